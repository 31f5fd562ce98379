// Far field W_0^(p) (Section 3.6): spreading -> FFT -> diagonal scaling ->
// inverse FFT -> interpolation on the Fourier grid M_0 x M_1 (x M_2), with no
// upsampling (rem:no_upsampling), in fractional coordinates.
//
// With the spreading window phi (exp(beta(sqrt(1-z^2)-1)), w cells wide) and its
// per-axis transform phi^(m), the scaling of eq:diag becomes
//   S(m) = What_0(|k_m|) / (V phi^(m)^2),  k_m = 2 pi L^{-T} m,  S(0) = 0,
// What_0(k) = psi~(k r_c / c) / k^2 (eq:W0hat), computed once per plan in FP64.
// The FFT is a hand-written mixed-radix (2, 3, 4, 5) Stockham transform; each
// workgroup transforms one grid line held in LDS.
#include <algorithm>
#include <climits>
#include <cmath>

#include "internal.h"

namespace pdmk {

static inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }

struct Radices {
  int n;
  int r[24];
};

static Radices factorize(int M) {
  Radices R{};
  int m = M;
  while (m % 4 == 0) { R.r[R.n++] = 4; m /= 4; }
  while (m % 2 == 0) { R.r[R.n++] = 2; m /= 2; }
  while (m % 3 == 0) { R.r[R.n++] = 3; m /= 3; }
  while (m % 5 == 0) { R.r[R.n++] = 5; m /= 5; }
  if (m != 1) throw Error{PDMK_ERR_UNSUPPORTED, "FFT size not 2,3,5-smooth"};
  return R;
}

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// y[k] = sum_r v[r] exp(sign 2 pi i r k / R) for R in {2, 3, 4, 5}, with the
// roots of unity as constants.
__device__ inline void small_dft(double2* v, int R, int sign) {
  const double sg = (double)sign;
  if (R == 2) {
    const double2 a = v[0], b = v[1];
    v[0] = make_double2(a.x + b.x, a.y + b.y);
    v[1] = make_double2(a.x - b.x, a.y - b.y);
  } else if (R == 4) {
    const double2 s0 = make_double2(v[0].x + v[2].x, v[0].y + v[2].y);
    const double2 d0 = make_double2(v[0].x - v[2].x, v[0].y - v[2].y);
    const double2 s1 = make_double2(v[1].x + v[3].x, v[1].y + v[3].y);
    const double2 d1 = make_double2(v[1].x - v[3].x, v[1].y - v[3].y);
    // sign i d1 = (-sign d1.y, sign d1.x)
    v[0] = make_double2(s0.x + s1.x, s0.y + s1.y);
    v[2] = make_double2(s0.x - s1.x, s0.y - s1.y);
    v[1] = make_double2(d0.x - sg * d1.y, d0.y + sg * d1.x);
    v[3] = make_double2(d0.x + sg * d1.y, d0.y - sg * d1.x);
  } else if (R == 3) {
    const double h = 0.8660254037844386;   // sin(2 pi / 3)
    const double2 a = v[0];
    const double2 t = make_double2(v[1].x + v[2].x, v[1].y + v[2].y);
    const double2 u = make_double2(v[1].x - v[2].x, v[1].y - v[2].y);
    const double2 m = make_double2(a.x - 0.5 * t.x, a.y - 0.5 * t.y);
    // sign i h u = (-sign h u.y, sign h u.x)
    v[0] = make_double2(a.x + t.x, a.y + t.y);
    v[1] = make_double2(m.x - sg * h * u.y, m.y + sg * h * u.x);
    v[2] = make_double2(m.x + sg * h * u.y, m.y - sg * h * u.x);
  } else {
    // cos and sin of 2 pi m / 5
    const double C[5] = {1.0, 0.30901699437494745, -0.8090169943749475, -0.8090169943749475,
                         0.30901699437494745};
    const double S[5] = {0.0, 0.9510565162951535, 0.5877852522924731, -0.5877852522924731,
                         -0.9510565162951535};
    double2 y[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      double sr = 0, si = 0;
#pragma unroll
      for (int r = 0; r < 5; ++r) {
        const int m = (r * k) % 5;
        const double c = C[m], sn = sg * S[m];
        sr += v[r].x * c - v[r].y * sn;
        si += v[r].x * sn + v[r].y * c;
      }
      y[k] = make_double2(sr, si);
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) v[k] = y[k];
  }
}

// One batch of grid lines for k_fft_lines: line l starts at
//   (l % nl0) so0 + ((l / nl0) % nl1) so1 + (l / (nl0 nl1)) so2
// and holds M elements `stride` apart.  tw is the twiddle table of the whole
// axis, exp(-2 pi i j / (M twmul)); the radix passes read tw[j twmul].  With
// post set, element i of line l is multiplied by tw[i (l % nl0)] after the
// transform (the inter-step twiddle of the four-step split).
struct FftLines {
  int M;
  int64_t stride;
  int nl0, nl1;
  int64_t so0, so1, so2;
  int nlines;
  int twmul;
  int post;
};

// Stockham FFT of `lpb` grid lines of length M per workgroup, in LDS (FP64
// twiddles from the host; sign = +1 uses their conjugates).  Lines along a
// strided direction are loaded line-fastest (the lines of a workgroup are
// adjacent in memory), lines along the contiguous direction element-fastest.
__global__ __launch_bounds__(256) void k_fft_lines(double2* __restrict__ data, FftLines f,
                                                   int lpb, int sign, Radices rad,
                                                   const double2* __restrict__ tw) {
  extern __shared__ double2 sh[];
  const int M = f.M;
  double2* b0 = sh;
  double2* b1 = sh + lpb * M;
  const int l0 = blockIdx.x * lpb;
  const int nl = min(lpb, f.nlines - l0);
  const int tot = nl * M;
  const bool contiguous = f.stride == 1;
  auto addr = [&](int l, int i) {
    const int line = l0 + l;
    const int r = line / f.nl0;
    return (int64_t)(line % f.nl0) * f.so0 + (int64_t)(r % f.nl1) * f.so1 +
           (int64_t)(r / f.nl1) * f.so2 + (int64_t)i * f.stride;
  };
  // eight loads in flight per thread
  for (int e0 = threadIdx.x; e0 < tot; e0 += 8 * 256) {
    double2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * 256;
      if (e < tot) {
        const int l = contiguous ? e / M : e % nl, i = contiguous ? e % M : e / nl;
        v[u] = data[addr(l, i)];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * 256;
      if (e < tot) {
        const int l = contiguous ? e / M : e % nl, i = contiguous ? e % M : e / nl;
        b0[l * M + i] = v[u];
      }
    }
  }
  __syncthreads();
  int Ns = 1;
  for (int pass = 0; pass < rad.n; ++pass) {
    const int R = rad.r[pass];
    const int nb = M / R;
    const int step = M / (Ns * R);   // twiddle index stride: exp(2 pi i jm / (Ns R))
    for (int jj = threadIdx.x; jj < nl * nb; jj += blockDim.x) {
      const int l = jj / nb, j = jj - l * nb;
      const double2* in = b0 + l * M;
      double2 v[5];
      for (int r = 0; r < R; ++r) v[r] = in[j + r * nb];
      const int jm = j % Ns;
      if (Ns > 1 && jm > 0) {
        double2 w1 = tw[(int64_t)jm * step * f.twmul];
        if (sign > 0) w1.y = -w1.y;
        double2 w = w1;
        for (int r = 1; r < R; ++r) {
          v[r] = cmul(v[r], w);
          w = cmul(w, w1);
        }
      }
      small_dft(v, R, sign);
      double2* out = b1 + l * M + (j / Ns) * Ns * R + jm;
      for (int r = 0; r < R; ++r) out[r * Ns] = v[r];
    }
    __syncthreads();
    double2* t = b0;
    b0 = b1;
    b1 = t;
    Ns *= R;
  }
  for (int e0 = threadIdx.x; e0 < tot; e0 += 256) {
    const int l = contiguous ? e0 / M : e0 % nl, i = contiguous ? e0 % M : e0 / nl;
    double2 v = b0[l * M + i];
    if (f.post) {
      double2 w = tw[(int64_t)i * ((l0 + l) % f.nl0)];
      if (sign > 0) w.y = -w.y;
      v = cmul(v, w);
    }
    data[addr(l, i)] = v;
  }
}

// Longest line a workgroup transforms in LDS (two FP64 complex buffers of
// 4096 points: 128 KB).  Longer axes use the four-step split below.
constexpr int kFftLineMax = 4096;

// Factor M = A B (A, B <= kFftLineMax, as balanced as possible), or A = M,
// B = 1 when M fits one line.
static void fft_split(int M, int& A, int& B) {
  A = M;
  B = 1;
  if (M <= kFftLineMax) return;
  int best = 0;
  for (int a = 2; a <= kFftLineMax; ++a)
    if (M % a == 0 && M / a <= kFftLineMax && (best == 0 || std::abs(a * a - M) <
                                                                std::abs(best * best - M)))
      best = a;
  if (best == 0)
    throw Error{PDMK_ERR_UNSUPPORTED, "Fourier grid axis has no split into two lines of at most " +
                                          std::to_string(kFftLineMax)};
  A = best;
  B = M / A;
}

static void fft_launch(double2* g, const FftLines& f, int sign, const double2* tw,
                       hipStream_t s) {
  Radices R = factorize(f.M);
  // several short lines per workgroup (at most 2048 points, 64 KB of LDS)
  const int lpb = std::max(1, std::min(2048 / f.M, 64));
  const int nblocks = (f.nlines + lpb - 1) / lpb;
  const size_t smem = 2 * (size_t)lpb * f.M * sizeof(double2);
  ensure_lds((const void*)&k_fft_lines, smem);
  hipLaunchKernelGGL(k_fft_lines, dim3(nblocks), dim3(256), smem, s, g, f, lpb, sign, R, tw);
  PDMK_HIP(hipGetLastError());
}

// In-place FFT of the grid along every axis.  An axis of length M = A B with
// M > kFftLineMax is split in four steps (n = B n1 + n2, k = k1 + A k2):
// forward, A-point transforms over n1, twiddle exp(-2 pi i n2 k1 / M),
// B-point transforms over n2, leaving X[k1 + A k2] at position B k1 + k2
// (transposed order, which the diagonal scaling table follows); the inverse
// takes that order back to natural order by the mirrored steps.
static void fft3(double2* g, const int* M, int dim, int sign, const double2* tw,
                 const int64_t* tw_off, hipStream_t s) {
  const int64_t M0 = M[0], M1 = M[1], M2 = dim == 3 ? M[2] : 1;
  for (int ax = 0; ax < dim; ++ax) {
    const int Ma = M[ax];
    if (Ma == 1) continue;
    // the other two axes: lines at (i % n_o0) s_o0 + (i / n_o0) s_o1
    int64_t sa, s_o0, s_o1;
    int n_o0, n_other;
    if (ax == 0) { sa = 1; n_o0 = (int)M1; s_o0 = M0; s_o1 = M0 * M1; n_other = (int)(M1 * M2); }
    else if (ax == 1) { sa = M0; n_o0 = (int)M0; s_o0 = 1; s_o1 = M0 * M1; n_other = (int)(M0 * M2); }
    else { sa = M0 * M1; n_o0 = (int)M0; s_o0 = 1; s_o1 = M0; n_other = (int)(M0 * M1); }
    int A, B;
    fft_split(Ma, A, B);
    const double2* t = tw + tw_off[ax];
    if (B == 1) {
      fft_launch(g, FftLines{Ma, sa, n_o0, INT_MAX, s_o0, s_o1, 0, n_other, 1, 0}, sign, t, s);
      continue;
    }
    // over n1 (or k1): lines n2 (k2 ... ) at offset n2 sa, elements B sa apart
    const FftLines over_a{A, B * sa, B, n_o0, sa, s_o0, s_o1, B * n_other, B, 0};
    // over n2 (or k2): lines k1 at offset B k1 sa, elements sa apart
    const FftLines over_b{B, sa, A, n_o0, B * sa, s_o0, s_o1, A * n_other, A, 0};
    if (sign < 0) {
      FftLines f1 = over_a;
      f1.post = 1;
      fft_launch(g, f1, sign, t, s);
      fft_launch(g, over_b, sign, t, s);
    } else {
      FftLines f1 = over_b;
      f1.post = 1;
      fft_launch(g, f1, sign, t, s);
      fft_launch(g, over_a, sign, t, s);
    }
  }
}

__device__ inline double es_win(double z, double beta) {
  double t = 1.0 - z * z;
  return t >= 0.0 ? exp(beta * (sqrt(t) - 1.0)) : 0.0;
}
__device__ inline float es_win(float z, float beta) {
  float t = 1.0f - z * z;
  return t >= 0.0f ? __expf(beta * (sqrtf(t) - 1.0f)) : 0.0f;
}

// LDS subgrid (doubles) of the spreading and interpolation blocks: the
// windows of 256 consecutive points in tree order cover a small box of cells.
constexpr int kSubCap = 4096;

template <int D>
__device__ inline void grid_coords(const KParams& kp, const double* __restrict__ x, int64_t n,
                                   int64_t i, const int* Ms, double* g) {
  // fractional coordinates u = L^{-1} x' of an oriented point, in grid units
  for (int a = 0; a < D; ++a) {
    double s = 0.0;
    for (int b = a; b < D; ++b) s += kp.Li[a + D * b] * x[b * n + i];
    s -= floor(s);
    g[a] = s * Ms[a];
  }
}

// Bounding box of the block's 256 points in grid cells (window start i0 per
// axis); returns the subgrid extent and whether it fits in LDS.
template <int D, int W, bool PAD = false>
__device__ inline bool block_box(const KParams& kp, int64_t n, const double* __restrict__ x,
                                 int64_t i, bool valid, const int* Ms, double* g, int* i0,
                                 int* lo_s, int* hi_s, int* lo, int* ext, int& vol) {
  constexpr double hw = 0.5 * W;
  if (threadIdx.x < 3) {
    lo_s[threadIdx.x] = INT_MAX;
    hi_s[threadIdx.x] = INT_MIN;
  }
  __syncthreads();
  for (int a = 0; a < D; ++a) {
    g[a] = 0;
    i0[a] = 0;
  }
  if (valid) {
    grid_coords<D>(kp, x, n, i, Ms, g);
    for (int a = 0; a < D; ++a) {
      i0[a] = (int)ceil(g[a] - hw);
      atomicMin(&lo_s[a], i0[a]);
      atomicMax(&hi_s[a], i0[a]);
    }
  }
  __syncthreads();
  long long v = 1;
  for (int a = 0; a < 3; ++a) {
    lo[a] = a < D ? lo_s[a] : 0;
    ext[a] = a < D ? hi_s[a] - lo_s[a] + W : 1;
    // PAD: row stride = 8 (mod 16) doubles, so that the 8 rows of a wave's
    // 8 x 8 stencil columns fall on alternating halves of the LDS banks
    // (padding cells are never written)
    if (PAD && a == 0) ext[0] += (24 - ext[0] % 16) % 16;
    if (a < D) v *= ext[a];
  }
  vol = v <= kSubCap ? (int)v : kSubCap + 1;
  return v <= kSubCap;
}

__device__ inline int wrap_index(int i, int M) {
  int r = i % M;
  return r < 0 ? r + M : r;
}

// Lane j's value, read by every lane (wave-uniform).
__device__ inline double rdlane(double v, int j) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), j);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), j);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline float rdlane(float v, int j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}

// Spreading (step one of Section 3.6): the block takes 256 consecutive
// sources in tree order and accumulates their windows in an LDS subgrid; each
// wave spreads its 64 sources one at a time, the lanes covering the W^D
// stencil entries (distinct addresses, so the LDS atomics do not collide).
// The subgrid is then added to the grid with one global atomic per touched
// cell.  A block whose box exceeds the LDS subgrid (sources straddling the
// periodic boundary) spreads straight into the grid with global atomics.
template <int D, int W, class Real>
__global__ __launch_bounds__(256) void k_spread_coop(KParams kp, int64_t n,
                                                     const double* __restrict__ x,
                                                     const double* __restrict__ q, int M0,
                                                     int M1, int M2, double beta,
                                                     double* __restrict__ grid) {
  __shared__ double sub[kSubCap];
  __shared__ int lo_s[3], hi_s[3];
  constexpr int NE = D == 3 ? W * W * W : W * W;
  constexpr Real hw = (Real)(0.5 * W);
  const int Ms[3] = {M0, M1, M2};
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool valid = i < n;
  double g[D];
  int i0[D], lo[3], ext[3], vol;
  const bool tiled =
      block_box<D, W, W == 8>(kp, n, x, i, valid, Ms, g, i0, lo_s, hi_s, lo, ext, vol);
  if (tiled) {
    for (int c = threadIdx.x; c < vol; c += 256) sub[c] = 0.0;
    __syncthreads();
  }
  const double qi = valid ? q[i] : 0.0;
  const int lane = threadIdx.x & 63;
  // lane l < D W holds the window value of axis l / W, offset l % W
  const int wa = lane / W, wk = lane - wa * W;
  for (int j = 0; j < 64; ++j) {
    // point j of this wave, broadcast from its lane (uniform values)
    const double qj = rdlane(qi, j);
    if (qj == 0.0) continue;   // also skips lanes past the end (uniform across the wave)
    double gj[D];
    int ij[D];
    for (int a = 0; a < D; ++a) {
      gj[a] = rdlane(g[a], j);
      ij[a] = __builtin_amdgcn_readlane(i0[a], j);
    }
    Real wv = 0;
    if (wa < D) {
      const double ga = wa == 0 ? gj[0] : (wa == 1 ? gj[1] : gj[D - 1]);
      const int ia = wa == 0 ? ij[0] : (wa == 1 ? ij[1] : ij[D - 1]);
      wv = es_win((Real)((ia + wk - ga) / (double)hw), (Real)beta);
      if (wa == 0) wv *= (Real)qj;
    }
    if (D == 3) {
      // lane = stencil column (k0, k1); the column's W values differ only
      // in the uniform last-axis weight
#pragma unroll
      for (int p0 = 0; p0 < W * W; p0 += 64) {
        const int pr = p0 + lane;
        const int k0 = pr % W, k1 = pr / W;
        const Real v01 = __shfl(wv, k0) * __shfl(wv, W + (k1 < W ? k1 : 0));
        if (pr < W * W) {
          if (tiled) {
            const int ob = ((ij[D - 1] - lo[D - 1]) * ext[1] + ij[1] - lo[1] + k1) * ext[0] +
                           ij[0] - lo[0] + k0;
            const int st = ext[0] * ext[1];
#pragma unroll
            for (int k2 = 0; k2 < W; ++k2) {
              const Real v2 = rdlane(wv, 2 * W + k2);
              atomicAdd(sub + ob + k2 * st, (double)(v01 * v2));
            }
          } else {
            const int64_t gb = wrap_index(ij[0] + k0, M0) + (int64_t)M0 * wrap_index(ij[1] + k1, M1);
#pragma unroll
            for (int k2 = 0; k2 < W; ++k2) {
              const Real v2 = rdlane(wv, 2 * W + k2);
              atomicAdd(grid + gb + (int64_t)M0 * M1 * wrap_index(ij[D - 1] + k2, M2),
                        (double)(v01 * v2));
            }
          }
        }
      }
    } else {
#pragma unroll
      for (int e0 = 0; e0 < NE; e0 += 64) {
        const int e = e0 + lane;
        const int k0 = e % W, k1 = (e / W) % W;
        const Real v = __shfl(wv, k0) * __shfl(wv, W + k1);
        if (e < NE) {
          if (tiled) {
            const int o = (ij[D - 1] - lo[D - 1] + k1) * ext[0] + ij[0] - lo[0] + k0;
            atomicAdd(sub + o, (double)v);
          } else {
            const int64_t gi = wrap_index(ij[0] + k0, M0) + (int64_t)M0 * wrap_index(ij[1] + k1, M1);
            atomicAdd(grid + gi, (double)v);
          }
        }
      }
    }
  }
  if (tiled) {
    __syncthreads();
    for (int c = threadIdx.x; c < vol; c += 256) {
      const double v = sub[c];
      if (v == 0.0) continue;
      const int c0 = c % ext[0], c1 = (c / ext[0]) % ext[1], c2 = c / (ext[0] * ext[1]);
      int64_t gi = wrap_index(lo[0] + c0, M0) + (int64_t)M0 * wrap_index(lo[1] + c1, M1);
      if (D == 3) gi += (int64_t)M0 * M1 * wrap_index(lo[2] + c2, M2);
      atomicAdd(grid + gi, v);
    }
  }
}

// Fixed-order spreading.  A block is one wave and takes 64 consecutive
// sources in tree order; its lanes cover distinct stencil entries of one
// source at a time, so the LDS subgrid is accumulated with plain adds in
// program order.  Each subgrid cell value v (|v| <= sum |q|, the window is at
// most 1) then goes to the grid as two 64-bit fixed-point words, hi = rint(v /
// u) and lo = rint((v - hi u) / u2) with u = sum |q| 2^-52 and u2 = u 2^-30,
// added with integer atomics: integer sums do not depend on their order, and
// k_fp_to_grid reads the grid back as HI u + LO u2.  Bounds: |hi| <= 2^52 and
// |lo| <= 1.5 2^30 per add, and a cell receives at most one add per source
// (2^30 sources), so neither word overflows; the representation error of an
// add is below u2.  Blocks whose box does not fit the subgrid add each
// stencil entry the same way.
__device__ inline void fp_add(unsigned long long* __restrict__ hi,
                              unsigned long long* __restrict__ lo, double v, double u,
                              double iu, double iu2, double u2) {
  const double h = rint(v * iu);
  const double r = fma(-h, u, v);
  const long long hl = (long long)h;
  const long long ll = (long long)rint(r * iu2);
  atomicAdd(hi, (unsigned long long)hl);
  atomicAdd(lo, (unsigned long long)ll);
  (void)u2;
}

template <int D, int W, class Real>
__global__ __launch_bounds__(64) void k_spread_det(KParams kp, int64_t n,
                                                   const double* __restrict__ x,
                                                   const double* __restrict__ q, int M0, int M1,
                                                   int M2, double beta,
                                                   const double* __restrict__ qsum,
                                                   unsigned long long* __restrict__ ghi,
                                                   unsigned long long* __restrict__ glo) {
  __shared__ double sub[kSubCap];
  __shared__ int lo_s[3], hi_s[3];
  constexpr int NE = D == 3 ? W * W * W : W * W;
  constexpr Real hw = (Real)(0.5 * W);
  const int Ms[3] = {M0, M1, M2};
  const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const bool valid = i < n;
  const double qa = qsum[1] > 0.0 ? qsum[1] : 1.0;
  const double u = ldexp(qa, -52), u2 = ldexp(qa, -82);
  const double iu = 1.0 / u, iu2 = 1.0 / u2;
  double g[D];
  int i0[D], lo[3], ext[3], vol;
  const bool tiled = block_box<D, W>(kp, n, x, i, valid, Ms, g, i0, lo_s, hi_s, lo, ext, vol);
  if (tiled) {
    for (int c = threadIdx.x; c < vol; c += 64) sub[c] = 0.0;
    __syncthreads();
  }
  const double qi = valid ? q[i] : 0.0;
  const int lane = threadIdx.x;
  const int wa = lane / W, wk = lane - wa * W;
  for (int j = 0; j < 64; ++j) {
    const double qj = rdlane(qi, j);
    if (qj == 0.0) continue;
    double gj[D];
    int ij[D];
    for (int a = 0; a < D; ++a) {
      gj[a] = rdlane(g[a], j);
      ij[a] = __builtin_amdgcn_readlane(i0[a], j);
    }
    Real wv = 0;
    if (wa < D) {
      const double ga = wa == 0 ? gj[0] : (wa == 1 ? gj[1] : gj[D - 1]);
      const int ia = wa == 0 ? ij[0] : (wa == 1 ? ij[1] : ij[D - 1]);
      wv = es_win((Real)((ia + wk - ga) / (double)hw), (Real)beta);
      if (wa == 0) wv *= (Real)qj;
    }
    for (int e0 = 0; e0 < NE; e0 += 64) {
      const int e = e0 + lane;
      const int k0 = e % W, k1 = (e / W) % W, k2 = D == 3 ? e / (W * W) : 0;
      Real v = __shfl(wv, k0) * __shfl(wv, W + (k1 < W ? k1 : 0));
      if (D == 3) v *= __shfl(wv, 2 * W + (k2 < W ? k2 : 0));
      if (e < NE) {
        if (tiled) {
          int o = (ij[1] - lo[1] + k1) * ext[0] + ij[0] - lo[0] + k0;
          if (D == 3) o += (ij[D - 1] - lo[D - 1] + k2) * ext[0] * ext[1];
          sub[o] += (double)v;   // distinct addresses across the wave
        } else {
          int64_t gi = wrap_index(ij[0] + k0, M0) + (int64_t)M0 * wrap_index(ij[1] + k1, M1);
          if (D == 3) gi += (int64_t)M0 * M1 * wrap_index(ij[D - 1] + k2, M2);
          fp_add(ghi + gi, glo + gi, (double)v, u, iu, iu2, u2);
        }
      }
    }
  }
  if (tiled) {
    __syncthreads();
    for (int c = threadIdx.x; c < vol; c += 64) {
      const double v = sub[c];
      if (v == 0.0) continue;
      const int c0 = c % ext[0], c1 = (c / ext[0]) % ext[1], c2 = c / (ext[0] * ext[1]);
      int64_t gi = wrap_index(lo[0] + c0, M0) + (int64_t)M0 * wrap_index(lo[1] + c1, M1);
      if (D == 3) gi += (int64_t)M0 * M1 * wrap_index(lo[2] + c2, M2);
      fp_add(ghi + gi, glo + gi, v, u, iu, iu2, u2);
    }
  }
}

// Fixed-point grid -> complex grid (HI u + LO u2, u from sum |q|).
__global__ void k_fp_to_grid(int64_t n, const unsigned long long* __restrict__ ghi,
                             const unsigned long long* __restrict__ glo,
                             const double* __restrict__ qsum, double2* __restrict__ c) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double qa = qsum[1] > 0.0 ? qsum[1] : 1.0;
  const double v = (double)(long long)ghi[i] * ldexp(qa, -52) +
                   (double)(long long)glo[i] * ldexp(qa, -82);
  c[i] = make_double2(v, 0.0);
}

// Interpolation (step five of Section 3.6) at targets in tree order, one
// target per lane; the block's subgrid is read into LDS once.  Results are
// added to the near-field arrays (tree order), gradients rotated by L^{-T}.
// comp: the grid's real (0) or imaginary (1) part is interpolated (the
// imaginary part carries the Bloch far field).
template <int D, int W, bool GRAD, class Real>
__global__ __launch_bounds__(256) void k_interp_t(KParams kp, int64_t n,
                                                  const double* __restrict__ x, int M0, int M1,
                                                  int M2, double beta,
                                                  const double2* __restrict__ grid,
                                                  double* __restrict__ pot,
                                                  double* __restrict__ grad, int comp) {
  __shared__ double sub[kSubCap];
  __shared__ int lo_s[3], hi_s[3];
  constexpr double hw = 0.5 * W;
  const int Ms[3] = {M0, M1, M2};
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool valid = i < n;
  double g[D];
  int i0[D], lo[3], ext[3], vol;
  const bool tiled = block_box<D, W>(kp, n, x, i, valid, Ms, g, i0, lo_s, hi_s, lo, ext, vol);
  if (tiled) {
    // the block's subgrid into LDS, eight loads in flight per thread
    for (int c0 = threadIdx.x; c0 < vol; c0 += 8 * 256) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = c0 + u * 256;
        v[u] = 0.0;
        if (c < vol) {
          const int a0 = c % ext[0], a1 = (c / ext[0]) % ext[1], a2 = c / (ext[0] * ext[1]);
          int64_t gi = wrap_index(lo[0] + a0, M0) + (int64_t)M0 * wrap_index(lo[1] + a1, M1);
          if (D == 3) gi += (int64_t)M0 * M1 * wrap_index(lo[2] + a2, M2);
          v[u] = comp ? grid[gi].y : grid[gi].x;
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (c0 + u * 256 < vol) sub[c0 + u * 256] = v[u];
    }
    __syncthreads();
  }
  if (!valid) return;
  // window values (and derivatives) of axes 0 and 1 in registers; axis 2 is
  // evaluated inside its loop
  auto win = [&](int a, int k, double& v, double& dv) {
    const Real z = (Real)((i0[a] + k - g[a]) / hw);
    const Real e = es_win(z, (Real)beta);
    v = (double)e;
    dv = 0.0;
    if (GRAD) {
      const Real t = (Real)1 - z * z;
      dv = (t > (Real)0) ? (double)(e * (Real)beta * (-z / sqrt(t))) * (-Ms[a] / hw) : 0.0;
    }
  };
  double wt0[W], dw0[W], wt1[W], dw1[W];
#pragma unroll
  for (int k = 0; k < W; ++k) {
    win(0, k, wt0[k], dw0[k]);
    win(1, k, wt1[k], dw1[k]);
  }
  double acc = 0.0, gu[3] = {0, 0, 0};
  constexpr int K2 = D == 3 ? W : 1;
  const int b0 = i0[0] - lo[0], b1 = i0[1] - lo[1], b2 = D == 3 ? i0[D - 1] - lo[D - 1] : 0;
  for (int k2 = 0; k2 < K2; ++k2) {
    double w2 = 1.0, d2 = 0.0;
    if (D == 3) win(D - 1, k2, w2, d2);
    double p2 = 0.0, g20 = 0.0, g21 = 0.0;   // this k2 plane: value, d/du0, d/du1
#pragma unroll
    for (int k1 = 0; k1 < W; ++k1) {
      double a0 = 0.0, ad0 = 0.0;
      if (tiled) {
        const double* row = sub + ((b2 + k2) * ext[1] + (b1 + k1)) * ext[0] + b0;
#pragma unroll
        for (int k0 = 0; k0 < W; ++k0) {
          const double v = row[k0];
          a0 = fma(v, wt0[k0], a0);
          if (GRAD) ad0 = fma(v, dw0[k0], ad0);
        }
      } else {
        int64_t row = (int64_t)M0 * wrap_index(i0[1] + k1, M1);
        if (D == 3) row += (int64_t)M0 * M1 * wrap_index(i0[D - 1] + k2, M2);
#pragma unroll
        for (int k0 = 0; k0 < W; ++k0) {
          const double2 gv = grid[row + wrap_index(i0[0] + k0, M0)];
          const double v = comp ? gv.y : gv.x;
          a0 = fma(v, wt0[k0], a0);
          if (GRAD) ad0 = fma(v, dw0[k0], ad0);
        }
      }
      p2 = fma(a0, wt1[k1], p2);
      if (GRAD) {
        g20 = fma(ad0, wt1[k1], g20);
        g21 = fma(a0, dw1[k1], g21);
      }
    }
    acc = fma(p2, w2, acc);
    if (GRAD) {
      gu[0] = fma(g20, w2, gu[0]);
      gu[1] = fma(g21, w2, gu[1]);
      if (D == 3) gu[2] = fma(p2, d2, gu[2]);
    }
  }
  pot[i] += acc;
  if (GRAD)
    for (int b = 0; b < D; ++b) {
      double s = 0.0;
      for (int a = 0; a <= b; ++a) s += kp.Li[a + D * b] * gu[a];
      grad[i * D + b] += s;
    }
}

template <int D, int W, class Real>
static void launch_spread_interp(pdmk_plan* P, Eval& E, const int* M, double beta, double* grid,
                                 double2* cg, bool want_grad, bool spread) {
  if (spread) {
    if (E.n_src > 0 && E.det)
      hipLaunchKernelGGL((k_spread_det<D, W, Real>), dim3(nblk(E.n_src, 64)), dim3(64), 0, E.s,
                         P->kp, E.n_src, E.ox, E.oq, M[0], M[1], M[2], beta, E.qsum,
                         E.far_hi, E.far_lo);
    else if (E.n_src > 0)
      hipLaunchKernelGGL((k_spread_coop<D, W, Real>), dim3(nblk(E.n_src, 256)), dim3(256), 0,
                         E.s, P->kp, E.n_src, E.ox, E.oq, M[0], M[1], M[2], beta, grid);
  } else if (E.n_trg > 0) {
    if (want_grad)
      hipLaunchKernelGGL((k_interp_t<D, W, true, Real>), dim3(nblk(E.n_trg, 256)), dim3(256), 0,
                         E.s, P->kp, E.n_trg, E.tx, M[0], M[1], M[2], beta, cg,
                         E.far_out ? E.far_out : E.pot_sorted, E.grad_sorted, E.far_comp);
    else
      hipLaunchKernelGGL((k_interp_t<D, W, false, Real>), dim3(nblk(E.n_trg, 256)), dim3(256),
                         0, E.s, P->kp, E.n_trg, E.tx, M[0], M[1], M[2], beta, cg,
                         E.far_out ? E.far_out : E.pot_sorted, E.grad_sorted, E.far_comp);
  }
}

template <int D, class Real>
static void spread_interp_w(pdmk_plan* P, Eval& E, const int* M, int w, double beta,
                            double* grid, double2* cg, bool want_grad, bool spread) {
  switch (w) {
#define PDMK_W(WW) \
  case WW: launch_spread_interp<D, WW, Real>(P, E, M, beta, grid, cg, want_grad, spread); break;
    PDMK_W(4) PDMK_W(5) PDMK_W(6) PDMK_W(7) PDMK_W(8) PDMK_W(9) PDMK_W(10) PDMK_W(11)
    PDMK_W(12) PDMK_W(13) PDMK_W(14) PDMK_W(15) PDMK_W(16)
#undef PDMK_W
    default: throw Error{PDMK_ERR_UNSUPPORTED, "window width outside 4..16"};
  }
}

static void spread_interp(pdmk_plan* P, Eval& E, const int* M, int w, double beta,
                          double* grid, double2* cg, bool want_grad, bool spread) {
  const bool f32 = P->kp.precision == PDMK_PREC_MIXED && (P->mixed_parts & 4);
  if (P->kp.dim == 3) {
    if (f32) spread_interp_w<3, float>(P, E, M, w, beta, grid, cg, want_grad, spread);
    else spread_interp_w<3, double>(P, E, M, w, beta, grid, cg, want_grad, spread);
  } else {
    if (f32) spread_interp_w<2, float>(P, E, M, w, beta, grid, cg, want_grad, spread);
    else spread_interp_w<2, double>(P, E, M, w, beta, grid, cg, want_grad, spread);
  }
}


__global__ void k_to_complex(int64_t n, const double* __restrict__ g, double2* __restrict__ c) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c[i] = make_double2(g[i], 0.0);
}

__global__ void k_to_complex2(int64_t n, const double* __restrict__ re,
                              const double* __restrict__ im, double2* __restrict__ c) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c[i] = make_double2(re[i], im[i]);
}

// Bloch source pre-modulation (Section 4.1): q~ = q_w e^{-i beta.x_w} for the
// originals in tree order (wrapped positions x_w and charges q_w).
__global__ void k_bloch_premod(KParams kp, int64_t n, const double* __restrict__ x,
                               const double* __restrict__ qr, const double* __restrict__ qi,
                               double* __restrict__ outr, double* __restrict__ outi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double ph = 0.0;
  for (int a = 0; a < kp.dim; ++a) ph += kp.beta[a] * x[a * n + i];
  double sn, cs;
  sincos(-ph, &sn, &cs);
  outr[i] = qr[i] * cs - qi[i] * sn;
  outi[i] = qr[i] * sn + qi[i] * cs;
}

__global__ void k_scale(int64_t n, double2* __restrict__ c, const double* __restrict__ s) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    double v = s[i];
    c[i] = make_double2(c[i].x * v, c[i].y * v);
  }
}

// Diagonal scaling table (FP64), once per plan.
// Spectrum order per axis: B > 1 for an axis transformed in four steps, whose
// storage position p holds frequency index p / B + A (p % B).
struct FftOrder {
  int A[3], B[3];
};

__global__ void k_farscale(KParams kp, int M0, int M1, int M2, int Mp0, int Mp1, int Mp2,
                           FftOrder ord, const double* __restrict__ wf0,
                           const double* __restrict__ wf1, const double* __restrict__ wf2,
                           const double* __restrict__ gx, const double* __restrict__ gwpsi, int nq,
                           double c, double c0, double V, double* __restrict__ out) {
  const int64_t n = (int64_t)M0 * M1 * M2;
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int d = kp.dim;
  int ii[3] = {(int)(idx % M0), (int)((idx / M0) % M1), (int)(idx / ((int64_t)M0 * M1))};
  for (int a = 0; a < 3; ++a)
    if (ord.B[a] > 1) ii[a] = ii[a] / ord.B[a] + ord.A[a] * (ii[a] % ord.B[a]);
  const int Ms[3] = {M0, M1, M2};
  int m[3] = {0, 0, 0};
  bool nyq = false, zero = true;
  const int Mp[3] = {Mp0, Mp1, Mp2};
  for (int a = 0; a < d; ++a) {
    m[a] = ii[a] < Ms[a] / 2 ? ii[a] : ii[a] - Ms[a];
    if (Ms[a] > 1 && Ms[a] % 2 == 0 && ii[a] == Ms[a] / 2) nyq = true;
    // only the modes of the grid of eq:Mi are kept (|m_a| < M_a / 2)
    if (2 * m[a] >= Mp[a] || 2 * m[a] < -Mp[a] + 1) nyq = true;
    if (m[a] != 0) zero = false;
  }
  // periodic: m = 0 omitted (charge neutrality); Bloch: every mode kept, at
  // the shifted wave vector k_m + beta (Section 4.1)
  if (nyq || (zero && !kp.bloch)) { out[idx] = 0.0; return; }
  double k2 = 0.0;
  for (int b = 0; b < d; ++b) {
    double s = 0.0;
    for (int a = 0; a < d; ++a) s += kp.Li[a + d * b] * m[a];
    s *= 2.0 * 3.14159265358979323846;
    if (kp.bloch) s += kp.beta[b];
    k2 += s * s;
  }
  const double x = sqrt(k2) * kp.rc / c;
  double ps = 0.0;
  for (int j = 0; j < nq; ++j) ps += gwpsi[j] * cos(c * x * gx[j]);
  ps /= 2.0 * c0;
  double den = wf0[ii[0]] * wf1[ii[1]];
  if (d == 3) den *= wf2[ii[2]];
  out[idx] = ps / k2 / V / (den * den);
}

void far_build_scale(pdmk_plan* P) {
  const Geometry& g = P->g;
  const int d = g.dim;
  int M[3] = {g.fgrid[0], g.fgrid[1], d == 3 ? g.fgrid[2] : 1};
  int64_t n = (int64_t)M[0] * M[1] * M[2];
  std::vector<double> wf[3];
  for (int a = 0; a < 3; ++a)
    wf[a] = (a < d) ? window_ft(M[a], P->mp.nufft_w, P->nufft_beta) : std::vector<double>(1, 1.0);
  const Pswf& ps = *P->P;
  std::vector<double> gwpsi(ps.qx.size());
  for (size_t i = 0; i < ps.qx.size(); ++i) gwpsi[i] = ps.qw[i] * ps.qpsi[i];
  std::vector<void*> tmp;
  auto up = [&](const std::vector<double>& v) {
    double* p;
    PDMK_HIP(hipMalloc(&p, v.size() * sizeof(double)));
    PDMK_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice));
    tmp.push_back(p);
    return p;
  };
  double* d0 = up(wf[0]);
  double* d1 = up(wf[1]);
  double* d2 = up(wf[2]);
  double* dgx = up(ps.qx);
  double* dgw = up(gwpsi);
  {
    // FFT twiddles exp(-2 pi i k / M_a), k < M_a, one table per axis
    std::vector<double2> tw;
    for (int a = 0; a < 3; ++a) {
      P->fftw_off[a] = (int64_t)tw.size();
      for (int k = 0; k < M[a]; ++k) {
        const double t = -2.0 * M_PI * (double)k / (double)M[a];
        tw.push_back(make_double2(std::cos(t), std::sin(t)));
      }
    }
    PDMK_HIP(hipMalloc(&P->d_fftw, tw.size() * sizeof(double2)));
    PDMK_HIP(hipMemcpy(P->d_fftw, tw.data(), tw.size() * sizeof(double2), hipMemcpyHostToDevice));
  }
  PDMK_HIP(hipMalloc(&P->d_farscale, n * sizeof(double)));
  FftOrder ord{};
  for (int a = 0; a < 3; ++a) fft_split(M[a], ord.A[a], ord.B[a]);
  hipLaunchKernelGGL(k_farscale, dim3(nblk(n, 256)), dim3(256), 0, 0, P->kp, M[0], M[1], M[2],
                     g.fgrid_paper[0], g.fgrid_paper[1], d == 3 ? g.fgrid_paper[2] : 1, ord, d0,
                     d1, d2, dgx, dgw, (int)ps.qx.size(), ps.c, ps.c0, g.volume, P->d_farscale);
  PDMK_HIP(hipDeviceSynchronize());
  for (void* p : tmp) (void)hipFree(p);
}

void stage_far_grid(pdmk_plan* P, Eval& E) {
  const Geometry& g = P->g;
  const int d = g.dim;
  int M[3] = {g.fgrid[0], g.fgrid[1], d == 3 ? g.fgrid[2] : 1};
  int64_t n = (int64_t)M[0] * M[1] * M[2];
  const int w = P->mp.nufft_w;
  const double beta = P->nufft_beta;
  double* grid = E.alloc<double>(n);
  double2* cg = E.alloc<double2>(n);
  E.far_grid = grid;
  E.far_cg = cg;
  const bool tm = E.timing && E.far_ev[0];
  if (tm) PDMK_HIP(hipEventRecord(E.far_ev[0], E.s));
  if (E.det) {
    // fixed-point grid (two words per cell), see k_spread_det
    E.far_hi = E.alloc<unsigned long long>(n);
    E.far_lo = E.alloc<unsigned long long>(n);
    fill_zero(E.far_hi, n * sizeof(unsigned long long), E.s);
    fill_zero(E.far_lo, n * sizeof(unsigned long long), E.s);
    spread_interp(P, E, M, w, beta, grid, cg, false, true);
    hipLaunchKernelGGL(k_fp_to_grid, dim3(nblk(n, 256)), dim3(256), 0, E.s, n, E.far_hi,
                       E.far_lo, E.qsum, cg);
  } else if (P->kp.bloch) {
    // complex pre-modulated charges: real and imaginary parts spread apart
    double* grid2 = E.alloc<double>(n);
    double* qtr = E.alloc<double>(E.n_src);
    double* qti = E.alloc<double>(E.n_src);
    if (E.n_src > 0)
      hipLaunchKernelGGL(k_bloch_premod, dim3(nblk(E.n_src, 256)), dim3(256), 0, E.s, P->kp,
                         E.n_src, E.ox, E.oq, E.oq_im, qtr, qti);
    double* keep = E.oq;
    E.oq = qtr;
    fill_zero(grid, n * sizeof(double), E.s);
    spread_interp(P, E, M, w, beta, grid, cg, false, true);
    E.oq = qti;
    fill_zero(grid2, n * sizeof(double), E.s);
    spread_interp(P, E, M, w, beta, grid2, cg, false, true);
    E.oq = keep;
    hipLaunchKernelGGL(k_to_complex2, dim3(nblk(n, 256)), dim3(256), 0, E.s, n, grid, grid2, cg);
  } else {
    fill_zero(grid, n * sizeof(double), E.s);
    spread_interp(P, E, M, w, beta, grid, cg, false, true);
    hipLaunchKernelGGL(k_to_complex, dim3(nblk(n, 256)), dim3(256), 0, E.s, n, grid, cg);
  }
  if (tm) PDMK_HIP(hipEventRecord(E.far_ev[1], E.s));
  fft3(cg, M, d, -1, P->d_fftw, P->fftw_off, E.s);
  hipLaunchKernelGGL(k_scale, dim3(nblk(n, 256)), dim3(256), 0, E.s, n, cg, P->d_farscale);
  fft3(cg, M, d, +1, P->d_fftw, P->fftw_off, E.s);
  if (tm) PDMK_HIP(hipEventRecord(E.far_ev[2], E.s));
}

void stage_far_interp(pdmk_plan* P, Eval& E, bool want_grad) {
  const Geometry& g = P->g;
  int M[3] = {g.fgrid[0], g.fgrid[1], g.dim == 3 ? g.fgrid[2] : 1};
  if (E.far_out) fill_zero(E.far_out, E.n_trg * sizeof(double), E.s);
  const bool tm = E.timing && E.far_ev[3];
  if (tm) PDMK_HIP(hipEventRecord(E.far_ev[3], E.s));
  spread_interp(P, E, M, P->mp.nufft_w, P->nufft_beta, E.far_grid, E.far_cg, want_grad, false);
  if (tm) PDMK_HIP(hipEventRecord(E.far_ev[4], E.s));
}

}  // namespace pdmk

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
#include <climits>

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

// y[k] = sum_r v[r] exp(sign 2 pi i r k / R), R <= 5
__device__ inline void small_dft(double2* v, int R, int sign) {
  double2 y[5];
  for (int k = 0; k < R; ++k) {
    double sr = 0, si = 0;
    for (int r = 0; r < R; ++r) {
      double c, s;
      sincospi(2.0 * (double)((r * k) % R) / (double)R, &s, &c);
      s *= sign;
      sr += v[r].x * c - v[r].y * s;
      si += v[r].x * s + v[r].y * c;
    }
    y[k] = make_double2(sr, si);
  }
  for (int k = 0; k < R; ++k) v[k] = y[k];
}

// One workgroup per grid line of length M along one axis.
__global__ void k_fft_lines(double2* __restrict__ data, int M, int64_t stride, int nl0,
                            int64_t so0, int64_t so1, int sign, Radices rad) {
  extern __shared__ double2 sh[];
  double2* b0 = sh;
  double2* b1 = sh + M;
  const int line = blockIdx.x;
  const int64_t base = (int64_t)(line % nl0) * so0 + (int64_t)(line / nl0) * so1;
  for (int i = threadIdx.x; i < M; i += blockDim.x) b0[i] = data[base + i * stride];
  __syncthreads();
  int Ns = 1;
  for (int pass = 0; pass < rad.n; ++pass) {
    const int R = rad.r[pass];
    const int nb = M / R;
    for (int j = threadIdx.x; j < nb; j += blockDim.x) {
      double2 v[5];
      for (int r = 0; r < R; ++r) v[r] = b0[j + r * nb];
      const int jm = j % Ns;
      if (Ns > 1) {
        double s, c;
        sincospi(2.0 * (double)jm / (double)(Ns * R), &s, &c);
        const double2 w1 = make_double2(c, sign * s);
        double2 w = w1;
        for (int r = 1; r < R; ++r) {
          v[r] = cmul(v[r], w);
          w = cmul(w, w1);
        }
      }
      small_dft(v, R, sign);
      const int idx = (j / Ns) * Ns * R + jm;
      for (int r = 0; r < R; ++r) b1[idx + r * Ns] = v[r];
    }
    __syncthreads();
    double2* t = b0;
    b0 = b1;
    b1 = t;
    Ns *= R;
  }
  for (int i = threadIdx.x; i < M; i += blockDim.x) data[base + i * stride] = b0[i];
}

static void fft3(double2* g, const int* M, int dim, int sign, hipStream_t s) {
  const int64_t M0 = M[0], M1 = M[1], M2 = dim == 3 ? M[2] : 1;
  for (int ax = 0; ax < dim; ++ax) {
    int Ma = M[ax];
    if (Ma == 1) continue;
    if (Ma > 4096) throw Error{PDMK_ERR_UNSUPPORTED, "Fourier grid axis longer than 4096"};
    Radices R = factorize(Ma);
    int64_t stride, so0, so1;
    int nl0, nlines;
    if (ax == 0) { stride = 1; nl0 = (int)M1; so0 = M0; so1 = M0 * M1; nlines = (int)(M1 * M2); }
    else if (ax == 1) { stride = M0; nl0 = (int)M0; so0 = 1; so1 = M0 * M1; nlines = (int)(M0 * M2); }
    else { stride = M0 * M1; nl0 = (int)M0; so0 = 1; so1 = M0; nlines = (int)(M0 * M1); }
    size_t smem = 2 * (size_t)Ma * sizeof(double2);
    hipLaunchKernelGGL(k_fft_lines, dim3(nlines), dim3(256), smem, s, g, Ma, stride, nl0, so0,
                       so1, sign, R);
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

// Tiled spreading: a block takes 256 consecutive sources in tree order; their
// windows cover a small box of grid cells, accumulated in an LDS subgrid with
// LDS atomics and then added to the grid with one global atomic per touched
// cell.  A block whose box exceeds the LDS subgrid (sources straddling the
// periodic boundary) falls back to global atomics.
constexpr int kSubCap = 8192;

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

template <int D, class Real>
__global__ __launch_bounds__(256) void k_spread_tiled(KParams kp, int64_t n,
                                                      const double* __restrict__ x,
                                                      const double* __restrict__ q, int M0,
                                                      int M1, int M2, int w, double beta,
                                                      double* __restrict__ grid) {
  __shared__ double sub[kSubCap];
  __shared__ int lo[3], hi[3];
  const int Ms[3] = {M0, M1, M2};
  const double hw = 0.5 * w;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool valid = i < n;
  if (threadIdx.x < 3) {
    lo[threadIdx.x] = INT_MAX;
    hi[threadIdx.x] = INT_MIN;
  }
  __syncthreads();
  double g[D];
  int i0[D];
  if (valid) {
    grid_coords<D>(kp, x, n, i, Ms, g);
    for (int a = 0; a < D; ++a) {
      i0[a] = (int)ceil(g[a] - hw);
      atomicMin(&lo[a], i0[a]);
      atomicMax(&hi[a], i0[a]);
    }
  }
  __syncthreads();
  int ext[3] = {1, 1, 1};
  long long vol = 1;
  for (int a = 0; a < D; ++a) {
    ext[a] = hi[a] - lo[a] + w;
    vol *= ext[a];
  }
  const bool tiled = vol <= kSubCap;
  if (tiled) {
    for (int c = threadIdx.x; c < vol; c += 256) sub[c] = 0.0;
    __syncthreads();
  }
  if (valid) {
    const double qi = q[i];
    double wt[D][16];
    for (int a = 0; a < D; ++a)
      for (int k = 0; k < w; ++k)
        wt[a][k] = (double)es_win((Real)((i0[a] + k - g[a]) / hw), (Real)beta);
    if (tiled) {
      const int o0 = i0[0] - lo[0], o1 = i0[1] - lo[1], o2 = D == 3 ? i0[2] - lo[2] : 0;
      if (D == 3) {
        for (int k2 = 0; k2 < w; ++k2)
          for (int k1 = 0; k1 < w; ++k1) {
            const double w12 = qi * wt[1][k1] * wt[D - 1][k2];
            double* row = sub + ((o2 + k2) * ext[1] + (o1 + k1)) * ext[0] + o0;
            for (int k0 = 0; k0 < w; ++k0) atomicAdd(row + k0, w12 * wt[0][k0]);
          }
      } else {
        for (int k1 = 0; k1 < w; ++k1) {
          const double w1 = qi * wt[1][k1];
          double* row = sub + (o1 + k1) * ext[0] + o0;
          for (int k0 = 0; k0 < w; ++k0) atomicAdd(row + k0, w1 * wt[0][k0]);
        }
      }
    } else {
      int ix[D][16];
      for (int a = 0; a < D; ++a)
        for (int k = 0; k < w; ++k) {
          int id = (i0[a] + k) % Ms[a];
          ix[a][k] = id < 0 ? id + Ms[a] : id;
        }
      if (D == 3) {
        for (int k2 = 0; k2 < w; ++k2)
          for (int k1 = 0; k1 < w; ++k1) {
            const double w12 = qi * wt[1][k1] * wt[D - 1][k2];
            const int64_t row = (int64_t)M0 * (ix[1][k1] + (int64_t)M1 * ix[D - 1][k2]);
            for (int k0 = 0; k0 < w; ++k0) atomicAdd(grid + row + ix[0][k0], w12 * wt[0][k0]);
          }
      } else {
        for (int k1 = 0; k1 < w; ++k1) {
          const double w1 = qi * wt[1][k1];
          const int64_t row = (int64_t)M0 * ix[1][k1];
          for (int k0 = 0; k0 < w; ++k0) atomicAdd(grid + row + ix[0][k0], w1 * wt[0][k0]);
        }
      }
    }
  }
  if (tiled) {
    __syncthreads();
    for (int c = threadIdx.x; c < vol; c += 256) {
      const double v = sub[c];
      if (v == 0.0) continue;
      int cc[3] = {c % ext[0], (c / ext[0]) % ext[1], c / (ext[0] * ext[1])};
      int64_t gi = 0, mul = 1;
      for (int a = 0; a < D; ++a) {
        int id = (lo[a] + cc[a]) % Ms[a];
        if (id < 0) id += Ms[a];
        gi += id * mul;
        mul *= Ms[a];
      }
      atomicAdd(grid + gi, v);
    }
  }
}

// Tiled interpolation at targets in tree order: the block's subgrid is read
// into LDS once; results are added to the near-field arrays (tree order).
template <int D, class Real>
__global__ __launch_bounds__(256) void k_interp_tiled(KParams kp, int64_t n,
                                                      const double* __restrict__ x, int M0,
                                                      int M1, int M2, int w, double beta,
                                                      const double2* __restrict__ grid,
                                                      double* __restrict__ pot,
                                                      double* __restrict__ grad, int want_grad) {
  __shared__ double sub[kSubCap];
  __shared__ int lo[3], hi[3];
  const int Ms[3] = {M0, M1, M2};
  const double hw = 0.5 * w;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool valid = i < n;
  if (threadIdx.x < 3) {
    lo[threadIdx.x] = INT_MAX;
    hi[threadIdx.x] = INT_MIN;
  }
  __syncthreads();
  double g[D];
  int i0[D];
  if (valid) {
    grid_coords<D>(kp, x, n, i, Ms, g);
    for (int a = 0; a < D; ++a) {
      i0[a] = (int)ceil(g[a] - hw);
      atomicMin(&lo[a], i0[a]);
      atomicMax(&hi[a], i0[a]);
    }
  }
  __syncthreads();
  int ext[3] = {1, 1, 1};
  long long vol = 1;
  for (int a = 0; a < D; ++a) {
    ext[a] = hi[a] - lo[a] + w;
    vol *= ext[a];
  }
  const bool tiled = vol <= kSubCap;
  if (tiled) {
    for (int c = threadIdx.x; c < vol; c += 256) {
      int cc[3] = {c % ext[0], (c / ext[0]) % ext[1], c / (ext[0] * ext[1])};
      int64_t gi = 0, mul = 1;
      for (int a = 0; a < D; ++a) {
        int id = (lo[a] + cc[a]) % Ms[a];
        if (id < 0) id += Ms[a];
        gi += id * mul;
        mul *= Ms[a];
      }
      sub[c] = grid[gi].x;
    }
    __syncthreads();
  }
  if (!valid) return;
  double wt[D][16], dw[D][16];
  int ix[D][16];
  for (int a = 0; a < D; ++a)
    for (int k = 0; k < w; ++k) {
      const Real z = (Real)((i0[a] + k - g[a]) / hw);
      const Real v = es_win(z, (Real)beta);
      wt[a][k] = (double)v;
      const Real t = (Real)1 - z * z;
      dw[a][k] = (t > (Real)0) ? (double)(v * (Real)beta * (-z / sqrt(t))) * (-Ms[a] / hw) : 0.0;
      if (tiled) {
        ix[a][k] = i0[a] + k - lo[a];
      } else {
        int id = (i0[a] + k) % Ms[a];
        ix[a][k] = id < 0 ? id + Ms[a] : id;
      }
    }
  const int s0 = tiled ? ext[0] : M0;
  const int s1 = tiled ? ext[1] : M1;
  double acc = 0.0, gu[3] = {0, 0, 0};
  if (D == 3) {
    for (int k2 = 0; k2 < w; ++k2)
      for (int k1 = 0; k1 < w; ++k1) {
        const int64_t row = (int64_t)s0 * (ix[1][k1] + (int64_t)s1 * ix[D - 1][k2]);
        double a0 = 0.0, ad0 = 0.0;
        for (int k0 = 0; k0 < w; ++k0) {
          const double v = tiled ? sub[row + ix[0][k0]] : grid[row + ix[0][k0]].x;
          a0 = fma(v, wt[0][k0], a0);
          if (want_grad) ad0 = fma(v, dw[0][k0], ad0);
        }
        const double w12 = wt[1][k1] * wt[D - 1][k2];
        acc = fma(a0, w12, acc);
        if (want_grad) {
          gu[0] = fma(ad0, w12, gu[0]);
          gu[1] = fma(a0, dw[1][k1] * wt[D - 1][k2], gu[1]);
          gu[2] = fma(a0, wt[1][k1] * dw[D - 1][k2], gu[2]);
        }
      }
  } else {
    for (int k1 = 0; k1 < w; ++k1) {
      const int64_t row = (int64_t)s0 * ix[1][k1];
      double a0 = 0.0, ad0 = 0.0;
      for (int k0 = 0; k0 < w; ++k0) {
        const double v = tiled ? sub[row + ix[0][k0]] : grid[row + ix[0][k0]].x;
        a0 = fma(v, wt[0][k0], a0);
        if (want_grad) ad0 = fma(v, dw[0][k0], ad0);
      }
      acc = fma(a0, wt[1][k1], acc);
      if (want_grad) {
        gu[0] = fma(ad0, wt[1][k1], gu[0]);
        gu[1] = fma(a0, dw[1][k1], gu[1]);
      }
    }
  }
  pot[i] += acc;
  if (want_grad)
    for (int b = 0; b < D; ++b) {
      double s = 0.0;
      for (int a = 0; a <= b; ++a) s += kp.Li[a + D * b] * gu[a];
      grad[i * D + b] += s;
    }
}

__global__ void k_to_complex(int64_t n, const double* __restrict__ g, double2* __restrict__ c) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c[i] = make_double2(g[i], 0.0);
}

__global__ void k_scale(int64_t n, double2* __restrict__ c, const double* __restrict__ s) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    double v = s[i];
    c[i] = make_double2(c[i].x * v, c[i].y * v);
  }
}

// Diagonal scaling table (FP64), once per plan.
__global__ void k_farscale(KParams kp, int M0, int M1, int M2, int Mp0, int Mp1, int Mp2,
                           const double* __restrict__ wf0,
                           const double* __restrict__ wf1, const double* __restrict__ wf2,
                           const double* __restrict__ gx, const double* __restrict__ gwpsi, int nq,
                           double c, double c0, double V, double* __restrict__ out) {
  const int64_t n = (int64_t)M0 * M1 * M2;
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int d = kp.dim;
  int ii[3] = {(int)(idx % M0), (int)((idx / M0) % M1), (int)(idx / ((int64_t)M0 * M1))};
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
  if (nyq || zero) { out[idx] = 0.0; return; }
  double k2 = 0.0;
  for (int b = 0; b < d; ++b) {
    double s = 0.0;
    for (int a = 0; a < d; ++a) s += kp.Li[a + d * b] * m[a];
    s *= 2.0 * 3.14159265358979323846;
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
  PDMK_HIP(hipMalloc(&P->d_farscale, n * sizeof(double)));
  hipLaunchKernelGGL(k_farscale, dim3(nblk(n, 256)), dim3(256), 0, 0, P->kp, M[0], M[1], M[2],
                     g.fgrid_paper[0], g.fgrid_paper[1], d == 3 ? g.fgrid_paper[2] : 1, d0,
                     d1, d2, dgx, dgw, (int)ps.qx.size(), ps.c, ps.c0, g.volume, P->d_farscale);
  PDMK_HIP(hipDeviceSynchronize());
  for (void* p : tmp) (void)hipFree(p);
}

void stage_far(pdmk_plan* P, Eval& E, const double* q, bool want_grad) {
  const Geometry& g = P->g;
  const int d = g.dim;
  int M[3] = {g.fgrid[0], g.fgrid[1], d == 3 ? g.fgrid[2] : 1};
  int64_t n = (int64_t)M[0] * M[1] * M[2];
  const int w = P->mp.nufft_w;
  const double beta = P->nufft_beta;
  double* grid = E.alloc<double>(n);
  double2* cg = E.alloc<double2>(n);
  PDMK_HIP(hipMemsetAsync(grid, 0, n * sizeof(double), E.s));
  const bool f32 = P->kp.precision == PDMK_PREC_MIXED;
#define PDMK_SP(DD, R)                                                                        \
  hipLaunchKernelGGL((k_spread_tiled<DD, R>), dim3(nblk(E.n_src, 256)), dim3(256), 0, E.s, \
                     P->kp, E.n_src, E.ox, E.oq, M[0], M[1], M[2], w, beta, grid)
#define PDMK_IN(DD, R)                                                                        \
  hipLaunchKernelGGL((k_interp_tiled<DD, R>), dim3(nblk(E.n_trg, 256)), dim3(256), 0, E.s, \
                     P->kp, E.n_trg, E.tx, M[0], M[1], M[2], w, beta, cg, E.pot_sorted,     \
                     E.grad_sorted, want_grad ? 1 : 0)
  if (E.n_src > 0) {
    if (d == 3) { if (f32) PDMK_SP(3, float); else PDMK_SP(3, double); }
    else { if (f32) PDMK_SP(2, float); else PDMK_SP(2, double); }
  }
  hipLaunchKernelGGL(k_to_complex, dim3(nblk(n, 256)), dim3(256), 0, E.s, n, grid, cg);
  fft3(cg, M, d, -1, E.s);
  hipLaunchKernelGGL(k_scale, dim3(nblk(n, 256)), dim3(256), 0, E.s, n, cg, P->d_farscale);
  fft3(cg, M, d, +1, E.s);
  if (E.n_trg > 0) {
    if (d == 3) { if (f32) PDMK_IN(3, float); else PDMK_IN(3, double); }
    else { if (f32) PDMK_IN(2, float); else PDMK_IN(2, double); }
  }
#undef PDMK_SP
#undef PDMK_IN
}

}  // namespace pdmk

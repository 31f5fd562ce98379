// Plane-wave transforms of one tree level on the matrix cores.
//
// Between colleague boxes of level l the difference kernel D_l is applied in a
// plane-wave basis of period 3h_l (Section 3.5 with eq:W0hat): proxy charges on
// the p^3 Chebyshev grid of a box become outgoing plane waves by three axis
// contractions with F[j][x] = exp(-i pi j xi_x / 3) (j = -J..J, Hermitian half
// j0 >= 0 on the first axis); incoming plane waves become proxy potentials by
// the conjugate contractions.  Each contraction is a small dense product, so
// here every one is a real GEMM on 16x16x4 MFMA tiles (FP32 or FP64), with the
// complex arithmetic folded into constant real matrices built on the host:
//
//   outgoing, for a group of g slabs j0 in [j0b, j0b + g):
//     X[(ri,b)][(jj,c)]   = sum_a      TA[(ri,j0)][a]      Q[a][(b,c)]
//     Z[(jj,j1)][(ro,c)]  = sum_(ri,b) TB[(ro,j1)][(ri,b)] X[(ri,b)][(jj,c)]
//     S[(j0,j1)][2j2+ro]  = sum_(ri,c) Z[(jj,j1)][(ri,c)]  TC[(ri,c)][2j2+ro]
//   incoming (after the colleague translation into I):
//     Y[2j1+ro][(jj,c)]   = sum_(j2,ri) I[(jj,j1)][2j2+ri] TC2[2j2+ri][2c+ro]
//     W[2jj+ro][(b,c)]    = sum_(j1,ri) TB2[2b+ro][2j1+ri] Y[2j1+ri][(jj,c)]
//     Phi[a][(b,c)]      += sum_(jj,ri) TA2[a][2j0+ri]    W[2jj+ri][(b,c)]
//
// ri / ro select real and imaginary parts; TA2 carries the weight 2 of the
// slabs j0 > 0 (Hermitian half).
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"
#include "lagrange.h"

namespace pdmk {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));

// 16x16x4 MFMA: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; the
// accumulator element r of lane l is C[row(l, r)][l % 16].
template <class Real> struct Mfma;
template <> struct Mfma<float> {
  using V = f4v;
  static __device__ V op(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <> struct Mfma<double> {
  using V = d4v;
  static __device__ V op(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ int row(int l, int r) { return (l >> 4) + 4 * r; }
};

// One matrix-core step over KB k-steps of 4.  KB = 1: the 16x16x4 product
// of Mfma<Real>.  KB = 4 (FP32 data): BF16 products with FP32 accumulation.
// Every operand is split as x = hi + lo with hi = bf16(x), lo = bf16(x - hi)
// (rounded to nearest even), and a b ~ hi_a hi_b + hi_a lo_b + lo_a hi_b,
// which keeps about 16 significant bits (a single BF16 product keeps 8, too
// few at eps = 1e-3 where the plane waves carry most of the potential).
// Each is one 16x16x16 product in which lane l supplies its four k-step
// values (A and B take the same permutation of the contraction index, so the
// sum is unchanged).
typedef short s4v __attribute__((ext_vector_type(4)));
__device__ inline unsigned bf16_bits(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u & 0xffff0000u;   // the BF16 value as FP32 bits
}
template <class Real, int KB> struct KStep;
template <class Real> struct KStep<Real, 1> {
  using F = Real;
  using V = typename Mfma<Real>::V;
  static __device__ F pack(const Real* v) { return v[0]; }
  static __device__ V op(F a, F b, V c) { return Mfma<Real>::op(a, b, c); }
};
struct Bf16x2 {
  s4v hi, lo;
};
template <> struct KStep<float, 4> {
  using F = Bf16x2;
  using V = f4v;
  static __device__ F pack(const float* v) {
    F r;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const unsigned h = bf16_bits(v[j]);
      const unsigned l = bf16_bits(v[j] - __uint_as_float(h));
      r.hi[j] = (short)(h >> 16);
      r.lo[j] = (short)(l >> 16);
    }
    return r;
  }
  static __device__ V op(const F& a, const F& b, V c) {
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.lo, b.hi, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, b.lo, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.hi, b.hi, c, 0, 0, 0);
  }
};

// Compile-time shape of one (p, J) pair; contraction depths are padded to
// multiples of 4 KB (KB k-steps of 4 per matrix-core instruction).
template <int P, int J, int KB = 1>
struct PwShape {
  static constexpr int KQ = 4 * KB;
  static constexpr int N1 = 2 * J + 1;                 // modes per axis
  static constexpr int KA = (P + KQ - 1) / KQ * KQ;    // stage A depth (a)
  static constexpr int K2P = (2 * P + KQ - 1) / KQ * KQ;    // depth over (ri, axis point)
  static constexpr int K2N = (2 * N1 + KQ - 1) / KQ * KQ;   // depth over (mode, ri)
  static constexpr int T2N = (2 * N1 + 15) / 16;       // 16-tiles over 2 N1
  static constexpr int T2P = (2 * P + 15) / 16;        // 16-tiles over 2 P
  static constexpr int TP = (P + 15) / 16;             // 16-tiles over P
  static constexpr int TPP = (P * P + 15) / 16;        // 16-tiles over P^2
};

__host__ __device__ constexpr int align16(int n) { return (n + 15) & ~15; }

// Workgroups of a launch are handed to the eight XCDs round-robin.  This maps
// the i-th workgroup an XCD receives to the i-th item of that XCD's
// contiguous share of [0, n), so neighbouring boxes (consecutive in key
// order) run on the same XCD and share its L2.
__device__ inline int xcd_contiguous(int b, int n) {
  const int x = b & 7, q = n >> 3, r = n & 7;
  return x * q + min(x, r) + (b >> 3);
}

// Fills dst[0, n) from load(e) with `B` loads in flight per thread (all
// loads of a batch are issued before its LDS stores).
template <int B, class Real, class Load>
__device__ inline void lds_fill(Real* dst, int n, Load load) {
  for (int e0 = threadIdx.x; e0 < n; e0 += B * 256) {
    Real v[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int e = e0 + u * 256;
      v[u] = e < n ? load(e) : (Real)0;
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int e = e0 + u * 256;
      if (e < n) dst[e] = v[u];
    }
  }
}

template <class Real> struct Cplx;
template <> struct Cplx<float> { using T = float2; };
template <> struct Cplx<double> { using T = double2; };

// Outgoing plane waves of the non-leaf boxes of one level (one block of 4
// waves per box).  The constant operands of stages B and C stay in registers
// for a whole group; the data operands are read from LDS without bounds tests
// (padding rows/columns of the LDS matrices are zero or only reach discarded
// outputs).
template <class Real, int P, int J, int KB>
__global__ __launch_bounds__(256, sizeof(Real) == 4 ? 2 : 1) void k_pw_out_mfma(
    const Real* __restrict__ Q, const Real* __restrict__ TA, const Real* __restrict__ TB,
    const Real* __restrict__ TC, const int2* __restrict__ brow, int nball,
    Real* __restrict__ S, int G, int sX, int sZ) {
  using SH = PwShape<P, J, KB>;
  using MF = Mfma<Real>;
  using V = typename MF::V;
  using KS = KStep<Real, KB>;
  using F = typename KS::F;
  constexpr int N1 = SH::N1, PP = P * P;
  extern __shared__ __align__(16) unsigned char smraw[];
  Real* X = reinterpret_cast<Real*>(smraw);   // K2P rows x sX: rows (ri, b), cols (jj, c)
  Real* Z = X + SH::K2P * sX;                 // align16(G N1) rows x sZ: cols (ro, c)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int k = blockIdx.x;
  // zero the padding rows of X and columns of Z once (never written later)
  for (int e = threadIdx.x; e < (SH::K2P - 2 * P) * sX; e += 256) X[2 * P * sX + e] = 0;
  for (int e = threadIdx.x; e < align16(G * N1) * (SH::K2P - 2 * P); e += 256) {
    const int r = e / (SH::K2P - 2 * P), c = e - r * (SH::K2P - 2 * P);
    Z[r * sZ + 2 * P + c] = 0;
  }
  const Real* Qk = Q + (int64_t)k * P * PP;
  Real* Sk = S + (int64_t)k * nball * 2;   // compact half-ball order, re/im interleaved
  // per row (j0, j1 + J) of the mode grid: {compact index of j2 = -J, half
  // width w}; the row's ball modes are |j2| <= w (w < 0: none)
  __shared__ int2 rows[(J + 1) * N1];
  for (int e = threadIdx.x; e < (J + 1) * N1; e += 256) rows[e] = brow[e];
  for (int j0b = 0; j0b <= J; j0b += G) {
    const int g = min(G, J + 1 - j0b);
    // stage A (transposed): X^T[bc][(ri,jj)] = sum_a Q[a][bc] TA[(ri, j0b+jj)][a]
    {
      Real bfr[SH::KA / 4];
#pragma unroll
      for (int s = 0; s < SH::KA / 4; ++s) {
        const int a = 4 * s + lk;
        const int ri = li >= g, jj = li - ri * g;
        bfr[s] = (a < P && li < 2 * g) ? TA[(ri * (J + 1) + j0b + jj) * P + a] : (Real)0;
      }
      F bf[SH::KA / 4 / KB];
#pragma unroll
      for (int s = 0; s < SH::KA / 4 / KB; ++s) bf[s] = KS::pack(bfr + KB * s);
      // the proxy charges of every tile of this wave are loaded first (one
      // memory round trip per group instead of one per tile)
      constexpr int NT = (SH::TPP + 3) / 4;
      Real qv[NT][SH::KA / 4];
#pragma unroll
      for (int i = 0; i < NT; ++i) {
        const int bc = 16 * (wave + 4 * i) + li;
#pragma unroll
        for (int s = 0; s < SH::KA / 4; ++s) {
          const int a = 4 * s + lk;
          qv[i][s] = (a < P && bc < PP) ? Qk[a * PP + bc] : (Real)0;
        }
      }
#pragma unroll
      for (int i = 0; i < NT; ++i) {
        const int t = wave + 4 * i;
        if (t >= SH::TPP) break;
        V acc = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < SH::KA / 4 / KB; ++s) acc = KS::op(KS::pack(qv[i] + KB * s), bf[s], acc);
        // acc element r: row bc' = 16 t + row(lane, r), column (ri, jj) = li
        const int ri = li >= g, jj = li - ri * g;
        if (li < 2 * g)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int e = 16 * t + MF::row(lane, r);
            if (e < PP) {
              const int b = e / P, c = e - b * P;
              X[(ri * P + b) * sX + jj * P + c] = acc[r];
            }
          }
      }
    }
    __syncthreads();
    // stage B: Z[(jj,j1)][(ro,c)] = sum_(ri,b) TB[(ro,j1)][(ri,b)] X[(ri,b)][(jj,c)]
    {
      F af[SH::T2N][SH::K2P / 4 / KB];
#pragma unroll
      for (int m = 0; m < SH::T2N; ++m)
#pragma unroll
        for (int s = 0; s < SH::K2P / 4 / KB; ++s) {
          Real v[KB];
#pragma unroll
          for (int u = 0; u < KB; ++u) v[u] = TB[(16 * m + li) * SH::K2P + 4 * (KB * s + u) + lk];
          af[m][s] = KS::pack(v);
        }
      const int nt = (g * P + 15) >> 4;
      for (int t = wave; t < nt; t += 4) {
        const Real* xb = X + lk * sX + 16 * t + li;
        V acc[SH::T2N];
#pragma unroll
        for (int m = 0; m < SH::T2N; ++m) acc[m] = V{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < SH::K2P / 4 / KB; ++s) {
          Real v[KB];
#pragma unroll
          for (int u = 0; u < KB; ++u) v[u] = xb[4 * (KB * s + u) * sX];
          const F bv = KS::pack(v);
#pragma unroll
          for (int m = 0; m < SH::T2N; ++m) acc[m] = KS::op(af[m][s], bv, acc[m]);
        }
        const int e = 16 * t + li;   // column (jj, c)
        if (e < g * P) {
          const int jj = e / P, c = e - jj * P;
#pragma unroll
          for (int m = 0; m < SH::T2N; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = 16 * m + MF::row(lane, r);   // (ro, j1)
              if (row < 2 * N1) {
                const int ro = row >= N1, j1 = row - ro * N1;
                Z[(jj * N1 + j1) * sZ + ro * P + c] = acc[m][r];
              }
            }
        }
      }
    }
    __syncthreads();
    // stage C: S[(j0,j1)][2 j2 + ro] = sum_(ri,c) Z[(jj,j1)][(ri,c)] TC[(ri,c)][2 j2 + ro]
    {
      F bf[SH::T2N][SH::K2P / 4 / KB];
#pragma unroll
      for (int m = 0; m < SH::T2N; ++m)
#pragma unroll
        for (int s = 0; s < SH::K2P / 4 / KB; ++s) {
          Real v[KB];
#pragma unroll
          for (int u = 0; u < KB; ++u) v[u] = TC[(4 * (KB * s + u) + lk) * (16 * SH::T2N) + 16 * m + li];
          bf[m][s] = KS::pack(v);
        }
      const int mt = (g * N1 + 15) >> 4;
      for (int t = wave; t < mt; t += 4) {
        const Real* zr = Z + (16 * t + li) * sZ + lk;
        V acc[SH::T2N];
#pragma unroll
        for (int m = 0; m < SH::T2N; ++m) acc[m] = V{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < SH::K2P / 4 / KB; ++s) {
          Real v[KB];
#pragma unroll
          for (int u = 0; u < KB; ++u) v[u] = zr[4 * (KB * s + u)];
          const F av = KS::pack(v);
#pragma unroll
          for (int m = 0; m < SH::T2N; ++m) acc[m] = KS::op(av, bf[m][s], acc[m]);
        }
        // only the modes of the ball |j| <= J are kept
#pragma unroll
        for (int m = 0; m < SH::T2N; ++m) {
          const int col = 16 * m + li;
          if (col < 2 * N1)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = 16 * t + MF::row(lane, r);   // (jj, j1)
              if (row < g * N1) {
                const int2 rw = rows[j0b * N1 + row];
                const int j2 = (col >> 1) - J;
                if (j2 <= rw.y && -j2 <= rw.y) Sk[2 * (rw.x + (col >> 1)) + (col & 1)] = acc[m][r];
              }
            }
        }
      }
    }
    __syncthreads();
  }
}

// Colleague translation of one level (Section 3.5): for each non-leaf box T
// with targets and each mode j of the half ball,
//   I_T[j] = levfac Dhat(|j|^2) sum_C omega^{j.delta} S_C[j],   omega = exp(2 pi i / 3),
// over the colleagues C of T that have children, delta = (c_T - c_S) / h.
// One block per (chunk of kTransChunk modes, box); blocks are numbered
// chunk-major and handed to the XCDs in contiguous ranges, so the boxes that
// run together on an XCD read the same mode chunk of overlapping colleague
// sets and find it in that XCD's L2.  Expansions are in compact half-ball
// order, so lanes read consecutive modes of each colleague.
constexpr int kTransChunk = 1024;
template <class Real>
__global__ __launch_bounds__(256) void k_pw_trans(Level L, const typename Cplx<Real>::T* __restrict__ S,
                                                  const double* __restrict__ dtab,
                                                  const int* __restrict__ ball, int nball, int J,
                                                  double levfac,
                                                  typename Cplx<Real>::T* __restrict__ Iw,
                                                  unsigned long long* __restrict__ npairs) {
  using C2 = typename Cplx<Real>::T;
  __shared__ const C2* cbase[27];
  __shared__ int cdl[27];
  __shared__ unsigned long long phc[27];
  __shared__ int ncol;
  const int nn = L.nnl;
  const int idx = xcd_contiguous(blockIdx.x, gridDim.x);
  const int ch = idx / nn, k = idx - ch * nn;
  const int b = L.nl_box[k];
  if (L.tend[b] <= L.tbeg[b]) return;   // no targets below this box
  if (threadIdx.x < 64) {
    // slot sl of the 3x3x3 neighbourhood: a colleague with children?
    const int sl = threadIdx.x;
    int kc = -1;
    if (sl < 27) {
      const int c = L.coll[b * 27 + sl];
      if (c >= 0) kc = L.nlid[c];
    }
    const unsigned long long mask = __ballot(kc >= 0);
    if (kc >= 0) {
      const int pos = __popcll(mask & ((1ull << sl) - 1));
      cbase[pos] = S + (int64_t)kc * nball;
      // delta = c_T - c_S in units of h, each component taken mod 3
      cdl[pos] = ((3 - (sl % 3 - 1)) % 3) | (((3 - ((sl / 3) % 3 - 1)) % 3) << 2) |
                 (((3 - (sl / 9 - 1)) % 3) << 4);
    }
    if (sl == 0) {
      const int m = __popcll(mask);
      ncol = m;
      if (npairs && ch == 0) {
        // one of 64 slot pairs per box (one address for every box would
        // serialise the atomics at the cache); the caller folds them
        unsigned long long* sp = npairs + 2 * (k & 63);
        atomicAdd(sp, (unsigned long long)m);
        atomicAdd(sp + 1, 1ull);
      }
    }
  }
  __syncthreads();
  const int nc = ncol;
  if (threadIdx.x < 27) {
    // per class (j mod 3 on each axis): the 2-bit phase index of every colleague
    const int t = threadIdx.x, p0 = t % 3, p1 = (t / 3) % 3, p2 = t / 9;
    unsigned long long code = 0;
    for (int m = 0; m < nc; ++m) {
      const int dl = cdl[m];
      code |= (unsigned long long)((p0 * (dl & 3) + p1 * ((dl >> 2) & 3) + p2 * (dl >> 4)) % 3)
              << (2 * m);
    }
    phc[t] = code;
  }
  __syncthreads();
  const Real s3 = (Real)0.8660254037844386;   // sin(2 pi / 3)
  const int ee = min(nball, (ch + 1) * kTransChunk);
  C2* out = Iw + (int64_t)k * nball;
  for (int e = ch * kTransChunk + (int)threadIdx.x; e < ee; e += 256) {
    const int code = ball[e];   // j0 | j1i << 8 | j2i << 16
    const int j0 = code & 255, j1 = ((code >> 8) & 255) - J, j2 = (code >> 16) - J;
    const int pc = j0 % 3 + 3 * ((j1 + 3 * J) % 3) + 9 * ((j2 + 3 * J) % 3);
    const unsigned long long ph = phc[pc];
    Real ar = 0, ai = 0;
    // colleagues nine at a time: all nine loads in flight, then their sum
#pragma unroll 1
    for (int m0 = 0; m0 < nc; m0 += 9) {
      C2 v[9];
#pragma unroll
      for (int u = 0; u < 9; ++u) {
        v[u].x = 0;
        v[u].y = 0;
        if (m0 + u < nc) v[u] = cbase[m0 + u][e];
      }
#pragma unroll
      for (int u = 0; u < 9; ++u) {
        const int q = (int)(ph >> (2 * (m0 + u))) & 3;
        const Real cr = q == 0 ? (Real)1 : (Real)-0.5;
        const Real ci = q == 0 ? (Real)0 : (q == 1 ? s3 : -s3);
        ar = fma(cr, v[u].x, ar);
        ar = fma(-ci, v[u].y, ar);
        ai = fma(cr, v[u].y, ai);
        ai = fma(ci, v[u].x, ai);
      }
    }
    const Real cf = (Real)(levfac * dtab[j0 * j0 + j1 * j1 + j2 * j2]);
    C2 r;
    r.x = ar * cf;
    r.y = ai * cf;
    out[e] = r;
  }
}

// Incoming plane waves of the non-leaf boxes of one level that hold targets
// (already translated and scaled, in compact half-ball order) become the
// box's proxy potential by the three conjugate contractions (accumulated in
// registers across the slab groups).
template <class Real, int P, int J, int KB>
__global__ __launch_bounds__(256, sizeof(Real) == 4 ? 2 : 1) void k_pw_in_mfma(
    Level L, const typename Cplx<Real>::T* __restrict__ Iw, const Real* __restrict__ TA2,
    const Real* __restrict__ TB2, const Real* __restrict__ TC2, const int* __restrict__ ball,
    const int* __restrict__ ball_beg, int nball, Real* __restrict__ Phi, int G, int sI, int sY,
    int sW) {
  using SH = PwShape<P, J, KB>;
  using MF = Mfma<Real>;
  using V = typename MF::V;
  using KS = KStep<Real, KB>;
  using F = typename KS::F;
  using C2 = typename Cplx<Real>::T;
  constexpr int N1 = SH::N1, PP = P * P;
  constexpr int NACC = (SH::TPP + 3) / 4;   // Phi column tiles per wave
  extern __shared__ __align__(16) unsigned char smraw[];
  const int k = blockIdx.x;
  const int b = L.nl_box[k];
  if (L.tend[b] <= L.tbeg[b]) {
    // no targets below this box: its proxy potential is zero, written here so
    // that the output needs no clearing beforehand
    Real* out = Phi + (int64_t)k * P * PP;
    for (int e = threadIdx.x; e < P * PP; e += 256) out[e] = 0;
    return;
  }
  Real* I = reinterpret_cast<Real*>(smraw);      // align16(G N1) rows x sI: cols 2 j2 + ri
  Real* Y = I + align16(G * N1) * sI;            // K2N rows x sY: rows 2 j1 + ri, cols (jj, c)
  Real* W = Y + SH::K2N * sY;                    // align(2G, 4 KB) rows x sW: cols (b, c)
  const int wrows = (2 * G + 4 * KB - 1) / (4 * KB) * (4 * KB);
  // zero the padding: I columns >= 2 N1, Y rows >= 2 N1, all of W
  for (int e = threadIdx.x; e < align16(G * N1) * (SH::K2N - 2 * N1); e += 256) {
    const int r = e / (SH::K2N - 2 * N1), c = e - r * (SH::K2N - 2 * N1);
    I[r * sI + 2 * N1 + c] = 0;
  }
  for (int e = threadIdx.x; e < (SH::K2N - 2 * N1) * sY; e += 256) Y[2 * N1 * sY + e] = 0;
  for (int e = threadIdx.x; e < wrows * sW; e += 256) W[e] = 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  V acc[SH::TP][NACC];
#pragma unroll
  for (int m = 0; m < SH::TP; ++m)
#pragma unroll
    for (int i = 0; i < NACC; ++i) acc[m][i] = V{0, 0, 0, 0};
  const C2* Ik = Iw + (int64_t)k * nball;
  for (int j0b = 0; j0b <= J; j0b += G) {
    const int g = min(G, J + 1 - j0b);
    // the group's half-ball modes into the zeroed slab matrix
    // I[(jj,j1)][2j2+ri] (modes outside the ball stay zero)
    for (int e = threadIdx.x; e < g * N1 * 2 * N1; e += blockDim.x) {
      const int r = e / (2 * N1), c = e - r * (2 * N1);
      I[r * sI + c] = 0;
    }
    __syncthreads();
    const int eb = ball_beg[j0b], ee = ball_beg[j0b + g];
    for (int e0 = eb + (int)threadIdx.x; e0 < ee; e0 += 4 * 256) {
      C2 v[4];
      int cd[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * 256;
        cd[u] = e < ee ? ball[e] : 0;
        if (e < ee) v[u] = Ik[e];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (e0 + u * 256 < ee) {
          const int j0 = cd[u] & 255, j1i = (cd[u] >> 8) & 255, j2i = cd[u] >> 16;
          Real* dst = I + ((j0 - j0b) * N1 + j1i) * sI + 2 * j2i;
          dst[0] = v[u].x;
          dst[1] = v[u].y;
        }
    }
    __syncthreads();
    // stage C': Y[2 j1 + ro][(jj, c)] = sum_q I[(jj,j1)][q] TC2[q][2 c + ro]
    {
      F bf[SH::T2P][SH::K2N / 4 / KB];
#pragma unroll
      for (int m = 0; m < SH::T2P; ++m)
#pragma unroll
        for (int s = 0; s < SH::K2N / 4 / KB; ++s) {
          Real v[KB];
#pragma unroll
          for (int u = 0; u < KB; ++u) v[u] = TC2[(4 * (KB * s + u) + lk) * (16 * SH::T2P) + 16 * m + li];
          bf[m][s] = KS::pack(v);
        }
      const int mt = (g * N1 + 15) >> 4;
      for (int t = wave; t < mt; t += 4) {
        const Real* ir = I + (16 * t + li) * sI + lk;
        V a2[SH::T2P];
#pragma unroll
        for (int m = 0; m < SH::T2P; ++m) a2[m] = V{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < SH::K2N / 4 / KB; ++s) {
          Real v[KB];
#pragma unroll
          for (int u = 0; u < KB; ++u) v[u] = ir[4 * (KB * s + u)];
          const F av = KS::pack(v);
#pragma unroll
          for (int m = 0; m < SH::T2P; ++m) a2[m] = KS::op(av, bf[m][s], a2[m]);
        }
#pragma unroll
        for (int m = 0; m < SH::T2P; ++m) {
          const int col = 16 * m + li;   // 2 c + ro
          if (col < 2 * P)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = 16 * t + MF::row(lane, r);   // (jj, j1)
              if (row < g * N1) {
                const int jj = row / N1, j1 = row - jj * N1;
                Y[(2 * j1 + (col & 1)) * sY + jj * P + (col >> 1)] = a2[m][r];
              }
            }
        }
      }
    }
    __syncthreads();
    // stage B': W[2 jj + ro][(b, c)] = sum_q TB2[2 b + ro][q] Y[q][(jj, c)]
    {
      F af[SH::T2P][SH::K2N / 4 / KB];
#pragma unroll
      for (int m = 0; m < SH::T2P; ++m)
#pragma unroll
        for (int s = 0; s < SH::K2N / 4 / KB; ++s) {
          Real v[KB];
#pragma unroll
          for (int u = 0; u < KB; ++u) v[u] = TB2[(16 * m + li) * SH::K2N + 4 * (KB * s + u) + lk];
          af[m][s] = KS::pack(v);
        }
      const int nt = (g * P + 15) >> 4;
      for (int t = wave; t < nt; t += 4) {
        const Real* yb = Y + lk * sY + 16 * t + li;
        V a2[SH::T2P];
#pragma unroll
        for (int m = 0; m < SH::T2P; ++m) a2[m] = V{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < SH::K2N / 4 / KB; ++s) {
          Real v[KB];
#pragma unroll
          for (int u = 0; u < KB; ++u) v[u] = yb[4 * (KB * s + u) * sY];
          const F bv = KS::pack(v);
#pragma unroll
          for (int m = 0; m < SH::T2P; ++m) a2[m] = KS::op(af[m][s], bv, a2[m]);
        }
        const int e = 16 * t + li;   // (jj, c)
        if (e < g * P) {
          const int jj = e / P, c = e - jj * P;
#pragma unroll
          for (int m = 0; m < SH::T2P; ++m)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = 16 * m + MF::row(lane, r);   // 2 b + ro
              if (row < 2 * P) W[(2 * jj + (row & 1)) * sW + (row >> 1) * P + c] = a2[m][r];
            }
        }
      }
    }
    __syncthreads();
    // stage A': Phi[a][bc] += sum_q TA2[a][2 j0b + q] W[q][bc], q < 2g
    {
      Real afr[SH::TP][4];
#pragma unroll
      for (int m = 0; m < SH::TP; ++m)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int a = 16 * m + li, q = 4 * s + lk;
          afr[m][s] = (a < P && q < 2 * g) ? TA2[a * 2 * (J + 1) + 2 * j0b + q] : (Real)0;
        }
      F af[SH::TP][4 / KB];
#pragma unroll
      for (int m = 0; m < SH::TP; ++m)
#pragma unroll
        for (int s = 0; s < 4 / KB; ++s) af[m][s] = KS::pack(afr[m] + KB * s);
      // k-steps that reach a row q < 2g (W rows past 2g are zero)
      const int ks = ((2 * g + 3) >> 2) + KB - 1;
#pragma unroll
      for (int i = 0; i < NACC; ++i) {
        const int t = wave + 4 * i;
        if (t < SH::TPP) {
          const Real* wb = W + lk * sW + 16 * t + li;
#pragma unroll
          for (int s = 0; s < 4 / KB; ++s)
            if (KB * s < ks - KB + 1) {
              Real v[KB];
#pragma unroll
              for (int u = 0; u < KB; ++u) v[u] = wb[4 * (KB * s + u) * sW];
              const F bv = KS::pack(v);
#pragma unroll
              for (int m = 0; m < SH::TP; ++m) acc[m][i] = KS::op(af[m][s], bv, acc[m][i]);
            }
        }
      }
    }
    __syncthreads();
  }
  Real* out = Phi + (int64_t)k * P * PP;
#pragma unroll
  for (int i = 0; i < NACC; ++i) {
    const int t = wave + 4 * i;
    const int bc = 16 * t + li;
    if (t < SH::TPP && bc < PP)
#pragma unroll
      for (int m = 0; m < SH::TP; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = 16 * m + MF::row(lane, r);
          if (a < P) out[a * PP + bc] = acc[m][i][r];
        }
  }
}

// Leaf targets evaluate their parent's proxy potential (3D):
//   phi(x) = sum_{i0,i1,i2} Phi[i0][i1][i2] l_i0(xi_0) l_i1(xi_1) l_i2(xi_2)
// For 16 targets at a time the contraction over i2 is a product
//   T[(i0,i1)][t] = sum_i2 Phi[(i0,i1)][i2] Lz[i2][t]
// on MFMA tiles; the remaining weights l_i0 l_i1 are applied as each tile
// leaves the accumulators.  The rows (i0, i1) are ordered so that the weights
// need no index arithmetic: an "A" tile holds one i0 with i1 = 0..15, a "B"
// tile (P > 16) the pair i0 = 2j, 2j + 1 with i1 = 16..23.  A lane's
// accumulator rows then keep the same i1 in every tile (those l_i1 stay in
// registers) and each tile needs one l_i0 per row block.  Rows with i0 or
// i1 >= P are zero.  One block of 4 waves per non-leaf parent; each wave
// takes whole 16-target chunks, so the waves never wait on each other.
template <int P> struct LeafRows {
  static_assert(P > 8 && P <= 24, "row layout covers 8 < P <= 24");
  static constexpr int P1 = (P + 7) & ~7;                            // i1 padded: 16 or 24
  static constexpr int NA = (P + 1) & ~1;                            // A tiles, even
  static constexpr int NB = P1 > 16 ? ((P + 1) / 2 + 1) & ~1 : 0;    // B tiles, even
  static constexpr int MT = NA + NB;
  // (i0, i1) of row rho of tile tl; both stay below P1
  __device__ static void map(int tl, int rho, int& i0, int& i1) {
    if (tl < NA) {
      i0 = tl;
      i1 = rho;
    } else {
      i0 = 2 * (tl - NA) + (rho >> 3);
      i1 = 16 + (rho & 7);
    }
  }
};

template <class Real, int P, bool GRAD>
__global__ __launch_bounds__(256) void k_eval_leaf_mfma(
    KParams kp, Level Lp, Level Lc, int lvl, const double* __restrict__ tx, int64_t ntrg,
    const double* __restrict__ nodes, const double* __restrict__ bw, double* __restrict__ pot,
    double* __restrict__ grad) {
  using MF = Mfma<Real>;
  using V = typename MF::V;
  using LR = LeafRows<P>;
  constexpr int KA = (P + 3) & ~3, SP = KA | 1, P1 = LR::P1, SL = P1 | 1;
  constexpr int MT = LR::MT, NA = LR::NA;
  constexpr int NR = GRAD ? 2 : 1;
  extern __shared__ __align__(16) unsigned char smraw[];
  Real* PhiA = reinterpret_cast<Real*>(smraw);        // 16 MT rows x SP (i2)
  Real* wrow = PhiA + 16 * MT * SP;                     // per wave: rows of 16 targets
  __shared__ int cb[8], cpre[9];
  const int k = blockIdx.x;
  const int Pb = Lp.nl_box[k];
  const int c0 = Lp.child0[Pb];
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int o = 0; o < 8; ++o) {
      const int c = c0 + o;
      cpre[o] = acc;
      if (Lc.child0[c] < 0) {
        cb[o] = Lc.tbeg[c];
        acc += Lc.tend[c] - Lc.tbeg[c];
      } else {
        cb[o] = 0;
      }
    }
    cpre[8] = acc;
  }
  __syncthreads();
  const int total = cpre[8];
  if (total == 0) return;
  const Real* Phi = static_cast<const Real*>(Lp.proxy_phi) + (int64_t)k * P * P * P;
  lds_fill<8>(PhiA, 16 * MT * SP, [&](int e) {
    const int R = e / SP, c = e - R * SP;
    int i0, i1;
    LR::map(R >> 4, R & 15, i0, i1);
    return (i0 < P && i1 < P && c < P) ? Phi[(i0 * P + i1) * P + c] : (Real)0;
  });
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  // wave-private rows: Lx, Ly [16][SL] (zero past P), Lz as B operand [KA][16],
  // and their derivatives
  Real* Lx = wrow + wave * NR * (2 * 16 * SL + KA * 16);
  Real* Ly = Lx + 16 * SL;
  Real* Lz = Ly + 16 * SL;
  Real* dLx = Lz + KA * 16;
  Real* dLy = dLx + 16 * SL;
  Real* dLz = dLy + 16 * SL;
  const double hP = kp.rc / (double)(1 << lvl);
  const double sc = 2.0 / hP;
  // target of lane li in chunk ch, and (lanes lk < 3) its coordinate lk; the
  // next chunk's coordinate is loaded while this chunk is evaluated
  auto target = [&](int ch, bool& valid) {
    const int j = 16 * ch + li;
    valid = j < total;
    int t = 0;
    if (valid) {
      int o = 0;
      while (o < 7 && cpre[o + 1] <= j) ++o;
      t = cb[o] + (j - cpre[o]);
    }
    return t;
  };
  bool vnext = false;
  int tnext = target(wave, vnext);
  double xnext = (lk < 3 && vnext) ? tx[lk * ntrg + tnext] : 0.0;
  for (int ch = wave; 16 * ch < total; ch += 4) {
    const int t = tnext;
    const bool valid = vnext;
    const double xraw = xnext;
    if (16 * (ch + 4) < total) {
      tnext = target(ch + 4, vnext);
      xnext = (lk < 3 && vnext) ? tx[lk * ntrg + tnext] : 0.0;
    }
    // rows: lane (li, axis lk < 3) computes l_i(xi) for its target
    if (lk < 3) {
      const int a = lk;
      const double cen = kp.origin[a] + (Lp.coord[Pb * 3 + a] + 0.5) * hP;
      const double xi = valid ? (xraw - cen) * sc : 0.0;
      double rl[P], dl[P];
      lagrange_rows_reg<P, GRAD, sizeof(Real) == 4 ? 1 : 2>(P, nodes, bw, xi, rl, dl);
      // the lane's row (x, y: SL-strided rows; z: the transposed B operand)
      // chosen once, so that the writes take no branch per entry
      const int off = a == 2 ? li : li * SL, str = a == 2 ? 16 : 1;
      Real* dst = (a == 0 ? Lx : (a == 1 ? Ly : Lz)) + off;
      Real* ddst = (a == 0 ? dLx : (a == 1 ? dLy : dLz)) + off;
      const double f = valid ? 1.0 : 0.0;
#pragma unroll
      for (int i = 0; i < P; ++i) {
        dst[i * str] = (Real)(f * rl[i]);
        if (GRAD) ddst[i * str] = (Real)(f * dl[i]);
      }
      const int iend = a == 2 ? KA : P1;
      for (int i = P; i < iend; ++i) {
        dst[i * str] = 0;
        if (GRAD) ddst[i * str] = 0;
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    Real bz[KA / 4], bd[KA / 4];
#pragma unroll
    for (int s = 0; s < KA / 4; ++s) {
      bz[s] = Lz[(4 * s + lk) * 16 + li];
      bd[s] = GRAD ? dLz[(4 * s + lk) * 16 + li] : (Real)0;
    }
    // l_i1 (and derivatives) of the lane's accumulator rows: A tiles, B tiles
    Real ya[4], yb[4], dya[4], dyb[4];
    int bo[4];   // i0 offset of the row within a B tile's pair
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int rho = MF::row(lane, r);
      ya[r] = Ly[li * SL + rho];
      yb[r] = P1 > 16 ? Ly[li * SL + 16 + (rho & 7)] : (Real)0;
      dya[r] = GRAD ? dLy[li * SL + rho] : (Real)0;
      dyb[r] = (GRAD && P1 > 16) ? dLy[li * SL + 16 + (rho & 7)] : (Real)0;
      bo[r] = rho >> 3;
    }
    Real acc = 0, g0 = 0, g1 = 0, g2 = 0;
    // two row tiles per step: independent accumulator chains overlap on the
    // matrix pipe (both tiles of a step are of the same kind: NA is even)
    auto tiles = [&](int mt, V (&c)[2], V (&cd)[2]) {
      const Real* ar = PhiA + (16 * mt + li) * SP + lk;
#pragma unroll
      for (int h = 0; h < 2; ++h) c[h] = cd[h] = V{0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < KA / 4; ++s) {
        const Real a0 = ar[4 * s], a1 = ar[16 * SP + 4 * s];
        c[0] = MF::op(a0, bz[s], c[0]);
        c[1] = MF::op(a1, bz[s], c[1]);
        if (GRAD) {
          cd[0] = MF::op(a0, bd[s], cd[0]);
          cd[1] = MF::op(a1, bd[s], cd[1]);
        }
      }
    };
    // software pipeline: the next pair's products are issued before this
    // pair's weights are applied
    V c[2], cd[2];
    tiles(0, c, cd);
#pragma unroll
    for (int mt = 0; mt < MT; mt += 2) {
      V cn[2], cdn[2];
      if (mt + 2 < MT) tiles(mt + 2, cn, cdn);
      if (mt < NA) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const Real x0 = Lx[li * SL + mt + h];
          Real sy = 0, sdy = 0, sdz = 0;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            sy = fma(c[h][r], ya[r], sy);
            if (GRAD) {
              sdy = fma(c[h][r], dya[r], sdy);
              sdz = fma(cd[h][r], ya[r], sdz);
            }
          }
          acc = fma(x0, sy, acc);
          if (GRAD) {
            g0 = fma(dLx[li * SL + mt + h], sy, g0);
            g1 = fma(x0, sdy, g1);
            g2 = fma(x0, sdz, g2);
          }
        }
      } else {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int i0 = 2 * (mt + h - NA);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const Real x0 = Lx[li * SL + i0 + bo[r]];
            acc = fma(c[h][r], x0 * yb[r], acc);
            if (GRAD) {
              g0 = fma(c[h][r], dLx[li * SL + i0 + bo[r]] * yb[r], g0);
              g1 = fma(c[h][r], x0 * dyb[r], g1);
              g2 = fma(cd[h][r], x0 * yb[r], g2);
            }
          }
        }
      }
      if (mt + 2 < MT) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          c[h] = cn[h];
          cd[h] = cdn[h];
        }
      }
    }
    // lanes li, li + 16, li + 32, li + 48 hold parts of target li
    for (int m = 16; m < 64; m <<= 1) {
      acc += __shfl_xor(acc, m);
      if (GRAD) {
        g0 += __shfl_xor(g0, m);
        g1 += __shfl_xor(g1, m);
        g2 += __shfl_xor(g2, m);
      }
    }
    // one add per target in this kernel (its leaf has one parent): an atomic
    // without return keeps the wave from waiting on the old value, and the
    // result does not depend on the order
    if (valid && lk == 0) {
      atomicAdd(&pot[t], (double)acc);
      if (GRAD) {
        atomicAdd(&grad[(int64_t)t * 3 + 0], (double)g0 * sc);
        atomicAdd(&grad[(int64_t)t * 3 + 1], (double)g1 * sc);
        atomicAdd(&grad[(int64_t)t * 3 + 2], (double)g2 * sc);
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

template <class Real, int PP>
static size_t eval_leaf_lds(bool grad) {
  constexpr int KA = (PP + 3) & ~3, SP = KA | 1, SL = LeafRows<PP>::P1 | 1,
                MT = LeafRows<PP>::MT;
  const int NR = grad ? 2 : 1;
  return ((size_t)16 * MT * SP + (size_t)4 * NR * (2 * 16 * SL + KA * 16)) * sizeof(Real);
}

template <class Real, int PP>
static bool eval_leaf_launch(const pdmk_plan* P, const Level& Lp, const Level& Lc, int l,
                             const double* tx, int64_t ntrg, double* pot, double* grad,
                             hipStream_t s) {
  const size_t lds = eval_leaf_lds<Real, PP>(grad != nullptr);
  if (lds > 150 * 1024) return false;
  if (grad) {
    ensure_lds((const void*)&k_eval_leaf_mfma<Real, PP, true>, lds);
    hipLaunchKernelGGL((k_eval_leaf_mfma<Real, PP, true>), dim3(Lp.nnl), dim3(256), lds, s,
                       P->kp, Lp, Lc, l, tx, ntrg, P->d_nodes, P->d_bw, pot, grad);
  } else {
    ensure_lds((const void*)&k_eval_leaf_mfma<Real, PP, false>, lds);
    hipLaunchKernelGGL((k_eval_leaf_mfma<Real, PP, false>), dim3(Lp.nnl), dim3(256), lds, s,
                       P->kp, Lp, Lc, l, tx, ntrg, P->d_nodes, P->d_bw, pot, grad);
  }
  return true;
}

template <class Real>
bool eval_leaf_mfma(const pdmk_plan* P, const Level& Lp, const Level& Lc, int l,
                    const double* tx, int64_t ntrg, double* pot, double* grad, hipStream_t s) {
  if (P->kp.dim != 3 || !P->pw_mfma) return false;
  if (P->kp.p == 22) return eval_leaf_launch<Real, 22>(P, Lp, Lc, l, tx, ntrg, pot, grad, s);
  if (P->kp.p == 13) return eval_leaf_launch<Real, 13>(P, Lp, Lc, l, tx, ntrg, pot, grad, s);
  return false;
}

template bool eval_leaf_mfma<float>(const pdmk_plan*, const Level&, const Level&, int,
                                    const double*, int64_t, double*, double*, hipStream_t);
template bool eval_leaf_mfma<double>(const pdmk_plan*, const Level&, const Level&, int,
                                     const double*, int64_t, double*, double*, hipStream_t);

// Proxy charges of a non-leaf box from the sources of its childless children
// (3D): Q[i0][i1][i2] = sum_s q_s l_i0(xi_0) l_i1(xi_1) l_i2(xi_2), i.e. the
// product (q l_i0 l_i1)[(i0,i1)][s] x l_i2[s][i2] over the sources, on MFMA
// tiles with the sources in chunks of 64 (3 x 64 threads form a chunk's
// Lagrange rows).  One block of 4 waves per box; each wave owns the same
// M-tiles of Q for every chunk (accumulators in registers).
// MWP > 0: each block computes MWP tile slots per wave (blockIdx.y selects
// which), so that large orders keep their accumulators in registers; the
// sources are then read once per block.
template <class Real, int P, int MWP = 0>
__global__ __launch_bounds__(256, sizeof(Real) == 4 ? 3 : 1) void k_anterp_mfma(KParams kp, Level L, Level C, int lvl,
                                                     const double* __restrict__ sx,
                                                     const double* __restrict__ sq,
                                                     int64_t nimg,
                                                     const double* __restrict__ nodes,
                                                     const double* __restrict__ bw,
                                                     Real* __restrict__ Q) {
  using MF = Mfma<Real>;
  using V = typename MF::V;
  constexpr int PP = P * P, SL = P | 1, CH = 64, NT = (P + 15) / 16, NW = 16 * NT;
  constexpr int MT = (PP + 15) / 16, MW = MWP > 0 ? MWP : (MT + 3) / 4;
  const int mt0 = MWP > 0 ? (int)blockIdx.y * 4 * MWP : 0;   // first tile of the block
  __shared__ Real qLx[CH * SL], Ly[CH * SL], Lz[CH * NW];
  __shared__ int cb[8], cpre[9];
  const int k = blockIdx.x;
  const int b = L.nl_box[k];
  const int c0 = L.child0[b];
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int o = 0; o < 8; ++o) {
      const int c = c0 + o;
      cpre[o] = acc;
      if (C.child0[c] < 0) {
        cb[o] = C.sbeg[c];
        acc += C.send[c] - C.sbeg[c];
      } else {
        cb[o] = 0;
      }
    }
    cpre[8] = acc;
  }
  // B operand padding columns stay zero
  for (int e = threadIdx.x; e < CH * NW; e += 256) Lz[e] = 0;
  __syncthreads();
  const int total = cpre[8];
  const double h = kp.rc / (double)(1 << lvl);
  const double sc = 2.0 / h;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  V acc[MW][NT];
  int ri0[MW], ri1[MW];   // (i0, i1) of the lane's A-operand row in each tile slot
#pragma unroll
  for (int i = 0; i < MW; ++i) {
    const int m = min(16 * (mt0 + wave + 4 * i) + li, PP - 1);
    ri0[i] = m / P;
    ri1[i] = m - ri0[i] * P;
#pragma unroll
    for (int n = 0; n < NT; ++n) acc[i][n] = V{0, 0, 0, 0};
  }
  for (int s0 = 0; s0 < total; s0 += CH) {
    // Lagrange rows of the chunk: thread (source, axis)
    if (threadIdx.x < 3 * CH) {
      const int si = threadIdx.x / 3, a = threadIdx.x - 3 * si;
      const int j = s0 + si;
      const bool valid = j < total;
      int sidx = 0;
      if (valid) {
        int o = 0;
        while (o < 7 && cpre[o + 1] <= j) ++o;
        sidx = cb[o] + (j - cpre[o]);
      }
      const double cen = kp.origin[a] + (L.coord[b * 3 + a] + 0.5) * h;
      const double xi = valid ? (sx[a * nimg + sidx] - cen) * sc : 0.0;
      const double qs = (valid && a == 0) ? sq[sidx] : 1.0;
      double rl[P], dl[P];
      lagrange_rows_reg<P, false, sizeof(Real) == 4 ? 1 : 2>(P, nodes, bw, xi, rl, dl);
      // the thread's row and factor chosen once (no branch per entry)
      Real* dst = a == 0 ? qLx + si * SL : (a == 1 ? Ly + si * SL : Lz + si * NW);
      const double f = valid ? qs : 0.0;
#pragma unroll
      for (int i = 0; i < P; ++i) dst[i] = (Real)(f * rl[i]);
    }
    __syncthreads();
    // Every tile slot of the wave is computed (a slot past the last tile
    // yields rows m >= P^2, whose clamped indices stay inside the rows and
    // whose results are never stored).
    if constexpr (sizeof(Real) == 4) {
      // k-step outer, tile slots inner: consecutive products go to different
      // accumulators
#pragma unroll 4
      for (int st = 0; st < CH / 4; ++st) {
        const int si = 4 * st + lk;
        Real bz[NT];
#pragma unroll
        for (int n = 0; n < NT; ++n) bz[n] = Lz[si * NW + 16 * n + li];
#pragma unroll
        for (int i = 0; i < MW; ++i) {
          const Real av = qLx[si * SL + ri0[i]] * Ly[si * SL + ri1[i]];
#pragma unroll
          for (int n = 0; n < NT; ++n) acc[i][n] = MF::op(av, bz[n], acc[i][n]);
        }
      }
    } else {
      // FP64 (one wave per SIMD): the chunk's B operand in registers, tile
      // slots outer (measured faster at this occupancy)
      Real bz[CH / 4][NT];
#pragma unroll
      for (int st = 0; st < CH / 4; ++st)
#pragma unroll
        for (int n = 0; n < NT; ++n) bz[st][n] = Lz[(4 * st + lk) * NW + 16 * n + li];
#pragma unroll
      for (int i = 0; i < MW; ++i) {
#pragma unroll
        for (int st = 0; st < CH / 4; ++st) {
          const int si = 4 * st + lk;
          const Real av = qLx[si * SL + ri0[i]] * Ly[si * SL + ri1[i]];
#pragma unroll
          for (int n = 0; n < NT; ++n) acc[i][n] = MF::op(av, bz[st][n], acc[i][n]);
        }
      }
    }
    __syncthreads();
  }
  Real* out = Q + (int64_t)k * P * PP;
#pragma unroll
  for (int i = 0; i < MW; ++i) {
    const int mt = mt0 + wave + 4 * i;
    if (mt < MT)
#pragma unroll
      for (int n = 0; n < NT; ++n) {
        const int i2 = 16 * n + li;
        if (i2 < P)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int m = 16 * mt + MF::row(lane, r);
            if (m < PP) out[m * P + i2] = acc[i][n][r];
          }
      }
  }
}

// Row tiles of the proxy-charge product with compile-time (i0, i1): the
// P^2 rows (i0, i1) of Q are cut into "full" tiles (one i0, i1 = 16 b .. 16 b
// + 15) and, for the last P % 16 values of i1, "pair" tiles (i0 = 2u and
// 2u + 1 with eight i1 each, when P % 16 <= 8) or "single" tiles (one i0,
// sixteen i1, when P % 16 > 8).  Wave w of the block owns tiles w, w + 4,
// ...; with w a template parameter each tile's i0 is a constant, so the A
// operand of a k-step (source s, row i0 i1) is q_s l_i0(s) taken from a
// register row times l_i1(s), one product per tile.
template <int P>
struct AnterpTiles {
  static constexpr int A = P / 16, R = P % 16;
  static constexpr bool PAIR = R > 0 && R <= 8;
  static constexpr int NTA = P * A;
  static constexpr int NTB = R == 0 ? 0 : (PAIR ? (P + 1) / 2 : P);
  static constexpr int NTILE = NTA + NTB;
  // tiles 0 .. NDEAL - 1 are dealt to the waves round-robin (MW each); the
  // NREM others are shared: wave w takes their k-steps st = w mod 4, and the
  // four partial sums are added at the end (no wave does a tile more)
  static constexpr int MW = NTILE / 4;
  static constexpr int NDEAL = 4 * MW;
  static constexpr int NREM = NTILE - NDEAL;
  static constexpr int NT = (P + 15) / 16;     // column tiles (i2)
  // row stride of the Lagrange rows: holds index P (zero, the missing
  // partner of an odd pair) and, for single tiles, 16 (A + 1) entries
  static constexpr int SL0 = ((P + 1 + 3) / 4) * 4;
  static constexpr int SL = (R > 8 && 16 * (A + 1) > SL0) ? 16 * (A + 1) : SL0;
  // B operand row stride: the four sources of a k-step start 16 banks apart
  static constexpr int NWP = NT % 2 ? 16 * NT : 16 * NT + 16;
  static constexpr int CH = 64;                // sources per chunk
  // i0 of a tile for lanes li < 8 (lo) and li >= 8 (hi); first i1 and
  // whether i1 advances with li (full, single) or with li & 7 (pair)
  __host__ __device__ static constexpr int i0lo(int t) {
    return t < NTA ? t / A : (PAIR ? 2 * (t - NTA) : t - NTA);
  }
  __host__ __device__ static constexpr int i0hi(int t) {
    return t < NTA ? t / A : (PAIR ? 2 * (t - NTA) + 1 : t - NTA);
  }
  __host__ __device__ static constexpr int i1b(int t) { return t < NTA ? 16 * (t % A) : 16 * A; }
  __host__ __device__ static constexpr bool paired(int t) { return t >= NTA && PAIR; }
};

template <class Real, int P, int W>
__device__ __forceinline__ void anterp_rows_wave(const KParams& kp, const Level& L, int b,
                                                 int total, const int* cb, const int* cpre,
                                                 double h, const double* __restrict__ sx,
                                                 const double* __restrict__ sq, int64_t nimg,
                                                 const double* __restrict__ nodes,
                                                 const double* __restrict__ bw, Real* qLx,
                                                 Real* Ly, Real* Lz, Real* __restrict__ out) {
  using TT = AnterpTiles<P>;
  using MF = Mfma<Real>;
  using V = typename MF::V;
  constexpr int SL = TT::SL, NWP = TT::NWP, CH = TT::CH, MW = TT::MW, NT = TT::NT;
  const double sc = 2.0 / h;
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const bool hi = li >= 8;
  constexpr int NREM = TT::NREM;
  V acc[MW][NT], accr[NREM > 0 ? NREM : 1][NT];
#pragma unroll
  for (int i = 0; i < MW; ++i)
#pragma unroll
    for (int n = 0; n < NT; ++n) acc[i][n] = V{0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < (NREM > 0 ? NREM : 1); ++i)
#pragma unroll
    for (int n = 0; n < NT; ++n) accr[i][n] = V{0, 0, 0, 0};
  for (int s0 = 0; s0 < total; s0 += CH) {
    // Lagrange rows of the chunk: thread (source, axis)
    if (threadIdx.x < 3 * CH) {
      const int si = threadIdx.x / 3, a = threadIdx.x - 3 * si;
      const int j = s0 + si;
      const bool valid = j < total;
      int sidx = 0;
      if (valid) {
        int o = 0;
        while (o < 7 && cpre[o + 1] <= j) ++o;
        sidx = cb[o] + (j - cpre[o]);
      }
      const double cen = kp.origin[a] + (L.coord[b * 3 + a] + 0.5) * h;
      const double xi = valid ? (sx[a * nimg + sidx] - cen) * sc : 0.0;
      const double qs = (valid && a == 0) ? sq[sidx] : 1.0;
      double rl[P], dl[P];
      lagrange_rows_reg<P, false, sizeof(Real) == 4 ? 1 : 2>(P, nodes, bw, xi, rl, dl);
      // the thread's row and factor chosen once (no branch per entry)
      Real* dst = a == 0 ? qLx + si * SL : (a == 1 ? Ly + si * SL : Lz + si * NWP);
      const double f = valid ? qs : 0.0;
#pragma unroll
      for (int i = 0; i < P; ++i) dst[i] = (Real)(f * rl[i]);
    }
    __syncthreads();
#pragma unroll 2
    for (int st = 0; st < CH / 4; ++st) {
      const int si = 4 * st + lk;
      Real bz[NT];
#pragma unroll
      for (int n = 0; n < NT; ++n) bz[n] = Lz[si * NWP + 16 * n + li];
      // the source's row q l_i0 (every i0; broadcast within 16 lanes)
      Real qx[SL];
#pragma unroll
      for (int i = 0; i < SL; ++i) qx[i] = qLx[si * SL + i];
      Real ly[TT::A + 1];
#pragma unroll
      for (int c = 0; c < TT::A; ++c) ly[c] = Ly[si * SL + 16 * c + li];
      if constexpr (TT::R > 0) ly[TT::A] = Ly[si * SL + 16 * TT::A + (TT::PAIR ? (li & 7) : li)];
      auto tile_av = [&](int t) {
        const int c = t < TT::NTA ? t % TT::A : TT::A;
        const Real q0 = qx[TT::i0lo(t)];
        const Real qsel = TT::paired(t) ? (hi ? qx[TT::i0hi(t)] : q0) : q0;
        return qsel * ly[c];
      };
#pragma unroll
      for (int i = 0; i < MW; ++i) {
        const Real av = tile_av(W + 4 * i);
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[i][n] = MF::op(av, bz[n], acc[i][n]);
      }
      if (NREM > 0 && (st & 3) == W) {
#pragma unroll
        for (int i = 0; i < NREM; ++i) {
          const Real av = tile_av(TT::NDEAL + i);
#pragma unroll
          for (int n = 0; n < NT; ++n) accr[i][n] = MF::op(av, bz[n], accr[i][n]);
        }
      }
    }
    __syncthreads();
  }
  // shared tiles: the four waves' partial sums through LDS (the Lagrange rows
  // are no longer read), added by the wave that owns the tile's store
  Real* red = qLx;   // qLx and Ly are consecutive (one array): NREM * NT * 4 * 256 entries
  static_assert(NREM * NT * 4 * 256 <= 2 * CH * SL, "partial sums fit the row buffers");
  if constexpr (NREM > 0) {
#pragma unroll
    for (int i = 0; i < NREM; ++i)
#pragma unroll
      for (int n = 0; n < NT; ++n)
#pragma unroll
        for (int r = 0; r < 4; ++r) red[(((i * NT + n) * 4 + W) * 4 + r) * 64 + lane] = accr[i][n][r];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NREM; ++i)
      if ((i & 3) == W)
#pragma unroll
        for (int n = 0; n < NT; ++n)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            Real v = 0;
#pragma unroll
            for (int w = 0; w < 4; ++w) v += red[(((i * NT + n) * 4 + w) * 4 + r) * 64 + lane];
            accr[i][n][r] = v;
          }
  }
  auto store = [&](int t, const V* a) {
#pragma unroll
    for (int n = 0; n < NT; ++n) {
      const int i2 = 16 * n + li;
      if (i2 < P)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int rr = MF::row(lane, r);
          const int i0 = TT::paired(t) ? (rr >= 8 ? TT::i0hi(t) : TT::i0lo(t)) : TT::i0lo(t);
          const int i1 = TT::i1b(t) + (TT::paired(t) ? (rr & 7) : rr);
          if (i0 < P && i1 < P) out[(i0 * P + i1) * P + i2] = a[n][r];
        }
    }
  };
#pragma unroll
  for (int i = 0; i < MW; ++i) store(W + 4 * i, acc[i]);
#pragma unroll
  for (int i = 0; i < NREM; ++i)
    if ((i & 3) == W) store(TT::NDEAL + i, accr[i]);
}

// Proxy charges of a non-leaf box from the sources of its childless children
// (3D) on the row tiles of AnterpTiles; one block of 4 waves per box.
template <class Real, int P>
__global__ __launch_bounds__(256, sizeof(Real) == 4 ? 3 : 1) void k_anterp_rows(
    KParams kp, Level L, Level C, int lvl, const double* __restrict__ sx,
    const double* __restrict__ sq, int64_t nimg, const double* __restrict__ nodes,
    const double* __restrict__ bw, Real* __restrict__ Q) {
  using TT = AnterpTiles<P>;
  // the two row buffers in one array: the shared tiles' partial sums use both
  __shared__ Real rows[2 * TT::CH * TT::SL], Lz[TT::CH * TT::NWP];
  __shared__ int cb[8], cpre[9];
  Real* qLx = rows;
  Real* Ly = rows + TT::CH * TT::SL;
  const int k = blockIdx.x;
  const int b = L.nl_box[k];
  const int c0 = L.child0[b];
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int o = 0; o < 8; ++o) {
      const int c = c0 + o;
      cpre[o] = acc;
      if (C.child0[c] < 0) {
        cb[o] = C.sbeg[c];
        acc += C.send[c] - C.sbeg[c];
      } else {
        cb[o] = 0;
      }
    }
    cpre[8] = acc;
  }
  // padding entries (i >= P) stay zero for every chunk
  for (int e = threadIdx.x; e < TT::CH * TT::SL; e += 256) {
    qLx[e] = 0;
    Ly[e] = 0;
  }
  for (int e = threadIdx.x; e < TT::CH * TT::NWP; e += 256) Lz[e] = 0;
  __syncthreads();
  const int total = cpre[8];
  const double h = kp.rc / (double)(1 << lvl);
  Real* out = Q + (int64_t)k * P * P * P;
  switch (threadIdx.x >> 6) {
    case 0:
      anterp_rows_wave<Real, P, 0>(kp, L, b, total, cb, cpre, h, sx, sq, nimg, nodes, bw, qLx,
                                   Ly, Lz, out);
      break;
    case 1:
      anterp_rows_wave<Real, P, 1>(kp, L, b, total, cb, cpre, h, sx, sq, nimg, nodes, bw, qLx,
                                   Ly, Lz, out);
      break;
    case 2:
      anterp_rows_wave<Real, P, 2>(kp, L, b, total, cb, cpre, h, sx, sq, nimg, nodes, bw, qLx,
                                   Ly, Lz, out);
      break;
    default:
      anterp_rows_wave<Real, P, 3>(kp, L, b, total, cb, cpre, h, sx, sq, nimg, nodes, bw, qLx,
                                   Ly, Lz, out);
      break;
  }
}

template <class Real>
bool anterp_mfma(const pdmk_plan* P, const Level& L, const Level& C, int l, const double* sx,
                 const double* sq, int64_t nimg, void* Q, hipStream_t s) {
  if (P->kp.dim != 3 || !P->pw_mfma) return false;
  if (P->kp.p == 22)
    hipLaunchKernelGGL((k_anterp_rows<Real, 22>), dim3(L.nnl), dim3(256), 0, s, P->kp, L, C, l,
                       sx, sq, nimg, P->d_nodes, P->d_bw, static_cast<Real*>(Q));
  else if (P->kp.p == 13)
    hipLaunchKernelGGL((k_anterp_rows<Real, 13>), dim3(L.nnl), dim3(256), 0, s, P->kp, L, C, l,
                       sx, sq, nimg, P->d_nodes, P->d_bw, static_cast<Real*>(Q));
  else if constexpr (sizeof(Real) == 8) {
    // the orders of eps = 1e-9 and 1e-12 (FP64 only: mixed plans compute in
    // FP64 there; at p = 40 the row tiles are split over several blocks)
    if (P->kp.p == 31) {
      hipLaunchKernelGGL((k_anterp_mfma<Real, 31>), dim3(L.nnl), dim3(256), 0, s, P->kp, L, C,
                         l, sx, sq, nimg, P->d_nodes, P->d_bw, static_cast<Real*>(Q));
    } else if (P->kp.p == 40) {
      // 100 row tiles in 5 blocks of 5 tile slots per wave (all in registers)
      constexpr int MWP = 5, MT = (40 * 40 + 15) / 16;
      const int npass = (MT + 4 * MWP - 1) / (4 * MWP);
      hipLaunchKernelGGL((k_anterp_mfma<Real, 40, MWP>), dim3(L.nnl, npass), dim3(256), 0, s,
                         P->kp, L, C, l, sx, sq, nimg, P->d_nodes, P->d_bw,
                         static_cast<Real*>(Q));
    } else {
      return false;
    }
  } else {
    return false;
  }
  return true;
}

template bool anterp_mfma<float>(const pdmk_plan*, const Level&, const Level&, int,
                                 const double*, const double*, int64_t, void*, hipStream_t);
template bool anterp_mfma<double>(const pdmk_plan*, const Level&, const Level&, int,
                                  const double*, const double*, int64_t, void*, hipStream_t);

// Proxy transfer between a non-leaf child (level l+1) and its parent (level
// l): a 1D Lagrange matrix applied along each axis (up: child charges into
// the parent's, summed over siblings with atomics; down: parent potentials
// into the child's).  Each axis is one product C[o][(j,k)] = sum_i M[i][o]
// X[i][(j,k)] that contracts the slowest axis, stored with o as the fastest
// axis, so three products return to the original layout.  The first product
// reads the input from memory, the other two from one LDS buffer; each
// product's tiles stay in registers until every wave has read the buffer.
template <class Real, int P, bool UP>
__global__ __launch_bounds__(256) void k_transfer_mfma(Level Lp, Level Lc,
                                                       const Real* __restrict__ src,
                                                       Real* __restrict__ dst,
                                                       const double* __restrict__ Tm, int SB,
                                                       int oct_only) {
  using MF = Mfma<Real>;
  using V = typename MF::V;
  constexpr int PP = P * P, KA = (P + 3) & ~3, NTILE = (PP + 15) / 16, MTL = (P + 15) / 16;
  constexpr int NW = (NTILE + 3) / 4;
  extern __shared__ __align__(16) unsigned char smraw[];
  Real* buf = reinterpret_cast<Real*>(smraw);   // KA rows x SB
  const int kc = blockIdx.x;
  const int c = Lc.nl_box[kc];
  const int pb = Lc.parent[c];
  const int kpar = Lp.nlid[pb];
  const int oct = c - Lp.child0[pb];
  // fixed-order mode: one octant per launch, so a parent receives one add
  if (oct_only >= 0 && oct != oct_only) return;
  const Real* in = src + (int64_t)(UP ? kc : kpar) * P * PP;
  Real* out = dst + (int64_t)(UP ? kpar : kc) * P * PP;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  for (int e = threadIdx.x; e < (KA - P) * SB; e += 256) buf[P * SB + e] = 0;
  V acc[NW][MTL];
  for (int st = 0; st < 3; ++st) {
    // A fragments: A[o][i] = M[i][o]; up: M[i][o] = Tm[sel][o][i], down: Tm[sel][i][o]
    const int sel = (oct >> st) & 1;
    Real af[MTL][KA / 4];
#pragma unroll
    for (int m = 0; m < MTL; ++m)
#pragma unroll
      for (int q = 0; q < KA / 4; ++q) {
        const int o = 16 * m + li, i = 4 * q + lk;
        af[m][q] = (o < P && i < P)
                       ? (Real)(UP ? Tm[sel * PP + o * P + i] : Tm[sel * PP + i * P + o])
                       : (Real)0;
      }
    if (st == 0) {
      // every input value of this wave's tiles is loaded before the products
      Real bq[NW][KA / 4];
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const int n = 16 * (wave + 4 * w) + li;
#pragma unroll
        for (int q = 0; q < KA / 4; ++q) {
          const int i = 4 * q + lk;
          bq[w][q] = (i < P && n < PP) ? in[i * PP + n] : (Real)0;
        }
      }
#pragma unroll
      for (int w = 0; w < NW; ++w) {
#pragma unroll
        for (int m = 0; m < MTL; ++m) acc[w][m] = V{0, 0, 0, 0};
        if (wave + 4 * w < NTILE)
#pragma unroll
          for (int q = 0; q < KA / 4; ++q)
#pragma unroll
            for (int m = 0; m < MTL; ++m) acc[w][m] = MF::op(af[m][q], bq[w][q], acc[w][m]);
      }
    } else {
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const int t = wave + 4 * w;
#pragma unroll
        for (int m = 0; m < MTL; ++m) acc[w][m] = V{0, 0, 0, 0};
        if (t < NTILE) {
          const int n = 16 * t + li;
#pragma unroll
          for (int q = 0; q < KA / 4; ++q) {
            const Real bv = buf[(4 * q + lk) * SB + n];
#pragma unroll
            for (int m = 0; m < MTL; ++m) acc[w][m] = MF::op(af[m][q], bv, acc[w][m]);
          }
        }
      }
    }
    __syncthreads();   // every wave has read the buffer
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const int t = wave + 4 * w;
      const int n = 16 * t + li;   // (j, k)
      if (t < NTILE && n < PP) {
        const int j = n / P, kk = n - j * P;
#pragma unroll
        for (int m = 0; m < MTL; ++m)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int o = 16 * m + MF::row(lane, r);
            if (o < P) buf[j * SB + kk * P + o] = acc[w][m][r];
          }
      }
    }
    __syncthreads();
  }
  // after the third product buf holds the tensor in its natural order (row j
  // of P^2 entries at stride SB): coalesced update of the output, eight
  // entries per thread in flight
  constexpr int NE = P * PP;
  for (int e0 = threadIdx.x; e0 < NE; e0 += 8 * 256) {
    Real v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * 256;
      v[u] = 0;
      if (e < NE) {
        const int j = e / PP;
        v[u] = buf[j * SB + (e - j * PP)];
      }
    }
    if (UP) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 256;
        if (e < NE) atomicAdd(out + e, v[u]);
      }
    } else {
      Real o[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 256;
        o[u] = e < NE ? out[e] : (Real)0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * 256;
        if (e < NE) out[e] = o[u] + v[u];
      }
    }
  }
}

template <class Real, int PPP>
static void transfer_launch(const pdmk_plan* P, const Level& Lp, const Level& Lc, bool up,
                            const void* src, void* dst, bool det, hipStream_t s) {
  constexpr int KA = (PPP + 3) & ~3, PP = PPP * PPP;
  const int SB = sizeof(Real) == 4 ? ((PP + 31) & ~31) + 16 : ((PP + 15) & ~15) + 8;
  const size_t lds = (size_t)KA * SB * sizeof(Real);
  if (up) {
    ensure_lds((const void*)&k_transfer_mfma<Real, PPP, true>, lds);
    // fixed-order mode: the children add into their parents one octant at a time
    for (int o = det ? 0 : -1; o < (det ? 8 : 0); ++o)
      hipLaunchKernelGGL((k_transfer_mfma<Real, PPP, true>), dim3(Lc.nnl), dim3(256), lds, s,
                         Lp, Lc, static_cast<const Real*>(src), static_cast<Real*>(dst),
                         P->d_Tm, SB, o);
  } else {
    ensure_lds((const void*)&k_transfer_mfma<Real, PPP, false>, lds);
    hipLaunchKernelGGL((k_transfer_mfma<Real, PPP, false>), dim3(Lc.nnl), dim3(256), lds, s, Lp,
                       Lc, static_cast<const Real*>(src), static_cast<Real*>(dst), P->d_Tm, SB,
                       -1);
  }
}

// 3D proxy transfers on the matrix cores for the (p, J) pairs that have
// matrix-core plane-wave kernels (FP32 and FP64 tensors).
template <class Real>
bool transfer_mfma(const pdmk_plan* P, const Level& Lp, const Level& Lc, bool up,
                   const void* src, void* dst, bool det, hipStream_t s) {
  if (P->kp.dim != 3 || !P->pw_mfma) return false;
  if (P->kp.p == 22) transfer_launch<Real, 22>(P, Lp, Lc, up, src, dst, det, s);
  else if (P->kp.p == 13) transfer_launch<Real, 13>(P, Lp, Lc, up, src, dst, det, s);
  else return false;
  return true;
}

template bool transfer_mfma<float>(const pdmk_plan*, const Level&, const Level&, bool,
                                   const void*, void*, bool, hipStream_t);
template bool transfer_mfma<double>(const pdmk_plan*, const Level&, const Level&, bool,
                                    const void*, void*, bool, hipStream_t);

// ------------------------------------------------------------------ host
// (p, J) pairs with matrix-core kernels: the defaults at eps = 1e-3 and 1e-6.
static bool pw_mfma_supported(int p, int J) {
  return (p == 22 && J == 16) || (p == 13 && J == 9);
}

static int stride_a(int n) { return n | 1; }   // rows read across lanes: odd stride
static int stride_b(int n, size_t rs) {
  // rows read along a row (B operand): lanes 0-15 and 16-31 fall on disjoint
  // halves of the LDS banks
  return rs == 4 ? ((n + 31) & ~31) + 16 : ((n + 15) & ~15) + 8;
}

PwMfmaShape pw_mfma_shape(int p, int J, size_t rs, int kb) {
  PwMfmaShape s{};
  s.ok = pw_mfma_supported(p, J);
  if (!s.ok) return s;
  const int n = 2 * J + 1, kq = 4 * kb;
  const int k2p = (2 * p + kq - 1) / kq * kq, k2n = (2 * n + kq - 1) / kq * kq;
  // LDS budget per block: FP32 keeps two blocks per CU (80 KB); FP64 takes
  // the largest slab groups that fit one block per CU (fewer groups, so
  // fewer barriers and operand reloads; measured 7.5 -> 5.4 ms incoming,
  // 5.5 -> 4.2 ms outgoing at p = 22, J = 16)
  const size_t hard = 150 * 1024, budget = rs == 8 ? hard : 80 * 1024;
  auto out_lds = [&](int g) {
    return ((size_t)k2p * stride_b(align16(g * p), rs) +
            (size_t)align16(g * n) * stride_a(k2p)) * rs;
  };
  auto in_lds = [&](int g) {
    return ((size_t)align16(g * n) * stride_a(k2n) +
            (size_t)k2n * stride_b(align16(g * p), rs) +
            (size_t)((2 * g + kq - 1) / kq * kq) * stride_b(align16(p * p), rs)) * rs;
  };
  auto pick = [&](auto lds, int& G, size_t& bytes) {
    int gmax = 0;
    for (int g = 1; g <= J + 1 && g <= 8; ++g)
      if (lds(g) <= budget) gmax = g;
    if (gmax == 0)
      for (int g = 1; g <= J + 1 && g <= 8; ++g)
        if (lds(g) <= hard) gmax = g;
    if (gmax == 0) return false;
    const int ng = (J + 1 + gmax - 1) / gmax;
    G = (J + 1 + ng - 1) / ng;
    bytes = lds(G);
    return true;
  };
  s.ok = pick(out_lds, s.g_out, s.lds_out) && pick(in_lds, s.g_in, s.lds_in);
  if (!s.ok) return s;
  s.sX = stride_b(align16(s.g_out * p), rs);
  s.sZ = stride_a(k2p);
  s.sI = stride_a(k2n);
  s.sY = stride_b(align16(s.g_in * p), rs);
  s.sW = stride_b(align16(p * p), rs);
  return s;
}

// Real matrices of the complex contractions (layouts in the file header),
// zero-padded to the tile grid the kernels read without bounds tests.
template <class Real>
static std::vector<Real> pw_mfma_tables_t(const std::vector<double>& nodes, int p, int J,
                                          size_t off[6], int kb) {
  const int n = 2 * J + 1, kq = 4 * kb;
  const int k2p = (2 * p + kq - 1) / kq * kq, k2n = (2 * n + kq - 1) / kq * kq;
  const int r2n = 16 * ((2 * n + 15) / 16), r2p = 16 * ((2 * p + 15) / 16);
  auto Fr = [&](int j, int x) { return std::cos(-kPi * j * nodes[x] / 3.0); };
  auto Fi = [&](int j, int x) { return std::sin(-kPi * j * nodes[x] / 3.0); };
  std::vector<Real> t;
  // TA: 2(J+1) x p, rows (ri, j0)
  off[0] = t.size();
  for (int ri = 0; ri < 2; ++ri)
    for (int j0 = 0; j0 <= J; ++j0)
      for (int a = 0; a < p; ++a) t.push_back((Real)(ri ? Fi(j0, a) : Fr(j0, a)));
  // TB: r2n x k2p, rows (ro, j1), columns (ri, b): [[Fr, -Fi], [Fi, Fr]]
  off[1] = t.size();
  for (int row = 0; row < r2n; ++row)
    for (int col = 0; col < k2p; ++col) {
      double v = 0;
      if (row < 2 * n && col < 2 * p) {
        const int ro = row / n, j1 = row % n, ri = col / p, b = col % p;
        const double fr = Fr(j1 - J, b), fi = Fi(j1 - J, b);
        v = ro == ri ? fr : (ro ? fi : -fi);
      }
      t.push_back((Real)v);
    }
  // TC: k2p x r2n, rows (ri, c), columns 2 j2 + ro
  off[2] = t.size();
  for (int row = 0; row < k2p; ++row)
    for (int col = 0; col < r2n; ++col) {
      double v = 0;
      if (row < 2 * p && col < 2 * n) {
        const int ri = row / p, c = row % p, j2 = col / 2, ro = col % 2;
        const double fr = Fr(j2 - J, c), fi = Fi(j2 - J, c);
        v = ri == ro ? fr : (ri ? -fi : fi);
      }
      t.push_back((Real)v);
    }
  // TA2: p x 2(J+1), columns 2 j0 + ri, weight 2 for j0 > 0
  off[3] = t.size();
  for (int a = 0; a < p; ++a)
    for (int j0 = 0; j0 <= J; ++j0)
      for (int ri = 0; ri < 2; ++ri) {
        const double w = j0 == 0 ? 1.0 : 2.0;
        t.push_back((Real)(w * (ri ? Fi(j0, a) : Fr(j0, a))));
      }
  // TB2: r2p x k2n, rows 2 b + ro, columns 2 j1 + ri: conj(F) acting on Y
  off[4] = t.size();
  for (int row = 0; row < r2p; ++row)
    for (int col = 0; col < k2n; ++col) {
      double v = 0;
      if (row < 2 * p && col < 2 * n) {
        const int b = row / 2, ro = row % 2, j1 = col / 2, ri = col % 2;
        const double fr = Fr(j1 - J, b), fi = Fi(j1 - J, b);
        v = ro == ri ? fr : (ro ? -fi : fi);
      }
      t.push_back((Real)v);
    }
  // TC2: k2n x r2p, rows 2 j2 + ri, columns 2 c + ro: I conj(F)^T
  off[5] = t.size();
  for (int row = 0; row < k2n; ++row)
    for (int col = 0; col < r2p; ++col) {
      double v = 0;
      if (row < 2 * n && col < 2 * p) {
        const int j2 = row / 2, ri = row % 2, c = col / 2, ro = col % 2;
        const double fr = Fr(j2 - J, c), fi = Fi(j2 - J, c);
        v = ri == ro ? fr : (ri ? fi : -fi);
      }
      t.push_back((Real)v);
    }
  return t;
}

void pw_mfma_upload(pdmk_plan* P) {
  const int p = P->mp.porder, J = P->mp.npw;
  {
    // modes of the Hermitian half ball |j| <= J, slab by slab (j0 | j1 << 8 | j2 << 16
    // with j1, j2 shifted by J), followed by the J + 2 slab starts
    const int n = 2 * J + 1;
    std::vector<int> ball, beg;
    for (int j0 = 0; j0 <= J; ++j0) {
      beg.push_back((int)ball.size());
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
          const int j1 = a - J, j2 = b - J;
          if (j0 * j0 + j1 * j1 + j2 * j2 <= J * J) ball.push_back(j0 | (a << 8) | (b << 16));
        }
    }
    beg.push_back((int)ball.size());
    P->nball = (int)ball.size();
    // per row (j0, j1 + J): {compact index of the row's mode j2 = -J (may lie
    // outside the row), half width w of the row's ball modes, -1 if none}
    std::vector<int> brow((size_t)(J + 1) * n * 2, 0);
    for (size_t r = 0; r < (size_t)(J + 1) * n; ++r) brow[2 * r + 1] = -1;
    for (int e = 0; e < P->nball; ++e) {
      const int c = ball[e];
      const int j0 = c & 255, a = (c >> 8) & 255, b = c >> 16;
      const size_t r = (size_t)j0 * n + a;
      if (brow[2 * r + 1] < 0) {
        brow[2 * r] = e - b;
        brow[2 * r + 1] = J - b;
      }
    }
    ball.insert(ball.end(), beg.begin(), beg.end());
    void* d = nullptr;
    PDMK_HIP(hipMalloc(&d, ball.size() * sizeof(int)));
    PDMK_HIP(hipMemcpy(d, ball.data(), ball.size() * sizeof(int), hipMemcpyHostToDevice));
    P->d_ball = static_cast<int*>(d);
    PDMK_HIP(hipMalloc(&d, brow.size() * sizeof(int)));
    PDMK_HIP(hipMemcpy(d, brow.data(), brow.size() * sizeof(int), hipMemcpyHostToDevice));
    P->d_brow = static_cast<int2*>(d);
  }
  // the compact half-ball tables above serve every order (the colleague
  // translation of the library-GEMM path uses them too); the matrix-core
  // contraction tables only the supported (p, J)
  if (!pw_mfma_supported(p, J)) return;
  std::vector<double> nodes, bw;
  cheb_nodes(p, nodes, bw);
  {
    auto t = pw_mfma_tables_t<float>(nodes, p, J, P->pwt_off, 1);
    void* d = nullptr;
    PDMK_HIP(hipMalloc(&d, t.size() * sizeof(float)));
    PDMK_HIP(hipMemcpy(d, t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice));
    P->d_pwt_f = static_cast<float*>(d);
  }
  {
    // the same matrices padded for the BF16 products (depths multiple of 16)
    auto t = pw_mfma_tables_t<float>(nodes, p, J, P->pwt_off_b, 4);
    void* d = nullptr;
    PDMK_HIP(hipMalloc(&d, t.size() * sizeof(float)));
    PDMK_HIP(hipMemcpy(d, t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice));
    P->d_pwt_b = static_cast<float*>(d);
  }
  {
    auto t = pw_mfma_tables_t<double>(nodes, p, J, P->pwt_off, 1);
    void* d = nullptr;
    PDMK_HIP(hipMalloc(&d, t.size() * sizeof(double)));
    PDMK_HIP(hipMemcpy(d, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice));
    P->d_pwt_d = static_cast<double*>(d);
  }
}

// Colleague translation of one level in compact half-ball order (FP64), for
// the plane-wave path whose contractions run as library GEMMs.
void pw_translate(const pdmk_plan* P, const Level& L, const double2* S, double2* Iw,
                  double levfac, unsigned long long* npairs, hipStream_t s) {
  const int nn = L.nnl;
  if (nn == 0) return;
  const int nchunk = (P->nball + kTransChunk - 1) / kTransChunk;
  hipLaunchKernelGGL(k_pw_trans<double>, dim3(nchunk * nn), dim3(256), 0, s, L, S, P->d_dtab,
                     P->d_ball, P->nball, P->kp.J, levfac, Iw, npairs);
  PDMK_HIP(hipGetLastError());
}

template <class Real, int PP, int JJ, int KB>
static void pw_mfma_launch(const pdmk_plan* P, const Level& L, int nn, const void* proxy_q,
                           void* S, void* Iw, void* proxy_phi, double levfac,
                           unsigned long long* npairs, hipEvent_t ev_out, hipEvent_t ev_tr,
                           hipStream_t s) {
  using C2 = typename Cplx<Real>::T;
  const PwMfmaShape sh = pw_mfma_shape(PP, JJ, sizeof(Real), KB);
  const Real* T;
  const size_t* o;
  if constexpr (sizeof(Real) == 8) {
    T = P->d_pwt_d;
    o = P->pwt_off;
  } else {
    T = KB == 4 ? P->d_pwt_b : P->d_pwt_f;
    o = KB == 4 ? P->pwt_off_b : P->pwt_off;
  }
  ensure_lds((const void*)&k_pw_out_mfma<Real, PP, JJ, KB>, sh.lds_out);
  ensure_lds((const void*)&k_pw_in_mfma<Real, PP, JJ, KB>, sh.lds_in);
  hipLaunchKernelGGL((k_pw_out_mfma<Real, PP, JJ, KB>), dim3(nn), dim3(256), sh.lds_out, s,
                     static_cast<const Real*>(proxy_q), T + o[0], T + o[1], T + o[2], P->d_brow,
                     P->nball, static_cast<Real*>(S), sh.g_out, sh.sX, sh.sZ);
  if (ev_out) PDMK_HIP(hipEventRecord(ev_out, s));
  const int nchunk = (P->nball + kTransChunk - 1) / kTransChunk;
  hipLaunchKernelGGL(k_pw_trans<Real>, dim3(nchunk * nn), dim3(256), 0, s, L,
                     static_cast<const C2*>(S), P->d_dtab, P->d_ball, P->nball, JJ, levfac,
                     static_cast<C2*>(Iw), npairs);
  if (ev_tr) PDMK_HIP(hipEventRecord(ev_tr, s));
  hipLaunchKernelGGL((k_pw_in_mfma<Real, PP, JJ, KB>), dim3(nn), dim3(256), sh.lds_in, s, L,
                     static_cast<const C2*>(Iw), T + o[3], T + o[4], T + o[5], P->d_ball,
                     P->d_ball + P->nball, P->nball, static_cast<Real*>(proxy_phi), sh.g_in,
                     sh.sI, sh.sY, sh.sW);
}

// BF16 products with FP32 accumulation for FP32 data at eps >= 1e-3
// (PDMK_MIXED_PARTS bit 8 clears it for diagnostics).
static bool pw_use_bf16(const pdmk_plan* P, size_t rs) {
  return rs == 4 && P->o.eps >= 1e-3 && (P->mixed_parts & 8);
}

template <class Real>
void pw_mfma_level(const pdmk_plan* P, const Level& L, int nn, const void* proxy_q, void* S,
                   void* Iw, void* proxy_phi, double levfac, unsigned long long* npairs,
                   hipEvent_t ev_out, hipEvent_t ev_tr, hipStream_t s) {
  const KParams& kp = P->kp;
  const bool bf = pw_use_bf16(P, sizeof(Real));
  if (kp.p == 22 && kp.J == 16) {
    if (bf) pw_mfma_launch<Real, 22, 16, sizeof(Real) == 4 ? 4 : 1>(P, L, nn, proxy_q, S, Iw, proxy_phi, levfac, npairs, ev_out, ev_tr, s);
    else pw_mfma_launch<Real, 22, 16, 1>(P, L, nn, proxy_q, S, Iw, proxy_phi, levfac, npairs, ev_out, ev_tr, s);
  } else if (kp.p == 13 && kp.J == 9) {
    if (bf) pw_mfma_launch<Real, 13, 9, sizeof(Real) == 4 ? 4 : 1>(P, L, nn, proxy_q, S, Iw, proxy_phi, levfac, npairs, ev_out, ev_tr, s);
    else pw_mfma_launch<Real, 13, 9, 1>(P, L, nn, proxy_q, S, Iw, proxy_phi, levfac, npairs, ev_out, ev_tr, s);
  } else {
    throw Error{PDMK_ERR_UNSUPPORTED, "no matrix-core plane-wave kernel for this (p, J)"};
  }
}

template void pw_mfma_level<float>(const pdmk_plan*, const Level&, int, const void*, void*,
                                   void*, void*, double, unsigned long long*, hipEvent_t,
                                   hipEvent_t, hipStream_t);
template void pw_mfma_level<double>(const pdmk_plan*, const Level&, int, const void*, void*,
                                    void*, void*, double, unsigned long long*, hipEvent_t,
                                    hipEvent_t, hipStream_t);

}  // namespace pdmk

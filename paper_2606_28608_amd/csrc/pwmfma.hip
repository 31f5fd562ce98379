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

// C (M x N) = A (M x K) B (K x N) over 16x16 tiles dealt round-robin to the
// block's waves.  A(m, k), B(k, n) read one element; out(m, n, v) stores one.
template <class Real, class AF, class BF, class OF>
__device__ inline void tile_gemm(int M, int N, int K, AF A, BF B, OF out) {
  using MF = Mfma<Real>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int tn = (N + 15) >> 4, nt = ((M + 15) >> 4) * tn, ks = (K + 3) >> 2;
  const int li = lane & 15, lk = lane >> 4;
  for (int t = wave; t < nt; t += nw) {
    const int r0 = (t / tn) << 4, c0 = (t % tn) << 4;
    const int ar = r0 + li, bc = c0 + li;
    const bool arow = ar < M, bcol = bc < N;
    typename MF::V acc = {0, 0, 0, 0};
#pragma unroll 4
    for (int s = 0; s < ks; ++s) {
      const int k = (s << 2) + lk;
      const bool kin = k < K;
      const Real a = (arow && kin) ? A(ar, k) : (Real)0;
      const Real b = (kin && bcol) ? B(k, bc) : (Real)0;
      acc = MF::op(a, b, acc);
    }
    if (bcol)
      for (int r = 0; r < 4; ++r) {
        const int row = r0 + MF::row(lane, r);
        if (row < M) out(row, bc, acc[r]);
      }
  }
}

// Outgoing plane waves of the non-leaf boxes of one level (one block per box).
template <class Real>
__global__ __launch_bounds__(256) void k_pw_out_mfma(KParams kp, const Real* __restrict__ Q,
                                                     const Real* __restrict__ TA,
                                                     const Real* __restrict__ TB,
                                                     const Real* __restrict__ TC,
                                                     Real* __restrict__ S, int G, int sX,
                                                     int sZ) {
  extern __shared__ __align__(16) unsigned char smraw[];
  const int p = kp.p, J = kp.J, n = 2 * J + 1, p2 = p * p;
  Real* X = reinterpret_cast<Real*>(smraw);   // 2p rows x sX
  Real* Z = X + 2 * p * sX;                   // G n rows x sZ
  const int k = blockIdx.x;
  const Real* Qk = Q + (int64_t)k * p * p2;
  Real* Sk = S + (int64_t)k * (J + 1) * n * n * 2;
  for (int j0b = 0; j0b <= J; j0b += G) {
    const int g = min(G, J + 1 - j0b);
    tile_gemm<Real>(
        2 * g, p2, p,
        [&](int m, int a) {
          const int ri = m >= g, jj = m - ri * g;
          return TA[(ri * (J + 1) + j0b + jj) * p + a];
        },
        [&](int a, int e) { return Qk[a * p2 + e]; },
        [&](int m, int e, Real v) {
          const int ri = m >= g, jj = m - ri * g;
          const int b = e / p, c = e - b * p;
          X[(ri * p + b) * sX + jj * p + c] = v;
        });
    __syncthreads();
    tile_gemm<Real>(
        2 * n, g * p, 2 * p, [&](int m, int q) { return TB[m * 2 * p + q]; },
        [&](int q, int e) { return X[q * sX + e]; },
        [&](int m, int e, Real v) {
          const int ro = m >= n, j1 = m - ro * n;
          const int jj = e / p, c = e - jj * p;
          Z[(jj * n + j1) * sZ + ro * p + c] = v;
        });
    __syncthreads();
    tile_gemm<Real>(
        g * n, 2 * n, 2 * p, [&](int m, int q) { return Z[m * sZ + q]; },
        [&](int q, int e) { return TC[q * 2 * n + e]; },
        [&](int m, int e, Real v) { Sk[(int64_t)(j0b * n + m) * 2 * n + e] = v; });
    __syncthreads();
  }
}

// Incoming plane waves of the non-leaf boxes of one level that hold targets:
// translation from the colleagues that have children, scaled by the
// difference-kernel multiplier, then the three conjugate contractions into
// the box's proxy potential.  MAXT = accumulator tiles of Phi per wave.
template <class Real, int MAXT>
__global__ __launch_bounds__(256) void k_pw_in_mfma(
    KParams kp, Level L, const Real* __restrict__ S, const Real* __restrict__ TA2,
    const Real* __restrict__ TB2, const Real* __restrict__ TC2, const double* __restrict__ dtab,
    double levfac, Real* __restrict__ Phi, unsigned long long* __restrict__ npairs, int G,
    int sI, int sY, int sW) {
  using MF = Mfma<Real>;
  extern __shared__ __align__(16) unsigned char smraw[];
  __shared__ int ckc[27], cph[27][3];
  __shared__ int ncol;
  const int p = kp.p, J = kp.J, n = 2 * J + 1, p2 = p * p;
  const int k = blockIdx.x;
  const int b = L.nl_box[k];
  if (L.tend[b] <= L.tbeg[b]) return;   // no targets below this box
  Real* I = reinterpret_cast<Real*>(smraw);   // G n rows x sI   (W aliases it)
  Real* W = I;                                // 2G rows x sW
  Real* Y = I + (size_t)G * n * sI;           // 2n rows x sY
  if (threadIdx.x == 0) {
    int m = 0;
    for (int sl = 0; sl < 27; ++sl) {
      const int c = L.coll[b * 27 + sl];
      if (c < 0 || L.nlid[c] < 0) continue;
      ckc[m] = L.nlid[c];
      cph[m][0] = -(sl % 3 - 1);
      cph[m][1] = -((sl / 3) % 3 - 1);
      cph[m][2] = -(sl / 9 - 1);
      ++m;
    }
    ncol = m;
    if (npairs) atomicAdd(npairs, (unsigned long long)m);
  }
  __syncthreads();
  const int nc = ncol;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int tn = (p2 + 15) >> 4, ntile = ((p + 15) >> 4) * tn;
  typename MF::V acc[MAXT];
#pragma unroll
  for (int i = 0; i < MAXT; ++i) acc[i] = typename MF::V{0, 0, 0, 0};
  const int64_t msz = (int64_t)(J + 1) * n * n;   // complex entries per box
  const Real w3r[3] = {(Real)1, (Real)-0.5, (Real)-0.5};
  const Real w3i[3] = {(Real)0, (Real)0.8660254037844386, (Real)-0.8660254037844386};
  for (int j0b = 0; j0b <= J; j0b += G) {
    const int g = min(G, J + 1 - j0b);
    // translation: I[(jj,j1)][2j2+ri] = c(|j|^2) sum_C omega^{j.delta} S_C[j0][j1][j2]
    for (int e = threadIdx.x; e < g * n * n; e += blockDim.x) {
      const int jj = e / (n * n), r = e - jj * n * n;
      const int j1i = r / n, j2i = r - j1i * n;
      const int j0 = j0b + jj, j1 = j1i - J, j2 = j2i - J;
      const int nn = j0 * j0 + j1 * j1 + j2 * j2;
      Real ar = 0, ai = 0;
      if (nn <= J * J) {
        const int64_t off = ((int64_t)j0 * n * n + r) * 2;
        for (int m = 0; m < nc; ++m) {
          int ph = (j0 * cph[m][0] + j1 * cph[m][1] + j2 * cph[m][2]) % 3;
          if (ph < 0) ph += 3;
          const Real* v = S + (int64_t)ckc[m] * msz * 2 + off;
          const Real vr = v[0], vi = v[1];
          ar = fma(w3r[ph], vr, ar);
          ar = fma(-w3i[ph], vi, ar);
          ai = fma(w3r[ph], vi, ai);
          ai = fma(w3i[ph], vr, ai);
        }
        const Real cf = (Real)(levfac * dtab[nn]);
        ar *= cf;
        ai *= cf;
      }
      Real* dst = I + (jj * n + j1i) * sI + 2 * j2i;
      dst[0] = ar;
      dst[1] = ai;
    }
    __syncthreads();
    tile_gemm<Real>(
        g * n, 2 * p, 2 * n, [&](int m, int q) { return I[m * sI + q]; },
        [&](int q, int e) { return TC2[q * 2 * p + e]; },
        [&](int m, int e, Real v) {
          const int jj = m / n, j1 = m - jj * n;
          Y[(2 * j1 + (e & 1)) * sY + jj * p + (e >> 1)] = v;
        });
    __syncthreads();
    tile_gemm<Real>(
        2 * p, g * p, 2 * n, [&](int m, int q) { return TB2[m * 2 * n + q]; },
        [&](int q, int e) { return Y[q * sY + e]; },
        [&](int m, int e, Real v) {
          const int jj = e / p, c = e - jj * p;
          W[(2 * jj + (m & 1)) * sW + (m >> 1) * p + c] = v;
        });
    __syncthreads();
    // Phi[a][(b,c)] += sum_q TA2[a][2 j0b + q] W[q][(b,c)], accumulators in registers
    const int ks = (2 * g + 3) >> 2;
#pragma unroll
    for (int i = 0; i < MAXT; ++i) {
      const int t = wave + 4 * i;
      if (t < ntile) {
        const int ar = ((t / tn) << 4) + li, bc = ((t % tn) << 4) + li;
        for (int s = 0; s < ks; ++s) {
          const int q = (s << 2) + lk;
          const bool qin = q < 2 * g;
          const Real a = (ar < p && qin) ? TA2[ar * 2 * (J + 1) + 2 * j0b + q] : (Real)0;
          const Real bv = (qin && bc < p2) ? W[q * sW + bc] : (Real)0;
          acc[i] = MF::op(a, bv, acc[i]);
        }
      }
    }
    __syncthreads();
  }
  Real* out = Phi + (int64_t)k * p * p2;
#pragma unroll
  for (int i = 0; i < MAXT; ++i) {
    const int t = wave + 4 * i;
    if (t < ntile) {
      const int bc = ((t % tn) << 4) + li;
      if (bc < p2)
        for (int r = 0; r < 4; ++r) {
          const int row = ((t / tn) << 4) + MF::row(lane, r);
          if (row < p) out[row * p2 + bc] += acc[i][r];
        }
    }
  }
}

// ------------------------------------------------------------------ host
static int stride_b(int n, size_t rs) {
  // row stride of a matrix read along rows (B operand): lanes 0-15 and 16-31
  // then fall on disjoint halves of the 32 LDS banks
  return rs == 4 ? ((n + 31) & ~31) + 16 : ((n + 15) & ~15) + 8;
}

PwMfmaShape pw_mfma_shape(int p, int J, size_t rs) {
  PwMfmaShape s{};
  const int n = 2 * J + 1;
  const int tiles = ((p + 15) / 16) * ((p * p + 15) / 16);
  s.ok = tiles <= 4 * kPwMaxTiles;
  if (!s.ok) return s;
  const size_t budget = 80 * 1024, hard = 150 * 1024;
  auto out_lds = [&](int g) {
    return ((size_t)2 * p * stride_b(g * p, rs) + (size_t)g * n * (2 * p + 1)) * rs;
  };
  auto in_lds = [&](int g) {
    const size_t iw = std::max((size_t)g * n * (2 * n + 1),
                               (size_t)2 * g * stride_b(p * p, rs));
    return (iw + (size_t)2 * n * stride_b(g * p, rs)) * rs;
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
  s.sX = stride_b(s.g_out * p, rs);
  s.sZ = 2 * p + 1;
  s.sI = 2 * n + 1;
  s.sY = stride_b(s.g_in * p, rs);
  s.sW = stride_b(p * p, rs);
  return s;
}

// Real matrices of the complex contractions (layouts in the file header).
template <class Real>
static std::vector<Real> pw_mfma_tables_t(const std::vector<double>& nodes, int p, int J,
                                          size_t off[6]) {
  const int n = 2 * J + 1;
  auto Fr = [&](int j, int x) { return std::cos(-kPi * j * nodes[x] / 3.0); };
  auto Fi = [&](int j, int x) { return std::sin(-kPi * j * nodes[x] / 3.0); };
  std::vector<Real> t;
  // TA: 2(J+1) x p
  off[0] = t.size();
  for (int ri = 0; ri < 2; ++ri)
    for (int j0 = 0; j0 <= J; ++j0)
      for (int a = 0; a < p; ++a) t.push_back((Real)(ri ? Fi(j0, a) : Fr(j0, a)));
  // TB: 2n x 2p, [[Fr, -Fi], [Fi, Fr]]
  off[1] = t.size();
  for (int ro = 0; ro < 2; ++ro)
    for (int j1 = 0; j1 < n; ++j1)
      for (int ri = 0; ri < 2; ++ri)
        for (int b = 0; b < p; ++b) {
          const double fr = Fr(j1 - J, b), fi = Fi(j1 - J, b);
          t.push_back((Real)(ro == ri ? fr : (ro ? fi : -fi)));
        }
  // TC: 2p x 2n, rows (ri, c), columns 2 j2 + ro
  off[2] = t.size();
  for (int ri = 0; ri < 2; ++ri)
    for (int c = 0; c < p; ++c)
      for (int j2 = 0; j2 < n; ++j2)
        for (int ro = 0; ro < 2; ++ro) {
          const double fr = Fr(j2 - J, c), fi = Fi(j2 - J, c);
          t.push_back((Real)(ri == ro ? fr : (ri ? -fi : fi)));
        }
  // TA2: p x 2(J+1), columns 2 j0 + ri, weight 2 for j0 > 0
  off[3] = t.size();
  for (int a = 0; a < p; ++a)
    for (int j0 = 0; j0 <= J; ++j0)
      for (int ri = 0; ri < 2; ++ri) {
        const double w = j0 == 0 ? 1.0 : 2.0;
        t.push_back((Real)(w * (ri ? Fi(j0, a) : Fr(j0, a))));
      }
  // TB2: 2p x 2n, rows 2 b + ro, columns 2 j1 + ri: conj(F) acting on Y
  off[4] = t.size();
  for (int b = 0; b < p; ++b)
    for (int ro = 0; ro < 2; ++ro)
      for (int j1 = 0; j1 < n; ++j1)
        for (int ri = 0; ri < 2; ++ri) {
          const double fr = Fr(j1 - J, b), fi = Fi(j1 - J, b);
          t.push_back((Real)(ro == ri ? fr : (ro ? -fi : fi)));
        }
  // TC2: 2n x 2p, rows 2 j2 + ri, columns 2 c + ro: I conj(F)^T
  off[5] = t.size();
  for (int j2 = 0; j2 < n; ++j2)
    for (int ri = 0; ri < 2; ++ri)
      for (int c = 0; c < p; ++c)
        for (int ro = 0; ro < 2; ++ro) {
          const double fr = Fr(j2 - J, c), fi = Fi(j2 - J, c);
          t.push_back((Real)(ri == ro ? fr : (ri ? fi : -fi)));
        }
  return t;
}

void pw_mfma_upload(pdmk_plan* P) {
  const int p = P->mp.porder, J = P->mp.npw;
  std::vector<double> nodes, bw;
  cheb_nodes(p, nodes, bw);
  {
    auto t = pw_mfma_tables_t<float>(nodes, p, J, P->pwt_off);
    void* d = nullptr;
    PDMK_HIP(hipMalloc(&d, t.size() * sizeof(float)));
    PDMK_HIP(hipMemcpy(d, t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice));
    P->d_pwt_f = static_cast<float*>(d);
  }
  {
    auto t = pw_mfma_tables_t<double>(nodes, p, J, P->pwt_off);
    void* d = nullptr;
    PDMK_HIP(hipMalloc(&d, t.size() * sizeof(double)));
    PDMK_HIP(hipMemcpy(d, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice));
    P->d_pwt_d = static_cast<double*>(d);
  }
}

template <class Real>
static const Real* pw_tables(const pdmk_plan* P);
template <>
const float* pw_tables<float>(const pdmk_plan* P) { return P->d_pwt_f; }
template <>
const double* pw_tables<double>(const pdmk_plan* P) { return P->d_pwt_d; }

template <class Real>
void pw_mfma_level(const pdmk_plan* P, const Level& L, int nn, const void* proxy_q, void* S,
                   void* proxy_phi, double levfac, unsigned long long* npairs, hipStream_t s) {
  const KParams& kp = P->kp;
  const PwMfmaShape sh = pw_mfma_shape(kp.p, kp.J, sizeof(Real));
  const Real* T = pw_tables<Real>(P);
  const size_t* o = P->pwt_off;
  PDMK_HIP(hipFuncSetAttribute((const void*)&k_pw_out_mfma<Real>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds_out));
  PDMK_HIP(hipFuncSetAttribute((const void*)&k_pw_in_mfma<Real, kPwMaxTiles>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds_in));
  hipLaunchKernelGGL(k_pw_out_mfma<Real>, dim3(nn), dim3(256), sh.lds_out, s, kp,
                     static_cast<const Real*>(proxy_q), T + o[0], T + o[1], T + o[2],
                     static_cast<Real*>(S), sh.g_out, sh.sX, sh.sZ);
  hipLaunchKernelGGL((k_pw_in_mfma<Real, kPwMaxTiles>), dim3(nn), dim3(256), sh.lds_in, s, kp,
                     L, static_cast<const Real*>(S), T + o[3], T + o[4], T + o[5], P->d_dtab,
                     levfac, static_cast<Real*>(proxy_phi), npairs, sh.g_in, sh.sI, sh.sY,
                     sh.sW);
}

template void pw_mfma_level<float>(const pdmk_plan*, const Level&, int, const void*, void*, void*,
                                   double, unsigned long long*, hipStream_t);
template void pw_mfma_level<double>(const pdmk_plan*, const Level&, int, const void*, void*,
                                    void*, double, unsigned long long*, hipStream_t);

}  // namespace pdmk

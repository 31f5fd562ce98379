// Preprocessing and tree construction (Algorithm 1, preprocessing and tree
// construction steps):
//   - orientation x' = Q^T x and wrap into the cell in FP64 (Section 3.2,
//     fractional coordinates eq:fractional_coords),
//   - image sources of the extended root grid (Sections 3.3-3.4),
//   - keys = root cube index + Morton code inside the cube, radix sort,
//   - level-synchronous adaptive refinement of every box holding more than
//     n_s sources, colleague lists (boxes at the same level sharing a
//     boundary point, bounded by the rectangular root grid),
//   - the residual interaction lists of the target leaves.
#include <cstring>
#include <rocprim/rocprim.hpp>

#include "internal.h"

namespace pdmk {

void exclusive_scan_int(const int* in, int* out, int n, Eval& E) {
  if (n <= 0) return;
  size_t tb = 0;
  PDMK_HIP(rocprim::exclusive_scan(nullptr, tb, in, out, 0, (size_t)n,
                                   rocprim::plus<int>(), E.s));
  void* tmp = E.alloc<char>(tb);
  PDMK_HIP(rocprim::exclusive_scan(tmp, tb, in, out, 0, (size_t)n,
                                   rocprim::plus<int>(), E.s));
}

int read_int(const int* dptr, hipStream_t s) {
  int v = 0;
  PDMK_HIP(hipMemcpyAsync(&v, dptr, sizeof(int), hipMemcpyDeviceToHost, s));
  PDMK_HIP(hipStreamSynchronize(s));
  return v;
}

static inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }

// ------------------------------------------------------------- orientation
// x' = Q^T x ; u = L^{-1} x' wrapped to [0,1) ; x' = L u  (FP64)
// theta (Bloch conditions only, else null): beta.(wrapped - given) = beta.L w
// for the lattice vector L w that wraps the point (the phase its charge, or
// its value as a target, carries across the wrap).
__global__ void k_prepare(KParams kp, int64_t n, const double* __restrict__ xin,
                          double* __restrict__ xo, double* __restrict__ uo,
                          int* __restrict__ bad, double* __restrict__ theta) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int d = kp.dim;
  double x[3] = {0, 0, 0}, xr[3] = {0, 0, 0}, u[3] = {0, 0, 0};
  bool ok = true;
  for (int a = 0; a < d; ++a) {
    x[a] = xin[i * d + a];
    ok = ok && isfinite(x[a]);
  }
  if (!ok) {
    atomicOr(bad, 1);
    for (int a = 0; a < d; ++a) x[a] = 0.0;
  }
  for (int a = 0; a < d; ++a) {
    double s = 0;
    for (int b = 0; b < d; ++b) s += kp.Q[b + d * a] * x[b];
    xr[a] = s;
  }
  for (int a = 0; a < d; ++a) {
    double s = 0;
    for (int b = 0; b < d; ++b) s += kp.Li[a + d * b] * xr[b];
    s -= floor(s);
    if (s >= 1.0 || s < 0.0) s = 0.0;
    u[a] = s;
  }
  double th = 0.0;
  for (int a = 0; a < d; ++a) {
    double s = 0;
    for (int b = a; b < d; ++b) s += kp.L[a + d * b] * u[b];
    xo[a * n + i] = s;
    uo[a * n + i] = u[a];
    th += kp.beta[a] * (s - xr[a]);
  }
  if (theta) theta[i] = th;
}

// Wrapped Bloch charges q e^{i theta} (real and imaginary parts).
__global__ void k_bloch_charges(int64_t n, const double* __restrict__ q,
                                const double* __restrict__ theta, double* __restrict__ qr,
                                double* __restrict__ qi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double sn, cs;
  sincos(theta[i], &sn, &cs);
  qr[i] = q[i] * cs;
  qi[i] = q[i] * sn;
}

// ------------------------------------------------------------------ images
__device__ inline bool in_extended(const KParams& kp, const double* y) {
  for (int a = 0; a < kp.dim; ++a) {
    double t = (y[a] - kp.origin[a]) / kp.rc;
    if (!(t >= 0.0 && t < (double)kp.next[a])) return false;
  }
  return true;
}

// Images y = x + L n of one point inside the extended domain (Section 3.4).
// L is upper triangular after orientation, so the admissible n_d follows from
// the last coordinate alone, then n_{d-1} given n_d, and so on: each axis is
// scanned over the range its bounds allow (one extra candidate on each side;
// the per-axis tests only prune), and every candidate that survives is
// decided by in_extended on the full image.  The shift vector is summed in
// the same order as the host shift table.
template <class F>
__device__ inline void for_each_image(const KParams& kp, const double* x, F f) {
  const int d = kp.dim;
  const double* L = kp.L;
  double lo[3], hi[3];
  for (int a = 0; a < d; ++a) {
    lo[a] = kp.origin[a];
    hi[a] = kp.origin[a] + kp.next[a] * kp.rc;
  }
  const double tol = 1e-9 * kp.rc;
  auto range = [&](double base, double lo_, double hi_, double Lii, int& nlo, int& nhi) {
    nlo = (int)floor((lo_ - base) / Lii) - 1;
    nhi = (int)ceil((hi_ - base) / Lii) + 1;
  };
  auto ok = [&](double v, int a) { return v >= lo[a] - tol && v < hi[a] + tol; };
  if (d == 3) {
    int a3, b3;
    range(x[2], lo[2], hi[2], L[8], a3, b3);
    for (int n3 = a3; n3 <= b3; ++n3) {
      if (!ok(x[2] + L[8] * n3, 2)) continue;
      int a2, b2;
      range(x[1] + L[7] * n3, lo[1], hi[1], L[4], a2, b2);
      for (int n2 = a2; n2 <= b2; ++n2) {
        if (!ok(x[1] + (L[4] * n2 + L[7] * n3), 1)) continue;
        int a1, b1;
        range(x[0] + (L[3] * n2 + L[6] * n3), lo[0], hi[0], L[0], a1, b1);
        for (int n1 = a1; n1 <= b1; ++n1) {
          double y[3];
          y[0] = x[0] + __dadd_rn(__dadd_rn(__dmul_rn(L[0], n1), __dmul_rn(L[3], n2)),
                                  __dmul_rn(L[6], n3));
          y[1] = x[1] + __dadd_rn(__dadd_rn(__dmul_rn(L[1], n1), __dmul_rn(L[4], n2)),
                                  __dmul_rn(L[7], n3));
          y[2] = x[2] + __dadd_rn(__dadd_rn(__dmul_rn(L[2], n1), __dmul_rn(L[5], n2)),
                                  __dmul_rn(L[8], n3));
          if (in_extended(kp, y)) f(y);
        }
      }
    }
  } else {
    int a2, b2;
    range(x[1], lo[1], hi[1], L[3], a2, b2);
    for (int n2 = a2; n2 <= b2; ++n2) {
      if (!ok(x[1] + L[3] * n2, 1)) continue;
      int a1, b1;
      range(x[0] + L[2] * n2, lo[0], hi[0], L[0], a1, b1);
      for (int n1 = a1; n1 <= b1; ++n1) {
        double y[3] = {0, 0, 0};
        y[0] = x[0] + __dadd_rn(__dmul_rn(L[0], n1), __dmul_rn(L[2], n2));
        y[1] = x[1] + __dadd_rn(__dmul_rn(L[1], n1), __dmul_rn(L[3], n2));
        if (in_extended(kp, y)) f(y);
      }
    }
  }
}

// Images per source; also their total in 64 bits (total64), so that a count
// past the int32 range of the offsets and tree indices is detected before the
// offsets are used.  Grid-stride over a bounded grid: one atomic per block on
// the one total (tens of thousands of them would serialise at the cache).
__global__ __launch_bounds__(256) void k_img_count(KParams kp, int64_t n,
                                                   const double* __restrict__ xs,
                                                   int* __restrict__ cnt, int* __restrict__ missing,
                                                   unsigned long long* __restrict__ total64) {
  __shared__ unsigned long long part[256];
  unsigned long long mine = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int d = kp.dim;
    double x[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) x[a] = xs[a * n + i];
    int c = 0;
    bool orig = false;
    if (kp.vimg) {
      // virtual images: the original alone
      c = 1;
      orig = true;
    } else {
      for_each_image(kp, x, [&](const double* y) {
        ++c;
        orig = orig || (y[0] == x[0] && y[1] == x[1] && y[2] == x[2]);
      });
    }
    cnt[i] = c;
    mine += (unsigned long long)c;
    if (!orig) atomicAdd(missing, 1);   // the unshifted copy was not emitted
  }
  part[threadIdx.x] = mine;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) part[threadIdx.x] += part[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(total64, part[0]);
}

// Images of source i at off[i]...; isrc[o] = i for the unshifted copy, -1
// for the shifted ones; iall[o] = i for every image (when iall is given).
// Bloch conditions (qim, qi_im not null): the source's charge q + i qim and
// its image at y = x + L n carries (q + i qim) e^{i beta.L n} (Section 4.1).
__global__ void k_img_emit(KParams kp, int64_t n, const double* __restrict__ xs,
                           const double* __restrict__ q, const int* __restrict__ off,
                           int64_t nimg, double4* __restrict__ xq,
                           int* __restrict__ isrc, int* __restrict__ iall,
                           const double* __restrict__ qim, double* __restrict__ qi_im) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int d = kp.dim;
  double x[3] = {0, 0, 0};
  for (int a = 0; a < d; ++a) x[a] = xs[a * n + i];
  const double qq = q[i];
  const double qm = qim ? qim[i] : 0.0;
  int64_t o = off[i];
  if (kp.vimg) {
    // virtual images: the original alone, whatever rounding did to its
    // distance from the cell's far faces
    xq[o] = make_double4(x[0], x[1], x[2], qq);
    isrc[o] = (int)i;
    if (iall) iall[o] = (int)i;
    return;
  }
  for_each_image(kp, x, [&](const double* y) {
    double qo = qq;
    if (qi_im) {
      double ph = 0.0;
      for (int a = 0; a < d; ++a) ph += kp.beta[a] * (y[a] - x[a]);
      double sn, cs;
      sincos(ph, &sn, &cs);
      qo = qq * cs - qm * sn;
      qi_im[o] = qq * sn + qm * cs;
    }
    xq[o] = make_double4(y[0], y[1], d == 3 ? y[2] : 0.0, qo);
    isrc[o] = (y[0] == x[0] && y[1] == x[1] && y[2] == x[2]) ? (int)i : -1;
    if (iall) iall[o] = (int)i;
    ++o;
  });
}

// Targets that are the sources: the sorted targets are the unshifted copies
// in the sorted images (equal coordinates give equal keys, and the stable
// radix sort keeps both in source-index order among equal keys).
// osrc[p]: source index of sorted image p if it is an unshifted copy, else -1
// (read in sorted order by the pick below).
__global__ void k_orig_flag(int64_t nimg, const int* __restrict__ perm,
                            const int* __restrict__ isrc, int* __restrict__ flag,
                            int* __restrict__ osrc) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nimg) return;
  const int s = isrc[perm[p]];
  osrc[p] = s;
  flag[p] = s >= 0 ? 1 : 0;
}
// Also the charges of the sorted originals (oq) from the sorted image charges,
// and itrg[p]: the sorted target that sorted image p is (-1: a shifted copy).
__global__ void k_orig_pick(int64_t nimg, int64_t n, int d, const int* __restrict__ osrc,
                            const int* __restrict__ pos, const uint64_t* __restrict__ skey,
                            const double* __restrict__ sx, const double* __restrict__ sq,
                            uint64_t* __restrict__ tkey, double* __restrict__ tx,
                            int* __restrict__ tperm, double* __restrict__ oq,
                            const double* __restrict__ sq_im, double* __restrict__ oq_im,
                            int* __restrict__ itrg) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nimg) return;
  const int src = osrc[p];
  itrg[p] = src >= 0 ? pos[p] : -1;
  if (src < 0) return;
  const int t = pos[p];
  tperm[t] = src;
  tkey[t] = skey[p];
  oq[t] = sq[p];
  if (oq_im) oq_im[t] = sq_im[p];
  for (int a = 0; a < d; ++a) tx[a * n + t] = sx[a * nimg + p];
}

// -------------------------------------------------------------------- keys
__device__ inline uint64_t morton_interleave(const uint32_t* c, int d, int B) {
  uint64_t k = 0;
  for (int b = 0; b < B; ++b)
    for (int a = 0; a < d; ++a) k |= (uint64_t)((c[a] >> b) & 1u) << (d * b + a);
  return k;
}

// Coordinate a of point i is x[a * sa + i * si]: (n, 1) for separate
// coordinate arrays, (1, 4) for packed (x, y, z, q) records.
__global__ void k_keys(KParams kp, int64_t n, const double* __restrict__ x, int64_t sa, int si,
                       uint64_t* __restrict__ key, int* __restrict__ idx) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int d = kp.dim;
  const double scale = (double)(1ull << kp.B);
  uint32_t c[3] = {0, 0, 0};
  int r[3] = {0, 0, 0};
  for (int a = 0; a < d; ++a) {
    double t = (x[a * sa + i * si] - kp.origin[a]) / kp.rc;
    int ra = (int)floor(t);
    ra = ra < 0 ? 0 : (ra >= kp.next[a] ? kp.next[a] - 1 : ra);
    double f = (t - ra) * scale;
    long long qa = (long long)floor(f);
    if (qa < 0) qa = 0;
    if (qa >= (1ll << kp.B)) qa = (1ll << kp.B) - 1;
    c[a] = (uint32_t)qa;
    r[a] = ra;
  }
  uint64_t root = (uint64_t)r[0] + (uint64_t)kp.next[0] * ((uint64_t)r[1] + (uint64_t)kp.next[1] * (uint64_t)r[2]);
  key[i] = (root << (d * kp.B)) | morton_interleave(c, d, kp.B);
  idx[i] = (int)i;
}

// out[i] = in[perm[i]] (int)
__global__ void k_gather_int(int64_t n, const int* __restrict__ perm, const int* __restrict__ in,
                             int* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[perm[i]];
}

__global__ void k_gather(int64_t n, int d, const int* __restrict__ perm,
                         const double* __restrict__ xin, int64_t nin,
                         const double* __restrict__ qin, double* __restrict__ xout,
                         double* __restrict__ qout) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int j = perm[i];
  for (int a = 0; a < d; ++a) xout[a * n + i] = xin[a * nin + j];
  if (qout) qout[i] = qin[j];
}

// Sorted images from packed (x, y, z, q) records: one 32-byte read per point
// at its random source index, where separate arrays cost a scattered line
// per coordinate and for the charge.
__global__ void k_gather_packed(int64_t n, int d, const int* __restrict__ perm,
                                const double4* __restrict__ xq, double* __restrict__ xout,
                                double* __restrict__ qout) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double4 v = xq[perm[i]];
  xout[i] = v.x;
  xout[n + i] = v.y;
  if (d == 3) xout[2 * n + i] = v.z;
  qout[i] = v.w;
}

// Sorts n points by key.  Either x_in (dim * n, separate coordinate arrays)
// with optional charges q_in, or packed (x, y, z, q) records xq_in.
static void sort_points(pdmk_plan* P, Eval& E, int64_t n, const double* x_in,
                        const double* q_in, uint64_t*& key_sorted, double*& x_sorted,
                        double*& q_sorted, int*& perm, const double4* xq_in = nullptr) {
  const KParams& kp = P->kp;
  hipStream_t s = E.s;
  uint64_t* k0 = E.alloc<uint64_t>(n);
  int* i0 = E.alloc<int>(n);
  key_sorted = E.alloc<uint64_t>(n);
  perm = E.alloc<int>(n);
  if (n > 0) {
    if (xq_in)
      hipLaunchKernelGGL(k_keys, dim3(nblk(n, 256)), dim3(256), 0, s, kp, n,
                         (const double*)xq_in, (int64_t)1, 4, k0, i0);
    else
      hipLaunchKernelGGL(k_keys, dim3(nblk(n, 256)), dim3(256), 0, s, kp, n, x_in, n, 1, k0,
                         i0);
    int rootbits = 1;
    int64_t nroot = (int64_t)kp.next[0] * kp.next[1] * (kp.dim == 3 ? kp.next[2] : 1);
    while ((1ll << rootbits) < nroot) ++rootbits;
    unsigned end_bit = (unsigned)(rootbits + kp.dim * kp.B);
    if (end_bit > 64) end_bit = 64;
    size_t tb = 0;
    PDMK_HIP(rocprim::radix_sort_pairs(nullptr, tb, k0, key_sorted, i0, perm, (size_t)n, 0u,
                                       end_bit, s));
    void* tmp = E.alloc<char>(tb);
    PDMK_HIP(rocprim::radix_sort_pairs(tmp, tb, k0, key_sorted, i0, perm, (size_t)n, 0u,
                                       end_bit, s));
  }
  x_sorted = E.alloc<double>(n * kp.dim);
  q_sorted = (q_in || xq_in) ? E.alloc<double>(n) : nullptr;
  if (n > 0 && xq_in)
    hipLaunchKernelGGL(k_gather_packed, dim3(nblk(n, 256)), dim3(256), 0, s, n, kp.dim, perm,
                       xq_in, x_sorted, q_sorted);
  else if (n > 0)
    hipLaunchKernelGGL(k_gather, dim3(nblk(n, 256)), dim3(256), 0, s, n, kp.dim, perm, x_in, n,
                       q_in, x_sorted, q_sorted);
}

// Orientation and wrap.  Non-finite coordinates are replaced by 0 and flagged
// in E.d_flags[1] (read by the caller once the call's stream has finished),
// so every later index stays valid.
void stage_prepare(pdmk_plan* P, Eval& E, const double* src, const double* trg) {
  const KParams& kp = P->kp;
  int* bad = E.d_flags + 1;
  E.xs = E.alloc<double>(E.n_src * kp.dim);
  E.us = E.alloc<double>(E.n_src * kp.dim);
  if (kp.bloch) E.theta_s = E.alloc<double>(E.n_src);
  if (E.n_src > 0)
    hipLaunchKernelGGL(k_prepare, dim3(nblk(E.n_src, 256)), dim3(256), 0, E.s, kp, E.n_src, src,
                       E.xs, E.us, bad, E.theta_s);
  if (E.self_targets) {
    E.xt = E.xs;
    E.ut = E.us;
    E.theta_t = E.theta_s;
  } else {
    E.xt = E.alloc<double>(E.n_trg * kp.dim);
    E.ut = E.alloc<double>(E.n_trg * kp.dim);
    if (kp.bloch) E.theta_t = E.alloc<double>(E.n_trg);
    if (E.n_trg > 0)
      hipLaunchKernelGGL(k_prepare, dim3(nblk(E.n_trg, 256)), dim3(256), 0, E.s, kp, E.n_trg,
                         trg, E.xt, E.ut, bad, E.theta_t);
  }
}

void stage_images(pdmk_plan* P, Eval& E, const double* q) {
  const KParams& kp = P->kp;
  int64_t n = E.n_src;
  const double* qim = nullptr;   // Bloch: imaginary part of the wrapped charges
  if (kp.bloch) {
    double* qr = E.alloc<double>(n);
    double* qm = E.alloc<double>(n);
    if (n > 0)
      hipLaunchKernelGGL(k_bloch_charges, dim3(nblk(n, 256)), dim3(256), 0, E.s, n, q,
                         E.theta_s, qr, qm);
    q = qr;
    qim = qm;
    E.q = qr;
    E.q_im = qm;
  }
  int* cnt = E.alloc<int>(n + 2);   // [n + 1]: sources whose unshifted copy is missing
  int* off = E.alloc<int>(n + 1);
  unsigned long long* total64 = E.alloc<unsigned long long>(1);
  PDMK_HIP(hipMemsetAsync(cnt + n, 0, 2 * sizeof(int), E.s));
  PDMK_HIP(hipMemsetAsync(total64, 0, sizeof(unsigned long long), E.s));
  if (n > 0)
    hipLaunchKernelGGL(k_img_count, dim3(std::min(nblk(n, 256), 2048)), dim3(256), 0, E.s, kp,
                       n, E.xs, cnt, cnt + n + 1, total64);
  exclusive_scan_int(cnt, off, (int)(n + 1), E);
  int hv[2] = {0, 0};
  unsigned long long tot = 0;
  PDMK_HIP(hipMemcpyAsync(&hv[0], off + n, sizeof(int), hipMemcpyDeviceToHost, E.s));
  PDMK_HIP(hipMemcpyAsync(&hv[1], cnt + n + 1, sizeof(int), hipMemcpyDeviceToHost, E.s));
  PDMK_HIP(hipMemcpyAsync(&tot, total64, sizeof(tot), hipMemcpyDeviceToHost, E.s));
  PDMK_HIP(hipStreamSynchronize(E.s));
  if (tot > (unsigned long long)kMaxImages)
    throw Error{PDMK_ERR_UNSUPPORTED,
                "sources plus images exceed " + std::to_string(kMaxImages) +
                    " (int32 tree indices): " + std::to_string(tot) +
                    "; use fewer sources or a larger kappa"};
  E.n_img = hv[0];
  const bool from_images = E.self_targets && hv[1] == 0;
  double4* xq = E.alloc<double4>(E.n_img);   // (x, y, z, q) per image, emit order
  int* isrc = E.alloc<int>(E.n_img);
  int* iall = E.keep_map ? E.alloc<int>(E.n_img) : nullptr;
  double* qi_im = qim ? E.alloc<double>(E.n_img) : nullptr;
  if (n > 0)
    hipLaunchKernelGGL(k_img_emit, dim3(nblk(n, 256)), dim3(256), 0, E.s, kp, n, E.xs, q, off,
                       E.n_img, xq, isrc, iall, qim, qi_im);
  int* perm = nullptr;
  sort_points(P, E, E.n_img, nullptr, nullptr, E.skey, E.sx, E.sq, perm, xq);
  if (qim) {
    E.sq_im = E.alloc<double>(E.n_img);
    if (E.n_img > 0)
      hipLaunchKernelGGL(k_gather, dim3(nblk(E.n_img, 256)), dim3(256), 0, E.s, E.n_img, 0, perm,
                         (const double*)nullptr, E.n_img, qi_im, (double*)nullptr, E.sq_im);
  }
  if (E.keep_map) {
    // source index of every sorted image, for re-gathering charges and
    // displacements on the kept tree
    E.img_src = E.alloc<int>(E.n_img);
    if (E.n_img > 0)
      hipLaunchKernelGGL(k_gather_int, dim3(nblk(E.n_img, 256)), dim3(256), 0, E.s, E.n_img,
                         perm, iall, E.img_src);
  }
  if (from_images) {
    E.tkey = E.alloc<uint64_t>(E.n_trg);
    E.tx = E.alloc<double>(E.n_trg * kp.dim);
    E.tperm = E.alloc<int>(E.n_trg);
    E.ox = E.tx;
    E.oq = E.alloc<double>(n);
    if (qim) E.oq_im = E.alloc<double>(n);
    int* flag = E.alloc<int>(E.n_img + 1);
    int* pos = E.alloc<int>(E.n_img + 1);
    int* osrc = E.alloc<int>(E.n_img + 1);
    E.img_trg = E.alloc<int>(E.n_img + 1);
    if (E.n_img > 0) {
      hipLaunchKernelGGL(k_orig_flag, dim3(nblk(E.n_img, 256)), dim3(256), 0, E.s, E.n_img,
                         perm, isrc, flag, osrc);
      exclusive_scan_int(flag, pos, (int)E.n_img, E);
      hipLaunchKernelGGL(k_orig_pick, dim3(nblk(E.n_img, 256)), dim3(256), 0, E.s, E.n_img,
                         E.n_trg, kp.dim, osrc, pos, E.skey, E.sx, E.sq, E.tkey, E.tx, E.tperm,
                         E.oq, E.sq_im, E.oq_im, E.img_trg);
    }
    return;   // original sources in tree order: the picked copies
  } else {
    double* dummyq = nullptr;
    sort_points(P, E, E.n_trg, E.xt, nullptr, E.tkey, E.tx, dummyq, E.tperm);
  }
  // original sources in tree order (spatially coherent spreading)
  if (E.self_targets) {
    E.ox = E.tx;
    E.oq = E.alloc<double>(n);
    if (n > 0)
      hipLaunchKernelGGL(k_gather, dim3(nblk(n, 256)), dim3(256), 0, E.s, n, 0, E.tperm, E.xs, n,
                         q, (double*)nullptr, E.oq);
    if (qim) {
      E.oq_im = E.alloc<double>(n);
      if (n > 0)
        hipLaunchKernelGGL(k_gather, dim3(nblk(n, 256)), dim3(256), 0, E.s, n, 0, E.tperm, E.xs,
                           n, qim, (double*)nullptr, E.oq_im);
    }
  } else {
    uint64_t* okey = nullptr;
    int* operm = nullptr;
    sort_points(P, E, n, E.xs, q, okey, E.ox, E.oq, operm);
    E.operm = operm;
    if (qim) {
      E.oq_im = E.alloc<double>(n);
      if (n > 0)
        hipLaunchKernelGGL(k_gather, dim3(nblk(n, 256)), dim3(256), 0, E.s, n, 0, operm, E.xs, n,
                           qim, (double*)nullptr, E.oq_im);
    }
  }
}

// -------------------------------------------------------------------- tree
__device__ inline int lower_bound_u64(const uint64_t* __restrict__ a, int lo, int hi, uint64_t v) {
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < v) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Range [beg, end) of keys in [kbeg, kbeg + 2^span) within a[lo, hi).
__device__ inline void key_range(const uint64_t* a, int lo, int hi, uint64_t kbeg, int span,
                                 int& beg, int& end) {
  beg = lower_bound_u64(a, lo, hi, kbeg);
  uint64_t kend = kbeg + (span >= 64 ? 0ull : (1ull << span));
  if (span >= 64 || kend <= kbeg) end = hi;
  else end = lower_bound_u64(a, beg, hi, kend);
}

__device__ inline int coll_slot(const int* dl, int d) {
  int s = 0, m = 1;
  for (int a = 0; a < d; ++a) {
    s += (dl[a] + 1) * m;
    m *= 3;
  }
  return s;
}

__global__ void k_level0(KParams kp, Level L, const uint64_t* __restrict__ skey, int nimg,
                         const uint64_t* __restrict__ tkey, int ntrg) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= L.n) return;
  const int d = kp.dim;
  int r[3] = {b % kp.next[0], (b / kp.next[0]) % kp.next[1], d == 3 ? b / (kp.next[0] * kp.next[1]) : 0};
  uint64_t key = (uint64_t)b << (d * kp.B);
  L.key[b] = key;
  for (int a = 0; a < d; ++a) L.coord[b * d + a] = r[a];
  int sb, se, tb, te;
  key_range(skey, 0, nimg, key, d * kp.B, sb, se);
  key_range(tkey, 0, ntrg, key, d * kp.B, tb, te);
  L.sbeg[b] = sb; L.send[b] = se; L.tbeg[b] = tb; L.tend[b] = te;
  L.parent[b] = -1;
  L.child0[b] = -1;
  L.nlid[b] = -1;
  int ncoll = d == 3 ? 27 : 9;
  for (int sl = 0; sl < ncoll; ++sl) {
    int dl[3] = {sl % 3 - 1, (sl / 3) % 3 - 1, sl / 9 - 1};
    int idx = 0, m = 1, sh[3] = {0, 0, 0};
    bool ok = true;
    for (int a = 0; a < d; ++a) {
      int c = r[a] + dl[a];
      if (kp.vimg) {
        // across a face of the cell: the box on the other side, shifted by
        // L n with n_a = -1 (c < 0) or +1 (c >= m_a)
        if (c < 0) { c += kp.next[a]; sh[a] = -1; }
        else if (c >= kp.next[a]) { c -= kp.next[a]; sh[a] = 1; }
      }
      ok = ok && c >= 0 && c < kp.next[a];
      idx += c * m;
      m *= kp.next[a];
    }
    L.coll[b * ncoll + sl] = ok ? idx : -1;
    if (L.cshift) L.cshift[b * ncoll + sl] = (unsigned char)shift_code(sh, d);
  }
}

// Split flags of a level: more than n_s sources, or a split forced by the
// 2:1 balance (the box's (key, level) in the forced list, sorted by key).
__global__ void k_split_flags(Level L, int lvl, int ns, int maxlev, int* __restrict__ flag,
                              const uint64_t* __restrict__ fkey, const int* __restrict__ flev,
                              int nforced) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b > L.n) return;
  if (b == L.n) { flag[b] = 0; return; }
  bool split = L.send[b] - L.sbeg[b] > ns;
  if (!split && nforced > 0) {
    const uint64_t key = L.key[b];
    int lo = 0, hi = nforced;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (fkey[mid] < key) lo = mid + 1; else hi = mid;
    }
    for (int i = lo; i < nforced && fkey[i] == key; ++i)
      if (flev[i] == lvl) split = true;
  }
  flag[b] = (split && lvl < maxlev) ? 1 : 0;
}

// 2:1 balance check of level l (its boxes and those of levels l+1, l+2
// exist): a leaf holding points with a colleague that has a non-leaf child
// is appended to the forced list (key, level) at the next free slot.
__global__ void k_balance_check(Level L, Level C1, int lvl, int d, uint64_t* __restrict__ fkey,
                                int* __restrict__ flev, int* __restrict__ nforced, int cap) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= L.n) return;
  if (L.child0[b] >= 0) return;
  if (L.send[b] <= L.sbeg[b] && L.tend[b] <= L.tbeg[b]) return;
  const int ncoll = d == 3 ? 27 : 9;
  bool viol = false;
  for (int sl = 0; sl < ncoll && !viol; ++sl) {
    const int c = L.coll[b * ncoll + sl];
    if (c < 0) continue;
    const int c0 = L.child0[c];
    if (c0 < 0) continue;
    for (int o = 0; o < (1 << d); ++o)
      if (C1.child0[c0 + o] >= 0) { viol = true; break; }
  }
  if (viol) {
    const int slot = atomicAdd(nforced, 1);
    if (slot < cap) {
      fkey[slot] = L.key[b];
      flev[slot] = lvl;
    }
  }
}

__global__ void k_mark_parents(Level L, const int* __restrict__ flag, const int* __restrict__ off,
                               int d) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= L.n) return;
  if (flag[b]) {
    int s = off[b];
    L.nlid[b] = s;
    L.child0[b] = s << d;
    L.nl_box[s] = b;
  } else {
    L.nlid[b] = -1;
    L.child0[b] = -1;
  }
}

__global__ void k_make_children(KParams kp, Level P, Level C, int lvl,
                                const uint64_t* __restrict__ skey,
                                const uint64_t* __restrict__ tkey) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C.n) return;
  const int d = kp.dim;
  int s = c >> d, o = c & ((1 << d) - 1);
  int b = P.nl_box[s];
  int shift = d * (kp.B - lvl - 1);
  uint64_t key = P.key[b] | ((uint64_t)o << shift);
  C.key[c] = key;
  for (int a = 0; a < d; ++a) C.coord[c * d + a] = 2 * P.coord[b * d + a] + ((o >> a) & 1);
  int sb, se, tb, te;
  key_range(skey, P.sbeg[b], P.send[b], key, shift, sb, se);
  key_range(tkey, P.tbeg[b], P.tend[b], key, shift, tb, te);
  C.sbeg[c] = sb; C.send[c] = se; C.tbeg[c] = tb; C.tend[c] = te;
  C.parent[c] = b;
  C.child0[c] = -1;
  C.nlid[c] = -1;
}

// Colleagues of the boxes of a child level, one thread per (box, slot): the
// neighbour at offset dl lies in the child octant ((g + dl) & 1) of the
// parent's colleague at offset ((g + dl) >> 1) - (g >> 1) (children are made
// in octant order, coordinates are 2 * parent + bit).
__global__ void k_colleagues(Level P, Level C, int d) {
  const int ncoll = d == 3 ? 27 : 9;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)C.n * ncoll) return;
  const int c = (int)(gid / ncoll), sl = (int)(gid - (int64_t)c * ncoll);
  const int b = C.parent[c];
  int ps = 0, m = 1, oct = 0, t = sl;
  for (int a = 0; a < d; ++a) {
    const int dl = t % 3 - 1;
    t /= 3;
    const int g = C.coord[c * d + a];
    const int n = g + dl;
    ps += ((n >> 1) - (g >> 1) + 1) * m;
    m *= 3;
    oct |= (n & 1) << a;
  }
  int cc = -1;
  const int pb = P.coll[b * ncoll + ps];
  if (pb >= 0) {
    const int c0 = P.child0[pb];
    if (c0 >= 0) cc = c0 + oct;
  }
  C.coll[c * ncoll + sl] = cc;
  // a child of a shifted colleague carries the same shift
  if (C.cshift) C.cshift[c * ncoll + sl] = P.cshift[b * ncoll + ps];
}

static void alloc_level(Eval& E, Level& L, int n, int d, bool vimg) {
  L.n = n;
  int ncoll = d == 3 ? 27 : 9;
  L.cshift = vimg ? E.alloc<unsigned char>((size_t)n * ncoll) : nullptr;
  L.key = E.alloc<uint64_t>(n);
  L.coord = E.alloc<int>((size_t)n * d);
  L.sbeg = E.alloc<int>(n);
  L.send = E.alloc<int>(n);
  L.tbeg = E.alloc<int>(n);
  L.tend = E.alloc<int>(n);
  L.parent = E.alloc<int>(n);
  L.child0 = E.alloc<int>(n);
  L.coll = E.alloc<int>((size_t)n * ncoll);
  L.nlid = E.alloc<int>(n);
}

static void build_tree(pdmk_plan* P, Eval& E, const uint64_t* fkey, const int* flev,
                       int nforced);

__global__ void k_set_int(int* p, int v) { *p = v; }

// The adaptive tree; with PDMK_BALANCE rebuilt with forced splits until it is
// 2:1 balanced (Algorithm 1).  Each round's tree is dropped by rewinding the
// workspace to the mark before it (stream order keeps the reuse safe).
void stage_tree(pdmk_plan* P, Eval& E) {
  if (!(P->o.flags & PDMK_BALANCE)) {
    build_tree(P, E, nullptr, nullptr, 0);
    return;
  }
  const int d = P->kp.dim;
  int cap = 0, nforced = 0, rounds = 0;
  uint64_t* fkey = nullptr;
  uint64_t* fkey2 = nullptr;
  int* flev = nullptr;
  int* flev2 = nullptr;
  int* dcount = E.alloc<int>(1);
  for (;;) {
    ++rounds;
    const size_t mark = E.ws->used;
    build_tree(P, E, fkey, flev, nforced);
    if (cap == 0) {
      // the forced list lives below every later round's mark
      int64_t nb = 0;
      for (auto& L : E.lev) nb += L.n;
      cap = (int)std::min<int64_t>(INT32_MAX / 2, 8 * nb + 1024);
      E.ws->used = mark;
      fkey = E.alloc<uint64_t>(cap);
      flev = E.alloc<int>(cap);
      fkey2 = E.alloc<uint64_t>(cap);
      flev2 = E.alloc<int>(cap);
      continue;   // rebuild above the list (the same tree: nothing forced yet)
    }
    const int nlev = (int)E.lev.size();
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, E.s, dcount, nforced);
    for (int l = 0; l + 2 < nlev; ++l)
      hipLaunchKernelGGL(k_balance_check, dim3(nblk(E.lev[l].n, 256)), dim3(256), 0, E.s,
                         E.lev[l], E.lev[l + 1], l, d, fkey, flev, dcount, cap);
    const int total = read_int(dcount, E.s);
    if (total > cap) throw Error{PDMK_ERR_UNSUPPORTED, "2:1 balance: forced-split list overflow"};
    if (total == nforced || rounds > 64) break;
    // keep the list sorted by key (the level decides among equal keys)
    size_t tb = 0;
    PDMK_HIP(rocprim::radix_sort_pairs(nullptr, tb, fkey, fkey2, flev, flev2, (size_t)total, 0u,
                                       64u, E.s));
    void* tmp = E.alloc<char>(tb);
    PDMK_HIP(rocprim::radix_sort_pairs(tmp, tb, fkey, fkey2, flev, flev2, (size_t)total, 0u, 64u,
                                       E.s));
    PDMK_HIP(hipMemcpyAsync(fkey, fkey2, (size_t)total * sizeof(uint64_t),
                            hipMemcpyDeviceToDevice, E.s));
    PDMK_HIP(hipMemcpyAsync(flev, flev2, (size_t)total * sizeof(int), hipMemcpyDeviceToDevice,
                            E.s));
    nforced = total;
    E.ws->used = mark;   // the next round's tree replaces this one
  }
  E.st.n_forced_splits = nforced;
  E.st.balance_rounds = rounds;
}

static void build_tree(pdmk_plan* P, Eval& E, const uint64_t* fkey, const int* flev,
                       int nforced) {
  const KParams& kp = P->kp;
  const int d = kp.dim;
  E.lev.clear();
  int n0 = kp.next[0] * kp.next[1] * (d == 3 ? kp.next[2] : 1);
  Level L0;
  alloc_level(E, L0, n0, d, kp.vimg != 0);
  hipLaunchKernelGGL(k_level0, dim3(nblk(n0, 128)), dim3(128), 0, E.s, kp, L0, E.skey,
                     (int)E.n_img, E.tkey, (int)E.n_trg);
  E.lev.push_back(L0);
  const int maxlev = kp.B;
  for (int l = 0;; ++l) {
    Level& Lp = E.lev[l];
    int* flag = E.alloc<int>(Lp.n + 1);
    int* off = E.alloc<int>(Lp.n + 1);
    hipLaunchKernelGGL(k_split_flags, dim3(nblk(Lp.n + 1, 256)), dim3(256), 0, E.s, Lp, l,
                       P->mp.n_s, maxlev, flag, fkey, flev, nforced);
    exclusive_scan_int(flag, off, Lp.n + 1, E);
    int nsplit = read_int(off + Lp.n, E.s);
    Lp.nnl = nsplit;
    Lp.nl_box = E.alloc<int>(nsplit);
    hipLaunchKernelGGL(k_mark_parents, dim3(nblk(Lp.n, 256)), dim3(256), 0, E.s, Lp, flag, off,
                       d);
    if (nsplit == 0) break;
    Level C;
    alloc_level(E, C, nsplit << d, d, kp.vimg != 0);
    Level Pcopy = E.lev[l];
    hipLaunchKernelGGL(k_make_children, dim3(nblk(C.n, 128)), dim3(128), 0, E.s, kp, Pcopy, C, l,
                       E.skey, E.tkey);
    hipLaunchKernelGGL(k_colleagues, dim3(nblk((int64_t)C.n * (d == 3 ? 27 : 9), 256)),
                       dim3(256), 0, E.s, Pcopy, C, d);
    E.lev.push_back(C);
  }
  E.d_lev = E.alloc<Level>(E.lev.size());
  PDMK_HIP(hipMemcpyAsync(E.d_lev, E.lev.data(), sizeof(Level) * E.lev.size(),
                          hipMemcpyHostToDevice, E.s));
  int64_t nb = 0, nnl = 0;
  for (auto& L : E.lev) {
    nb += L.n;
    nnl += L.nnl;
  }
  E.st.n_levels = (int)E.lev.size();
  E.st.n_boxes = nb;
  E.st.n_nonleaf = nnl;
  E.st.n_leaves = nb - nnl;
}

// ------------------------------------------------------------------- lists
// Residual interaction list of a target leaf T at level i (plane waves are
// exchanged only between colleagues that both have children):
//   (a) every colleague C of T: all sources of C, residual R_i;
//   (b) for every ancestor A of T at level j < i: every colleague D of A
//       without children: all sources of D, residual R_j.
// Mode 0 counts entries (and direct pairs), mode 1 writes them.  Slots of
// boxes that are not target leaves get no entries.
// The rule is symmetric: a point pair (x in T, y in S) meets in T's list
// through an entry holding S's box and in S's list through one holding T's
// box, with the same level (a virtual colleague under shift n is met again
// under -n).  sym (targets = sources, pairs evaluated once): an entry whose
// box precedes T in source order and holds only points of the cell (no
// shifted copies: as many sources as targets) is left out, since the leaves
// after it add its pairs to both ends.
// One list slot; returns its listed pairs (sources x targets) in mode 0.
__device__ inline unsigned long long leaf_list_one(int d, int i, const Level* __restrict__ lev,
                                                   const int* __restrict__ lf_level,
                                                   const int* __restrict__ lf_box,
                                                   int* __restrict__ cnt,
                                                   const int* __restrict__ beg,
                                                   int4* __restrict__ list,
                                                   int* __restrict__ nsrc, int sym) {
  const int ncoll = d == 3 ? 27 : 9;
  int lvl = lf_level[i], b = lf_box[i];
  const Level& T = lev[lvl];
  if (T.child0[b] >= 0 || T.tend[b] <= T.tbeg[b]) {
    // not a target leaf: no list, no residual work
    if (cnt) {
      cnt[i] = 0;
      nsrc[i] = 0;
    }
    return 0;
  }
  int k = 0;
  long long np = 0;
  int o = beg ? beg[i] : 0;
  const int tsb = T.sbeg[b];
  // .w of an entry: the shift_code of a virtual image's colleague (0: none)
  for (int sl = 0; sl < ncoll; ++sl) {
    int c = T.coll[b * ncoll + sl];
    if (c < 0) continue;
    int sb = T.sbeg[c], se = T.send[c];
    if (se <= sb) continue;
    const int sh = T.cshift ? T.cshift[b * ncoll + sl] : 0;
    if (sym && se <= tsb && se - sb == T.tend[c] - T.tbeg[c]) continue;
    if (list) list[o + k] = make_int4(sb, se, lvl, sh);
    ++k;
    np += se - sb;
  }
  int a = T.parent[b];
  for (int l = lvl - 1; l >= 0 && a >= 0; --l) {
    const Level& A = lev[l];
    for (int sl = 0; sl < ncoll; ++sl) {
      int D = A.coll[a * ncoll + sl];
      if (D < 0 || A.child0[D] >= 0) continue;
      int sb = A.sbeg[D], se = A.send[D];
      if (se <= sb) continue;
      const int sh = A.cshift ? A.cshift[a * ncoll + sl] : 0;
      if (sym && se <= tsb && se - sb == A.tend[D] - A.tbeg[D]) continue;
      if (list) list[o + k] = make_int4(sb, se, l, sh);
      ++k;
      np += se - sb;
    }
    a = A.parent[a];
  }
  if (!cnt) return 0;
  const long long nt = T.tend[b] - T.tbeg[b];
  cnt[i] = k;
  nsrc[i] = (int)np;
  return (unsigned long long)(np * nt);
}

// The listed pairs are summed per wave before one atomic (one address for
// every slot would serialise the atomics at the cache).
__global__ void k_leaf_lists(int d, int nleaf, const Level* __restrict__ lev,
                             const int* __restrict__ lf_level, const int* __restrict__ lf_box,
                             int* __restrict__ cnt, const int* __restrict__ beg,
                             int4* __restrict__ list, unsigned long long* __restrict__ pairs,
                             int* __restrict__ nsrc, int sym) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long pc = 0;
  if (i < nleaf) pc = leaf_list_one(d, i, lev, lf_level, lf_box, cnt, beg, list, nsrc, sym);
  if (pairs) {
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) pc += __shfl_xor(pc, m);
    if ((threadIdx.x & 63) == 0) atomicAdd(pairs, pc);
  }
}

// Work items of the residual sums: leaf i's targets are cut into chunks of
// kDirectTgt and its concatenated source list into segments of kDirectSeg
// sources; item = (leaf, chunk * nseg + segment).
__global__ void k_seg_count(int n, const Level* __restrict__ lev, const int* __restrict__ lf_level,
                            const int* __restrict__ lf_box, const int* __restrict__ nsrc,
                            int* __restrict__ segs) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Level& T = lev[lf_level[i]];
  const int b = lf_box[i];
  const int nt = T.tend[b] - T.tbeg[b];
  segs[i] = ((nsrc[i] + kDirectSeg - 1) / kDirectSeg) * ((nt + kDirectTgt - 1) / kDirectTgt);
}

// Also writes a sort key per item: larger cost (targets of the chunk, at
// least 8, times sources of the segment) sorts first.
__global__ void k_seg_fill(int n, const Level* __restrict__ lev, const int* __restrict__ lf_level,
                           const int* __restrict__ lf_box, const int* __restrict__ nsrc,
                           const int* __restrict__ beg, int2* __restrict__ items,
                           unsigned* __restrict__ key) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Level& T = lev[lf_level[i]];
  const int b = lf_box[i];
  const int nt = T.tend[b] - T.tbeg[b];
  const int ns = nsrc[i];
  const int nseg = (ns + kDirectSeg - 1) / kDirectSeg;
  for (int k = beg[i]; k < beg[i + 1]; ++k) {
    const int r = k - beg[i];
    const int seg = r % nseg, tc = r / nseg;
    const int ct = min(kDirectTgt, nt - tc * kDirectTgt);
    const int cs = min(kDirectSeg, ns - seg * kDirectSeg);
    items[k] = make_int2(i, r);
    key[k] = 0xffffffffu - (unsigned)(max(ct, 8) * cs);
  }
}

// Every box of every level (level by level, boxes in key order) is a list
// slot; boxes that are not target leaves get empty lists and no work items,
// so the slots need no compaction (and no host read of the leaf count).
__global__ void k_box_slots(Level L, int lvl, int* __restrict__ lf_level,
                            int* __restrict__ lf_box) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= L.n) return;
  lf_level[b] = lvl;
  lf_box[b] = b;
}

void stage_lists(pdmk_plan* P, Eval& E) {
  const int d = P->kp.dim;
  int total = 0;
  for (auto& L : E.lev) total += L.n;
  const int n = total;
  E.nleaf_t = n;
  E.lf_level = E.alloc<int>(n);
  E.lf_box = E.alloc<int>(n);
  {
    int off = 0;
    for (size_t l = 0; l < E.lev.size(); ++l) {
      if (E.lev[l].n > 0)
        hipLaunchKernelGGL(k_box_slots, dim3(nblk(E.lev[l].n, 256)), dim3(256), 0, E.s,
                           E.lev[l], (int)l, E.lf_level + off, E.lf_box + off);
      off += E.lev[l].n;
    }
  }
  int* cnt = E.alloc<int>(n + 1);
  E.lf_list_beg = E.alloc<int>(n + 1);
  unsigned long long* pairs = E.alloc<unsigned long long>(1);
  PDMK_HIP(hipMemsetAsync(pairs, 0, sizeof(unsigned long long), E.s));
  PDMK_HIP(hipMemsetAsync(cnt + n, 0, sizeof(int), E.s));
  E.lf_nsrc = E.alloc<int>(n > 0 ? n : 1);
  int* segs = E.alloc<int>(n + 1);
  int* sbeg = E.alloc<int>(n + 1);
  PDMK_HIP(hipMemsetAsync(segs + n, 0, sizeof(int), E.s));
  if (n > 0) {
    hipLaunchKernelGGL(k_leaf_lists, dim3(nblk(n, 128)), dim3(128), 0, E.s, d, n, E.d_lev,
                       E.lf_level, E.lf_box, cnt, (const int*)nullptr, (int4*)nullptr, pairs,
                       E.lf_nsrc, E.sym ? 1 : 0);
    // work items of the residual sums: segments of each leaf's source list
    hipLaunchKernelGGL(k_seg_count, dim3(nblk(n, 256)), dim3(256), 0, E.s, n, E.d_lev, E.lf_level,
                       E.lf_box, E.lf_nsrc, segs);
  }
  // visited pairs (statistics): read with the call's other counters at its end
  PDMK_HIP(hipMemcpyAsync(P->h_cnt + 3, pairs, sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, E.s));
  exclusive_scan_int(segs, sbeg, n + 1, E);
  exclusive_scan_int(cnt, E.lf_list_beg, n + 1, E);
  {
    int hv[2] = {0, 0};
    PDMK_HIP(hipMemcpyAsync(&hv[0], sbeg + n, sizeof(int), hipMemcpyDeviceToHost, E.s));
    PDMK_HIP(hipMemcpyAsync(&hv[1], E.lf_list_beg + n, sizeof(int), hipMemcpyDeviceToHost, E.s));
    PDMK_HIP(hipStreamSynchronize(E.s));
    E.nitems = hv[0];
    E.nlist = hv[1];
  }
  E.item_beg = sbeg;
  if (E.nitems > 0) {
    int2* items = E.alloc<int2>(E.nitems);
    E.items_u = items;
    unsigned* key = E.alloc<unsigned>(E.nitems);
    hipLaunchKernelGGL(k_seg_fill, dim3(nblk(n, 256)), dim3(256), 0, E.s, n, E.d_lev,
                       E.lf_level, E.lf_box, E.lf_nsrc, sbeg, items, key);
    // launch order: most expensive items first, so that no long block forms
    // the tail of the grid
    E.items = E.alloc<int2>(E.nitems);
    unsigned* key2 = E.alloc<unsigned>(E.nitems);
    size_t tb = 0;
    PDMK_HIP(rocprim::radix_sort_pairs(nullptr, tb, key, key2, items, E.items,
                                       (size_t)E.nitems, 0u, 32u, E.s));
    void* tmp = E.alloc<char>(tb);
    PDMK_HIP(rocprim::radix_sort_pairs(tmp, tb, key, key2, items, E.items, (size_t)E.nitems, 0u,
                                       32u, E.s));
  }
  E.list = E.alloc<int4>(E.nlist > 0 ? E.nlist : 1);
  if (n > 0 && E.nlist > 0)
    hipLaunchKernelGGL(k_leaf_lists, dim3(nblk(n, 128)), dim3(128), 0, E.s, d, n, E.d_lev,
                       E.lf_level, E.lf_box, (int*)nullptr, E.lf_list_beg, E.list,
                       (unsigned long long*)nullptr, (int*)nullptr, E.sym ? 1 : 0);
}

}  // namespace pdmk

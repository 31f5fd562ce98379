// C interface (include/pdmk.h): plans, evaluation pipeline of Algorithm 1,
// assembly with the self-interaction correction (Section 3.8), status codes.
#include <cmath>
#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <set>
#include <thread>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <string>
#include <system_error>

#include "internal.h"

using namespace pdmk;

static thread_local std::string g_last_error;

static int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

static inline int nblk(int64_t n, int b) { return (int)((n + b - 1) / b); }

static ChebSeries cheb_derivative(const ChebSeries& S) {
  // d/ds of sum a_k T_k(2s-1): derivative in t by the standard recurrence, times 2
  int n = (int)S.a.size();
  ChebSeries D;
  if (n < 2) {
    D.a.assign(1, 0.0);
    return D;
  }
  std::vector<double> d(n + 1, 0.0);
  for (int k = n - 1; k >= 1; --k) d[k - 1] = d[k + 1] + 2.0 * k * S.a[k];
  d[0] *= 0.5;
  D.a.assign(d.begin(), d.begin() + (n - 1));
  for (double& v : D.a) v *= 2.0;
  return D;
}

static std::vector<double> pw_table(const Pswf& P, double c, int J, int dim) {
  int nmax = dim * J * J;
  std::vector<double> t(nmax + 1, 0.0);
  t[0] = -P.psit_dd0 / (24.0 * c * c);
  for (int n = 1; n <= nmax; ++n) {
    double jn = std::sqrt((double)n);
    t[n] = (P.psit(kPi * jn / (3.0 * c)) - P.psit(2.0 * kPi * jn / (3.0 * c))) /
           (4.0 * kPi * kPi * n);
  }
  return t;
}

template <class T>
static T* upload(const std::vector<T>& v) {
  T* p = nullptr;
  PDMK_HIP(hipMalloc(&p, std::max<size_t>(1, v.size()) * sizeof(T)));
  if (!v.empty()) PDMK_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return p;
}

namespace pdmk {
__global__ void k_fill_zero(uint64_t* __restrict__ w, int64_t nw, unsigned char* __restrict__ tail,
                            int ntail) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nw) w[i] = 0ull;
  if (i < ntail) tail[i] = 0;
}

__global__ void k_fill_zero_bytes(unsigned char* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = 0;
}

void fill_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  if (reinterpret_cast<uintptr_t>(p) % 8 != 0) {
    hipLaunchKernelGGL(k_fill_zero_bytes, dim3(nblk((int64_t)bytes, 256)), dim3(256), 0, s,
                       static_cast<unsigned char*>(p), (int64_t)bytes);
    return;
  }
  // whole 8-byte words, then the last bytes % 8
  const int64_t nw = (int64_t)(bytes / 8);
  const int ntail = (int)(bytes % 8);
  const int64_t n = std::max<int64_t>(nw, ntail);
  hipLaunchKernelGGL(k_fill_zero, dim3(nblk(n, 256)), dim3(256), 0, s,
                     static_cast<uint64_t*>(p), nw, static_cast<unsigned char*>(p) + 8 * nw,
                     ntail);
}

void ensure_lds(const void* kernel, size_t bytes) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, size_t> limit;
  int dev = 0;
  PDMK_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  size_t& cur = limit[{dev, kernel}];
  if (bytes <= cur) return;
  PDMK_HIP(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  cur = bytes;
}

void plan_upload_tables(pdmk_plan* P) {
  const int d = P->g.dim;
  const int p = P->mp.porder, J = P->mp.npw;
  ChebSeries Ed = cheb_derivative(P->T->E), F2d = cheb_derivative(P->T->F2);
  // The kernels evaluate each series sum_k c_k T_k(u) by Horner's rule in the
  // monomial basis of u = 2 s - 1 (half the operations of Clenshaw's
  // recurrence).  For these series sum_j |a_j| stays within a factor 5 of
  // max |E| on [-1, 1] (a factor 1.0-1.2 except for the 2D derivative at
  // eps = 1e-3), so the monomial form costs no accuracy.  FP32 evaluation
  // uses the series cut where |c_k| drops below 1e-8 max |c| (below FP32
  // resolution).  Zero-padded to 32 + 32 entries.
  auto mono = [](std::vector<double> c, bool fp32) {
    if (fp32) {
      double mx = 0;
      for (double v : c) mx = std::max(mx, std::fabs(v));
      while (c.size() > 1 && std::fabs(c.back()) < 1e-8 * mx) c.pop_back();
    }
    const size_t n = c.size();
    std::vector<double> a(n, 0.0), tm(n, 0.0), tk(n, 0.0), tp(n, 0.0);
    if (n > 0) tm[0] = 1.0;            // T_0
    if (n > 1) tk[1] = 1.0;            // T_1
    for (size_t k = 0; k < n; ++k) {
      const std::vector<double>& T = k == 0 ? tm : tk;
      for (size_t j = 0; j < n; ++j) a[j] += c[k] * T[j];
      if (k >= 1) {
        // T_{k+1} = 2 u T_k - T_{k-1}
        for (size_t j = 0; j < n; ++j) tp[j] = (j ? 2.0 * tk[j - 1] : 0.0) - tm[j];
        tm = tk;
        tk = tp;
      }
    }
    return a;
  };
  auto both = [&](const std::vector<double>& c, int& n64, int& n32) {
    std::vector<double> a = mono(c, false), b = mono(c, true);
    if (a.size() > 32) throw Error{PDMK_ERR_UNSUPPORTED, "kernel series longer than 32 terms"};
    n64 = (int)a.size();
    n32 = (int)b.size();
    a.resize(32, 0.0);
    b.resize(32, 0.0);
    a.insert(a.end(), b.begin(), b.end());
    return a;
  };
  KParams& kq = P->kp;
  P->d_E = upload(both(P->T->E.a, kq.nE, kq.nE32));
  P->d_Ed = upload(both(Ed.a, kq.nEd, kq.nEd32));
  P->d_F2 = upload(both(P->T->F2.a, kq.nF2, kq.nF232));
  P->d_F2d = upload(both(F2d.a, kq.nF2d, kq.nF2d32));
  std::vector<double> nodes, bw;
  cheb_nodes(p, nodes, bw);
  P->d_nodes = upload(nodes);
  P->d_bw = upload(bw);
  std::vector<double> Tm(2 * p * p), row(p);
  for (int sel = 0; sel < 2; ++sel) {
    double sg = sel ? 1.0 : -1.0;
    for (int i = 0; i < p; ++i) {
      lagrange_row(p, nodes.data(), bw.data(), 0.5 * sg + 0.5 * nodes[i], row.data());
      for (int Pp = 0; Pp < p; ++Pp) Tm[sel * p * p + Pp * p + i] = row[Pp];
    }
  }
  P->d_Tm = upload(Tm);
  std::vector<double2> F((2 * J + 1) * p);
  for (int j = -J; j <= J; ++j)
    for (int i = 0; i < p; ++i) {
      double a = -kPi * j * nodes[i] / 3.0;
      F[(j + J) * p + i] = make_double2(std::cos(a), std::sin(a));
    }
  P->d_F = upload(F);
  {
    std::vector<double2> Fc(F.size()), Fw(F.size());
    for (int j = -J; j <= J; ++j)
      for (int i = 0; i < p; ++i) {
        const double2 f = F[(j + J) * p + i];
        Fc[(j + J) * p + i] = make_double2(f.x, -f.y);
        const double w = j > 0 ? 2.0 : 1.0;
        Fw[(j + J) * p + i] = make_double2(w * f.x, -w * f.y);
      }
    P->d_Fc = upload(Fc);
    P->d_Fw = upload(Fw);
  }
  std::vector<float2> Ff(F.size());
  for (size_t i = 0; i < F.size(); ++i) Ff[i] = make_float2((float)F[i].x, (float)F[i].y);
  P->d_Ff = upload(Ff);
  P->d_dtab = upload(pw_table(*P->P, P->P->c, J, d));
  std::vector<double> sv;
  for (size_t s = 0; s < P->g.shifts.size() / d; ++s)
    for (int a = 0; a < d; ++a) {
      double v = 0;
      for (int b = 0; b < d; ++b) v += P->g.L[a + d * b] * P->g.shifts[s * d + b];
      sv.push_back(v);
    }
  P->nshift = (int)(P->g.shifts.size() / d);
  P->d_shiftvec = upload(sv);
}
}  // namespace pdmk

static void unbind(pdmk_plan* P);

static void free_plan_tables(pdmk_plan* P) {
  void* ptrs[] = {P->d_E, P->d_Ed, P->d_F2, P->d_F2d, P->d_nodes, P->d_bw, P->d_Tm,
                  P->d_F, P->d_Ff, P->d_dtab, P->d_farscale, P->d_shiftvec, P->d_pwt_f,
                  P->d_pwt_d, P->adj_buf, P->d_ball, P->d_brow, P->d_fftw, P->d_pwt_b,
                  P->d_Fc, P->d_Fw};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  pdmk::gemm_release(P);
  for (hipEvent_t e : P->ev_pool) (void)hipEventDestroy(e);
  P->ev_pool.clear();
  P->ev_next = 0;
  if (P->h_cnt) (void)hipHostFree(P->h_cnt);
  P->h_cnt = nullptr;
  if (P->s_aux) {
    (void)hipStreamSynchronize(P->s_aux);
    (void)hipStreamDestroy(P->s_aux);
    P->s_aux = nullptr;
  }
  if (P->arena) {
    // every evaluation synchronises its stream before returning, so the
    // arena is no longer in use
    (void)hipFree(P->arena);
    P->arena = nullptr;
    P->arena_size = 0;
  }
}

// After a call: free this call's overflow blocks and grow the arena to the
// call's total, so that the next call of this size takes no allocation.
static void finish_workspace(char*& arena, size_t& arena_size, Workspace& ws) {
  const bool grow = !ws.overflow.empty();
  ws.release_overflow();
  if (grow) {
    if (arena) PDMK_HIP(hipFree(arena));
    arena = nullptr;
    arena_size = 0;
    const size_t want = ws.used + ws.used / 8;
    void* p = nullptr;
    if (hipMalloc(&p, want) == hipSuccess) {
      arena = static_cast<char*>(p);
      arena_size = want;
    } else {
      (void)hipGetLastError();   // the next call allocates per request again
    }
  }
}

// Method parameters for the options: defaults for (dim, eps), overridden by
// every positive field.  With PDMK_WANT_GRAD the default window is two cells
// wider: the gradient of the far field differentiates the window, which
// loses about a factor 10-50 of accuracy at the default width.
static MethodParams resolve_params(const pdmk_opts* o) {
  MethodParams m = default_params(o->dim, o->eps);
  if (o->flags & PDMK_WANT_GRAD) m.nufft_w = std::min(16, m.nufft_w + 2);
  if (o->kappa > 0) m.kappa = o->kappa;
  if (o->n_s > 0) m.n_s = o->n_s;
  if (o->porder > 0) m.porder = o->porder;
  if (o->npw > 0) m.npw = o->npw;
  if (o->sigma > 0) m.sigma = o->sigma;
  if (o->nufft_w > 0) m.nufft_w = o->nufft_w;
  m.beta = window_beta(m.nufft_w, m.sigma);
  return m;
}

// ---------------------------------------------------------------- kernels
// Charge sum and sum of magnitudes: per-block partials (part[2 b], part[2 b + 1]).
__global__ void k_charge_stats(int64_t n, const double* __restrict__ q, double* __restrict__ part,
                               int* __restrict__ bad) {
  __shared__ double s1[256], s2[256];
  double a = 0.0, b = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double v = q[i];
    if (!isfinite(v)) atomicOr(bad, 1);
    else {
      a += v;
      b += fabs(v);
    }
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      s1[threadIdx.x] += s1[threadIdx.x + st];
      s2[threadIdx.x] += s2[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s1[0];
    part[2 * blockIdx.x + 1] = s2[0];
  }
}

// Sum of the per-block partials of k_charge_stats in a fixed order (one
// block), so the charge sum -- and the uniform-background constant it
// scales -- does not depend on the order blocks finish in.
__global__ void k_charge_stats_final(int nblocks, const double* __restrict__ part,
                                     double* __restrict__ out) {
  __shared__ double s1[256], s2[256];
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nblocks; k += 256) {
    a += part[2 * k];
    b += part[2 * k + 1];
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      s1[threadIdx.x] += s1[threadIdx.x + st];
      s2[threadIdx.x] += s2[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = s1[0];
    out[1] = s2[0];
  }
}

// Final assembly: un-permute, add the uniform-background constant
// -(sum q) cnn, rotate gradients back.  Writes nothing when the input was
// rejected (non-finite values, or charges not neutral without
// allow_nonneutral), so the caller's outputs stay untouched on error.
__global__ void k_assemble(int64_t n, int d, const int* __restrict__ tperm,
                           const double* __restrict__ ps, const double* __restrict__ gs,
                           const double* __restrict__ qs, const int* __restrict__ flags,
                           double cnn, int allow_nonneutral, KParams kp,
                           double* __restrict__ pot, double* __restrict__ grad) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  if (flags[0] || flags[1]) return;
  if (!allow_nonneutral && fabs(qs[0]) > 1e-8 * qs[1]) return;
  const double shift = -qs[0] * cnn;
  const int o = tperm[t];
  pot[o] = ps[t] + shift;
  if (grad) {
    double g[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) g[a] = gs[t * d + a];
    for (int a = 0; a < d; ++a) {
      double s = 0;
      for (int b = 0; b < d; ++b) s += kp.Q[a + d * b] * g[b];
      grad[(int64_t)o * d + a] = s;
    }
  }
}

// Adjoint combination (targets = sources when gphi_self is set):
//   dq_j = Psi(y_j),  dsrc_j = q_j grad Psi(y_j) [+ g_j grad Phi(y_j)],
//   dtrg_i = g_i grad Phi(x_i)
__global__ void k_adjoint_combine(int64_t ns, int64_t nt, int d, const double* __restrict__ q,
                                  const double* __restrict__ g,
                                  const double* __restrict__ gphi, int self_t,
                                  const double* __restrict__ psi,
                                  const double* __restrict__ gpsi, double* __restrict__ dq,
                                  double* __restrict__ dsrc, double* __restrict__ dtrg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ns) {
    if (dq) dq[i] = psi[i];
    if (dsrc)
      for (int a = 0; a < d; ++a) {
        double v = q[i] * gpsi[i * d + a];
        if (self_t) v = fma(g[i], gphi[i * d + a], v);
        dsrc[i * d + a] = v;
      }
  }
  if (dtrg && i < nt)
    for (int a = 0; a < d; ++a) dtrg[i * d + a] = g[i] * gphi[i * d + a];
}

// ------------------------------------------------------------------- C ABI
extern "C" {

const char* pdmk_status_string(int s) {
  switch (s) {
    case PDMK_OK: return "ok";
    case PDMK_ERR_INVALID_ARG: return "invalid argument";
    case PDMK_ERR_SINGULAR_LATTICE: return "singular or ill-conditioned lattice";
    case PDMK_ERR_NOT_NEUTRAL: return "charges are not neutral";
    case PDMK_ERR_EPS_RANGE: return "eps outside [1e-12, 1e-2]";
    case PDMK_ERR_NONFINITE: return "non-finite input";
    case PDMK_ERR_OUT_OF_MEMORY: return "device out of memory";
    case PDMK_ERR_HIP: return "HIP runtime error";
    case PDMK_ERR_NO_DEVICE: return "no HIP device";
    case PDMK_ERR_UNSUPPORTED: return "unsupported option";
    case PDMK_ERR_SCRATCH: return "input too large for the fixed device scratch";
  }
  return "unknown status";
}

const char* pdmk_last_error(void) { return g_last_error.c_str(); }

int pdmk_default_opts(int dim, double eps, pdmk_opts* out) {
  if (!out) return fail(PDMK_ERR_INVALID_ARG, "null output");
  if (dim != 2 && dim != 3) return fail(PDMK_ERR_INVALID_ARG, "dim must be 2 or 3");
  if (!(eps >= 1e-12 && eps <= 1e-2)) return fail(PDMK_ERR_EPS_RANGE, "eps out of range");
  MethodParams m = default_params(dim, eps);
  std::memset(out, 0, sizeof(*out));
  out->dim = dim;
  out->eps = eps;
  out->precision = PDMK_PREC_FP64;
  out->kappa = m.kappa;
  out->n_s = m.n_s;
  out->porder = m.porder;
  out->npw = m.npw;
  out->nufft_w = 0;   // chosen at plan creation (it depends on PDMK_WANT_GRAD)
  out->sigma = m.sigma;
  return PDMK_OK;
}

int pdmk_kernel_info_get(int dim, double eps, pdmk_kernel_info* out) {
  if (!out || (dim != 2 && dim != 3)) return fail(PDMK_ERR_INVALID_ARG, "bad argument");
  if (!(eps >= 1e-12 && eps <= 1e-2)) return fail(PDMK_ERR_EPS_RANGE, "eps out of range");
  const Pswf& P = pswf_for_eps(eps);
  const SplitTables& T = tables_for_eps(eps);
  out->c = P.c;
  out->lambda0 = P.lambda0;
  out->c0_over_psi0 = P.c0 / P.psi0;
  out->w0_zero = T.w0_unit(dim);
  return PDMK_OK;
}

int pdmk_kernel_eval_residual(int dim, double eps, double h, int64_t n, const double* r,
                              double* out) {
  if ((dim != 2 && dim != 3) || n < 0 || (n > 0 && (!r || !out)) || !(h > 0))
    return fail(PDMK_ERR_INVALID_ARG, "bad argument");
  if (!(eps >= 1e-12 && eps <= 1e-2)) return fail(PDMK_ERR_EPS_RANGE, "eps out of range");
  const SplitTables& T = tables_for_eps(eps);
  for (int64_t i = 0; i < n; ++i) out[i] = T.residual(dim, r[i], h);
  return PDMK_OK;
}

int pdmk_kernel_eval_w0hat(int dim, double eps, double rc, int64_t n, const double* k,
                           double* out) {
  if ((dim != 2 && dim != 3) || n < 0 || (n > 0 && (!k || !out)) || !(rc > 0))
    return fail(PDMK_ERR_INVALID_ARG, "bad argument");
  if (!(eps >= 1e-12 && eps <= 1e-2)) return fail(PDMK_ERR_EPS_RANGE, "eps out of range");
  const Pswf& P = pswf_for_eps(eps);
  for (int64_t i = 0; i < n; ++i) out[i] = P.psit(k[i] * rc / P.c) / (k[i] * k[i]);
  return PDMK_OK;
}

static int validate_opts(const pdmk_opts* o) {
  if (!o) return fail(PDMK_ERR_INVALID_ARG, "null options");
  if (o->dim != 2 && o->dim != 3) return fail(PDMK_ERR_INVALID_ARG, "dim must be 2 or 3");
  if (!(o->eps >= 1e-12 && o->eps <= 1e-2)) return fail(PDMK_ERR_EPS_RANGE, "eps out of range");
  if (o->precision != PDMK_PREC_FP64 && o->precision != PDMK_PREC_MIXED)
    return fail(PDMK_ERR_INVALID_ARG, "unknown precision");
  if (o->porder > 40 || o->npw > 64 || o->nufft_w > 16 || o->sigma > 4.0)
    return fail(PDMK_ERR_INVALID_ARG, "porder <= 40, npw <= 64, nufft_w <= 16, sigma <= 4");
  if (o->flags & ~(unsigned)(PDMK_WANT_GRAD | PDMK_ALLOW_NONNEUTRAL | PDMK_DETERMINISTIC |
                             PDMK_VECTOR_PLANE_WAVES | PDMK_ONE_STREAM | PDMK_BLOCH |
                             PDMK_VIRTUAL_IMAGES | PDMK_BALANCE | PDMK_ALL_PAIRS))
    return fail(PDMK_ERR_INVALID_ARG, "unknown flag");
  if ((o->flags & PDMK_BLOCH) && (o->flags & PDMK_VIRTUAL_IMAGES))
    return fail(PDMK_ERR_UNSUPPORTED, "PDMK_BLOCH does not support PDMK_VIRTUAL_IMAGES");
  if (o->flags & PDMK_BLOCH) {
    for (int a = 0; a < o->dim; ++a)
      if (!std::isfinite(o->bloch[a])) return fail(PDMK_ERR_INVALID_ARG, "non-finite Bloch vector");
    if (o->flags & (PDMK_WANT_GRAD | PDMK_DETERMINISTIC))
      return fail(PDMK_ERR_UNSUPPORTED,
                  "PDMK_BLOCH does not support PDMK_WANT_GRAD or PDMK_DETERMINISTIC");
  }
  if (o->fp32_stages & ~15u) return fail(PDMK_ERR_INVALID_ARG, "unknown fp32_stages bit");
  return PDMK_OK;
}

// Status of a make_geometry message.
static int geometry_status(const std::string& msg) {
  if (msg.rfind("unsupported:", 0) == 0) return PDMK_ERR_UNSUPPORTED;
  return msg.find("kappa") != std::string::npos ? PDMK_ERR_INVALID_ARG
                                                : PDMK_ERR_SINGULAR_LATTICE;
}

static double bloch_norm(const pdmk_opts* o) {
  if (!(o->flags & PDMK_BLOCH)) return 0.0;
  double s = 0.0;
  for (int a = 0; a < o->dim; ++a) s += o->bloch[a] * o->bloch[a];
  return std::sqrt(s);
}

// Oriented Bloch vector beta' = Q^T beta (beta.x is invariant under the
// rotation).  False when beta lies in the reciprocal lattice (L^T beta / 2 pi
// integral): that is the periodic case.
static bool oriented_bloch(const Geometry& g, const pdmk_opts* opts, double* beta) {
  const int d = g.dim;
  for (int a = 0; a < d; ++a) {
    double v = 0.0;
    for (int b = 0; b < d; ++b) v += g.Q[b + d * a] * opts->bloch[b];
    beta[a] = v;
  }
  for (int a = 0; a < d; ++a) {
    double u = 0.0;
    for (int b = 0; b < d; ++b) u += g.L[b + d * a] * beta[b];
    u /= 2.0 * kPi;
    if (std::fabs(u - std::rint(u)) > 1e-9) return true;
  }
  return false;
}

int pdmk_plan_create(const pdmk_opts* opts, const double* L, pdmk_plan** out) {
  if (!out || !L) return fail(PDMK_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  int st = validate_opts(opts);
  if (st) return st;
  for (int i = 0; i < opts->dim * opts->dim; ++i)
    if (!std::isfinite(L[i])) return fail(PDMK_ERR_SINGULAR_LATTICE, "non-finite lattice");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0)
    return fail(PDMK_ERR_NO_DEVICE, "no HIP device");
  pdmk_plan* P = new pdmk_plan();
  try {
    P->o = *opts;
    const int d = opts->dim;
    P->mp = resolve_params(opts);
    P->nufft_beta = P->mp.beta;
    P->P = &pswf_for_eps(opts->eps);
    P->T = &tables_for_eps(opts->eps);
    std::string msg = make_geometry(d, L, P->mp.kappa, P->P->c, P->mp.sigma, P->g,
                                    bloch_norm(opts), (opts->flags & PDMK_VIRTUAL_IMAGES) != 0);
    if (!msg.empty()) {
      delete P;
      return fail(geometry_status(msg), msg);
    }
    PDMK_HIP(hipGetDevice(&P->device));
    KParams& kp = P->kp;
    std::memset(&kp, 0, sizeof(kp));
    kp.dim = d;
    kp.p = P->mp.porder;
    kp.J = P->mp.npw;
    kp.rc = P->g.rc;
    kp.irc = 1.0 / P->g.rc;
    kp.precision = opts->precision;
    kp.vimg = P->g.virtual_images ? 1 : 0;
    int64_t nroot = 1;
    for (int a = 0; a < 3; ++a) {
      kp.next[a] = a < d ? P->g.next[a] : 1;
      kp.origin[a] = a < d ? P->g.origin[a] : 0.0;
      nroot *= kp.next[a];
    }
    int rootbits = 1;
    while ((1ll << rootbits) < nroot) ++rootbits;
    if (rootbits > 40) throw Error{PDMK_ERR_UNSUPPORTED, "root grid too large"};
    kp.B = std::min(d == 3 ? 20 : 30, (64 - rootbits) / d);
    for (int k = 0; k < 9; ++k) {
      kp.L[k] = P->g.L[k];
      kp.Li[k] = P->g.Li[k];
      kp.Q[k] = P->g.Q[k];
    }
    kp.w0unit = P->T->w0_unit(d);
    if (opts->flags & PDMK_BLOCH) {
      kp.bloch = 1;
      if (!oriented_bloch(P->g, opts, kp.beta))
        throw Error{PDMK_ERR_INVALID_ARG,
                    "Bloch vector in the reciprocal lattice: this is the periodic case"};
    }
    plan_upload_tables(P);
    if (d == 3) pw_mfma_upload(P);
    P->pw_mfma = !(opts->flags & PDMK_VECTOR_PLANE_WAVES);
    // stages in FP32 (mixed plans): the caller's mask, all by default; none
    // below eps = 1e-6, where FP32 rounding (about 6e-8 per operation, and the
    // FP32 residual series cut at 1e-8 of its largest coefficient) cannot
    // reach the tolerance
    P->mixed_parts = opts->fp32_stages ? (opts->fp32_stages & 15u) : 15u;
    if (opts->precision != PDMK_PREC_MIXED || opts->eps < kMixedEpsFloor) P->mixed_parts = 0;
    far_build_scale(P);
    PDMK_HIP(hipHostMalloc((void**)&P->h_cnt, 12 * sizeof(unsigned long long)));
  } catch (const Error& e) {
    free_plan_tables(P);
    delete P;
    return fail(e.code, e.msg);
  }
  *out = P;
  return PDMK_OK;
}

void pdmk_plan_destroy(pdmk_plan* P) {
  if (!P) return;
  unbind(P);
  free_plan_tables(P);
  delete P;
}

int pdmk_plan_geometry(const pdmk_plan* P, pdmk_geometry* out) {
  if (!P || !out) return fail(PDMK_ERR_INVALID_ARG, "null argument");
  std::memset(out, 0, sizeof(*out));
  const Geometry& g = P->g;
  out->dim = g.dim;
  for (int k = 0; k < g.dim * g.dim; ++k) {
    out->L_oriented[k] = g.L[k];
    out->Q[k] = g.Q[k];
  }
  for (int a = 0; a < g.dim; ++a) {
    out->perm[a] = g.perm[a];
    out->nroot[a] = g.nroot[a];
    out->origin[a] = g.origin[a];
    out->fgrid[a] = g.fgrid[a];
    out->fgrid_paper[a] = g.fgrid_paper[a];
  }
  out->volume = g.volume;
  out->rc = g.rc;
  out->n_shifts = (int)(g.shifts.size() / g.dim);
  out->c = P->P->c;
  out->w0_zero_rc = P->T->w0_unit(g.dim);
  out->porder = P->mp.porder;
  out->npw = P->mp.npw;
  out->nufft_w = P->mp.nufft_w;
  out->n_s = P->mp.n_s;
  out->nufft_beta = P->nufft_beta;
  out->kappa = P->mp.kappa;
  return PDMK_OK;
}

int pdmk_geometry_get(const pdmk_opts* opts, const double* L, pdmk_geometry* out) {
  if (!L || !out) return fail(PDMK_ERR_INVALID_ARG, "null argument");
  int st = validate_opts(opts);
  if (st) return st;
  pdmk_plan tmp;
  tmp.o = *opts;
  tmp.mp = resolve_params(opts);
  tmp.nufft_beta = tmp.mp.beta;
  tmp.P = &pswf_for_eps(opts->eps);
  tmp.T = &tables_for_eps(opts->eps);
  std::string msg = make_geometry(opts->dim, L, tmp.mp.kappa, tmp.P->c, tmp.mp.sigma, tmp.g,
                                  bloch_norm(opts), (opts->flags & PDMK_VIRTUAL_IMAGES) != 0);
  if (!msg.empty()) return fail(geometry_status(msg), msg);
  double ob[3];
  if ((opts->flags & PDMK_BLOCH) && !oriented_bloch(tmp.g, opts, ob))
    return fail(PDMK_ERR_INVALID_ARG,
                "Bloch vector in the reciprocal lattice: this is the periodic case");
  return pdmk_plan_geometry(&tmp, out);
}

int pdmk_plan_stats(const pdmk_plan* P, pdmk_stats* out) {
  if (!P || !out) return fail(PDMK_ERR_INVALID_ARG, "null argument");
  *out = P->last;
  return PDMK_OK;
}

}  // extern "C"

// One evaluation; `flags` replaces the plan's flags (PDMK_ALLOW_NONNEUTRAL is
// honoured, gradients are computed iff grad is not null).
// Sources + targets from which a call runs the far field's grid steps on a
// second stream.
constexpr int64_t kForkMin = 1 << 18;

// Tree kept by pdmk_plan_bind: the evaluation state after the list stage
// (sorted sources and targets, levels, lists, work items) in its own device
// memory, the map from sorted images to sources, the bound positions, and the
// execute workspace.
struct pdmk::BoundState {
  Eval E;                        // state after the lists (host copy of the level table)
  Workspace tree_ws;             // device memory of E (arena + overflow), owned
  char* tree_arena = nullptr;
  char* xarena = nullptr;        // execute workspace (sized at bind)
  size_t xarena_size = 0;
  std::vector<void*> pending;    // execute overflow blocks, freed at the next status
  size_t pending_need = 0;       // bytes the largest overflowing execute needed
  double* src0 = nullptr;        // bound positions (caller layout, n x d)
  double* trg0 = nullptr;
  double* sx0 = nullptr;         // bound sorted images, targets, originals (SoA)
  double* tx0 = nullptr;
  double* ox0 = nullptr;
  double* dsrc = nullptr;        // displacements (SoA) of a moved execute
  double* dtrg = nullptr;
  int* status_dev = nullptr;     // sticky device status bits of the executes
  bool moved = false;            // sorted arrays hold displaced positions
  hipStream_t last = nullptr;    // stream of the last execute
  unsigned flags = 0;
  ~BoundState() {
    tree_ws.release_overflow();
    for (void* p : pending) (void)hipFree(p);
    void* ptrs[] = {tree_arena, xarena, src0, trg0, sx0, tx0, ox0, dsrc, dtrg, status_dev};
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
  }
};

static void unbind(pdmk_plan* P) {
  if (!P->bound) return;
  if (P->bound->last) (void)hipStreamSynchronize(P->bound->last);
  if (P->s_aux) (void)hipStreamSynchronize(P->s_aux);
  delete P->bound;
  P->bound = nullptr;
}

// aux: the second stream of the call (null: the plan's own, created on first
// use; a batch worker passes its own).  keep: bind mode -- the call keeps its
// tree in a new BoundState (the workspace arena passes to it).
static int eval_impl(pdmk_plan* P, int64_t n_src, const double* src, const double* q,
                     int64_t n_trg, const double* trg, double* pot, double* grad, void* stream,
                     unsigned flags, char*& arena, size_t& arena_size,
                     hipStream_t aux = nullptr, BoundState** keep = nullptr,
                     bool noalloc = false, double* pot_far = nullptr) {
  if (!P) return fail(PDMK_ERR_INVALID_ARG, "null plan");
  if (P->kp.bloch)
    return fail(PDMK_ERR_UNSUPPORTED, "a Bloch plan evaluates with pdmk_plan_eval_bloch");
  const int d = P->g.dim;
  const bool self_t = (trg == nullptr);
  if (self_t) n_trg = n_src;
  const bool want_grad = grad != nullptr;
  if (n_src < 0 || n_trg < 0) return fail(PDMK_ERR_INVALID_ARG, "negative count");
  if (n_src > (int64_t)1 << 30 || n_trg > (int64_t)1 << 30)
    return fail(PDMK_ERR_INVALID_ARG, "more than 2^30 points");
  if ((n_src > 0 && (!src || !q)) || (n_trg > 0 && !pot))
    return fail(PDMK_ERR_INVALID_ARG, "null array");
  if (keep && (n_src == 0 || n_trg == 0))
    return fail(PDMK_ERR_INVALID_ARG, "binding needs sources and targets");
  hipStream_t s = (hipStream_t)stream;
  const auto wall0 = std::chrono::steady_clock::now();
  Workspace ws;
  ws.base = arena;
  ws.size = arena_size;
  ws.fixed = noalloc;
  Eval E;
  E.s = s;
  E.ws = &ws;
  E.n_src = n_src;
  E.n_trg = n_trg;
  E.self_targets = self_t;
  E.q = q;
  E.keep_map = keep != nullptr;
  E.timing = !noalloc;   // stage events only where the call may create them
  E.lib_gemm = !noalloc;
  E.det = (flags & PDMK_DETERMINISTIC) != 0;
  try {
    int cur = -1;
    PDMK_HIP(hipGetDevice(&cur));
    if (cur != P->device) throw Error{PDMK_ERR_INVALID_ARG, "plan bound to another device"};
    if (n_trg == 0) return PDMK_OK;
    if (n_src == 0) {
      PDMK_HIP(hipMemsetAsync(pot, 0, n_trg * sizeof(double), s));
      if (want_grad) PDMK_HIP(hipMemsetAsync(grad, 0, n_trg * d * sizeof(double), s));
      PDMK_HIP(hipStreamSynchronize(s));
      return PDMK_OK;
    }
    // the second stream pays off only for large inputs: for small ones the
    // fork's events and the extra stream's share of the hardware queues cost
    // more than the overlap (measured on batches of small cells)
    const bool fork = !noalloc && !(flags & PDMK_ONE_STREAM) && n_src + n_trg >= kForkMin;
    if (fork && !aux) {
      if (!P->s_aux) PDMK_HIP(hipStreamCreateWithFlags(&P->s_aux, hipStreamNonBlocking));
      aux = P->s_aux;
    }
    if (!fork) aux = s;
    P->ev_next = 0;
    E.plan = P;
    // timing events (none in the allocation-free mode, which creates nothing)
    const bool tm = E.timing;
    hipEvent_t ev[5] = {}, fev[3] = {};
    if (tm) {
      for (auto& e : ev) e = E.event();
      for (auto& e : fev) e = E.event();
      for (auto& e : E.far_ev) e = E.event();
    }
    auto record = [&](hipEvent_t e, hipStream_t st) {
      if (tm) PDMK_HIP(hipEventRecord(e, st));
    };
    record(ev[0], s);
    // input checks (charge sums, non-finite charges and positions) stay on
    // the device and are read after the call's final synchronisation; the
    // pipeline runs on sanitised data in between and the assembly writes
    // nothing for a rejected input
    double* qs = E.alloc<double>(2);
    E.d_flags = E.alloc<int>(2);
    fill_zero(E.d_flags, 2 * sizeof(int), s);
    {
      const int nb = std::min(1024, nblk(n_src, 256));
      double* part = E.alloc<double>(2 * nb);
      hipLaunchKernelGGL(k_charge_stats, dim3(nb), dim3(256), 0, s, n_src, q, part, E.d_flags);
      hipLaunchKernelGGL(k_charge_stats_final, dim3(1), dim3(256), 0, s, nb, part, qs);
    }
    E.qsum = qs;
    stage_prepare(P, E, src, trg);
    stage_images(P, E, q);
    // the far field's grid steps need only the sorted sources: they run on
    // the plan's second stream beside the tree, lists and near field, and are
    // joined before the interpolation (which adds into pot_sorted).  A bind
    // builds the tree first, so that everything allocated after the lists is
    // the state an execute rebuilds.
    auto far_fork = [&]() {
      if (fork) {
        PDMK_HIP(hipEventRecord(fev[0], s));
        PDMK_HIP(hipStreamWaitEvent(aux, fev[0], 0));
      }
      record(fev[1], aux);
      E.s = aux;
      stage_far_grid(P, E);
      E.s = s;
      record(fev[2], aux);
    };
    if (!keep) far_fork();
    // residual pairs evaluated once where the call allows it (a kept tree of
    // a plan made with PDMK_WANT_GRAD keeps both-way lists: its executes may
    // ask for gradients; one of another plan rejects such executes)
    E.sym = self_t && !want_grad && !E.det && E.img_trg != nullptr &&
            !(flags & PDMK_ALL_PAIRS) && (!keep || !(flags & PDMK_WANT_GRAD));
    stage_tree(P, E);
    stage_lists(P, E);
    const size_t mark = ws.used;
    Eval kept;
    if (keep) {
      kept = E;   // the state an execute starts from
      far_fork();
    }
    record(ev[1], s);
    stage_near(P, E, want_grad);
    record(ev[2], s);
    if (fork) PDMK_HIP(hipStreamWaitEvent(s, fev[2], 0));
    if (pot_far) E.far_out = E.alloc<double>(n_trg);
    stage_far_interp(P, E, want_grad);
    record(ev[3], s);
    // uniform-background constant: the method with m = 0 dropped returns the
    // tin-foil potential plus (sum q) * Rhat_0(0) / V
    const double cc = P->P->c;
    const double cnn = -P->P->psit_dd0 * P->g.rc * P->g.rc / (2.0 * cc * cc * P->g.volume);
    hipLaunchKernelGGL(k_assemble, dim3(nblk(n_trg, 256)), dim3(256), 0, s, n_trg, d, E.tperm,
                       E.pot_sorted, E.grad_sorted, qs, E.d_flags, cnn,
                       (flags & PDMK_ALLOW_NONNEUTRAL) ? 1 : 0, P->kp, pot,
                       want_grad ? grad : nullptr);
    if (pot_far)
      hipLaunchKernelGGL(k_assemble, dim3(nblk(n_trg, 256)), dim3(256), 0, s, n_trg, d,
                         E.tperm, E.far_out, nullptr, qs, E.d_flags, 0.0,
                         (flags & PDMK_ALLOW_NONNEUTRAL) ? 1 : 0, P->kp, pot_far, nullptr);
    PDMK_HIP(hipMemcpyAsync(P->h_cnt + 4, qs, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    PDMK_HIP(hipMemcpyAsync(P->h_cnt + 6, E.d_flags, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    float t1 = 0, t2 = 0, t3 = 0, t4 = 0, tg = 0;
    if (tm) {
      PDMK_HIP(hipEventRecord(ev[4], s));
      PDMK_HIP(hipEventSynchronize(ev[4]));
      near_finish(P, E);
      PDMK_HIP(hipEventElapsedTime(&t1, ev[0], ev[1]));
      PDMK_HIP(hipEventElapsedTime(&t2, ev[1], ev[2]));
      PDMK_HIP(hipEventElapsedTime(&t3, ev[2], ev[3]));
      PDMK_HIP(hipEventElapsedTime(&t4, ev[0], ev[4]));
      PDMK_HIP(hipEventElapsedTime(&tg, fev[1], fev[2]));
      t3 += tg;   // far field: grid steps (overlapped with the build and near field) + interpolation
      float a = 0, b = 0, c = 0;
      PDMK_HIP(hipEventElapsedTime(&a, E.far_ev[0], E.far_ev[1]));
      PDMK_HIP(hipEventElapsedTime(&b, E.far_ev[1], E.far_ev[2]));
      PDMK_HIP(hipEventElapsedTime(&c, E.far_ev[3], E.far_ev[4]));
      E.st.t_spread_ms = a;
      E.st.t_fft_ms = b;
      E.st.t_interp_ms = c;
    } else {
      PDMK_HIP(hipStreamSynchronize(s));
    }
    {
      double hq[2];
      int hf[2];
      std::memcpy(hq, P->h_cnt + 4, sizeof(hq));
      std::memcpy(hf, P->h_cnt + 6, sizeof(hf));
      if (hf[0]) throw Error{PDMK_ERR_NONFINITE, "non-finite charge"};
      if (hf[1]) throw Error{PDMK_ERR_NONFINITE, "non-finite position"};
      if (std::fabs(hq[0]) > 1e-8 * hq[1] && !(flags & PDMK_ALLOW_NONNEUTRAL))
        throw Error{PDMK_ERR_NOT_NEUTRAL, "sum of charges is not zero"};
    }
    E.st.n_src = n_src;
    E.st.n_trg = n_trg;
    E.st.n_images = E.n_img;
    {
      // length of the series the residual kernel evaluated
      const bool f32 = P->kp.precision == PDMK_PREC_MIXED && (P->mixed_parts & 1);
      E.st.series_len = d == 3 ? (f32 ? P->kp.nE32 : P->kp.nE) : (f32 ? P->kp.nF232 : P->kp.nF2);
      E.st.pairs_once = E.sym ? 1 : 0;
    }
    E.st.t_build_ms = t1;
    E.st.t_near_ms = t2;
    E.st.t_far_ms = t3;
    E.st.t_total_ms = t4;
    P->last = E.st;
    PDMK_HIP(hipStreamSynchronize(s));
    if (keep) {
      // the workspace (arena and overflow blocks) now holds the kept tree
      BoundState* B = new BoundState();
      *keep = B;
      B->E = kept;
      B->E.lib_gemm = false;   // executes only enqueue kernels (graph-capturable)
      B->tree_ws.overflow.swap(ws.overflow);
      B->tree_arena = arena;
      arena = nullptr;
      arena_size = 0;
      B->flags = flags;
      // an execute allocates what this call allocated after the lists, plus
      // its charge sums and (whether or not this call had them) gradients
      size_t need = ws.used - mark + 2 * 1024 * sizeof(double) + 8 * 256 +
                    (want_grad ? 0 : (size_t)n_trg * d * sizeof(double) + 256);
      PDMK_HIP(hipMalloc((void**)&B->xarena, need));
      B->xarena_size = need;
      P->last.workspace_bytes = (int64_t)(ws.used + need);
    } else if (!noalloc) {
      finish_workspace(arena, arena_size, ws);
      P->last.workspace_bytes = (int64_t)ws.used;
    } else {
      P->last.workspace_bytes = (int64_t)ws.used;
    }
    P->last.t_call_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - wall0)
            .count();
  } catch (const Error& e) {
    (void)hipStreamSynchronize(s);
    if (aux) (void)hipStreamSynchronize(aux);   // far-field steps forked before the error
    ws.release_overflow();
    return fail(e.code, e.msg);
  }
  return PDMK_OK;
}

// ------------------------------------------------------------ Bloch conditions
// Phi(x_w) = near_re + i near_im + e^{i beta.x_w} (far_re + i far_im) at the
// sorted (wrapped) targets, carried back to the given target by the phase of
// its wrap, Phi(x) = e^{-i theta} Phi(x_w) (Section 4.1: post-modulation and
// quasi-periodicity); written as (real, imaginary) pairs in the caller's order.
__global__ void k_assemble_bloch(KParams kp, int64_t n, const int* __restrict__ tperm,
                                 const double* __restrict__ tx, const double* __restrict__ nr,
                                 const double* __restrict__ ni, const double* __restrict__ fr,
                                 const double* __restrict__ fi,
                                 const double* __restrict__ theta_t,
                                 const int* __restrict__ flags, double* __restrict__ pot) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  if (flags[0] || flags[1]) return;
  double ph = 0.0;
  for (int a = 0; a < kp.dim; ++a) ph += kp.beta[a] * tx[a * n + t];
  double sn, cs;
  sincos(ph, &sn, &cs);
  const double re = nr[t] + (cs * fr[t] - sn * fi[t]);
  const double im = ni[t] + (sn * fr[t] + cs * fi[t]);
  const int o = tperm[t];
  double s2, c2;
  sincos(theta_t[o], &s2, &c2);
  pot[2 * (int64_t)o] = re * c2 + im * s2;
  pot[2 * (int64_t)o + 1] = im * c2 - re * s2;
}

// One Bloch evaluation: the periodic pipeline with phased image charges, two
// real near fields (real and imaginary parts of the image charges) and the
// modulated far field of eq:qp_far; every stage on the caller's stream.
static int bloch_impl(pdmk_plan* P, int64_t n_src, const double* src, const double* q,
                      int64_t n_trg, const double* trg, double* pot, void* stream) {
  if (!P) return fail(PDMK_ERR_INVALID_ARG, "null plan");
  if (!P->kp.bloch) return fail(PDMK_ERR_INVALID_ARG, "the plan was made without PDMK_BLOCH");
  const int d = P->g.dim;
  const bool self_t = (trg == nullptr);
  if (self_t) n_trg = n_src;
  if (n_src < 0 || n_trg < 0) return fail(PDMK_ERR_INVALID_ARG, "negative count");
  if (n_src > (int64_t)1 << 30 || n_trg > (int64_t)1 << 30)
    return fail(PDMK_ERR_INVALID_ARG, "more than 2^30 points");
  if ((n_src > 0 && (!src || !q)) || (n_trg > 0 && !pot))
    return fail(PDMK_ERR_INVALID_ARG, "null array");
  hipStream_t s = (hipStream_t)stream;
  const auto wall0 = std::chrono::steady_clock::now();
  Workspace ws;
  ws.base = P->arena;
  ws.size = P->arena_size;
  Eval E;
  E.s = s;
  E.ws = &ws;
  E.plan = P;
  E.n_src = n_src;
  E.n_trg = n_trg;
  E.self_targets = self_t;
  E.q = q;
  E.timing = false;
  try {
    int cur = -1;
    PDMK_HIP(hipGetDevice(&cur));
    if (cur != P->device) throw Error{PDMK_ERR_INVALID_ARG, "plan bound to another device"};
    if (n_trg == 0) return PDMK_OK;
    if (n_src == 0) {
      fill_zero(pot, 2 * n_trg * sizeof(double), s);
      PDMK_HIP(hipStreamSynchronize(s));
      return PDMK_OK;
    }
    P->ev_next = 0;
    double* qs = E.alloc<double>(2);
    E.d_flags = E.alloc<int>(2);
    fill_zero(E.d_flags, 2 * sizeof(int), s);
    {
      const int nb = std::min(1024, nblk(n_src, 256));
      double* part = E.alloc<double>(2 * nb);
      hipLaunchKernelGGL(k_charge_stats, dim3(nb), dim3(256), 0, s, n_src, q, part, E.d_flags);
      hipLaunchKernelGGL(k_charge_stats_final, dim3(1), dim3(256), 0, s, nb, part, qs);
    }
    E.qsum = qs;
    stage_prepare(P, E, src, trg);
    stage_images(P, E, q);   // wrapped complex charges and phased images
    stage_far_grid(P, E);    // pre-modulated charges, shifted-mode scaling
    stage_tree(P, E);
    // residual pairs evaluated once: each pass is a plain sum over the phased
    // image charges (the targets are modulated afterwards), and a target's
    // charge as a source is its unshifted image's (oq / oq_im)
    E.sym = self_t && E.img_trg != nullptr && E.oq_im != nullptr &&
            !(P->o.flags & PDMK_ALL_PAIRS);
    stage_lists(P, E);
    // the near field is real-linear in the charges: one pass per part
    double* sq_re = E.sq;
    const double* q_re = E.q;
    double* oq_re = E.oq;
    stage_near(P, E, false);
    double* near_re = E.pot_sorted;
    E.sq = E.sq_im;
    E.q = E.q_im;
    E.oq = E.oq_im;
    stage_near(P, E, false);
    double* near_im = E.pot_sorted;
    E.sq = sq_re;
    E.q = q_re;
    E.oq = oq_re;
    double* far_re = E.alloc<double>(n_trg);
    double* far_im = E.alloc<double>(n_trg);
    E.far_out = far_re;
    E.far_comp = 0;
    stage_far_interp(P, E, false);
    E.far_out = far_im;
    E.far_comp = 1;
    stage_far_interp(P, E, false);
    hipLaunchKernelGGL(k_assemble_bloch, dim3(nblk(n_trg, 256)), dim3(256), 0, s, P->kp, n_trg,
                       E.tperm, E.tx, near_re, near_im, far_re, far_im, E.theta_t, E.d_flags,
                       pot);
    PDMK_HIP(hipGetLastError());
    PDMK_HIP(hipMemcpyAsync(P->h_cnt + 6, E.d_flags, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    PDMK_HIP(hipStreamSynchronize(s));
    int hf[2];
    std::memcpy(hf, P->h_cnt + 6, sizeof(hf));
    if (hf[0]) throw Error{PDMK_ERR_NONFINITE, "non-finite charge"};
    if (hf[1]) throw Error{PDMK_ERR_NONFINITE, "non-finite position"};
    E.st.n_src = n_src;
    E.st.n_trg = n_trg;
    E.st.n_images = E.n_img;
    E.st.pairs_once = E.sym ? 1 : 0;
    P->last = E.st;
    finish_workspace(P->arena, P->arena_size, ws);
    P->last.workspace_bytes = (int64_t)ws.used;
    P->last.t_call_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - wall0)
            .count();
  } catch (const Error& e) {
    (void)hipStreamSynchronize(s);
    ws.release_overflow();
    return fail(e.code, e.msg);
  }
  return PDMK_OK;
}

// ------------------------------------------------- allocation-free entry
// The workspace of pdmk_plan_eval_noalloc: one fixed array per device (each
// device holds its own copy from the code object's load until the process
// ends).  Host code must not use the array's name as a device address: the
// address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[PDMK_NOALLOC_SCRATCH_BYTES];

struct ScratchSlot {
  std::mutex mu;             // held for a whole call: calls on one device do not overlap
  char* ptr = nullptr;       // device address of this device's copy of scratch
};

static ScratchSlot& scratch_slot(int dev) {
  static std::mutex mu;
  static std::map<int, ScratchSlot> slots;
  std::lock_guard<std::mutex> lock(mu);
  return slots[dev];   // node-based map: the reference stays valid
}

// ------------------------------------------------------ kept-tree execute
// d[a * n + i] = Q^T (x[i] - x0[i]) (oriented displacement); flags a
// non-finite position
__global__ void k_displacement(KParams kp, int64_t n, const double* __restrict__ x,
                               const double* __restrict__ x0, double* __restrict__ dsp,
                               int* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int d = kp.dim;
  double v[3] = {0, 0, 0};
  bool ok = true;
  for (int a = 0; a < d; ++a) {
    v[a] = x[i * d + a] - x0[i * d + a];
    ok = ok && isfinite(v[a]);
  }
  if (!ok) {
    atomicOr(bad, 1);
    for (int a = 0; a < d; ++a) v[a] = 0.0;
  }
  for (int a = 0; a < d; ++a) {
    double s = 0;
    for (int b = 0; b < d; ++b) s += kp.Q[b + d * a] * v[b];
    dsp[a * n + i] = s;
  }
}

// out[a * m + k] = base[a * m + k] + dsp[a * n + map[k]] (dsp == null: base)
__global__ void k_displace(int64_t m, int d, const int* __restrict__ map,
                           const double* __restrict__ base, const double* __restrict__ dsp,
                           int64_t n, double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const int j = dsp ? map[k] : 0;
  for (int a = 0; a < d; ++a)
    out[a * m + k] = base[a * m + k] + (dsp ? dsp[a * n + j] : 0.0);
}

// out[k] = q[map[k]]
__global__ void k_gather_q(int64_t m, const int* __restrict__ map, const double* __restrict__ q,
                           double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) out[k] = q[map[k]];
}

// status bits of one execute, kept until pdmk_plan_status reads them:
// 1 non-finite charge, 2 non-finite position, 4 charges not neutral
__global__ void k_status_accum(const int* __restrict__ flags, const double* __restrict__ qs,
                               int allow_nonneutral, int* __restrict__ status) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int v = status[0];
  if (flags[0]) v |= 1;
  if (flags[1]) v |= 2;
  if (!allow_nonneutral && fabs(qs[0]) > 1e-8 * qs[1]) v |= 4;
  status[0] = v;
}

static int execute_impl(pdmk_plan* P, const double* src, const double* trg, const double* q,
                        double* pot, double* grad, hipStream_t s) {
  BoundState& B = *P->bound;
  const int d = P->g.dim;
  Eval E = B.E;
  Workspace xws;
  xws.base = B.xarena;
  xws.size = B.xarena_size;
  E.ws = &xws;
  E.s = s;
  E.plan = P;
  E.timing = false;
  E.q = q;
  E.st = pdmk_stats{};
  E.det = (B.flags & PDMK_DETERMINISTIC) != 0;
  const bool want_grad = grad != nullptr;
  if (want_grad && E.sym)
    return fail(PDMK_ERR_UNSUPPORTED,
                "the tree was bound for potentials (residual pairs evaluated once); bind on "
                "a plan made with PDMK_WANT_GRAD to execute with gradients");
  const int64_t n = E.n_src, m = E.n_trg;
  const bool fork = n + m >= kForkMin;
  hipStream_t aux = fork ? P->s_aux : s;
  try {
    if (fork && !aux) throw Error{PDMK_ERR_INVALID_ARG, "plan has no second stream"};
    P->ev_next = 0;
    double* qs = E.alloc<double>(2);
    E.d_flags = E.alloc<int>(2);
    fill_zero(E.d_flags, 2 * sizeof(int), s);
    {
      const int nb = std::min(1024, nblk(n, 256));
      double* part = E.alloc<double>(2 * nb);
      hipLaunchKernelGGL(k_charge_stats, dim3(nb), dim3(256), 0, s, n, q, part, E.d_flags);
      hipLaunchKernelGGL(k_charge_stats_final, dim3(1), dim3(256), 0, s, nb, part, qs);
    }
    E.qsum = qs;
    // positions: the bound ones, or displaced from them on the kept tree
    const bool move = src != nullptr || (trg != nullptr && !E.self_targets);
    if (move || B.moved) {
      const double* ds = nullptr;
      const double* dt = nullptr;
      if (src) {
        hipLaunchKernelGGL(k_displacement, dim3(nblk(n, 256)), dim3(256), 0, s, P->kp, n, src,
                           B.src0, B.dsrc, E.d_flags + 1);
        ds = B.dsrc;
      }
      if (E.self_targets) dt = ds;
      else if (trg) {
        hipLaunchKernelGGL(k_displacement, dim3(nblk(m, 256)), dim3(256), 0, s, P->kp, m, trg,
                           B.trg0, B.dtrg, E.d_flags + 1);
        dt = B.dtrg;
      }
      hipLaunchKernelGGL(k_displace, dim3(nblk(E.n_img, 256)), dim3(256), 0, s, E.n_img, d,
                         E.img_src, B.sx0, ds, n, E.sx);
      hipLaunchKernelGGL(k_displace, dim3(nblk(m, 256)), dim3(256), 0, s, m, d, E.tperm, B.tx0,
                         dt, m, E.tx);
      if (!E.self_targets)
        hipLaunchKernelGGL(k_displace, dim3(nblk(n, 256)), dim3(256), 0, s, n, d, E.operm,
                           B.ox0, ds, n, E.ox);
      B.moved = move;
    }
    // charges of the sorted images and of the originals in tree order
    hipLaunchKernelGGL(k_gather_q, dim3(nblk(E.n_img, 256)), dim3(256), 0, s, E.n_img,
                       E.img_src, q, E.sq);
    hipLaunchKernelGGL(k_gather_q, dim3(nblk(n, 256)), dim3(256), 0, s, n,
                       E.self_targets ? E.tperm : E.operm, q, E.oq);
    hipEvent_t f0 = nullptr, f1 = nullptr;
    if (fork) {
      f0 = E.event();
      f1 = E.event();
      PDMK_HIP(hipEventRecord(f0, s));
      PDMK_HIP(hipStreamWaitEvent(aux, f0, 0));
    }
    E.s = aux;
    stage_far_grid(P, E);
    E.s = s;
    if (fork) PDMK_HIP(hipEventRecord(f1, aux));
    stage_near(P, E, want_grad);
    if (fork) PDMK_HIP(hipStreamWaitEvent(s, f1, 0));
    stage_far_interp(P, E, want_grad);
    const double cc = P->P->c;
    const double cnn = -P->P->psit_dd0 * P->g.rc * P->g.rc / (2.0 * cc * cc * P->g.volume);
    const int allow = (B.flags & PDMK_ALLOW_NONNEUTRAL) ? 1 : 0;
    hipLaunchKernelGGL(k_assemble, dim3(nblk(m, 256)), dim3(256), 0, s, m, d, E.tperm,
                       E.pot_sorted, E.grad_sorted, qs, E.d_flags, cnn, allow, P->kp, pot,
                       want_grad ? grad : nullptr);
    hipLaunchKernelGGL(k_status_accum, dim3(1), dim3(64), 0, s, E.d_flags, qs, allow,
                       B.status_dev);
    PDMK_HIP(hipGetLastError());
    B.last = s;
    if (!xws.overflow.empty()) {
      // more than the bind measured (should not happen): keep the blocks
      // until the stream has finished, then grow the workspace
      for (void* p : xws.overflow) B.pending.push_back(p);
      xws.overflow.clear();
      B.pending_need = std::max(B.pending_need, xws.used);
    }
  } catch (const Error& e) {
    (void)hipStreamSynchronize(s);
    if (aux) (void)hipStreamSynchronize(aux);
    xws.release_overflow();
    return fail(e.code, e.msg);
  }
  return PDMK_OK;
}

__global__ void k_copy_soa(int64_t n, const double* __restrict__ in, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i];
}

extern "C" {

int pdmk_plan_eval(pdmk_plan* P, int64_t n_src, const double* src, const double* q,
                   int64_t n_trg, const double* trg, double* pot, double* grad, void* stream) {
  if (!P) return fail(PDMK_ERR_INVALID_ARG, "null plan");
  return eval_impl(P, n_src, src, q, n_trg, trg, pot, grad, stream, P->o.flags, P->arena,
                   P->arena_size);
}

int pdmk_plan_eval_bloch(pdmk_plan* P, int64_t n_src, const double* src, const double* q,
                         int64_t n_trg, const double* trg, double* pot, void* stream) {
  return bloch_impl(P, n_src, src, q, n_trg, trg, pot, stream);
}

int pdmk_plan_eval_parts(pdmk_plan* P, int64_t n_src, const double* src, const double* q,
                         int64_t n_trg, const double* trg, double* pot_near, double* pot_far,
                         void* stream) {
  if (!P) return fail(PDMK_ERR_INVALID_ARG, "null plan");
  if ((trg ? n_trg : n_src) > 0 && (!pot_near || !pot_far))
    return fail(PDMK_ERR_INVALID_ARG, "null output");
  return eval_impl(P, n_src, src, q, n_trg, trg, pot_near, nullptr, stream, P->o.flags,
                   P->arena, P->arena_size, nullptr, nullptr, false, pot_far);
}

int pdmk_plan_eval_noalloc(pdmk_plan* P, int64_t n_src, const double* src, const double* q,
                           int64_t n_trg, const double* trg, double* pot, double* grad,
                           void* stream) {
  if (!P) return fail(PDMK_ERR_INVALID_ARG, "null plan");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(PDMK_ERR_HIP, "hipGetDevice failed");
  if (dev != P->device) return fail(PDMK_ERR_INVALID_ARG, "plan bound to another device");
  // a lower bound of the workspace: wrapped and fractional positions, sorted
  // copies, keys and permutations of every source and target
  const int64_t nt = trg ? n_trg : n_src;
  const int d = P->g.dim;
  const int64_t low = (n_src + nt) * (int64_t)(4 * d * sizeof(double) + 24);
  if (low > (int64_t)PDMK_NOALLOC_SCRATCH_BYTES)
    return fail(PDMK_ERR_SCRATCH, "the input needs more than the " +
                                      std::to_string(PDMK_NOALLOC_SCRATCH_BYTES >> 20) +
                                      " MiB of device scratch of the allocation-free entry point");
  ScratchSlot& slot = scratch_slot(dev);
  std::lock_guard<std::mutex> lock(slot.mu);
  if (!slot.ptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(PDMK_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                    hipGetErrorString(e));
    slot.ptr = static_cast<char*>(p);
  }
  char* base = slot.ptr;
  size_t size = PDMK_NOALLOC_SCRATCH_BYTES;
  return eval_impl(P, n_src, src, q, n_trg, trg, pot, grad, stream, P->o.flags, base, size,
                   nullptr, nullptr, true);
}

int pdmk_plan_bind(pdmk_plan* P, int64_t n_src, const double* src, const double* q,
                   int64_t n_trg, const double* trg, double* pot, double* grad, void* stream) {
  if (!P) return fail(PDMK_ERR_INVALID_ARG, "null plan");
  unbind(P);
  const int d = P->g.dim;
  BoundState* B = nullptr;
  int st = eval_impl(P, n_src, src, q, n_trg, trg, pot, grad, stream, P->o.flags, P->arena,
                     P->arena_size, nullptr, &B);
  if (st != PDMK_OK) return st;
  P->bound = B;
  try {
    Eval& E = B->E;
    const int64_t n = E.n_src, m = E.n_trg;
    hipStream_t s = (hipStream_t)stream;
    // bound positions: the caller's arrays and the sorted arrays they made
    PDMK_HIP(hipMalloc((void**)&B->src0, (size_t)n * d * sizeof(double)));
    PDMK_HIP(hipMemcpyAsync(B->src0, src, (size_t)n * d * sizeof(double),
                            hipMemcpyDeviceToDevice, s));
    PDMK_HIP(hipMalloc((void**)&B->dsrc, (size_t)n * d * sizeof(double)));
    PDMK_HIP(hipMalloc((void**)&B->sx0, (size_t)E.n_img * d * sizeof(double)));
    hipLaunchKernelGGL(k_copy_soa, dim3(nblk(E.n_img * d, 256)), dim3(256), 0, s, E.n_img * d,
                       E.sx, B->sx0);
    PDMK_HIP(hipMalloc((void**)&B->tx0, (size_t)m * d * sizeof(double)));
    hipLaunchKernelGGL(k_copy_soa, dim3(nblk(m * d, 256)), dim3(256), 0, s, m * d, E.tx, B->tx0);
    if (!E.self_targets) {
      PDMK_HIP(hipMalloc((void**)&B->trg0, (size_t)m * d * sizeof(double)));
      PDMK_HIP(hipMemcpyAsync(B->trg0, trg, (size_t)m * d * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
      PDMK_HIP(hipMalloc((void**)&B->dtrg, (size_t)m * d * sizeof(double)));
      PDMK_HIP(hipMalloc((void**)&B->ox0, (size_t)n * d * sizeof(double)));
      hipLaunchKernelGGL(k_copy_soa, dim3(nblk(n * d, 256)), dim3(256), 0, s, n * d, E.ox,
                         B->ox0);
    }
    PDMK_HIP(hipMalloc((void**)&B->status_dev, sizeof(int)));
    PDMK_HIP(hipMemsetAsync(B->status_dev, 0, sizeof(int), s));
    if (n + m >= kForkMin && !P->s_aux)
      PDMK_HIP(hipStreamCreateWithFlags(&P->s_aux, hipStreamNonBlocking));
    PDMK_HIP(hipStreamSynchronize(s));
  } catch (const Error& e) {
    unbind(P);
    return fail(e.code, e.msg);
  }
  return PDMK_OK;
}

int pdmk_plan_execute(pdmk_plan* P, const double* src, const double* trg, const double* q,
                      double* pot, double* grad, void* stream) {
  if (!P) return fail(PDMK_ERR_INVALID_ARG, "null plan");
  if (!P->bound) return fail(PDMK_ERR_INVALID_ARG, "no bound tree (call pdmk_plan_bind)");
  if (!q || !pot) return fail(PDMK_ERR_INVALID_ARG, "null array");
  if (trg && P->bound->E.self_targets)
    return fail(PDMK_ERR_INVALID_ARG, "the bound targets are the sources");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != P->device)
    return fail(PDMK_ERR_INVALID_ARG, "plan bound to another device");
  return execute_impl(P, src, trg, q, pot, grad, (hipStream_t)stream);
}

int pdmk_plan_status(pdmk_plan* P) {
  if (!P) return fail(PDMK_ERR_INVALID_ARG, "null plan");
  BoundState* B = P->bound;
  if (!B) return fail(PDMK_ERR_INVALID_ARG, "no bound tree");
  int v = 0;
  try {
    if (B->last) PDMK_HIP(hipStreamSynchronize(B->last));
    if (P->s_aux) PDMK_HIP(hipStreamSynchronize(P->s_aux));
    PDMK_HIP(hipMemcpy(&v, B->status_dev, sizeof(int), hipMemcpyDeviceToHost));
    PDMK_HIP(hipMemset(B->status_dev, 0, sizeof(int)));
    if (!B->pending.empty()) {
      for (void* p : B->pending) (void)hipFree(p);
      B->pending.clear();
      const size_t want = B->pending_need + B->pending_need / 8;
      (void)hipFree(B->xarena);
      B->xarena = nullptr;
      B->xarena_size = 0;
      PDMK_HIP(hipMalloc((void**)&B->xarena, want));
      B->xarena_size = want;
    }
  } catch (const Error& e) {
    return fail(e.code, e.msg);
  }
  if (v & 1) return fail(PDMK_ERR_NONFINITE, "non-finite charge");
  if (v & 2) return fail(PDMK_ERR_NONFINITE, "non-finite position");
  if (v & 4) return fail(PDMK_ERR_NOT_NEUTRAL, "sum of charges is not zero");
  return PDMK_OK;
}

void pdmk_plan_unbind(pdmk_plan* P) {
  if (P) unbind(P);
}

int pdmk_plan_adjoint(pdmk_plan* P, int64_t n_src, const double* src, const double* q,
                      int64_t n_trg, const double* trg, const double* g, const double* grad_phi,
                      double* dq, double* dsrc, double* dtrg, void* stream) {
  if (!P) return fail(PDMK_ERR_INVALID_ARG, "null plan");
  const int d = P->g.dim;
  const bool self_t = trg == nullptr;
  if (self_t) n_trg = n_src;
  if (n_src < 0 || n_trg < 0) return fail(PDMK_ERR_INVALID_ARG, "negative count");
  if (n_src > 0 && !src) return fail(PDMK_ERR_INVALID_ARG, "null src");
  if (n_trg > 0 && !g) return fail(PDMK_ERR_INVALID_ARG, "null g");
  if (dsrc && n_src > 0 && !q) return fail(PDMK_ERR_INVALID_ARG, "dsrc needs q");
  if (((dsrc && self_t) || (dtrg && !self_t)) && n_trg > 0 && !grad_phi)
    return fail(PDMK_ERR_INVALID_ARG, "grad_phi is needed for the position adjoint");
  if (dtrg && self_t) return fail(PDMK_ERR_INVALID_ARG, "dtrg needs separate targets");
  hipStream_t s = (hipStream_t)stream;
  try {
    int cur = -1;
    PDMK_HIP(hipGetDevice(&cur));
    if (cur != P->device) throw Error{PDMK_ERR_INVALID_ARG, "plan bound to another device"};
    // Psi and grad Psi at the sources: the potential of the charges g placed
    // at the targets (the kernel is symmetric), uniform background allowed
    const size_t need = (size_t)n_src * (d + 1);
    if (need > P->adj_size) {
      if (P->adj_buf) PDMK_HIP(hipFree(P->adj_buf));
      P->adj_buf = nullptr;
      P->adj_size = 0;
      PDMK_HIP(hipMalloc((void**)&P->adj_buf, need * sizeof(double)));
      P->adj_size = need;
    }
    double* psi = P->adj_buf;
    double* gpsi = P->adj_buf + n_src;
    if (n_src > 0) {
      const int st = self_t ? eval_impl(P, n_src, src, g, 0, nullptr, psi, dsrc ? gpsi : nullptr,
                                        stream, PDMK_ALLOW_NONNEUTRAL, P->arena, P->arena_size)
                            : eval_impl(P, n_trg, trg, g, n_src, src, psi,
                                        dsrc ? gpsi : nullptr, stream, PDMK_ALLOW_NONNEUTRAL,
                                        P->arena, P->arena_size);
      if (st != PDMK_OK) return st;
    }
    const int64_t nmax = std::max(n_src, n_trg);
    if (nmax > 0)
      hipLaunchKernelGGL(k_adjoint_combine, dim3(nblk(nmax, 256)), dim3(256), 0, s, n_src,
                         n_trg, d, q, g, grad_phi, self_t ? 1 : 0, psi, gpsi, dq, dsrc, dtrg);
    PDMK_HIP(hipGetLastError());
    PDMK_HIP(hipStreamSynchronize(s));
  } catch (const Error& e) {
    (void)hipStreamSynchronize(s);
    return fail(e.code, e.msg);
  }
  return PDMK_OK;
}

int pdmk_eval(const pdmk_opts* opts, const double* L, int64_t n_src, const double* src,
              const double* q, int64_t n_trg, const double* trg, double* pot, double* grad,
              void* stream) {
  if (opts && (opts->flags & PDMK_WANT_GRAD) && !grad && (trg ? n_trg : n_src) > 0)
    return fail(PDMK_ERR_INVALID_ARG, "PDMK_WANT_GRAD set but grad is null");
  pdmk_plan* P = nullptr;
  int st = pdmk_plan_create(opts, L, &P);
  if (st) return st;
  st = pdmk_plan_eval(P, n_src, src, q, n_trg, trg, pot, grad, stream);
  pdmk_plan_destroy(P);
  return st;
}

// ------------------------------------------------------------------ batches
// Many independent systems: one plan per system, evaluated by a pool of host
// workers, each with its own HIP stream and device workspace, so that the
// small per-system pipelines of different systems overlap on the GPU.
struct pdmk_batch {
  pdmk_opts o{};
  int device = 0;
  std::vector<pdmk_plan*> plans;
  std::vector<double> L;          // lattices, d x d per system (column-major)
  std::vector<hipStream_t> streams;
  std::vector<hipStream_t> aux;   // each worker's second stream
  std::vector<char*> arenas;
  std::vector<size_t> arena_sizes;
  // kept trees of every system (pdmk_batch_bind): the bound offsets, and the
  // fork / join events of an execute over the worker streams
  std::vector<int64_t> bound_off;
  hipEvent_t ev_fork = nullptr;
  std::vector<hipEvent_t> ev_join;
};

int pdmk_batch_create(const pdmk_opts* opts, int n_sys, const double* L, int n_workers,
                      pdmk_batch** out) {
  if (!opts || !L || !out || n_sys < 0) return fail(PDMK_ERR_INVALID_ARG, "null argument");
  const int d = opts->dim;
  if (d != 2 && d != 3) return fail(PDMK_ERR_INVALID_ARG, "dim must be 2 or 3");
  pdmk_batch* B = new pdmk_batch;
  B->o = *opts;
  B->L.assign(L, L + (size_t)n_sys * d * d);
  try {
    PDMK_HIP(hipGetDevice(&B->device));
    for (int sy = 0; sy < n_sys; ++sy) {
      pdmk_plan* P = nullptr;
      const int st = pdmk_plan_create(opts, L + (size_t)sy * d * d, &P);
      if (st) {
        pdmk_batch_destroy(B);
        return st;
      }
      B->plans.push_back(P);
    }
    const int nw = std::max(1, std::min(n_workers > 0 ? n_workers : 8, std::max(1, n_sys)));
    for (int w = 0; w < nw; ++w) {
      hipStream_t st = nullptr, sa = nullptr;
      PDMK_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      B->streams.push_back(st);
      PDMK_HIP(hipStreamCreateWithFlags(&sa, hipStreamNonBlocking));
      B->aux.push_back(sa);
      B->arenas.push_back(nullptr);
      B->arena_sizes.push_back(0);
      hipEvent_t ev = nullptr;
      PDMK_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      B->ev_join.push_back(ev);
    }
    PDMK_HIP(hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming));
  } catch (const Error& e) {
    pdmk_batch_destroy(B);
    return fail(e.code, e.msg);
  }
  *out = B;
  return PDMK_OK;
}

int pdmk_batch_eval(pdmk_batch* B, const int64_t* offsets, const double* src, const double* q,
                    double* pot, double* grad, void* stream) {
  if (!B || !offsets) return fail(PDMK_ERR_INVALID_ARG, "null argument");
  const int n_sys = (int)B->plans.size();
  const int d = B->o.dim;
  for (int sy = 0; sy < n_sys; ++sy)
    if (offsets[sy + 1] < offsets[sy]) return fail(PDMK_ERR_INVALID_ARG, "offsets decrease");
  if (offsets[n_sys] > offsets[0] && (!src || !q || !pot))
    return fail(PDMK_ERR_INVALID_ARG, "null array");
  if ((B->o.flags & PDMK_WANT_GRAD) && !grad) return fail(PDMK_ERR_INVALID_ARG, "null grad");
  // the caller's stream is joined before and after (its earlier work, e.g.
  // the inputs, is complete before any worker starts)
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
    return fail(PDMK_ERR_HIP, "stream synchronise failed");
  const int nw = (int)B->streams.size();
  std::vector<int> status(nw, PDMK_OK);
  std::vector<std::string> msg(nw);
  // largest cells first, so that no worker starts a large cell near the end
  std::vector<int> order(n_sys);
  for (int sy = 0; sy < n_sys; ++sy) order[sy] = sy;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return offsets[a + 1] - offsets[a] > offsets[b + 1] - offsets[b];
  });
  std::atomic<int> next(0);
  auto work = [&](int w) {
    if (hipSetDevice(B->device) != hipSuccess) {
      status[w] = PDMK_ERR_HIP;
      msg[w] = "hipSetDevice failed";
      return;
    }
    for (;;) {
      const int k = next.fetch_add(1);
      if (k >= n_sys) break;
      const int sy = order[k];
      const int64_t o = offsets[sy], n = offsets[sy + 1] - offsets[sy];
      const int st = eval_impl(B->plans[sy], n, src + o * d, q + o, 0, nullptr, pot + o,
                               grad ? grad + o * d : nullptr, B->streams[w], B->o.flags,
                               B->arenas[w], B->arena_sizes[w], B->aux[w]);
      if (st != PDMK_OK) {
        status[w] = st;
        msg[w] = g_last_error;
        next.store(n_sys);
        break;
      }
    }
  };
  std::vector<std::thread> th;
  try {
    for (int w = 1; w < nw; ++w) th.emplace_back(work, w);
  } catch (const std::system_error&) {
    // fewer threads than workers: the threads that exist take every system
  }
  work(0);
  for (auto& t : th) t.join();
  for (int w = 0; w < nw; ++w)
    if (status[w] != PDMK_OK) return fail(status[w], msg[w]);
  return PDMK_OK;
}

int pdmk_batch_bind(pdmk_batch* B, const int64_t* offsets, const double* src, const double* q,
                    double* pot, double* grad, void* stream) {
  if (!B || !offsets) return fail(PDMK_ERR_INVALID_ARG, "null argument");
  const int n_sys = (int)B->plans.size();
  const int d = B->o.dim;
  for (int sy = 0; sy < n_sys; ++sy)
    if (offsets[sy + 1] < offsets[sy]) return fail(PDMK_ERR_INVALID_ARG, "offsets decrease");
  if (offsets[n_sys] > offsets[0] && (!src || !q || !pot))
    return fail(PDMK_ERR_INVALID_ARG, "null array");
  if ((B->o.flags & PDMK_WANT_GRAD) && !grad) return fail(PDMK_ERR_INVALID_ARG, "null grad");
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
    return fail(PDMK_ERR_HIP, "stream synchronise failed");
  B->bound_off.clear();
  for (pdmk_plan* P : B->plans) unbind(P);
  const int nw = (int)B->streams.size();
  std::vector<int> status(nw, PDMK_OK);
  std::vector<std::string> msg(nw);
  std::atomic<int> next(0);
  auto work = [&](int w) {
    if (hipSetDevice(B->device) != hipSuccess) {
      status[w] = PDMK_ERR_HIP;
      msg[w] = "hipSetDevice failed";
      return;
    }
    for (;;) {
      const int sy = next.fetch_add(1);
      if (sy >= n_sys) break;
      const int64_t o = offsets[sy], n = offsets[sy + 1] - offsets[sy];
      if (n == 0) continue;   // an empty system keeps no tree
      const int st = pdmk_plan_bind(B->plans[sy], n, src + o * d, q + o, 0, nullptr, pot + o,
                                    grad ? grad + o * d : nullptr, B->streams[w]);
      if (st != PDMK_OK) {
        status[w] = st;
        msg[w] = g_last_error;
        next.store(n_sys);
        break;
      }
    }
  };
  std::vector<std::thread> th;
  try {
    for (int w = 1; w < nw; ++w) th.emplace_back(work, w);
  } catch (const std::system_error&) {
  }
  work(0);
  for (auto& t : th) t.join();
  for (int w = 0; w < nw; ++w)
    if (status[w] != PDMK_OK) {
      for (pdmk_plan* P : B->plans) unbind(P);
      return fail(status[w], msg[w]);
    }
  B->bound_off.assign(offsets, offsets + n_sys + 1);
  return PDMK_OK;
}

int pdmk_batch_execute(pdmk_batch* B, const double* q, double* pot, double* grad,
                       void* stream) {
  if (!B) return fail(PDMK_ERR_INVALID_ARG, "null batch");
  if (B->bound_off.empty()) return fail(PDMK_ERR_INVALID_ARG, "no bound trees (pdmk_batch_bind)");
  const int n_sys = (int)B->plans.size();
  const int d = B->o.dim;
  if (B->bound_off[n_sys] > B->bound_off[0] && (!q || !pot))
    return fail(PDMK_ERR_INVALID_ARG, "null array");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != B->device)
    return fail(PDMK_ERR_INVALID_ARG, "batch bound to another device");
  const int nw = (int)B->streams.size();
  hipStream_t cs = (hipStream_t)stream;
  try {
    // fork: every worker stream waits for the caller's stream; the systems'
    // executes are enqueued round-robin over them (this thread only, so a
    // caller can capture the whole call into one graph); join: the caller's
    // stream waits for every worker stream
    PDMK_HIP(hipEventRecord(B->ev_fork, cs));
    for (int w = 0; w < nw; ++w) PDMK_HIP(hipStreamWaitEvent(B->streams[w], B->ev_fork, 0));
    for (int sy = 0; sy < n_sys; ++sy)
      if (B->bound_off[sy + 1] > B->bound_off[sy] && !B->plans[sy]->bound)
        return fail(PDMK_ERR_INVALID_ARG, "a system has no bound tree (bind again)");
    // outside a capture the workers enqueue their shares concurrently (the
    // launches, not the device, bound a batch of small cells); inside one the
    // calling thread enqueues everything
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    PDMK_HIP(hipStreamIsCapturing(cs, &cap));
    const int nthreads = cap == hipStreamCaptureStatusNone ? nw : 1;
    std::vector<int> status(nw, PDMK_OK);
    std::vector<std::string> msg(nw);
    auto work = [&](int t) {
      if (t > 0 && hipSetDevice(B->device) != hipSuccess) {
        status[t] = PDMK_ERR_HIP;
        msg[t] = "hipSetDevice failed";
        return;
      }
      int k = 0;
      for (int sy = 0; sy < n_sys; ++sy) {
        const int64_t o = B->bound_off[sy], n = B->bound_off[sy + 1] - o;
        if (n == 0) continue;
        const int w = k++ % nw;
        if (w % nthreads != t) continue;
        const int st = execute_impl(B->plans[sy], nullptr, nullptr, q + o, pot + o,
                                    grad ? grad + o * d : nullptr, B->streams[w]);
        if (st != PDMK_OK) {
          status[t] = st;
          msg[t] = g_last_error;
          return;
        }
      }
    };
    std::vector<std::thread> th;
    try {
      for (int t = 1; t < nthreads; ++t) th.emplace_back(work, t);
    } catch (const std::system_error&) {
      for (auto& x : th) x.join();
      th.clear();
      throw Error{PDMK_ERR_HIP, "worker threads"};
    }
    work(0);
    for (auto& x : th) x.join();
    for (int t = 0; t < nthreads; ++t)
      if (status[t] != PDMK_OK) {
        for (int w = 0; w < nw; ++w) (void)hipStreamSynchronize(B->streams[w]);
        return fail(status[t], msg[t]);
      }
    for (int w = 0; w < nw; ++w) {
      PDMK_HIP(hipEventRecord(B->ev_join[w], B->streams[w]));
      PDMK_HIP(hipStreamWaitEvent(cs, B->ev_join[w], 0));
    }
  } catch (const Error& e) {
    return fail(e.code, e.msg);
  }
  return PDMK_OK;
}

int pdmk_batch_status(pdmk_batch* B) {
  if (!B) return fail(PDMK_ERR_INVALID_ARG, "null batch");
  if (B->bound_off.empty()) return fail(PDMK_ERR_INVALID_ARG, "no bound trees (pdmk_batch_bind)");
  const int n_sys = (int)B->plans.size();
  int first = PDMK_OK;
  std::string msg;
  for (int sy = 0; sy < n_sys; ++sy) {
    if (B->bound_off[sy + 1] == B->bound_off[sy]) continue;
    const int st = pdmk_plan_status(B->plans[sy]);
    if (st != PDMK_OK && first == PDMK_OK) {
      first = st;
      msg = g_last_error;
    }
  }
  return first == PDMK_OK ? PDMK_OK : fail(first, msg);
}

void pdmk_batch_destroy(pdmk_batch* B) {
  if (!B) return;
  for (hipEvent_t e : B->ev_join)
    if (e) (void)hipEventDestroy(e);
  if (B->ev_fork) (void)hipEventDestroy(B->ev_fork);
  for (pdmk_plan* P : B->plans) pdmk_plan_destroy(P);
  for (hipStream_t s : B->streams) (void)hipStreamDestroy(s);
  for (hipStream_t s : B->aux) (void)hipStreamDestroy(s);
  for (char* a : B->arenas)
    if (a) (void)hipFree(a);
  delete B;
}

int pdmk_batch_stats(const pdmk_batch* B, int sys, pdmk_stats* out) {
  if (!B || !out || sys < 0 || sys >= (int)B->plans.size())
    return fail(PDMK_ERR_INVALID_ARG, "bad system index");
  *out = B->plans[sys]->last;
  return PDMK_OK;
}

int pdmk_plan_tune(const pdmk_opts* opts, const double* L, int n_cand, const double* kappa,
                   const int* n_s, int trials, int64_t n_src, const double* src,
                   const double* q, int64_t n_trg, const double* trg, double* pot,
                   void* stream, double* times_ms, double* best_kappa, int* best_n_s) {
  if (!opts || !L || !kappa || !n_s || !best_kappa || !best_n_s || n_cand < 1 || trials < 1)
    return fail(PDMK_ERR_INVALID_ARG, "null argument, n_cand < 1 or trials < 1");
  double best = -1.0;
  int first_err = PDMK_OK;
  std::string first_msg;
  for (int c = 0; c < n_cand; ++c) {
    if (times_ms) times_ms[c] = -1.0;
    pdmk_opts o = *opts;
    if (kappa[c] > 0) o.kappa = kappa[c];
    if (n_s[c] > 0) o.n_s = n_s[c];
    pdmk_plan* P = nullptr;
    int st = pdmk_plan_create(&o, L, &P);
    if (st != PDMK_OK) {
      if (first_err == PDMK_OK) {
        first_err = st;
        first_msg = g_last_error;
      }
      continue;
    }
    // warm-up (grows the plan's workspace), then the timed evaluations
    st = pdmk_plan_eval(P, n_src, src, q, n_trg, trg, pot, nullptr, stream);
    double ms = 0.0;
    for (int t = 0; st == PDMK_OK && t < trials; ++t) {
      const auto t0 = std::chrono::steady_clock::now();
      st = pdmk_plan_eval(P, n_src, src, q, n_trg, trg, pot, nullptr, stream);
      ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                .count();
    }
    pdmk_plan_destroy(P);
    if (st != PDMK_OK) return st;   // an input error: the same for every candidate
    ms /= trials;
    if (times_ms) times_ms[c] = ms;
    if (best < 0 || ms < best) {
      best = ms;
      *best_kappa = o.kappa;
      *best_n_s = o.n_s;
    }
  }
  if (best < 0) return fail(first_err, first_msg);
  return PDMK_OK;
}

// Batch autotuner: systems are grouped by size class floor(log2 n).  For
// each class and candidate (kappa, n_s), up to one system per worker, spread
// evenly over the class's sizes, is planned and evaluated concurrently by the
// batch's workers, one system per worker stream, as the batch itself runs;
// the candidate with the shortest round is kept and every system of the class
// is re-planned with it.  Small cells are bound by launch and host-read
// latency shared among the workers, which a lone evaluation does not show.
int pdmk_batch_tune(pdmk_batch* B, const int64_t* offsets, const double* src, const double* q,
                    int n_cand, const double* kappa, const int* n_s, int trials, void* stream,
                    double* kappa_out, int* n_s_out) {
  if (!B || !offsets || !kappa || !n_s || n_cand < 1 || trials < 1)
    return fail(PDMK_ERR_INVALID_ARG, "null argument, n_cand < 1 or trials < 1");
  const int n_sys = (int)B->plans.size();
  const int d = B->o.dim;
  for (int sy = 0; sy < n_sys; ++sy)
    if (offsets[sy + 1] < offsets[sy]) return fail(PDMK_ERR_INVALID_ARG, "offsets decrease");
  if (offsets[n_sys] > offsets[0] && (!src || !q))
    return fail(PDMK_ERR_INVALID_ARG, "null array");
  B->bound_off.clear();   // re-planned systems keep no tree
  if (hipSetDevice(B->device) != hipSuccess) return fail(PDMK_ERR_HIP, "hipSetDevice failed");
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
    return fail(PDMK_ERR_HIP, "stream synchronise failed");
  const int nw = (int)B->streams.size();
  std::map<int, std::vector<int>> cls;
  for (int sy = 0; sy < n_sys; ++sy) {
    const int64_t n = offsets[sy + 1] - offsets[sy];
    if (n <= 0) continue;
    int c = 0;
    while ((2ll << c) <= n) ++c;
    cls[c].push_back(sy);
  }
  const bool want_grad = (B->o.flags & PDMK_WANT_GRAD) != 0;
  int status = PDMK_OK;
  std::string msg;
  std::vector<double*> buf(nw, nullptr);   // each worker's outputs (discarded)
  std::vector<size_t> buf_n(nw, 0);
  for (auto& kv : cls) {
    std::vector<int>& mem = kv.second;
    std::sort(mem.begin(), mem.end(), [&](int a, int b) {
      return offsets[a + 1] - offsets[a] < offsets[b + 1] - offsets[b];
    });
    const int ns = std::min<int>(nw, (int)mem.size());
    std::vector<int> sample(ns);
    for (int i = 0; i < ns; ++i) sample[i] = mem[(size_t)(2 * i + 1) * mem.size() / (2 * ns)];
    for (int i = 0; i < ns && status == PDMK_OK; ++i) {
      const size_t need = (size_t)(offsets[sample[i] + 1] - offsets[sample[i]]) *
                          (want_grad ? d + 1 : 1);
      if (need > buf_n[i]) {
        if (buf[i]) (void)hipFree(buf[i]);
        buf[i] = nullptr;
        buf_n[i] = 0;
        if (hipMalloc((void**)&buf[i], sizeof(double) * need) != hipSuccess) {
          status = PDMK_ERR_OUT_OF_MEMORY;
          msg = "tuning buffer";
        } else {
          buf_n[i] = need;
        }
      }
    }
    if (status != PDMK_OK) break;
    double best = -1.0, bk = 0.0;
    int bn = 0, first_err = PDMK_OK;
    std::string first_msg;
    for (int c = 0; c < n_cand && status == PDMK_OK; ++c) {
      pdmk_opts o = B->o;
      if (kappa[c] > 0) o.kappa = kappa[c];
      if (n_s[c] > 0) o.n_s = n_s[c];
      std::vector<pdmk_plan*> P(ns, nullptr);
      int st = PDMK_OK;
      for (int i = 0; i < ns && st == PDMK_OK; ++i)
        st = pdmk_plan_create(&o, B->L.data() + (size_t)sample[i] * d * d, &P[i]);
      if (st != PDMK_OK) {
        if (first_err == PDMK_OK) {
          first_err = st;
          first_msg = g_last_error;
        }
        for (pdmk_plan* p : P) pdmk_plan_destroy(p);
        continue;
      }
      std::vector<int> wst(ns, PDMK_OK);
      std::vector<std::string> wmsg(ns);
      auto one = [&](int i) {
        if (hipSetDevice(B->device) != hipSuccess) {
          wst[i] = PDMK_ERR_HIP;
          wmsg[i] = "hipSetDevice failed";
          return;
        }
        const int sy = sample[i];
        const int64_t o0 = offsets[sy], n = offsets[sy + 1] - offsets[sy];
        int r = eval_impl(P[i], n, src + o0 * d, q + o0, 0, nullptr, buf[i],
                          want_grad ? buf[i] + n : nullptr, B->streams[i], B->o.flags,
                          B->arenas[i], B->arena_sizes[i], B->aux[i]);
        if (r == PDMK_OK && hipStreamSynchronize(B->streams[i]) != hipSuccess)
          r = fail(PDMK_ERR_HIP, "stream synchronise failed");
        wst[i] = r;
        if (r != PDMK_OK) wmsg[i] = g_last_error;
      };
      double ms = 0.0;
      for (int t = 0; t <= trials && st == PDMK_OK; ++t) {   // t = 0: warm-up
        const auto t0 = std::chrono::steady_clock::now();
        std::vector<std::thread> th;
        int started = 1;
        try {
          for (int i = 1; i < ns; ++i, ++started) th.emplace_back(one, i);
        } catch (const std::system_error&) {
          // samples without a thread run on this one after its own
        }
        one(0);
        for (int i = started; i < ns; ++i) one(i);
        for (auto& x : th) x.join();
        if (t > 0)
          ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                    .count();
        for (int i = 0; i < ns && st == PDMK_OK; ++i)
          if (wst[i] != PDMK_OK) {
            st = wst[i];
            msg = wmsg[i];
          }
      }
      if (st == PDMK_OK && (best < 0 || ms < best)) {
        best = ms;
        bk = P[0]->mp.kappa;
        bn = P[0]->mp.n_s;
      }
      for (pdmk_plan* p : P) pdmk_plan_destroy(p);
      if (st != PDMK_OK) status = st;   // an input error: the same for every candidate
    }
    if (status != PDMK_OK) break;
    if (best < 0) {
      status = first_err;
      msg = first_msg;
      break;
    }
    for (int sy : mem) {
      pdmk_plan*& cur = B->plans[sy];
      if (cur->mp.kappa == bk && cur->mp.n_s == bn) continue;
      pdmk_opts o = B->o;
      o.kappa = bk;
      o.n_s = bn;
      pdmk_plan* P = nullptr;
      if (pdmk_plan_create(&o, B->L.data() + (size_t)sy * d * d, &P) != PDMK_OK)
        continue;   // this cell keeps its current (valid) plan
      pdmk_plan_destroy(cur);
      cur = P;
    }
  }
  for (double* b : buf)
    if (b) (void)hipFree(b);
  for (int sy = 0; sy < n_sys; ++sy) {
    if (kappa_out) kappa_out[sy] = B->plans[sy]->mp.kappa;
    if (n_s_out) n_s_out[sy] = B->plans[sy]->mp.n_s;
  }
  if (status != PDMK_OK) return fail(status, msg);
  return PDMK_OK;
}

int pdmk_eval_batched(const pdmk_opts* opts, int n_sys, const double* L, const int64_t* offsets,
                      const double* src, const double* q, double* pot, double* grad,
                      void* stream) {
  pdmk_batch* B = nullptr;
  int st = pdmk_batch_create(opts, n_sys, L, 0, &B);
  if (st) return st;
  st = pdmk_batch_eval(B, offsets, src, q, pot, grad, stream);
  pdmk_batch_destroy(B);
  return st;
}

}  // extern "C"

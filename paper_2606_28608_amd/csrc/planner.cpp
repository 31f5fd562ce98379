// Host-side planning for periodic DMK.  See planner.h.
#include "planner.h"

#include <algorithm>
#include <functional>
#include <cmath>
#include <map>
#include <mutex>
#include <numeric>

namespace pdmk {

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    double wi = 2.0 / ((1.0 - z * z) * dp * dp);
    w[i] = wi;
    w[n - 1 - i] = wi;
  }
}

static double legendre_series(const std::vector<double>& a, double x) {
  // sum a_k P_k(x) by the three-term recurrence
  double p0 = 1.0, p1 = x, s = a.empty() ? 0.0 : a[0];
  if (a.size() > 1) s += a[1] * x;
  for (size_t k = 2; k < a.size(); ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    s += a[k] * p2;
    p0 = p1;
    p1 = p2;
  }
  return s;
}

// Smallest eigenpair of a symmetric tridiagonal matrix (diag d, off e):
// Sturm-sequence bisection for the eigenvalue, inverse iteration for the vector.
static void tridiag_smallest(const std::vector<double>& d, const std::vector<double>& e,
                             double& lam, std::vector<double>& v) {
  int n = (int)d.size();
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < n; ++i) {
    double r = (i > 0 ? std::fabs(e[i - 1]) : 0) + (i + 1 < n ? std::fabs(e[i]) : 0);
    lo = std::min(lo, d[i] - r);
    hi = std::max(hi, d[i] + r);
  }
  auto count_below = [&](double x) {
    int cnt = 0;
    double q = d[0] - x;
    if (q < 0) ++cnt;
    for (int i = 1; i < n; ++i) {
      if (q == 0) q = 1e-300;
      q = d[i] - x - e[i - 1] * e[i - 1] / q;
      if (q < 0) ++cnt;
    }
    return cnt;
  };
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (count_below(mid) >= 1) hi = mid; else lo = mid;
    if (hi - lo < 1e-15 * std::max(1.0, std::fabs(hi))) break;
  }
  lam = 0.5 * (lo + hi);
  // inverse iteration with a slightly shifted matrix
  double shift = lam - 1e-10 * std::max(1.0, std::fabs(lam));
  v.assign(n, 1.0);
  std::vector<double> cp(n), dp(n), x(n);
  for (int it = 0; it < 6; ++it) {
    // solve (T - shift I) x = v  (Thomas algorithm)
    double b0 = d[0] - shift;
    cp[0] = n > 1 ? e[0] / b0 : 0;
    dp[0] = v[0] / b0;
    for (int i = 1; i < n; ++i) {
      double den = d[i] - shift - e[i - 1] * cp[i - 1];
      cp[i] = i + 1 < n ? e[i] / den : 0;
      dp[i] = (v[i] - e[i - 1] * dp[i - 1]) / den;
    }
    x[n - 1] = dp[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = dp[i] - cp[i] * x[i + 1];
    double nrm = 0;
    for (double t : x) nrm += t * t;
    nrm = std::sqrt(nrm);
    for (int i = 0; i < n; ++i) v[i] = x[i] / nrm;
  }
}

double Pswf::psi(double x) const { return legendre_series(leg, x); }

double Pswf::phi(double t) const {
  if (t >= 1.0) return 1.0;
  if (t <= 0.0) return -phi(-t);
  // (1/c0) int_0^t psi = (t/c0) int_0^1 psi(t v) dv, Gauss-Legendre on [0,1]
  double s = 0;
  for (size_t i = 0; i < qx.size(); ++i) {
    double v = 0.5 * (qx[i] + 1.0);
    s += 0.5 * qw[i] * psi(t * v);
  }
  return t * s / c0;
}

double Pswf::psit(double x) const {
  // psi~(x) = (1/(2 c0)) int_{-1}^{1} psi(t) cos(c x t) dt   (eq:pswf_eig)
  x = std::fabs(x);
  double s = 0;
  for (size_t i = 0; i < qx.size(); ++i) s += qw[i] * qpsi[i] * std::cos(c * x * qx[i]);
  return s / (2.0 * c0);
}

Pswf make_pswf_c(double c) {
  Pswf P;
  P.c = c;
  int n = (int)(2.0 * c + 40.0);
  // prolate operator in the normalised even Legendre basis: symmetric tridiagonal
  std::vector<double> d(n), e(n > 1 ? n - 1 : 1);
  for (int i = 0; i < n; ++i) {
    double k = 2.0 * i;
    d[i] = k * (k + 1) + c * c * (2 * k * (k + 1) - 1) / ((2 * k + 3) * (2 * k - 1));
    if (i + 1 < n)
      e[i] = c * c * (k + 1) * (k + 2) / ((2 * k + 3) * std::sqrt((2 * k + 1) * (2 * k + 5)));
  }
  double lam;
  std::vector<double> v;
  tridiag_smallest(d, e, lam, v);
  if (v[0] < 0)
    for (double& t : v) t = -t;
  P.leg.assign(2 * n, 0.0);
  for (int i = 0; i < n; ++i) P.leg[2 * i] = v[i] * std::sqrt(2.0 * i + 0.5);
  // trim negligible tail
  while (P.leg.size() > 2 && std::fabs(P.leg.back()) < 1e-30) P.leg.pop_back();
  gauss_legendre(std::max(96, (int)(2.0 * c) + 64), P.qx, P.qw);
  P.qpsi.resize(P.qx.size());
  for (size_t i = 0; i < P.qx.size(); ++i) P.qpsi[i] = P.psi(P.qx[i]);
  P.psi0 = P.psi(0.0);
  double s = 0, s2 = 0;
  for (size_t i = 0; i < P.qx.size(); ++i) {
    s += P.qw[i] * P.qpsi[i];
    s2 += P.qw[i] * P.qpsi[i] * P.qx[i] * P.qx[i];
  }
  P.c0 = 0.5 * s;                 // psi is even
  P.lambda0 = s / P.psi0;
  P.psit_dd0 = -c * c * s2 / (2.0 * P.c0);
  return P;
}

double calibrate_c(double eps) {
  double lo = 0.5, hi = 80.0;
  for (int it = 0; it < 90; ++it) {
    double mid = 0.5 * (lo + hi);
    Pswf P = make_pswf_c(mid);
    double r = P.psi(1.0) / P.psi0;
    if (r > eps) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

const Pswf& pswf_for_eps(double eps) {
  static std::mutex mu;
  static std::map<double, Pswf> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(eps);
  if (it != cache.end()) return it->second;
  Pswf P = make_pswf_c(calibrate_c(eps));
  P.eps = eps;
  return cache.emplace(eps, std::move(P)).first->second;
}

double ChebSeries::operator()(double s) const {
  double t = 2.0 * s - 1.0, b1 = 0, b2 = 0;
  for (int k = (int)a.size() - 1; k >= 1; --k) {
    double b0 = 2.0 * t * b1 - b2 + a[k];
    b2 = b1;
    b1 = b0;
  }
  return t * b1 - b2 + a[0];
}

double ChebSeries::deriv(double s) const {
  // derivative of sum a_k T_k(t), t = 2s-1: coefficients of the derivative series
  int n = (int)a.size();
  if (n < 2) return 0.0;
  std::vector<double> d(n + 1, 0.0);
  for (int k = n - 1; k >= 1; --k) d[k - 1] = d[k + 1] + 2.0 * k * a[k];
  d[0] *= 0.5;
  ChebSeries D;
  D.a.assign(d.begin(), d.begin() + (n - 1));
  return 2.0 * D(s);
}

static ChebSeries cheb_fit(int n, const std::function<double(double)>& f, double tol) {
  // interpolate at Chebyshev points of [0,1], coefficients by the DCT
  std::vector<double> fv(n);
  for (int j = 0; j < n; ++j) {
    double t = std::cos(kPi * (j + 0.5) / n);
    fv[j] = f(0.5 * (t + 1.0));
  }
  ChebSeries S;
  S.a.assign(n, 0.0);
  double amax = 0;
  for (int k = 0; k < n; ++k) {
    double s = 0;
    for (int j = 0; j < n; ++j) s += fv[j] * std::cos(kPi * k * (j + 0.5) / n);
    S.a[k] = (k == 0 ? 1.0 : 2.0) * s / n;
    amax = std::max(amax, std::fabs(S.a[k]));
  }
  // truncate at the first run of three coefficients below tol (the tail
  // beyond it is rounding noise of the samples)
  size_t keep = S.a.size();
  for (size_t k = 1; k + 2 < S.a.size(); ++k)
    if (std::fabs(S.a[k]) < tol * amax && std::fabs(S.a[k + 1]) < tol * amax &&
        std::fabs(S.a[k + 2]) < tol * amax) {
      keep = k;
      break;
    }
  S.a.resize(keep);
  return S;
}

double SplitTables::w0_unit(int dim) const {
  // 3D: eq:W0zero, W_h(0) = psi(0) / (4 pi c0 h)
  if (dim == 3) return pswf_for_eps(eps).psi0 / pswf_for_eps(eps).c0 / (4.0 * kPi);
  return -F2(0.0) / (2.0 * kPi);
}

double SplitTables::residual(int dim, double r, double h) const {
  if (r >= h || r <= 0) return 0.0;
  double s = (r / h) * (r / h);
  if (dim == 3) return (1.0 / r - E(s) / h) / (4.0 * kPi);
  return (-std::log(r / h) + F2(s)) / (2.0 * kPi);
}

double SplitTables::residual_dr(int dim, double r, double h) const {
  if (r >= h || r <= 0) return 0.0;
  double s = (r / h) * (r / h);
  if (dim == 3) return (-1.0 / (r * r) - E.deriv(s) * 2.0 * r / (h * h * h)) / (4.0 * kPi);
  return (-1.0 / r + F2.deriv(s) * 2.0 * r / (h * h)) / (2.0 * kPi);
}

void SplitTables::prepare_pw(int jmax, int dim) {
  const Pswf& P = pswf_for_eps(eps);
  int nmax = dim * jmax * jmax;
  dtab.assign(nmax + 1, 0.0);
  // (3h)^{2-d} * [psi~(pi|j|/(3c)) - psi~(2 pi|j|/(3c))] / (4 pi^2 |j|^2); the
  // factor (3h)^{2-d} is applied per level.
  dtab[0] = -P.psit_dd0 / (24.0 * c * c);
  for (int n = 1; n <= nmax; ++n) {
    double jn = std::sqrt((double)n);
    double a = P.psit(kPi * jn / (3.0 * c)), b = P.psit(2.0 * kPi * jn / (3.0 * c));
    dtab[n] = (a - b) / (4.0 * kPi * kPi * n);
  }
}

const SplitTables& tables_for_eps(double eps) {
  static std::mutex mu;
  static std::map<double, SplitTables> cache;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(eps);
    if (it != cache.end()) return it->second;
  }
  const Pswf& P = pswf_for_eps(eps);
  SplitTables T;
  T.eps = eps;
  T.c = P.c;
  // E(s) = phi(sqrt s)/sqrt s, E(0) = psi(0)/c0
  T.E = cheb_fit(64, [&](double s) {
    if (s <= 0) return P.psi0 / P.c0;
    double t = std::sqrt(s);
    return P.phi(t) / t;
  }, std::max(4e-15, 1e-4 * eps));
  // F2(s) = log(1 + sqrt(1-s)) - int_0^{sqrt(1-s)} E(s + v^2) dv
  std::vector<double> gx, gw;
  gauss_legendre(64, gx, gw);
  T.F2 = cheb_fit(64, [&](double s) {
    double a = std::sqrt(std::max(0.0, 1.0 - s));
    double integ = 0;
    for (size_t i = 0; i < gx.size(); ++i) {
      double v = 0.5 * a * (gx[i] + 1.0);
      double rr = std::sqrt(s + v * v);
      double e = rr > 0 ? P.phi(rr) / rr : P.psi0 / P.c0;
      integ += 0.5 * a * gw[i] * e;
    }
    return std::log(1.0 + a) - integ;
  }, std::max(4e-15, 1e-4 * eps));
  std::lock_guard<std::mutex> lk(mu);
  return cache.emplace(eps, std::move(T)).first->second;
}

MethodParams default_params(int dim, double eps) {
  const Pswf& P = pswf_for_eps(eps);
  MethodParams m;
  double l = -std::log10(eps);
  if (dim == 3) {
    m.kappa = 3.0;
    m.n_s = l <= 3.5 ? 80 : (l <= 6.5 ? 200 : (l <= 9.5 ? 500 : 600));
  } else {
    m.kappa = 7.0;
    m.n_s = l <= 3.5 ? 30 : (l <= 9.5 ? 40 : 60);
  }
  // proxy points per axis: 13 / 22 / 31 / 40 at eps = 1e-3 / 1e-6 / 1e-9 /
  // 1e-12; at 1e-12 one point fewer leaves the near field at 2e-12 on a
  // clustered cube (kappa = 3), one more point 3e-13
  m.porder = (int)std::ceil(1.28 * P.c + 0.8);
  m.npw = (int)std::ceil(3.0 * P.c / kPi);
  // Spreading window: without upsampling (the paper's grid) a width of
  // log10(1/eps) + 2 cells suffices down to eps ~ 1e-7; below that the
  // window would have to grow past 16 cells, so the grid is doubled instead.
  // On the doubled grid one cell less does: its far-field error at eps = 1e-9
  // / 1e-12 is 1.8e-11 / 1.5e-14 of |Phi| (clustered triclinic cell), against
  // 1.1e-12 / 1.8e-15 with the wider window, for (10/11)^3 / (13/14)^3 of the
  // spreading and interpolation work.
  m.sigma = eps >= 1e-7 ? 1.0 : 2.0;
  m.nufft_w = std::min(16, (int)std::ceil(l - 1e-9) + (m.sigma > 1.5 ? 1 : 2));
  m.beta = window_beta(m.nufft_w, m.sigma);
  return m;
}

double window_beta(int w, double sigma) { return (sigma > 1.5 ? 2.4 : 2.0) * w; }

int next_fft_size(int n) {
  if (n < 2) n = 2;
  if (n % 2) ++n;
  for (;; n += 2) {
    int t = n;
    while (t % 2 == 0) t /= 2;
    while (t % 3 == 0) t /= 3;
    while (t % 5 == 0) t /= 5;
    if (t == 1) return n;
  }
}

static void inv3(int d, const double* A, double* Ai) {
  if (d == 2) {
    double det = A[0] * A[3] - A[2] * A[1];
    Ai[0] = A[3] / det; Ai[2] = -A[2] / det; Ai[1] = -A[1] / det; Ai[3] = A[0] / det;
    return;
  }
  auto a = [&](int i, int j) { return A[i + 3 * j]; };
  double c00 = a(1, 1) * a(2, 2) - a(1, 2) * a(2, 1);
  double c01 = a(1, 2) * a(2, 0) - a(1, 0) * a(2, 2);
  double c02 = a(1, 0) * a(2, 1) - a(1, 1) * a(2, 0);
  double det = a(0, 0) * c00 + a(0, 1) * c01 + a(0, 2) * c02;
  double m[9];
  m[0] = c00; m[1] = c01; m[2] = c02;
  m[3] = a(0, 2) * a(2, 1) - a(0, 1) * a(2, 2);
  m[4] = a(0, 0) * a(2, 2) - a(0, 2) * a(2, 0);
  m[5] = a(0, 1) * a(2, 0) - a(0, 0) * a(2, 1);
  m[6] = a(0, 1) * a(1, 2) - a(0, 2) * a(1, 1);
  m[7] = a(0, 2) * a(1, 0) - a(0, 0) * a(1, 2);
  m[8] = a(0, 0) * a(1, 1) - a(0, 1) * a(1, 0);
  for (int k = 0; k < 9; ++k) Ai[k] = m[k] / det;
}

std::string make_geometry(int d, const double* Lin, double kappa, double c, double sigma,
                          Geometry& g, double beta_norm, bool virtual_images) {
  g = Geometry();
  g.dim = d;
  // sort lattice vectors by decreasing length (stable), Section 3.2
  double len[3];
  for (int j = 0; j < d; ++j) {
    double s = 0;
    for (int i = 0; i < d; ++i) s += Lin[i + d * j] * Lin[i + d * j];
    len[j] = std::sqrt(s);
    g.perm[j] = j;
  }
  std::stable_sort(g.perm, g.perm + d, [&](int a, int b) { return len[a] > len[b]; });
  double A[9] = {0}, Qm[9] = {0}, R[9] = {0};
  for (int j = 0; j < d; ++j)
    for (int i = 0; i < d; ++i) A[i + d * j] = Lin[i + d * g.perm[j]];
  // modified Gram-Schmidt: A = Q R, R upper triangular with positive diagonal
  for (int j = 0; j < d; ++j) {
    double v[3];
    for (int i = 0; i < d; ++i) v[i] = A[i + d * j];
    for (int k = 0; k < j; ++k) {
      double r = 0;
      for (int i = 0; i < d; ++i) r += Qm[i + d * k] * v[i];
      R[k + d * j] = r;
      for (int i = 0; i < d; ++i) v[i] -= r * Qm[i + d * k];
    }
    double nr = 0;
    for (int i = 0; i < d; ++i) nr += v[i] * v[i];
    nr = std::sqrt(nr);
    if (!(nr > 1e-300) || !std::isfinite(nr)) return "singular lattice";
    R[j + d * j] = nr;
    for (int i = 0; i < d; ++i) Qm[i + d * j] = v[i] / nr;
  }
  for (int k = 0; k < d * d; ++k) { g.L[k] = R[k]; g.Q[k] = Qm[k]; }
  if (virtual_images) {
    // a rectangular cell: R is diagonal up to rounding, which is removed
    double Lmx = 0;
    for (int i = 0; i < d; ++i) Lmx = std::max(Lmx, R[i + d * i]);
    for (int j = 0; j < d; ++j)
      for (int i = 0; i < j; ++i) {
        if (std::fabs(R[i + d * j]) > 1e-12 * Lmx)
          return "unsupported: virtual images need a rectangular cell";
        g.L[i + d * j] = 0.0;
      }
  }
  inv3(d, g.L, g.Li);
  g.volume = 1.0;
  g.Lmin = 1e300;
  for (int i = 0; i < d; ++i) {
    g.volume *= g.L[i + d * i];
    g.Lmin = std::min(g.Lmin, g.L[i + d * i]);
  }
  double Lmax = 0;
  for (int i = 0; i < d; ++i) Lmax = std::max(Lmax, g.L[i + d * i]);
  if (!(g.Lmin > 1e-12 * Lmax)) return "lattice too ill-conditioned";
  if (!(kappa >= 1.0)) return "kappa must be >= 1";
  g.rc = g.Lmin / kappa;
  if (virtual_images) {
    // rem:cube: root cubes of side r_c tile the cell exactly; a boundary
    // box's colleagues across a face are boxes of the other side, shifted by
    // L n, so no image is placed or sorted
    g.virtual_images = true;
    for (int i = 0; i < d; ++i) {
      const double e = g.L[i + d * i];
      const double m = std::nearbyint(e / g.rc);
      if (m < 1.0 || std::fabs(m * g.rc - e) > 1e-13 * e)
        return "unsupported: virtual images need cell edges that are whole multiples of "
               "r_c = L_min / kappa";
      g.xlo[i] = 0.0;
      g.width[i] = e;
      g.nroot[i] = (int)m;
      g.next[i] = (int)m;
      g.origin[i] = 0.0;
    }
    for (int k = 0; k < d; ++k) g.shifts.push_back(0);
  }
  // bounding box (eq:x1range .. eq:w1) and root cubes (eq:mi)
  for (int i = 0; i < d && !virtual_images; ++i) {
    double lo = 0, w = g.L[i + d * i];
    for (int j = i + 1; j < d; ++j) {
      lo += std::min(0.0, g.L[i + d * j]);
      w += std::fabs(g.L[i + d * j]);
    }
    g.xlo[i] = lo;
    g.width[i] = w;
    int m = (int)std::ceil(w / g.rc);
    while (m * g.rc < w) ++m;
    if (m < 1) m = 1;
    g.nroot[i] = m;
    g.next[i] = m + 2;
    g.origin[i] = lo - g.rc;
  }
  // lattice shifts passing eq:shift_bounds (n_d outermost)
  std::vector<int> n(d, 0);
  std::function<void(int)> rec = [&](int i) {
    if (i < 0) {
      for (int k = 0; k < d; ++k) g.shifts.push_back(n[k]);
      return;
    }
    double s = 0;
    for (int k = i + 1; k < d; ++k) s += g.L[i + d * k] * n[k];
    int nmax = (int)std::ceil(((g.nroot[i] + 1) * g.rc + std::fabs(s)) / g.L[i + d * i]);
    for (int v = -nmax; v <= nmax; ++v) {
      n[i] = v;
      rec(i - 1);
    }
    n[i] = 0;
  };
  if (!virtual_images) rec(d - 1);
  // Fourier grid (eq:Mi with eq:anorms); with a Bloch vector the active modes
  // |k_m + beta| <= c / r_c need M_i = 2 ceil((c / r_c + |beta|) |a_i| / 2 pi)
  // (Section 4.1, Fourier grid)
  for (int i = 0; i < d; ++i) {
    double an = 0;
    for (int k = 0; k <= i; ++k) an += g.L[k + d * i] * g.L[k + d * i];
    an = std::sqrt(an);
    int M = beta_norm == 0.0 ? 2 * (int)std::ceil(c * an / (2.0 * kPi * g.rc))
                             : 2 * (int)std::ceil((c / g.rc + beta_norm) * an / (2.0 * kPi));
    if (M < 2) M = 2;
    g.fgrid_paper[i] = M;
    g.fgrid[i] = next_fft_size((int)std::ceil(std::max(1.0, sigma) * M - 1e-9));
  }
  return "";
}

std::vector<double> window_ft(int M, int w, double beta) {
  std::vector<double> gx, gw;
  gauss_legendre(std::max(64, 4 * w + 40), gx, gw);
  double hw = 0.5 * w;
  std::vector<double> out(M);
  for (int n = 0; n < M; ++n) {
    int m = n < M / 2 ? n : n - M;
    double s = 0;
    for (size_t i = 0; i < gx.size(); ++i) {
      double z = gx[i];
      double ph = std::exp(beta * (std::sqrt(std::max(0.0, 1.0 - z * z)) - 1.0));
      s += gw[i] * hw * ph * std::cos(2.0 * kPi * m * hw * z / M);
    }
    out[n] = s;
  }
  return out;
}

void cheb_nodes(int p, std::vector<double>& x, std::vector<double>& bw) {
  x.resize(p);
  bw.resize(p);
  for (int j = 0; j < p; ++j) {
    double th = (2.0 * j + 1.0) * kPi / (2.0 * p);
    x[j] = std::cos(th);
    bw[j] = ((j % 2) ? -1.0 : 1.0) * std::sin(th);
  }
}

void lagrange_row(int p, const double* nodes, const double* bw, double x, double* out) {
  double s = 0;
  for (int j = 0; j < p; ++j) {
    double dx = x - nodes[j];
    if (dx == 0.0) {
      for (int k = 0; k < p; ++k) out[k] = (k == j) ? 1.0 : 0.0;
      return;
    }
    out[j] = bw[j] / dx;
    s += out[j];
  }
  for (int j = 0; j < p; ++j) out[j] /= s;
}

}  // namespace pdmk

/*
 * Reference Ewald summation for periodic Laplace (Coulomb) lattice sums.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, double-precision
 * oracle against which the GPU library is checked.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product library neither links nor calls it, and it shares no code with it.
 *
 * What is computed (Introduction, eq:potential and eq:greens; Section 3.5,
 * eq:W0p and the charge-neutrality paragraph):
 *
 *     Phi(x) = sum_n sum_j G(x - y_j - L n) q_j,
 *
 *   G = -log(r)/(2 pi) in 2D and 1/(4 pi r) in 3D, the singular self pair
 *   (n = 0, coincident source) removed, the sum taken in the tin-foil sense:
 *   the k = 0 Fourier mode of the periodic potential is zero.  Equivalently,
 *
 *     Phi(x) = (1/V) sum_{m != 0} |k_m|^-2 sum_j q_j exp(i k_m.(x - y_j)),
 *     k_m = 2 pi L^{-T} m.
 *
 * Method: the classical Ewald split 1/|k|^2 = e^{-k^2/4a^2}/k^2 +
 * (1 - e^{-k^2/4a^2})/k^2.  The first part is summed in reciprocal space,
 * the second in real space where its kernel is
 *     3D: erfc(a r) / (4 pi r)
 *     2D: E1(a^2 r^2) / (4 pi)
 * The smooth part evaluated at a coincident source contains the limit of the
 * smooth kernel at r = 0, which is removed:
 *     3D: a / (2 pi^{3/2}),   2D: (gamma + 2 ln a) / (4 pi).
 * The real-space kernel has mean (over R^d) 1/(4 a^2); its periodic sum thus
 * carries a k = 0 component (sum q)/(4 a^2 V), which is removed so that a
 * non-neutral input returns the potential of the charges plus a uniform
 * neutralising background (tin-foil, zero cell mean).  For neutral charges
 * this term is zero.
 *
 * Lattice convention: L is d x d, column-major, its columns are the lattice
 * vectors a_1..a_d: L[i + d*j] = (a_j)_i.
 *
 * Summations use Neumaier compensation.  OpenMP parallelises over targets
 * (real space and reciprocal evaluation) and over sources (structure factor).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846264338327950288
#define OR_EULER_GAMMA 0.57721566490153286060651209008240243

typedef struct { double s, c; } nsum;   /* Neumaier accumulator */

static inline void nsum_add(nsum* a, double v) {
  double t = a->s + v;
  if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
  else a->c += (v - t) + a->s;
  a->s = t;
}
static inline double nsum_get(const nsum* a) { return a->s + a->c; }

/* Exponential integral E1(x), x > 0 (Abramowitz & Stegun 5.1.11 power series
 * for x <= 1, 5.1.22 continued fraction evaluated by the modified Lentz
 * method for x > 1). */
double oracle_expint_e1(double x) {
  if (x <= 0.0) return INFINITY;
  if (x <= 1.0) {
    /* E1(x) = -gamma - ln x - sum_{k>=1} (-x)^k / (k k!) */
    double sum = 0.0, term = 1.0;
    for (int k = 1; k < 200; ++k) {
      term *= -x / k;                 /* (-x)^k / k! */
      double add = term / k;
      sum += add;
      if (fabs(add) < 1e-18 * fabs(sum)) break;
    }
    return -OR_EULER_GAMMA - log(x) - sum;
  }
  /* E1(x) = e^{-x} / (x + 1 - 1^2/(x + 3 - 2^2/(x + 5 - ...))) */
  const double tiny = 1e-300;
  double b = x + 1.0, c = 1.0 / tiny, d = 1.0 / b, h = d;
  for (int i = 1; i < 500; ++i) {
    double an = -(double)i * (double)i;
    b += 2.0;
    d = an * d + b; if (fabs(d) < tiny) d = tiny;
    c = b + an / c; if (fabs(c) < tiny) c = tiny;
    d = 1.0 / d;
    double del = c * d;
    h *= del;
    if (fabs(del - 1.0) < 1e-16) break;
  }
  return h * exp(-x);
}

/* Inverse of a d x d matrix (d = 2 or 3), column-major.  Returns det. */
static double inv_small(int d, const double* A, double* Ai) {
  if (d == 2) {
    double det = A[0] * A[3] - A[2] * A[1];
    Ai[0] = A[3] / det; Ai[2] = -A[2] / det;
    Ai[1] = -A[1] / det; Ai[3] = A[0] / det;
    return det;
  }
  /* 3x3 via cofactors; A(i,j) = A[i + 3 j] */
#define M_(i, j) A[(i) + 3 * (j)]
  double c00 = M_(1,1)*M_(2,2) - M_(1,2)*M_(2,1);
  double c01 = M_(1,2)*M_(2,0) - M_(1,0)*M_(2,2);
  double c02 = M_(1,0)*M_(2,1) - M_(1,1)*M_(2,0);
  double det = M_(0,0)*c00 + M_(0,1)*c01 + M_(0,2)*c02;
  double inv[9];
  inv[0 + 3*0] = c00;
  inv[1 + 3*0] = c01;
  inv[2 + 3*0] = c02;
  inv[0 + 3*1] = M_(0,2)*M_(2,1) - M_(0,1)*M_(2,2);
  inv[1 + 3*1] = M_(0,0)*M_(2,2) - M_(0,2)*M_(2,0);
  inv[2 + 3*1] = M_(0,1)*M_(2,0) - M_(0,0)*M_(2,1);
  inv[0 + 3*2] = M_(0,1)*M_(1,2) - M_(0,2)*M_(1,1);
  inv[1 + 3*2] = M_(0,2)*M_(1,0) - M_(0,0)*M_(1,2);
  inv[2 + 3*2] = M_(0,0)*M_(1,1) - M_(0,1)*M_(1,0);
#undef M_
  for (int k = 0; k < 9; ++k) Ai[k] = inv[k] / det;
  return det;
}

/* Real-space kernel (and d/dr) of the Ewald split. */
static inline void real_kernel(int d, double a, double r, double* k, double* dk) {
  if (d == 3) {
    double e = erfc(a * r);
    *k = e / (4.0 * OR_PI * r);
    *dk = -(e / (r * r) + 2.0 * a / sqrt(OR_PI) * exp(-a * a * r * r) / r) / (4.0 * OR_PI);
  } else {
    *k = oracle_expint_e1(a * a * r * r) / (4.0 * OR_PI);
    *dk = -exp(-a * a * r * r) / (2.0 * OR_PI * r);
  }
}

/*
 * Real-space part at n_trg targets.  self_idx[i] (or NULL) names the source
 * coincident with target i; that pair is skipped for n = 0 only.
 */
static void real_space(int d, const double* L, const double* Li, long n_src,
                       const double* src, const double* q, long n_trg,
                       const double* trg, const long* self_idx, double a,
                       double rcut, int want_grad, double* pot, double* grad) {
  double b[3] = {0, 0, 0};
  for (int i = 0; i < d; ++i) {            /* |row_i(L^-1)| * rcut */
    double s = 0;
    for (int j = 0; j < d; ++j) s += Li[i + d * j] * Li[i + d * j];
    b[i] = sqrt(s) * rcut;
  }
  const double rc2 = rcut * rcut;
#pragma omp parallel for schedule(dynamic, 4)
  for (long it = 0; it < n_trg; ++it) {
    nsum acc = {0, 0}, g[3] = {{0, 0}, {0, 0}, {0, 0}};
    const double* x = trg + d * it;
    long self = self_idx ? self_idx[it] : -1;
    for (long js = 0; js < n_src; ++js) {
      const double* y = src + d * js;
      double dx[3] = {0, 0, 0}, u[3] = {0, 0, 0};
      for (int i = 0; i < d; ++i) dx[i] = x[i] - y[i];
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) u[i] += Li[i + d * j] * dx[j];
      long lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
      for (int i = 0; i < d; ++i) {
        lo[i] = (long)ceil(u[i] - b[i]);
        hi[i] = (long)floor(u[i] + b[i]);
      }
      long n3lo = d == 3 ? lo[2] : 0, n3hi = d == 3 ? hi[2] : 0;
      for (long n3 = n3lo; n3 <= n3hi; ++n3)
        for (long n2 = lo[1]; n2 <= hi[1]; ++n2)
          for (long n1 = lo[0]; n1 <= hi[0]; ++n1) {
            long nn[3] = {n1, n2, n3};
            if (js == self && n1 == 0 && n2 == 0 && n3 == 0) continue;
            double z[3] = {0, 0, 0}, r2 = 0;
            for (int i = 0; i < d; ++i) {
              double s = dx[i];
              for (int j = 0; j < d; ++j) s -= L[i + d * j] * (double)nn[j];
              z[i] = s;
              r2 += s * s;
            }
            if (r2 >= rc2) continue;
            double r = sqrt(r2), k, dk;
            real_kernel(d, a, r, &k, &dk);
            nsum_add(&acc, q[js] * k);
            if (want_grad)
              for (int i = 0; i < d; ++i) nsum_add(&g[i], q[js] * dk * z[i] / r);
          }
    }
    pot[it] = nsum_get(&acc);
    if (want_grad)
      for (int i = 0; i < d; ++i) grad[d * it + i] = nsum_get(&g[i]);
  }
}

/* Enumerate reciprocal modes m != 0 with |k_m| <= kcut, one of each +-m pair
 * (the first nonzero component positive).  Returns the count; fills modes
 * (d ints each) and weights w(m) = e^{-k^2/4a^2}/k^2 and k-vectors. */
static long enum_modes(int d, const double* L, const double* Li, double a,
                       double kcut, int** modes_out, double** w_out,
                       double** kv_out) {
  long mmax[3] = {0, 0, 0};
  for (int i = 0; i < d; ++i) {
    double s = 0;
    for (int j = 0; j < d; ++j) s += L[j + d * i] * L[j + d * i];
    mmax[i] = (long)floor(sqrt(s) * kcut / (2.0 * OR_PI)) + 1;
  }
  long cap = 1;
  for (int i = 0; i < d; ++i) cap *= (2 * mmax[i] + 1);
  int* modes = (int*)malloc(sizeof(int) * d * cap);
  double* w = (double*)malloc(sizeof(double) * cap);
  double* kv = (double*)malloc(sizeof(double) * d * cap);
  long n = 0;
  long m3lo = d == 3 ? -mmax[2] : 0, m3hi = d == 3 ? mmax[2] : 0;
  for (long m3 = m3lo; m3 <= m3hi; ++m3)
    for (long m2 = -mmax[1]; m2 <= mmax[1]; ++m2)
      for (long m1 = -mmax[0]; m1 <= mmax[0]; ++m1) {
        long mm[3] = {m1, m2, m3};
        /* keep one representative of {m, -m}: first nonzero of (m_d..m_1) > 0 */
        int sgn = 0;
        for (int i = d - 1; i >= 0; --i)
          if (mm[i] != 0) { sgn = mm[i] > 0 ? 1 : -1; break; }
        if (sgn <= 0) continue;
        double k[3] = {0, 0, 0}, k2 = 0;
        for (int i = 0; i < d; ++i) {   /* k = 2 pi L^{-T} m: k_i = 2pi sum_j Li[j,i] m_j */
          double s = 0;
          for (int j = 0; j < d; ++j) s += Li[j + d * i] * (double)mm[j];
          k[i] = 2.0 * OR_PI * s;
          k2 += k[i] * k[i];
        }
        if (k2 > kcut * kcut) continue;
        for (int i = 0; i < d; ++i) { modes[d * n + i] = (int)mm[i]; kv[d * n + i] = k[i]; }
        w[n] = exp(-k2 / (4.0 * a * a)) / k2;
        ++n;
      }
  *modes_out = modes; *w_out = w; *kv_out = kv;
  return n;
}

/* Per-axis phase table e^{-2 pi i m v} for m in [-mmax, mmax], by direct sincos. */
static void axis_phases(double v, long mmax, double* re, double* im) {
  for (long m = -mmax; m <= mmax; ++m) {
    double t = -2.0 * OR_PI * (double)m * v;
    re[m + mmax] = cos(t);
    im[m + mmax] = sin(t);
  }
}

/* Fractional coordinate v = L^{-1} y */
static inline void frac(int d, const double* Li, const double* y, double* v) {
  for (int i = 0; i < d; ++i) {
    double s = 0;
    for (int j = 0; j < d; ++j) s += Li[i + d * j] * y[j];
    v[i] = s;
  }
}

/*
 * Structure factor S(m) = sum_j q_j e^{-2 pi i m.v_j} for the enumerated modes.
 */
static void structure_factor(int d, const double* Li, long n_src,
                             const double* src, const double* q, long nm,
                             const int* modes, double* Sre, double* Sim) {
  long mmax[3] = {0, 0, 0};
  for (long t = 0; t < nm; ++t)
    for (int i = 0; i < d; ++i) {
      long a = labs((long)modes[d * t + i]);
      if (a > mmax[i]) mmax[i] = a;
    }
  int nthreads = 1;
#ifdef _OPENMP
  nthreads = omp_get_max_threads();
#endif
  nsum* part = (nsum*)calloc((size_t)nthreads * 2 * nm, sizeof(nsum));
#pragma omp parallel
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    nsum* pr = part + (size_t)tid * 2 * nm;
    nsum* pi = pr + nm;
    double* tab = (double*)malloc(sizeof(double) * 2 * (2 * (mmax[0] + mmax[1] + mmax[2]) + 3));
    double *re[3], *im[3];
    long off = 0;
    for (int i = 0; i < d; ++i) {
      re[i] = tab + off; off += 2 * mmax[i] + 1;
      im[i] = tab + off; off += 2 * mmax[i] + 1;
    }
#pragma omp for schedule(static)
    for (long j = 0; j < n_src; ++j) {
      double v[3];
      frac(d, Li, src + d * j, v);
      for (int i = 0; i < d; ++i) axis_phases(v[i], mmax[i], re[i], im[i]);
      for (long t = 0; t < nm; ++t) {
        double cr = 1.0, ci = 0.0;
        for (int i = 0; i < d; ++i) {
          long m = modes[d * t + i] + mmax[i];
          double nr = cr * re[i][m] - ci * im[i][m];
          double ni = cr * im[i][m] + ci * re[i][m];
          cr = nr; ci = ni;
        }
        nsum_add(&pr[t], q[j] * cr);
        nsum_add(&pi[t], q[j] * ci);
      }
    }
    free(tab);
  }
  for (long t = 0; t < nm; ++t) {
    nsum a = {0, 0}, b = {0, 0};
    for (int th = 0; th < nthreads; ++th) {
      nsum_add(&a, nsum_get(&part[(size_t)th * 2 * nm + t]));
      nsum_add(&b, nsum_get(&part[(size_t)th * 2 * nm + nm + t]));
    }
    Sre[t] = nsum_get(&a);
    Sim[t] = nsum_get(&b);
  }
  free(part);
}

/*
 * Reciprocal part at targets: (1/V) sum_{m != 0} w(m) Re[e^{2 pi i m.u} S(m)]
 * (each +-m pair counted once, hence the factor 2), and its gradient
 * (1/V) sum w(m) Re[i k_m e^{2 pi i m.u} S(m)].
 */
static void reciprocal(int d, const double* Li, double V, long nm,
                       const int* modes, const double* w, const double* kv,
                       const double* Sre, const double* Sim, long n_trg,
                       const double* trg, int want_grad, double* pot,
                       double* grad) {
  long mmax[3] = {0, 0, 0};
  for (long t = 0; t < nm; ++t)
    for (int i = 0; i < d; ++i) {
      long a = labs((long)modes[d * t + i]);
      if (a > mmax[i]) mmax[i] = a;
    }
#pragma omp parallel
  {
    double* tab = (double*)malloc(sizeof(double) * 2 * (2 * (mmax[0] + mmax[1] + mmax[2]) + 3));
    double *re[3], *im[3];
    long off = 0;
    for (int i = 0; i < d; ++i) {
      re[i] = tab + off; off += 2 * mmax[i] + 1;
      im[i] = tab + off; off += 2 * mmax[i] + 1;
    }
#pragma omp for schedule(dynamic, 8)
    for (long it = 0; it < n_trg; ++it) {
      double u[3];
      frac(d, Li, trg + d * it, u);
      /* tables hold e^{-2 pi i m u}; conjugate gives e^{+2 pi i m u} */
      for (int i = 0; i < d; ++i) axis_phases(u[i], mmax[i], re[i], im[i]);
      nsum acc = {0, 0}, g[3] = {{0, 0}, {0, 0}, {0, 0}};
      for (long t = 0; t < nm; ++t) {
        double cr = 1.0, ci = 0.0;
        for (int i = 0; i < d; ++i) {
          long m = modes[d * t + i] + mmax[i];
          double er = re[i][m], ei = -im[i][m];
          double nr = cr * er - ci * ei;
          double ni = cr * ei + ci * er;
          cr = nr; ci = ni;
        }
        /* e^{2 pi i m u} S(m) */
        double pr = cr * Sre[t] - ci * Sim[t];
        double pim = cr * Sim[t] + ci * Sre[t];
        nsum_add(&acc, 2.0 * w[t] * pr);
        if (want_grad)   /* Re[i k z] = -k Im z */
          for (int i = 0; i < d; ++i) nsum_add(&g[i], -2.0 * w[t] * kv[d * t + i] * pim);
      }
      pot[it] = nsum_get(&acc) / V;
      if (want_grad)
        for (int i = 0; i < d; ++i) grad[d * it + i] = nsum_get(&g[i]) / V;
    }
    free(tab);
  }
}

/*
 * Full Ewald evaluation.
 *   d        : 2 or 3
 *   L        : lattice (column-major, columns are lattice vectors)
 *   src, q   : n_src positions (row-major n_src x d) and charges
 *   trg      : n_trg positions (row-major)
 *   self_idx : per target the index of its coincident source, or -1; NULL = none
 *   alpha    : Ewald splitting parameter; rcut, kcut the real / reciprocal cutoffs
 *   pot      : n_trg potentials (out); grad : n_trg x d gradients (out) or NULL
 * Returns 0 on success, nonzero on invalid input.
 */
int oracle_ewald(int d, const double* L, long n_src, const double* src,
                 const double* q, long n_trg, const double* trg,
                 const long* self_idx, double alpha, double rcut, double kcut,
                 double* pot, double* grad) {
  if ((d != 2 && d != 3) || n_src < 0 || n_trg < 0 || alpha <= 0) return 1;
  double Li[9];
  double det = inv_small(d, L, Li);
  if (!(fabs(det) > 0)) return 2;
  double V = fabs(det);
  int want_grad = grad != NULL;

  double* pr = (double*)calloc(n_trg > 0 ? n_trg : 1, sizeof(double));
  double* gr = want_grad ? (double*)calloc((n_trg > 0 ? n_trg : 1) * d, sizeof(double)) : NULL;
  real_space(d, L, Li, n_src, src, q, n_trg, trg, self_idx, alpha, rcut,
             want_grad, pot, grad);

  int* modes; double *w, *kv;
  long nm = enum_modes(d, L, Li, alpha, kcut, &modes, &w, &kv);
  double* Sre = (double*)calloc(nm > 0 ? nm : 1, sizeof(double));
  double* Sim = (double*)calloc(nm > 0 ? nm : 1, sizeof(double));
  structure_factor(d, Li, n_src, src, q, nm, modes, Sre, Sim);
  reciprocal(d, Li, V, nm, modes, w, kv, Sre, Sim, n_trg, trg, want_grad, pr, gr);

  nsum qs = {0, 0};
  for (long j = 0; j < n_src; ++j) nsum_add(&qs, q[j]);
  double qtot = nsum_get(&qs);
  double self_c = d == 3 ? alpha / (2.0 * pow(OR_PI, 1.5))
                         : (OR_EULER_GAMMA + 2.0 * log(alpha)) / (4.0 * OR_PI);
  double jell = qtot / (4.0 * alpha * alpha * V);
  for (long it = 0; it < n_trg; ++it) {
    nsum a = {0, 0};
    nsum_add(&a, pot[it]);
    nsum_add(&a, pr[it]);
    long s = self_idx ? self_idx[it] : -1;
    if (s >= 0) nsum_add(&a, -q[s] * self_c);
    nsum_add(&a, -jell);
    pot[it] = nsum_get(&a);
    if (want_grad)
      for (int i = 0; i < d; ++i) grad[d * it + i] += gr[d * it + i];
  }
  free(pr); free(gr); free(modes); free(w); free(kv); free(Sre); free(Sim);
  return 0;
}

/* Number of reciprocal modes (one per +-pair) the evaluation would use;
 * lets the caller balance alpha before committing to a run. */
long oracle_ewald_nmodes(int d, const double* L, double alpha, double kcut) {
  double Li[9];
  inv_small(d, L, Li);
  int* modes; double *w, *kv;
  long nm = enum_modes(d, L, Li, alpha, kcut, &modes, &w, &kv);
  free(modes); free(w); free(kv);
  return nm;
}

/* Brute-force image sum over whole cells n with |L n| <= R (a ball in 3D, a
 * disc in 2D), plain G, self pair skipped.  Used only to pin the Ewald code
 * against the definition by extrapolation in R. */
int oracle_ball_sum(int d, const double* L, long n_src, const double* src,
                    const double* q, long n_trg, const double* trg,
                    const long* self_idx, double R, double* pot) {
  double Li[9];
  inv_small(d, L, Li);
  long nmax[3] = {0, 0, 0};
  for (int i = 0; i < d; ++i) {
    double s = 0;
    for (int j = 0; j < d; ++j) s += Li[i + d * j] * Li[i + d * j];
    nmax[i] = (long)ceil(sqrt(s) * R) + 1;
  }
  long n3lo = d == 3 ? -nmax[2] : 0, n3hi = d == 3 ? nmax[2] : 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (long it = 0; it < n_trg; ++it) {
    nsum acc = {0, 0};
    const double* x = trg + d * it;
    long self = self_idx ? self_idx[it] : -1;
    for (long n3 = n3lo; n3 <= n3hi; ++n3)
      for (long n2 = -nmax[1]; n2 <= nmax[1]; ++n2)
        for (long n1 = -nmax[0]; n1 <= nmax[0]; ++n1) {
          long nn[3] = {n1, n2, n3};
          double t[3] = {0, 0, 0}, t2 = 0;
          for (int i = 0; i < d; ++i) {
            for (int j = 0; j < d; ++j) t[i] += L[i + d * j] * (double)nn[j];
            t2 += t[i] * t[i];
          }
          if (t2 > R * R) continue;
          for (long js = 0; js < n_src; ++js) {
            if (js == self && n1 == 0 && n2 == 0 && n3 == 0) continue;
            double r2 = 0;
            for (int i = 0; i < d; ++i) {
              double z = x[i] - src[d * js + i] - t[i];
              r2 += z * z;
            }
            double g = d == 3 ? 1.0 / (4.0 * OR_PI * sqrt(r2))
                              : -log(r2) / (4.0 * OR_PI);
            nsum_add(&acc, q[js] * g);
          }
        }
    pot[it] = nsum_get(&acc);
  }
  return 0;
}

/* Number of OpenMP threads the sums above run on. */
int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

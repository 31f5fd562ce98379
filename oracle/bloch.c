/*
 * Reference Ewald summation for quasi-periodic (Bloch) Laplace lattice sums.
 *
 * TEST INFRASTRUCTURE ONLY, like ewald.c (same library, same rules): the
 * slow, plain, double-precision oracle for the Bloch evaluation; it shares
 * no code with the GPU library.
 *
 * What is computed (Section 4.1, eq:qp_def): for a Bloch vector beta, real
 * charges q_j at positions y_j (anywhere in R^d, taken literally: the image
 * of y_j at y_j + L n carries the charge q_j e^{i beta.L n}),
 *
 *     Phi(x) = sum_n sum_j q_j e^{i beta.L n} G(x - y_j - L n),
 *
 * the singular self pair (n = 0, coincident source) removed.  It satisfies
 * Phi(x + L n) = e^{i beta.L n} Phi(x).  By Poisson summation the sum is
 *
 *     Phi(x) = (1/V) sum_{m in Z^d} |k_m + beta|^-2 sum_j q_j e^{i (k_m + beta).(x - y_j)},
 *
 * every mode kept (finite when beta is not in the reciprocal lattice; no
 * neutrality needed).  The Ewald split of ewald.c applies mode by mode: the
 * real-space sum carries the image phases, the reciprocal sum runs over the
 * shifted wave vectors k_m + beta with weights e^{-|k|^2/4a^2}/|k|^2, and the
 * smooth part's value at r = 0 is removed for a target coincident with a
 * source (the n = 0 image has phase 1):
 *     3D: a / (2 pi^{3/2}),   2D: (gamma + 2 ln a) / (4 pi).
 * No uniform-background term arises: the k = beta mode is an ordinary term.
 *
 * Lattice convention as in ewald.c (columns of the column-major L).
 */
#include <math.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define BL_PI 3.14159265358979323846264338327950288
#define BL_EULER_GAMMA 0.57721566490153286060651209008240243

typedef struct { double s, c; } bsum;   /* Neumaier accumulator */

static inline void bsum_add(bsum* a, double v) {
  double t = a->s + v;
  if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
  else a->c += (v - t) + a->s;
  a->s = t;
}
static inline double bsum_get(const bsum* a) { return a->s + a->c; }

double oracle_expint_e1(double x);   /* ewald.c */

static int inv_lattice(int d, const double* L, double* Li) {
  double det;
  if (d == 2) {
    det = L[0] * L[3] - L[2] * L[1];
    if (det == 0.0) return -1;
    Li[0] = L[3] / det; Li[3] = L[0] / det;
    Li[2] = -L[2] / det; Li[1] = -L[1] / det;
  } else {
    const double a = L[0], b = L[3], c = L[6], e = L[1], f = L[4], g = L[7];
    const double h = L[2], i = L[5], k = L[8];
    det = a * (f * k - g * i) - b * (e * k - g * h) + c * (e * i - f * h);
    if (det == 0.0) return -1;
    Li[0] = (f * k - g * i) / det; Li[3] = -(b * k - c * i) / det; Li[6] = (b * g - c * f) / det;
    Li[1] = -(e * k - g * h) / det; Li[4] = (a * k - c * h) / det; Li[7] = -(a * g - c * e) / det;
    Li[2] = (e * i - f * h) / det; Li[5] = -(a * i - b * h) / det; Li[8] = (a * f - b * e) / det;
  }
  return 0;
}

/*
 * Potential (real and imaginary parts) at n_trg targets.  self_idx[i] (or
 * NULL) names the source coincident with target i (its n = 0 pair is
 * skipped and the smooth part's value at 0 removed).  Returns 0, or -1 for a
 * singular lattice, -2 when beta lies in the reciprocal lattice.
 */
int oracle_ewald_bloch(int d, const double* L, const double* beta, long n_src,
                       const double* src, const double* q, long n_trg, const double* trg,
                       const long* self_idx, double a, double rcut, double kcut,
                       double* pot_re, double* pot_im) {
  double Li[9];
  if (inv_lattice(d, L, Li)) return -1;
  double V = 1.0;
  {
    /* |det L| from the inverse's determinant is avoided: direct formula */
    if (d == 2) V = fabs(L[0] * L[3] - L[2] * L[1]);
    else V = fabs(L[0] * (L[4] * L[8] - L[7] * L[5]) - L[3] * (L[1] * L[8] - L[7] * L[2]) +
                  L[6] * (L[1] * L[5] - L[4] * L[2]));
  }
  /* beta in the reciprocal lattice: L^T beta / 2 pi integral */
  {
    int all_int = 1;
    for (int i = 0; i < d; ++i) {
      double s = 0;
      for (int j = 0; j < d; ++j) s += L[j + d * i] * beta[j];
      s /= 2.0 * BL_PI;
      if (fabs(s - rint(s)) > 1e-12) all_int = 0;
    }
    if (all_int) return -2;
  }
  /* real space */
  double b[3] = {0, 0, 0};
  for (int i = 0; i < d; ++i) {
    double s = 0;
    for (int j = 0; j < d; ++j) s += Li[i + d * j] * Li[i + d * j];
    b[i] = sqrt(s) * rcut;
  }
  const double rc2 = rcut * rcut;
#pragma omp parallel for schedule(dynamic, 4)
  for (long it = 0; it < n_trg; ++it) {
    bsum ar = {0, 0}, ai = {0, 0};
    const double* x = trg + d * it;
    const long self = self_idx ? self_idx[it] : -1;
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
      const long n3lo = d == 3 ? lo[2] : 0, n3hi = d == 3 ? hi[2] : 0;
      for (long n3 = n3lo; n3 <= n3hi; ++n3)
        for (long n2 = lo[1]; n2 <= hi[1]; ++n2)
          for (long n1 = lo[0]; n1 <= hi[0]; ++n1) {
            const long nn[3] = {n1, n2, n3};
            if (js == self && n1 == 0 && n2 == 0 && n3 == 0) continue;
            double z[3] = {0, 0, 0}, r2 = 0, ph = 0;
            for (int i = 0; i < d; ++i) {
              double Ln = 0;
              for (int j = 0; j < d; ++j) Ln += L[i + d * j] * (double)nn[j];
              z[i] = dx[i] - Ln;
              r2 += z[i] * z[i];
              ph += beta[i] * Ln;
            }
            if (r2 >= rc2) continue;
            const double r = sqrt(r2);
            const double k = d == 3 ? erfc(a * r) / (4.0 * BL_PI * r)
                                    : oracle_expint_e1(a * a * r * r) / (4.0 * BL_PI);
            bsum_add(&ar, q[js] * k * cos(ph));
            bsum_add(&ai, q[js] * k * sin(ph));
          }
    }
    pot_re[it] = bsum_get(&ar);
    pot_im[it] = bsum_get(&ai);
  }
  /* reciprocal space: modes m with |k_m + beta| <= kcut */
  double bn = 0;
  for (int i = 0; i < d; ++i) bn += beta[i] * beta[i];
  bn = sqrt(bn);
  long mmax[3] = {0, 0, 0};
  for (int i = 0; i < d; ++i) {
    double s = 0;
    for (int j = 0; j < d; ++j) s += L[j + d * i] * L[j + d * i];
    mmax[i] = (long)floor(sqrt(s) * (kcut + bn) / (2.0 * BL_PI)) + 1;
  }
  long cap = 1;
  for (int i = 0; i < d; ++i) cap *= 2 * mmax[i] + 1;
  double* kv = (double*)malloc(sizeof(double) * 3 * cap);
  double* w = (double*)malloc(sizeof(double) * cap);
  long nm = 0;
  const long m3lo = d == 3 ? -mmax[2] : 0, m3hi = d == 3 ? mmax[2] : 0;
  for (long m3 = m3lo; m3 <= m3hi; ++m3)
    for (long m2 = -mmax[1]; m2 <= mmax[1]; ++m2)
      for (long m1 = -mmax[0]; m1 <= mmax[0]; ++m1) {
        const long mm[3] = {m1, m2, m3};
        double k[3] = {0, 0, 0}, k2 = 0;
        for (int i = 0; i < d; ++i) {   /* k = 2 pi L^{-T} m + beta */
          double s = 0;
          for (int j = 0; j < d; ++j) s += Li[j + d * i] * (double)mm[j];
          k[i] = 2.0 * BL_PI * s + beta[i];
          k2 += k[i] * k[i];
        }
        if (k2 > kcut * kcut) continue;
        for (int i = 0; i < 3; ++i) kv[3 * nm + i] = k[i];
        w[nm] = exp(-k2 / (4.0 * a * a)) / k2 / V;
        ++nm;
      }
  /* structure factor S(k) = sum_j q_j e^{-i k.y_j} */
  double* Sr = (double*)calloc(nm, sizeof(double));
  double* Si = (double*)calloc(nm, sizeof(double));
#pragma omp parallel for schedule(dynamic, 16)
  for (long t = 0; t < nm; ++t) {
    bsum sr = {0, 0}, si = {0, 0};
    for (long j = 0; j < n_src; ++j) {
      double ph = 0;
      for (int i = 0; i < d; ++i) ph += kv[3 * t + i] * src[d * j + i];
      bsum_add(&sr, q[j] * cos(ph));
      bsum_add(&si, -q[j] * sin(ph));
    }
    Sr[t] = bsum_get(&sr);
    Si[t] = bsum_get(&si);
  }
#pragma omp parallel for schedule(dynamic, 4)
  for (long it = 0; it < n_trg; ++it) {
    bsum ar = {0, 0}, ai = {0, 0};
    const double* x = trg + d * it;
    for (long t = 0; t < nm; ++t) {
      double ph = 0;
      for (int i = 0; i < d; ++i) ph += kv[3 * t + i] * x[i];
      const double c = cos(ph), s = sin(ph);
      /* w e^{i ph} S */
      bsum_add(&ar, w[t] * (c * Sr[t] - s * Si[t]));
      bsum_add(&ai, w[t] * (c * Si[t] + s * Sr[t]));
    }
    double self = 0.0;
    if (self_idx && self_idx[it] >= 0) {
      const double qs = q[self_idx[it]];
      self = d == 3 ? qs * a / (2.0 * pow(BL_PI, 1.5))
                    : qs * (BL_EULER_GAMMA + 2.0 * log(a)) / (4.0 * BL_PI);
    }
    pot_re[it] += bsum_get(&ar) - self;
    pot_im[it] += bsum_get(&ai);
  }
  free(kv);
  free(w);
  free(Sr);
  free(Si);
  return 0;
}

// Lagrange interpolation at Chebyshev nodes for the proxy grids (device
// helpers shared by the near-field translation units).
#pragma once
#include <hip/hip_runtime.h>

namespace pdmk {

// 1/d from the hardware reciprocal estimate refined by NR Newton steps
// (r <- r + r (1 - d r)); each step squares the relative error: two leave the
// result within a few units in the last place of the correctly rounded
// quotient, one is ample for rows that are rounded to FP32.
template <int NR = 2>
__device__ inline double recip_nr(double d) {
  double r = __builtin_amdgcn_rcp(d);
#pragma unroll
  for (int k = 0; k < NR; ++k) r = fma(r, fma(-d, r, 1.0), r);
  return r;
}

// Lagrange basis at the p Chebyshev nodes (barycentric form), and optionally
// its derivative.  x exactly at a node is moved by 1e-13.
template <class T>
__device__ inline void lagrange_rows(int p, const double* __restrict__ nodes,
                                     const double* __restrict__ bw, double x,
                                     T* row, T* drow) {
  for (int j = 0; j < p; ++j)
    if (x == nodes[j]) { x += 1e-13; break; }
  // reciprocals by Newton-refined hardware estimates (recomputed in the
  // second loop: cheaper than keeping p of them)
  double s = 0.0, s1 = 0.0;
  for (int j = 0; j < p; ++j) {
    double inv = recip_nr<2>(x - nodes[j]);
    double t = bw[j] * inv;
    s += t;
    s1 += t * inv;
  }
  double is = recip_nr<2>(s);
  for (int j = 0; j < p; ++j) {
    // l_j = (w_j/(x - x_j)) / S;  l_j' = l_j (-1/(x - x_j) + S1/S),  S1 = sum w_k/(x-x_k)^2
    const double inv = recip_nr<2>(x - nodes[j]);
    const double lj = bw[j] * inv * is;
    row[j] = (T)lj;
    if (drow) drow[j] = (T)(lj * (-inv + s1 * is));
  }
}


// Same as lagrange_rows with compile-time capacity PMAX (entries >= p are 0),
// so the rows stay in registers; NR Newton steps per reciprocal.
template <int PMAX, bool DER, int NR = 2>
__device__ inline void lagrange_rows_reg(int p, const double* __restrict__ nodes,
                                         const double* __restrict__ bw, double x,
                                         double (&row)[PMAX], double (&drow)[PMAX]) {
#pragma unroll
  for (int m = 0; m < PMAX; ++m)
    if (m < p && x == nodes[m]) x += 1e-13;
  double s = 0.0, s1 = 0.0;
  double inv[PMAX];
#pragma unroll
  for (int m = 0; m < PMAX; ++m) {
    if (m < p) {
      inv[m] = recip_nr<NR>(x - nodes[m]);
      const double t = bw[m] * inv[m];
      row[m] = t;
      s += t;
      s1 += t * inv[m];
    } else {
      inv[m] = 0.0;
      row[m] = 0.0;
    }
  }
  const double is = 1.0 / s;
#pragma unroll
  for (int m = 0; m < PMAX; ++m) {
    const double lj = row[m] * is;
    if (DER) drow[m] = lj * (s1 * is - inv[m]);
    row[m] = lj;
  }
}

}  // namespace pdmk

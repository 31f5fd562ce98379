// Host-side planning for periodic DMK: prolate spheroidal wave function,
// kernel-splitting tables, lattice orientation, root grid, image shifts,
// Fourier grid, spreading window.  Pure C++ (no device code).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace pdmk {

constexpr double kPi = 3.14159265358979323846264338327950288;

// Gauss-Legendre rule on [-1, 1].
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);

// Zeroth prolate spheroidal wave function psi_0^c (Section 2.2).
struct Pswf {
  double eps = 0, c = 0;
  std::vector<double> leg;   // coefficients in the standard Legendre basis P_k
  double psi0 = 0;           // psi(0)
  double c0 = 0;             // int_0^1 psi (eq:Phic)
  double lambda0 = 0;        // eigenvalue of eq:pswf_eig: lambda0 psi(0) = int_{-1}^1 psi
  double psit_dd0 = 0;       // second derivative at 0 of the normalised psi~
  // quadrature of psi on [-1,1] used for the entire extension of psi~
  std::vector<double> qx, qw, qpsi;

  double psi(double x) const;          // Legendre series, |x| <= 1
  double phi(double t) const;          // (1/c0) int_0^t psi, = 1 for t >= 1 (eq:Phic)
  double psit(double x) const;         // psi~(x) = psi(x)/psi(0) extended as an entire function
};

// psi with bandwidth c; calibrate_c finds c with psi(1)/psi(0) = eps.
Pswf make_pswf_c(double c);
double calibrate_c(double eps);
const Pswf& pswf_for_eps(double eps);   // cached per eps

// Chebyshev series on [0, 1] in the variable s: f(s) = sum_k a_k T_k(2s - 1).
struct ChebSeries {
  std::vector<double> a;
  double operator()(double s) const;
  double deriv(double s) const;        // d/ds
};

// Kernel-splitting tables for one eps (eq:pswf_split and its 2D analogue).
//   3D: R_h(r) = (1/4pi) [1/r - E(r^2/h^2)/h]            for r < h, else 0
//       with phi(t) = t E(t^2);  W_h(0) = E(0) / (4 pi h)
//   2D: R_h(r) = -(1/2pi) log(r/h) + F2(r^2/h^2)/(2pi)  for r < h, else 0
//       F2(s) = log(1 + sqrt(1-s)) - int_0^{sqrt(1-s)} E(s + v^2) dv
//       (the residual is the line integral of the 3D residual along the
//       third axis, both having the same radial Fourier profile);
//       W_h(0) = -(1/2pi) log h - F2(0)/(2pi)
struct SplitTables {
  double eps = 0, c = 0;
  ChebSeries E;     // phi(sqrt(s))/sqrt(s)
  ChebSeries F2;    // 2D smooth part
  double w0_unit(int dim) const;       // W_h(0) for h = 1
  double residual(int dim, double r, double h) const;
  double residual_dr(int dim, double r, double h) const;   // dR/dr
  // Fourier multiplier of level l's difference kernel divided by the
  // period volume, as a function of the integer mode norm^2 n = |j|^2 for
  // period 3h:  (3h)^{2-d} * dtab[n]
  std::vector<double> dtab;   // filled by prepare_pw
  void prepare_pw(int jmax, int dim);
};
const SplitTables& tables_for_eps(double eps);

// Default method parameters for (dim, eps).
struct MethodParams {
  double kappa;
  int n_s;
  int porder;   // proxy points per axis
  int npw;      // plane-wave half count J
  int nufft_w;  // window width (grid cells)
  double beta;  // ES window shape
  double sigma; // Fourier grid upsampling factor
};
// ES window shape for a width and an upsampling factor.
double window_beta(int w, double sigma);
MethodParams default_params(int dim, double eps);

// Geometry of one lattice (Sections 3.2-3.4, 3.7).
struct Geometry {
  int dim = 3;
  double L[9] = {0};        // oriented, upper triangular, column-major
  double Li[9] = {0};       // inverse of L, column-major
  double Q[9] = {0};        // x_oriented = Q^T x, column-major
  int perm[3] = {0, 1, 2};
  double volume = 0;
  double Lmin = 0;
  double rc = 0;
  double xlo[3] = {0};      // bounding box corner x^-
  double width[3] = {0};    // w_i
  int nroot[3] = {1, 1, 1}; // m_i
  int next[3] = {1, 1, 1};  // m_i + 2
  double origin[3] = {0};   // x^- - r_c
  std::vector<int> shifts;  // dim ints per surviving lattice shift
  int fgrid_paper[3] = {1, 1, 1};
  int fgrid[3] = {1, 1, 1};
  // images as virtual neighbours (rem:cube): the root grid tiles the cell and
  // colleagues wrap around it; no halo, no image points
  bool virtual_images = false;
};
// Returns empty string on success, else a message.
// beta_norm: |beta| of a Bloch vector (0: periodic), which enlarges the
// Fourier grid (Section 4.1).
// virtual_images: the cube-cell construction of rem:cube, for rectangular
// cells whose edges are whole multiples of r_c (a message starting with
// "unsupported:" otherwise).
std::string make_geometry(int dim, const double* Lin, double kappa, double c,
                          double sigma, Geometry& g, double beta_norm = 0.0,
                          bool virtual_images = false);

// Smallest even integer >= n whose prime factors are 2, 3, 5.
int next_fft_size(int n);

// Spreading window exp(beta (sqrt(1 - z^2) - 1)), |z| < 1, z = x / (w/2)
// with x in grid cells; its Fourier transform on the grid frequencies
// m = -M/2 .. M/2-1 (returned in FFT order: index n <-> m = n or n - M).
std::vector<double> window_ft(int M, int w, double beta);

// Chebyshev (first kind) nodes and barycentric weights on [-1, 1].
void cheb_nodes(int p, std::vector<double>& x, std::vector<double>& bw);
// l_j(x) for all j (Lagrange basis at Chebyshev nodes).
void lagrange_row(int p, const double* nodes, const double* bw, double x, double* out);

}  // namespace pdmk

// Host-side FP64 mathematics of the PSWF-LR path: the prolate window and
// mollifier, the Fourier kernels Phi_p, piecewise-polynomial tables for the
// device (FKAD-style fits), and parameter selection.
#pragma once

#include <cstdint>
#include <memory>
#include <vector>

namespace pswf {

// Gauss-Legendre nodes and weights on [a, b] (Newton on the Legendre
// recurrence; Golub-Welsch is not needed at these orders).
void gauss_legendre(int n, double a, double b, std::vector<double> &x, std::vector<double> &w);

// Order-zero prolate spheroidal wave function psi_0^c with psi(0) = 1
// (Methods, "Prolate spheroidal wave functions", eqs. formula and
// psidefinit).  Computed from the prolate differential operator, which
// commutes with F_c, by Chebyshev collocation and inverse iteration;
// evaluated anywhere by barycentric interpolation; lambda_0 = int psi
// (eq. psidefinit at x = 0).
class Prolate {
 public:
  explicit Prolate(double c, int N = 96);
  double c() const { return c_; }
  double lambda() const { return lam_; }
  double C0() const { return 0.5 * lam_; }          // int_0^1 psi
  double operator()(double x) const;                // psi(x), |x| <= 1
  double d1(double x) const;                        // psi'(x)
  double d2(double x) const;                        // psi''(x)
  double deriv0(int n) const;                       // psi^(n)(0), n even
  double chi() const { return chi_; }               // prolate ODE eigenvalue
  double I0(double k) const;                        // int_0^k psi
  double J1(double k) const;                        // int_k^1 u psi(u) du
  double J3(double k) const;                        // int_k^1 u^3 psi(u) du
  double T3(double k) const;                        // int_k^1 (psi(u)-1)/u du
  // Fourier transform of the compact window psi(x) on [-1, 1] at any s:
  // int_{-1}^{1} psi(t) cos(s t) dt  (equals lambda psi(s/c) for |s| <= c).
  double window_ft(double s) const;

 private:
  double bary(const std::vector<double> &f, double x) const;
  double c_ = 0, lam_ = 0, chi_ = 0;
  std::vector<double> x_, bw_, psi_, dpsi_, d2psi_;  // collocation nodes, values
  std::vector<double> qx_, qw_;                      // quadrature on [0,1] for integrals
  std::vector<double> fx_, fwpsi_;                   // window-transform nodes, 2 w psi
};

// Shared, cached instances (plan creation is cheap after the first call).
std::shared_ptr<const Prolate> prolate_cached(double c);

// Deconvolution factors of one grid axis, h^2 / What(k)^2 at the grid
// frequencies k = 2 pi f / (M h), f = 0 .. M / 2: the window transform
// depends on f / M only (What(k) / h = (P / 2) window_ft(pi P f / M)), so a
// table serves every box with that (c_s, P, M).  Cached.
std::shared_ptr<const std::vector<float>> deconvolution_cached(double c_s, int P, int M);

// Device representation of a smooth function on [0, 1]: nseg uniform
// segments, each a monomial in the local variable tau in [-1, 1] of degree
// deg (coefficients low to high).  Built by Chebyshev interpolation on each
// segment, dropping coefficients below 0.01 * eps * max (Methods,
// "Parameter selection", polynomial degree selection), then converting the
// truncated Chebyshev series to monomials.
struct PiecewisePoly {
  int nseg = 0, deg = 0;
  std::vector<double> coef;   // [nseg][deg + 1]
  double max_abs_err = 0;     // measured on a dense check grid
  double eval(double x) const;
};
template <class F>
PiecewisePoly fit_piecewise(F f, int nseg, int deg, double eps);

// psi_{c_s} on [0, 1] for the spreading window (even: the device uses |t|).
PiecewisePoly make_window_poly(double c_s, int nseg, int deg, double eps);

// Per-channel kernel representation used by the device (see kernels.hip):
//   Phi(k)      = A * kappa^eA * f(kappa) + B * kappa^eB * ln(kappa)
//   Phi'(k) / k = Cc * kappa^eC * g(kappa) + D * kappa^eD * ln(kappa)
// with kappa = k r_c / c in (0, 1], and Phi = 0 for kappa > 1.
struct ChannelKernel {
  int p = 1;
  double A = 0, B = 0, Cc = 0, D = 0;
  int eA = 0, eB = 0, eC = 0, eD = 0;
  PiecewisePoly f, g;
  double self_coef = 0;   // E_self = self_coef * sum q^2
  double zero_coef_V = 0; // E_0 = zero_coef_V / V * Q^2
};
ChannelKernel make_channel_kernel(int p, double c, double r_c, double eps);

// Real-space complement 1 - G_p(rho) of the mollifier (Eqs. G1, G6, G;
// rho = r / r_c, zero for rho >= 1), and its device representation on
// [0, 1] (the pair kernel is (1 - G_p(r / r_c)) / r^p; its derivative comes
// from the polynomial's).
double mollifier_complement(const Prolate &ps, int p, double rho);
PiecewisePoly make_complement_poly(int p, double c, int nseg, int deg, double eps);

// Exact (FP64) Phi_p(k) and Phi_p'(k) from the closed forms, for checks.
double phi_hat(const Prolate &ps, int p, double k, double c, double r_c);
double phi_hat_deriv(const Prolate &ps, int p, double k, double c, double r_c);

// Window-bandwidth selection: minimises a force-weighted RMS aliasing ratio
// of the truncated PSWF window over the k-ball (see host_math.cpp).
double estimate_spread_error(int P, double eta, double c_s, double c_mollifier);
double choose_c_spread(int P, double eta, double c_mollifier);
// estimate_spread_error at the next grid point of eta (step 1/40) with its
// chosen window bandwidth, cached: a conservative value for the support choice
double spread_error_bound(int P, double eta, double c_mollifier);

// Smallest M >= x whose only prime factors are 2, 3, 5 (and even if asked).
int smooth_size(double x, bool even);
bool is_smooth235(int m);

}  // namespace pswf

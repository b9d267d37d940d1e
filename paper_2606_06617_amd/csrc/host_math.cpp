// Host-side FP64 mathematics of the PSWF-LR path (see host_math.hpp).
#include "host_math.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <stdexcept>
#include <tuple>

namespace pswf {

static const double kPi = 3.14159265358979323846264338327950288;

void gauss_legendre(int n, double a, double b, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = 0.0;
      for (int k = 1; k <= n; ++k) {
        double p2 = p1;
        p1 = p0;
        p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
      }
      dp = n * (z * p0 - p1) / (z * z - 1.0);
      double dz = p0 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = 0.0;
    for (int k = 1; k <= n; ++k) {
      double p2 = p1;
      p1 = p0;
      p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
    }
    dp = n * (z * p0 - p1) / (z * z - 1.0);
    double wi = 2.0 / ((1.0 - z * z) * dp * dp);
    // z is the i-th largest root
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = wi;
    w[n - 1 - i] = wi;
  }
  for (int i = 0; i < n; ++i) {
    x[i] = 0.5 * (b - a) * (x[i] + 1.0) + a;
    w[i] *= 0.5 * (b - a);
  }
}

// LU factorisation with partial pivoting (row-major n x n), in place.
static bool lu_factor(int n, std::vector<double> &a, std::vector<int> &piv) {
  piv.resize(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(a[size_t(i) * n + k]) > std::fabs(a[size_t(p) * n + k])) p = i;
    piv[k] = p;
    if (a[size_t(p) * n + k] == 0.0) return false;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(a[size_t(k) * n + j], a[size_t(p) * n + j]);
    const double inv = 1.0 / a[size_t(k) * n + k];
    for (int i = k + 1; i < n; ++i) {
      const double f = a[size_t(i) * n + k] * inv;
      a[size_t(i) * n + k] = f;
      if (f != 0.0)
        for (int j = k + 1; j < n; ++j) a[size_t(i) * n + j] -= f * a[size_t(k) * n + j];
    }
  }
  return true;
}

static void lu_solve(int n, const std::vector<double> &lu, const std::vector<int> &piv, std::vector<double> &b) {
  // the factorisation swapped whole rows (multipliers included): apply all
  // interchanges to b first, then the unit-lower solve
  for (int k = 0; k < n; ++k) std::swap(b[k], b[piv[k]]);
  for (int k = 0; k < n; ++k)
    for (int i = k + 1; i < n; ++i) b[i] -= lu[size_t(i) * n + k] * b[k];
  for (int i = n - 1; i >= 0; --i) {
    double s = b[i];
    for (int j = i + 1; j < n; ++j) s -= lu[size_t(i) * n + j] * b[j];
    b[i] = s / lu[size_t(i) * n + i];
  }
}

// Chebyshev-Gauss-Lobatto nodes x_j = cos(pi j / N) and the collocation
// differentiation matrix (the classical closed form with the negative-sum
// diagonal).
static void cheb_matrix(int N, std::vector<double> &x, std::vector<double> &D) {
  const int n = N + 1;
  x.resize(n);
  for (int j = 0; j < n; ++j) x[j] = std::cos(kPi * j / N);
  x[N / 2] = (N % 2 == 0) ? 0.0 : x[N / 2];
  std::vector<double> cw(n, 1.0);
  cw[0] = cw[N] = 2.0;
  D.assign(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) {
    double rowsum = 0.0;
    for (int j = 0; j < n; ++j) {
      if (i == j) continue;
      const double sgn = ((i + j) % 2 == 0) ? 1.0 : -1.0;
      const double v = (cw[i] / cw[j]) * sgn / (x[i] - x[j]);
      D[size_t(i) * n + j] = v;
      rowsum += v;
    }
    D[size_t(i) * n + i] = -rowsum;
  }
}

// psi_0^c from the prolate differential operator (it commutes with F_c and
// has well-separated eigenvalues chi_0 < chi_2 < ..., unlike the eigenvalues
// of F_c itself, which cluster near sqrt(2 pi / c) for large c):
//   L psi = -(1 - x^2) psi'' + 2 x psi' + c^2 x^2 psi = chi psi,
// collocated at Chebyshev-Gauss-Lobatto points (the endpoint rows enforce
// regularity), smallest eigenvalue by inverse iteration from an even start.
Prolate::Prolate(double c, int N) : c_(c) {
  if (!(c > 0.0)) throw std::invalid_argument("prolate bandwidth must be positive");
  if (N % 2) ++N;
  const int n = N + 1;
  std::vector<double> D;
  cheb_matrix(N, x_, D);
  std::vector<double> D2(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      const double dik = D[size_t(i) * n + k];
      if (dik == 0.0) continue;
      for (int j = 0; j < n; ++j) D2[size_t(i) * n + j] += dik * D[size_t(k) * n + j];
    }
  std::vector<double> A(size_t(n) * n), Ash;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double v = -(1.0 - x_[i] * x_[i]) * D2[size_t(i) * n + j] + 2.0 * x_[i] * D[size_t(i) * n + j];
      if (i == j) v += c * c * x_[i] * x_[i];
      A[size_t(i) * n + j] = v;
    }
  // shift near chi_0 (about c^2/3 for small c and c - 3/4 for large c; the
  // next even eigenvalue is ~4c higher, the odd one ~2c), iterate in the
  // even subspace (the nodes are symmetric: x_{N-j} = -x_j)
  const double sigma = std::min(c * c / 3.0, c - 0.75);
  Ash = A;
  for (int i = 0; i < n; ++i) Ash[size_t(i) * n + i] -= sigma;
  std::vector<int> piv;
  if (!lu_factor(n, Ash, piv)) throw std::runtime_error("prolate collocation matrix is singular");
  std::vector<double> v(n, 1.0);
  for (int it = 0; it < 60; ++it) {
    lu_solve(n, Ash, piv, v);
    for (int i = 0; i < n / 2; ++i) {
      const double e = 0.5 * (v[i] + v[N - i]);
      v[i] = v[N - i] = e;
    }
    double nrm = 0.0;
    for (double e : v) nrm = std::max(nrm, std::fabs(e));
    for (double &e : v) e /= nrm;
  }
  // Rayleigh-like estimate of chi at x = 0 row is ill-posed; use the
  // residual-minimising quotient over all nodes
  std::vector<double> Av(n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Av[i] += A[size_t(i) * n + j] * v[j];
  double num = 0.0, den = 0.0;
  for (int i = 0; i < n; ++i) {
    num += Av[i] * v[i];
    den += v[i] * v[i];
  }
  chi_ = num / den;
  const double v0 = v[N / 2];
  psi_.resize(n);
  for (int i = 0; i < n; ++i) psi_[i] = v[i] / v0;
  // derivatives at the nodes
  dpsi_.assign(n, 0.0);
  d2psi_.assign(n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      dpsi_[i] += D[size_t(i) * n + j] * psi_[j];
      d2psi_[i] += D2[size_t(i) * n + j] * psi_[j];
    }
  // barycentric weights
  bw_.resize(n);
  for (int j = 0; j < n; ++j) bw_[j] = ((j % 2) ? -1.0 : 1.0) * ((j == 0 || j == N) ? 0.5 : 1.0);
  // lambda_0 = int_{-1}^{1} psi (eq. psidefinit at x = 0), Gauss quadrature
  gauss_legendre(64, 0.0, 1.0, qx_, qw_);
  std::vector<double> gx, gw;
  gauss_legendre(96, -1.0, 1.0, gx, gw);
  lam_ = 0.0;
  for (size_t i = 0; i < gx.size(); ++i) lam_ += gw[i] * (*this)(gx[i]);
  // quadrature for the window transform at frequencies up to ~200
  std::vector<double> fw;
  gauss_legendre(320, 0.0, 1.0, fx_, fw);
  fwpsi_.resize(fx_.size());
  for (size_t i = 0; i < fx_.size(); ++i) fwpsi_[i] = 2.0 * fw[i] * (*this)(fx_[i]);
}

double Prolate::bary(const std::vector<double> &f, double x) const {
  double num = 0.0, den = 0.0;
  for (size_t j = 0; j < x_.size(); ++j) {
    const double dx = x - x_[j];
    if (dx == 0.0) return f[j];
    const double t = bw_[j] / dx;
    num += t * f[j];
    den += t;
  }
  return num / den;
}

double Prolate::operator()(double x) const { return bary(psi_, x); }
double Prolate::d1(double x) const { return bary(dpsi_, x); }
double Prolate::d2(double x) const { return bary(d2psi_, x); }

// psi^(n)(0) for even n: psi''(0) = -chi from the ODE at x = 0, and the
// n-times differentiated ODE at 0:
//   psi^(n+2)(0) = (n (n + 1) - chi) psi^(n)(0) + c^2 n (n - 1) psi^(n-2)(0).
double Prolate::deriv0(int n) const {
  if (n == 0) return 1.0;
  if (n % 2) return 0.0;
  double prev = 1.0, cur = -chi_;  // psi(0), psi''(0)
  for (int m = 2; m < n; m += 2) {
    const double next = (m * (m + 1) - chi_) * cur + c_ * c_ * m * (m - 1) * prev;
    prev = cur;
    cur = next;
  }
  return cur;
}

double Prolate::I0(double k) const {
  double s = 0.0;
  for (size_t i = 0; i < qx_.size(); ++i) s += k * qw_[i] * (*this)(k * qx_[i]);
  return s;
}
double Prolate::J1(double k) const {
  double s = 0.0, L = 1.0 - k;
  for (size_t i = 0; i < qx_.size(); ++i) {
    double u = k + L * qx_[i];
    s += L * qw_[i] * u * (*this)(u);
  }
  return s;
}
double Prolate::J3(double k) const {
  double s = 0.0, L = 1.0 - k;
  for (size_t i = 0; i < qx_.size(); ++i) {
    double u = k + L * qx_[i];
    s += L * qw_[i] * u * u * u * (*this)(u);
  }
  return s;
}
double Prolate::T3(double k) const {
  double s = 0.0, L = 1.0 - k;
  for (size_t i = 0; i < qx_.size(); ++i) {
    double u = k + L * qx_[i];
    s += L * qw_[i] * ((*this)(u) - 1.0) / u;
  }
  return s;
}
double Prolate::window_ft(double s) const {
  double acc = 0.0;
  for (size_t i = 0; i < fx_.size(); ++i) acc += fwpsi_[i] * std::cos(s * fx_[i]);
  return acc;
}

std::shared_ptr<const Prolate> prolate_cached(double c) {
  static std::mutex mu;
  static std::map<double, std::shared_ptr<const Prolate>> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(c);
  if (it != cache.end()) return it->second;
  auto p = std::make_shared<const Prolate>(c);
  cache[c] = p;
  return p;
}

std::shared_ptr<const std::vector<float>> deconvolution_cached(double c_s, int P, int M) {
  static std::mutex mu;
  static std::map<std::tuple<double, int, int>, std::shared_ptr<const std::vector<float>>> cache;
  const auto key = std::make_tuple(c_s, P, M);
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  auto ws = prolate_cached(c_s);
  auto tab = std::make_shared<std::vector<float>>(M / 2 + 1);
  for (int f = 0; f <= M / 2; ++f) {
    const double what_over_h = 0.5 * P * ws->window_ft(kPi * P * double(f) / M);
    (*tab)[f] = float(1.0 / (what_over_h * what_over_h));
  }
  std::lock_guard<std::mutex> lock(mu);
  cache.emplace(key, tab);
  return tab;
}

// ---------------------------------------------------------------------------
double PiecewisePoly::eval(double x) const {
  double y = x * nseg;
  int s = std::min(nseg - 1, std::max(0, int(std::floor(y))));
  double tau = 2.0 * (y - s) - 1.0;
  const double *cf = &coef[size_t(s) * (deg + 1)];
  double r = cf[deg];
  for (int d = deg - 1; d >= 0; --d) r = r * tau + cf[d];
  return r;
}

template <class F>
PiecewisePoly fit_piecewise(F f, int nseg, int deg, double eps) {
  PiecewisePoly pp;
  pp.nseg = nseg;
  pp.deg = deg;
  pp.coef.assign(size_t(nseg) * (deg + 1), 0.0);
  const int n = deg + 1;
  // monomial expansions of T_0..T_deg
  std::vector<std::vector<double>> T(n, std::vector<double>(n, 0.0));
  T[0][0] = 1.0;
  if (n > 1) T[1][1] = 1.0;
  for (int m = 2; m < n; ++m)
    for (int d = 0; d < n; ++d) {
      double v = -T[m - 2][d];
      if (d > 0) v += 2.0 * T[m - 1][d - 1];
      T[m][d] = v;
    }
  for (int s = 0; s < nseg; ++s) {
    double a = double(s) / nseg, b = double(s + 1) / nseg;
    std::vector<double> fv(n), ch(n, 0.0);
    for (int j = 0; j < n; ++j) {
      double y = std::cos(kPi * (j + 0.5) / n);
      fv[j] = f(0.5 * (b - a) * (y + 1.0) + a);
    }
    double amax = 0.0;
    for (int m = 0; m < n; ++m) {
      double acc = 0.0;
      for (int j = 0; j < n; ++j) acc += fv[j] * std::cos(kPi * m * (j + 0.5) / n);
      ch[m] = (m == 0 ? 1.0 : 2.0) * acc / n;
      amax = std::max(amax, std::fabs(ch[m]));
    }
    for (int m = 0; m < n; ++m)
      if (std::fabs(ch[m]) <= 0.01 * eps * amax) ch[m] = 0.0;
    double *cf = &pp.coef[size_t(s) * n];
    for (int m = 0; m < n; ++m)
      for (int d = 0; d < n; ++d) cf[d] += ch[m] * T[m][d];
  }
  double err = 0.0;
  for (int i = 0; i <= 4000; ++i) {
    double x = i / 4000.0;
    err = std::max(err, std::fabs(pp.eval(x) - f(x)));
  }
  pp.max_abs_err = err;
  return pp;
}

PiecewisePoly make_window_poly(double c_s, int nseg, int deg, double eps) {
  // plans of a serving mix share a handful of bandwidths: cache the fits
  static std::mutex mu;
  static std::map<std::tuple<long, int, int, long>, PiecewisePoly> cache;
  const auto key = std::make_tuple(std::lround(c_s * 1e6), nseg, deg, std::lround(std::log10(eps) * 100));
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  auto ws = prolate_cached(c_s);
  PiecewisePoly fit = fit_piecewise([&](double x) { return (*ws)(x); }, nseg, deg, eps);
  std::lock_guard<std::mutex> lock(mu);
  cache.emplace(key, fit);
  return fit;
}

// ---------------------------------------------------------------------------
// Fourier kernels Phi_p (Eq. PhiH), band-limited reading: the Fourier-side
// integrals of lambda0 psi(x/c) run over [0, c], so Chat0 = lambda0 c C0
// and Phi_p vanishes for k > c / r_c.  With K = c / r_c, kappa = k / K:
//   Phi1 = 4 pi psi(kappa) / k^2
//   Phi2 = 2 pi^2 T2(kappa) / k,                T2 = 1 - I0/C0
//   Phi3 = 4 pi (T3(kappa) - ln kappa)
//   Phi4 = -pi^2 k T2 + pi^2 K J1 / C0
//   Phi5 = -(2 pi/3) (k^2 (T3 - ln kappa) - K^2 J1)
//   Phi6 = (pi^2/12) (k^3 T2 - (3 k^2 K / (2 C0)) J1 + K^3 J3 / (2 C0))
double phi_hat(const Prolate &ps, int p, double k, double c, double r_c) {
  const double K = c / r_c, kap = k / K;
  if (kap > 1.0) return 0.0;
  const double C0 = ps.C0();
  const double T2 = 1.0 - ps.I0(kap) / C0;
  switch (p) {
    case 1: return 4.0 * kPi * ps(kap) / (k * k);
    case 2: return 2.0 * kPi * kPi * T2 / k;
    case 3: return 4.0 * kPi * (ps.T3(kap) - std::log(kap));
    case 4: return -kPi * kPi * k * T2 + kPi * kPi * K * ps.J1(kap) / C0;
    case 5: return -(2.0 * kPi / 3.0) * (k * k * (ps.T3(kap) - std::log(kap)) - K * K * ps.J1(kap));
    case 6:
      return (kPi * kPi / 12.0) * (k * k * k * T2 - 1.5 * k * k * K * ps.J1(kap) / C0 +
                                   K * K * K * ps.J3(kap) / (2.0 * C0));
  }
  throw std::invalid_argument("p must be 1..6");
}

// d Phi_p / dk, differentiating under the integral sign (dI0/dkappa = psi,
// dJ1/dkappa = -kappa psi, dJ3/dkappa = -kappa^3 psi, dT3/dkappa =
// -(psi - 1)/kappa); the psi terms cancel for p = 4, 5, 6.
double phi_hat_deriv(const Prolate &ps, int p, double k, double c, double r_c) {
  const double K = c / r_c, kap = k / K;
  if (kap > 1.0) return 0.0;
  const double C0 = ps.C0();
  const double T2 = 1.0 - ps.I0(kap) / C0;
  switch (p) {
    case 1: return 4.0 * kPi * (kap * ps.d1(kap) - 2.0 * ps(kap)) / (k * k * k);
    case 2: return -2.0 * kPi * kPi * T2 / (k * k) - 2.0 * kPi * kPi * kap * ps(kap) / (C0 * k * k);
    case 3: return -4.0 * kPi * ps(kap) / k;
    case 4: return -kPi * kPi * T2;
    case 5: return -(4.0 * kPi / 3.0) * k * (ps.T3(kap) - std::log(kap));
    case 6: return (kPi * kPi / 4.0) * (k * k * T2 - k * K * ps.J1(kap) / C0);
  }
  throw std::invalid_argument("p must be 1..6");
}

static ChannelKernel build_channel_kernel(int p, double c, double r_c, double eps);

double mollifier_complement(const Prolate &ps, int p, double rho) {
  if (!(rho < 1.0)) return 0.0;
  const double x = rho < 0.0 ? 0.0 : rho;
  const double psi = ps(x), d1 = ps.d1(x), C0 = ps.C0();
  switch (p) {
    case 1: return 1.0 - ps.I0(x) / C0;                                  // G1 = I0 / C0
    case 2: return psi;                                                   // G2 = 1 - psi
    case 3: return 1.0 - (ps.I0(x) - x * psi) / C0;
    case 4: return psi - 0.5 * x * d1;
    case 5: return 1.0 - (ps.I0(x) - x * psi + x * x / 3.0 * d1) / C0;
    case 6: return psi - 5.0 * x / 8.0 * d1 + x * x / 8.0 * ps.d2(x);   // G6
  }
  return 0.0;
}

PiecewisePoly make_complement_poly(int p, double c, int nseg, int deg, double eps) {
  static std::mutex mu;
  static std::map<std::tuple<int, long, int, int, long>, PiecewisePoly> cache;
  const auto key = std::make_tuple(p, std::lround(c * 1e9), nseg, deg, std::lround(std::log10(eps) * 100));
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  auto ps = prolate_cached(c);
  PiecewisePoly fit = fit_piecewise([&](double x) { return mollifier_complement(*ps, p, x); }, nseg, deg, eps);
  std::lock_guard<std::mutex> lock(mu);
  cache.emplace(key, fit);
  return fit;
}

ChannelKernel make_channel_kernel(int p, double c, double r_c, double eps) {
  // box-independent: one fit per (p, c, r_c) serves every structure
  static std::mutex mu;
  static std::map<std::tuple<int, long, long, long>, ChannelKernel> cache;
  const auto key = std::make_tuple(p, std::lround(c * 1e9), std::lround(r_c * 1e9), std::lround(std::log10(eps) * 100));
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  ChannelKernel ck = build_channel_kernel(p, c, r_c, eps);
  std::lock_guard<std::mutex> lock(mu);
  cache.emplace(key, ck);
  return ck;
}

static ChannelKernel build_channel_kernel(int p, double c, double r_c, double eps) {
  auto psp = prolate_cached(c);
  const Prolate &ps = *psp;
  const double K = c / r_c, C0 = ps.C0();
  const int nseg = 16, deg = 11;
  ChannelKernel ck;
  ck.p = p;
  auto T2 = [&](double x) { return 1.0 - ps.I0(x) / C0; };
  switch (p) {
    case 1:
      ck.A = 4.0 * kPi / (K * K); ck.eA = -2;
      ck.f = fit_piecewise([&](double x) { return ps(x); }, nseg, deg, eps);
      ck.Cc = 4.0 * kPi / (K * K * K * K); ck.eC = -4;
      ck.g = fit_piecewise([&](double x) { return x * ps.d1(x) - 2.0 * ps(x); }, nseg, deg, eps);
      break;
    case 2:
      ck.A = 2.0 * kPi * kPi / K; ck.eA = -1;
      ck.f = fit_piecewise(T2, nseg, deg, eps);
      ck.Cc = 2.0 * kPi * kPi / (K * K * K); ck.eC = -3;
      ck.g = fit_piecewise([&](double x) { return -T2(x) - x * ps(x) / C0; }, nseg, deg, eps);
      break;
    case 3:
      ck.A = 4.0 * kPi; ck.eA = 0;
      ck.f = fit_piecewise([&](double x) { return ps.T3(x); }, nseg, deg, eps);
      ck.B = -4.0 * kPi; ck.eB = 0;
      ck.Cc = -4.0 * kPi / (K * K); ck.eC = -2;
      ck.g = fit_piecewise([&](double x) { return ps(x); }, nseg, deg, eps);
      break;
    case 4:
      ck.A = 1.0; ck.eA = 0;
      ck.f = fit_piecewise([&](double x) { return -kPi * kPi * K * x * T2(x) + kPi * kPi * K * ps.J1(x) / C0; },
                           nseg, deg, eps);
      ck.Cc = -kPi * kPi / K; ck.eC = -1;
      ck.g = fit_piecewise(T2, nseg, deg, eps);
      break;
    case 5:
      ck.A = 1.0; ck.eA = 0;
      ck.f = fit_piecewise([&](double x) { return -(2.0 * kPi / 3.0) * K * K * (x * x * ps.T3(x) - ps.J1(x)); },
                           nseg, deg, eps);
      ck.B = (2.0 * kPi / 3.0) * K * K; ck.eB = 2;
      ck.Cc = -4.0 * kPi / 3.0; ck.eC = 0;
      ck.g = fit_piecewise([&](double x) { return ps.T3(x); }, nseg, deg, eps);
      ck.D = 4.0 * kPi / 3.0; ck.eD = 0;
      break;
    case 6:
      ck.A = kPi * kPi * K * K * K / 12.0; ck.eA = 0;
      ck.f = fit_piecewise([&](double x) {
        return x * x * x * T2(x) - 1.5 * x * x * ps.J1(x) / C0 + ps.J3(x) / (2.0 * C0);
      }, nseg, deg, eps);
      ck.Cc = kPi * kPi * K / 4.0; ck.eC = 0;
      ck.g = fit_piecewise([&](double x) { return x * T2(x) - ps.J1(x) / C0; }, nseg, deg, eps);
      break;
    default:
      throw std::invalid_argument("p must be 1..6");
  }
  // Self term (Methods, "Implementation details"): E_self = s_p sum q^2.
  const double d2 = ps.deriv0(2), d4 = ps.deriv0(4), d6 = ps.deriv0(6);
  switch (p) {
    case 1: ck.self_coef = 1.0 / (2.0 * C0 * r_c); break;
    case 2: ck.self_coef = -d2 / (4.0 * r_c * r_c); break;
    case 3: ck.self_coef = -d2 / (6.0 * C0 * std::pow(r_c, 3)); break;
    case 4: ck.self_coef = d4 / (48.0 * std::pow(r_c, 4)); break;
    case 5: ck.self_coef = d4 / (90.0 * C0 * std::pow(r_c, 5)); break;
    case 6: ck.self_coef = -d6 / (1440.0 * std::pow(r_c, 6)); break;
  }
  // Zero-frequency term E_0 = (zero_coef_V / V) Q_net^2 (Eqs. Correction,
  // Correction3r; p > 3 is Phi_p(0)/2).  For p = 1 the k -> 0 limit of
  // (Phi1 - 4 pi / k^2) / 2 = -pi chi0 / K^2 is used (tin-foil boundary,
  // E_IB = 0), which keeps the total independent of (c, r_c).
  switch (p) {
    case 1: ck.zero_coef_V = -kPi * ps.chi() / (K * K); break;
    case 2: ck.zero_coef_V = -2.0 * kPi * r_c * C0; break;
    case 3: ck.zero_coef_V = 2.0 * kPi * (std::log(c / r_c) + ps.T3(0.0)); break;
    case 4: ck.zero_coef_V = 0.5 * kPi * kPi * K * ps.J1(0.0) / C0; break;
    case 5: ck.zero_coef_V = 0.5 * (2.0 * kPi / 3.0) * K * K * ps.J1(0.0); break;
    case 6: ck.zero_coef_V = 0.5 * (kPi * kPi / 12.0) * K * K * K * ps.J3(0.0) / (2.0 * C0); break;
  }
  return ck;
}

// ---------------------------------------------------------------------------
// Spreading-error estimate.  In grid units (h = 1) the truncated window has
// the transform What(s) = omega * int_{-1}^{1} psi_s(t) cos(s omega t) dt,
// omega = P/2.  Sampling on the grid aliases every mode k with k + 2 pi j,
// so the relative error of the deconvolved mode is approximately
//   r(k) = sum_{j != 0} |What(k + 2 pi j)| / What(k)   per axis.
// The estimate is the RMS of r(k_x) + r(k_y) + r(k_z) over the k-ball
// |k| <= eta pi, weighted by the force spectrum of the p = 1 kernel for
// uncorrelated charges (Phi_1^2 k^2 per mode, i.e. psi_c(kappa)^2 per
// radial shell).  Its minimiser over c_s tracks the measured optimum of the
// force error closely; its magnitude is about 1/25 of that error.
double estimate_spread_error(int P, double eta, double c_s, double c_moll) {
  auto ws = prolate_cached(c_s);
  auto pc = prolate_cached(c_moll);
  const double omega = 0.5 * P, kmax = eta * kPi;
  const int nk = 97;
  std::vector<double> rk(nk);
  for (int i = 0; i < nk; ++i) {
    double k = kmax * i / (nk - 1);
    double w0 = omega * ws->window_ft(k * omega);
    double a = 0.0;
    for (int j = 1; j <= 4; ++j)
      a += std::fabs(omega * ws->window_ft((k + 2 * kPi * j) * omega)) +
           std::fabs(omega * ws->window_ft((k - 2 * kPi * j) * omega));
    rk[i] = a / std::fabs(w0);
  }
  auto interp = [&](double k) {
    double y = std::fabs(k) / kmax * (nk - 1);
    int i = std::min(nk - 2, int(y));
    double f = y - i;
    return rk[i] * (1 - f) + rk[i + 1] * f;
  };
  std::vector<double> rx, rw, cx, cw;
  gauss_legendre(20, 0.0, 1.0, rx, rw);
  gauss_legendre(12, -1.0, 1.0, cx, cw);
  double num = 0.0, den = 0.0;
  for (size_t i = 0; i < rx.size(); ++i) {
    double wr = rw[i] * std::pow((*pc)(rx[i]), 2);
    for (size_t j = 0; j < cx.size(); ++j) {
      double ct = cx[j], st = std::sqrt(std::max(0.0, 1 - ct * ct));
      for (int m = 0; m < 24; ++m) {
        double ph = 2 * kPi * (m + 0.5) / 24;
        double kx = kmax * rx[i] * st * std::cos(ph), ky = kmax * rx[i] * st * std::sin(ph),
               kz = kmax * rx[i] * ct;
        double e = interp(kx) + interp(ky) + interp(kz);
        double wgt = wr * cw[j];
        num += wgt * e * e;
        den += wgt;
      }
    }
  }
  return std::sqrt(num / den);
}

// minimiser of the estimate at one eta (golden-section search on [2.2 P, 3.2 P])
static double search_c_spread(int P, double eta, double c_moll) {
  double a = 2.2 * P, b = 3.2 * P;
  const double g = 0.5 * (std::sqrt(5.0) - 1.0);
  double x1 = b - g * (b - a), x2 = a + g * (b - a);
  double f1 = estimate_spread_error(P, eta, x1, c_moll), f2 = estimate_spread_error(P, eta, x2, c_moll);
  for (int it = 0; it < 14; ++it) {  // bracket 0.01 P: the estimate is flat near its minimum
    if (f1 < f2) {
      b = x2; x2 = x1; f2 = f1; x1 = b - g * (b - a);
      f1 = estimate_spread_error(P, eta, x1, c_moll);
    } else {
      a = x1; x1 = x2; f1 = f2; x2 = a + g * (b - a);
      f2 = estimate_spread_error(P, eta, x2, c_moll);
    }
  }
  return 0.5 * (a + b);
}

double spread_error_bound(int P, double eta, double c_moll) {
  // The estimate grows with eta, so it is taken at the grid point of step
  // 1/40 at or above eta, with that point's window bandwidth: an upper
  // bound for the plan's own eta.  Grid points are computed on first use
  // and cached, so choosing the support costs no quadrature once plans of
  // a similar coarseness have been made (each evaluation takes a few ms).
  static std::mutex mu;
  static std::map<std::tuple<int, long, long>, double> cache;
  const double step = 1.0 / 40.0;
  const long i = std::max(1L, long(std::ceil(eta / step - 1e-9)));
  const auto key = std::make_tuple(P, i, std::lround(c_moll * 1e6));
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  const double eu = std::min(0.99, i * step);
  const double v = estimate_spread_error(P, eu, choose_c_spread(P, eu, c_moll), c_moll);
  std::lock_guard<std::mutex> lock(mu);
  cache[key] = v;
  return v;
}

double choose_c_spread(int P, double eta, double c_moll) {
  // The minimiser is a smooth, slowly varying function of eta (the error
  // is flat near it), so it is searched on a grid of eta with step 1/40 and
  // interpolated linearly; grid points are computed on first use and cached,
  // so plans for boxes of any shape after the first few cost no search.
  static std::mutex mu;
  static std::map<std::tuple<int, long, long>, double> cache;
  const double step = 1.0 / 40.0;
  const double u = std::max(eta, step) / step;
  const long i0 = long(std::floor(u));
  double v[2];
  for (int j = 0; j < 2; ++j) {
    const long i = i0 + j;
    const auto key = std::make_tuple(P, i, std::lround(c_moll * 1e6));
    bool hit = false;
    {
      std::lock_guard<std::mutex> lock(mu);
      auto it = cache.find(key);
      if (it != cache.end()) {
        v[j] = it->second;
        hit = true;
      }
    }
    if (!hit) {
      v[j] = search_c_spread(P, std::min(0.99, i * step), c_moll);
      std::lock_guard<std::mutex> lock(mu);
      cache[key] = v[j];
    }
  }
  // rounded to 0.05 (well inside the flat minimum): boxes of nearby eta then
  // share one window bandwidth, so the window polynomial built for it is
  // reused from its cache instead of refitted per box
  const double f = u - double(i0);
  return std::round(((1.0 - f) * v[0] + f * v[1]) * 20.0) / 20.0;
}

bool is_smooth235(int m) {
  if (m < 1) return false;
  for (int p : {2, 3, 5})
    while (m % p == 0) m /= p;
  return m == 1;
}

int smooth_size(double x, bool even) {
  int m = std::max(1, int(std::ceil(x - 1e-9)));
  while (!is_smooth235(m) || (even && (m % 2))) ++m;
  return m;
}

}  // namespace pswf

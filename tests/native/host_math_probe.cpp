// Prints the library's host-side FP64 math for comparison with the oracle
// (tests/test_host_math.py).  Built with g++ from the library's sources.
#include <cstdio>
#include <cmath>
#include <cstdlib>

#include "host_math.hpp"

int main(int argc, char **argv) {
  const double c = argc > 1 ? std::atof(argv[1]) : 12.024;
  const double rc = 5.0;
  pswf::Prolate ps(c);
  std::printf("lam %.17g\nchi %.17g\nC0 %.17g\n", ps.lambda(), ps.chi(), ps.C0());
  for (double x : {0.0, 0.25, 0.5, 0.75, 1.0}) std::printf("psi %.17g %.17g %.17g\n", x, ps(x), ps.d1(x));
  std::printf("d4 %.17g\nd6 %.17g\n", ps.deriv0(4), ps.deriv0(6));
  for (double kap : {0.0, 0.3, 0.7}) std::printf("int %.17g %.17g %.17g %.17g %.17g\n", kap, ps.I0(kap), ps.J1(kap), ps.J3(kap), ps.T3(kap));
  const double kc = c / rc;
  for (int p = 1; p <= 6; ++p) {
    auto ck = pswf::make_channel_kernel(p, c, rc, 1e-9);
    std::printf("coef %d %.17g %.17g %.3g %.3g\n", p, ck.self_coef, ck.zero_coef_V, ck.f.max_abs_err, ck.g.max_abs_err);
    for (double f : {0.05, 0.3, 0.6, 0.95}) {
      const double k = f * kc, kap = f;
      // the device representation: A kap^eA f + B kap^eB ln kap, and Phi'/k
      auto pw = [](double x, int e) { double r = 1; for (int i = 0; i < (e < 0 ? -e : e); ++i) r *= x; return e < 0 ? 1 / r : r; };
      const double phi_dev = ck.A * pw(kap, ck.eA) * ck.f.eval(kap) + (ck.B != 0 ? ck.B * pw(kap, ck.eB) * std::log(kap) : 0.0);
      const double dph_dev = ck.Cc * pw(kap, ck.eC) * ck.g.eval(kap) + (ck.D != 0 ? ck.D * pw(kap, ck.eD) * std::log(kap) : 0.0);
      std::printf("phi %d %.17g %.17g %.17g %.17g %.17g\n", p, k, pswf::phi_hat(ps, p, k, c, rc),
                  pswf::phi_hat_deriv(ps, p, k, c, rc), phi_dev, dph_dev);
    }
  }
  auto wp = pswf::make_window_poly(20.0, 8, 11, 1e-9);
  pswf::Prolate w20(20.0);
  for (double t : {0.0, 0.33, 0.8, 0.999}) std::printf("win %.17g %.17g %.17g\n", t, wp.eval(t), w20(t));
  for (double s : {0.0, 5.0, 19.0}) std::printf("wft %.17g %.17g %.17g\n", s, w20.window_ft(s), w20.lambda() * w20(s / 20.0));
  std::printf("cs6 %.6f\ncs8 %.6f\n", pswf::choose_c_spread(6, 0.54, 12.024), pswf::choose_c_spread(8, 0.54, 12.024));
  // the support choice's cached bound against the estimate itself
  for (int P : {5, 7, 8})
    for (double eta : {0.31, 0.4603, 0.54, 0.6442})
      std::printf("ebound %d %.6f %.17g %.17g\n", P, eta,
                  pswf::estimate_spread_error(P, eta, pswf::choose_c_spread(P, eta, 12.024), 12.024),
                  pswf::spread_error_bound(P, eta, 12.024));
  return 0;
}

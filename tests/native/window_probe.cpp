// Reads lines "O x L M P" (orthorhombic: u = x M / L) or
// "G x y z T0 T1 T2 M P" (general cell: u = T . r, T one row of
// diag(M) H^-T) and prints the window start and offset the binning kernel
// computes for them (grid_coord, window_start_dw: FP32 double-word
// arithmetic), for comparison with exact rational arithmetic
// (tests/test_window_start_cpu.py).
#include <cstdio>

#include "device_types.hpp"

int main() {
  char mode[4];
  while (std::scanf("%3s", mode) == 1) {
    int n0 = -1, M, P;
    float delta = -1.0f;
    if (mode[0] == 'O') {
      double x, L;
      if (std::scanf("%lf %lf %d %d", &x, &L, &M, &P) != 4) return 1;
      const double s = double(M) / L;
      const float sh = float(s), sl = float(s - double(sh));
      pswf::window_start(float(x), sh, sl, M, P, &n0, &delta);
    } else {
      double r[3], T[3];
      if (std::scanf("%lf %lf %lf %lf %lf %lf %d %d", &r[0], &r[1], &r[2], &T[0], &T[1], &T[2], &M, &P) != 8)
        return 1;
      float rf[3], th[3], tl[3];
      for (int b = 0; b < 3; ++b) {
        rf[b] = float(r[b]);
        th[b] = float(T[b]);
        tl[b] = float(T[b] - double(th[b]));
      }
      float hi, lo;
      pswf::grid_coord(rf, th, tl, &hi, &lo);
      pswf::window_start_dw(hi, lo, M, P, &n0, &delta);
    }
    std::printf("%d %.9g\n", n0, double(delta));
  }
  return 0;
}

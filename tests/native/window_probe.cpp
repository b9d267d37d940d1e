// Reads lines "x L M P" and prints the window start and offset the binning
// kernel computes for them (window_start, FP32 double-word arithmetic), for
// comparison with exact rational arithmetic (tests/test_window_start_cpu.py).
#include <cstdio>

#include "device_types.hpp"

int main() {
  double x, L;
  int M, P;
  while (std::scanf("%lf %lf %d %d", &x, &L, &M, &P) == 4) {
    const double s = double(M) / L;
    const float sh = float(s), sl = float(s - double(sh));
    int n0 = -1;
    float delta = -1.0f;
    pswf::window_start(float(x), sh, sl, M, P, &n0, &delta);
    std::printf("%d %.9g\n", n0, double(delta));
  }
  return 0;
}

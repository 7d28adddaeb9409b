// Host-side check of the library's symmetric 3x3 inverse (mpl_math.h):
// reads blocks (xx yy zz xy yz xz) from stdin, one per line, and prints the
// success flag and the six inverse entries.
#include <cstdio>

#include "../../paper_2602_07853_amd/csrc/mpl_math.h"

int main() {
  double h[6];
  while (std::scanf("%lf %lf %lf %lf %lf %lf", &h[0], &h[1], &h[2], &h[3], &h[4], &h[5]) == 6) {
    double inv[6];
    const bool ok = mpl::sym3_inverse(h, inv);
    std::printf("%d %.17g %.17g %.17g %.17g %.17g %.17g\n", ok ? 1 : 0, inv[0], inv[1], inv[2], inv[3],
                inv[4], inv[5]);
  }
  return 0;
}

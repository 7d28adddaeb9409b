// Host-side check of the two-level reduction's partition (mpl_math.h): reads
// array lengths nm from stdin, one per line, and prints for each the number
// of workgroups G (at most 64) followed by the G ranges lo hi.
#include <cstdio>

#include "../../paper_2602_07853_amd/csrc/mpl_math.h"

int main() {
  int nm;
  while (std::scanf("%d", &nm) == 1) {
    const int G = mpl::red2_groups(nm, 64);
    std::printf("%d", G);
    for (int g = 0; g < G; ++g) {
      int lo, hi;
      mpl::red2_range(g, G, nm, lo, hi);
      std::printf(" %d %d", lo, hi);
    }
    std::printf("\n");
  }
  return 0;
}

// Host-side check of the library's SplitMix64 counter generator (mpl_math.h):
// reads counters from stdin, one per line, and prints each output in hex.
#include <cstdio>

#include "../../paper_2602_07853_amd/csrc/mpl_math.h"

int main() {
  unsigned long long q;
  while (std::scanf("%llu", &q) == 1) std::printf("%016llx\n", (unsigned long long)mpl::splitmix64(q));
  return 0;
}

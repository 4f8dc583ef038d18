// Host-side check of the recursion kernel's workgroup -> (tile, part) mapping,
// built from the library's own functions (xcd_tile, split_tile, split_count in
// q2x_internal.hpp, the code the kernel and the host call): for every launch
// of 1..max_tiles tiles in both precisions, every (tile, part) is covered
// exactly once, a tile has two parts iff it is one of the split_count(n) split
// tiles, and the virtual ids are a permutation of the workgroups.  Prints the
// number of launches checked; exits non-zero on the first mismatch.
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "../paper_2107_10942_amd/csrc/q2x_internal.hpp"

int main(int argc, char** argv) {
  const int max_tiles = argc > 1 ? atoi(argv[1]) : 2199;
  int checked = 0;
  for (int prec = 0; prec < 2; ++prec) {
    for (int64_t n = 1; n <= max_tiles; ++n) {
      const int64_t s = q2x::split_count(n, prec);
      if (s < 0 || s > n || (s > 0 && n > 2048)) {
        printf("bad split count n=%lld s=%lld\n", (long long)n, (long long)s);
        return 1;
      }
      const int64_t nblk = n + s;
      std::vector<int> seen_v(nblk, 0), seen_tp(2 * n, 0), parts_of(n, 0);
      for (int64_t b = 0; b < nblk; ++b) {
        const int64_t v = q2x::xcd_tile(b, nblk);
        if (v < 0 || v >= nblk || seen_v[v]++) {
          printf("virtual id %lld repeated or out of range (n=%lld b=%lld)\n", (long long)v, (long long)n, (long long)b);
          return 1;
        }
        uint32_t t = (uint32_t)v;
        int part = 0, parts = 1;
        if (s > 0) q2x::split_tile((uint32_t)v, (uint32_t)n, (uint32_t)s, t, part, parts);
        if (t >= (uint64_t)n || part < 0 || part >= parts || seen_tp[2 * t + part]++) {
          printf("tile/part out of range or repeated (n=%lld v=%lld t=%u part=%d)\n", (long long)n, (long long)v, t,
                 part);
          return 1;
        }
        if (parts_of[t] && parts_of[t] != parts) {
          printf("inconsistent part count (n=%lld t=%u)\n", (long long)n, t);
          return 1;
        }
        parts_of[t] = parts;
      }
      int64_t split = 0;
      for (int64_t t = 0; t < n; ++t) {
        const bool want = (t + 1) * s / n > t * s / n;
        if ((parts_of[t] == 2) != want || seen_tp[2 * t] != 1 || seen_tp[2 * t + 1] != (want ? 1 : 0)) {
          printf("tile %lld covered wrongly (n=%lld s=%lld)\n", (long long)t, (long long)n, (long long)s);
          return 1;
        }
        split += want;
      }
      if (split != s) {
        printf("split %lld tiles, expected %lld (n=%lld)\n", (long long)split, (long long)s, (long long)n);
        return 1;
      }
      ++checked;
    }
  }
  printf("checked %d launches\n", checked);
  return 0;
}

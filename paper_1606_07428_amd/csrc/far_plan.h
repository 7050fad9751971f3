// Source chunks of the all-pairs sums (host side, plain C++): split s < s1 covers c1
// sources from s c1, split s >= s1 covers c2 sources from s1 c1 + (s - s1) c2, each
// clipped to N; a split that starts at or past N is empty and its slot holds zeros.
// Workgroups are dispatched split by split, so the long chunks (85% of the sources, the
// first half of the splits) run first and the grid drains on the short ones.
#pragma once
#include <algorithm>

namespace rbm {

struct FarChunks {
  int s1, c1, c2;
};

inline FarChunks far_chunks(int N, int nsplit) {
  if (nsplit < 2) return {0, N, N};
  const int s1 = nsplit / 2, s2 = nsplit - s1;
  const long c1 = std::min((17L * N + 20L * s1 - 1) / (20L * s1), (long)N / s1);
  const long rest = N - s1 * c1;
  const long c2 = std::max(1L, (rest + s2 - 1) / s2);
  return {s1, (int)c1, (int)c2};
}

}  // namespace rbm

// Source chunks of the all-pairs sums (host side, plain C++): split s < s1 covers c1
// sources from s c1, split s >= s1 covers c2 sources from s1 c1 + (s - s1) c2, each
// clipped to N; a split that starts at or past N is empty and its slot holds zeros.
// Workgroups are dispatched split by split, so the long chunks (85% of the sources, the
// first half of the splits) run first and the grid drains on the short ones.
#pragma once
#include <algorithm>
#include <cstddef>

namespace rbm {

struct FarChunks {
  int s1, c1, c2;
};

// Source chunks per all-pairs sum for N points.  The grid has nbx = ceil(N/256) target
// blocks (one target per lane) times `split` source chunks; 256 CUs hold 2048 resident
// 4-wave workgroups, and about six rounds of them balance the waves' finish times
// (measured on MI355X: at 20k points six rounds are 5 % faster in float64 and 12 % in
// float32 than one), so split >= ceil(6 * 2048 / nbx).  Workgroups run split by split and
// every XCD sweeps the sources of the current chunks; at most kChunkSources sources (2 MiB
// of float64 records, half an XCD's 4 MB L2) in the longest chunk keeps that sweep in L2
// instead of streaming the Infinity Cache.  The long chunks of far_chunks hold 1.7 times
// the mean over floor(split / 2) slots, so split >= 1.7 N / kChunkSources + 2 (at 1.25 M
// points 67 chunks instead of 3).  At most 96 and nbx.
constexpr int kChunkSources = 32768;

inline int far_l2_split(long N) { return (int)((17 * N + 10L * kChunkSources - 1) / (10L * kChunkSources)) + 2; }

inline int far_split(int N) {
  const int nbx = (N + 255) / 256;
  const int rounds = (6 * 2048 + nbx - 1) / nbx;
  const int l2 = N > kChunkSources ? far_l2_split(N) : 1;
  return std::max(1, std::min(std::max(rounds, l2), std::min(96, nbx)));
}

// Bound, non-decreasing in N, of split * points over all sizes up to N: with nbx' target
// blocks the product is at most min(96, nbx') N', and each of the two lower bounds of the
// split gives at most (6*2048/nbx' + 1) * 256 nbx' or far_l2_split(N') N'.  The partial-sum
// buffer holds that many points' worth of slots.
inline size_t far_part_cap(size_t N) {
  const size_t nbx = (N + 255) / 256;
  const size_t rounds = (size_t)6 * 2048 * 256 + N + 256;
  const size_t l2 = (size_t)far_l2_split((long)N) * N;
  return std::min(std::min<size_t>(96, nbx) * N, std::max(rounds, l2));
}

inline FarChunks far_chunks(int N, int nsplit) {
  if (nsplit < 2) return {0, N, N};
  const int s1 = nsplit / 2, s2 = nsplit - s1;
  const long c1 = std::min((17L * N + 20L * s1 - 1) / (20L * s1), (long)N / s1);
  const long rest = N - s1 * c1;
  const long c2 = std::max(1L, (rest + s2 - 1) / s2);
  return {s1, (int)c1, (int)c2};
}

}  // namespace rbm

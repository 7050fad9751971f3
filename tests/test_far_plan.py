"""Host logic of the all-pairs sums: the source chunks of the partial-sum slots
(`csrc/far_plan.h`) cover every source exactly once, in order, within bounds, for every
slot count up to 96, and give the first half of the slots the long chunks at the slot
counts the library chooses.
Built with g++ from the header alone (no GPU)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1606_07428_amd", "csrc")

CHECK = r"""
#include <cstdio>
#include "far_plan.h"
int main() {
  long bad = 0, cases = 0, ordered_bad = 0;
  auto check = [&](int N, int ns) {
    const rbm::FarChunks fc = rbm::far_chunks(N, ns);
    long covered = 0, prev = 0;
    for (int s = 0; s < ns; ++s) {
      const long b0 = s < fc.s1 ? (long)s * fc.c1 : (long)fc.s1 * fc.c1 + (long)(s - fc.s1) * fc.c2;
      const long b1 = b0 + (s < fc.s1 ? fc.c1 : fc.c2) < N ? b0 + (s < fc.s1 ? fc.c1 : fc.c2) : N;
      if (b0 < 0) ++bad;
      if (b1 > b0) {
        if (b0 != prev) ++bad;
        prev = b1;
        covered += b1 - b0;
      }
    }
    if (covered != N) ++bad;
    // the library chooses at most one slot per 256 targets' block
    if (ns >= 2 && ns <= (N + 255) / 256 && fc.c1 < fc.c2) ++ordered_bad;
    ++cases;
  };
  for (int N = 1; N <= 3000; ++N)
    for (int ns = 1; ns <= 96; ++ns) check(N, ns);
  const int big[] = {19968, 59904, 73728, 160000, 544000, 1248000, 4000000};
  for (int N : big)
    for (int ns = 1; ns <= 96; ++ns) check(N, ns);
  // the slot buffer bound covers the split of every size up to N, and the chosen split's
  // chunks stay within the L2 share once the split is not capped at 96
  long cap_bad = 0, l2_bad = 0;
  for (long N = 1; N <= 4000000; N += (N < 100000 ? 1 : 997)) {
    const int ns = rbm::far_split((int)N);
    if ((size_t)ns * N > rbm::far_part_cap(N)) ++cap_bad;
    if (rbm::far_part_cap(N) < rbm::far_part_cap(N - 1 > 0 ? N - 1 : 1)) ++cap_bad;
    const rbm::FarChunks fc = rbm::far_chunks((int)N, ns);
    if (ns < 96 && ns < (N + 255) / 256 && fc.c1 > rbm::kChunkSources) ++l2_bad;
  }
  std::printf("%ld %ld %ld %ld %ld\n", cases, bad, ordered_bad, cap_bad, l2_bad);
  return 0;
}
"""


def test_far_chunks_cover_every_source_once(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    src = tmp_path / "check.cpp"
    src.write_text(CHECK)
    exe = tmp_path / "check"
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    cases, bad, ordered_bad, cap_bad, l2_bad = map(int, subprocess.run(
        [str(exe)], check=True, capture_output=True, text=True).stdout.split())
    assert cases > 280000
    assert bad == 0
    # at the slot counts the library uses, the first half of the slots take the long chunks
    assert ordered_bad == 0
    assert cap_bad == 0 and l2_bad == 0

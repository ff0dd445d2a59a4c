"""The rule that picks which entries of an item the exact path recomputes
(csrc/exact_rule.h, shared by every kernel's exact path), checked on the host:
a plain C++ program built with g++ calls it.

When the total is starved, every bit side must be recomputed, also a side
that sits above the bound while the total is below it (the total and a side
are summed in different orders, so a side can exceed the total by an ulp);
otherwise exactly the starved sides (NaN counts as starved)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2108_07001_amd", "csrc")

PROG = r"""
#include <cmath>
#include <cstdio>
#include <limits>
#include "exact_rule.h"
int main() {
  const float thr = std::ldexp(1.0f, 6 - 126 + 20);
  const float below = std::nextafter(thr, 0.0f), above = std::nextafter(thr, 1.0f);
  const float nan = std::numeric_limits<float>::quiet_NaN();
  float side[6] = {above, 1.0f, below, 2.0f, 3.0f, nan};
  // total below the bound, some sides above it: every side
  std::printf("%u\n", air::exact_entries<float>(below, side, 3, thr));
  // total above: only the starved sides (2: below, 5: NaN)
  std::printf("%u\n", air::exact_entries<float>(above, side, 3, thr));
  // total NaN: every side
  std::printf("%u\n", air::exact_entries<float>(nan, side, 3, thr));
  // nothing starved
  float ok[4] = {1.0f, 1.0f, thr, 2.0f};
  std::printf("%u\n", air::exact_entries<float>(5.0f, ok, 2, thr));
  // double, m = 12: all 24 bits when the total straddles
  double sd[24];
  for (int i = 0; i < 24; ++i) sd[i] = 1.0;
  std::printf("%u\n", air::exact_entries<double>(0.5, sd, 12, 0.75));
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_exact_entries_rule(tmp_path):
    src = tmp_path / "rule.cpp"
    src.write_text(PROG)
    exe = tmp_path / "rule"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    assert [int(x) for x in out] == [0b111111, 0b100100, 0b111111, 0, (1 << 24) - 1]

"""CPU test of how the resident-key kernel's workers share the ring
(paper_2004_09252_amd/csrc/resident_shares.h): for every worker count the
kernel can be started with, the positions each worker owns cover every
residue exactly once, and consecutive positions belong to workers `step`
apart (different workgroups of 4 waves).  A residue no worker owned would
never be served."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2004_09252_amd", "csrc")

PROGRAM = r"""
#include <cstdio>
#include <vector>
#include "resident_shares.h"
int main() {
  for (uint32_t W = 1; W < 4096; ++W) {
    const uint32_t inv = ms::share_stride_inverse(W);
    std::vector<int> owner(W, -1);
    for (uint32_t w = 0; w < W; ++w) {
      const uint32_t r = (uint32_t)((uint64_t)w * inv % W);
      if (owner[r] != -1) { std::printf("W=%u residue %u twice\n", W, r); return 1; }
      owner[r] = (int)w;
    }
    if (W >= 5) {
      // the documented stride: the smallest integer >= 4 coprime to W
      uint32_t want = 4;
      for (;; ++want) {
        uint32_t x = want, y = W;
        while (y) { const uint32_t t = x % y; x = y; y = t; }
        if (x == 1) break;
      }
      const uint32_t step = (uint32_t)((owner[1] - owner[0] + W) % W);
      if (step != want % W) { std::printf("W=%u step %u\n", W, step); return 1; }
      for (uint32_t r = 0; r + 1 < W; ++r)
        if ((uint32_t)((owner[r + 1] - owner[r] + W) % W) != step) {
          std::printf("W=%u uneven stride at %u\n", W, r); return 1;
        }
    }
    if ((uint64_t)(W - 1) * inv >= (1ull << 32)) { std::printf("overflow\n"); return 1; }
  }
  std::printf("ok\n");
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not present")
def test_worker_shares_cover_every_position_once(tmp_path):
    src = tmp_path / "shares.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "shares"
    r = subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, str(src),
                        "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout

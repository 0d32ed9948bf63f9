"""CPU test of how a predictor matrix product splits its K range
(paper_2004_09252_amd/csrc/gemm_split.h): for every output shape up to
1024 x 1024 (steps of 8, plus 1) and every K up to 4096, the slices are
whole K steps, non-empty, tile [0, K) exactly, number at most 4, and their
partial products fit the workspace's partial buffer; only products with
fewer than 128 output tiles split.  A slice past K would read past the
operands, and a partial buffer overrun would write past the workspace."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2004_09252_amd", "csrc")

PROGRAM = r"""
#include <cstdio>
#include <vector>
#include "gemm_split.h"
int main() {
  std::vector<int> dims = {1};
  for (int d = 8; d <= 1024; d += 8) dims.push_back(d);
  long plans = 0, split = 0;
  for (int M : dims)
    for (int N : dims) {
      const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
      for (int K = 1; K <= 4096; ++K) {
        const ms::SplitPlan p = ms::split_plan(M, N, K);
        ++plans;
        if (p.splits == 1) {
          if (p.k_split != K) { std::printf("M=%d N=%d K=%d unsplit k_split %d\n", M, N, K, p.k_split); return 1; }
          continue;
        }
        ++split;
        if (tiles >= ms::kSplitMaxTiles || p.splits > ms::kSplitMax ||
            K < 2 * ms::kSplitMinK) {
          std::printf("M=%d N=%d K=%d split %d\n", M, N, K, p.splits); return 1;
        }
        if (p.k_split <= 0 || p.k_split % ms::kGemmTileK) {
          std::printf("M=%d N=%d K=%d k_split %d\n", M, N, K, p.k_split); return 1;
        }
        // slices [z*k, min(K,(z+1)*k)) for z < splits: non-empty, cover K
        if ((long)(p.splits - 1) * p.k_split >= K || (long)p.splits * p.k_split < K) {
          std::printf("M=%d N=%d K=%d cover %d x %d\n", M, N, K, p.splits, p.k_split); return 1;
        }
        if ((unsigned long long)p.splits * M * N > ms::kSplitPartFloats) {
          std::printf("M=%d N=%d K=%d partials overrun\n", M, N, K); return 1;
        }
      }
    }
  if (split == 0) { std::printf("nothing split\n"); return 1; }
  std::printf("ok %ld plans, %ld split\n", plans, split);
  return 0;
}
"""


@pytest.mark.skipif(not shutil.which("g++"), reason="g++ not present")
def test_split_plans_stay_in_bounds(tmp_path):
    src = tmp_path / "split.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "split"
    r = subprocess.run(["g++", "-std=c++17", "-O2", "-I", CSRC, str(src),
                        "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout

// How a predictor matrix product splits its K range (host side;
// mlp_kernels.hip launches the plan).  Plain C++, no device code.
#pragma once

#include <stdint.h>

namespace ms {

// Output tile and K step of the product kernel.
constexpr int kGemmTile = 64;
constexpr int kGemmTileK = 128;
// A product with fewer output tiles than kSplitMaxTiles and K of at least
// twice kSplitMinK runs its K range in up to kSplitMax slices, each on its
// own workgroups, into a partial buffer of kSplitPartFloats floats.
constexpr int kSplitMaxTiles = 128;
constexpr int kSplitMax = 4;
constexpr int kSplitMinK = 256;
constexpr uint64_t kSplitPartFloats =
    (uint64_t)kSplitMax * kSplitMaxTiles * kGemmTile * kGemmTile;

struct SplitPlan {
  int splits;   // slices (1: no split)
  int k_split;  // K per slice: slice z covers [z * k_split, min(K, (z+1) * k_split))
};

// The plan for an M x N x K product: slices of whole K steps, every slice
// non-empty, splits * M * N <= kSplitPartFloats.
inline SplitPlan split_plan(int M, int N, int K) {
  const int tiles = ((N + kGemmTile - 1) / kGemmTile) *
                    ((M + kGemmTile - 1) / kGemmTile);
  int splits = 1;
  if (tiles < kSplitMaxTiles) {
    splits = K / kSplitMinK;
    if (splits > kSplitMax) splits = kSplitMax;
  }
  if (splits <= 1) return SplitPlan{1, K};
  // whole K steps per slice; rounding up can leave fewer slices
  const int k_split =
      ((K + splits - 1) / splits + kGemmTileK - 1) / kGemmTileK * kGemmTileK;
  splits = (K + k_split - 1) / k_split;
  return splits > 1 ? SplitPlan{splits, k_split} : SplitPlan{1, K};
}

}  // namespace ms

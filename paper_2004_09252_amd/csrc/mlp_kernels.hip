// Page-access predictor kernels for gfx950 (include/memshield_mlp.h).
//
// Matrix products use gfx950's bf16 matrix-core instruction
// v_mfma_f32_16x16x32_bf16: a wave multiplies a 16x32 bf16 tile of A by a
// 32x16 bf16 tile of B into a 16x16 float32 accumulator.  Operand layout for
// lane l of the wave: A row (l % 16), K elements 8*(l/16)..+7; B column
// (l % 16), K elements 8*(l/16)..+7; accumulator column (l % 16), rows
// 4*(l/16)..+3.  A workgroup of four waves computes a 64x64 output tile,
// each wave a 32x32 quarter (2x2 MFMA tiles), staging 64x128 bf16 tiles of A
// and B through LDS per K step of 128: four 16-byte global loads per
// operand and thread, the next step's loads in flight during the current
// step's MFMAs.  Transposed operands are handled in the LDS staging, so one kernel
// serves the forward products and both gradient products.  The epilogue adds a bias, applies ReLU or a ReLU
// mask taken from a stored activation, and writes float32 and/or bf16.
//
// Everything else (embedding gather and its deterministic scatter-add,
// softmax cross-entropy, bias gradients, Adam, top-k) is elementwise or a
// small reduction on the vector ALUs.  Reductions run in a fixed order, so
// results are bit-reproducible run to run.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>

#include "gemm_split.h"
#include "memshield_mlp.h"

namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kTile = ms::kGemmTile;
constexpr int kTileK = ms::kGemmTileK;

__device__ __forceinline__ float bf2f(uint16_t h) {
  return __uint_as_float((uint32_t)h << 16);
}

// float32 -> bfloat16, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

struct GemmArgs {
  const uint16_t* A;  // logical M x K: A[m*lda+k], or A[k*lda+m] if transA
  const uint16_t* B;  // logical K x N: B[k*ldb+n], or B[n*ldb+k] if transB
  const uint16_t* bias;  // N entries or null
  const uint16_t* mask;  // M x N (ld ldm) or null: out *= (mask > 0)
  float* outF;           // M x N float32 (ld ldo) or null
  uint16_t* outH;        // M x N bf16 (ld ldh) or null
  int M, N, K;
  int lda, ldb, ldm, ldo, ldh;
  int transA, transB, relu;
  // split K: blockIdx.z takes k in [z * k_split, (z + 1) * k_split); with
  // splits > 1 each slice stores its float32 partial product in `part`
  // (splits x M x N) and gemm_reduce_kernel adds the slices in order and
  // applies the epilogue
  float* part;
  int splits, k_split;
};

// the split plan and the partial buffer's size (gemm_split.h)
using ms::kSplitPartFloats;

// The epilogue: bias, ReLU, mask, then the float32 and/or bf16 output.
__device__ __forceinline__ void gemm_store(const GemmArgs& g, int row, int col,
                                           float v);

// Eight consecutive bf16 of a row starting at p, of which `valid` (0..8)
// lie inside the matrix (the rest read as zero): one 16-byte load when all
// eight are inside and the row is 16-byte aligned, element loads otherwise.
__device__ __forceinline__ uint4 load8(const uint16_t* p, int valid,
                                       bool vec) {
  if (vec && valid == 8) return *reinterpret_cast<const uint4*>(p);
  uint16_t e[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) e[i] = i < valid ? p[i] : (uint16_t)0;
  return make_uint4(e[0] | (uint32_t)e[1] << 16, e[2] | (uint32_t)e[3] << 16,
                    e[4] | (uint32_t)e[5] << 16, e[6] | (uint32_t)e[7] << 16);
}

__device__ __forceinline__ int clamp8(int64_t left) {
  return left <= 0 ? 0 : (left >= 8 ? 8 : (int)left);
}

__device__ __forceinline__ uint16_t half_of(const uint4& v, int i) {
  const uint32_t w = i < 2 ? v.x : (i < 4 ? v.y : (i < 6 ? v.z : v.w));
  return (uint16_t)(w >> (16 * (i & 1)));
}

// Both LDS tiles hold their K dimension contiguous (A as [m][k], B as
// [n][k]), so an MFMA operand (4 consecutive k) is one 8-byte LDS read.  A
// row is kTileK k plus 8 of padding, which spreads the rows a wave reads at
// once over the LDS banks.
constexpr int kLdsRow = kTileK + 8;
// 8-element chunks per operand tile (64 x kTileK) and per thread
constexpr int kChunks = kTile * kTileK / 8 / 256;
static_assert(kChunks * 256 * 8 == kTile * kTileK, "tile split");

// Workgroup barrier for the LDS tiles only: the LDS accesses before it are
// complete (lgkmcnt) and visible after it, while global loads stay in
// flight across it.  __syncthreads() would also wait for every outstanding
// global load (it is a fence as well), which drains the next step's
// prefetch at each step.  The memory clobber keeps the compiler from moving
// LDS accesses across it.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" : : : "memory");
}

__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g) {
  __shared__ __align__(16) uint16_t As[kTile][kLdsRow];
  __shared__ __align__(16) uint16_t Bt[kTile][kLdsRow];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int m0 = blockIdx.y * kTile, n0 = blockIdx.x * kTile;
  // 16-byte global loads need 16-byte aligned rows
  const bool vecA = (reinterpret_cast<uintptr_t>(g.A) & 15) == 0 &&
                    (g.lda & 7) == 0;
  const bool vecB = (reinterpret_cast<uintptr_t>(g.B) & 15) == 0 &&
                    (g.ldb & 7) == 0;
  // Each thread moves kChunks 8-element chunks of A and of B per K step,
  // along the dimension that is contiguous in memory; chunk c = tid + 256j
  // of a tile of 64 rows (m or n) by kTileK k is, with R = kTileK / 8:
  //   A [m][k], B^T [n][k] (k contiguous): row c / R, k 8 * (c % R); one
  //     16-byte LDS store;
  //   A^T [k][m], B [k][n] (m or n contiguous): k c % kTileK, rows
  //     8 * (c / kTileK) + 0..7; eight 2-byte LDS stores, and since a wave's
  //     lanes hold 64 consecutive k of the same rows, each of those stores
  //     spreads over all the LDS banks.
  constexpr int R = kTileK / 8;
  uint4 ra[kChunks], rb[kChunks];
  auto fetch = [&](int k0) {
    // A tile wholly inside both matrices, with 16-byte aligned rows, takes
    // straight-line 16-byte loads; the test is uniform across the
    // workgroup, so no lane waits on another's element loads
    const bool interior = vecA && vecB && m0 + kTile <= g.M &&
                          n0 + kTile <= g.N && k0 + kTileK <= g.K;
    if (interior) {
#pragma unroll
      for (int j = 0; j < kChunks; ++j) {
        const int c = tid + 256 * j;
        const int64_t ao =
            !g.transA ? (int64_t)(m0 + c / R) * g.lda + k0 + 8 * (c % R)
                      : (int64_t)(k0 + c % kTileK) * g.lda + m0 +
                            8 * (c / kTileK);
        const int64_t bo =
            !g.transB ? (int64_t)(k0 + c % kTileK) * g.ldb + n0 +
                            8 * (c / kTileK)
                      : (int64_t)(n0 + c / R) * g.ldb + k0 + 8 * (c % R);
        ra[j] = *reinterpret_cast<const uint4*>(g.A + ao);
        rb[j] = *reinterpret_cast<const uint4*>(g.B + bo);
      }
      return;
    }
#pragma unroll
    for (int j = 0; j < kChunks; ++j) {
      const int c = tid + 256 * j;
      if (!g.transA) {
        const int64_t m = m0 + c / R, k = k0 + 8 * (c % R);
        const int valid = m < g.M ? clamp8(g.K - k) : 0;
        ra[j] = load8(g.A + (valid ? m * g.lda + k : 0), valid, vecA);
      } else {
        const int64_t k = k0 + c % kTileK, m = m0 + 8 * (c / kTileK);
        const int valid = k < g.K ? clamp8(g.M - m) : 0;
        ra[j] = load8(g.A + (valid ? k * g.lda + m : 0), valid, vecA);
      }
      if (!g.transB) {
        const int64_t k = k0 + c % kTileK, n = n0 + 8 * (c / kTileK);
        const int valid = k < g.K ? clamp8(g.N - n) : 0;
        rb[j] = load8(g.B + (valid ? k * g.ldb + n : 0), valid, vecB);
      } else {
        const int64_t n = n0 + c / R, k = k0 + 8 * (c % R);
        const int valid = n < g.N ? clamp8(g.K - k) : 0;
        rb[j] = load8(g.B + (valid ? n * g.ldb + k : 0), valid, vecB);
      }
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int j = 0; j < kChunks; ++j) {
      const int c = tid + 256 * j;
      if (!g.transA) {
        *reinterpret_cast<uint4*>(&As[c / R][8 * (c % R)]) = ra[j];
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i)
          As[8 * (c / kTileK) + i][c % kTileK] = half_of(ra[j], i);
      }
      if (g.transB) {
        *reinterpret_cast<uint4*>(&Bt[c / R][8 * (c % R)]) = rb[j];
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i)
          Bt[8 * (c / kTileK) + i][c % kTileK] = half_of(rb[j], i);
      }
    }
  };
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (v4f){0.f, 0.f, 0.f, 0.f};

  // this workgroup's K slice (the whole K unless split); k_split is a
  // multiple of kTileK, so only the last slice can end inside a K step, and
  // the loads mask that step against K
  const int kbeg = blockIdx.z * g.k_split;
  const int kend = min(g.K, kbeg + g.k_split);
  fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += kTileK) {
    stash();
    lds_barrier();
    // the next step's global loads are in flight during this step's MFMAs
    if (k0 + kTileK < kend) fetch(k0 + kTileK);
#pragma unroll
    for (int kk = 0; kk < kTileK; kk += 32) {
      // one 16-byte LDS read per operand tile: 8 consecutive K elements
      const int kb = kk + 8 * (lane >> 4);
      v8bf a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        a[i] = *reinterpret_cast<const v8bf*>(
            &As[wm * 32 + i * 16 + (lane & 15)][kb]);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        b[j] = *reinterpret_cast<const v8bf*>(
            &Bt[wn * 32 + j * 16 + (lane & 15)][kb]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              a[i], b[j], acc[i][j], 0, 0, 0);
    }
    lds_barrier();
  }

#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + r;
        const int col = n0 + wn * 32 + j * 16 + (lane & 15);
        if (row >= g.M || col >= g.N) continue;
        if (g.splits > 1)
          g.part[((size_t)blockIdx.z * g.M + row) * g.N + col] = acc[i][j][r];
        else
          gemm_store(g, row, col, acc[i][j][r]);
      }
}

__device__ __forceinline__ void gemm_store(const GemmArgs& g, int row, int col,
                                           float v) {
  if (g.bias) v += bf2f(g.bias[col]);
  if (g.relu) v = v > 0.f ? v : 0.f;
  if (g.mask && !(bf2f(g.mask[(size_t)row * g.ldm + col]) > 0.f)) v = 0.f;
  if (g.outF) g.outF[(size_t)row * g.ldo + col] = v;
  if (g.outH) g.outH[(size_t)row * g.ldh + col] = f2bf(v);
}

// The K slices of a split GEMM added in slice order (so the sum does not
// depend on which slice finished first), then the epilogue.
__global__ __launch_bounds__(256) void gemm_reduce_kernel(GemmArgs g) {
  const size_t mn = (size_t)g.M * g.N;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < mn;
       i += (size_t)gridDim.x * blockDim.x) {
    float v = g.part[i];
    for (int z = 1; z < g.splits; ++z) v += g.part[z * mn + i];
    gemm_store(g, (int)(i / g.N), (int)(i % g.N), v);
  }
}

// x[b][s*D + d] = E[ids[b][s]][d]; ids outside [0, V) are clamped.
__global__ void embed_gather_kernel(const uint16_t* __restrict__ E,
                                    const int32_t* __restrict__ ids, int B,
                                    int C, int D, int V,
                                    uint16_t* __restrict__ x) {
  const int64_t n = (int64_t)B * C * D;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t bs = i / D;
    const int d = (int)(i % D);
    int id = ids[bs];
    id = id < 0 ? 0 : (id >= V ? V - 1 : id);
    x[i] = E[(int64_t)id * D + d];
  }
}

// dE[v][d] = sum over positions i, in increasing order, with ids[i] == v of
// dx[i][d] (ids clamped into [0, V) as the forward pass clamps them).
// A workgroup of four waves owns four consecutive rows v, one per wave.  It
// stages the ids, kScatterChunk at a time, into LDS as 16-bit values (V is
// at most 65536) with all its threads, 32 loads per thread in flight; each
// wave then scans the chunk for its row, 512 positions per step (eight LDS
// reads in flight, one ballot that skips a step without a match, then one
// per 64 positions in order), and appends the matching positions, lowest
// first, to a list of its own in LDS.  When the list is full, and at
// the end, the wave adds the dx rows it names with up to 16 loads in flight,
// in list order.  So every row's sum runs over its positions in increasing
// order, one after another, whatever the chunk and list sizes (the sum is
// deterministic), and the ids are read from memory once per workgroup
// instead of once per row.  Embedding widths above 64 take one pass per 64
// columns.
constexpr int kScatterChunk = 16384;
constexpr int kScatterList = 256;
static_assert(kScatterChunk % 512 == 0, "scan steps of 512 stay in the chunk");
__global__ __launch_bounds__(256) void embed_scatter_kernel(
    const float* __restrict__ dx, const int32_t* __restrict__ ids, int B,
    int C, int D, int V, float* __restrict__ dE) {
  __shared__ uint16_t sid[kScatterChunk];
  __shared__ int64_t plist[4][kScatterList];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int v = blockIdx.x * 4 + wave;  // >= V: stages ids, writes nothing
  const int64_t n = (int64_t)B * C;
  const unsigned long long below = (1ull << lane) - 1;
  int64_t* list = plist[wave];
  for (int d0 = 0; d0 < D; d0 += 64) {
    const int d = d0 + lane;
    float acc = 0.f;
    int cnt = 0;
    // add the listed rows in list order, 16 loads in flight
    auto flush = [&]() {
      for (int t0 = 0; t0 < cnt; t0 += 16) {
        float val[16];
#pragma unroll
        for (int t = 0; t < 16; ++t)
          val[t] = (t0 + t < cnt && d < D)
                       ? dx[list[t0 + t] * D + d]
                       : 0.f;
#pragma unroll
        for (int t = 0; t < 16; ++t)
          if (t0 + t < cnt) acc += val[t];
      }
      cnt = 0;
    };
    for (int64_t base = 0; base < n; base += kScatterChunk) {
      const int len = (int)(n - base < kScatterChunk ? n - base : kScatterChunk);
      __syncthreads();  // the previous chunk's scans are done
      // 32 loads of each thread in flight before their stores
      for (int j0 = 0; j0 < len; j0 += 256 * 32) {
        int x[32];
#pragma unroll
        for (int q = 0; q < 32; ++q) {
          const int j = j0 + 256 * q + (int)threadIdx.x;
          x[q] = j < len ? ids[base + j] : 0;
        }
#pragma unroll
        for (int q = 0; q < 32; ++q) {
          const int j = j0 + 256 * q + (int)threadIdx.x;
          if (j < len)
            sid[j] = (uint16_t)(x[q] < 0 ? 0 : (x[q] >= V ? V - 1 : x[q]));
        }
      }
      __syncthreads();
      if (v < V) {
        // 512 positions per step: eight LDS reads in flight, one ballot
        // that skips the step when none matches, else one per 64 in order
        for (int j0 = 0; j0 < len; j0 += 512) {
          bool hit[8];
          bool any = false;
          // (j0 + 511 stays inside the chunk buffer, whose size is a
          // multiple of 512: the reads need no guard, entries past len are
          // masked out)
          uint32_t sv[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) sv[q] = sid[j0 + 64 * q + lane];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            hit[q] = (j0 + 64 * q + lane < len) & (sv[q] == (uint32_t)v);
            any = any | hit[q];
          }
          if (!__ballot(any)) continue;
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const unsigned long long m = __ballot(hit[q]);
            if (!m) continue;
            const int k = __popcll(m);
            if (cnt + k > kScatterList) flush();
            if (hit[q])
              list[cnt + __popcll(m & below)] = base + j0 + 64 * q + lane;
            cnt += k;
          }
        }
      }
    }
    if (v < V) {
      flush();
      if (d < D) dE[(int64_t)v * D + d] = acc;
    }
  }
}

// One workgroup per row: loss_row[b] and dlogits = (softmax - onehot) / B.
__global__ __launch_bounds__(256) void softmax_ce_kernel(
    const float* __restrict__ logits, const int32_t* __restrict__ targets,
    int B, int V, float* __restrict__ row_loss, float* __restrict__ dlF,
    uint16_t* __restrict__ dlH) {
  __shared__ float red[256];
  const int b = blockIdx.x;
  const float* row = logits + (int64_t)b * V;
  float mx = -INFINITY;
  for (int i = threadIdx.x; i < V; i += 256) mx = fmaxf(mx, row[i]);
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  mx = red[0];
  __syncthreads();
  float sum = 0.f;
  for (int i = threadIdx.x; i < V; i += 256) sum += expf(row[i] - mx);
  red[threadIdx.x] = sum;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  sum = red[0];
  int t = targets[b];
  t = t < 0 ? 0 : (t >= V ? V - 1 : t);
  const float inv_b = 1.f / (float)B;
  for (int i = threadIdx.x; i < V; i += 256) {
    float p = expf(row[i] - mx) / sum;
    if (i == t) p -= 1.f;
    p *= inv_b;
    dlF[(int64_t)b * V + i] = p;
    dlH[(int64_t)b * V + i] = f2bf(p);
  }
  if (threadIdx.x == 0) row_loss[b] = logf(sum) + mx - row[t];
}

// loss = mean of row_loss (one workgroup, fixed order).
__global__ void mean_kernel(const float* __restrict__ v, int n,
                            float* __restrict__ out) {
  __shared__ float red[256];
  float s = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) s += v[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0] / (float)n;
}

// out[n] = sum over m of in[m][n] (float32).  A workgroup takes 64 columns;
// its 16 waves sum the rows g, g+16, g+32, ... of each column, and the 16
// partial sums are added in a fixed tree order (deterministic).
constexpr int kColsumGroups = 16;
constexpr int kColsumMaxSlices = 32;

// Row slices for a column sum over M rows: enough to fill the device with
// (N / 64) x slices workgroups, each slice at least 64 rows.
int colsum_slices(int M) {
  const int s = (M + 63) / 64;
  return s < 1 ? 1 : (s > kColsumMaxSlices ? kColsumMaxSlices : s);
}

// Partial column sums: workgroup (x, s) sums rows [s*R, (s+1)*R) (R =
// ceil(M / slices)) of columns 64x..64x+63 into part[s][n].  Sixteen waves
// take rows g, g+16, ... of the slice; an LDS tree in fixed order combines
// them.
__global__ __launch_bounds__(64 * kColsumGroups) void colsum_partial_kernel(
    const float* __restrict__ in, int M, int N, int ld,
    float* __restrict__ part) {
  __shared__ float acc[kColsumGroups][64];
  const int c = threadIdx.x & 63;
  const int g = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + c;
  const int rows = (M + gridDim.y - 1) / gridDim.y;
  const int r0 = blockIdx.y * rows;
  const int r1 = r0 + rows < M ? r0 + rows : M;
  float s = 0.f;
  if (n < N)
    for (int m = r0 + g; m < r1; m += kColsumGroups)
      s += in[(int64_t)m * ld + n];
  acc[g][c] = s;
  __syncthreads();
  for (int k = kColsumGroups / 2; k > 0; k >>= 1) {
    if (g < k) acc[g][c] += acc[g + k][c];
    __syncthreads();
  }
  if (g == 0 && n < N) part[(int64_t)blockIdx.y * N + n] = acc[0][c];
}

// out[n] = part[0][n] + part[1][n] + ... in slice order (deterministic).
__global__ __launch_bounds__(256) void colsum_final_kernel(
    const float* __restrict__ part, int slices, int N,
    float* __restrict__ out) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int i = 0; i < slices; ++i) s += part[(int64_t)i * N + n];
  out[n] = s;
}

__global__ void adam_kernel(float* __restrict__ w, float* __restrict__ m,
                            float* __restrict__ v, const float* __restrict__ g,
                            uint16_t* __restrict__ wh, uint64_t n, float lr,
                            float b1, float b2, float eps, float c1,
                            float c2) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi * c1;
    const float vh = vi * c2;
    const float wi = w[i] - lr * mh / (sqrtf(vh) + eps);
    w[i] = wi;
    wh[i] = f2bf(wi);
  }
}

__global__ void to_bf16_kernel(const float* __restrict__ s,
                               uint16_t* __restrict__ d, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    d[i] = f2bf(s[i]);
}

// One wave per row: k rounds of (lane-local best, wave reduction); the
// order is (value descending, id ascending); NaN counts as -inf.  With
// `prob` set, also the softmax probability of each chosen id over the whole
// row.
// a ranks before b: larger value, or the same value and a lower index
__device__ __forceinline__ bool ranks_before(float av, int ai, float bv,
                                             int bi) {
  return av > bv || (av == bv && ai < bi);
}

// Values a lane loads at once: the loads of a chunk are independent, so
// the row costs one memory round trip per chunk instead of one per value.
constexpr int kTopkChunk = 16;

__global__ __launch_bounds__(64) void topk_kernel(
    const float* __restrict__ logits, int V, int k, int exclude,
    int32_t* __restrict__ out, float* __restrict__ prob) {
  const int b = blockIdx.x;
  const int lane = threadIdx.x;
  const float* row = logits + (int64_t)b * V;
  // This lane's running maximum and sum of exp(x - max) over its positions
  // (one pass; the lanes' sums are rescaled to the row maximum at the end).
  float mx = -INFINITY, sum = 0.f;
  // Each lane keeps the best 16 of its positions lane, lane + 64, ...
  // (NaN counts as -inf, `exclude` and positions past the row are left out)
  // sorted in registers; an entry enters by swapping down the list.  The
  // best k of the row are the best k of the lanes' lists.
  float lv[16];
  int li[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    lv[t] = -INFINITY;
    li[t] = 0x7fffffff;
  }
  for (int base = 0; base < V; base += 64 * kTopkChunk) {
    float x[kTopkChunk];
#pragma unroll
    for (int t = 0; t < kTopkChunk; ++t) {
      const int i = base + 64 * t + lane;
      x[t] = i < V ? row[i] : -INFINITY;
    }
    if (prob) {
      float m = mx;
#pragma unroll
      for (int t = 0; t < kTopkChunk; ++t) m = fmaxf(m, x[t]);
      if (m != -INFINITY) {
        float s2 = sum * expf(mx - m);
#pragma unroll
        for (int t = 0; t < kTopkChunk; ++t) s2 += expf(x[t] - m);
        sum = s2;
        mx = m;
      }
    }
#pragma unroll
    for (int t = 0; t < kTopkChunk; ++t) {
      const int i = base + 64 * t + lane;
      // a left-out position becomes (-inf, INT_MAX), which never ranks
      // before an entry of the list (the list starts full of those)
      const bool in = i < V && i != exclude;
      float cv = in ? (x[t] != x[t] ? -INFINITY : x[t]) : -INFINITY;
      int ci = in ? i : 0x7fffffff;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const bool before = ranks_before(cv, ci, lv[u], li[u]);
        const float tv = lv[u];
        const int ti = li[u];
        lv[u] = before ? cv : tv;
        li[u] = before ? ci : ti;
        cv = before ? tv : cv;
        ci = before ? ti : ci;
      }
    }
  }
  if (prob) {
    // the row maximum, then each lane's sum rescaled to it
    float rm = mx;
    for (int off = 32; off > 0; off >>= 1)
      rm = fmaxf(rm, __shfl_xor(rm, off, 64));
    float rs = mx == -INFINITY ? 0.f : sum * expf(mx - rm);
    for (int off = 32; off > 0; off >>= 1) rs += __shfl_xor(rs, off, 64);
    mx = rm;
    sum = rs;
  }
  // k rounds: the best list head over the wave, popped by its lane
  for (int r = 0; r < k; ++r) {
    float bv = lv[0];
    int bi = li[0];
    for (int off = 32; off > 0; off >>= 1) {
      const float ov = __shfl_xor(bv, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ranks_before(ov, oi, bv, bi)) { bv = ov; bi = oi; }
    }
    const bool mine = li[0] == bi;
#pragma unroll
    for (int t = 0; t < 15; ++t) {
      lv[t] = mine ? lv[t + 1] : lv[t];
      li[t] = mine ? li[t + 1] : li[t];
    }
    lv[15] = mine ? -INFINITY : lv[15];
    li[15] = mine ? 0x7fffffff : li[15];
    if (lane == 0) {
      out[(int64_t)b * k + r] = bi;
      if (prob) prob[(int64_t)b * k + r] = expf(bv - mx) / sum;
    }
  }
}

uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

bool shape_ok(const ms_mlp_shape* s) {
  if (!s) return false;
  const int64_t cd = (int64_t)s->context * s->embed;
  return s->vocab >= 64 && s->vocab % 64 == 0 && s->context >= 1 &&
         s->embed >= 1 && cd % 32 == 0 && s->hidden >= 32 &&
         s->hidden % 32 == 0 && cd <= (1 << 16) && s->hidden <= (1 << 14) &&
         s->vocab <= (1 << 16);
}

struct Ws {
  uint16_t *x, *h1, *h2, *dlH, *dz2H, *dz1H;
  float *logits, *dlF, *dz2F, *dz1F, *dxF, *row_loss, *colpart, *part;
  uint64_t bytes;
};

Ws carve(const ms_mlp_shape* s, int64_t Bm, uint8_t* base) {
  const int64_t CD = (int64_t)s->context * s->embed, H = s->hidden,
                V = s->vocab;
  Ws w;
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    uint8_t* p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  w.x = (uint16_t*)take(Bm * CD * 2);
  w.h1 = (uint16_t*)take(Bm * H * 2);
  w.h2 = (uint16_t*)take(Bm * H * 2);
  w.dlH = (uint16_t*)take(Bm * V * 2);
  w.dz2H = (uint16_t*)take(Bm * H * 2);
  w.dz1H = (uint16_t*)take(Bm * H * 2);
  w.logits = (float*)take(Bm * V * 4);
  w.dlF = (float*)take(Bm * V * 4);
  w.dz2F = (float*)take(Bm * H * 4);
  w.dz1F = (float*)take(Bm * H * 4);
  w.dxF = (float*)take(Bm * CD * 4);
  w.row_loss = (float*)take(Bm * 4);
  w.colpart = (float*)take((uint64_t)kColsumMaxSlices * (V > H ? V : H) * 4);
  w.part = (float*)take(kSplitPartFloats * 4);
  w.bytes = off;
  return w;
}

// Column sums of an M x N float32 matrix (leading dimension ld) into out,
// through per-slice partial sums in `part` (kColsumMaxSlices x N floats).
hipError_t colsum(const float* in, int M, int N, int ld, float* out,
                  float* part, hipStream_t st) {
  const int slices = colsum_slices(M);
  hipLaunchKernelGGL(colsum_partial_kernel, dim3((N + 63) / 64, slices),
                     dim3(64 * kColsumGroups), 0, st, in, M, N, ld, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(colsum_final_kernel, dim3((N + 255) / 256), dim3(256), 0,
                     st, part, slices, N, out);
  return hipGetLastError();
}

// Launch one GEMM; one with few output tiles and a long K is split over K
// into the workspace's partial buffer, then reduced.
hipError_t gemm(GemmArgs g, const Ws& w, hipStream_t s) {
  const int tn = (g.N + kTile - 1) / kTile, tm = (g.M + kTile - 1) / kTile;
  // splits * M * N <= kSplitPartFloats (tests/test_gemm_split_cpu.py)
  const ms::SplitPlan plan = ms::split_plan(g.M, g.N, g.K);
  g.splits = plan.splits;
  g.k_split = plan.k_split;
  g.part = w.part;
  hipLaunchKernelGGL(gemm_bf16_kernel, dim3(tn, tm, g.splits), dim3(256), 0,
                     s, g);
  if (g.splits == 1) return hipGetLastError();
  const uint64_t mn = (uint64_t)g.M * g.N;
  hipLaunchKernelGGL(gemm_reduce_kernel,
                     dim3((unsigned)std::min<uint64_t>((mn + 255) / 256, 1024)),
                     dim3(256), 0, s, g);
  return hipGetLastError();
}

GemmArgs gemm_args(const uint16_t* A, int lda, int transA, const uint16_t* B,
                   int ldb, int transB, int M, int N, int K) {
  GemmArgs g;
  memset(&g, 0, sizeof(g));
  g.A = A; g.lda = lda; g.transA = transA;
  g.B = B; g.ldb = ldb; g.transB = transB;
  g.M = M; g.N = N; g.K = K;
  return g;
}

int grid_for(uint64_t n) {
  uint64_t b = (n + 255) / 256;
  return (int)(b > 4096 ? 4096 : (b ? b : 1));
}

// Forward into the workspace; logits to `logits`.
hipError_t forward_impl(const ms_mlp_shape* s, const uint16_t* P,
                        const uint64_t off[7], const int32_t* ids, int B,
                        float* logits, const Ws& w, hipStream_t st) {
  const int CD = s->context * s->embed, H = s->hidden, V = s->vocab;
  const int64_t n = (int64_t)B * CD;
  hipLaunchKernelGGL(embed_gather_kernel, dim3(grid_for(n)), dim3(256), 0, st,
                     P + off[0], ids, B, s->context, s->embed, V, w.x);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  GemmArgs g = gemm_args(w.x, CD, 0, P + off[1], H, 0, B, H, CD);
  g.bias = P + off[2]; g.relu = 1; g.outH = w.h1; g.ldh = H;
  if ((e = gemm(g, w, st)) != hipSuccess) return e;
  g = gemm_args(w.h1, H, 0, P + off[3], H, 0, B, H, H);
  g.bias = P + off[4]; g.relu = 1; g.outH = w.h2; g.ldh = H;
  if ((e = gemm(g, w, st)) != hipSuccess) return e;
  g = gemm_args(w.h2, H, 0, P + off[5], V, 0, B, V, H);
  g.bias = P + off[6]; g.outF = logits; g.ldo = V;
  return gemm(g, w, st);
}

}  // namespace

extern "C" {

uint64_t ms_mlp_offsets(const ms_mlp_shape* s, uint64_t off[7]) {
  if (!shape_ok(s) || !off) return 0;
  const uint64_t CD = (uint64_t)s->context * s->embed, H = s->hidden,
                 V = s->vocab, D = s->embed;
  const uint64_t sizes[7] = {V * D, CD * H, H, H * H, H, H * V, V};
  uint64_t o = 0;
  for (int i = 0; i < 7; ++i) {
    off[i] = o;
    o += sizes[i];
  }
  return o;
}

uint64_t ms_mlp_workspace_bytes(const ms_mlp_shape* s, int32_t max_batch) {
  if (!shape_ok(s) || max_batch < 1 || max_batch > (1 << 20)) return 0;
  return carve(s, max_batch, nullptr).bytes;
}

ms_status ms_mlp_forward(const ms_mlp_shape* s, const uint16_t* params,
                         const int32_t* ids, int32_t batch, float* logits,
                         void* workspace, uint64_t ws_bytes, void* stream) {
  uint64_t off[7];
  if (!ms_mlp_offsets(s, off) || !params || !ids || !logits || !workspace ||
      batch < 1)
    return MS_EINVAL;
  const Ws w = carve(s, batch, static_cast<uint8_t*>(workspace));
  if (w.bytes > ws_bytes) return MS_EINVAL;
  hipError_t e = forward_impl(s, params, off, ids, batch, logits, w,
                              static_cast<hipStream_t>(stream));
  return e == hipSuccess ? MS_OK : MS_EDEVICE;
}

ms_status ms_mlp_backward(const ms_mlp_shape* s, const uint16_t* P,
                          const int32_t* ids, const int32_t* targets,
                          int32_t B, float* G, float* loss, void* workspace,
                          uint64_t ws_bytes, void* stream) {
  uint64_t off[7];
  if (!ms_mlp_offsets(s, off) || !P || !ids || !targets || !G || !loss ||
      !workspace || B < 1)
    return MS_EINVAL;
  const Ws w = carve(s, B, static_cast<uint8_t*>(workspace));
  if (w.bytes > ws_bytes) return MS_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int CD = s->context * s->embed, H = s->hidden, V = s->vocab;
  hipError_t e = forward_impl(s, P, off, ids, B, w.logits, w, st);
  if (e != hipSuccess) return MS_EDEVICE;
  hipLaunchKernelGGL(softmax_ce_kernel, dim3(B), dim3(256), 0, st, w.logits,
                     targets, B, V, w.row_loss, w.dlF, w.dlH);
  hipLaunchKernelGGL(mean_kernel, dim3(1), dim3(256), 0, st, w.row_loss, B,
                     loss);
  // output layer: dW3 = h2^T dl, db3 = colsum(dl), dz2 = (dl W3^T) * (h2>0)
  GemmArgs g = gemm_args(w.h2, H, 1, w.dlH, V, 0, H, V, B);
  g.outF = G + off[5]; g.ldo = V;
  if (gemm(g, w, st) != hipSuccess) return MS_EDEVICE;
  if (colsum(w.dlF, B, V, V, G + off[6], w.colpart, st) != hipSuccess)
    return MS_EDEVICE;
  g = gemm_args(w.dlH, V, 0, P + off[5], V, 1, B, H, V);
  g.mask = w.h2; g.ldm = H; g.outF = w.dz2F; g.ldo = H; g.outH = w.dz2H;
  g.ldh = H;
  if (gemm(g, w, st) != hipSuccess) return MS_EDEVICE;
  // layer 2: dW2 = h1^T dz2, db2 = colsum(dz2), dz1 = (dz2 W2^T) * (h1>0)
  g = gemm_args(w.h1, H, 1, w.dz2H, H, 0, H, H, B);
  g.outF = G + off[3]; g.ldo = H;
  if (gemm(g, w, st) != hipSuccess) return MS_EDEVICE;
  if (colsum(w.dz2F, B, H, H, G + off[4], w.colpart, st) != hipSuccess)
    return MS_EDEVICE;
  g = gemm_args(w.dz2H, H, 0, P + off[3], H, 1, B, H, H);
  g.mask = w.h1; g.ldm = H; g.outF = w.dz1F; g.ldo = H; g.outH = w.dz1H;
  g.ldh = H;
  if (gemm(g, w, st) != hipSuccess) return MS_EDEVICE;
  // layer 1: dW1 = x^T dz1, db1 = colsum(dz1), dx = dz1 W1^T
  g = gemm_args(w.x, CD, 1, w.dz1H, H, 0, CD, H, B);
  g.outF = G + off[1]; g.ldo = H;
  if (gemm(g, w, st) != hipSuccess) return MS_EDEVICE;
  if (colsum(w.dz1F, B, H, H, G + off[2], w.colpart, st) != hipSuccess)
    return MS_EDEVICE;
  g = gemm_args(w.dz1H, H, 0, P + off[1], H, 1, B, CD, H);
  g.outF = w.dxF; g.ldo = CD;
  if (gemm(g, w, st) != hipSuccess) return MS_EDEVICE;
  hipLaunchKernelGGL(embed_scatter_kernel, dim3((V + 3) / 4), dim3(256), 0,
                     st, w.dxF, ids, B, s->context, s->embed, V, G + off[0]);
  return hipGetLastError() == hipSuccess ? MS_OK : MS_EDEVICE;
}

ms_status ms_mlp_adam(const ms_mlp_shape* s, float* master, float* m,
                      float* v, const float* grads, uint16_t* params,
                      float lr, float beta1, float beta2, float eps,
                      int32_t step, void* stream) {
  uint64_t off[7];
  const uint64_t n = ms_mlp_offsets(s, off);
  if (!n || !master || !m || !v || !grads || !params || step < 1)
    return MS_EINVAL;
  const float c1 = (float)(1.0 / (1.0 - pow((double)beta1, step)));
  const float c2 = (float)(1.0 / (1.0 - pow((double)beta2, step)));
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), master, m, v, grads,
                     params, n, lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? MS_OK : MS_EDEVICE;
}

ms_status ms_mlp_to_bf16(const float* src, uint16_t* dst, uint64_t n,
                         void* stream) {
  if (!src || !dst) return MS_EINVAL;
  if (!n) return MS_OK;
  hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(n)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), src, dst, n);
  return hipGetLastError() == hipSuccess ? MS_OK : MS_EDEVICE;
}

ms_status ms_mlp_topk(const float* logits, int32_t batch, int32_t vocab,
                      int32_t k, int32_t exclude, int32_t* out_ids,
                      float* out_prob, void* stream) {
  if (!logits || !out_ids || batch < 1 || vocab < 1 || k < 1 || k > 16 ||
      k > vocab - (exclude >= 0 && exclude < vocab ? 1 : 0))
    return MS_EINVAL;
  hipLaunchKernelGGL(topk_kernel, dim3(batch), dim3(64), 0,
                     static_cast<hipStream_t>(stream), logits, vocab, k,
                     exclude, out_ids, out_prob);
  return hipGetLastError() == hipSuccess ? MS_OK : MS_EDEVICE;
}

}  // extern "C"

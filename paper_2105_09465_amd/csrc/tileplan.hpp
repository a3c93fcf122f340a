// Tile plan of the matrix-free kernel product: the points in a spatially
// coherent order, the bounding box of every row tile (64 points) and column
// chunk (32 points), and for every row tile the ascending list of chunks that
// can hold a non-zero kernel value in the chosen precision.
//
// A (row tile, chunk) pair is dropped only when the box gap g satisfies
// s2 g^2 >= threshold, with s2 = log2(e)/(2 l^2) the exp2 scale of the RBF
// kernel (Sec. 3.1, eq. "grbf"): then every exp tile entry of the pair is
// exactly zero in the form that evaluates it (below the smallest FP16
// subnormal after the 2^11 scale of the precision form, below the smallest
// FP32 subnormal in the FP32 form), so the product over the listed pairs
// equals the product over all pairs term for term.
#pragma once

#include <cstdint>

#include "common.hpp"

namespace gpl {

constexpr int kRowTile = 64;     // rows per wave (four 16-row MFMA tiles)
constexpr int kChunk = 32;       // source points per chunk
constexpr int kSegChunks = 32;   // chunks per work item that trigger one more item
constexpr int kMaxSeg = 8;       // work items per row tile
constexpr int kMaxPlanChunks = 65535;  // chunk indices are 16-bit

// Skip thresholds on s2 g^2 (exp2 arguments: 11 - s2 d^2 <= -25 leaves the FP16
// hi and lo parts zero; -s2 d^2 <= -152 underflows FP32 to zero; each with
// margin for the FP32 rounding of the box gap and of d^2).
constexpr float kSkipF16x3 = 36.f;
constexpr float kSkipFp32 = 152.f;

struct TilePlan {
  int n;     // points
  int nrt;   // row tiles = ceil(n / 64)
  int nch;   // chunks = 2 nrt
  int npad;  // 64 nrt
  const int* perm;  // sorted position -> caller index; nullptr = identity
  float *xs, *ys;   // [npad] points in sorted order, zero padded
  float4* cbox;     // [nch] (xmin, xmax, ymin, ymax); empty chunks have xmin = +inf
  int* count;       // [nrt] live chunks of each row tile
  int* nseg;        // [nrt] work items of each row tile, in [1, kMaxSeg]
  uint16_t* list;   // [nrt][nch] live chunks of each row tile, ascending
};

// Bytes of the plan buffers for n points (0 for n <= 0).
size_t plan_workspace(int n);
// Carve the plan buffers (nullptr fields when the carver overflows).
template <class C>
void plan_carve(C& cv, int n, TilePlan& p) {
  p.n = n;
  p.nrt = cdiv(n, kRowTile);
  p.nch = 2 * p.nrt;
  p.npad = p.nrt * kRowTile;
  p.perm = nullptr;
  int* perm = cv.template take<int>((size_t)p.npad);
  p.perm = perm;
  p.xs = cv.template take<float>((size_t)p.npad);
  p.ys = cv.template take<float>((size_t)p.npad);
  p.cbox = cv.template take<float4>((size_t)p.nch);
  p.count = cv.template take<int>((size_t)p.nrt);
  p.nseg = cv.template take<int>((size_t)p.nrt);
  p.list = cv.template take<uint16_t>((size_t)p.nrt * p.nch);
}

// Build the plan on `stream`. With `grid` the points are the fine grid of that
// grid in row-major order and are sorted along the Z-order curve of the fine
// grid; without it they keep the caller's order. `s2` is the exp2 scale,
// `threshold` one of kSkipF16x3 / kSkipFp32.
int plan_build(TilePlan& p, int n, const float* px, const float* py, const gpl_grid* grid, float s2, float threshold,
               hipStream_t stream);

// Device: Z-order rank of fine pixel (fx, fy) among the pixels of an m x m grid.
__device__ __forceinline__ int zorder_rank(int fx, int fy, int m) {
  int side = 1;
  while (side < m) side <<= 1;
  int rank = 0, x0 = 0, y0 = 0;
  for (int s = side >> 1; s >= 1; s >>= 1) {
    const int qx = fx >= x0 + s, qy = fy >= y0 + s;
    const int q = qx + 2 * qy;
    // valid pixels of the quadrants that precede q in Z-order
    for (int t = 0; t < q; ++t) {
      const int ax = x0 + (t & 1) * s, ay = y0 + (t >> 1) * s;
      const int wx = min(max(m - ax, 0), s), wy = min(max(m - ay, 0), s);
      rank += wx * wy;
    }
    x0 += qx * s;
    y0 += qy * s;
  }
  return rank;
}

}  // namespace gpl

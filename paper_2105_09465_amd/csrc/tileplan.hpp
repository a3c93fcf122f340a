// Tile plan of the matrix-free kernel product: the points sorted along a Hilbert
// curve of their own positions (the ray-traced source-plane points, so that the
// images of one source region share tiles), the bounding box of every 16-point subtile and 32-point
// chunk, and for every row tile (64 points, four subtiles) the ascending list of
// chunks that can hold a non-zero kernel value in the chosen precision, each
// with a mask of the subtiles that can.
//
// A (subtile, chunk) pair is dropped only when the box gap g satisfies
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
constexpr int kSubTile = 16;     // rows of one MFMA tile
constexpr int kChunk = 32;       // source points per chunk
constexpr int kSubsPerTile = kRowTile / kSubTile;
constexpr int kChunksPerTile = kRowTile / kChunk;
constexpr int kMaxPlanWaves = 3072;    // waves of one product launch (3 per SIMD)
constexpr int kMaxPlanChunks = 65535;  // chunk indices are 16-bit

// Skip thresholds on s2 g^2. Precision form: the exp2 argument 11 - s2 d^2 <= -25
// leaves the FP16 hi and lo parts exactly zero (margin for the FP32 rounding of
// the box gap and of d^2), so nothing is dropped. FP32 form: the same cutoff
// drops terms k_ij v_j with k_ij <= 2^-36 a^2, an error-bounded cutoff rather than
// an exact zero: per row the dropped terms sum to at most 2^-36 a^2 sum_j |v_j|
// (5.8e-7 a^2 max|v| at 40,000 points), and both forms evaluate the same pairs.
// -s2 d^2 <= -152 underflows FP32 itself to zero (kept for the adjoint's plan,
// whose own per-chunk cutoff is applied on top).
constexpr float kSkipF16x3 = 36.f;
constexpr float kSkipFp32 = 36.f;
constexpr float kSkipFp32Exact = 152.f;
// In the precision form a (subtile, chunk) pair with s2 g^2 >= kLoF16x3 has
// every kernel value k <= 2^-20, so the lo part of its exp tile (below 2^-10 k)
// is below 2^-30 per entry, under a 2^-20 share of the FP32 rounding of an
// entry of size one: such pairs multiply the hi part only.
constexpr float kLoF16x3 = 20.f;

// s2 g^2 < threshold for the gap g between two boxes (x0, x1, y0, y1) (NaN-free:
// an infinite box gives a zero gap, an empty one an infinite gap).
__device__ __forceinline__ bool boxes_live(const float4& a, const float4& q, float s2, float threshold) {
  const float gx = fmaxf(0.f, fmaxf(q.x - a.y, a.x - q.y));
  const float gy = fmaxf(0.f, fmaxf(q.z - a.w, a.z - q.w));
  return !(s2 * fmaf(gx, gx, gy * gy) >= threshold);
}

// List entries: chunk index in the low 16 bits, bit 16 + t set when subtile t of
// the row tile can see the chunk (entries with no such bit are not listed), bit
// 20 + t set when that pair also needs the lo part of the exp tile (the same
// bits as the first mask in the FP32 form).
__host__ __device__ inline int entry_chunk(uint32_t e) { return (int)(e & 0xffffu); }
__host__ __device__ inline unsigned entry_mask(uint32_t e) { return (e >> 16) & 0xfu; }
__host__ __device__ inline unsigned entry_lomask(uint32_t e) { return (e >> 20) & 0xfu; }

// The evaluated work is a sequence of units, the live (row tile, chunk) pairs in
// row-tile order (T units in all). A product launch of nw waves gives each wave
// a contiguous range of units; a wave writes one partial row block per row tile
// it touches, into consecutive slots starting at wslot[w]. The slots of one row
// tile are then consecutive too, in wave order, and are summed in that order.
//
// The ranges balance a cost estimate, not the unit count: a unit costs in
// proportion to its live subtiles plus a fixed part, and a row tile has a fixed
// cost of its own (row loads, the partial store). They are also sized for how
// the waves share a SIMD. Workgroups are dispatched in order, one per compute
// unit at a time, so the waves of the r-th group of wround = 4 x (compute
// units) waves sit as the r-th wave on their SIMDs, and the SIMD issues for its
// oldest wave first. With equal costs the first group ends early and the last
// one runs on alone at the rate of a single wave; costs in the ratio of
// kRoundWeight let the three waves of a SIMD end together.
struct TilePlan {
  int n;     // points
  int nrt;   // row tiles = ceil(n / 64)
  int nch;   // chunks = 2 nrt (kChunksPerTile nrt)
  int npad;  // 64 nrt
  int nw;    // waves of a product launch (multiple of 4)
  int wround;  // waves dispatched per round (4 per compute unit)
  const int* perm;  // [npad] sorted position -> caller index (-1 past n)
  const int* irank; // [npad] caller index -> sorted position (first n entries)
  float *xs, *ys;   // [npad] points in sorted order, zero padded
  // The same points for the precision form's product: scaled by sqrt(s2) and
  // taken relative to the scaled centre of their 64-point block, cen[j / 64]
  // (a multiple of 2^-12, 0 for a block without a finite box), so that
  // sqrt(s2) (p_i - p_j) = (xc_i + (cen_i - cen_j)) - xc_j with every term of
  // the size of the blocks, not of the coordinates.
  float *xc, *yc;   // [npad]
  float2* cen;      // [nrt]
  float4* cbox;     // [nch] (xmin, xmax, ymin, ymax); empty chunks have xmin = +inf
  float4* sbox;     // [kSubsPerTile nrt] the same for every 16-point subtile
  int* count;       // [nrt] live chunks of each row tile
  uint32_t* list;   // [nrt][nch] entries of the live chunks of each row tile, ascending
  int* unit_off;    // [nrt] first unit of each row tile (exclusive prefix of count)
  int* total;       // [1] T
  int* wrow;        // [nw] row tile of each wave's first unit (-1: no units)
  int* wslot;       // [nw + 1] first partial slot of each wave
  int2* rslot;      // [nrt] first partial slot of each row tile and their number
  int4* wdesc;      // [nw] per wave: first row tile, first slot, list range [kb, ke) in that row tile
  int* wrest;       // [nw] the wave's units in later row tiles
  int* wunit;       // [nw + 1] first unit of each wave (wunit[nw] = T)
  int* roww;        // [nrt] cost estimate of each row tile
  long long* rowwoff;  // [nrt] exclusive prefix of roww
  long long* wtot;     // [1] total cost
  // scratch of the sort that orders the points (used while the plan is built;
  // its Hilbert keys and extent live in xc, yc and cbox, written after the sort)
  int* sval;                // [npad] caller indices, ping-pong partner of perm
  int* shist;               // [kSortDigits nsb] digit counts per sort block, then their offsets
};

// Sort of the points: Hilbert index of 12 bits per axis over the square that
// holds every finite point, radix-sorted 8 bits a pass in blocks of 256 points.
constexpr int kHilbertBits = 12;
constexpr int kSortBlock = 256;
constexpr int kSortDigits = 256;
constexpr int kSortPasses = (2 * kHilbertBits + 7) / 8;
__host__ __device__ inline int sort_blocks(int n) { return (n + kSortBlock - 1) / kSortBlock; }

// Waves of a product launch for n points, and partial slots it may write.
__host__ __device__ inline int plan_waves(int n) {
  const int nrt = (n + kRowTile - 1) / kRowTile;
  const int w = nrt * 8 < kMaxPlanWaves ? nrt * 8 : kMaxPlanWaves;
  return (w + 3) / 4 * 4;
}
__host__ __device__ inline int plan_slots(int n) { return plan_waves(n) + (n + kRowTile - 1) / kRowTile; }

// Position of entry (column c, sorted point j) in a right-hand-side buffer of ncp
// columns: chunk-major, each chunk's columns of 32 consecutive points together,
// so that the 16 columns of a column block of one chunk are 1 KB (FP16) or 2 KB
// (FP32) of contiguous memory.
__host__ __device__ inline size_t rhs_at(int c, int j, int ncp) {
  return ((size_t)(j >> 5) * ncp + c) * kChunk + (j & (kChunk - 1));
}

// The precision form's last block of 16 columns, when it holds at most 8 of the
// nrhs columns, is packed: column c of it keeps both FP16 parts in the hi buffer,
// hi at column slot 16 b + 2 (c - 16 b) and lo in the slot after it (b the block),
// so that two MFMAs (hi and lo of the exp tile, each times [hi, lo] of the RHS)
// give the column's product instead of three; the lo buffer's block is unused.
__host__ __device__ inline bool last_block_packed(int nrhs) { return nrhs > 0 && nrhs - 16 * ((nrhs - 1) / 16) <= 8; }
__host__ __device__ inline int packed_block_start(int nrhs) { return 16 * ((nrhs - 1) / 16); }
// Column slot of the hi part of column c (the lo part: the same slot of the lo
// buffer, or the next slot of the hi buffer when c is in a packed block).
__host__ __device__ inline int hi_slot(int c, int nrhs) {
  const int b0 = packed_block_start(nrhs);
  return last_block_packed(nrhs) && c >= b0 ? b0 + 2 * (c - b0) : c;
}

// Bytes of the plan buffers for n points (0 for n <= 0).
size_t plan_workspace(int n);
// Carve the plan buffers (nullptr fields when the carver overflows).
template <class C>
void plan_carve(C& cv, int n, TilePlan& p) {
  p.n = n;
  p.nrt = cdiv(n, kRowTile);
  p.nch = kChunksPerTile * p.nrt;
  p.npad = p.nrt * kRowTile;
  p.nw = plan_waves(n);
  p.wround = 1024;
  p.perm = cv.template take<int>((size_t)p.npad);
  p.irank = cv.template take<int>((size_t)p.npad);
  p.xs = cv.template take<float>((size_t)p.npad);
  p.ys = cv.template take<float>((size_t)p.npad);
  p.xc = cv.template take<float>((size_t)p.npad);
  p.yc = cv.template take<float>((size_t)p.npad);
  p.cen = cv.template take<float2>((size_t)p.nrt);
  p.cbox = cv.template take<float4>((size_t)p.nch);
  p.sbox = cv.template take<float4>((size_t)p.nrt * kSubsPerTile);
  p.count = cv.template take<int>((size_t)p.nrt);
  p.list = cv.template take<uint32_t>((size_t)p.nrt * p.nch);
  p.unit_off = cv.template take<int>((size_t)p.nrt);
  p.total = cv.template take<int>(1);
  p.wrow = cv.template take<int>((size_t)p.nw);
  p.wslot = cv.template take<int>((size_t)p.nw + 1);
  p.rslot = cv.template take<int2>((size_t)p.nrt);
  p.wdesc = cv.template take<int4>((size_t)p.nw);
  p.wrest = cv.template take<int>((size_t)p.nw);
  p.wunit = cv.template take<int>((size_t)p.nw + 1);
  p.roww = cv.template take<int>((size_t)p.nrt);
  p.rowwoff = cv.template take<long long>((size_t)p.nrt);
  p.wtot = cv.template take<long long>(1);
  p.sval = cv.template take<int>((size_t)p.npad);
  p.shist = cv.template take<int>((size_t)kSortDigits * sort_blocks(n));
}

// Build the plan on `stream`. The points are sorted along the Hilbert curve of
// their positions (ties in caller order, so the plan depends only on the
// points). `grid` (nullable) is checked against n: with one, the points are its
// fine grid in row-major order, which is what irank is indexed by in the fused
// PSF adjoint. `s2` is the exp2 scale, `threshold` the skip threshold of the
// form and `lo_threshold` that of the lo masks (kLoF16x3 in the precision form;
// equal to `threshold` where the form has no lo part).
int plan_build(TilePlan& p, int n, const float* px, const float* py, const gpl_grid* grid, float s2, float threshold,
               float lo_threshold, hipStream_t stream);
// The first part of plan_build alone: the Hilbert sort (perm, irank, xs, ys)
// and the chunk and subtile boxes.
int plan_sort(TilePlan& p, int n, const float* px, const float* py, hipStream_t stream);

// Relative work of a wave in the first, second and later dispatch rounds.
constexpr int kRounds = 3;
constexpr int kRoundWeight[kRounds] = {16, 9, 4};
constexpr int kPlanWaves = 4;  // waves per workgroup of a product launch
constexpr int kXcds = 8;       // workgroup b of a launch runs on XCD b % kXcds

// Order of a launch's waves along the unit sequence. Workgroups are dispatched
// in order, wround / kPlanWaves per round, round-robin over the XCDs. Within
// each round the workgroups are permuted so that those an XCD takes hold one
// contiguous eighth of the round's range: neighbouring row tiles then read
// their right-hand-side chunks through one L2 instead of eight. The first
// multiple of kXcds workgroups of a round are permuted among themselves; the
// rest of a partial round keep their places. (One contiguous share of the whole
// sequence per XCD, the rounds alternating in it, fetched more than this from
// HBM.)
__host__ __device__ inline int plan_block(int b, int nw, int wround) {
  const int R = wround / kPlanWaves;
  const int r0 = b - b % R;
  const int m = min(R, nw / kPlanWaves - r0) & ~(kXcds - 1);
  const int i = b - r0;
  return i < m ? r0 + (i % kXcds) * (m / kXcds) + i / kXcds : b;
}

// Weight of waves [0, w): sum over rounds of the round's weight x its waves below
// w (the permutation of plan_block keeps every wave in its round).
__host__ __device__ inline long long wave_weight_below(int w, int wround) {
  long long c = 0;
  for (int k = 0; k < kRounds; ++k) {
    const int lo = k * wround;
    const int hi = k == kRounds - 1 ? w : min(w, (k + 1) * wround);
    if (hi > lo) c += (long long)kRoundWeight[k] * (hi - lo);
  }
  return c;
}

// Cost estimate of a unit (per live subtile, per subtile that also needs the lo
// part, and fixed) and of a row tile, in the ratio measured for the precision form.
constexpr int kCostSubtile = 3;
constexpr int kCostSubtileLo = 2;
constexpr int kCostUnit = 5;
constexpr int kCostRowTile = 36;
__host__ __device__ inline int unit_cost(uint32_t e) {
  return kCostSubtile * __builtin_popcount(entry_mask(e)) + kCostSubtileLo * __builtin_popcount(entry_lomask(e)) +
         kCostUnit;
}

}  // namespace gpl

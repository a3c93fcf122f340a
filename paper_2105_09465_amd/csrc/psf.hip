// Observation operator B = D o P (PSF on the fine grid, then local averaging to
// image pixels) and its adjoint B^T = P^T D^T (Sec. 2 and Sec. 3.3 footnote on a
// PSF as deterministic post-processing of the fluxes; Sec. 4.1 local averaging).
//
// Both are applied through the composite 1-D filter g of the PSF taps and the
// ss-point block sum (Taps::g): per axis, B maps fine index f to pixel I with
// weight g(f - ss I) / ss, and B^T maps pixel I back to f with the same weight,
// so B is a separable strided convolution with 2r + ss taps and B^T a polyphase
// one with at most ceil((2r + ss) / ss) taps per output. This is the same linear
// map as the PSF followed by the block mean; only the FP32 rounding order
// differs. One workgroup per (tile, column): the input window of the tile (fine
// values for B, pixel values for B^T) is staged in LDS, filtered along x into a
// second LDS buffer, then along y. The taps are a normalised 1-D Gaussian,
// computed on the host in FP64.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "internal.hpp"

namespace gpl {

constexpr int kFineTile = 32;  // fine-grid tile side
constexpr int kMaxWin = kFineTile + 2 * GPL_PSF_MAX_RADIUS;

// Row stride of the adjoint's x-convolved buffer: 40 = 8 (mod 32), so the 8 x 8
// pixel block a wave reads in the Z-order walk falls on distinct LDS banks.
constexpr int kAdjStride = 40;
constexpr int kOutPer = kFineTile * kFineTile / 256;  // output pixels per thread of a forward tile

// Dynamic LDS of the tiles (floats), sized for the PSF radius r and the
// supersampling ss of the launch.
__host__ __device__ inline int fwd_tile_dims(int r, int ss, int& TP, int& W) {
  TP = kFineTile / ss > 0 ? kFineTile / ss : 1;
  W = TP * ss + 2 * r;
  return W * W + W * (TP + 1) + 2 * r + ss;
}
__host__ __device__ inline int adj_tile_dims(int r, int ss, int& WC, int& K) {
  const int L = 2 * r + ss;
  WC = (kFineTile + 2 * r + ss - 2) / ss + 1;
  K = (L - 1) / ss + 1;
  return WC * WC + (WC + K - 1) * kAdjStride + ss + L;
}
__host__ __device__ inline size_t fwd_lds_bytes(int r, int ss) {
  int a, b;
  return sizeof(float) * (size_t)fwd_tile_dims(r, ss, a, b);
}
__host__ __device__ inline size_t adj_lds_bytes(int r, int ss) {
  int a, b;
  return sizeof(float) * (size_t)adj_tile_dims(r, ss, a, b);
}

// A W x W window (W <= kMaxWin) staged into LDS through registers: thread
// (lx, ly) of the 32 x 8 workgroup holds rows ly + 8k and columns lx + 32m, and
// every global load of the window is issued before the first LDS store, so the
// loads overlap instead of each waiting for the previous one.
constexpr int kWinRows = (kMaxWin + 7) / 8, kWinCols = (kMaxWin + 31) / 32;
static_assert(kWinRows * kWinCols <= 32, "one mask bit per window slot");
struct WinRegs {
  float v[kWinRows][kWinCols];
  unsigned ok;  // bit k * kWinCols + m: slot inside the window and the grid
};

__device__ __forceinline__ int clamp_idx(int v, int m) { return min(max(v, 0), m - 1); }

// at(wy, wx, ok) returns the value at window position (wy, wx) read from the
// nearest grid pixel, always at a valid address, and sets ok when the position
// lies inside the window and the grid. Slots that are not ok are stored as 0 in
// win_store: keeping the selection out of the load blocks lets all loads be in
// flight together.
template <class At>
__device__ __forceinline__ void win_load(WinRegs& R, int W, At&& at) {
  const int lx = threadIdx.x & 31, ly = threadIdx.x >> 5;
  R.ok = 0u;
#pragma unroll
  for (int k = 0; k < kWinRows; ++k)
#pragma unroll
    for (int m = 0; m < kWinCols; ++m)
      if (8 * k < W && 32 * m < W) {
        bool ok;
        R.v[k][m] = at(ly + 8 * k, lx + 32 * m, ok);
        R.ok |= (ok ? 1u : 0u) << (k * kWinCols + m);
      }
}

__device__ __forceinline__ void win_store(const WinRegs& R, int W, float* S) {
  const int lx = threadIdx.x & 31, ly = threadIdx.x >> 5;
#pragma unroll
  for (int k = 0; k < kWinRows; ++k)
#pragma unroll
    for (int m = 0; m < kWinCols; ++m)
      if (8 * k < W && 32 * m < W) {
        const int wy = ly + 8 * k, wx = lx + 32 * m;
        if (wy < W && wx < W) S[wy * W + wx] = (R.ok >> (k * kWinCols + m)) & 1u ? R.v[k][m] : 0.f;
      }
}

// g[t + r] = sum_{s < ss} w[s - t] / sum for t in [-r, ss - 1 + r], in FP64.
static void composite_taps(int ss, int r, const double* w, double sum, Taps& t) {
  t.L = 2 * r + ss;
  for (int k = 0; k < t.L; ++k) {
    const int tt = k - r;
    double a = 0.0;
    for (int s = 0; s < ss; ++s) {
      const int j = s - tt;
      if (j >= -r && j <= r) a += w[j + r];
    }
    t.g[k] = (float)(a / sum);
  }
}

int make_taps(const gpl_grid* g, const gpl_psf* psf, Taps& t) {
  GPL_REQUIRE(psf != nullptr, "psf is NULL");
  GPL_REQUIRE(psf->fwhm >= 0 && std::isfinite(psf->fwhm), "psf fwhm must be >= 0");
  GPL_REQUIRE(psf->radius >= 0 && psf->radius <= GPL_PSF_MAX_RADIUS, "psf radius must be in [0, %d]",
              GPL_PSF_MAX_RADIUS);
  GPL_REQUIRE(g->ss >= 1 && g->ss <= kFineTile, "ss=%d outside [1, %d]", g->ss, kFineTile);
  if (psf->fwhm == 0.0) {
    const double one[1] = {1.0};
    t.r = 0;
    t.w[0] = 1.f;
    composite_taps(g->ss, 0, one, 1.0, t);
    return GPL_OK;
  }
  const double h = g->pix_scale / g->ss;
  const double s = psf->fwhm / (2.0 * std::sqrt(2.0 * std::log(2.0)));
  int r = psf->radius > 0 ? psf->radius : (int)std::ceil(4.0 * s / h);
  GPL_REQUIRE(r <= GPL_PSF_MAX_RADIUS, "psf radius %d (fwhm %g, h %g) exceeds %d", r, psf->fwhm, h,
              GPL_PSF_MAX_RADIUS);
  double w[2 * GPL_PSF_MAX_RADIUS + 1], sum = 0.0;
  for (int k = -r; k <= r; ++k) {
    const double u = k * h / s;
    w[k + r] = std::exp(-0.5 * u * u);
    sum += w[k + r];
  }
  t.r = r;
  for (int k = 0; k < 2 * r + 1; ++k) t.w[k] = (float)(w[k] / sum);
  composite_taps(g->ss, r, w, sum, t);
  return GPL_OK;
}

// floor(v / ss) for 0 <= v < 2^15 and 1 <= ss <= 32, rss = 1 / ss in FP32:
// (v + 1/2) / ss stays at least 1/64 away from an integer, far more than the
// FP32 rounding of the product. Branch-free, so the loads it addresses are not
// split into separately waited blocks.
__device__ __forceinline__ int div_ss(int v, float rss) { return (int)(((float)v + 0.5f) * rss); }

// Floor and ceiling of a / b for b > 0 and any sign of a.
__device__ __forceinline__ int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
__device__ __forceinline__ int ceil_div(int a, int b) { return -floor_div(-a, b); }

// Forward y pass for this thread's NU pixels o = tid + 256 u (a pixel past the
// tile repeats the last one and is not used).
template <int NU>
__device__ __forceinline__ void forward_ypass(const float* S2, const float* tg, int L, int LS, int ss, int TP,
                                              float (&acc)[kOutPer]) {
  const float* col[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int o = min((int)threadIdx.x + u * 256, TP * TP - 1);
    const int oy = o / TP, ox = o - oy * TP;
    col[u] = S2 + ss * oy * LS + ox;
  }
#pragma unroll 2
  for (int k = 0; k < L; ++k) {
    const float w = tg[k];
#pragma unroll
    for (int u = 0; u < NU; ++u) acc[u] = fmaf(w, col[u][k * LS], acc[u]);
  }
}

// Forward: out[I] = alpha * (B in)[I] + beta * out[I] + gamma * extra[I];
// optional FP64 partial sums of dotv[I] * out[I] per (column, tile).
// `skip()` (uniform over the workgroup) is evaluated once the window loads are in
// flight; when it is true the workgroup leaves without writing anything.
template <class Skip>
__device__ __forceinline__ void psf_forward_body(Skip&& skip, int tile, int c, int n, int ss, const Taps& taps,
                                                 const float* __restrict__ in, int ld_in, float* __restrict__ out,
                                                 int ld_out, float alpha, float beta, const float* __restrict__ extra,
                                                 int ld_extra, float gamma, const float* __restrict__ dotv,
                                                 int ld_dotv, double* __restrict__ partial, int ntiles) {
  extern __shared__ float psf_lds[];
  __shared__ double red[4];
  const int M = n * ss, r = taps.r, L = taps.L;
  int TP, W;  // output pixels per tile side, window side
  fwd_tile_dims(r, ss, TP, W);
  const int F = TP * ss, LS = TP + 1;
  float* const S1 = psf_lds;           // [W][W] fine window
  float* const S2 = S1 + W * W;        // [W][LS] filtered along x
  float* const tg = S2 + W * LS;       // [L] composite taps
  const int tiles_x = (n + TP - 1) / TP;
  const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
  const int fy0 = ty * F, fx0 = tx * F;
  const float* src = in + (size_t)c * ld_in;
  // this thread's output pixels (at most kOutPer) and their operands, loaded
  // together with the window
  int I[kOutPer];
  float o_old[kOutPer], o_ext[kOutPer], o_dot[kOutPer];
#pragma unroll
  for (int u = 0; u < kOutPer; ++u) {
    const int o = threadIdx.x + u * 256;
    const int oy = o / TP, ox = o - oy * TP;
    const int Iy = ty * TP + oy, Ix = tx * TP + ox;
    I[u] = (o < TP * TP && Iy < n && Ix < n) ? Iy * n + Ix : -1;
  }
  // unconditional loads at valid addresses (pixel 0 for a pixel past the grid),
  // all issued after the indices are known; the values are only looked at where
  // they are used (a select or a branch here would wait for them before the
  // window loads are issued). An absent or unused operand (out when beta is 0)
  // reads the same pixels of another, so it adds no memory traffic.
  {
    const float* pe = extra ? extra + (size_t)c * ld_extra : src;
    const float* po = beta != 0.f ? out + (size_t)c * ld_out : pe;
    const float* pd = dotv ? dotv + (size_t)c * ld_dotv : pe;
#pragma unroll
    for (int u = 0; u < kOutPer; ++u) {
      const int Ic = max(I[u], 0);
      o_old[u] = po[Ic];
      o_ext[u] = pe[Ic];
      o_dot[u] = pd[Ic];
    }
  }
  {
    WinRegs R;
    win_load(R, W, [&](int wy, int wx, bool& ok) {
      const int fy = fy0 - r + wy, fx = fx0 - r + wx;
      ok = wy < W && wx < W && fy >= 0 && fy < M && fx >= 0 && fx < M;
      return src[(size_t)clamp_idx(fy, M) * M + clamp_idx(fx, M)];
    });
    if (skip()) return;
    if ((int)threadIdx.x < L) tg[threadIdx.x] = taps.g[threadIdx.x];
    win_store(R, W, S1);
  }
  __syncthreads();
  // x: S2[wy][ox] = sum_t g(t) S1[wy][ss ox + t + r], window rows wy < W, pixel
  // columns ox < TP; three rows at a time share each tap
  for (int o0 = threadIdx.x; o0 < W * TP; o0 += 3 * 256) {
    int at[3];
    float acc[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int o = min(o0 + 256 * i, W * TP - 1);
      const int wy = o / TP, ox = o - wy * TP;
      at[i] = wy * W + ss * ox;
    }
#pragma unroll 2
    for (int k = 0; k < L; ++k) {
      const float w = tg[k];
#pragma unroll
      for (int i = 0; i < 3; ++i) acc[i] = fmaf(w, S1[at[i] + k], acc[i]);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int o = o0 + 256 * i;
      if (o < W * TP) {
        const int wy = o / TP, ox = o - wy * TP;
        S2[wy * LS + ox] = acc[i];
      }
    }
  }
  __syncthreads();
  // y: pixel (oy, ox) = sum_t g(t) S2[ss oy + t + r][ox] / ss^2
  const float inv_ss2 = 1.f / (float)(ss * ss);
  float acc[kOutPer] = {};
  if (TP * TP > 256)
    forward_ypass<kOutPer>(S2, tg, L, LS, ss, TP, acc);
  else
    forward_ypass<1>(S2, tg, L, LS, ss, TP, acc);
  double dot = 0.0;
#pragma unroll
  for (int u = 0; u < kOutPer; ++u) {
    if (I[u] < 0) continue;
    float res = alpha * (acc[u] * inv_ss2);
    if (beta != 0.f) res += beta * o_old[u];
    if (extra) res += gamma * o_ext[u];
    out[(size_t)c * ld_out + I[u]] = res;
    if (dotv) dot += (double)o_dot[u] * (double)res;
  }
  if (partial) {
    const double s = block_sum_double(dot, red);
    if (threadIdx.x == 0) partial[(size_t)c * ntiles + tile] = s;
  }
}

__global__ __launch_bounds__(256) void psf_forward_kernel(int n, int ss, Taps taps, const float* __restrict__ in,
                                                          int ld_in, float* __restrict__ out, int ld_out,
                                                          float alpha, float beta, const float* __restrict__ extra,
                                                          int ld_extra, float gamma, const float* __restrict__ dotv,
                                                          int ld_dotv, double* __restrict__ partial, int ntiles,
                                                          CgGate gate) {
  psf_forward_body([&] { return gate.skip(blockIdx.y); }, blockIdx.x, blockIdx.y, n, ss, taps, in, ld_in, out, ld_out, alpha, beta, extra, ld_extra, gamma,
                   dotv, ld_dotv, partial, ntiles);
}

// Adjoint on one fine tile: v = (P^T D^T in)(fy, fx) for every fine point of the
// tile. Thread t takes the points u = 0..3 of the tile's walk (position t + 256 u:
// Z-order within the tile when ZWALK, else row-major); fetch(u, fy, fx) runs for
// each while the window loads are in flight (coordinates clamped into the grid)
// and store(fy, fx, v, u) at the end for the points inside the grid. P^T is the
// correlation with the taps: (P^T g)(y, x) = sum_{a,b} w_a w_b g(y + a, x + b).
template <bool ZWALK, class Skip, class Pre, class Fetch, class Store>
__device__ __forceinline__ void psf_adjoint_tile(Skip&& skip, int tile, int c, int n, int ss, const Taps& taps,
                                                 const float* __restrict__ in, int ld_in, Pre&& pre, Fetch&& fetch,
                                                 Store&& store) {
  extern __shared__ float psf_lds[];
  const int M = n * ss, r = taps.r, L = taps.L;
  int WC, K;  // window side in pixels; pixels that reach one fine point along an axis
  adj_tile_dims(r, ss, WC, K);
  static_assert(kFineTile == 32, "the Z-order decode below takes 5 bits per axis");
  const int F = kFineTile, LS = kAdjStride;
  float* const S1 = psf_lds;                 // [WC][WC] pixel window
  float* const S2 = S1 + WC * WC;            // [WC + K - 1][LS] filtered along x, zero rows at the end
  float* const tz = S2 + (WC + K - 1) * LS;  // [ss + L]: ss zeros, then g
  const int tiles_x = (M + F - 1) / F;
  const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
  const int fy0 = ty * F, fx0 = tx * F;
  // pixels whose composite filter reaches the tile: from ceil((f0 - ss + 1 - r) / ss) on, WC of them
  const int cy0 = ceil_div(fy0 - ss + 1 - r, ss), cx0 = ceil_div(fx0 - ss + 1 - r, ss);
  const float* src = in + (size_t)c * ld_in;
  const float inv_ss2 = 1.f / (float)(ss * ss);
  const int lx = threadIdx.x & 31, ly = threadIdx.x >> 5;  // 32 x 8 threads
  // the thread's points: position o = tid + 256 u of the walk
  constexpr int kPer = kFineTile * kFineTile / 256;
  int px[kPer], py[kPer], b0[kPer];
  const float* col[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int o = threadIdx.x + u * 256;
    int x = 0, y = 0;
    if (ZWALK) {
#pragma unroll
      for (int bit = 0; bit < 5; ++bit) {
        x |= ((o >> (2 * bit)) & 1) << bit;
        y |= ((o >> (2 * bit + 1)) & 1) << bit;
      }
    } else {
      y = o >> 5;
      x = o & 31;
    }
    px[u] = x;
    py[u] = y;
    const int fy = fy0 + y;
    const int ilo = ceil_div(fy - ss + 1 - r, ss) - cy0;
    b0[u] = ss + (fy - ss * (cy0 + ilo)) + r;
    col[u] = S2 + ilo * LS + x;
  }
  {
    WinRegs R;
    win_load(R, WC, [&](int wy, int wx, bool& ok) {
      const int iy = cy0 + wy, ix = cx0 + wx;
      ok = wy < WC && wx < WC && iy >= 0 && iy < n && ix >= 0 && ix < n;
      return src[(size_t)clamp_idx(iy, n) * n + clamp_idx(ix, n)];
    });
    if (skip()) return;
    if ((int)threadIdx.x < ss + L) tz[threadIdx.x] = (int)threadIdx.x < ss ? 0.f : taps.g[threadIdx.x - ss];
    for (int i = threadIdx.x; i < (K - 1) * LS; i += 256) S2[WC * LS + i] = 0.f;
    pre();  // runs while the window loads are in flight
#pragma unroll
    for (int u = 0; u < kPer; ++u) fetch(u, min(fy0 + py[u], M - 1), min(fx0 + px[u], M - 1));
    win_store(R, WC, S1);
  }
  __syncthreads();
  // x: S2[wy][x] = sum_k g(t0 - ss k) S1[wy][jlo + k], the pixels jlo.. that reach
  // fine column fx0 + x (weights past the last one are the zeros in front of g)
  {
    const int fx = fx0 + lx;
    const int jlo = ceil_div(fx - ss + 1 - r, ss) - cx0;
    const int b0 = ss + (fx - ss * (cx0 + jlo)) + r;  // tz index of k = 0
    const int nk = (WC + 7) / 8;
#pragma unroll 1
    for (int k0 = 0; k0 < nk; k0 += 3) {
      int wy[3];
      float acc[3] = {0.f, 0.f, 0.f};
#pragma unroll
      for (int i = 0; i < 3; ++i) wy[i] = min(ly + 8 * (k0 + i), WC - 1);
#pragma unroll 2
      for (int k = 0; k < K; ++k) {
        const float w = tz[b0 - ss * k];
        const int j = min(jlo + k, WC - 1);
#pragma unroll
        for (int i = 0; i < 3; ++i) acc[i] = fmaf(w, S1[wy[i] * WC + j], acc[i]);
      }
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const int row = ly + 8 * (k0 + i);
        if (row < WC) S2[row * LS + lx] = acc[i];
      }
    }
  }
  __syncthreads();
  // y, for the points of the walk, four chains per thread
  float v[kPer] = {};
#pragma unroll 2
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) v[u] = fmaf(tz[b0[u] - ss * k], col[u][k * LS], v[u]);
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int fy = fy0 + py[u], fx = fx0 + px[u];
    if (fy < M && fx < M) store(fy, fx, v[u] * inv_ss2, u);
  }
}

// out (fine, row-major) = alpha * B^T in + beta * out.
template <class Skip>
__device__ __forceinline__ void psf_adjoint_body(Skip&& skip, int tile, int c, int n, int ss, const Taps& taps,
                                                 const float* __restrict__ in, int ld_in, float* __restrict__ out,
                                                 int ld_out, float alpha, float beta) {
  const int M = n * ss;
  psf_adjoint_tile<false>(skip, tile, c, n, ss, taps, in, ld_in, [] {}, [](int, int, int) {},
                          [&](int fy, int fx, float v, int) {
    const size_t o_idx = (size_t)c * ld_out + (size_t)fy * M + fx;
    float res = alpha * v;
    if (beta != 0.f) res += beta * out[o_idx];
    out[o_idx] = res;
  });
}

// B^T P written straight into the RHS buffers of the product: fine
// point (fx, fy) goes to its sorted position in the product's plan (irank,
// loaded while the window loads are in flight); the precision form scales column c by
// 2^e_c, chosen from the bound max |B^T P| <= max |P| / ss^2 (nonnegative taps
// summing to one) so that the largest entry stays below 2^14, and splits it
// into FP16 hi (nearest) and lo.
template <class Skip>
__device__ __forceinline__ void psf_adjoint_rhs_body(Skip&& skip, int tile, int c, int n, int ss, const Taps& taps,
                                                     const float* __restrict__ in, int ld_in, const RhsOut& o) {
  __shared__ float red[4];
  __shared__ float s_scale;
  const int M = n * ss;
  int jr[kFineTile * kFineTile / 256];
  const bool f16 = o.prec == GPL_PREC_F16X3;
  // column scale, folded while the tile's window loads are in flight (the tile
  // synchronises the workgroup before its first use of s_scale)
  auto fold_scale = [&] {
    if (!f16) return;
    float m = 0.f;
    for (int k = threadIdx.x; k < o.npart; k += blockDim.x) m = fmaxf(m, __uint_as_float(o.pmax[c * o.npart + k]));
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      const float mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3])) / (float)(ss * ss);
      int e = 0;
      // bound * 2^e in [2^13, 2^14), e capped so that 2^e stays a finite float
      if (mx > 0.f && isfinite(mx)) e = min(14 - ilogbf(mx) - 1, 126);
      s_scale = ldexpf(1.f, e);
      if (tile == 0) o.inv_scale[c] = ldexpf(1.f, -e) / 2048.f;  // with the 2^11 of the exp tile
    }
  };
  // one instantiation of the tile (its LDS buffers) for both forms
  auto fetch = [&](int u, int fy, int fx) { jr[u] = o.irank[fy * M + fx]; };
  // FP16 parts of column c: hi at slot hs of Vh, lo at the same slot of Vl or,
  // in a packed last block, at the next slot of Vh
  const int hs = hi_slot(c, o.nrhs);
  const bool packed = last_block_packed(o.nrhs) && c >= packed_block_start(o.nrhs);
  psf_adjoint_tile<true>(skip, tile, c, n, ss, taps, in, ld_in, fold_scale, fetch, [&](int, int, float v, int u) {
    const float scale = f16 ? s_scale : 1.f;
    if (f16) {
      const size_t j = rhs_at(hs, jr[u], o.ncp);
      const float sv = v * scale;
      const _Float16 h = (_Float16)sv;
      const _Float16 l = (_Float16)(sv - (float)h);
      o.Vh[j] = h;
      if (packed) o.Vh[j + kChunk] = l;  // slot hs + 1 of the same chunk
      else o.Vl[j] = l;
    } else {
      o.Vp[rhs_at(c, jr[u], o.ncp)] = v;
    }
  });
}

__global__ __launch_bounds__(256) void psf_adjoint_rhs_kernel(int n, int ss, Taps taps, const float* __restrict__ in,
                                                              int ld_in, RhsOut o, CgGate gate) {
  psf_adjoint_rhs_body([&] { return gate.skip(blockIdx.y); }, blockIdx.x, blockIdx.y, n, ss, taps, in, ld_in, o);
}

__global__ __launch_bounds__(256) void psf_adjoint_kernel(int n, int ss, Taps taps, const float* __restrict__ in,
                                                          int ld_in, float* __restrict__ out, int ld_out,
                                                          float alpha, float beta, CgGate gate) {
  psf_adjoint_body([&] { return gate.skip(blockIdx.y); }, blockIdx.x, blockIdx.y, n, ss, taps, in, ld_in, out, ld_out,
                   alpha, beta);
}

// ---- grouped launches (serving): workgroup b of slot s handles (tile, column) =
// (local % tiles, local / tiles), local = b - off[s].

__global__ __launch_bounds__(256) void psf_adjoint_grouped_kernel(SlotBatch B, int p) {
  const int s = B.find(blockIdx.x);
  const ServeSlotDev& S = *B.slot[s];
  const int local = blockIdx.x - B.off[s];
  const int tile = local % S.ntiles_adj, c = local / S.ntiles_adj;
  const RhsOut o{S.prec, S.nrhs, S.ncp, S.Vh, S.Vl, S.Vp, S.inv_scale, S.pmax, S.nb_upd, S.plan.irank};
  psf_adjoint_rhs_body([&] { return S.n_active[p] == 0 || S.st[p][c].active == 0; }, tile, c, S.n, S.ss, S.taps, S.P, S.ldv, o);
}

__global__ __launch_bounds__(256) void psf_forward_grouped_kernel(SlotBatch B, int p) {
  const int s = B.find(blockIdx.x);
  const ServeSlotDev& S = *B.slot[s];
  const int local = blockIdx.x - B.off[s];
  const int tile = local % S.ntiles_fwd, c = local / S.ntiles_fwd;
  psf_forward_body([&] { return S.n_active[p] == 0 || S.st[p][c].active == 0; }, tile, c, S.n, S.ss, S.taps, S.T2, S.ldf, S.AP, S.ldv, 1.f, 0.f, S.P, S.ldv, S.sigma2, S.P, S.ldv,
                   S.pap_part, S.ntiles_fwd);
}

int psf_adjoint_tiles(int n, int ss) {
  const int M = n * ss, t = (M + kFineTile - 1) / kFineTile;
  return t * t;
}

static int grouped_launch(void (*kern)(SlotBatch, int), const ServeSlotDev* const* hslots,
                          const ServeSlotDev* const* dslots, int nslots, int p, int (*tiles_of)(const ServeSlotDev&),
                          size_t (*lds_of)(int, int), hipStream_t stream) {
  SlotBatch B;
  B.nslots = nslots;
  B.off[0] = 0;
  size_t lds = 0;
  for (int s = 0; s < nslots; ++s) {
    B.slot[s] = dslots[s];
    B.off[s + 1] = B.off[s] + tiles_of(*hslots[s]);
    lds = std::max(lds, lds_of(hslots[s]->taps.r, hslots[s]->ss));
  }
  if (B.off[nslots] == 0) return GPL_OK;
  hipLaunchKernelGGL(kern, dim3(B.off[nslots]), dim3(256), lds, stream, B, p);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

int psf_adjoint_grouped(const ServeSlotDev* const* hslots, const ServeSlotDev* const* dslots, int nslots, int p,
                        hipStream_t stream) {
  return grouped_launch(psf_adjoint_grouped_kernel, hslots, dslots, nslots, p,
                        [](const ServeSlotDev& S) { return S.ntiles_adj * S.nrhs; }, adj_lds_bytes, stream);
}

int psf_forward_grouped(const ServeSlotDev* const* hslots, const ServeSlotDev* const* dslots, int nslots, int p,
                        hipStream_t stream) {
  return grouped_launch(psf_forward_grouped_kernel, hslots, dslots, nslots, p,
                        [](const ServeSlotDev& S) { return S.ntiles_fwd * S.nrhs; }, fwd_lds_bytes, stream);
}

// Grid limits of the PSF tiles: ss <= kFineTile and a fine side below 2^15 (the
// range of the branch-free division by ss).
static int check_psf_grid(int n, int ss) {
  GPL_REQUIRE(ss >= 1 && ss <= kFineTile, "ss=%d outside [1, %d]", ss, kFineTile);
  GPL_REQUIRE(n >= 1 && (long)n * ss < 32768, "fine grid side %ld exceeds 32767", (long)n * ss);
  return GPL_OK;
}

int psf_forward_tiles(int n, int ss) {
  const int TP = kFineTile / ss > 0 ? kFineTile / ss : 1;
  const int t = (n + TP - 1) / TP;
  return t * t;
}

int psf_forward_launch(int n, int ss, const Taps& taps, int nrhs, const float* in, int ld_in, float* out, int ld_out,
                       float alpha, float beta, const float* extra, int ld_extra, float gamma, const float* dotv,
                       int ld_dotv, double* partial, CgGate gate, hipStream_t stream) {
  GPL_TRY(check_psf_grid(n, ss));
  const int ntiles = psf_forward_tiles(n, ss);
  hipLaunchKernelGGL(psf_forward_kernel, dim3(ntiles, nrhs), dim3(256), fwd_lds_bytes(taps.r, ss), stream, n, ss, taps,
                     in, ld_in, out,
                     ld_out, alpha, beta, extra, ld_extra, gamma, dotv, ld_dotv, partial, ntiles, gate);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

int psf_adjoint_rhs_launch(int n, int ss, const Taps& taps, int nrhs, const float* P, int ldp, const RhsOut& out,
                           CgGate gate, hipStream_t stream) {
  GPL_TRY(check_psf_grid(n, ss));
  const int M = n * ss, t = (M + kFineTile - 1) / kFineTile;
  hipLaunchKernelGGL(psf_adjoint_rhs_kernel, dim3(t * t, nrhs), dim3(256), adj_lds_bytes(taps.r, ss), stream, n, ss,
                     taps, P, ldp, out, gate);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

int psf_adjoint_launch(int n, int ss, const Taps& taps, int nrhs, const float* in, int ld_in, float* out, int ld_out,
                       float alpha, float beta, CgGate gate, hipStream_t stream) {
  GPL_TRY(check_psf_grid(n, ss));
  const int M = n * ss, t = (M + kFineTile - 1) / kFineTile;
  hipLaunchKernelGGL(psf_adjoint_kernel, dim3(t * t, nrhs), dim3(256), adj_lds_bytes(taps.r, ss), stream, n, ss, taps,
                     in, ld_in, out, ld_out,
                     alpha, beta, gate);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

}  // namespace gpl

using namespace gpl;

extern "C" int gpl_psf_conv(const gpl_grid* grid, const gpl_psf* psf, int nrhs, const float* in, int ld_in,
                            float* out, int ld_out, float alpha, float beta, int adjoint, hipStream_t stream) {
  GPL_REQUIRE(grid != nullptr && grid->n >= 1 && grid->ss >= 1 && grid->pix_scale > 0, "bad grid");
  GPL_REQUIRE(nrhs >= 0 && nrhs <= 65535, "nrhs=%d must be in [0, 65535]", nrhs);
  if (nrhs == 0) return GPL_OK;
  GPL_REQUIRE(in && out && in != out, "in/out NULL or aliased");
  const int N = grid->n * grid->ss * grid->n * grid->ss, npix = grid->n * grid->n;
  Taps taps;
  GPL_TRY(make_taps(grid, psf, taps));
  if (adjoint == 0) {
    GPL_REQUIRE(ld_in >= N && ld_out >= npix, "ld_in=%d (>= %d) / ld_out=%d (>= %d)", ld_in, N, ld_out, npix);
    return psf_forward_launch(grid->n, grid->ss, taps, nrhs, in, ld_in, out, ld_out, alpha, beta, nullptr, 0, 0.f,
                              nullptr, 0, nullptr, CgGate{}, stream);
  }
  GPL_REQUIRE(ld_in >= npix && ld_out >= N, "ld_in=%d (>= %d) / ld_out=%d (>= %d)", ld_in, npix, ld_out, N);
  return psf_adjoint_launch(grid->n, grid->ss, taps, nrhs, in, ld_in, out, ld_out, alpha, beta, CgGate{}, stream);
}

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
constexpr int kOutPer = kFineTile * kFineTile / 256;  // output pixels per thread of a forward tile, at most
// Output pixels per thread of a forward tile: (kFineTile / ss)^2 over 256 threads.
__host__ __device__ inline int fwd_pixels_per_thread(int ss) { return ss == 1 ? kOutPer : 1; }
static_assert(kFineTile * kFineTile / 4 <= 256, "a tile with ss >= 2 has at most 256 output pixels");

// Dynamic LDS of the tiles (floats), sized for the PSF radius r and the
// supersampling ss of the launch.
// Forward: the composite taps (padded to a multiple of 4), the W x W fine window
// with rows of W rounded up to 4 floats, and the x-filtered window stored
// transposed, [TP][LT] with an odd row stride.
__host__ __device__ inline int fwd_tile_dims(int r, int ss, int& TP, int& W, int& LT) {
  TP = kFineTile / ss > 0 ? kFineTile / ss : 1;
  W = TP * ss + 2 * r;
  LT = W | 1;
  return (2 * r + ss + 3) / 4 * 4 + W * ((W + 3) / 4 * 4) + TP * LT;
}
// Adjoint: the taps by phase [ss][K4], the WC x WC pixel window with WCP = WC + 8
// floats a row (the last 8 zero) and the x-filtered rows [WC + K4 - 1][kAdjStride]
// (the last K4 - 1 zero). K = ceil(L / ss) pixels reach a fine point along an
// axis, K4 is K rounded up to a multiple of 4.
__host__ __device__ inline int adj_tile_dims(int r, int ss, int& WC, int& K4, int& WCP) {
  const int L = 2 * r + ss;
  WC = (kFineTile + 2 * r + ss - 2) / ss + 1;
  K4 = ((L - 1) / ss + 4) / 4 * 4;
  WCP = WC + 8;
  return ss * K4 + WC * WCP + (WC + K4 - 1) * kAdjStride;
}
__host__ __device__ inline size_t fwd_lds_bytes(int r, int ss) {
  int a, b, c;
  return sizeof(float) * (size_t)fwd_tile_dims(r, ss, a, b, c);
}
__host__ __device__ inline size_t adj_lds_bytes(int r, int ss) {
  int a, b, c;
  return sizeof(float) * (size_t)adj_tile_dims(r, ss, a, b, c);
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

// Window values are read from the nearest grid pixel, always at a valid
// address; a slot's ok bit is set when its position lies inside the window and
// the grid, and win_store stores the slots that are not ok as 0: keeping the
// selection out of the load blocks lets all loads be in flight together. The
// address and the in-grid test split into a row part row(wy, ok) (an element
// offset from src) and a column part col(wx, ok), so that each slot costs one
// address add; ok of a slot = ok of its row and of its column.
template <class Row, class Col>
__device__ __forceinline__ void win_load_sep(WinRegs& R, int W, const float* __restrict__ src, Row&& row, Col&& col) {
  const int lx = threadIdx.x & 31, ly = threadIdx.x >> 5;
  int coff[kWinCols];
  unsigned cok = 0u;
#pragma unroll
  for (int m = 0; m < kWinCols; ++m) {
    bool ok = false;
    coff[m] = 32 * m < W ? col(lx + 32 * m, ok) : 0;
    cok |= (ok ? 1u : 0u) << m;
  }
  R.ok = 0u;
#pragma unroll
  for (int k = 0; k < kWinRows; ++k)
    if (8 * k < W) {
      bool rok;
      const float* p = src + row(ly + 8 * k, rok);
#pragma unroll
      for (int m = 0; m < kWinCols; ++m)
        if (32 * m < W) {
          R.v[k][m] = p[coff[m]];
          R.ok |= (rok && ((cok >> m) & 1u) ? 1u : 0u) << (k * kWinCols + m);
        }
    }
}

// Row wy of the window goes to S + wy * stride.
__device__ __forceinline__ void win_store(const WinRegs& R, int W, float* S, int stride) {
  const int lx = threadIdx.x & 31, ly = threadIdx.x >> 5;
#pragma unroll
  for (int k = 0; k < kWinRows; ++k)
#pragma unroll
    for (int m = 0; m < kWinCols; ++m)
      if (8 * k < W && 32 * m < W) {
        const int wy = ly + 8 * k, wx = lx + 32 * m;
        if (wy < W && wx < W) S[wy * stride + wx] = (R.ok >> (k * kWinCols + m)) & 1u ? R.v[k][m] : 0.f;
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

// floor(v / d) for 0 <= v < 2^16 and 1 <= d <= 32, rd = 1 / d in FP32:
// (v + 1/2) / d stays at least 1/64 away from an integer, more than the FP32
// rounding of the product and of rd (together below 2^-7). Branch-free, so the
// loads it addresses are not split into separately waited blocks.
__device__ __forceinline__ int div_ss(int v, float rd) { return (int)(((float)v + 0.5f) * rd); }

// Forward y pass for this thread's NU pixels o = tid + 256 u (a pixel past the
// tile repeats the last one and is not used), from the transposed x-filtered
// window S2T[ox][wy]: the taps of one pixel are consecutive, so four of them
// are read with one base address.
template <int NU>
__device__ __forceinline__ void forward_ypass(const float* S2T, const float* tg, int L, int LT, int ss, int TP,
                                              float rTP, float (&acc)[NU]) {
  int base[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int o = min((int)threadIdx.x + u * 256, TP * TP - 1);
    const int oy = div_ss(o, rTP), ox = o - oy * TP;
    base[u] = ox * LT + ss * oy;
  }
  int k = 0;
#pragma unroll 1
  for (; k + 4 <= L; k += 4) {
    const float4 w = *reinterpret_cast<const float4*>(tg + k);
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const float* q = S2T + base[u] + k;
      acc[u] = fmaf(w.x, q[0], acc[u]);
      acc[u] = fmaf(w.y, q[1], acc[u]);
      acc[u] = fmaf(w.z, q[2], acc[u]);
      acc[u] = fmaf(w.w, q[3], acc[u]);
    }
  }
  for (; k < L; ++k) {
    const float w = tg[k];
#pragma unroll
    for (int u = 0; u < NU; ++u) acc[u] = fmaf(w, S2T[base[u] + k], acc[u]);
  }
}

// Forward: out[I] = alpha * (B in)[I] + beta * out[I] + gamma * extra[I];
// optional FP64 partial sums of dotv[I] * out[I] per (column, tile).
// `skip()` (uniform over the workgroup) is evaluated once the window loads are in
// flight; when it is true the workgroup leaves without writing anything. NU:
// output pixels per thread, fwd_pixels_per_thread(ss).
template <int NU, class Skip>
__device__ __forceinline__ void psf_forward_body(Skip&& skip, int tile, int c, int n, int ss, const Taps& taps,
                                                 const float* __restrict__ in, int ld_in, float* __restrict__ out,
                                                 int ld_out, float alpha, float beta, const float* __restrict__ extra,
                                                 int ld_extra, float gamma, const float* __restrict__ dotv,
                                                 int ld_dotv, double* __restrict__ partial, int ntiles) {
  extern __shared__ __align__(16) float psf_lds[];
  __shared__ double red[4];
  const int M = n * ss, r = taps.r, L = taps.L;
  int TP, W, LT;  // output pixels per tile side, window side, row stride of S2T
  fwd_tile_dims(r, ss, TP, W, LT);
  const int F = TP * ss;
  const float rTP = 1.f / (float)TP;
  float* const tg = psf_lds;                    // [L, padded to 4] composite taps
  const int W4 = (W + 3) / 4 * 4;               // row stride of S1
  float* const S1 = tg + (L + 3) / 4 * 4;       // [W][W4] fine window
  float* const S2T = S1 + W * W4;               // [TP][LT] filtered along x, transposed
  const int tiles_x = (n + TP - 1) / TP;
  const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
  const int fy0 = ty * F, fx0 = tx * F;
  const float* src = in + (size_t)c * ld_in;
  // this thread's output pixels and their operands, loaded together with the
  // window
  int I[NU];
  float o_old[NU], o_ext[NU], o_dot[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int o = threadIdx.x + u * 256;
    const int oy = div_ss(o, rTP), ox = o - oy * TP;
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
    for (int u = 0; u < NU; ++u) {
      const int Ic = max(I[u], 0);
      o_old[u] = po[Ic];
      o_ext[u] = pe[Ic];
      o_dot[u] = pd[Ic];
    }
  }
  // A window inside the grid, W4 columns included, whose rows of W4 floats take
  // at most four float4 loads a thread: staged by float4 (no clamps or masks).
  // Any other window: by single floats with clamped addresses and masks.
  const int wq = W4 >> 2, wtot = W * wq;
  if (fy0 - r >= 0 && fy0 - r + W <= M && fx0 - r >= 0 && fx0 - r + W4 <= M && wtot <= 4 * 256) {
    typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
    const float* base = src + (size_t)(fy0 - r) * M + (fx0 - r);
    const float rq = 1.f / (float)wq;
    f4u v[4];
    int li[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (u * 256 < wtot) {
        const int i = min((int)threadIdx.x + u * 256, wtot - 1);
        const int row = div_ss(i, rq), q = i - row * wq;
        v[u] = *reinterpret_cast<const f4u*>(base + (size_t)row * M + 4 * q);
        li[u] = row * W4 + 4 * q;
      }
    if (skip()) return;
    if ((int)threadIdx.x < (L + 3) / 4 * 4) tg[threadIdx.x] = (int)threadIdx.x < L ? taps.g[threadIdx.x] : 0.f;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (u * 256 < wtot) *reinterpret_cast<float4*>(S1 + li[u]) = float4{v[u][0], v[u][1], v[u][2], v[u][3]};
  } else {
    WinRegs R;
    win_load_sep(
        R, W, src,
        [&](int wy, bool& ok) {
          const int fy = fy0 - r + wy;
          ok = wy < W && fy >= 0 && fy < M;
          return clamp_idx(fy, M) * M;
        },
        [&](int wx, bool& ok) {
          const int fx = fx0 - r + wx;
          ok = wx < W && fx >= 0 && fx < M;
          return clamp_idx(fx, M);
        });
    if (skip()) return;
    if ((int)threadIdx.x < (L + 3) / 4 * 4) tg[threadIdx.x] = (int)threadIdx.x < L ? taps.g[threadIdx.x] : 0.f;
    win_store(R, W, S1, W4);
  }
  __syncthreads();
  // x: S2T[ox][wy] = sum_t g(t) S1[wy][ss ox + t], window rows wy < W, pixel
  // columns ox < TP; three outputs per thread share each group of four taps
  for (int o0 = threadIdx.x; o0 < W * TP; o0 += 3 * 256) {
    int at[3];
    float acc[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int o = min(o0 + 256 * i, W * TP - 1);
      const int wy = div_ss(o, rTP), ox = o - wy * TP;
      at[i] = wy * W4 + ss * ox;
    }
    int k = 0;
#pragma unroll 1
    for (; k + 4 <= L; k += 4) {
      const float4 w = *reinterpret_cast<const float4*>(tg + k);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const float* q = S1 + at[i] + k;
        acc[i] = fmaf(w.x, q[0], acc[i]);
        acc[i] = fmaf(w.y, q[1], acc[i]);
        acc[i] = fmaf(w.z, q[2], acc[i]);
        acc[i] = fmaf(w.w, q[3], acc[i]);
      }
    }
    for (; k < L; ++k) {
      const float w = tg[k];
#pragma unroll
      for (int i = 0; i < 3; ++i) acc[i] = fmaf(w, S1[at[i] + k], acc[i]);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int o = o0 + 256 * i;
      if (o < W * TP) {
        const int wy = div_ss(o, rTP), ox = o - wy * TP;
        S2T[ox * LT + wy] = acc[i];
      }
    }
  }
  __syncthreads();
  // y: pixel (oy, ox) = sum_t g(t) S2T[ox][ss oy + t] / ss^2
  const float inv_ss2 = 1.f / (float)(ss * ss);
  float acc[NU] = {};
  forward_ypass<NU>(S2T, tg, L, LT, ss, TP, rTP, acc);
  double dot = 0.0;
#pragma unroll
  for (int u = 0; u < NU; ++u) {
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

template <int NU>
__global__ __launch_bounds__(256) void psf_forward_kernel(int n, int ss, Taps taps, const float* __restrict__ in,
                                                          int ld_in, float* __restrict__ out, int ld_out,
                                                          float alpha, float beta, const float* __restrict__ extra,
                                                          int ld_extra, float gamma, const float* __restrict__ dotv,
                                                          int ld_dotv, double* __restrict__ partial, int ntiles,
                                                          CgGate gate) {
  psf_forward_body<NU>([&] { return gate.skip(blockIdx.y); }, blockIdx.x, blockIdx.y, n, ss, taps, in, ld_in, out, ld_out, alpha, beta, extra, ld_extra, gamma,
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
  extern __shared__ __align__(16) float psf_lds[];
  const int M = n * ss, r = taps.r, L = taps.L;
  int WC, K4, WCP;  // window side in pixels, taps per phase (padded), window row stride
  adj_tile_dims(r, ss, WC, K4, WCP);
  static_assert(kFineTile == 32, "the Z-order decode below takes 5 bits per axis");
  const int F = kFineTile, LS = kAdjStride;
  float* const T = psf_lds;           // [ss][K4] taps by phase
  float* const S1 = T + ss * K4;      // [WC][WCP] pixel window
  float* const S2 = S1 + WC * WCP;    // [WC + K4 - 1][LS] filtered along x
  const float rss = 1.f / (float)ss;
  // The pixels reaching fine point f along an axis are J(f) + k, k < K, with
  // J(f) = floor((f - r) / ss); the weight of pixel J(f) + k is the composite
  // tap g[q + 2r - ss k] (zero outside [0, L)), q = f - r - ss J(f) the phase.
  // D, a multiple of ss above r, keeps the argument of the division positive.
  const int D = ss * ((32 + ss - 1) / ss);
  auto pix = [&](int f) { return div_ss(f - r + D, rss) - D / ss; };
  const int tiles_x = (M + F - 1) / F;
  const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
  const int fy0 = ty * F, fx0 = tx * F;
  const int cy0 = pix(fy0), cx0 = pix(fx0);  // first pixel row and column of the window
  const float* src = in + (size_t)c * ld_in;
  const float inv_ss2 = 1.f / (float)(ss * ss);
  const int lx = threadIdx.x & 31, ly = threadIdx.x >> 5;  // 32 x 8 threads
  // the thread's points: position o = tid + 256 u of the walk
  constexpr int kPer = kFineTile * kFineTile / 256;
  int px[kPer], py[kPer], tb[kPer];
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
    const int fy = fy0 + y, J = pix(fy);
    tb[u] = (fy - r - ss * J) * K4;
    col[u] = S2 + (J - cy0) * LS + x;
  }
  {
    WinRegs R;
    win_load_sep(
        R, WC, src,
        [&](int wy, bool& ok) {
          const int iy = cy0 + wy;
          ok = wy < WC && iy >= 0 && iy < n;
          return clamp_idx(iy, n) * n;
        },
        [&](int wx, bool& ok) {
          const int ix = cx0 + wx;
          ok = wx < WC && ix >= 0 && ix < n;
          return clamp_idx(ix, n);
        });
    if (skip()) return;
    for (int i = threadIdx.x; i < ss * K4; i += 256) {
      const int q = i / K4, k = i - q * K4, t = q + 2 * r - ss * k;
      T[i] = t >= 0 && t < L ? taps.g[t] : 0.f;
    }
    for (int i = threadIdx.x; i < WC * 8; i += 256) S1[(i >> 3) * WCP + WC + (i & 7)] = 0.f;
    for (int i = threadIdx.x; i < (K4 - 1) * LS; i += 256) S2[WC * LS + i] = 0.f;
    pre();  // runs while the window loads are in flight
#pragma unroll
    for (int u = 0; u < kPer; ++u) fetch(u, min(fy0 + py[u], M - 1), min(fx0 + px[u], M - 1));
    win_store(R, WC, S1, WCP);
  }
  __syncthreads();
  // x: S2[wy][x] = sum_k T[qx][k] S1[wy][jlo + k] for the pixels jlo + k that
  // reach fine column fx0 + x (their reads stay inside the row's zero padding)
  {
    const int fx = fx0 + lx, J = pix(fx);
    const int jlo = J - cx0;
    const float* tq = T + (fx - r - ss * J) * K4;
    const int nk = (WC + 7) / 8;
#pragma unroll 1
    for (int k0 = 0; k0 < nk; k0 += 3) {
      int at[3];
      float acc[3] = {0.f, 0.f, 0.f};
#pragma unroll
      for (int i = 0; i < 3; ++i) at[i] = min(ly + 8 * (k0 + i), WC - 1) * WCP + jlo;
#pragma unroll 1
      for (int k = 0; k < K4; k += 4) {
        const float4 w = *reinterpret_cast<const float4*>(tq + k);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const float* q = S1 + at[i] + k;
          acc[i] = fmaf(w.x, q[0], acc[i]);
          acc[i] = fmaf(w.y, q[1], acc[i]);
          acc[i] = fmaf(w.z, q[2], acc[i]);
          acc[i] = fmaf(w.w, q[3], acc[i]);
        }
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
#pragma unroll 1
  for (int k = 0; k < K4; k += 4) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const float4 w = *reinterpret_cast<const float4*>(T + tb[u] + k);
      const float* q = col[u] + k * LS;
      v[u] = fmaf(w.x, q[0], v[u]);
      v[u] = fmaf(w.y, q[LS], v[u]);
      v[u] = fmaf(w.z, q[2 * LS], v[u]);
      v[u] = fmaf(w.w, q[3 * LS], v[u]);
    }
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
  auto skip = [&] { return S.n_active[p] == 0 || S.st[p][c].active == 0; };
  if (S.ss == 1)
    psf_forward_body<kOutPer>(skip, tile, c, S.n, S.ss, S.taps, S.T2, S.ldf, S.AP, S.ldv, 1.f, 0.f, S.P, S.ldv,
                              S.sigma2, S.P, S.ldv, S.pap_part, S.ntiles_fwd);
  else
    psf_forward_body<1>(skip, tile, c, S.n, S.ss, S.taps, S.T2, S.ldf, S.AP, S.ldv, 1.f, 0.f, S.P, S.ldv, S.sigma2,
                        S.P, S.ldv, S.pap_part, S.ntiles_fwd);
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
  auto kern = fwd_pixels_per_thread(ss) == 1 ? psf_forward_kernel<1> : psf_forward_kernel<kOutPer>;
  hipLaunchKernelGGL(kern, dim3(ntiles, nrhs), dim3(256), fwd_lds_bytes(taps.r, ss), stream, n, ss, taps, in, ld_in,
                     out, ld_out, alpha, beta, extra, ld_extra, gamma, dotv, ld_dotv, partial, ntiles, gate);
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

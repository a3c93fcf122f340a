// Observation operator B = D o P (PSF on the fine grid, then local averaging to
// image pixels) and its adjoint B^T = P^T D^T (Sec. 2 and Sec. 3.3 footnote on a
// PSF as deterministic post-processing of the fluxes; Sec. 4.1 local averaging).
//
// One workgroup per (tile, column). The fine window of the tile plus the PSF
// halo is staged in LDS, convolved along x into a second LDS buffer, then along
// y; the forward direction averages each ss x ss block on the fly, the adjoint
// generates D^T x while loading the window. The taps are a normalised 1-D
// Gaussian (outer product in 2-D), computed on the host in FP64.
#include <cmath>

#include "common.hpp"
#include "internal.hpp"

namespace gpl {

constexpr int kFineTile = 32;  // fine-grid tile side
constexpr int kMaxWin = kFineTile + 2 * GPL_PSF_MAX_RADIUS;

int make_taps(const gpl_grid* g, const gpl_psf* psf, Taps& t) {
  GPL_REQUIRE(psf != nullptr, "psf is NULL");
  GPL_REQUIRE(psf->fwhm >= 0 && std::isfinite(psf->fwhm), "psf fwhm must be >= 0");
  GPL_REQUIRE(psf->radius >= 0 && psf->radius <= GPL_PSF_MAX_RADIUS, "psf radius must be in [0, %d]",
              GPL_PSF_MAX_RADIUS);
  if (psf->fwhm == 0.0) {
    t.r = 0;
    t.w[0] = 1.f;
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
  return GPL_OK;
}

// Forward: out[I] = alpha * (B in)[I] + beta * out[I] + gamma * extra[I];
// optional FP64 partial sums of dotv[I] * out[I] per (column, tile).
// Integer division by the supersampling factor (1 and 2 without a divide).
__device__ __forceinline__ int div_ss(int v, int ss) { return ss == 1 ? v : ss == 2 ? (v >> 1) : v / ss; }

__device__ __forceinline__ void psf_forward_body(int tile, int c, int n, int ss, const Taps& taps,
                                                 const float* __restrict__ in, int ld_in, float* __restrict__ out,
                                                 int ld_out, float alpha, float beta, const float* __restrict__ extra,
                                                 int ld_extra, float gamma, const float* __restrict__ dotv,
                                                 int ld_dotv, double* __restrict__ partial, int ntiles) {
  __shared__ float S1[kMaxWin * kMaxWin];
  __shared__ float S2[kMaxWin * (kFineTile + 1)];
  __shared__ float tw[2 * GPL_PSF_MAX_RADIUS + 1];
  __shared__ double red[4];
  const int M = n * ss, r = taps.r;
  if ((int)threadIdx.x <= 2 * r) tw[threadIdx.x] = taps.w[threadIdx.x];
  const int TP = kFineTile / ss > 0 ? kFineTile / ss : 1;  // output pixels per tile side
  const int F = TP * ss, W = F + 2 * r, LS = F + 1;
  const int tiles_x = (n + TP - 1) / TP;
  const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
  const int fy0 = ty * F, fx0 = tx * F;
  const float* src = in + (size_t)c * ld_in;
  const int lx = threadIdx.x & 31, ly = threadIdx.x >> 5;  // 32 x 8 threads
  for (int wy = ly; wy < W; wy += 8) {
    const int fy = fy0 - r + wy;
    const bool rowok = fy >= 0 && fy < M;
    for (int wx = lx; wx < W; wx += 32) {
      const int fx = fx0 - r + wx;
      S1[wy * W + wx] = (rowok && fx >= 0 && fx < M) ? src[(size_t)fy * M + fx] : 0.f;
    }
  }
  __syncthreads();
  for (int wy = ly; wy < W; wy += 8)
    for (int x = lx; x < F; x += 32) {
      const float* row = S1 + wy * W + x + r;
      float s = 0.f;
#pragma unroll 4
      for (int b = -r; b <= r; ++b) s += tw[b + r] * row[-b];
      S2[wy * LS + x] = s;
    }
  __syncthreads();
  const float inv_ss2 = 1.f / (float)(ss * ss);
  double dot = 0.0;
  for (int o = threadIdx.x; o < TP * TP; o += blockDim.x) {
    const int oy = o / TP, ox = o - oy * TP;
    const int Iy = ty * TP + oy, Ix = tx * TP + ox;
    if (Iy >= n || Ix >= n) continue;
    float acc = 0.f;
    for (int sy = 0; sy < ss; ++sy)
      for (int sx = 0; sx < ss; ++sx) {
        const int y = oy * ss + sy, x = ox * ss + sx;
        const float* col = S2 + (y + r) * LS + x;
        float v = 0.f;
#pragma unroll 4
        for (int a = -r; a <= r; ++a) v += tw[a + r] * col[-a * LS];
        acc += v;
      }
    const int I = Iy * n + Ix;
    float res = alpha * (acc * inv_ss2);
    if (beta != 0.f) res += beta * out[(size_t)c * ld_out + I];
    if (extra) res += gamma * extra[(size_t)c * ld_extra + I];
    out[(size_t)c * ld_out + I] = res;
    if (dotv) dot += (double)dotv[(size_t)c * ld_dotv + I] * (double)res;
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
  if (gate.skip(blockIdx.y)) return;
  psf_forward_body(blockIdx.x, blockIdx.y, n, ss, taps, in, ld_in, out, ld_out, alpha, beta, extra, ld_extra, gamma,
                   dotv, ld_dotv, partial, ntiles);
}

// Adjoint on one fine tile: v = (P^T D^T in)(fy, fx) for every fine point of the
// tile, handed to store(fy, fx, v, z) with z the point's Z-order index within
// the tile when ZWALK and the tile lies inside the grid (else -1). P^T is the correlation with the taps:
// (P^T g)(y, x) = sum_{a,b} w_a w_b g(y + a, x + b).
template <bool ZWALK, class Store>
__device__ __forceinline__ void psf_adjoint_tile(int tile, int c, int n, int ss, const Taps& taps,
                                                 const float* __restrict__ in, int ld_in, Store&& store) {
  __shared__ float S1[kMaxWin * kMaxWin];
  __shared__ float S2[kMaxWin * (kFineTile + 1)];
  __shared__ float tw[2 * GPL_PSF_MAX_RADIUS + 1];
  const int M = n * ss, r = taps.r;
  static_assert(kFineTile == 32, "the Z-order decode below takes 5 bits per axis");
  const int F = kFineTile, W = F + 2 * r, LS = F + 1;
  if ((int)threadIdx.x <= 2 * r) tw[threadIdx.x] = taps.w[threadIdx.x];
  const int tiles_x = (M + F - 1) / F;
  const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
  const int fy0 = ty * F, fx0 = tx * F;
  const float* src = in + (size_t)c * ld_in;
  const float inv_ss2 = 1.f / (float)(ss * ss);
  const int lx = threadIdx.x & 31, ly = threadIdx.x >> 5;  // 32 x 8 threads
  for (int wy = ly; wy < W; wy += 8) {
    const int fy = fy0 - r + wy;
    const bool rowok = fy >= 0 && fy < M;
    const float* srow = src + (size_t)div_ss(rowok ? fy : 0, ss) * n;
    for (int wx = lx; wx < W; wx += 32) {
      const int fx = fx0 - r + wx;
      S1[wy * W + wx] = (rowok && fx >= 0 && fx < M) ? srow[div_ss(fx, ss)] * inv_ss2 : 0.f;
    }
  }
  __syncthreads();
  for (int wy = ly; wy < W; wy += 8) {
    const float* row = S1 + wy * W + lx + r;
    float s = 0.f;
#pragma unroll 4
    for (int b = -r; b <= r; ++b) s += tw[b + r] * row[b];
    S2[wy * LS + lx] = s;
  }
  __syncthreads();
  // A tile fully inside the grid holds consecutive Z-order ranks (it is an
  // aligned power-of-two square): z is the point's Z-order index in the tile.
  const bool zwalk = ZWALK && fy0 + F <= M && fx0 + F <= M;
  for (int o = threadIdx.x; o < F * F; o += blockDim.x) {
    int x = 0, y = 0;
    if (zwalk) {
#pragma unroll
      for (int bit = 0; bit < 5; ++bit) {
        x |= ((o >> (2 * bit)) & 1) << bit;
        y |= ((o >> (2 * bit + 1)) & 1) << bit;
      }
    } else {
      y = o >> 5;
      x = o & 31;
    }
    const int fy = fy0 + y, fx = fx0 + x;
    if (fy >= M || fx >= M) continue;
    const float* col = S2 + (y + r) * LS + x;
    float v = 0.f;
#pragma unroll 4
    for (int a = -r; a <= r; ++a) v += tw[a + r] * col[a * LS];
    const int z = zwalk ? o : -1;
    store(fy, fx, v, z);
  }
}

// out (fine, row-major) = alpha * B^T in + beta * out.
__device__ __forceinline__ void psf_adjoint_body(int tile, int c, int n, int ss, const Taps& taps,
                                                 const float* __restrict__ in, int ld_in, float* __restrict__ out,
                                                 int ld_out, float alpha, float beta) {
  const int M = n * ss;
  psf_adjoint_tile<false>(tile, c, n, ss, taps, in, ld_in, [&](int fy, int fx, float v, int) {
    const size_t o_idx = (size_t)c * ld_out + (size_t)fy * M + fx;
    float res = alpha * v;
    if (beta != 0.f) res += beta * out[o_idx];
    out[o_idx] = res;
  });
}

// B^T P written straight into the RHS buffers of a grid-ordered product: fine
// point (fx, fy) goes to its Z-order rank; the precision form scales column c by
// 2^e_c, chosen from the bound max |B^T P| <= max |P| / ss^2 (nonnegative taps
// summing to one) so that the largest entry stays below 2^14, and splits it
// into FP16 hi (nearest) and lo.
__device__ __forceinline__ void psf_adjoint_rhs_body(int tile, int c, int n, int ss, const Taps& taps,
                                                     const float* __restrict__ in, int ld_in, const RhsOut& o) {
  __shared__ float red[4];
  __shared__ float s_scale;
  const int M = n * ss;
  const int tiles_x = (M + kFineTile - 1) / kFineTile;
  const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
  const int base = zorder_rank(tx * kFineTile, ty * kFineTile, M);  // first rank of an interior tile
  const bool f16 = o.prec == GPL_PREC_F16X3;
  if (f16) {
    float m = 0.f;
    for (int k = threadIdx.x; k < o.npart; k += blockDim.x) m = fmaxf(m, __uint_as_float(o.pmax[c * o.npart + k]));
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      const float mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3])) / (float)(ss * ss);
      int e = 0;
      if (mx > 0.f && isfinite(mx)) e = 14 - ilogbf(mx) - 1;  // bound * 2^e in [2^13, 2^14)
      s_scale = ldexpf(1.f, e);
      if (tile == 0) o.inv_scale[c] = ldexpf(1.f, -e) / 2048.f;  // with the 2^11 of the exp tile
    }
    __syncthreads();
  }
  const float scale = f16 ? s_scale : 1.f;
  // one instantiation of the tile (its LDS buffers) for both forms
  psf_adjoint_tile<true>(tile, c, n, ss, taps, in, ld_in, [&](int fy, int fx, float v, int z) {
    const size_t j = (size_t)c * o.ldh + (z >= 0 ? base + z : zorder_rank(fx, fy, M));
    if (f16) {
      const float sv = v * scale;
      const _Float16 h = (_Float16)sv;
      o.Vh[j] = h;
      o.Vl[j] = (_Float16)(sv - (float)h);
    } else {
      o.Vp[j] = v;
    }
  });
}

__global__ __launch_bounds__(256) void psf_adjoint_rhs_kernel(int n, int ss, Taps taps, const float* __restrict__ in,
                                                              int ld_in, RhsOut o, CgGate gate) {
  if (gate.skip(blockIdx.y)) return;
  psf_adjoint_rhs_body(blockIdx.x, blockIdx.y, n, ss, taps, in, ld_in, o);
}

__global__ __launch_bounds__(256) void psf_adjoint_kernel(int n, int ss, Taps taps, const float* __restrict__ in,
                                                          int ld_in, float* __restrict__ out, int ld_out,
                                                          float alpha, float beta, CgGate gate) {
  if (gate.skip(blockIdx.y)) return;
  psf_adjoint_body(blockIdx.x, blockIdx.y, n, ss, taps, in, ld_in, out, ld_out, alpha, beta);
}

// ---- grouped launches (serving): workgroup b of slot s handles (tile, column) =
// (local % tiles, local / tiles), local = b - off[s].

__global__ __launch_bounds__(256) void psf_adjoint_grouped_kernel(SlotBatch B, int p) {
  const int s = B.find(blockIdx.x);
  const ServeSlotDev& S = *B.slot[s];
  if (S.n_active[p] == 0) return;
  const int local = blockIdx.x - B.off[s];
  const int tile = local % S.ntiles_adj, c = local / S.ntiles_adj;
  if (S.st[p][c].active == 0) return;
  const RhsOut o{S.prec, S.ldh, S.Vh, S.Vl, S.Vp, S.inv_scale, S.pmax, S.nb_upd};
  psf_adjoint_rhs_body(tile, c, S.n, S.ss, S.taps, S.P, S.ldv, o);
}

__global__ __launch_bounds__(256) void psf_forward_grouped_kernel(SlotBatch B, int p) {
  const int s = B.find(blockIdx.x);
  const ServeSlotDev& S = *B.slot[s];
  if (S.n_active[p] == 0) return;
  const int local = blockIdx.x - B.off[s];
  const int tile = local % S.ntiles_fwd, c = local / S.ntiles_fwd;
  if (S.st[p][c].active == 0) return;
  psf_forward_body(tile, c, S.n, S.ss, S.taps, S.T2, S.ldf, S.AP, S.ldv, 1.f, 0.f, S.P, S.ldv, S.sigma2, S.P, S.ldv,
                   S.pap_part, S.ntiles_fwd);
}

int psf_adjoint_tiles(int n, int ss) {
  const int M = n * ss, t = (M + kFineTile - 1) / kFineTile;
  return t * t;
}

static int grouped_launch(void (*kern)(SlotBatch, int), const ServeSlotDev* const* hslots,
                          const ServeSlotDev* const* dslots, int nslots, int p, int (*tiles_of)(const ServeSlotDev&),
                          hipStream_t stream) {
  SlotBatch B;
  B.nslots = nslots;
  B.off[0] = 0;
  for (int s = 0; s < nslots; ++s) {
    B.slot[s] = dslots[s];
    B.off[s + 1] = B.off[s] + tiles_of(*hslots[s]);
  }
  if (B.off[nslots] == 0) return GPL_OK;
  hipLaunchKernelGGL(kern, dim3(B.off[nslots]), dim3(256), 0, stream, B, p);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

int psf_adjoint_grouped(const ServeSlotDev* const* hslots, const ServeSlotDev* const* dslots, int nslots, int p,
                        hipStream_t stream) {
  return grouped_launch(psf_adjoint_grouped_kernel, hslots, dslots, nslots, p,
                        [](const ServeSlotDev& S) { return S.ntiles_adj * S.nrhs; }, stream);
}

int psf_forward_grouped(const ServeSlotDev* const* hslots, const ServeSlotDev* const* dslots, int nslots, int p,
                        hipStream_t stream) {
  return grouped_launch(psf_forward_grouped_kernel, hslots, dslots, nslots, p,
                        [](const ServeSlotDev& S) { return S.ntiles_fwd * S.nrhs; }, stream);
}

int psf_forward_tiles(int n, int ss) {
  const int TP = kFineTile / ss > 0 ? kFineTile / ss : 1;
  const int t = (n + TP - 1) / TP;
  return t * t;
}

int psf_forward_launch(int n, int ss, const Taps& taps, int nrhs, const float* in, int ld_in, float* out, int ld_out,
                       float alpha, float beta, const float* extra, int ld_extra, float gamma, const float* dotv,
                       int ld_dotv, double* partial, CgGate gate, hipStream_t stream) {
  GPL_REQUIRE(ss <= kFineTile, "ss=%d exceeds %d", ss, kFineTile);
  const int ntiles = psf_forward_tiles(n, ss);
  hipLaunchKernelGGL(psf_forward_kernel, dim3(ntiles, nrhs), dim3(256), 0, stream, n, ss, taps, in, ld_in, out,
                     ld_out, alpha, beta, extra, ld_extra, gamma, dotv, ld_dotv, partial, ntiles, gate);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

int psf_adjoint_rhs_launch(int n, int ss, const Taps& taps, int nrhs, const float* P, int ldp, const RhsOut& out,
                           CgGate gate, hipStream_t stream) {
  const int M = n * ss, t = (M + kFineTile - 1) / kFineTile;
  hipLaunchKernelGGL(psf_adjoint_rhs_kernel, dim3(t * t, nrhs), dim3(256), 0, stream, n, ss, taps, P, ldp, out, gate);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

int psf_adjoint_launch(int n, int ss, const Taps& taps, int nrhs, const float* in, int ld_in, float* out, int ld_out,
                       float alpha, float beta, CgGate gate, hipStream_t stream) {
  const int M = n * ss, t = (M + kFineTile - 1) / kFineTile;
  hipLaunchKernelGGL(psf_adjoint_kernel, dim3(t * t, nrhs), dim3(256), 0, stream, n, ss, taps, in, ld_in, out, ld_out,
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

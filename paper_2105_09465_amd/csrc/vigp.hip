// Variationally optimised GP source: one reparametrised ELBO sample and its
// gradient (Sec. 3.3 eqs. "gp-gen2", "decomposition"; Sec. 3.4 eq.
// "transmission" with the k-th-neighbour density; Sec. 3.5 image- and
// source-plane layers; Sec. 3.6 eqs. "elbo", "reparam"; Sec. 4.2 eq. "guide"),
// and the Adam update of Sec. 4.3.
//
// Layers: f = mu(p) + sum_k T_k y_k, T_k[i][j] = A_j N(p_i - q_j, Zt_i + l_k^2 I / 2),
// A_j = sqrt(2 pi l_k^2) w_j with w_j = rho_j^{-1/2} = r_j sqrt(pi / k) (r_j the
// distance to the k-th closest other inducing point). Image-plane layers: q = p,
// Zt = the pixel shapes; the source-plane layer: q = a fixed grid, Zt = 0. All
// products are the Gaussian products of gauss.hip (every pair in FP32).
//
// Step: the lens sample theta (device FP64), the source samples y (FP32),
// ray tracing from the device-held theta, pixel shapes, k-NN weights, the
// layered fluxes, residual r = d - B f; backward g_f = B^T r / sigma^2, per
// layer T_k^T g_f, then dE/dp from the Sersic mean, both sides of every
// transmission product, the pixel shapes and the k-NN weights, and dE/dtheta
// by the ray-tracing adjoint. A final one-thread kernel folds the FP64 sums
// into the ELBO pieces and the gradient of the small FP64 parameter block.
#include <cmath>

#include "common.hpp"
#include "internal.hpp"

namespace gpl {

constexpr int kVMaxLayers = 8;
constexpr int kVSums = 1 + 3 * kVMaxLayers;  // |r|^2, then per layer |y|^2, sum log s, |e|^2

struct VLayout {
  int nl, nip, sp;  // layers, image-plane layers, index of the source-plane layer (-1: none)
  int N, M, G, npix;
  size_t n64, n32, ne32;
  size_t mean[kVMaxLayers], logs[kVMaxLayers], cross;  // P32 offsets of each layer's blocks
  size_t e[kVMaxLayers];                               // e32 offset of each layer's noise
  int n[kVMaxLayers];                                  // source parameters per layer
};

static int vigp_layout(const gpl_vigp_model* m, const gpl_grid* grid, int G, VLayout& L) {
  GPL_REQUIRE(m != nullptr && grid != nullptr, "model/grid are NULL");
  GPL_REQUIRE(m->n_layers >= 1 && m->n_layers <= kVMaxLayers, "n_layers=%d must be in [1, %d]", m->n_layers,
              kVMaxLayers);
  GPL_REQUIRE(grid->n >= 1 && grid->ss >= 1, "bad grid");
  L.nl = m->n_layers;
  L.M = grid->n * grid->ss;
  L.N = L.M * L.M;
  L.npix = grid->n * grid->n;
  L.G = G;
  L.sp = -1;
  L.nip = 0;
  for (int k = 0; k < L.nl; ++k) {
    GPL_REQUIRE(m->lengthscale[k] > 0 && std::isfinite(m->lengthscale[k]), "lengthscale[%d] must be > 0", k);
    if (m->kind[k] == GPL_VIGP_SOURCE_PLANE) {
      GPL_REQUIRE(L.sp < 0, "at most one source-plane layer");
      L.sp = k;
    } else {
      GPL_REQUIRE(m->kind[k] == GPL_VIGP_IMAGE_PLANE, "kind[%d]=%d unknown", k, m->kind[k]);
      ++L.nip;
    }
  }
  GPL_REQUIRE(m->knn_k >= 1 && m->knn_k <= 32, "knn_k=%d must be in [1, 32]", m->knn_k);
  GPL_REQUIRE(L.nip == 0 || L.N > m->knn_k, "need more than knn_k traced points");
  GPL_REQUIRE(L.sp < 0 || G > m->knn_k, "a source-plane layer needs more than knn_k grid points (G=%d)", G);
  GPL_REQUIRE(m->shear_sd > 0, "shear_sd must be > 0");
  L.n64 = 56 + (size_t)L.nl;
  size_t o = 0, oe = 0;
  if (L.sp >= 0) {
    L.mean[L.sp] = o;
    L.logs[L.sp] = o + G;
    L.cross = o + 2 * (size_t)G;
    L.n[L.sp] = G;
    L.e[L.sp] = oe;
    o += 9 * (size_t)G;
    oe += G;
  }
  for (int k = 0; k < L.nl; ++k) {
    if (k == L.sp) continue;
    L.mean[k] = o;
    L.logs[k] = o + L.N;
    L.n[k] = L.N;
    L.e[k] = oe;
    o += 2 * (size_t)L.N;
    oe += L.N;
  }
  L.n32 = o;
  L.ne32 = oe;
  return GPL_OK;
}

// bump allocation inside the caller's workspace
struct Bump {
  char* p;
  size_t used = 0;
  template <class T>
  T* take(size_t n) {
    T* r = p ? reinterpret_cast<T*>(p + used) : nullptr;
    used += align_up(n * sizeof(T));
    return r;
  }
};

struct VBufs {
  double *lens, *g_lens, *g_src, *sums, *gq, *rt_partial, *se_partial;
  void* knn_ws;
  size_t knn_bytes;
  float *px, *py, *Z, *f, *resid, *g_f, *gpx, *gpy, *gZ, *gw, *gab, *r, *w, *w_sp, *r_sp, *y;
  int *nn, *nn_sp;
};

static size_t vigp_carve(const VLayout& L, void* ws, VBufs& b) {
  Bump B{static_cast<char*>(ws)};
  const size_t N = L.N, G = std::max(L.G, 1);
  b.lens = B.take<double>(8);
  b.g_lens = B.take<double>(8);
  b.g_src = B.take<double>(2);
  b.sums = B.take<double>(kVSums);
  b.gq = B.take<double>(2 * N);
  b.rt_partial = B.take<double>(8 * (size_t)cdiv(L.N, 256));
  b.se_partial = B.take<double>(2 * (size_t)cdiv(L.N, 256));
  b.px = B.take<float>(N);
  b.py = B.take<float>(N);
  b.Z = B.take<float>(3 * N);
  b.f = B.take<float>(N);
  b.resid = B.take<float>(L.npix);
  b.g_f = B.take<float>(N);
  b.gpx = B.take<float>(N);
  b.gpy = B.take<float>(N);
  b.gZ = B.take<float>(3 * N);
  b.gw = B.take<float>(N);
  b.gab = B.take<float>(4 * N);
  b.r = B.take<float>(N);
  b.w = B.take<float>(N);
  b.nn = B.take<int>(N);
  b.w_sp = B.take<float>(G);
  b.r_sp = B.take<float>(G);
  b.nn_sp = B.take<int>(G);
  b.y = B.take<float>(L.ne32 ? L.ne32 : 1);
  b.knn_bytes = knn_workspace(std::max(L.nip > 0 ? L.N : 0, L.sp >= 0 ? L.G : 0));
  b.knn_ws = B.take<char>(std::max<size_t>(b.knn_bytes, 1));
  return B.used;
}

struct VSeg {
  const float* a[kVSums];
  int n[kVSums];
  int square[kVSums];
};

// sums[s] = sum_i a_s[i]^2 (square) or sum_i a_s[i], FP64, one workgroup per
// segment in a fixed order.
__global__ __launch_bounds__(256) void vigp_sums_kernel(VSeg seg, double* sums) {
  __shared__ double red[4];
  const int s = blockIdx.x;
  const float* a = seg.a[s];
  const int n = seg.n[s];
  double acc = 0.0;
  if (a != nullptr)
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const double v = (double)a[i];
      acc += seg.square[s] ? v * v : v;
    }
  acc = block_sum_double(acc, red);
  if (threadIdx.x == 0) sums[s] = acc;
}

// theta = m_l + L_l e_l (L_l: strictly lower part of raw, exp of its diagonal),
// with the fixed slope in position 3 of the 8-vector.
__global__ void vigp_lens_sample_kernel(const double* __restrict__ P64, const double* __restrict__ e_l, double slope,
                                        double* lens) {
  if (threadIdx.x != 0) return;
  const int free_idx[7] = {0, 1, 2, 4, 5, 6, 7};
  for (int a = 0; a < 7; ++a) {
    double t = P64[a];
    for (int b = 0; b < a; ++b) t += P64[7 + a * 7 + b] * e_l[b];
    t += exp(P64[7 + a * 7 + a]) * e_l[a];
    lens[free_idx[a]] = t;
  }
  lens[3] = slope;
}

// y = m + C e_l + exp(logs) e (C nullable: n x 7, column b at b * n)
__global__ void vigp_sample_y_kernel(int n, const float* __restrict__ m, const float* __restrict__ logs,
                                     const float* __restrict__ C, const double* __restrict__ e_l,
                                     const float* __restrict__ e, float* y) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  float v = m[j];
  if (C)
    for (int b = 0; b < 7; ++b) v = fmaf(C[(size_t)b * n + j], (float)e_l[b], v);
  y[j] = fmaf(expf(logs[j]), e[j], v);
}

__global__ void vigp_knn_weight_kernel(int n, const float* __restrict__ r, float c, float* w) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) w[j] = c * r[j];
}

__global__ void vigp_fill_kernel(size_t n, float* a, float v) {
  const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) a[j] = v;
}

__global__ void vigp_fill_double_kernel(size_t n, double* a) {
  const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) a[j] = 0.0;
}

__global__ void vigp_copy_kernel(int n, const float* __restrict__ a, float* b) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) b[j] = a[j];
}

// Per-parameter gradients of one layer, from t = T^T g_f held in gmean:
// g_y = t - y / alpha^2 (alpha = exp(log_amp)); dE/dm = g_y,
// dE/dlog s = s g_y e + 1, dE/dC[:, b] = g_y e_l[b] (source-plane layer).
__global__ void vigp_layer_grad_kernel(int n, const float* __restrict__ y, const double* __restrict__ log_amp,
                                       const float* __restrict__ logs, const float* __restrict__ e,
                                       const double* __restrict__ e_l, float* gmean, float* glogs, float* gcross) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const float ia2 = (float)exp(-2.0 * log_amp[0]);
  const float g = gmean[j] - y[j] * ia2;
  gmean[j] = g;
  glogs[j] = fmaf(expf(logs[j]) * g, e[j], 1.f);
  if (gcross)
    for (int b = 0; b < 7; ++b) gcross[(size_t)b * n + j] = g * (float)e_l[b];
}

struct VFinal {
  int nl, npix, n[kVMaxLayers];
  double sigma, lo[5], hi[5], shear_sd;
};

// ELBO pieces and the FP64 gradient block (lens mean 7, lens raw 49, log amp).
__global__ void vigp_finalize_kernel(VFinal F, const double* __restrict__ P64, const double* __restrict__ e_l,
                                     const double* __restrict__ lens, const double* __restrict__ sums,
                                     const double* __restrict__ g_lens, double* out, double* G64) {
  if (threadIdx.x != 0) return;
  const double l2pi = log(2.0 * M_PI);
  const double sig = F.sigma;
  const double loglik = -0.5 * sums[0] / (sig * sig) - F.npix * log(sig) - 0.5 * F.npix * l2pi;
  double lpy = 0.0, nlq = 0.0;
  double ntot = 7.0;
  for (int a = 0; a < 7; ++a) nlq += 0.5 * e_l[a] * e_l[a] + P64[7 + a * 7 + a];
  for (int k = 0; k < F.nl; ++k) {
    const double la = P64[56 + k], a2 = exp(2.0 * la);
    const double sy = sums[1 + 3 * k], sl = sums[2 + 3 * k], se = sums[3 + 3 * k];
    lpy += -0.5 * sy / a2 - F.n[k] * la - 0.5 * F.n[k] * l2pi;
    nlq += 0.5 * se + sl;
    ntot += F.n[k];
    G64[56 + k] = sy / a2 - F.n[k];
  }
  nlq += 0.5 * ntot * l2pi;
  const int box[5] = {0, 1, 2, 4, 5};
  bool inside = true;
  double lpt = 0.0;
  for (int i = 0; i < 5; ++i) {
    inside = inside && lens[box[i]] >= F.lo[i] && lens[box[i]] <= F.hi[i];
    lpt -= log(F.hi[i] - F.lo[i]);
  }
  if (!inside) lpt = -INFINITY;
  double gt8[8];
  for (int k = 0; k < 8; ++k) gt8[k] = g_lens[k];
  for (int k = 6; k < 8; ++k) {
    const double t = lens[k] / F.shear_sd;
    lpt += -0.5 * t * t - log(F.shear_sd) - 0.5 * l2pi;
    gt8[k] -= lens[k] / (F.shear_sd * F.shear_sd);
  }
  out[0] = loglik + lpy + lpt + nlq;
  out[1] = loglik;
  out[2] = lpy;
  out[3] = lpt;
  out[4] = nlq;
  for (int k = 0; k < 8; ++k) out[5 + k] = lens[k];
  const int free_idx[7] = {0, 1, 2, 4, 5, 6, 7};
  for (int a = 0; a < 7; ++a) {
    const double g = gt8[free_idx[a]];
    G64[a] = g;
    for (int b = 0; b < 7; ++b) {
      double v = 0.0;
      if (b < a) v = g * e_l[b];
      if (b == a) v = g * e_l[a] * exp(P64[7 + a * 7 + a]) + 1.0;
      G64[7 + a * 7 + b] = v;
    }
  }
}

// Adam (torch's form) minimising -E: the loss gradient is -G. The weights
// 1 - beta come from the host in double precision (1 - 0.999f in FP32 would be
// 1.3e-5 off 0.001).
template <class T>
__global__ void vigp_adam_kernel(size_t n, T* p, const T* __restrict__ g, T* m, T* v, T lr_bc1, T b1, T omb1, T b2,
                                 T omb2, T inv_sqrt_bc2, T eps) {
  const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const T gl = -g[j];
  const T mj = b1 * m[j] + omb1 * gl;
  const T vj = b2 * v[j] + omb2 * gl * gl;
  m[j] = mj;
  v[j] = vj;
  p[j] -= lr_bc1 * mj / (sqrt(vj) * inv_sqrt_bc2 + eps);
}

static inline dim3 blocks_for(size_t n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace gpl

using namespace gpl;

extern "C" int gpl_vigp_sizes(const gpl_vigp_model* model, const gpl_grid* grid, int G, size_t* n64, size_t* n32,
                              size_t* ne32) {
  VLayout L;
  GPL_TRY(vigp_layout(model, grid, G, L));
  if (n64) *n64 = L.n64;
  if (n32) *n32 = L.n32;
  if (ne32) *ne32 = L.ne32;
  return GPL_OK;
}

extern "C" size_t gpl_vigp_workspace(const gpl_vigp_model* model, const gpl_grid* grid, int G) {
  VLayout L;
  if (vigp_layout(model, grid, G, L) != GPL_OK) return 0;
  VBufs b;
  return vigp_carve(L, nullptr, b);
}

extern "C" int gpl_vigp_elbo(const gpl_vigp_model* model, const gpl_grid* grid, const gpl_psf* psf,
                             const gpl_source* src, double noise_sigma, int G, const float* gx, const float* gy,
                             const float* d, const double* P64, const float* P32, const double* e64,
                             const float* e32, double* out, double* G64, float* G32, void* ws, size_t ws_bytes,
                             hipStream_t stream) {
  VLayout L;
  GPL_TRY(vigp_layout(model, grid, G, L));
  GPL_REQUIRE(noise_sigma > 0 && std::isfinite(noise_sigma), "noise_sigma must be > 0");
  GPL_REQUIRE(src != nullptr && psf != nullptr, "source/psf are NULL");
  GPL_REQUIRE(d && P64 && P32 && e64 && e32 && out && G64 && G32, "NULL argument");
  GPL_REQUIRE(L.sp < 0 || (gx && gy), "source-plane layer without grid points");
  for (int i = 0; i < 5; ++i)
    GPL_REQUIRE(model->prior_hi[i] > model->prior_lo[i], "prior box %d is empty", i);
  VBufs b;
  const size_t need = vigp_carve(L, nullptr, b);
  GPL_TRY(check_ws(ws, ws_bytes, need));
  vigp_carve(L, ws, b);
  const int N = L.N;
  const size_t N3 = 3 * (size_t)N;
  const double kk = model->knn_k;
  const float wscale = (float)std::sqrt(M_PI / kk);

  // ---- samples
  hipLaunchKernelGGL(vigp_lens_sample_kernel, dim3(1), dim3(64), 0, stream, P64, e64, model->slope, b.lens);
  GPL_LAUNCH_CHECK();
  float* y[kVMaxLayers];
  for (int k = 0; k < L.nl; ++k) {
    y[k] = b.y + L.e[k];
    const bool sp = k == L.sp;
    hipLaunchKernelGGL(vigp_sample_y_kernel, blocks_for(L.n[k]), dim3(256), 0, stream, L.n[k], P32 + L.mean[k],
                       P32 + L.logs[k], sp ? P32 + L.cross : nullptr, e64, e32 + L.e[k], y[k]);
    GPL_LAUNCH_CHECK();
  }
  // ---- forward
  GPL_TRY(raytrace_dev_launch(grid, b.lens, b.px, b.py, stream));
  GPL_TRY(pixel_shapes_launch(L.M, b.px, b.py, b.Z, stream));
  if (L.nip > 0) {
    GPL_TRY(knn_index_launch(N, b.px, b.py, model->knn_k, nullptr, b.r, b.nn, b.knn_ws, b.knn_bytes, stream));
    hipLaunchKernelGGL(vigp_knn_weight_kernel, blocks_for(N), dim3(256), 0, stream, N, b.r, wscale, b.w);
    GPL_LAUNCH_CHECK();
  }
  if (L.sp >= 0) {
    GPL_TRY(knn_index_launch(G, gx, gy, model->knn_k, nullptr, b.r_sp, b.nn_sp, b.knn_ws, b.knn_bytes, stream));
    hipLaunchKernelGGL(vigp_knn_weight_kernel, blocks_for(G), dim3(256), 0, stream, G, b.r_sp, wscale, b.w_sp);
    GPL_LAUNCH_CHECK();
  }
  GPL_TRY(gpl_sersic_eval(src, N, b.px, b.py, b.f, stream));
  const GSide Pz{b.px, b.py, b.Z, nullptr, N}, P0{b.px, b.py, nullptr, nullptr, N};
  const GSide Qip{b.px, b.py, nullptr, b.w, N}, Qsp{gx, gy, nullptr, b.w_sp, G};
  double norm[kVMaxLayers], base[kVMaxLayers];
  for (int k = 0; k < L.nl; ++k) {
    const double ell = model->lengthscale[k];
    base[k] = 0.5 * ell * ell;
    norm[k] = std::sqrt(2.0 * M_PI * ell * ell) / (2.0 * M_PI);
    const bool sp = k == L.sp;
    GPL_TRY(gauss_product_launch(sp ? P0 : Pz, sp ? Qsp : Qip, base[k], norm[k], 1, y[k], L.n[k], b.f, N, 1.f,
                                 stream));
  }
  hipLaunchKernelGGL(vigp_copy_kernel, blocks_for(L.npix), dim3(256), 0, stream, L.npix, d, b.resid);
  GPL_LAUNCH_CHECK();
  GPL_TRY(gpl_psf_conv(grid, psf, 1, b.f, N, b.resid, L.npix, -1.f, 1.f, 0, stream));  // r = d - B f
  // ---- backward
  GPL_TRY(gpl_psf_conv(grid, psf, 1, b.resid, L.npix, b.g_f, N, (float)(1.0 / (noise_sigma * noise_sigma)), 0.f, 1,
                       stream));  // g_f = B^T r / sigma^2
  for (int k = 0; k < L.nl; ++k) {
    const bool sp = k == L.sp;
    // T_k^T g_f: targets are the inducing points (weights A), sources the traced points
    const GSide Tq = sp ? GSide{gx, gy, nullptr, b.w_sp, G} : GSide{b.px, b.py, nullptr, b.w, N};
    const GSide Sp = sp ? P0 : Pz;
    float* gmean = G32 + L.mean[k];
    GPL_TRY(gauss_product_launch(Tq, Sp, base[k], norm[k], 1, b.g_f, N, gmean, L.n[k], 0.f, stream));
    hipLaunchKernelGGL(vigp_layer_grad_kernel, blocks_for(L.n[k]), dim3(256), 0, stream, L.n[k], y[k], P64 + 56 + k,
                       P32 + L.logs[k], e32 + L.e[k], e64, gmean, G32 + L.logs[k], sp ? G32 + L.cross : nullptr);
    GPL_LAUNCH_CHECK();
  }
  // dE/dp
  hipLaunchKernelGGL(vigp_fill_kernel, blocks_for(N), dim3(256), 0, stream, (size_t)N, b.gpx, 0.f);
  hipLaunchKernelGGL(vigp_fill_kernel, blocks_for(N), dim3(256), 0, stream, (size_t)N, b.gpy, 0.f);
  hipLaunchKernelGGL(vigp_fill_kernel, blocks_for(N3), dim3(256), 0, stream, N3, b.gZ, 0.f);
  hipLaunchKernelGGL(vigp_fill_kernel, blocks_for(N), dim3(256), 0, stream, (size_t)N, b.gw, 0.f);
  hipLaunchKernelGGL(vigp_fill_double_kernel, blocks_for(2 * (size_t)N), dim3(256), 0, stream, 2 * (size_t)N, b.gq);
  GPL_LAUNCH_CHECK();
  GPL_TRY(gpl_sersic_backward(src, N, b.px, b.py, b.g_f, b.gpx, b.gpy, b.g_src, b.se_partial,
                              gpl_sersic_backward_workspace(N), stream));
  for (int k = 0; k < L.nl; ++k) {
    if (k == L.sp)
      GPL_TRY(gauss_backward_launch(P0, Qsp, base[k], norm[k], y[k], b.g_f, b.gpx, b.gpy, nullptr, nullptr, nullptr,
                                    nullptr, stream));
    else
      GPL_TRY(gauss_backward_launch(Pz, Qip, base[k], norm[k], y[k], b.g_f, b.gpx, b.gpy, b.gZ, b.gpx, b.gpy, b.gw,
                                    stream));
  }
  if (L.nip > 0) {
    GPL_TRY(pixel_shapes_backward_launch(L.M, b.px, b.py, b.gZ, b.gab, b.gpx, b.gpy, stream));
    // A_j = sqrt(2 pi l^2) w_j: dE/dw_j summed over the layers came with norm folded in
    GPL_TRY(knn_weight_backward_launch(N, b.px, b.py, b.r, b.nn, b.w, b.gw, b.gq, b.gpx, b.gpy, stream));
  }
  GPL_TRY(raytrace_dev_backward_launch(grid, b.lens, b.gpx, b.gpy, b.g_lens, b.rt_partial, stream));
  // ---- scalars
  VSeg seg{};
  int ns = 0;
  seg.a[ns] = b.resid;
  seg.n[ns] = L.npix;
  seg.square[ns++] = 1;
  for (int k = 0; k < L.nl; ++k) {
    seg.a[ns] = y[k];
    seg.n[ns] = L.n[k];
    seg.square[ns++] = 1;
    seg.a[ns] = P32 + L.logs[k];
    seg.n[ns] = L.n[k];
    seg.square[ns++] = 0;
    seg.a[ns] = e32 + L.e[k];
    seg.n[ns] = L.n[k];
    seg.square[ns++] = 1;
  }
  hipLaunchKernelGGL(vigp_sums_kernel, dim3(ns), dim3(256), 0, stream, seg, b.sums);
  GPL_LAUNCH_CHECK();
  VFinal F{};
  F.nl = L.nl;
  F.npix = L.npix;
  for (int k = 0; k < L.nl; ++k) F.n[k] = L.n[k];
  F.sigma = noise_sigma;
  for (int i = 0; i < 5; ++i) {
    F.lo[i] = model->prior_lo[i];
    F.hi[i] = model->prior_hi[i];
  }
  F.shear_sd = model->shear_sd;
  hipLaunchKernelGGL(vigp_finalize_kernel, dim3(1), dim3(64), 0, stream, F, P64, e64, b.lens, b.sums, b.g_lens, out,
                     G64);
  GPL_LAUNCH_CHECK();
  return GPL_OK;
}

extern "C" int gpl_vigp_adam(size_t n64, double* P64, const double* G64, double* M64, double* V64, size_t n32,
                             float* P32, const float* G32, float* M32, float* V32, int t, double lr, double beta1,
                             double beta2, double eps, hipStream_t stream) {
  GPL_REQUIRE(t >= 1, "step t=%d must be >= 1", t);
  GPL_REQUIRE(lr > 0 && beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0, "bad Adam constants");
  const double bc1 = 1.0 - std::pow(beta1, t), bc2 = 1.0 - std::pow(beta2, t);
  if (n64) {
    GPL_REQUIRE(P64 && G64 && M64 && V64, "NULL FP64 block");
    hipLaunchKernelGGL(vigp_adam_kernel<double>, blocks_for(n64), dim3(256), 0, stream, n64, P64, G64, M64, V64,
                       lr / bc1, beta1, 1.0 - beta1, beta2, 1.0 - beta2, 1.0 / std::sqrt(bc2), eps);
    GPL_LAUNCH_CHECK();
  }
  if (n32) {
    GPL_REQUIRE(P32 && G32 && M32 && V32, "NULL FP32 block");
    hipLaunchKernelGGL(vigp_adam_kernel<float>, blocks_for(n32), dim3(256), 0, stream, n32, P32, G32, M32, V32,
                       (float)(lr / bc1), (float)beta1, (float)(1.0 - beta1), (float)beta2, (float)(1.0 - beta2),
                       (float)(1.0 / std::sqrt(bc2)), (float)eps);
    GPL_LAUNCH_CHECK();
  }
  return GPL_OK;
}

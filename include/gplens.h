/*
 * gplens: GPU library for the Gaussian-process evidence of a lensed source.
 *
 * Karchev, Coogan & Weniger (2021), "Strong-lensing source reconstruction with
 * variationally optimised Gaussian processes". Supersampled image-plane pixels
 * are ray-traced through an SPLE lens with external shear (Sec. 2.1, 2.2); a
 * Gaussian-process source with an RBF kernel (Sec. 3.1, eq. "grbf") is observed
 * through a PSF and local averaging (Sec. 2, Sec. 4.1) with i.i.d. noise. The
 * library evaluates the marginal likelihood (Sec. 3.1, eq. "gp-mll") with
 * matrix-free kernel products, conjugate gradients and stochastic Lanczos
 * quadrature, the posterior mean (Sec. 3.7, eq. "gp-exact-mean"), the
 * variational objective of App. D.1 (eq. "hyper-loss"), and their gradients.
 *
 * Conventions shared by every entry point:
 *  - Array arguments are DEVICE pointers owned by the caller. The library never
 *    keeps them after a call returns and never frees them.
 *  - Parameter structs are HOST pointers, read during the call.
 *  - Work is enqueued on `stream` (0 = the null stream). Calls are asynchronous
 *    unless their comment says the host waits; none synchronises the device.
 *  - Scratch memory is passed in as (ws, ws_bytes); the matching
 *    gpl_*_workspace() call gives the size needed. ws must be 256-byte aligned.
 *    The library allocates no device memory.
 *  - Points: structure-of-arrays float px[n], py[n] in arcsec, any n >= 1.
 *  - Blocks of vectors: column-major float with leading dimension ld >= rows.
 *  - Return value: GPL_OK or a negative error code; gpl_strerror() names it and
 *    gpl_last_error() gives the detail of the last failure on this thread.
 *    Invalid arguments are rejected before anything is enqueued.
 */
#ifndef GPLENS_H
#define GPLENS_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GPL_OK 0
#define GPL_EINVAL (-1)       /* bad size, leading dimension, NULL or parameter */
#define GPL_EWORKSPACE (-2)   /* workspace missing, misaligned or too small */
#define GPL_EHIP (-3)         /* a HIP runtime call or kernel launch failed */
#define GPL_EUNSUPPORTED (-4) /* requested precision/kind is not available */

/* Arithmetic of the kernel-matrix product. */
#define GPL_PREC_FP32 0  /* exp tile FP32, tile x RHS product FP32 (VALU or FP32 MFMA) */
#define GPL_PREC_F16X3 1 /* exp tile FP32, product as FP16 hi/lo split on MFMA (3 terms), FP32 accumulate */

/* Per-column CG status. */
#define GPL_CG_CONVERGED 0
#define GPL_CG_MAXITER 1
#define GPL_CG_BREAKDOWN 2 /* p^T A p <= 0 */
#define GPL_CG_NONFINITE 3

/* Image grid: n x n pixels of side pix_scale (arcsec), each split into ss x ss
 * sub-pixels; the image centre sits at (cx, cy). Fine point j = fy*M + fx,
 * M = n*ss, has coordinates (cx + (fx - (M-1)/2) h, cy + (fy - (M-1)/2) h),
 * h = pix_scale/ss, and lies in image pixel (fy/ss)*n + fx/ss (Sec. 2 pixel
 * centres; Sec. 4.1 supersampling and local averaging). */
typedef struct {
  int n;
  int ss;
  double pix_scale;
  double cx, cy;
} gpl_grid;

/* SPLE + external shear (Sec. 2.2): Einstein radius, axis ratio q in (0,1],
 * position angle phi (rad), power-law slope in (1,3), centre (x0, y0), shear. */
typedef struct {
  double theta_E, q, phi, slope, x0, y0, gamma1, gamma2;
} gpl_lens;

/* Circular Sersic mean function mu = I_e exp(-b_n ((r/R_e)^(1/n) - 1)),
 * r = |p - (xs, ys)| (mean function of Sec. 3.1, footnote). */
typedef struct {
  double I_e, R_e, n_sersic, b_n, xs, ys;
} gpl_source;

/* kind 0: RBF kernel k = amplitude^2 exp(-|x1-x2|^2 / (2 lengthscale^2))
 * (eq. "grbf", isotropic Sigma = lengthscale^2 I).
 * kind 1: pixel-shape (windowed) kernel of Sec. 3.2, eq. "covariance":
 * K_ij = amplitude^2 2 pi lengthscale^2 N(p_i - p_j, Z_i + Z_j + lengthscale^2 I),
 * Z_i = (a a^T + b b^T) / (4 pi) from the pixel axes a, b (half the distance
 * between the projected centres of the neighbouring grid points along each
 * grid axis; one-sided at the grid edges; eq. "window-kernel" and its
 * footnote); needs the grid (the points are its fine grid in row-major order),
 * runs in the FP32 form, and is accepted by gpl_gp_kernel_mvm and gpl_apply_A
 * (the other entry points take kind 0). */
typedef struct {
  int kind;
  double lengthscale, amplitude;
} gpl_kernel;

/* Gaussian PSF on the fine grid: FWHM in arcsec (0 = no PSF), taps radius in
 * fine pixels (0 = ceil(4 sigma / h)); 1-D taps normalised to unit sum, applied
 * separably with zero padding. radius <= GPL_PSF_MAX_RADIUS. */
typedef struct {
  double fwhm;
  int radius;
} gpl_psf;
#define GPL_PSF_MAX_RADIUS 24

/* One reconstruction: grid, kernel, PSF, noise and the ray-traced points
 * (device px, py of length (n*ss)^2). */
typedef struct {
  gpl_grid grid;
  gpl_kernel kernel;
  gpl_psf psf;
  double noise_sigma;
  const float* px;
  const float* py;
} gpl_problem;

const char* gpl_strerror(int code);
const char* gpl_last_error(void);
int gpl_version(void);

/* Half-light Sersic constant: root b of P(2n, b) = 1/2 (host, FP64). */
double gpl_sersic_bn(double n_sersic);

/* ---------------------------------------------------------------- forward */

/* Fine-grid coordinates and fine->pixel index map (grid convention above).
 * Outputs of length (n*ss)^2; any of the three may be NULL. */
int gpl_grid_map(const gpl_grid* grid, float* xi_x, float* xi_y, int* pixel_of_fine, hipStream_t stream);

/* Ray tracing p = xi - alpha_SPLE(xi) - Gamma xi (Sec. 2.1 eq. "lens", Sec. 2.2
 * eq. "dispsple" and the shear term) for every fine point of the grid. 2F1 is
 * summed from its series; alpha_SPLE is rotated back to the sky frame by -phi;
 * R is floored at 1e-9 arcsec. Writes px, py (length (n*ss)^2). */
int gpl_lens_raytrace(const gpl_grid* grid, const gpl_lens* lens, float* px, float* py, hipStream_t stream);

/* Sersic mean at n points: mu[i] = mu(px[i], py[i]). */
int gpl_sersic_eval(const gpl_source* src, int n, const float* px, const float* py, float* mu, hipStream_t stream);

/* Observation operator B = D o P and its adjoint, on nrhs columns.
 * adjoint = 0: in is fine (N rows, ld_in >= N), out = alpha * B in + beta * out
 *             with out image pixels (n*n rows, ld_out >= n*n).
 * adjoint = 1: in is image pixels, out = alpha * B^T in + beta * out (fine).
 * B^T = P^T D^T: D^T replicates a pixel value / ss^2 to its sub-pixels.
 * in and out must not overlap. */
int gpl_psf_conv(const gpl_grid* grid, const gpl_psf* psf, int nrhs, const float* in, int ld_in, float* out,
                 int ld_out, float alpha, float beta, int adjoint, hipStream_t stream);

/* Matrix-free kernel product Y = K V + beta * Y, K_ij = k(p_i, p_j) (eq. "grbf";
 * formed on demand, never stored, as in Sec. 3.3), over n points, nrhs columns
 * (V, Y column-major with ld >= n, device memory, must not overlap).
 * prec = GPL_PREC_FP32 or GPL_PREC_F16X3. beta is 0 (overwrite) or any float.
 * Pairs of 16-point subtiles and 32-point chunks whose bounding boxes are so far
 * apart that every kernel value is at most 2^-36 amplitude^2 are not evaluated:
 * in the precision form those values are exactly zero (the result equals the
 * all-pairs product up to FP32 summation order); in the FP32 form each dropped
 * term is below 2^-36 amplitude^2 |v_j|. The points are taken along a Hilbert
 * curve of their own positions (ties in caller order), so tiles are compact in
 * the plane the kernel is evaluated in; Y is returned in the caller's order.
 * grid (nullable): if given, n must equal its fine point count (the points are
 * then its fine grid in row-major order, as gpl_lens_raytrace writes them).
 * n <= 2,097,120. */
size_t gpl_gp_kernel_mvm_workspace(int n, int nrhs, int prec);
int gpl_gp_kernel_mvm(const gpl_kernel* kern, const gpl_grid* grid, int n, const float* px, const float* py, int nrhs,
                      const float* V, int ldv, float* Y, int ldy, float beta, int prec, void* ws, size_t ws_bytes,
                      hipStream_t stream);

/* Work of the product above for these points: *live_tiles = the (64-point row
 * tile, 32-point chunk) pairs it visits, *live_subtiles (nullable) = the
 * (16-point subtile, 32-point chunk) pairs it evaluates, 512 kernel values each
 * (the rest are below the cutoff), *live_lo (nullable) = those of the evaluated
 * pairs whose exp tile also needs its lo part in the precision form (equal to
 * *live_subtiles in the FP32 form). Host outputs; synchronises `stream`. A
 * measurement helper, not needed for the product itself. */
size_t gpl_gp_kernel_mvm_plan_workspace(int n);
int gpl_gp_kernel_mvm_plan_stats(const gpl_kernel* kern, const gpl_grid* grid, int n, const float* px,
                                 const float* py, int prec, long long* live_tiles, long long* live_subtiles,
                                 long long* live_lo, void* ws, size_t ws_bytes, hipStream_t stream);

/* Gaussian products with per-point shape covariances (Sec. 3.2 eq.
 * "covariance", Sec. 3.4 eq. "transmission", Sec. 3.5 eq. "gp-reconstruction"):
 *   Y[i][c] = beta Y[i][c] + norm wt_i sum_j ws_j |C_ij|^{-1/2} exp(-d^T C_ij^{-1} d / 2) V[j][c],
 *   d = (tx_i - sx_j, ty_i - sy_j),  C_ij = Zt_i + Zs_j + base_var I.
 * Targets (nt points tx, ty) and sources (ns points sx, sy) each take an
 * optional shape covariance tz / sz (NULL or three device arrays of n floats
 * stored one after another: zxx, zxy, zyy) and an optional weight tw / sw (NULL
 * = 1). V (ns x nrhs, ld ldv) and Y (nt x nrhs, ld ldy) must not overlap. The
 * windowed kernel is norm = amplitude^2 lengthscale^2, base_var =
 * lengthscale^2 with Z on both sides; the transmission T_ik = A_k N(p_i - q_k,
 * Z_i + lengthscale^2 I / 2) is norm = 1 / (2 pi), base_var = lengthscale^2 / 2,
 * tz = Z, sw = A; its transpose swaps the sides. Every pair is evaluated in
 * FP32. */
typedef struct {
  double base_var, norm;
} gpl_gauss;
int gpl_gauss_product(const gpl_gauss* g, int nt, const float* tx, const float* ty, const float* tz, const float* tw,
                      int ns, const float* sx, const float* sy, const float* sz, const float* sw, int nrhs,
                      const float* V, int ldv, float* Y, int ldy, float beta, hipStream_t stream);

/* Adjoint of one column of gpl_gauss_product for sources without shape
 * covariances: with F = sum_i U_i Y_i, Y = the product of V (one column, ns),
 * accumulates (+=, FP32, device) the gradients gtx/gty (nt, nullable pair) of
 * the target positions, gtz (3 x nt as for tz, nullable; needs tz) of the
 * target shapes as the symmetric matrix gradient (entries xx, xy, yy of
 * dF/dZ), gsx/gsy (ns, nullable pair) of the source positions and gsw (ns,
 * nullable) of the source weights. The derivatives of the normal density:
 * dN/dd = -N C^{-1} d, dN/dC = N (C^{-1} d d^T C^{-1} - C^{-1}) / 2. */
int gpl_gauss_product_backward(const gpl_gauss* g, int nt, const float* tx, const float* ty, const float* tz,
                               const float* tw, int ns, const float* sx, const float* sy, const float* sw,
                               const float* V, const float* U, float* gtx, float* gty, float* gtz, float* gsx,
                               float* gsy, float* gsw, hipStream_t stream);

/* The same Gaussian entries as gpl_gauss_product written out as a dense
 * nt x ns matrix M (column-major, ld ldm >= nt): M[j*ldm + i] = norm wt_i ws_j
 * |C_ij|^{-1/2} exp(-d^T C_ij^{-1} d / 2). With the RBF parameters (norm =
 * amplitude^2 lengthscale^2, base_var = lengthscale^2) and targets p, sources x,
 * column j is K(p, x_j), the cross-covariance that the posterior variance at x_j
 * (Sec. 3.7, eq. "gp-exact-var") needs. */
int gpl_gauss_matrix(const gpl_gauss* g, int nt, const float* tx, const float* ty, const float* tz, const float* tw,
                     int ns, const float* sx, const float* sy, const float* sz, const float* sw, float* M, int ldm,
                     hipStream_t stream);

/* Pixel shapes Z (three arrays of (n*ss)^2 floats: zxx, zxy, zyy) of the
 * ray-traced fine grid px, py (eq. "window-kernel", axes as for kind 1). */
int gpl_pixel_shapes(const gpl_grid* grid, const float* px, const float* py, float* z, hipStream_t stream);

/* Adjoint of gpl_pixel_shapes: gpx/gpy (+=) receive dF/dp from gz, the
 * symmetric matrix gradient dF/dZ per point (3 arrays xx, xy, yy). Workspace:
 * 16 (n ss)^2 bytes. */
int gpl_pixel_shapes_backward(const gpl_grid* grid, const float* px, const float* py, const float* gz, float* gpx,
                              float* gpy, void* ws, size_t ws_bytes, hipStream_t stream);

/* Density of the inducing points q for the transmission weights (Sec. 3.4,
 * footnote to eq. "transmission"): rho_i = k / (pi r_k^2), r_k the distance
 * from q_i to its k-th closest other point (1 <= k <= 32, n > k; squared
 * distances ranked in FP32, equal ones by the lower index). The points are
 * sorted along a Hilbert curve in the workspace and only 32-point chunks whose
 * bounding box lies within reach are visited. n <= 2,097,120. */
size_t gpl_knn_density_workspace(int n);
int gpl_knn_density(int n, const float* qx, const float* qy, int k, float* rho, void* ws, size_t ws_bytes,
                    hipStream_t stream);

/* Y = A X with A = B K B^T + noise_sigma^2 I (image pixels, nrhs columns). */
size_t gpl_apply_A_workspace(const gpl_problem* prob, int nrhs, int prec);
int gpl_apply_A(const gpl_problem* prob, int nrhs, const float* X, int ldx, float* Y, int ldy, int prec, void* ws,
                size_t ws_bytes, hipStream_t stream);

/* Conjugate gradients on A X = Bm, A = B K B^T + noise^2 I: the solves of the
 * evidence (Sec. 3.1, eq. "gp-mll": u = A^{-1} r for the quadratic term) and
 * of the probe vectors of the stochastic log-determinant, by the conjugate
 * gradient method Sec. 3.3 names for evaluating eq. "gp-mll" (as in GPyTorch,
 * with the CG coefficients giving the Lanczos tridiagonal of each probe).
 * One independent recurrence per column (x_0 = 0), all columns sharing each
 * product with A. FP32 vectors; dot products, alpha/beta recurrences and the
 * recorded coefficients in FP64.
 * Column c stops when |r|/|b| <= tol (recursive residual) or, if
 * fixed_iters > 0, after exactly fixed_iters steps; max_iter caps the count.
 * Outputs (device): X (n*n x nrhs, ld ldx), lanczos_ab [nrhs][n_lanczos][2]
 * (alpha_k, beta_k for the first n_lanczos steps; 0 beyond a column's count),
 * bnorm2[nrhs] = |b_c|^2, iters[nrhs], relres[nrhs] (recursive residual at
 * the stop), status[nrhs]; true_relres[nrhs] (nullable) = |b - A x|/|b| of the
 * returned iterate, from one more product with A after the last iteration.
 * check_every = 0: fully asynchronous; every iteration up to the cap is
 * enqueued and those after the last column has stopped return at once.
 * check_every > 0: the host waits (on events, never synchronising the device)
 * every check_every iterations for the number of active columns and stops
 * enqueueing once it is zero; this mode keeps two pinned host ints and two
 * events per host thread, created on first use and kept until the process ends. */
size_t gpl_cg_solve_workspace(const gpl_problem* prob, int nrhs, int prec);
int gpl_cg_solve(const gpl_problem* prob, int nrhs, const float* Bm, int ldb, float* X, int ldx, double tol,
                 int max_iter, int fixed_iters, int n_lanczos, double* lanczos_ab, double* bnorm2, int* iters,
                 double* relres, double* true_relres, int* status, int prec, int check_every, void* ws,
                 size_t ws_bytes, hipStream_t stream);

/* Stochastic Lanczos quadrature of ln|A|: the stochastic log-determinant that
 * Sec. 3.3 names for the ln|2 pi A| term of eq. "gp-mll" (Hutchinson probes,
 * Gauss quadrature from the Lanczos tridiagonal of each probe). Probe j uses the
 * first k_j = min(iters[j], n_lanczos) steps: the tridiagonal
 * T_kk = 1/a_k + b_{k-1}/a_{k-1}, T_{k,k+1} = sqrt(b_k)/a_k, and
 * contrib[j] = bnorm2[j] * e_1^T ln(T) e_1 (Gauss quadrature on T's Ritz
 * values), evaluated in FP64 from the integral representation
 * ln x = int e^s (1/(1+e^s) - 1/(x+e^s)) ds with the trapezoidal rule and
 * continued-fraction resolvents of T.
 * logdet = scale * sum_j contrib[j] + *offset (scale 1/nprobe for Hutchinson
 * probes, 1 for all unit vectors; offset a device scalar, nullable: ln|P| for
 * the preconditioned estimate below); stderr = scale * sqrt(nprobe) * sd(contrib).
 * lanczos_ab, iters, bnorm2 as written by gpl_cg_solve (probe columns only);
 * n_lanczos <= 4096. Outputs (device): contrib[nprobe], logdet[1], stderr[1].
 * A probe whose tridiagonal is not positive definite contributes NaN.
 * The workspace size is 0 (ws may be NULL). */
size_t gpl_lanczos_logdet_workspace(int nprobe, int n_lanczos);
int gpl_lanczos_logdet(int nprobe, int n_lanczos, const double* lanczos_ab, const int* iters, const double* bnorm2,
                       double scale, const double* offset, double* contrib, double* logdet, double* stderr_out,
                       void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------- preconditioned evidence
 * The stochastic log-determinant of eq. "gp-mll" carries a noise Sec. 3.3
 * names as the reason the paper avoids it (1-2% in GPyTorch). GPyTorch, which
 * Sec. 3.3 cites for CG and that estimate, lowers the noise and the iteration
 * count with a preconditioner P = L L^T + sigma^2 I from a partial pivoted
 * Cholesky factor L of M = B K B^T (Gardner et al. 2018): ln|A| = ln|P| +
 * ln|P^{-1/2} A P^{-1/2}|, the first term exact by the determinant lemma, the
 * second estimated by SLQ on preconditioned CG with probes z ~ N(0, P).
 *
 * gpl_pchol: L (n*n x k, FP64, column-major, ld ldl) with k a multiple of 64,
 * built 64 pivots at a time. The candidates of a block are the 64 largest
 * entries of the residual diagonal of M - L L^T (ranked in FP32, ties by lower
 * pixel index); their columns of M come from the matrix-free product applied
 * to unit vectors (in precision `prec`), minus L L^T; a pivoted Cholesky of
 * the 64 x 64 residual block takes them largest-first while the residual
 * pivot exceeds 1e-5 of the largest diagonal entry of M (below that the FP32
 * columns are rounding noise). pivots[j] = the pixel
 * of column j, -1 for a zero column (a candidate not taken). G (k x k, ld ldg)
 * receives the inverse of sigma^2 I + L^T L (both triangles), built by
 * bordering in 64 x 64 blocks (Schur complements and their Cholesky factors);
 * logdet_P (device scalar) = ln|P| = (n*n - k) ln sigma^2 + ln|sigma^2 I + L^T L|
 * from those factors; info (device) = 0, or 1 + the index of the first pivot of
 * a Schur complement found not positive (the outputs are then meaningless).
 * noise_sigma > 0. Part of the work runs on a second stream of the calling
 * thread; it starts after the work already enqueued on `stream` and `stream`
 * waits for it before anything enqueued after this call. */
size_t gpl_pchol_workspace(const gpl_problem* prob, int k, int prec);
int gpl_pchol(const gpl_problem* prob, int k, int prec, double* L, int ldl, double* G, int ldg, int* pivots,
              double* logdet_P, int* info, void* ws, size_t ws_bytes, hipStream_t stream);

/* Probes z_j = L g_j + noise_sigma h_j, distributed as N(0, P) for standard
 * normals g (k x m, FP64, ld ldg) and h (n*n x m, FP32, ld ldh) supplied by the
 * caller; Z (n*n x m, FP32, ld ldz). */
size_t gpl_pchol_probes_workspace(int npix, int m);
int gpl_pchol_probes(int npix, int k, const double* L, int ldl, double noise_sigma, int m, const double* g, int ldg,
                     const float* h, int ldh, float* Z, int ldz, void* ws, size_t ws_bytes, hipStream_t stream);

/* Preconditioned CG on A X = Bm with P from gpl_pchol (L, G as written there):
 * z = P^{-1} r by the Woodbury identity (FP64 products: L^T r, one symmetric
 * product with G's lower triangle, L times that), alpha = r.z/p.Ap,
 * beta = r'.z'/r.z, p = z' + beta p; one recurrence per column, FP32 vectors,
 * FP64 scalars. Outputs as gpl_cg_solve, with rz0[c] = b_c^T P^{-1} b_c (the
 * quadrature weight of a probe column) in place of |b|^2: pass rz0 as
 * `bnorm2`, scale 1/m and offset ln|P| to gpl_lanczos_logdet for the
 * preconditioned estimate of ln|A|. Stops on the recursive residual |r|/|b|;
 * check_every as in gpl_cg_solve. */
size_t gpl_pcg_solve_workspace(const gpl_problem* prob, int k, int nrhs, int prec);
int gpl_pcg_solve(const gpl_problem* prob, int k, const double* L, int ldl, const double* G, int ldg, int nrhs,
                  const float* Bm, int ldb, float* X, int ldx, double tol, int max_iter, int fixed_iters,
                  int n_lanczos, double* lanczos_ab, double* rz0, int* iters, double* relres, double* true_relres,
                  int* status, int prec, int check_every, void* ws, size_t ws_bytes, hipStream_t stream);

/* Evidence scalars (Sec. 3.1 eq. "gp-mll" with the sign reading
 * -2 ln p = r^T A^{-1} r + ln|2 pi A|; App. D.1 eq. "hyper-loss"):
 * out[0] = quad = r . u, out[1] = ln p = -(quad + logdet + n_pix ln 2 pi)/2,
 * out[2] = L_VI = quad + n_points ln(amplitude^2 + noise_sigma^2).
 * r, u of length n_pix (device), logdet device scalar. */
int gpl_evidence_scalars(int n_pix, int n_points, const float* r, const float* u, const double* logdet,
                         double amplitude, double noise_sigma, double* out, hipStream_t stream);

/* Amplitude derivatives of the evidence and of the App. D.1 loss, from the
 * identity alpha dA/dalpha = 2 (A - sigma^2 I) (K is proportional to alpha^2):
 * out[0] = d ln p/d alpha = ((quad - sigma^2 u.u) - scale sum_j (|z_j|^2 - sigma^2 z_j.x_j)) / alpha,
 * the second term the probe estimate of tr(A^{-1} B K B^T) (Sec. 3.1 eq.
 * "gp-mll" differentiated; Sec. 3.3 stochastic trace), x_j = A^{-1} z_j;
 * out[1] = d L_VI/d alpha = -2 (quad - sigma^2 u.u)/alpha + 2 n_points alpha/(alpha^2 + sigma^2)
 * (App. D.1 eq. "hyper-loss"). u = A^{-1} r (n_pix), Z and X the probe columns
 * and their solves (ld >= n_pix; nprobe may be 0), quad a device scalar
 * (r.u, as gpl_evidence_scalars writes it), scale the probe weight (1/nprobe
 * for Hutchinson probes, 1 for all unit vectors). FP64 dot products. */
int gpl_evidence_amplitude_grad(int n_pix, int n_points, int nprobe, const float* u, const float* Z, int ldz,
                                const float* X, int ldx, const double* quad, double scale, double amplitude,
                                double noise_sigma, double* out, hipStream_t stream);

/* Posterior variance from solved columns (Sec. 3.7, eq. "gp-exact-var" with
 * the observation operator): out[c] = prior - sum_i W[c*ldw + i] X[c*ldx + i]
 * in FP64, c < ncols, i < n, for W = B K(p, x_c) and X = A^{-1} W; prior =
 * k(x_c, x_c) (amplitude^2 for the RBF). */
int gpl_posterior_variance(int n, int ncols, const float* W, int ldw, const float* X, int ldx, double prior,
                           double* out, hipStream_t stream);

/* Column-wise dot products in FP64: out[c] = sum_i X[c*ldx + i] * Y[c*ldy + i],
 * c < ncols, i < n. Used for quadratic forms and trace estimates
 * (z_j . A^{-1} z_j) of the evidence and its gradient. */
int gpl_block_dot(int n, int ncols, const float* X, int ldx, const float* Y, int ldy, double* out,
                  hipStream_t stream);

/* Opt-in timing of the kernel-product launches (main product kernel only, not
 * its preparation or reduction), for measuring achieved rates. With stride
 * k >= 1, every k-th such launch on this host thread (counted from the enable
 * call) is bracketed by HIP events recorded on its stream; 0 turns timing off.
 * Each event pair delays the stream by a few microseconds, so a stride above 1
 * keeps timed runs close to untimed ones. gpl_timing_read waits for the
 * recorded events (host wait, no device synchronisation) and returns the summed
 * elapsed milliseconds and number of timed launches since the last reset;
 * gpl_timing_samples copies up to `cap` of the per-launch times (ms, in launch
 * order) to host memory `ms` and sets *count to how many there are. Both reset
 * the samples if `reset` is non-zero. */
int gpl_timing_enable(int stride);
int gpl_timing_read(double* total_ms, long* launches, int reset);
int gpl_timing_samples(float* ms, int cap, int* count, int reset);

/* ---------------------------------------------------------------- backward */

/* Gradient of F = sum_c w[c] a_c^T K b_c (a_c, b_c columns of A and Bv, n rows)
 * with respect to the points, the lengthscale and the amplitude, kernel tiles
 * recomputed: gpx[i] += dF/dpx_i, gpy[i] += dF/dpy_i (FP32, accumulated),
 * g_hyp[0] = dF/d lengthscale, g_hyp[1] = dF/d amplitude (FP64, overwritten).
 * w is a HOST array of npairs weights. The points are sorted as for the product
 * (a tile plan is built in the workspace, so n is bounded as there), and pairs
 * whose FP32 kernel value is exactly zero are skipped. */
size_t gpl_gp_kernel_mvm_backward_workspace(int n, int npairs);
int gpl_gp_kernel_mvm_backward(const gpl_kernel* kern, int n, const float* px, const float* py, int npairs,
                               const float* A, int lda, const float* Bv, int ldb, const double* w, float* gpx,
                               float* gpy, double* g_hyp, void* ws, size_t ws_bytes, hipStream_t stream);

/* Adjoint of ray tracing: g_lens[k] = sum_i (dp_i/dtheta_k) . (gpx_i, gpy_i) for
 * theta = (theta_E, q, phi, slope, x0, y0, gamma1, gamma2) (FP64, overwritten).
 * Per-point Jacobians come from forward-mode derivatives through the series. */
size_t gpl_lens_raytrace_backward_workspace(const gpl_grid* grid);
int gpl_lens_raytrace_backward(const gpl_grid* grid, const gpl_lens* lens, const float* gpx, const float* gpy,
                               double* g_lens, void* ws, size_t ws_bytes, hipStream_t stream);

/* Allocation-free form of gpl_lens_raytrace_backward, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same kernels and the same result
 * (bitwise), with the partial sums in a static device array of 1 MiB that each
 * device holds from its first call until the process ends. No workspace
 * argument; nothing is allocated. Grids of more than 4,194,304 fine points
 * ((n ss)^2) are rejected with GPL_EINVAL. Every call on one device shares that
 * array and overwrites it completely before reading it, so calls that overlap
 * in time on one device (different streams, several host threads) race. */
int gpl_lens_raytrace_backward_noalloc(const gpl_grid* grid, const gpl_lens* lens, const float* gpx,
                                       const float* gpy, double* g_lens, hipStream_t stream);

/* Adjoint of the Sersic mean: gpx[i] += gmu[i] dmu_i/dpx, gpy[i] += gmu[i] dmu_i/dpy,
 * g_src[0..1] = d/d(xs, ys) of sum_i gmu[i] mu_i (FP64, overwritten). */
size_t gpl_sersic_backward_workspace(int n);
int gpl_sersic_backward(const gpl_source* src, int n, const float* px, const float* py, const float* gmu, float* gpx,
                        float* gpy, double* g_src, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------- variational GP source
 * The paper's fitting loop (Sec. 3.3-3.7, 4.2, 4.3): the source is a sum of
 * GP layers written as transmission products (Sec. 3.3 eqs. "gp-gen2",
 * "decomposition"; Sec. 3.4 eq. "transmission"):
 *   f = mu(p) + sum_k T_k y_k,  T_k[i][j] = A_j N(p_i - q_j, Zt_i + l_k^2 I / 2),
 *   A_j = sqrt(2 pi l_k^2) / sqrt(rho(q_j)),  rho = knn_k / (pi r^2),
 * r the distance from q_j to its knn_k-th closest other inducing point. An
 * image-plane layer (GPL_VIGP_IMAGE_PLANE) uses the traced points as inducing
 * points (q = p) and their pixel shapes Zt (eq. "window-kernel"); the
 * source-plane layer (GPL_VIGP_SOURCE_PLANE, at most one, Sec. 3.5) uses a
 * fixed grid of G points and no shapes. Data d ~ N(B f, noise_sigma^2 I), prior
 * y_k ~ N(0, alpha_k^2 I); lens prior: uniform boxes on theta_E, q, phi, x0, y0
 * (prior_lo/hi) and N(0, shear_sd^2) on each shear component (Table
 * "lens-params"). The slope, the Sersic mean and the noise are fixed.
 *
 * Guide (Sec. 4.2 eq. "guide", Table "gparams"): the 7 free lens parameters
 * (theta_E, q, phi, x0, y0, gamma1, gamma2) and the source-plane parameters are
 * jointly normal with scale [[L_l, 0], [C, diag(s_sp)]]; image-plane layers are
 * diagonal normals; the amplitudes alpha_k are point estimates. Positive
 * quantities are held as logarithms.
 *
 * Parameter blocks (device):
 *   P64 (n64 = 56 + n_layers doubles): [0, 7) lens mean m_l; [7, 56) L_l raw,
 *     row-major 7 x 7: entries below the diagonal as they are, diagonal entries
 *     as ln L_l[a][a], entries above ignored; [56, 56 + n_layers) ln alpha_k.
 *   P32 (n32 floats): the source-plane layer first (if any): m_sp (G), ln s_sp
 *     (G), C (G x 7, column b at offset 2G + bG); then each image-plane layer
 *     in layer order: m_k (N), ln s_k (N), N = (n ss)^2.
 *   Noise of one sample (standard normals, drawn by the caller): e64 (7 doubles,
 *     e_l) and e32 (ne32 floats: e_sp (G) first, then e_k (N) per image-plane
 *     layer in layer order).
 * gpl_vigp_elbo: one reparametrised sample (Sec. 3.6 eq. "reparam")
 *   theta = m_l + L_l e_l, y_sp = m_sp + C e_l + s_sp e_sp, y_k = m_k + s_k e_k,
 * and the ELBO sample (eq. "elbo") E = ln N(d | B f) + sum_k ln N(y_k | 0, alpha_k^2)
 * + ln p(theta) - ln q(theta, y); out (device, 13 doubles): E, ln N(d | B f),
 * sum_k ln p(y_k), ln p(theta) (-inf outside the boxes), -ln q, then the
 * sampled 8-vector theta (gpl_lens order). G64 / G32 (device, shaped like
 * P64 / P32) receive dE/dparameter (entries of L_l above the diagonal: 0),
 * through the traced points, their pixel shapes and the k-NN weights of
 * image-plane inducing points (each point's k-th neighbour held at its current
 * index; its share is added with FP64 atomics, so the last FP32 bit of a
 * gradient may vary between runs). All products are dense Gaussian products
 * (every pair in FP32), FP64 sums for the scalars. */
#define GPL_VIGP_IMAGE_PLANE 0
#define GPL_VIGP_SOURCE_PLANE 1
typedef struct {
  int n_layers;              /* 1..8 */
  int kind[8];               /* GPL_VIGP_IMAGE_PLANE or GPL_VIGP_SOURCE_PLANE */
  double lengthscale[8];     /* l_k, arcsec */
  int knn_k;                 /* neighbours of the density estimate (Sec. 3.4: 20), 1..32 */
  double slope;              /* fixed SPLE slope */
  double prior_lo[5], prior_hi[5]; /* boxes for theta_E, q, phi, x0, y0 */
  double shear_sd;           /* prior standard deviation of gamma1, gamma2 */
} gpl_vigp_model;
int gpl_vigp_sizes(const gpl_vigp_model* model, const gpl_grid* grid, int G, size_t* n64, size_t* n32,
                   size_t* ne32);
size_t gpl_vigp_workspace(const gpl_vigp_model* model, const gpl_grid* grid, int G);
int gpl_vigp_elbo(const gpl_vigp_model* model, const gpl_grid* grid, const gpl_psf* psf, const gpl_source* src,
                  double noise_sigma, int G, const float* gx, const float* gy, const float* d, const double* P64,
                  const float* P32, const double* e64, const float* e32, double* out, double* G64, float* G32,
                  void* ws, size_t ws_bytes, hipStream_t stream);

/* One Adam step (Sec. 4.3: torch's Adam; Kingma & Ba 2015) on both parameter
 * blocks minimising -E, i.e. with loss gradient -G: m = b1 m + (1 - b1) g,
 * v = b2 v + (1 - b2) g^2, p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
 * elementwise (FP64 for the P64 block, FP32 for P32); t >= 1 is the step
 * number; M*, V* hold the moments (zero before the first step). */
int gpl_vigp_adam(size_t n64, double* P64, const double* G64, double* M64, double* V64, size_t n32, float* P32,
                  const float* G32, float* M32, float* V32, int t, double lr, double beta1, double beta2, double eps,
                  hipStream_t stream);

/* ---------------------------------------------------------------- serving
 * A continuous-batching request loop keeps every admitted reconstruction (a
 * slot) resident in its own device workspace: points, residual and probe
 * columns, CG vectors and state, Lanczos coefficients. gpl_serve_step advances
 * any set of slots by a number of CG iterations; each stage of an iteration is
 * ONE grouped launch over the tiles of all those slots, so requests of uneven
 * sizes share the device. Results of a slot do not depend on which other slots
 * it is batched with (bitwise). Iteration counters are global: iteration k of
 * the loop uses state parity k & 1, and a slot may join at any k. */
typedef struct {
  void* ws;       /* the slot's device workspace (set by init) */
  void* dev;      /* device address of the slot descriptor inside ws (set by init) */
  int N, npix, nrhs;
  unsigned char opaque[1024]; /* host copy of the descriptor (library use) */
} gpl_serve_slot;

/* Bytes of device workspace of one slot (nrhs <= 32 columns: the solve column
 * plus nrhs - 1 probes). This is the slot's HBM footprint for admission. */
size_t gpl_serve_slot_workspace(const gpl_grid* grid, int nrhs, int n_lanczos, int prec);

/* Admit one request into `ws`: ray tracing, Sersic mean, residual d - B mu in
 * column 0, probes (nrhs - 1 columns, ld ldz) after it, CG initial state. prob
 * supplies grid, kernel, PSF and noise (its px/py are ignored). Enqueued on
 * `stream`; d and probes may be reused once the stream has passed this call. */
int gpl_serve_slot_init(gpl_serve_slot* slot, const gpl_problem* prob, const gpl_lens* lens, const gpl_source* src,
                        const float* d, const float* probes, int ldz, int nrhs, double tol, int max_iter,
                        int n_lanczos, int prec, void* ws, size_t ws_bytes, hipStream_t stream);

/* Advance the slots (host array of nslots <= 64 pointers) by `iters` CG
 * iterations, the first being global iteration iter0. Slots whose columns have
 * all stopped do no work. */
int gpl_serve_step(gpl_serve_slot* const* slots, int nslots, int iters, long iter0, hipStream_t stream);

/* Write each slot's number of still-active columns after global iteration
 * `iter` - 1 (i.e. at parity iter & 1) to host_active[s], a host buffer the
 * device can write (pinned, mapped). Read it after the stream passes this call. */
int gpl_serve_snapshot(gpl_serve_slot* const* slots, int nslots, long iter, int* host_active, hipStream_t stream);

/* Finish a slot whose columns have stopped, `iter` being the global iteration
 * count reached: out[0..4] = quad, ln p, L_VI, ln|A| (SLQ, scale logdet_scale),
 * its standard error; iters/relres/status per column (device, nrhs entries);
 * optionally the posterior mean fhat (N) and the predicted image (n*n). */
int gpl_serve_slot_finish(gpl_serve_slot* slot, long iter, double logdet_scale, double* out, int* iters,
                          double* relres, int* status, float* fhat, float* image, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* GPLENS_H */

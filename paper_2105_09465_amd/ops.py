"""Thin torch-facing wrappers over the gplens C-ABI.

Blocks of column vectors are torch tensors of shape (ncols, rows) on the GPU:
row k is column k of the column-major block, and the leading dimension is the
tensor's stride(0). Each wrapper checks shapes, allocates outputs and workspace
with torch (device memory only), and passes pointers plus torch's current HIP
stream to the library. No arithmetic happens here.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from .params import Grid, Kernel, Lens, Problem, PSF, Sersic

PREC = {"fp32": _lib.PREC_FP32, "f16x3": _lib.PREC_F16X3}


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor, dtype=None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("gplens expects GPU tensors")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return C.c_void_p(t.data_ptr())


def _block(t: torch.Tensor, rows: int, name: str):
    if t.dim() != 2 or t.shape[1] != rows or t.stride(1) != 1:
        raise ValueError(f"{name}: expected a (ncols, {rows}) tensor with unit stride along rows, got "
                         f"{tuple(t.shape)} strides {t.stride()}")
    if t.dtype != torch.float32:
        raise TypeError(f"{name}: expected float32")
    return t.stride(0) if t.shape[0] > 1 else max(t.stride(0), rows)


def workspace(nbytes: int, device=None):
    if nbytes == 0:
        return None, 0
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device or "cuda"), int(nbytes)


def _wsptr(ws):
    return None if ws is None else C.c_void_p(ws.data_ptr())


def prec_code(prec):
    return PREC[prec] if isinstance(prec, str) else int(prec)


# ------------------------------------------------------------------ forward

def grid_map(grid: Grid, device="cuda"):
    x = torch.empty(grid.N, dtype=torch.float32, device=device)
    y = torch.empty_like(x)
    pix = torch.empty(grid.N, dtype=torch.int32, device=device)
    g = grid.c()
    _lib.call("gpl_grid_map", C.byref(g), _ptr(x), _ptr(y), _ptr(pix), _stream())
    return x, y, pix


def lens_raytrace(grid: Grid, lens: Lens, out=None, device="cuda"):
    if out is None:
        out = torch.empty(2, grid.N, dtype=torch.float32, device=device)
    g, L = grid.c(), lens.c()
    _lib.call("gpl_lens_raytrace", C.byref(g), C.byref(L), _ptr(out[0]), _ptr(out[1]), _stream())
    return out


def sersic_eval(src: Sersic, px, py, out=None):
    n = px.numel()
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=px.device)
    s = src.c()
    _lib.call("gpl_sersic_eval", C.byref(s), n, _ptr(px), _ptr(py), _ptr(out), _stream())
    return out


def psf_conv(grid: Grid, psf: PSF, inp, adjoint: bool, out=None, alpha=1.0, beta=0.0):
    """adjoint=False: B inp (fine -> image); True: B^T inp (image -> fine)."""
    rows_in, rows_out = (grid.n_pix, grid.N) if adjoint else (grid.N, grid.n_pix)
    squeeze = inp.dim() == 1
    inp2 = inp.unsqueeze(0) if squeeze else inp
    ld_in = _block(inp2, rows_in, "inp")
    if out is None:
        out = torch.zeros(inp2.shape[0], rows_out, dtype=torch.float32, device=inp.device)
        ld_out = rows_out
        ret = out
    else:
        ret = out
        out = out.unsqueeze(0) if out.dim() == 1 else out
        ld_out = _block(out, rows_out, "out")
    g, p = grid.c(), psf.c()
    _lib.call("gpl_psf_conv", C.byref(g), C.byref(p), inp2.shape[0], _ptr(inp2), ld_in, _ptr(out), ld_out,
              float(alpha), float(beta), 1 if adjoint else 0, _stream())
    return ret[0] if (squeeze and ret.dim() == 2) else ret


def kernel_mvm(kernel: Kernel, px, py, V, prec="fp32", out=None, beta=0.0, grid: Grid | None = None):
    """Y = K V (+ beta Y) over the points (px, py); grid (optional): the points
    are that grid's fine points in row-major order (checked against n)."""
    n = px.numel()
    squeeze = V.dim() == 1
    V2 = V.unsqueeze(0) if squeeze else V
    ldv = _block(V2, n, "V")
    if out is None:
        out = torch.zeros(V2.shape[0], n, dtype=torch.float32, device=V.device)
    out2 = out.unsqueeze(0) if out.dim() == 1 else out
    ldy = _block(out2, n, "Y")
    pc = prec_code(prec)
    ws, wsb = workspace(_lib.lib.gpl_gp_kernel_mvm_workspace(n, V2.shape[0], pc), V.device)
    k = kernel.c()
    g = C.byref(grid.c()) if grid is not None else None
    _lib.call("gpl_gp_kernel_mvm", C.byref(k), g, n, _ptr(px), _ptr(py), V2.shape[0], _ptr(V2), ldv, _ptr(out2), ldy,
              float(beta), pc, _wsptr(ws), wsb, _stream())
    return out[0] if (squeeze and out.dim() == 2) else out


def gauss_product(base_var, norm, tx, ty, sx, sy, V, tz=None, tw=None, sz=None, sw=None, out=None, beta=0.0):
    """Y[i] = beta Y[i] + norm wt_i sum_j ws_j |C_ij|^{-1/2} exp(-d^T C_ij^{-1} d / 2) V[j], C_ij = Zt_i + Zs_j +
    base_var I, d = t_i - s_j: targets (tx, ty), sources (sx, sy); V (ncols, ns); shapes tz/sz as (3, n)
    (zxx, zxy, zyy), weights tw/sw (n,), all float32 on the GPU."""
    nt, ns = tx.numel(), sx.numel()
    squeeze = V.dim() == 1
    V2 = V.unsqueeze(0) if squeeze else V
    ldv = _block(V2, ns, "V")
    if out is None:
        out = torch.zeros(V2.shape[0], nt, dtype=torch.float32, device=V.device)
    out2 = out.unsqueeze(0) if out.dim() == 1 else out
    ldy = _block(out2, nt, "Y")
    g = _lib.gpl_gauss(float(base_var), float(norm))
    for z, n in ((tz, nt), (sz, ns)):
        if z is not None and (tuple(z.shape) != (3, n) or not z.is_contiguous()):
            raise ValueError("shape covariances must be contiguous (3, n) tensors")
    _lib.call("gpl_gauss_product", C.byref(g), nt, _ptr(tx), _ptr(ty), _ptr(tz), _ptr(tw), ns, _ptr(sx), _ptr(sy),
              _ptr(sz), _ptr(sw), V2.shape[0], _ptr(V2), ldv, _ptr(out2), ldy, float(beta), _stream())
    return out[0] if (squeeze and out.dim() == 2) else out


def gauss_matrix(base_var, norm, tx, ty, sx, sy, tz=None, tw=None, sz=None, sw=None, out=None):
    """Dense Gaussian entries as a (ns, nt) float32 tensor: row j is column j of
    the nt x ns matrix M_ij = norm wt_i ws_j |C_ij|^{-1/2} exp(-d^T C_ij^{-1} d / 2)."""
    nt, ns = tx.numel(), sx.numel()
    if out is None:
        out = torch.empty(ns, nt, dtype=torch.float32, device=tx.device)
    ldm = _block(out, nt, "M")
    for z, n in ((tz, nt), (sz, ns)):
        if z is not None and (tuple(z.shape) != (3, n) or not z.is_contiguous()):
            raise ValueError("shape covariances must be contiguous (3, n) tensors")
    g = _lib.gpl_gauss(float(base_var), float(norm))
    _lib.call("gpl_gauss_matrix", C.byref(g), nt, _ptr(tx), _ptr(ty), _ptr(tz), _ptr(tw), ns, _ptr(sx), _ptr(sy),
              _ptr(sz), _ptr(sw), _ptr(out), ldm, _stream())
    return out


def pixel_shapes(grid: Grid, px, py):
    """Pixel-shape covariances (3, N): zxx, zxy, zyy of the ray-traced fine grid."""
    z = torch.empty(3, grid.N, dtype=torch.float32, device=px.device)
    g = grid.c()
    _lib.call("gpl_pixel_shapes", C.byref(g), _ptr(px), _ptr(py), _ptr(z), _stream())
    return z


def knn_density(qx, qy, k=20):
    """k-th closest neighbour density of the points (q_x, q_y)."""
    n = qx.numel()
    rho = torch.empty(n, dtype=torch.float32, device=qx.device)
    ws, wsb = workspace(_lib.lib.gpl_knn_density_workspace(n), qx.device)
    _lib.call("gpl_knn_density", n, _ptr(qx), _ptr(qy), int(k), _ptr(rho), _wsptr(ws), wsb, _stream())
    return rho


def kernel_mvm_live_tiles(kernel: Kernel, px, py, prec="fp32", grid: Grid | None = None, with_lo=False):
    """Work of the product for these points: (64-point row tile, 32-point chunk)
    pairs visited and (16-point subtile, 32-point chunk) pairs evaluated (512
    kernel values each), and with with_lo also those evaluated pairs that need
    the lo part of the exp tile in the precision form; synchronises the stream."""
    n = px.numel()
    ws, wsb = workspace(_lib.lib.gpl_gp_kernel_mvm_plan_workspace(n), px.device)
    tiles, subtiles, lo = C.c_longlong(0), C.c_longlong(0), C.c_longlong(0)
    k = kernel.c()
    g = C.byref(grid.c()) if grid is not None else None
    _lib.call("gpl_gp_kernel_mvm_plan_stats", C.byref(k), g, n, _ptr(px), _ptr(py), prec_code(prec), C.byref(tiles),
              C.byref(subtiles), C.byref(lo), _wsptr(ws), wsb, _stream())
    if with_lo:
        return int(tiles.value), int(subtiles.value), int(lo.value)
    return int(tiles.value), int(subtiles.value)


def problem_c(problem: Problem, px, py):
    return _lib.gpl_problem(problem.grid.c(), problem.kernel.c(), problem.psf.c(), problem.noise_sigma,
                            C.c_void_p(px.data_ptr()), C.c_void_p(py.data_ptr()))


def apply_A(problem: Problem, px, py, X, prec="fp32"):
    npix = problem.grid.n_pix
    ldx = _block(X, npix, "X")
    Y = torch.empty(X.shape[0], npix, dtype=torch.float32, device=X.device)
    pc = prec_code(prec)
    pr = problem_c(problem, px, py)
    ws, wsb = workspace(_lib.lib.gpl_apply_A_workspace(C.byref(pr), X.shape[0], pc), X.device)
    _lib.call("gpl_apply_A", C.byref(pr), X.shape[0], _ptr(X), ldx, _ptr(Y), npix, pc, _wsptr(ws), wsb, _stream())
    return Y


def cg_solve(problem: Problem, px, py, Bm, tol=1e-6, max_iter=1000, fixed_iters=0, n_lanczos=30, prec="fp32",
             check_every=8, ws=None, true_residual=True):
    """CG on A X = Bm for every column of Bm (ncols, n_pix). Returns device tensors.
    check_every = 0 enqueues every iteration up to the cap without any host
    wait; k > 0 lets the library wait for the active count every k iterations
    and stop enqueueing once all columns have stopped. true_residual adds
    |b - A x|/|b| of the returned iterate (one more product with A)."""
    npix = problem.grid.n_pix
    ldb = _block(Bm, npix, "Bm")
    m = Bm.shape[0]
    dev = Bm.device
    X = torch.empty(m, npix, dtype=torch.float32, device=dev)
    nl = max(int(n_lanczos), 0)
    ab = torch.zeros(m, max(nl, 1), 2, dtype=torch.float64, device=dev)
    bnorm2 = torch.empty(m, dtype=torch.float64, device=dev)
    iters = torch.empty(m, dtype=torch.int32, device=dev)
    relres = torch.empty(m, dtype=torch.float64, device=dev)
    true_relres = torch.empty(m, dtype=torch.float64, device=dev) if true_residual else None
    status = torch.empty(m, dtype=torch.int32, device=dev)
    pc = prec_code(prec)
    pr = problem_c(problem, px, py)
    need = _lib.lib.gpl_cg_solve_workspace(C.byref(pr), m, pc)
    if ws is None or ws.numel() < need:
        ws, _ = workspace(need, dev)
    _lib.call("gpl_cg_solve", C.byref(pr), m, _ptr(Bm), ldb, _ptr(X), npix, float(tol), int(max_iter),
              int(fixed_iters), nl, _ptr(ab), _ptr(bnorm2), _ptr(iters), _ptr(relres), _ptr(true_relres),
              _ptr(status), pc, int(check_every), _wsptr(ws), int(need), _stream())
    return dict(X=X, ab=ab[:, :nl], bnorm2=bnorm2, iters=iters, relres=relres, true_relres=true_relres,
                status=status, n_lanczos=nl)


def lanczos_logdet(ab, iters, bnorm2, scale, offset=None):
    """SLQ log-determinant from CG coefficients of the probe columns (plus a
    device scalar offset, e.g. ln|P| of a preconditioner)."""
    m, nl = ab.shape[0], ab.shape[1]
    ab = ab.contiguous()
    dev = ab.device
    contrib = torch.empty(m, dtype=torch.float64, device=dev)
    logdet = torch.empty(1, dtype=torch.float64, device=dev)
    stderr = torch.empty(1, dtype=torch.float64, device=dev)
    ws, wsb = workspace(_lib.lib.gpl_lanczos_logdet_workspace(m, nl), dev)
    _lib.call("gpl_lanczos_logdet", m, nl, _ptr(ab), _ptr(iters.contiguous()), _ptr(bnorm2.contiguous()),
              float(scale), _ptr(offset, torch.float64) if offset is not None else None, _ptr(contrib),
              _ptr(logdet), _ptr(stderr), _wsptr(ws), wsb, _stream())
    return logdet, stderr, contrib


def pchol(problem: Problem, px, py, k, prec="f16x3"):
    """Partial pivoted Cholesky preconditioner of A: dict with L (k, n_pix)
    float64 (column j of L is row j), G (k, k) the factor of sigma^2 I + L^T L
    (column-major: row j of the tensor is column j), pivots (k,), logdet_P and
    info (device scalars)."""
    npix = problem.grid.n_pix
    dev = px.device
    L = torch.empty(k, npix, dtype=torch.float64, device=dev)
    Gm = torch.empty(k, k, dtype=torch.float64, device=dev)
    piv = torch.empty(k, dtype=torch.int32, device=dev)
    ldp = torch.empty(1, dtype=torch.float64, device=dev)
    info = torch.empty(1, dtype=torch.int32, device=dev)
    pc = prec_code(prec)
    pr = problem_c(problem, px, py)
    ws, wsb = workspace(_lib.lib.gpl_pchol_workspace(C.byref(pr), k, pc), dev)
    _lib.call("gpl_pchol", C.byref(pr), int(k), pc, _ptr(L), npix, _ptr(Gm), k, _ptr(piv), _ptr(ldp), _ptr(info),
              _wsptr(ws), wsb, _stream())
    return dict(L=L, G=Gm, pivots=piv, logdet_P=ldp, info=info, k=int(k))


def pchol_probes(pc: dict, noise_sigma, g, h):
    """Probes z = L g + sigma h for normals g (m, k) float64 and h (m, n_pix)
    float32 on the device; returns (m, n_pix) float32."""
    L = pc["L"]
    k, npix = L.shape
    m = g.shape[0]
    Z = torch.empty(m, npix, dtype=torch.float32, device=L.device)
    ws, wsb = workspace(_lib.lib.gpl_pchol_probes_workspace(npix, m), L.device)
    _lib.call("gpl_pchol_probes", npix, k, _ptr(L), npix, float(noise_sigma), m, _ptr(g.contiguous(), torch.float64),
              k, _ptr(h.contiguous(), torch.float32), npix, _ptr(Z), npix, _wsptr(ws), wsb, _stream())
    return Z


def pcg_solve(problem: Problem, px, py, pc: dict, Bm, tol=1e-6, max_iter=1000, fixed_iters=0, n_lanczos=30,
              prec="f16x3", check_every=2, ws=None, true_residual=True):
    """Preconditioned CG on A X = Bm (ncols, n_pix) with the factor from pchol().
    Returns device tensors; rz0 = b^T P^{-1} b per column."""
    npix = problem.grid.n_pix
    ldb = _block(Bm, npix, "Bm")
    m = Bm.shape[0]
    dev = Bm.device
    k = pc["k"]
    X = torch.empty(m, npix, dtype=torch.float32, device=dev)
    nl = max(int(n_lanczos), 0)
    ab = torch.zeros(m, max(nl, 1), 2, dtype=torch.float64, device=dev)
    rz0 = torch.empty(m, dtype=torch.float64, device=dev)
    iters = torch.empty(m, dtype=torch.int32, device=dev)
    relres = torch.empty(m, dtype=torch.float64, device=dev)
    true_relres = torch.empty(m, dtype=torch.float64, device=dev) if true_residual else None
    status = torch.empty(m, dtype=torch.int32, device=dev)
    pcode = prec_code(prec)
    pr = problem_c(problem, px, py)
    need = _lib.lib.gpl_pcg_solve_workspace(C.byref(pr), k, m, pcode)
    if ws is None or ws.numel() < need:
        ws, _ = workspace(need, dev)
    _lib.call("gpl_pcg_solve", C.byref(pr), k, _ptr(pc["L"]), npix, _ptr(pc["G"]), k, m, _ptr(Bm), ldb, _ptr(X),
              npix, float(tol), int(max_iter), int(fixed_iters), nl, _ptr(ab), _ptr(rz0), _ptr(iters), _ptr(relres),
              _ptr(true_relres), _ptr(status), pcode, int(check_every), _wsptr(ws), int(need), _stream())
    return dict(X=X, ab=ab[:, :nl], bnorm2=rz0, rz0=rz0, iters=iters, relres=relres, true_relres=true_relres,
                status=status, n_lanczos=nl)


def evidence_scalars(n_pix, n_points, r, u, logdet, amplitude, noise_sigma):
    out = torch.empty(3, dtype=torch.float64, device=r.device)
    _lib.call("gpl_evidence_scalars", n_pix, n_points, _ptr(r), _ptr(u), _ptr(logdet), float(amplitude),
              float(noise_sigma), _ptr(out), _stream())
    return out


def evidence_amplitude_grad(n_points, u, Z, X, quad, scale, amplitude, noise_sigma):
    """(d ln p/d alpha, d L_VI/d alpha) as a float64 2-vector on the device; Z, X:
    (m, n_pix) probes and their solves (m may be 0), quad a device scalar."""
    npix = u.numel()
    m = 0 if Z is None else Z.shape[0]
    ldz = _block(Z, npix, "Z") if m else npix
    ldx = _block(X, npix, "X") if m else npix
    out = torch.empty(2, dtype=torch.float64, device=u.device)
    _lib.call("gpl_evidence_amplitude_grad", npix, int(n_points), m, _ptr(u), _ptr(Z) if m else None, ldz,
              _ptr(X) if m else None, ldx, _ptr(quad, torch.float64), float(scale), float(amplitude),
              float(noise_sigma), _ptr(out), _stream())
    return out


def block_dot(X, Y):
    """Per-column FP64 dot products of two (ncols, n) blocks."""
    n = X.shape[-1]
    X2 = X.unsqueeze(0) if X.dim() == 1 else X
    Y2 = Y.unsqueeze(0) if Y.dim() == 1 else Y
    ldx, ldy = _block(X2, n, "X"), _block(Y2, n, "Y")
    out = torch.empty(X2.shape[0], dtype=torch.float64, device=X.device)
    _lib.call("gpl_block_dot", n, X2.shape[0], _ptr(X2), ldx, _ptr(Y2), ldy, _ptr(out), _stream())
    return out


def posterior_variance(W, X, prior):
    """prior - W[c] . X[c] per column in FP64 (W, X as (ncols, n) blocks)."""
    n = W.shape[-1]
    ldw, ldx = _block(W, n, "W"), _block(X, n, "X")
    out = torch.empty(W.shape[0], dtype=torch.float64, device=W.device)
    _lib.call("gpl_posterior_variance", n, W.shape[0], _ptr(W), ldw, _ptr(X), ldx, float(prior), _ptr(out),
              _stream())
    return out


# ------------------------------------------------------------------ backward

def kernel_mvm_backward(kernel: Kernel, px, py, A, Bv, weights, gpx=None, gpy=None):
    """Gradient of F = sum_c w_c a_c^T K b_c w.r.t. points (accumulated into gpx,
    gpy), lengthscale and amplitude (returned as a 2-vector of float64)."""
    n = px.numel()
    lda, ldb = _block(A, n, "A"), _block(Bv, n, "Bv")
    npairs = A.shape[0]
    if Bv.shape[0] != npairs or len(weights) != npairs:
        raise ValueError("A, Bv and weights must have the same number of columns")
    if gpx is None:
        gpx = torch.zeros(n, dtype=torch.float32, device=px.device)
        gpy = torch.zeros(n, dtype=torch.float32, device=px.device)
    ghyp = torch.empty(2, dtype=torch.float64, device=px.device)
    w = (C.c_double * npairs)(*[float(v) for v in weights])
    ws, wsb = workspace(_lib.lib.gpl_gp_kernel_mvm_backward_workspace(n, npairs), px.device)
    k = kernel.c()
    _lib.call("gpl_gp_kernel_mvm_backward", C.byref(k), n, _ptr(px), _ptr(py), npairs, _ptr(A), lda, _ptr(Bv), ldb,
              w, _ptr(gpx), _ptr(gpy), _ptr(ghyp), _wsptr(ws), wsb, _stream())
    return gpx, gpy, ghyp


def lens_raytrace_backward(grid: Grid, lens: Lens, gpx, gpy):
    g, L = grid.c(), lens.c()
    out = torch.empty(8, dtype=torch.float64, device=gpx.device)
    ws, wsb = workspace(_lib.lib.gpl_lens_raytrace_backward_workspace(C.byref(g)), gpx.device)
    _lib.call("gpl_lens_raytrace_backward", C.byref(g), C.byref(L), _ptr(gpx), _ptr(gpy), _ptr(out), _wsptr(ws), wsb,
              _stream())
    return out


def lens_raytrace_backward_noalloc(grid: Grid, lens: Lens, gpx, gpy, out):
    """The adjoint into a caller-owned FP64 buffer of 8, with no allocation in
    the library (its scratch is a static device array; calls on one device must
    not overlap)."""
    g, L = grid.c(), lens.c()
    _lib.call("gpl_lens_raytrace_backward_noalloc", C.byref(g), C.byref(L), _ptr(gpx), _ptr(gpy), _ptr(out), _stream())
    return out


def sersic_backward(src: Sersic, px, py, gmu, gpx, gpy):
    n = px.numel()
    s = src.c()
    out = torch.empty(2, dtype=torch.float64, device=px.device)
    ws, wsb = workspace(_lib.lib.gpl_sersic_backward_workspace(n), px.device)
    _lib.call("gpl_sersic_backward", C.byref(s), n, _ptr(px), _ptr(py), _ptr(gmu), _ptr(gpx), _ptr(gpy), _ptr(out),
              _wsptr(ws), wsb, _stream())
    return out


# ------------------------------------------------------------------ timing

def timing_enable(on: bool | int = True):
    """Time every kernel-product launch (True), every k-th one (an int k >= 1),
    or none (False / 0)."""
    stride = int(on) if not isinstance(on, bool) else (1 if on else 0)
    _lib.call("gpl_timing_enable", stride)


def timing_read(reset: bool = True):
    """(total milliseconds, launches) of the timed kernel-product launches."""
    ms, n = C.c_double(0.0), C.c_long(0)
    _lib.call("gpl_timing_read", C.byref(ms), C.byref(n), 1 if reset else 0)
    return ms.value, n.value


def timing_samples(reset: bool = True):
    """Per-launch milliseconds of the timed kernel-product launches, in order."""
    n = C.c_int(0)
    _lib.call("gpl_timing_samples", None, 0, C.byref(n), 0)
    buf = (C.c_float * max(n.value, 1))()
    _lib.call("gpl_timing_samples", buf, n.value, C.byref(n), 1 if reset else 0)
    return [float(buf[k]) for k in range(n.value)]

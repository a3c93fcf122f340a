"""ctypes binding of libgplens.so (the C-ABI declared in include/gplens.h).

Only argument marshalling lives here: structs, pointer/stream conversion and
error translation. Every computation runs in the HIP library. Importing this
module never falls back to anything else: if the library is missing or does not
load, the import raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("GPLENS_LIB", os.path.join(HERE, "libgplens.so"))

GPL_OK, GPL_EINVAL, GPL_EWORKSPACE, GPL_EHIP, GPL_EUNSUPPORTED = 0, -1, -2, -3, -4
PREC_FP32, PREC_F16X3 = 0, 1
CG_CONVERGED, CG_MAXITER, CG_BREAKDOWN, CG_NONFINITE = 0, 1, 2, 3
PSF_MAX_RADIUS = 24


class GplError(RuntimeError):
    def __init__(self, code, func, detail):
        super().__init__(f"{func} failed ({code}): {detail}")
        self.code = code


class gpl_grid(C.Structure):
    _fields_ = [("n", C.c_int), ("ss", C.c_int), ("pix_scale", C.c_double), ("cx", C.c_double), ("cy", C.c_double)]


class gpl_lens(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("theta_E", "q", "phi", "slope", "x0", "y0", "gamma1", "gamma2")]


class gpl_source(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("I_e", "R_e", "n_sersic", "b_n", "xs", "ys")]


class gpl_kernel(C.Structure):
    _fields_ = [("kind", C.c_int), ("lengthscale", C.c_double), ("amplitude", C.c_double)]


class gpl_gauss(C.Structure):
    _fields_ = [("base_var", C.c_double), ("norm", C.c_double)]


class gpl_vigp_model(C.Structure):
    _fields_ = [("n_layers", C.c_int), ("kind", C.c_int * 8), ("lengthscale", C.c_double * 8), ("knn_k", C.c_int),
                ("slope", C.c_double), ("prior_lo", C.c_double * 5), ("prior_hi", C.c_double * 5),
                ("shear_sd", C.c_double)]


class gpl_psf(C.Structure):
    _fields_ = [("fwhm", C.c_double), ("radius", C.c_int)]


class gpl_problem(C.Structure):
    _fields_ = [("grid", gpl_grid), ("kernel", gpl_kernel), ("psf", gpl_psf), ("noise_sigma", C.c_double),
                ("px", C.c_void_p), ("py", C.c_void_p)]


class gpl_serve_slot(C.Structure):
    _fields_ = [("ws", C.c_void_p), ("dev", C.c_void_p), ("N", C.c_int), ("npix", C.c_int), ("nrhs", C.c_int),
                ("opaque", C.c_ubyte * 1024)]


_P = C.c_void_p
_I = C.c_int
_D = C.c_double
_F = C.c_float
_Z = C.c_size_t

# name -> (restype, argtypes)
SIGNATURES = {
    "gpl_strerror": (C.c_char_p, [_I]),
    "gpl_last_error": (C.c_char_p, []),
    "gpl_version": (_I, []),
    "gpl_sersic_bn": (_D, [_D]),
    "gpl_grid_map": (_I, [C.POINTER(gpl_grid), _P, _P, _P, _P]),
    "gpl_lens_raytrace": (_I, [C.POINTER(gpl_grid), C.POINTER(gpl_lens), _P, _P, _P]),
    "gpl_sersic_eval": (_I, [C.POINTER(gpl_source), _I, _P, _P, _P, _P]),
    "gpl_psf_conv": (_I, [C.POINTER(gpl_grid), C.POINTER(gpl_psf), _I, _P, _I, _P, _I, _F, _F, _I, _P]),
    "gpl_gp_kernel_mvm_workspace": (_Z, [_I, _I, _I]),
    "gpl_gp_kernel_mvm": (_I, [C.POINTER(gpl_kernel), C.POINTER(gpl_grid), _I, _P, _P, _I, _P, _I, _P, _I, _F, _I,
                               _P, _Z, _P]),
    "gpl_gp_kernel_mvm_plan_workspace": (_Z, [_I]),
    "gpl_gp_kernel_mvm_plan_stats": (_I, [C.POINTER(gpl_kernel), C.POINTER(gpl_grid), _I, _P, _P, _I,
                                          C.POINTER(C.c_longlong), C.POINTER(C.c_longlong),
                                          C.POINTER(C.c_longlong), _P, _Z, _P]),
    "gpl_apply_A_workspace": (_Z, [C.POINTER(gpl_problem), _I, _I]),
    "gpl_apply_A": (_I, [C.POINTER(gpl_problem), _I, _P, _I, _P, _I, _I, _P, _Z, _P]),
    "gpl_cg_solve_workspace": (_Z, [C.POINTER(gpl_problem), _I, _I]),
    "gpl_cg_solve": (_I, [C.POINTER(gpl_problem), _I, _P, _I, _P, _I, _D, _I, _I, _I, _P, _P, _P, _P, _P, _P, _I,
                          _I, _P, _Z, _P]),
    "gpl_lanczos_logdet_workspace": (_Z, [_I, _I]),
    "gpl_lanczos_logdet": (_I, [_I, _I, _P, _P, _P, _D, _P, _P, _P, _P, _P, _Z, _P]),
    "gpl_pchol_workspace": (_Z, [C.POINTER(gpl_problem), _I, _I]),
    "gpl_pchol": (_I, [C.POINTER(gpl_problem), _I, _I, _P, _I, _P, _I, _P, _P, _P, _P, _Z, _P]),
    "gpl_pchol_probes_workspace": (_Z, [_I, _I]),
    "gpl_pchol_probes": (_I, [_I, _I, _P, _I, _D, _I, _P, _I, _P, _I, _P, _I, _P, _Z, _P]),
    "gpl_pcg_solve_workspace": (_Z, [C.POINTER(gpl_problem), _I, _I, _I]),
    "gpl_pcg_solve": (_I, [C.POINTER(gpl_problem), _I, _P, _I, _P, _I, _I, _P, _I, _P, _I, _D, _I, _I, _I, _P, _P,
                           _P, _P, _P, _P, _I, _I, _P, _Z, _P]),
    "gpl_evidence_scalars": (_I, [_I, _I, _P, _P, _P, _D, _D, _P, _P]),
    "gpl_gp_kernel_mvm_backward_workspace": (_Z, [_I, _I]),
    "gpl_gp_kernel_mvm_backward": (_I, [C.POINTER(gpl_kernel), _I, _P, _P, _I, _P, _I, _P, _I, C.POINTER(_D), _P, _P,
                                        _P, _P, _Z, _P]),
    "gpl_lens_raytrace_backward_workspace": (_Z, [C.POINTER(gpl_grid)]),
    "gpl_lens_raytrace_backward": (_I, [C.POINTER(gpl_grid), C.POINTER(gpl_lens), _P, _P, _P, _P, _Z, _P]),
    "gpl_lens_raytrace_backward_noalloc": (_I, [C.POINTER(gpl_grid), C.POINTER(gpl_lens), _P, _P, _P, _P]),
    "gpl_sersic_backward_workspace": (_Z, [_I]),
    "gpl_sersic_backward": (_I, [C.POINTER(gpl_source), _I, _P, _P, _P, _P, _P, _P, _P, _Z, _P]),
    "gpl_block_dot": (_I, [_I, _I, _P, _I, _P, _I, _P, _P]),
    "gpl_posterior_variance": (_I, [_I, _I, _P, _I, _P, _I, _D, _P, _P]),
    "gpl_gauss_product": (_I, [C.POINTER(gpl_gauss), _I, _P, _P, _P, _P, _I, _P, _P, _P, _P, _I, _P, _I, _P, _I,
                               C.c_float, _P]),
    "gpl_gauss_matrix": (_I, [C.POINTER(gpl_gauss), _I, _P, _P, _P, _P, _I, _P, _P, _P, _P, _P, _I, _P]),
    "gpl_pixel_shapes": (_I, [C.POINTER(gpl_grid), _P, _P, _P, _P]),
    "gpl_gauss_product_backward": (_I, [C.POINTER(gpl_gauss), _I, _P, _P, _P, _P, _I, _P, _P, _P, _P, _P, _P, _P, _P,
                                        _P, _P, _P, _P]),
    "gpl_pixel_shapes_backward": (_I, [C.POINTER(gpl_grid), _P, _P, _P, _P, _P, _P, _Z, _P]),
    "gpl_vigp_sizes": (_I, [C.POINTER(gpl_vigp_model), C.POINTER(gpl_grid), _I, C.POINTER(_Z), C.POINTER(_Z),
                            C.POINTER(_Z)]),
    "gpl_vigp_workspace": (_Z, [C.POINTER(gpl_vigp_model), C.POINTER(gpl_grid), _I]),
    "gpl_vigp_elbo": (_I, [C.POINTER(gpl_vigp_model), C.POINTER(gpl_grid), C.POINTER(gpl_psf), C.POINTER(gpl_source),
                           _D, _I, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _Z, _P]),
    "gpl_vigp_adam": (_I, [_Z, _P, _P, _P, _P, _Z, _P, _P, _P, _P, _I, _D, _D, _D, _D, _P]),
    "gpl_knn_density_workspace": (_Z, [_I]),
    "gpl_knn_density": (_I, [_I, _P, _P, _I, _P, _P, _Z, _P]),
    "gpl_evidence_amplitude_grad": (_I, [_I, _I, _I, _P, _P, _I, _P, _I, _P, _D, _D, _D, _P, _P]),
    "gpl_timing_enable": (_I, [_I]),
    "gpl_serve_slot_workspace": (_Z, [C.POINTER(gpl_grid), _I, _I, _I]),
    "gpl_serve_slot_init": (_I, [C.POINTER(gpl_serve_slot), C.POINTER(gpl_problem), C.POINTER(gpl_lens),
                                 C.POINTER(gpl_source), _P, _P, _I, _I, _D, _I, _I, _I, _P, _Z, _P]),
    "gpl_serve_step": (_I, [C.POINTER(C.POINTER(gpl_serve_slot)), _I, _I, C.c_long, _P]),
    "gpl_serve_snapshot": (_I, [C.POINTER(C.POINTER(gpl_serve_slot)), _I, C.c_long, _P, _P]),
    "gpl_serve_slot_finish": (_I, [C.POINTER(gpl_serve_slot), C.c_long, _D, _P, _P, _P, _P, _P, _P, _P]),
    "gpl_timing_read": (_I, [C.POINTER(_D), C.POINTER(C.c_long), _I]),
    "gpl_timing_samples": (_I, [C.POINTER(C.c_float), _I, C.POINTER(_I), _I]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"gplens library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def call(name, *args):
    """Call an int-returning entry point and raise GplError on failure."""
    rc = getattr(lib, name)(*args)
    if rc != GPL_OK:
        raise GplError(rc, name, lib.gpl_last_error().decode(errors="replace"))
    return rc


def exported_symbols():
    return sorted(SIGNATURES)

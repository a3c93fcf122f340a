"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every
symbol the header declares, rejects invalid arguments before touching the
device, and its host helpers agree with the oracle."""
import ctypes as C
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gplens.h")


def _lib():
    try:
        from paper_2105_09465_amd import _lib
    except ImportError as e:  # the library must be built before the tests
        pytest.fail(f"libgplens.so not loadable: {e}")
    return _lib


def header_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gpl_[A-Za-z0-9_]+)\s*\(", text)))


def test_header_symbols_exported_and_bound():
    L = _lib()
    syms = header_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(L.lib, s), f"{s} declared in gplens.h but not exported"
    assert sorted(L.SIGNATURES) == syms, "Python binding and header disagree"


def test_version_and_strerror():
    L = _lib()
    assert L.lib.gpl_version() >= 100
    for code in (0, -1, -2, -3, -4):
        assert L.lib.gpl_strerror(code)


def test_sersic_bn_matches_oracle():
    L = _lib()
    from oracle import source
    for n in (0.5, 1.0, 1.5, 2.5, 4.0, 8.0):
        assert math.isclose(L.lib.gpl_sersic_bn(n), source.sersic_bn(n), rel_tol=1e-12)
    assert math.isnan(L.lib.gpl_sersic_bn(-1.0))


def test_invalid_arguments_rejected_on_host():
    L = _lib()
    g = L.gpl_grid(10, 2, 0.05, 0.0, 0.0)
    bad_lens = L.gpl_lens(1.0, 1.5, 0.0, 2.0, 0.0, 0.0, 0.0, 0.0)  # q > 1
    p = C.c_void_p(16)  # never dereferenced: validation fails first
    assert L.lib.gpl_lens_raytrace(C.byref(g), C.byref(bad_lens), p, p, None) == L.GPL_EINVAL
    assert b"q=" in L.lib.gpl_last_error()
    k = L.gpl_kernel(0, -1.0, 0.3)
    assert L.lib.gpl_gp_kernel_mvm(C.byref(k), None, 10, p, p, 1, p, 10, p, 10, 0.0, 0, None, 0, None) == L.GPL_EINVAL
    k = L.gpl_kernel(0, 0.04, 0.3)
    assert L.lib.gpl_gp_kernel_mvm(C.byref(k), None, 10, p, p, 1, p, 5, p, 10, 0.0, 0, None, 0, None) == L.GPL_EINVAL
    assert L.lib.gpl_gp_kernel_mvm(C.byref(k), None, 10, p, p, 1, p, 10, p, 10, 0.0, 7, None, 0, None) == L.GPL_EINVAL
    big = L.gpl_psf(5.0, 0)  # radius beyond the maximum
    assert L.lib.gpl_psf_conv(C.byref(g), C.byref(big), 1, p, 400, C.c_void_p(32), 100, 1.0, 0.0, 0, None) == \
        L.GPL_EINVAL
    # workspace checks
    need = L.lib.gpl_gp_kernel_mvm_workspace(40000, 17, 0)
    assert need > 0
    assert L.lib.gpl_gp_kernel_mvm(C.byref(k), None, 40000, p, p, 17, p, 40000, C.c_void_p(64), 40000, 0.0, 0, None, 0,
                                   None) == L.GPL_EWORKSPACE
    assert L.lib.gpl_lanczos_logdet(0, 30, p, p, p, 1.0, None, p, p, p, None, 0, None) == L.GPL_EINVAL
    # preconditioner: rank not a multiple of 64, zero noise
    prob = L.gpl_problem(g, k, L.gpl_psf(0.1, 0), 0.02, p, p)
    assert L.lib.gpl_pchol(C.byref(prob), 100, 1, p, 100, p, 100, p, p, p, None, 0, None) == L.GPL_EINVAL
    assert b"multiple of 64" in L.lib.gpl_last_error()
    prob0 = L.gpl_problem(g, k, L.gpl_psf(0.1, 0), 0.0, p, p)
    assert L.lib.gpl_pchol(C.byref(prob0), 64, 1, p, 100, p, 64, p, p, p, None, 0, None) == L.GPL_EINVAL
    assert L.lib.gpl_pchol(C.byref(prob), 64, 1, p, 100, p, 64, p, p, p, None, 0, None) == L.GPL_EWORKSPACE


def test_workspace_sizes_monotone():
    L = _lib()
    prob = L.gpl_problem(L.gpl_grid(100, 2, 0.05, 0, 0), L.gpl_kernel(0, 0.04, 0.3), L.gpl_psf(0.1, 0), 0.02,
                         C.c_void_p(16), C.c_void_p(16))
    a = L.lib.gpl_cg_solve_workspace(C.byref(prob), 17, 0)
    b = L.lib.gpl_cg_solve_workspace(C.byref(prob), 33, 0)
    assert 0 < a < b
    assert a % 256 == 0
    assert L.lib.gpl_lanczos_logdet_workspace(16, 30) == 0  # the quadrature runs in LDS
    assert L.lib.gpl_gp_kernel_mvm_workspace(160000, 64, 1) > L.lib.gpl_gp_kernel_mvm_workspace(40000, 17, 1) > 0


def test_noalloc_adjoint_size_limit_on_host():
    """The allocation-free adjoint refuses grids beyond its static scratch
    (4,194,304 fine points) before any device call."""
    L = _lib()
    p = C.c_void_p(16)  # never dereferenced: validation fails first
    lens = L.gpl_lens(1.0, 0.8, 0.0, 2.0, 0.0, 0.0, 0.0, 0.0)
    big = L.gpl_grid(2049, 1, 0.05, 0.0, 0.0)
    assert L.lib.gpl_lens_raytrace_backward_noalloc(C.byref(big), C.byref(lens), p, p, p, None) == L.GPL_EINVAL
    assert b"static scratch" in L.lib.gpl_last_error()

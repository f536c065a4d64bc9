"""The C-ABI library loads and exports every entry point include/magnus.h
declares; host-side argument checks run without a GPU."""
import ctypes
import os
import re

import pytest

import paper_2207_09776_amd as mg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "magnus.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(mg.LIB_PATH):
        pytest.fail("libmagnus.so is not built (run python -m paper_2207_09776_amd.build)")
    return mg.load_library()


def test_header_declares_the_five_entry_points():
    names = declared_functions()
    for n in ("mg_build_operators", "mg_iterated_integrals", "mg_magnus_expmv", "mg_euler_step",
              "mg_error_vs_exact"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(mg.EXPORTS) <= set(declared_functions())


def test_version_and_error_string(lib):
    assert b"gfx950" in lib.mg_version()
    assert lib.mg_last_error() is not None


def test_shape_checks_before_any_device_call(lib):
    vp = ctypes.c_void_p
    # Nf not a multiple of K
    assert lib.mg_iterated_integrals(vp(8), 2, 100, 1.0, 3, 2, vp(8), None, None) == mg.MG_ESHAPE
    assert b"multiple" in lib.mg_last_error()
    # negative P, bad order, bad T
    assert lib.mg_iterated_integrals(vp(8), -1, 96, 1.0, 3, 2, vp(8), None, None) == mg.MG_ESHAPE
    assert lib.mg_iterated_integrals(vp(8), 2, 96, 1.0, 3, 4, vp(8), None, None) == mg.MG_EINVAL
    assert lib.mg_iterated_integrals(vp(8), 2, 96, 0.0, 3, 2, vp(8), None, None) == mg.MG_EINVAL
    # P = 0 is a no-op even with NULL buffers
    assert lib.mg_iterated_integrals(None, 0, 96, 1.0, 3, 2, None, None, None) == mg.MG_OK
    # NULL ops
    assert lib.mg_magnus_expmv(None, None, 1, 1, None, 1, None, 0, 0.0, None, 0, None, None,
                               None) == mg.MG_EINVAL
    assert lib.mg_magnus_expmv_noalloc(None, None, 1, 1, None, 1, None, 0, 0.0, None, None,
                                       None) == mg.MG_EINVAL
    assert lib.mg_euler_step(None, None, 1, None, 1, 0.1, 0, None, 0, None, None) == mg.MG_EINVAL
    assert lib.mg_workspace_bytes(None, 4, 4, 0) == 0


def test_build_operators_argument_checks(lib):
    g = mg.mg_grid(0, 8, -1.0, 1.0, -1.0, 1.0)
    c = mg.mg_coeffs()
    h = ctypes.c_void_p()
    assert lib.mg_build_operators(ctypes.byref(g), ctypes.byref(c), 2, ctypes.byref(h)) == mg.MG_EINVAL
    g = mg.mg_grid(8, 8, 1.0, -1.0, -1.0, 1.0)
    assert lib.mg_build_operators(ctypes.byref(g), ctypes.byref(c), 2, ctypes.byref(h)) == mg.MG_EINVAL
    g = mg.mg_grid(8, 8, -1.0, 1.0, -1.0, 1.0)
    assert lib.mg_build_operators(ctypes.byref(g), ctypes.byref(c), 4, ctypes.byref(h)) == mg.MG_EINVAL
    assert lib.mg_build_operators(None, ctypes.byref(c), 2, ctypes.byref(h)) == mg.MG_EINVAL


def test_error_vs_exact_argument_checks(lib):
    g = mg.mg_grid(8, 8, -1.0, 1.0, -1.0, 1.0)
    ex = mg.mg_exact(1.0, 1.5, 0.25, 1.0)        # sigma^2 >= a: no closed form
    vp = ctypes.c_void_p
    assert lib.mg_error_vs_exact(ctypes.byref(g), ctypes.byref(ex), vp(8), vp(8), None, 1, 0,
                                 vp(8), None) == mg.MG_EINVAL
    ex = mg.mg_exact(1.0, 0.5, 0.25, 1.0)
    assert lib.mg_error_vs_exact(ctypes.byref(g), ctypes.byref(ex), vp(8), vp(8), None, 1, 4,
                                 vp(8), None) == mg.MG_EINVAL      # 8 >> 4 == 0: empty window


def _build_status(coeffs, n, order, lo=-5.0, hi=5.0):
    """Status of mg_build_operators; combinations the factored form cannot hold
    fail in the host build, before any device call, so this runs on the CPU."""
    import workloads as wl
    arrays = wl.sample_coefficients(coeffs, n, n, lo, hi, lo, hi)
    try:
        mg.build_operators(n, n, lo, hi, lo, hi, arrays, order)
    except mg.MagnusError as e:
        return e.code
    return mg.MG_OK


def test_unsupported_coefficient_combinations_are_reported():
    import numpy as np
    import workloads as wl
    # x-dependent diffusion with the x transport at order 3: [[B,A],B] pairs
    # a power of D^x with an x-dependent factor
    assert _build_status(wl.langevin_variable_sigma_beta(), 16, 3) == mg.MG_EUNSUPPORTED
    # the paper's variable set: x-dependent noise through d/dv meets D^x in
    # [B,A] (words diag(a) D^x diag(b)) and twice in [[B,A],B] (words
    # diag(a) D^x diag(b) D^x diag(c)): built at every order
    assert _build_status(wl.langevin_paper_variable(1.1, 0.3), 16, 2) != mg.MG_EUNSUPPORTED
    assert _build_status(wl.langevin_paper_variable(1.1, 0.3), 16, 3) != mg.MG_EUNSUPPORTED
    # x-dependent coefficients of x derivatives and the second difference in
    # x are x-terms (words diag(a) D^x, D^xx), built at every order ...
    assert _build_status(wl.Coefficients(fx=lambda x, v: -v * (1 + 0.1 * x)), 16, 3) != mg.MG_EUNSUPPORTED
    assert _build_status(wl.Coefficients(gxx=lambda x, v: 1.0 + 0 * x), 16, 3) != mg.MG_EUNSUPPORTED
    # ... but x-dependent noise through D^x puts three x derivatives into
    # [[B,A],A] at order 3
    sx = wl.Coefficients(fx=lambda x, v: -v, gvv=lambda x, v: 1.0 + 0 * x,
                         sx=lambda x, v: 0.3 * (1.0 + 0.5 / (1.0 + x * x)) + 0 * v)
    assert _build_status(sx, 16, 2) != mg.MG_EUNSUPPORTED
    assert _build_status(sx, 16, 3) == mg.MG_EUNSUPPORTED
    # a coefficient grid of full rank is not a short sum of products b(v) a(x)
    rng = np.random.default_rng(0)
    noise = rng.random((16, 16))
    assert _build_status(wl.Coefficients(gvv=lambda x, v: 1.0 + 0.1 * noise), 16, 2) == mg.MG_EUNSUPPORTED
    # non-finite coefficients
    assert _build_status(wl.Coefficients(gvv=lambda x, v: np.where(x > 0, np.nan, 1.0)), 16, 2) in (
        mg.MG_EINVAL, mg.MG_EUNSUPPORTED)


def test_multi_job_argument_checks(lib):
    """mg_magnus_expmv_multi checks every job before launching anything."""
    lib.mg_magnus_expmv_multi.restype = ctypes.c_int32
    assert lib.mg_magnus_expmv_multi(None, 0, None, 0, None) == mg.MG_OK
    assert lib.mg_magnus_expmv_multi(None, -1, None, 0, None) == mg.MG_EINVAL
    assert lib.mg_magnus_expmv_multi(None, 2, None, 0, None) == mg.MG_EINVAL
    jobs = (mg.mg_job * 2)()
    jobs[0] = mg.mg_job(None, None, 4, 4, None, 1, None, 0, 0.0, None, None)   # NULL ops
    assert lib.mg_magnus_expmv_multi(jobs, 2, None, 0, None) == mg.MG_EINVAL
    assert b"job 0" in lib.mg_last_error()
    assert lib.mg_workspace_bytes_multi(None, 1) == 0
    assert lib.mg_workspace_bytes_multi(jobs, 2) == 0


def test_adaptive_argument_checks(lib):
    """mg_magnus_adaptive rejects NULL outputs and operators before any
    device call."""
    vp = ctypes.c_void_p
    lvl = (ctypes.c_int32 * 4)()
    gp = (ctypes.c_double * 4)()
    assert lib.mg_magnus_adaptive(None, None, vp(8), 1, 64, 1.0, vp(8), 1, vp(8), 4, 2, 1, 1e-3,
                                  0, None, None, None) == mg.MG_EINVAL
    assert lib.mg_magnus_adaptive(None, None, vp(8), 1, 64, 1.0, vp(8), 1, vp(8), 4, 2, 1, 1e-3,
                                  0, lvl, gp, None) == mg.MG_EINVAL
    assert b"NULL" in lib.mg_last_error()

"""Host-side checks of the C ABI (no GPU compute): the library loads, exports
every function include/fmmprec.h declares, and rejects bad arguments before
touching the device."""
import ctypes
import os
import re

import pytest

import paper_1308_3339_amd as fp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fmmprec.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fmm_\w+|precond_gmres_solve\w*)\s*\(", src)))


def test_header_declares_the_entry_points():
    assert set(_declared()) == set(fp.exported_symbols)


def test_library_exports_every_declared_symbol():
    lib = fp.load_library()
    for name in _declared():
        assert hasattr(lib, name), name


def test_version_string():
    assert "gfx950" in fp.fmm_version()


def _setup_raw(kind=0, n=64, p=10, leaf=64, prec=0, bem=1, eps=0.0, theta=0.0):
    from paper_1308_3339_amd._binding import fmm_params, fmm_problem
    lib = fp.load_library()
    prob = fmm_problem(kind, n, None, None, 0.0, 0.0, 1.0)
    prm = fmm_params(p, leaf, prec, bem, eps, theta)
    out = ctypes.c_void_p(123)
    code = lib.fmm_setup(ctypes.byref(prob), ctypes.byref(prm), None, ctypes.byref(out))
    return code, out.value, lib.fmm_last_error(None).decode()


@pytest.mark.parametrize("kw,frag", [
    (dict(p=1), "p must"),
    (dict(p=21), "p must"),
    (dict(leaf=32), "leaf"),
    (dict(n=12), "8 * 2^L"),
    (dict(n=4), "8 * 2^L"),
    (dict(kind=7), "kind"),
    (dict(eps=-1.0), "self_eps"),
    (dict(theta=0.2), "theta"),
    (dict(theta=1.5), "theta"),
    (dict(theta=-0.5), "theta"),
])
def test_setup_rejects_bad_arguments(kw, frag):
    code, ptr, msg = _setup_raw(**kw)
    assert code == fp.FMM_ERR_ARG
    assert not ptr
    assert frag in msg


def test_precision_enum_values():
    # fmm_precision as declared in include/fmmprec.h
    src = open(os.path.join(ROOT, "include", "fmmprec.h")).read()
    vals = dict((k, int(v)) for k, v in re.findall(r"\b(FMM_(?:FP64|FP32|SPLIT_BF16|SPLIT_FP16))\s*=\s*(\d+)", src))
    assert vals == {"FMM_FP64": 0, "FMM_FP32": 1, "FMM_SPLIT_BF16": 2, "FMM_SPLIT_FP16": 3}
    assert (fp.FMM_FP64, fp.FMM_FP32, fp.FMM_SPLIT_BF16, fp.FMM_SPLIT_FP16) == (0, 1, 2, 3)


@pytest.mark.parametrize("prec", [4, -1])
def test_setup_rejects_unbuilt_precision(prec):
    code, ptr, msg = _setup_raw(prec=prec)
    assert code == fp.FMM_ERR_UNSUPPORTED and not ptr


@pytest.mark.parametrize("prec", [2, 3])
def test_split_precision_needs_a_grid(prec):
    code, ptr, msg = _setup_raw(kind=1, n=100, prec=prec)
    assert code == fp.FMM_ERR_UNSUPPORTED and not ptr
    assert "GRID" in msg


@pytest.mark.parametrize("kw", [dict(theta=0.4, prec=1, kind=1), dict(theta=0.4, prec=2),
                                dict(theta=0.4, prec=3),
                                dict(theta=0.3, p=11), dict(theta=0.4, p=14)])
def test_setup_rejects_unbuilt_theta_combinations(kw):
    # small theta: FP64 plans and FP32 grid plans with p <= 12 only, and the M2L
    # source tile must fit in LDS
    code, ptr, msg = _setup_raw(**kw)
    assert code == fp.FMM_ERR_UNSUPPORTED and not ptr
    assert "theta" in msg


def test_null_arguments():
    lib = fp.load_library()
    assert lib.fmm_setup(None, None, None, None) == fp.FMM_ERR_ARG
    assert lib.fmm_apply(None, None, None, 1, None) == fp.FMM_ERR_ARG
    assert lib.fmm_precond_apply(None, None, None, 1, None) == fp.FMM_ERR_ARG
    assert lib.fmm_stencil_apply(None, None, None, 1, None) == fp.FMM_ERR_ARG
    assert lib.precond_gmres_solve(None, None, None, None, None, None, None) == fp.FMM_ERR_ARG
    assert lib.fmm_destroy(None) == fp.FMM_OK
    assert lib.precond_gmres_solve_batch(None, 1, None, None, None, None, None, 0, None) == fp.FMM_ERR_ARG
    assert lib.fmm_tune(None, None, None) == fp.FMM_ERR_ARG
    assert lib.fmm_tune_m2l(None, None, None) == fp.FMM_ERR_ARG
    assert lib.fmm_set_m2l_split(None, 2) == fp.FMM_ERR_ARG
    assert lib.fmm_get_m2l_split(None, None) == fp.FMM_ERR_ARG
    assert lib.precond_gmres_solve_var(None, None, None, None, None, None, None, None) == fp.FMM_ERR_ARG
    assert lib.fmm_bumps_eval(None, 1, None, None, None, None, None, None) == fp.FMM_ERR_ARG


@pytest.mark.parametrize("n", [0, 100])
def test_points_setup_rejects_missing_coordinates(n):
    code, ptr, msg = _setup_raw(kind=1, n=n)
    assert code == fp.FMM_ERR_ARG and not ptr
    assert "POINTS" in msg

"""The C-ABI library loads and exports every entry point the header declares
(CPU only; no compute calls), and argument validation fails cleanly before
any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "anova.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(anova_\w+|krr_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2111_10140_amd import _lib
    return _lib.load()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ["anova_fastsum_plan", "anova_matvec", "krr_cg_solve",
                     "anova_plan_destroy", "anova_last_error"]:
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_invalid_arguments_return_status(lib):
    from paper_2111_10140_amd import _lib
    h = ctypes.c_void_p()
    w = _lib.make_windows([((0, 1, 2), 1.0)])
    prm = _lib.make_params(0.1)
    # NULL X
    st = lib.anova_fastsum_plan(ctypes.byref(h), None, 10, 3, 3, w, 1, ctypes.byref(prm), None)
    assert st == _lib.ANOVA_E_INVALID and "X" in _lib.anova_last_error()
    assert h.value is None
    # NULL out handle
    st = lib.anova_fastsum_plan(None, None, 10, 3, 3, w, 1, ctypes.byref(prm), None)
    assert st == _lib.ANOVA_E_INVALID
    # NULL plan in the other entry points
    assert lib.anova_matvec(None, None, None, 1, 10, 1.0, None) == _lib.ANOVA_E_INVALID
    info = (_lib.krr_cg_info * 1)()
    assert lib.krr_cg_solve(None, None, None, 1, 10, 1.0, 1e-6, 10, info, None) == _lib.ANOVA_E_INVALID
    assert lib.anova_plan_destroy(None) == _lib.ANOVA_OK


@pytest.mark.parametrize("field,value,needle", [
    ("ell", 0.0, "ell"), ("M", 7, "M"), ("n", 48, "n"), ("m", 9, "m"), ("residual", 2, "residual"), ("tune", 3, "tune"),
    ("precision", 5, "precision"), ("center", 2, "center"),
])
def test_invalid_params_rejected_before_device_work(lib, field, value, needle):
    from paper_2111_10140_amd import _lib
    h = ctypes.c_void_p()
    w = _lib.make_windows([((0, 1, 2), 1.0)])
    prm = _lib.make_params(0.1)
    setattr(prm, field, value)
    # a non-NULL but never dereferenced X: validation happens first
    st = lib.anova_fastsum_plan(ctypes.byref(h), ctypes.c_void_p(16), 10, 3, 3, w, 1,
                                ctypes.byref(prm), None)
    assert st == _lib.ANOVA_E_INVALID
    assert needle in _lib.anova_last_error()


@pytest.mark.parametrize("wins,needle", [
    ([((0, 1, 5), 1.0)], "range"), ([((0, 0), 1.0)], "repeated"), ([((), 1.0)], "d_A"),
    ([((0,), float("nan"))], "eta"),
])
def test_invalid_windows_rejected(lib, wins, needle):
    from paper_2111_10140_amd import _lib
    h = ctypes.c_void_p()
    w = _lib.make_windows(wins)
    prm = _lib.make_params(0.1)
    st = lib.anova_fastsum_plan(ctypes.byref(h), ctypes.c_void_p(16), 10, 3, 3, w, len(wins),
                                ctypes.byref(prm), None)
    assert st == _lib.ANOVA_E_INVALID
    assert needle in _lib.anova_last_error()


def test_newer_entry_points_validate_before_device_work(lib):
    from paper_2111_10140_amd import _lib
    i64 = ctypes.c_int64
    h = ctypes.c_void_p()
    wins = _lib.make_windows([((0, 1, 2), 1.0)])
    prm = _lib.make_params(0.2)
    # host-memory plan: NULL points, bad sizes
    assert lib.anova_fastsum_plan_host(ctypes.byref(h), None, 10, 3, 3, wins, 1,
                                       ctypes.byref(prm)) == _lib.ANOVA_E_INVALID
    X = (ctypes.c_double * 30)()
    assert lib.anova_fastsum_plan_host(ctypes.byref(h), X, 10, 3, 2, wins, 1,
                                       ctypes.byref(prm)) == _lib.ANOVA_E_INVALID  # ldx < d
    assert lib.anova_fastsum_plan_host(None, X, 10, 3, 3, wins, 1,
                                       ctypes.byref(prm)) == _lib.ANOVA_E_INVALID
    # footprint of no plan, solve handles without a plan or list
    a, b = i64(), i64()
    assert lib.anova_plan_footprint(None, 1, ctypes.byref(a), ctypes.byref(b)) == _lib.ANOVA_E_INVALID
    sv = ctypes.c_void_p()
    assert lib.krr_cg_start(ctypes.byref(sv), None, None, None, 1, 10, 1.0, 1e-6, 10,
                            None) == _lib.ANOVA_E_INVALID
    assert lib.krr_cg_start(None, None, None, None, 1, 10, 1.0, 1e-6, 10,
                            None) == _lib.ANOVA_E_INVALID
    assert lib.krr_cg_iterate(None, 0, 1, None) == _lib.ANOVA_E_INVALID
    assert lib.krr_cg_poll(None, None, None, None) == _lib.ANOVA_E_INVALID
    assert lib.krr_cg_finish(None, None, None) == _lib.ANOVA_E_INVALID
    assert lib.krr_cg_destroy(None) == _lib.ANOVA_OK  # NULL is a no-op
    assert lib.krr_cg_solve_batched(0, None, None, None, None, None, None, 1e-6, 10, None,
                                    None) == _lib.ANOVA_E_INVALID
    assert lib.anova_plan_destroy(None) == _lib.ANOVA_OK


def test_prediction_entry_points_validate_before_device_work(lib):
    from paper_2111_10140_amd import _lib
    h = ctypes.c_void_p()
    wins = _lib.make_windows([((0, 1, 2), 1.0)])
    prm = _lib.make_params(0.2)
    X = (ctypes.c_double * 30)()
    Z = (ctypes.c_double * 12)()
    # NULL targets, empty target set, short target rows, NULL handle
    assert lib.anova_predict_plan_host(ctypes.byref(h), X, 10, None, 4, 3, 3, 3, wins, 1,
                                       ctypes.byref(prm)) == _lib.ANOVA_E_INVALID
    assert "Z" in _lib.anova_last_error()
    assert lib.anova_predict_plan_host(ctypes.byref(h), X, 10, Z, 0, 3, 3, 3, wins, 1,
                                       ctypes.byref(prm)) == _lib.ANOVA_E_INVALID
    assert "Nz" in _lib.anova_last_error()
    assert lib.anova_predict_plan_host(ctypes.byref(h), X, 10, Z, 4, 3, 3, 2, wins, 1,
                                       ctypes.byref(prm)) == _lib.ANOVA_E_INVALID
    assert "ldz" in _lib.anova_last_error()
    assert lib.anova_predict_plan_host(None, X, 10, Z, 4, 3, 3, 3, wins, 1,
                                       ctypes.byref(prm)) == _lib.ANOVA_E_INVALID
    # the training-point checks still apply
    assert lib.anova_predict_plan_host(ctypes.byref(h), None, 10, Z, 4, 3, 3, 3, wins, 1,
                                       ctypes.byref(prm)) == _lib.ANOVA_E_INVALID
    assert lib.anova_predict_plan(ctypes.byref(h), ctypes.c_void_p(16), 10, None, 4, 3, 3, 3,
                                  wins, 1, ctypes.byref(prm), None) == _lib.ANOVA_E_INVALID
    assert h.value is None
    assert lib.anova_predict(None, None, None, 1, 10, 4, None) == _lib.ANOVA_E_INVALID


def test_shifted_cg_validates_before_device_work(lib):
    from paper_2111_10140_amd import _lib
    sh = (ctypes.c_double * 2)(1.0, 10.0)
    info = (_lib.krr_cg_info * 2)()
    assert lib.krr_cg_solve_shifts(None, None, None, 2, sh, 10, 1e-6, 10, info,
                                   None) == _lib.ANOVA_E_INVALID
    assert "plan" in _lib.anova_last_error()


def test_reg_q_validated(lib):
    from paper_2111_10140_amd import _lib
    h = ctypes.c_void_p()
    w = _lib.make_windows([((0, 1, 2), 1.0)])
    for bad in (-1, 13):
        prm = _lib.make_params(0.1, reg_q=bad)
        st = lib.anova_fastsum_plan(ctypes.byref(h), ctypes.c_void_p(16), 10, 3, 3, w, 1,
                                    ctypes.byref(prm), None)
        assert st == _lib.ANOVA_E_INVALID and "reg_q" in _lib.anova_last_error()

"""CPU-side checks of the C ABI: the library loads, exports every function that
include/fr.h declares, validates arguments before touching a device, and its
host-built operators agree with the oracle's independently built ones."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2107_14027_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "fr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fr_\w+)\s*\(", src)))


def test_library_exports_every_declared_function():
    L = B.lib()
    names = header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(B.EXPORTED)


def test_binding_constants_match_header():
    """Every FR_ constant the binding defines has the value include/fr.h gives
    it (enumerators with an explicit value)."""
    src = open(os.path.join(ROOT, "include", "fr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    header = {k: int(v) for k, v in re.findall(r"\b(FR_\w+)\s*=\s*(-?\d+)", src)}
    checked = 0
    for name in dir(B):
        if name.startswith("FR_") and isinstance(getattr(B, name), int) and name in header:
            assert getattr(B, name) == header[name], name
            checked += 1
    assert checked >= 30
    for name in ("FR_INFO_RESIDUAL_FORM", "FR_INFO_STAGE_PATH", "FR_STAGE_HALO", "FR_FORM_HALO"):
        assert name in header and hasattr(B, name), name


def test_strerror_and_invalid_arguments_fail_before_device_work():
    assert B.lib().fr_strerror(B.FR_ENOCONV).decode().startswith("pseudo-time")
    for args in [(0, 4, 4, 4, None, 4.0, (1e-3, 1.0)),      # order out of range
                 (7, 4, 4, 4, None, 4.0, (1e-3, 1.0)),
                 (2, 0, 4, 4, None, 4.0, (1e-3, 1.0)),      # empty lattice
                 (2, 4, 4, 4, None, -1.0, (1e-3, 1.0)),     # zeta <= 0
                 (2, 4, 4, 4, None, 4.0, (1e-3, 0.0)),      # T <= 0
                 (2, 4, 4, 4, None, 4.0, (-1.0, 1.0)),      # nu < 0
                 (2, 4, 4, 4, -np.eye(3), 4.0, (1e-3, 1.0))]:  # det J < 0
        with pytest.raises(B.FrError) as ei:
            B.fr_plan_create(*args)
        assert ei.value.code == B.FR_EINVAL
    L = B.lib()
    assert L.fr_residual(None, None, None, None) == B.FR_EINVAL
    assert L.fr_residual_noalloc(None, None, None, None) == B.FR_EINVAL
    assert L.fr_rk_step(None, None, 1e-3, 1, None) == B.FR_EINVAL
    assert L.fr_state_len(None) == 0
    assert L.fr_plan_set_int(None, 1, 0) == B.FR_EINVAL


@pytest.mark.parametrize("p", range(1, 7))
def test_library_operators_match_oracle(p):
    ops = B.fr_plan_operators(p)
    x, w = oracle.gauss_legendre(p + 1)
    assert np.allclose(ops["x"], x, atol=1e-15)
    assert np.allclose(ops["w"], w, atol=1e-14)
    D = oracle.lagrange_deriv(x)
    assert np.allclose(ops["D"], D, atol=1e-12 * max(1.0, np.abs(D).max()))
    assert np.allclose(ops["lm"], oracle.lagrange_eval(x, -1.0), atol=1e-13)
    assert np.allclose(ops["lp"], oracle.lagrange_eval(x, 1.0), atol=1e-13)
    dhl, dhr = oracle.correction_deriv(p, x)
    assert np.allclose(ops["gl"], dhl, atol=1e-11)
    assert np.allclose(ops["gr"], dhr, atol=1e-11)
    Dt = D - np.outer(dhl, oracle.lagrange_eval(x, -1.0)) - np.outer(dhr, oracle.lagrange_eval(x, 1.0))
    assert np.allclose(ops["Dt"], Dt, atol=1e-11)
    with pytest.raises(B.FrError):
        B.fr_plan_operators(7)

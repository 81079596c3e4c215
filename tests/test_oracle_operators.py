"""Pins of the oracle's 1D FR operators (paper Sec. 2.1) against closed forms,
numpy's Legendre routines and the exactness properties the method relies on."""
import math

import numpy as np
import numpy.polynomial.legendre as npleg
import pytest

import oracle


@pytest.mark.parametrize("m", range(1, 9))
def test_gauss_matches_library(m):
    x, w = oracle.gauss_legendre(m)
    xr, wr = npleg.leggauss(m)
    assert np.allclose(x, xr, atol=1e-15, rtol=0)
    assert np.allclose(w, wr, atol=2e-15, rtol=0)


def test_gauss_closed_forms():
    x, w = oracle.gauss_legendre(2)
    assert np.allclose(x, [-1 / math.sqrt(3), 1 / math.sqrt(3)], atol=1e-16)
    assert np.allclose(w, [1.0, 1.0], atol=1e-15)
    x, w = oracle.gauss_legendre(3)
    assert np.allclose(x, [-math.sqrt(0.6), 0.0, math.sqrt(0.6)], atol=1e-16)
    assert np.allclose(w, [5 / 9, 8 / 9, 5 / 9], atol=1e-15)


@pytest.mark.parametrize("p", range(1, 7))
def test_quadrature_exact_to_degree_2p_plus_1(p):
    x, w = oracle.gauss_legendre(p + 1)
    for k in range(2 * p + 2):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-14


@pytest.mark.parametrize("p", range(1, 7))
def test_lagrange_basis(p):
    x, _ = oracle.gauss_legendre(p + 1)
    for j, xj in enumerate(x):
        assert np.allclose(oracle.lagrange_eval(x, xj), np.eye(p + 1)[j], atol=1e-14)
    for t in (-1.0, 1.0, 0.3):
        l = oracle.lagrange_eval(x, t)
        assert abs(l.sum() - 1.0) < 1e-13
        for k in range(p + 1):   # interpolation of x^k is exact
            assert abs(np.dot(l, x ** k) - t ** k) < 1e-13


@pytest.mark.parametrize("p", range(1, 7))
def test_derivative_exact_on_degree_p(p):
    x, _ = oracle.gauss_legendre(p + 1)
    D = oracle.lagrange_deriv(x)
    for k in range(p + 1):
        exact = k * x ** (k - 1) if k else np.zeros_like(x)
        assert np.allclose(D @ x ** k, exact, atol=5e-13)
    # and the derivative of an arbitrary degree-p polynomial via numpy
    rng = np.random.default_rng(p)
    c = rng.standard_normal(p + 1)
    assert np.allclose(D @ np.polynomial.polynomial.polyval(x, c),
                       np.polynomial.polynomial.polyval(x, np.polynomial.polynomial.polyder(c)),
                       atol=5e-12)


@pytest.mark.parametrize("p", range(1, 7))
def test_correction_functions_radau(p):
    """h_l, h_r: endpoint conditions of Sec. 2.1 and the DG (Radau) member."""
    x, w = oracle.gauss_legendre(p + 1)
    dhl, dhr = oracle.correction_deriv(p, x)
    # Legendre-series definitions evaluated with numpy
    el = np.zeros(p + 2)
    el[p], el[p + 1] = 0.5 * (-1) ** p, -0.5 * (-1) ** p
    er = np.zeros(p + 2)
    er[p], er[p + 1] = 0.5, 0.5
    assert np.allclose(npleg.legval([-1.0, 1.0], el), [1.0, 0.0], atol=1e-14)
    assert np.allclose(npleg.legval([-1.0, 1.0], er), [0.0, 1.0], atol=1e-14)
    assert np.allclose(dhl, npleg.legval(x, npleg.legder(el)), atol=1e-12)
    assert np.allclose(dhr, npleg.legval(x, npleg.legder(er)), atol=1e-12)
    # h' has degree p, so Gauss integrates it exactly: h(1) - h(-1)
    assert abs(np.dot(w, dhl) + 1.0) < 1e-13
    assert abs(np.dot(w, dhr) - 1.0) < 1e-13
    # DG lifting identity on Gauss points: h_r'(x_i) = l_i(1)/w_i, h_l'(x_i) = -l_i(-1)/w_i
    assert np.allclose(dhr, oracle.lagrange_eval(x, 1.0) / w, atol=1e-12)
    assert np.allclose(dhl, -oracle.lagrange_eval(x, -1.0) / w, atol=1e-12)


@pytest.mark.parametrize("p", range(1, 7))
def test_partially_corrected_operator_unique_constants(p):
    """The partially corrected divergence operator has ceil((p+1)^2/2) or fewer
    distinct magnitudes (paper Sec. 4.1, the constant-memory optimisation)."""
    x, _ = oracle.gauss_legendre(p + 1)
    D = oracle.lagrange_deriv(x)
    dhl, dhr = oracle.correction_deriv(p, x)
    Dt = D - np.outer(dhl, oracle.lagrange_eval(x, -1.0)) - np.outer(dhr, oracle.lagrange_eval(x, 1.0))
    m = p + 1
    # centro-antisymmetry of the operator on a symmetric point set
    assert np.allclose(Dt[::-1, ::-1], -Dt, atol=1e-12)
    mags = np.unique(np.round(np.abs(Dt).ravel(), 10))
    assert len(mags) <= math.ceil(m * m / 2)
    if p >= 2:
        assert len(mags) == math.ceil(m * m / 2)

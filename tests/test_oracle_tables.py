"""Pins for the oracle's 1D tables (Gauss-Legendre points, Lagrange
derivative and extrapolation rows, Radau correction derivatives), checked
against closed forms and 50-digit mpmath evaluations, never against the
routines the oracle itself calls."""

import math

import mpmath as mp
import numpy as np
import pytest

from oracle import tables

PS = [1, 2, 3, 4]


@pytest.mark.parametrize("P", PS)
def test_nodes_are_legendre_roots(P):
    T = tables.get(P)
    mp.mp.dps = 40
    for x in T.xi:
        # |L_{P+1}(x)| small relative to its derivative scale
        val = mp.legendre(P + 1, mp.mpf(float(x)))
        assert abs(float(val)) < 1e-14
    assert np.all(np.diff(T.xi) > 0)
    np.testing.assert_allclose(T.xi, -T.xi[::-1], atol=1e-15)


@pytest.mark.parametrize("P", PS)
def test_quadrature_exact_to_degree_2P_plus_1(P):
    T = tables.get(P)
    for m in range(2 * P + 2):
        exact = 0.0 if m % 2 else 2.0 / (m + 1)
        assert abs(np.sum(T.w * T.xi ** m) - exact) < 1e-14
    # degree 2P+2 is not integrated exactly (Gauss rule has degree 2n-1)
    m = 2 * P + 2
    assert abs(np.sum(T.w * T.xi ** m) - 2.0 / (m + 1)) > 1e-6


@pytest.mark.parametrize("P", PS)
def test_derivative_matrix_exact_on_monomials(P):
    T = tables.get(P)
    np.testing.assert_allclose(T.D @ np.ones(P + 1), 0.0, atol=1e-13)
    for m in range(1, P + 1):
        np.testing.assert_allclose(T.D @ T.xi ** m, m * T.xi ** (m - 1), atol=1e-12)
    # a degree P+1 monomial is not differentiated exactly
    m = P + 1
    assert np.max(np.abs(T.D @ T.xi ** m - m * T.xi ** (m - 1))) > 1e-6


@pytest.mark.parametrize("P", PS)
def test_extrapolation_rows_exact_on_monomials(P):
    T = tables.get(P)
    for m in range(P + 1):
        assert abs(T.em @ T.xi ** m - (-1.0) ** m) < 1e-13
        assert abs(T.ep @ T.xi ** m - 1.0) < 1e-13
    np.testing.assert_allclose(T.em, T.ep[::-1], atol=1e-14)


@pytest.mark.parametrize("P", PS)
def test_radau_end_values_and_orthogonality(P):
    """g_L is the right Radau polynomial of degree P+1: 1 at -1, 0 at +1,
    orthogonal to all polynomials of degree <= P-1 (checked at 40 digits
    with mpmath's own Legendre functions and quadrature)."""
    mp.mp.dps = 40
    c = tables.radau_left_coeffs(P)
    gl = lambda x: sum(mp.mpf(float(c[n])) * mp.legendre(n, x) for n in range(len(c)))
    gr = lambda x: gl(-x)
    assert abs(gl(-1) - 1) < 1e-30 and abs(gl(1)) < 1e-30
    assert abs(gr(1) - 1) < 1e-30 and abs(gr(-1)) < 1e-30
    for m in range(P):
        assert abs(mp.quad(lambda x: gl(x) * x ** m, [-1, 1])) < 1e-25
    # degree P+1 exactly
    assert abs(float(c[P + 1])) == 0.5


@pytest.mark.parametrize("P", PS)
def test_radau_derivatives_match_mpmath_and_dg_identity(P):
    """gL'(xi_i), gR'(xi_i) against mpmath differentiation of the
    polynomial, and the DG-equivalence identity of the Radau correction:
    gL'(xi_i) = -l_i(-1)/w_i and gR'(xi_i) = l_i(+1)/w_i."""
    mp.mp.dps = 40
    T = tables.get(P)
    c = tables.radau_left_coeffs(P)
    gl = lambda x: sum(mp.mpf(float(c[n])) * mp.legendre(n, x) for n in range(len(c)))
    for i, x in enumerate(T.xi):
        d = float(mp.diff(gl, mp.mpf(float(x))))
        assert abs(d - T.gLp[i]) < 1e-12 * max(1.0, abs(d))
        d2 = float(mp.diff(lambda s: gl(-s), mp.mpf(float(x))))
        assert abs(d2 - T.gRp[i]) < 1e-12 * max(1.0, abs(d2))
    np.testing.assert_allclose(T.gLp, -T.em / T.w, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(T.gRp, T.ep / T.w, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("P", PS)
def test_correction_integrals(P):
    """Integral of gL' over [-1,1] is g_L(1)-g_L(-1) = -1, of gR' is +1; the
    Gauss rule integrates these degree-P polynomials exactly."""
    T = tables.get(P)
    assert abs(np.sum(T.w * T.gLp) + 1.0) < 1e-13
    assert abs(np.sum(T.w * T.gRp) - 1.0) < 1e-13


def test_bad_order_rejected():
    with pytest.raises(ValueError):
        tables.build(0)

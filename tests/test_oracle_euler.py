"""Pins for the oracle's Euler physics: fluxes against hand-evaluated
states, Jacobians against complex-step derivatives of the fluxes,
eigenvectors against the Jacobians, Rusanov consistency and symmetry."""

import numpy as np
import pytest

import inputs
from oracle import euler

G = 1.4


def test_flux_hand_values():
    # rho=2, u=3, v=-1, p=5 -> e = 5/0.4 + 0.5*2*10 = 22.5
    q = inputs.conserved_from_primitive(2.0, 3.0, -1.0, 5.0, G)
    np.testing.assert_allclose(q, [2.0, 6.0, -2.0, 22.5])
    assert abs(euler.pressure(q, G) - 5.0) < 1e-14
    np.testing.assert_allclose(euler.flux_x(q, G), [6.0, 6 * 3 + 5, -6.0, 3 * 27.5], rtol=1e-15)
    np.testing.assert_allclose(euler.flux_y(q, G), [-2.0, -6.0, 2 + 5, -27.5], rtol=1e-15)
    c = np.sqrt(1.4 * 5 / 2)
    assert abs(euler.sound_speed(q, G) - c) < 1e-15
    assert abs(euler.normal_wave_speed(q, G, 0) - (3 + c)) < 1e-14
    assert abs(euler.normal_wave_speed(q, G, 1) - (1 + c)) < 1e-14
    assert abs(euler.max_wave_speed(q, G) - (np.sqrt(10) + c)) < 1e-14


@pytest.mark.parametrize("axis", [0, 1])
def test_jacobian_matches_complex_step(axis):
    q = inputs.random_state((7,), seed=3)
    A = euler.flux_jacobian(q, G, axis)
    F = euler.flux_x if axis == 0 else euler.flux_y
    h = 1e-30
    for b in range(4):
        dq = np.zeros((4, 7), dtype=complex)
        dq[b] = 1j * h
        col = F(q + dq, G).imag / h
        np.testing.assert_allclose(A[:, b], col, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("axis", [0, 1])
def test_eigenvectors_diagonalise_jacobian(axis):
    q = inputs.random_state((5,), seed=4)
    A = euler.flux_jacobian(q, G, axis)
    R, L = euler.eigenvectors(q, G, axis)
    un = q[1 + axis] / q[0]
    c = euler.sound_speed(q, G)
    for n in range(5):
        a, r, l = A[..., n], R[..., n], L[..., n]
        np.testing.assert_allclose(l @ r, np.eye(4), atol=1e-13)
        lam = np.diag([un[n] - c[n], un[n], un[n], un[n] + c[n]])
        np.testing.assert_allclose(l @ a @ r, lam, atol=1e-12)


@pytest.mark.parametrize("axis", [0, 1])
def test_rusanov_consistency_and_conservation(axis):
    qa = inputs.random_state((9,), seed=5)
    qb = inputs.random_state((9,), seed=6)
    F = euler.flux_x if axis == 0 else euler.flux_y
    np.testing.assert_allclose(euler.rusanov(qa, qa, G, axis), F(qa, G), rtol=1e-15)
    # lam = max of the two one-sided speeds
    lam = np.maximum(euler.normal_wave_speed(qa, G, axis), euler.normal_wave_speed(qb, G, axis))
    expect = 0.5 * (F(qa, G) + F(qb, G)) - 0.5 * lam * (qb - qa)
    np.testing.assert_allclose(euler.rusanov(qa, qb, G, axis), expect, rtol=1e-14)


def test_rusanov_mirror_symmetry():
    """Reflecting x -> -x swaps the sides and negates the normal momentum;
    the normal flux changes sign in every component except the normal
    momentum flux."""
    qa = inputs.random_state((9,), seed=7)
    qb = inputs.random_state((9,), seed=8)
    m = np.array([1.0, -1.0, 1.0, 1.0])[:, None]
    F1 = euler.rusanov(qa, qb, G, 0)
    F2 = euler.rusanov(m * qb, m * qa, G, 0)
    np.testing.assert_allclose(F2, -m * F1, rtol=1e-13, atol=1e-14)


def test_xy_swap_relates_fluxes():
    q = inputs.random_state((6,), seed=9)
    s = q[[0, 2, 1, 3]]
    np.testing.assert_allclose(euler.flux_y(s, G), euler.flux_x(q, G)[[0, 2, 1, 3]], rtol=1e-15)

"""Pins of the deviation form of the residual (oracle/deviation.py).

In float64 the form is an exact rewriting of the residual of Section 2.2, so
it must reproduce cpr.residual to rounding for every scheme, degree and
boundary; its flux deviation must equal the difference of two Euler flux
evaluations. In float32 its rounding must scale with the deviations inside
an element, not with the full flux."""

import numpy as np
import pytest

import inputs
from oracle import cpr, deviation, euler, tables


def _random_ref_and_dev(seed, shape=(50,)):
    rng = np.random.default_rng(seed)
    ref = inputs.conserved_from_primitive(rng.uniform(0.5, 1.5, shape), rng.uniform(-1, 1, shape),
                                          rng.uniform(-1, 1, shape), rng.uniform(0.5, 1.5, shape))
    q = inputs.conserved_from_primitive(rng.uniform(0.5, 1.5, shape), rng.uniform(-1, 1, shape),
                                        rng.uniform(-1, 1, shape), rng.uniform(0.5, 1.5, shape))
    return ref, q


@pytest.mark.parametrize("axis", [0, 1])
def test_deviation_flux_is_the_flux_difference(axis):
    ref, q = _random_ref_and_dev(1)
    c = deviation._ref_constants(ref, 1.4, axis, np.float64)
    dF, un, p, rho = deviation.deviation_flux(q - ref, c, 1.4, axis)
    F = euler.flux_x if axis == 0 else euler.flux_y
    want = F(q, 1.4) - F(ref, 1.4)
    assert np.max(np.abs(dF - want)) <= 1e-14 * np.max(np.abs(F(q, 1.4)))
    assert np.allclose(un, q[1 + axis] / q[0], rtol=1e-14, atol=1e-15)
    assert np.allclose(p, euler.pressure(q, 1.4), rtol=1e-13)
    assert np.allclose(rho, q[0], rtol=1e-15)


def test_deviation_flux_hand_values():
    """One state worked by hand: ref (rho, u, v, p) = (1, 0.5, 0, 1),
    q = (2, 1, 0.5, 2) in primitives, gamma = 1.4."""
    ref = inputs.conserved_from_primitive(1.0, 0.5, 0.0, 1.0)
    q = inputs.conserved_from_primitive(2.0, 1.0, 0.5, 2.0)
    c = deviation._ref_constants(ref, 1.4, 0, np.float64)
    dF, _, _, _ = deviation.deviation_flux(q - ref, c, 1.4, 0)
    # f(ref) = (0.5, 0.25 + 1, 0, 0.5 (2.5 + 0.125 + 1)) = (0.5, 1.25, 0, 1.8125)
    # e(q) = 2/0.4 + 0.5*2*(1 + 0.25) = 6.25; f(q) = (2, 2 + 2, 1, 1 (6.25 + 2)) = (2, 4, 1, 8.25)
    assert np.allclose(dF, [1.5, 2.75, 1.0, 6.4375], rtol=0, atol=1e-14)


SCHEMES = ["gl_lp", "gll_chain", "gll_lp"]


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("P", [1, 2, 3, 4])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_deviation_residual_equals_plain_residual(scheme, P, bc):
    g = cpr.Grid(P=P, nx=7, ny=5, x0=0.0, x1=2.0, y0=-1.0, y1=0.5, bc=bc, scheme=scheme)
    q = inputs.random_state((5, 7, P + 1, P + 1), seed=40 + P)
    R = cpr.residual(q, g)
    Rd = deviation.residual_deviation(q, g)
    assert np.max(np.abs(Rd - R)) <= 1e-13 * max(1.0, np.max(np.abs(R)))


@pytest.mark.parametrize("scheme", SCHEMES)
def test_deviation_residual_vortex_and_one_element(scheme):
    """Smooth data, and a 1 x 1 periodic mesh (an element is its own
    neighbour across every face)."""
    for nx, ny in ((12, 10), (1, 1)):
        g = cpr.Grid(P=3, nx=nx, ny=ny, scheme=scheme)
        x, y = g.coords()
        q = inputs.Vortex().conserved(x, y)
        R = cpr.residual(q, g)
        Rd = deviation.residual_deviation(q, g)
        assert np.max(np.abs(Rd - R)) <= 1e-13 * max(1.0, np.max(np.abs(R))), (nx, ny)


@pytest.mark.parametrize("n", [32, 64])
def test_float32_deviation_form_rounds_with_the_deviations(n):
    """On the P=3 vortex the float32 deviation form stays within
    64 u32 (2/h)(||D|| + 2||g'||) S of the float64 residual, S the
    largest flux deviation a line meets, and S is small against the full
    flux: the rounding no longer grows with |F| / h."""
    g = cpr.Grid(P=3, nx=n, ny=n)
    x, y = g.coords()
    q = inputs.Vortex().conserved(x, y)
    R = cpr.residual(q, g)
    R32 = deviation.residual_deviation(q, g, dtype=np.float32)
    T = tables.get(3)
    normD = np.max(np.sum(np.abs(T.D), axis=1))
    normg = max(np.max(np.abs(T.gLp)), np.max(np.abs(T.gRp)))
    S, _ = deviation.deviation_scales(q, g)
    Fmax = max(np.max(np.abs(euler.flux_x(q, 1.4))), np.max(np.abs(euler.flux_y(q, 1.4))))
    bound = 64 * 2.0 ** -24 * (2.0 / g.dx * (normD + 2 * normg) * S + np.max(np.abs(R)))
    err = np.max(np.abs(R32 - R))
    print(f"n={n}: max err {err:.3e}, deviation bound {bound:.3e}, S/Fmax {S / Fmax:.3e}")
    assert err <= bound
    assert S < 0.5 * Fmax
    # and the error of the float32 form does not grow with the mesh as
    # (2/h) u32 max|F| would: it stays below that scale by the ratio S/Fmax
    assert err <= 0.25 * 2.0 ** -24 * 2.0 / g.dx * (normD + 2 * normg) * Fmax

"""Pins for the oracle's second scheme, the paper's own CPR (Section 2.2
with Gauss-Lobatto solution points and the chain-rule divergence of its CPR
flux kernel, Algorithms 7 and 8): the Gauss-Lobatto rule against its closed
forms, the tables' exactness, a 30-digit brute force of the residual on tiny
meshes, free-stream preservation, and the consistency order of the residual
against the exact time derivative of a smooth entropy wave."""

import math

import numpy as np
import pytest

import inputs
from oracle import cpr, tables
from tests import mp_cpr

G = 1.4

# closed forms of the Gauss-Lobatto-Legendre rules (nodes ascending)
_GLL = {
    1: ([-1.0, 1.0], [1.0, 1.0]),
    2: ([-1.0, 0.0, 1.0], [1 / 3, 4 / 3, 1 / 3]),
    3: ([-1.0, -1 / math.sqrt(5), 1 / math.sqrt(5), 1.0], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    4: ([-1.0, -math.sqrt(3 / 7), 0.0, math.sqrt(3 / 7), 1.0],
        [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
}


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_lobatto_rule_closed_form(P):
    T = tables.get(P, "gll")
    xi, w = _GLL[P]
    np.testing.assert_allclose(T.xi, xi, rtol=0, atol=1e-15)
    np.testing.assert_allclose(T.w, w, rtol=1e-14, atol=0)


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_lobatto_tables_exactness(P):
    T = tables.get(P, "gll")
    # the rule integrates x^m exactly for m <= 2P-1
    for m in range(2 * P):
        exact = (1 - (-1) ** (m + 1)) / (m + 1)
        assert abs(np.sum(T.w * T.xi ** m) - exact) <= 1e-14
    # face values are end values: l_l(-1), l_l(+1) are unit vectors
    e0 = np.zeros(P + 1)
    e0[0] = 1.0
    assert np.array_equal(T.em, e0) and np.array_equal(T.ep, e0[::-1])
    # D differentiates every polynomial of degree <= P exactly
    for m in range(P + 1):
        d = T.D @ T.xi ** m
        ref = m * T.xi ** (m - 1) if m > 0 else 0 * T.xi
        assert np.max(np.abs(d - ref)) <= 1e-13
    # Radau derivatives at the end points from L_n'(+-1) = (+-1)^(n+1) n (n+1) / 2
    dL = lambda n, s: s ** (n + 1) * n * (n + 1) / 2
    s = (-1) ** (P + 1) / 2
    for i, x in ((0, -1), (P, 1)):
        assert abs(T.gLp[i] - s * (dL(P + 1, x) - dL(P, x))) <= 1e-13
        assert abs(T.gRp[i] - 0.5 * (dL(P + 1, x) + dL(P, x))) <= 1e-13


@pytest.mark.parametrize("P", [1, 2, 3, 4])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_bruteforce_2x2_gll_chain(P, bc):
    grid = cpr.Grid(P=P, nx=2, ny=2, x0=0.0, x1=2.0, y0=-1.0, y1=0.5, bc=bc, gamma=G,
                    scheme="gll_chain")
    q = inputs.random_state((2, 2, P + 1, P + 1), seed=40 + P)
    R = cpr.residual(q, grid)
    Rm = mp_cpr.residual(q.tolist(), P, 2, 2, 0.0, 2.0, -1.0, 0.5, bc, G, dps=30,
                         scheme="gll_chain")
    Rb = np.array([[[[[float(v) for v in r] for r in e] for e in row] for row in var]
                   for var in Rm])
    assert np.max(np.abs(R - Rb)) <= 1e-13 * np.max(np.abs(Rb))


@pytest.mark.parametrize("P", [1, 2, 3, 4])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_free_stream_preserved_gll_chain(P, bc):
    grid = cpr.Grid(P=P, nx=5, ny=4, bc=bc, scheme="gll_chain")
    q = np.zeros(grid.shape)
    q[0], q[1], q[2], q[3] = 1.3, 0.4, -0.7, 3.1
    assert np.max(np.abs(cpr.residual(q, grid))) <= 1e-13


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_residual_consistency_order_gll_chain(P):
    """Periodic entropy wave rho = 1 + 0.2 sin(2 pi (x + y)/10), u = v = 1,
    p = 1: the exact time derivative is -(d/dx + d/dy) q. The residual's
    pointwise error must fall at least like h^P under refinement."""
    errs = []
    for n in (6, 12):
        grid = cpr.Grid(P=P, nx=n, ny=n, scheme="gll_chain")
        x, y = grid.coords()
        q = inputs.entropy_wave(x, y)
        drho = -2 * (0.2 * 2 * np.pi / 10) * np.cos(2 * np.pi * (x + y) / 10)
        # u = v = 1 and p constant: rho u, rho v and e = p/(g-1) + rho move with rho
        exact = np.stack([drho, drho, drho, drho])
        R = cpr.residual(q, grid)
        errs.append(np.max(np.abs(R - exact)))
    assert errs[0] / errs[1] >= 2.0 ** P * 0.8, errs

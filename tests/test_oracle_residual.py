"""Pins for the oracle's CPR residual: 50-digit brute force on tiny meshes,
free-stream preservation, polynomial exactness, discrete conservation,
x<->y symmetry and mirror symmetry."""

import numpy as np
import pytest

import inputs
from oracle import cpr
from tests import mp_cpr

G = 1.4


def _grid(P, nx, ny, bc, x0=0.0, x1=1.0, y0=0.0, y1=1.0):
    return cpr.Grid(P=P, nx=nx, ny=ny, x0=x0, x1=x1, y0=y0, y1=y1, bc=bc, gamma=G)


@pytest.mark.parametrize("P", [1, 2, 3, 4])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_bruteforce_2x2(P, bc):
    grid = _grid(P, 2, 2, bc, 0.0, 2.0, -1.0, 0.5)
    q = inputs.random_state((grid.ny, grid.nx, grid.n1, grid.n1), seed=10 + P)
    R = cpr.residual(q, grid)
    Rm = mp_cpr.residual(q.tolist(), P, grid.nx, grid.ny, grid.x0, grid.x1, grid.y0,
                         grid.y1, bc, G, dps=30)
    Rb = np.array([[[[[float(v) for v in r] for r in e] for e in row] for row in var]
                   for var in Rm])
    scale = np.max(np.abs(Rb))
    assert np.max(np.abs(R - Rb)) <= 1e-13 * scale


def test_bruteforce_3x1_rectangular():
    grid = _grid(2, 3, 1, "periodic", 0.0, 3.0, 0.0, 0.5)
    q = inputs.random_state((grid.ny, grid.nx, grid.n1, grid.n1), seed=99)
    R = cpr.residual(q, grid)
    Rm = mp_cpr.residual(q.tolist(), 2, 3, 1, 0.0, 3.0, 0.0, 0.5, "periodic", G, dps=30)
    Rb = np.array([[[[[float(v) for v in r] for r in e] for e in row] for row in var]
                   for var in Rm])
    assert np.max(np.abs(R - Rb)) <= 1e-13 * np.max(np.abs(Rb))


@pytest.mark.parametrize("P", [1, 2, 3, 4])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_free_stream_preserved(P, bc):
    grid = _grid(P, 5, 3, bc)
    qf = inputs.conserved_from_primitive(0.8, 0.3, -0.7, 1.3, G)
    q = np.broadcast_to(qf[:, None, None, None, None], grid.shape).copy()
    assert np.max(np.abs(cpr.residual(q, grid))) < 1e-13


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_polynomial_density_wave_exact(P):
    """rho a tensor polynomial of degree <= P in x and y, constant u, v, p:
    all fluxes are affine in rho, face states agree, so the residual is the
    exact -(u rho_x + v rho_y)(1, u, v, (u^2+v^2)/2) at every point
    (transmissive mesh, so nothing has to be periodic)."""
    grid = _grid(P, 4, 3, "transmissive", -1.0, 1.0, 0.0, 1.5)
    x, y = grid.coords()
    u, v, p = 0.6, -0.4, 1.0
    a = np.linspace(0.05, 0.01, P + 1)
    rho = 1.0 + sum(a[m] * x ** m * 0.5 for m in range(1, P + 1)) + 0.1 * y ** P * x
    rx = sum(m * a[m] * x ** (m - 1) * 0.5 for m in range(1, P + 1)) + 0.1 * y ** P
    ry = 0.1 * P * y ** (P - 1) * x
    q = inputs.conserved_from_primitive(rho, u + 0 * x, v + 0 * x, p + 0 * x, G)
    R = cpr.residual(q, grid)
    adv = -(u * rx + v * ry)
    expect = np.stack([adv, u * adv, v * adv, 0.5 * (u * u + v * v) * adv])
    np.testing.assert_allclose(R, expect, atol=1e-12)


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_discrete_conservation_periodic(P):
    grid = _grid(P, 6, 5, "periodic", 0.0, 3.0, 0.0, 2.0)
    q = inputs.random_state((grid.ny, grid.nx, grid.n1, grid.n1), seed=20 + P)
    R = cpr.residual(q, grid)
    tot = cpr.integrals(R, grid)
    scale = np.max(np.abs(R)) * (grid.x1 - grid.x0) * (grid.y1 - grid.y0)
    assert np.max(np.abs(tot)) < 1e-14 * scale


@pytest.mark.parametrize("P", [2, 3])
def test_transmissive_boundary_flux_balance(P):
    """On a transmissive mesh, d/dt of the totals equals minus the net
    boundary flux, where each boundary face carries F(q_inside face)."""
    from oracle import euler, tables
    grid = _grid(P, 4, 3, "transmissive", 0.0, 2.0, 0.0, 1.5)
    q = inputs.random_state((grid.ny, grid.nx, grid.n1, grid.n1), seed=30 + P)
    R = cpr.residual(q, grid)
    T = tables.get(P)
    w = T.w
    qW = q[:, :, 0] @ T.em      # west column of elements, (4, ny, n1_j)
    qE = q[:, :, -1] @ T.ep
    qS = np.einsum("l,kIli->kIi", T.em, q[:, 0])
    qN = np.einsum("l,kIli->kIi", T.ep, q[:, -1])
    hy, hx = grid.dy / 2, grid.dx / 2
    flux = (np.einsum("kJj,j->k", euler.flux_x(qE, G) - euler.flux_x(qW, G), w) * hy
            + np.einsum("kIi,i->k", euler.flux_y(qN, G) - euler.flux_y(qS, G), w) * hx)
    np.testing.assert_allclose(cpr.integrals(R, grid), -flux, atol=1e-12)


@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_xy_transpose_symmetry(bc):
    grid = _grid(3, 4, 4, bc)
    q = inputs.random_state((4, 4, 4, 4), seed=41)
    qt = q[[0, 2, 1, 3]].transpose(0, 2, 1, 4, 3)
    R = cpr.residual(q, grid)
    Rt = cpr.residual(qt, grid)
    np.testing.assert_allclose(Rt, R[[0, 2, 1, 3]].transpose(0, 2, 1, 4, 3), atol=1e-12)


def test_mirror_symmetry_x():
    grid = _grid(2, 5, 3, "periodic")
    q = inputs.random_state((3, 5, 3, 3), seed=42)
    m = np.array([1.0, -1.0, 1.0, 1.0])[:, None, None, None, None]
    qm = (m * q)[:, :, ::-1, :, ::-1]
    R = cpr.residual(q, grid)
    Rm = cpr.residual(qm, grid)
    np.testing.assert_allclose(Rm, (m * R)[:, :, ::-1, :, ::-1], atol=1e-12)


def test_y_independent_data_has_no_y_terms():
    """Data constant along y: the y-flux divergence and y-corrections cancel,
    so each row evolves as the same 1D problem."""
    grid = _grid(3, 5, 4, "periodic")
    row = inputs.random_state((1, 5, 1, 4), seed=43)
    q = np.broadcast_to(row, (4, 4, 5, 4, 4)).copy()
    R = cpr.residual(q, grid)
    np.testing.assert_allclose(R, np.broadcast_to(R[:, :1, :, :1, :], R.shape), atol=1e-12)
    # and matches a one-element-tall mesh
    g1 = _grid(3, 5, 1, "periodic", y1=0.25)
    R1 = cpr.residual(q[:, :1], g1)
    np.testing.assert_allclose(R[:, :1], R1, atol=1e-12)

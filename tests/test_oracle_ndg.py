"""Pins for the oracle's "gll_lp" scheme, the paper's nodal DG (Section 2.4):
D f plus the lift L [F.n - F_com] with D = M^-1 S and L = M^-1 M^A, on
Gauss-Lobatto points. The oracle evaluates it in the differential form, as
CPR with the Radau correction on those points; the identities that make the
two the same operator are pinned here (the Radau derivatives at the nodes
are the lift columns of the exact mass matrix, and the derivative matrix is
M^-1 S), together with a 30-digit brute force of the residual, free-stream
preservation and discrete conservation."""

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import inputs
from oracle import cpr, tables
from tests import mp_cpr

G = 1.4


def exact_matrices(P):
    """M_ij = int l_i l_j and S_ij = int l_i l_j' over [-1, 1] for the
    Lobatto Lagrange basis, by a Gauss rule with P+2 points (exact for the
    degree-2P integrands)."""
    T = tables.get(P, "gll")
    x, w = npleg.leggauss(P + 2)
    Lx = tables.lagrange_eval(T.xi, x)          # (npts, n1)
    dLx = tables.lagrange_deriv(T.xi, x)
    M = np.einsum("a,ai,aj->ij", w, Lx, Lx)
    S = np.einsum("a,ai,aj->ij", w, Lx, dLx)
    return T, M, S


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_lift_is_radau_derivative(P):
    """The lift of a unit jump at the right face, M^-1 e_N (the face mass
    matrix of a 1D element is the end-point evaluation), equals gR' at the
    nodes, and at the left face -M^-1 e_0 equals gL'."""
    T, M, _ = exact_matrices(P)
    n1 = P + 1
    eN = np.zeros(n1)
    eN[-1] = 1.0
    e0 = np.zeros(n1)
    e0[0] = 1.0
    np.testing.assert_allclose(np.linalg.solve(M, eN), T.gRp, rtol=0, atol=1e-11)
    np.testing.assert_allclose(-np.linalg.solve(M, e0), T.gLp, rtol=0, atol=1e-11)


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_derivative_matrix_is_minv_s(P):
    T, M, S = exact_matrices(P)
    np.testing.assert_allclose(np.linalg.solve(M, S), T.D, rtol=0, atol=1e-11)


@pytest.mark.parametrize("P", [1, 2, 3, 4])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_bruteforce_2x2_gll_lp(P, bc):
    grid = cpr.Grid(P=P, nx=2, ny=2, x0=0.0, x1=2.0, y0=-1.0, y1=0.5, bc=bc, gamma=G,
                    scheme=cpr.GLL_LP)
    q = inputs.random_state((2, 2, P + 1, P + 1), seed=60 + P)
    R = cpr.residual(q, grid)
    Rm = mp_cpr.residual(q.tolist(), P, 2, 2, 0.0, 2.0, -1.0, 0.5, bc, G, dps=30,
                         scheme="gll_lp")
    Rb = np.array([[[[[float(v) for v in r] for r in e] for e in row] for row in var]
                   for var in Rm])
    assert np.max(np.abs(R - Rb)) <= 1e-13 * np.max(np.abs(Rb))


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_free_stream_and_conservation_gll_lp(P):
    g = cpr.Grid(P=P, nx=5, ny=4, scheme=cpr.GLL_LP)
    q = np.zeros(g.shape)
    q[0], q[1], q[2], q[3] = 1.3, 0.4, -0.7, 3.1
    assert np.max(np.abs(cpr.residual(q, g))) <= 1e-13
    q = inputs.random_state((4, 5, P + 1, P + 1), seed=70 + P)
    R = cpr.residual(q, g)
    assert np.max(np.abs(cpr.integrals(R, g))) <= 1e-13 * np.max(np.abs(R)) * 6.0

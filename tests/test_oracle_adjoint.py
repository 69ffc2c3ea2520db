"""Pins for the oracle's hand-written adjoint: each transpose is checked
against complex-step directional derivatives of the oracle's forward
(exact to roundoff, with |.| and max branch-fixed by real part), and the
full gradient against central finite differences."""

import numpy as np
import pytest

import inputs
from oracle import adjoint, cpr, euler

G = 1.4
H = 1e-30


def _cs_jvp(fn, q, d):
    return fn(q + 1j * H * d).imag / H


@pytest.mark.parametrize("axis", [0, 1])
def test_rusanov_vjp_dot_product(axis):
    qL = inputs.random_state((11,), seed=50)
    qR = inputs.random_state((11,), seed=51)
    # force a few ties and sign changes in u_n
    qR[:, 0] = qL[:, 0]
    qL[1 + axis, 1] = 0.0
    rng = np.random.default_rng(52)
    s = rng.standard_normal((4, 11))
    dL = rng.standard_normal((4, 11))
    dR = rng.standard_normal((4, 11))
    jv = (_cs_jvp(lambda z: euler.rusanov(z, qR, G, axis), qL, dL)
          + _cs_jvp(lambda z: euler.rusanov(qL, z, G, axis), qR, dR))
    cL, cR = adjoint.rusanov_vjp(qL, qR, s, G, axis)
    lhs = np.sum(s * jv, axis=0)
    rhs = np.sum(cL * dL + cR * dR, axis=0)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("P", [1, 2, 3, 4])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
@pytest.mark.parametrize("scheme", [cpr.GL_LP, cpr.GLL_LP, cpr.GLL_CHAIN])
def test_residual_vjp_dot_product(P, bc, scheme):
    g = cpr.Grid(P=P, nx=3, ny=4, x0=0.0, x1=1.5, y0=0.0, y1=2.0, bc=bc, scheme=scheme)
    q = inputs.random_state((g.ny, g.nx, g.n1, g.n1), seed=60 + P)
    rng = np.random.default_rng(70 + P)
    for _ in range(3):
        v = rng.standard_normal(g.shape)
        w = rng.standard_normal(g.shape)
        Jw = _cs_jvp(lambda z: cpr.residual(z, g), q, w)
        JTv = adjoint.residual_vjp(q, v, g)
        lhs, rhs = np.sum(v * Jw), np.sum(JTv * w)
        assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), np.sum(np.abs(v * Jw)))


def test_residual_vjp_full_matrix_small():
    """Every column of the Jacobian on a 2x1 P=1 mesh, against the VJP
    applied to every unit vector."""
    g = cpr.Grid(P=1, nx=2, ny=1, x1=1.0, y1=0.5)
    q = inputs.random_state((1, 2, 2, 2), seed=80)
    n = q.size
    J_cols = np.zeros((n, n))     # J_cols[:, a] = J e_a (complex step)
    J_rows = np.zeros((n, n))     # J_rows[a, :] = (J^T e_a)^T (adjoint)
    for a in range(n):
        e = np.zeros(n)
        e[a] = 1.0
        J_cols[:, a] = _cs_jvp(lambda z: cpr.residual(z, g), q, e.reshape(q.shape)).ravel()
        J_rows[a, :] = adjoint.residual_vjp(q, e.reshape(q.shape), g).ravel()
    np.testing.assert_allclose(J_rows, J_cols, rtol=1e-12, atol=1e-12 * np.abs(J_cols).max())


@pytest.mark.parametrize("scheme", [cpr.GL_LP, cpr.GLL_LP, cpr.GLL_CHAIN])
def test_rk3_adjoint_step_dot_product(scheme):
    g = cpr.Grid(P=2, nx=3, ny=3, x1=3.0, y1=3.0, scheme=scheme)
    q = inputs.random_state((3, 3, 3, 3), seed=90)
    dt = 0.05
    rng = np.random.default_rng(91)
    lam = rng.standard_normal(g.shape)
    w = rng.standard_normal(g.shape)
    jw = _cs_jvp(lambda z: cpr.rk3_step(z, dt, g), q, w)
    jtl = adjoint.rk3_adjoint_step(q, dt, lam, g)
    lhs, rhs = np.sum(lam * jw), np.sum(jtl * w)
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(lam * jw))


def test_gradient_matches_central_differences():
    """Misfit J = 1/2 ||rho(T) - rho_exact||^2 of a perturbed vortex after
    a few steps; directional derivatives by central differences with
    h = 1e-6 ||q||_inf/||d||_inf agree with <grad, d> to 1e-6 relative."""
    g = cpr.Grid(P=2, nx=5, ny=5)
    x, y = g.coords()
    V = inputs.Vortex()
    q0 = V.conserved(x, y)
    q0[0] += inputs.gaussian_perturbation(q0[0].shape, 1e-3, 0)
    dt, n = 0.05, 4
    rho_ex = V.conserved(x, y, dt * n)[0]
    J, grad = adjoint.gradient(q0, dt, n, g, rho_ex)

    def Jof(q):
        return adjoint.misfit(cpr.run(q, g, dt, n), rho_ex, g)

    for d in inputs.random_directions(g.shape, [1000, 1001, 1002]):
        h = 1e-6 * np.max(np.abs(q0)) / np.max(np.abs(d))
        fd = (Jof(q0 + h * d) - Jof(q0 - h * d)) / (2 * h)
        ad = np.sum(grad * d)
        assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)


@pytest.mark.parametrize("P", [1, 3])
def test_chain_rule_vjp_full_matrix(P):
    """Every column of the chain-rule residual's Jacobian on a 2x2 mesh by
    complex step, against the transpose applied to unit vectors."""
    g = cpr.Grid(P=P, nx=2, ny=2, x1=1.0, y1=0.8, scheme=cpr.GLL_CHAIN)
    q = inputs.random_state((2, 2, P + 1, P + 1), seed=90 + P)
    n = q.size
    J = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        J[:, c] = _cs_jvp(lambda z: cpr.residual(z, g), q, e.reshape(q.shape)).ravel()
    JT = np.zeros((n, n))
    for r in range(n):
        e = np.zeros(n)
        e[r] = 1.0
        JT[r, :] = adjoint.residual_vjp(q, e.reshape(q.shape), g).ravel()
    assert np.max(np.abs(JT - J)) <= 1e-12 * np.max(np.abs(J))

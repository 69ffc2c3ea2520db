"""Hand-written discrete adjoint of the CPR residual and of one SSP-RK3 step
(oracle, NumPy FP64).

residual_vjp(q, v) returns (dR/dq)^T v for the residual of oracle.cpr (all
three schemes), transposing each of its operations in reverse order: flux
evaluation (or, for the chain rule, the Jacobian-vector products and their
second derivatives), extrapolation to the faces, the Rusanov flux (including the derivative of
its wave-speed bound lam = max(|u_n|+c); sign(0) = +1 for |u_n|), the
correction lift and the derivative contraction. Where the two one-sided
speeds tie, |lamL - lamR| <= 1e-12 max(lamL, lamR), max is not
differentiable and its gradient is taken as the mean of the two sides'
gradients (a valid subgradient that does not depend on which side rounding
happens to favour; such ties occur exactly on the symmetry lines of the
isentropic vortex). rk3_adjoint_step transposes the Shu-Osher stages:
    lam2 = 2/3 (lam3 + dt J(q2)^T lam3)
    lam1 = 1/4 (lam2 + dt J(q1)^T lam2)
    lamn = lam1 + dt J(qn)^T lam1 + 1/3 lam3 + 3/4 lam2
The paper has no adjoint; this follows the definitions of the forward
operations above (Section 2.2 residual, Section 4 time stepping).
"""

from __future__ import annotations

import numpy as np

from . import cpr, euler
from .cpr import PERIODIC, Grid

TIE_REL = 1e-12   # relative gap below which the two Rusanov speeds count as tied


def _jac_t_apply(q, s, gamma, axis):
    """A(q)^T s (axis 0) or B(q)^T s (axis 1) pointwise."""
    A = euler.flux_jacobian(q, gamma, axis)
    return np.einsum("ab...,a...->b...", A, s)


def _wave_speed_grad(q, gamma, axis):
    """Gradient of |u_n| + c with respect to the conserved state."""
    rho, mx, my, e = q[0], q[1], q[2], q[3]
    u = mx / rho
    v = my / rho
    un = u if axis == 0 else v
    sgn = np.where(un >= 0.0, 1.0, -1.0)
    gg = gamma * (gamma - 1.0)
    c = euler.sound_speed(q, gamma)
    dc2 = np.stack([gg * (-e / (rho * rho) + (u * u + v * v) / rho),
                    -gg * u / rho, -gg * v / rho, gg / rho + 0.0 * rho])
    grad = dc2 / (2.0 * c)
    grad[0] = grad[0] - sgn * un / rho
    grad[1 + axis] = grad[1 + axis] + sgn / rho
    return grad


def rusanov_vjp(qL, qR, s, gamma, axis):
    """Cotangents (of qL, of qR) of the Rusanov flux for output cotangent s."""
    lamL = euler.normal_wave_speed(qL, gamma, axis)
    lamR = euler.normal_wave_speed(qR, gamma, axis)
    lam = np.where(lamL >= lamR, lamL, lamR)
    tie = np.abs(lamL - lamR) <= TIE_REL * np.maximum(lamL, lamR)
    wL = np.where(tie, 0.5, np.where(lamL > lamR, 1.0, 0.0))
    wR = 1.0 - wL
    jump = np.sum(s * (qR - qL), axis=0)
    cL = 0.5 * _jac_t_apply(qL, s, gamma, axis) + 0.5 * lam * s
    cR = 0.5 * _jac_t_apply(qR, s, gamma, axis) - 0.5 * lam * s
    cL = cL - 0.5 * jump * wL * _wave_speed_grad(qL, gamma, axis)
    cR = cR - 0.5 * jump * wR * _wave_speed_grad(qR, gamma, axis)
    return cL, cR


def _hess_apply(q, a, d, gamma, axis, h=1e-30):
    """d/dq [a . A(q) d] at every point (A = B for axis 1): the second
    derivatives of the flux contracted with a and d, by complex-step
    differentiation of the flux Jacobian along each conserved variable
    (exact to rounding for these rational formulas)."""
    out = np.zeros(q.shape)
    for m in range(4):
        qc = q.astype(complex)
        qc[m] = qc[m] + 1j * h
        A = euler.flux_jacobian(qc, gamma, axis)
        out[m] = np.imag(np.einsum("ab...,a...,b...->...", A, a, d)) / h
    return out


def residual_vjp(q, v, grid: Grid):
    """(dR/dq)^T v for R = oracle.cpr.residual; same shape as q. For the
    chain-rule scheme the divergence A(q_i)(Dq)_i transposes into
    D^T (A(q)^T a) (through Dq) plus the second-derivative term
    d/dq [a . A(q) (Dq)] at each point (through A); the face terms are those
    of the other schemes with the flux interpolant's face values."""
    chain = grid.scheme == cpr.GLL_CHAIN
    T = grid.tables()
    g = grid.gamma
    out = np.zeros_like(q)

    # ---------------- x direction ----------------
    a = -(2.0 / grid.dx) * v
    sW = a @ T.gLp                          # cotangent of F_W, (4, ny, nx, n1_j)
    sE = a @ T.gRp
    if chain:
        dq = np.einsum("il,kJIjl->kJIji", T.D, q)
        out += np.einsum("kJIji,il->kJIjl", _jac_t_apply(q, a, g, 0), T.D)
        out += _hess_apply(q, a, dq, g, 0)
        cot_f = np.zeros_like(q)
    else:
        cot_f = np.einsum("kJIji,il->kJIjl", a, T.D)
    cot_f -= sW[..., None] * T.em + sE[..., None] * T.ep
    # face fluxes 0..nx
    nx = grid.nx
    cot_F = np.zeros((4, grid.ny, nx + 1, grid.n1), dtype=q.dtype)
    cot_F[:, :, :-1, :] += sW
    cot_F[:, :, 1:, :] += sE
    left, right = cpr._x_face_states(q, grid)
    cl, cr = rusanov_vjp(left, right, cot_F, g, 0)
    cot_qE = cl[:, :, 1:, :].copy()
    cot_qW = cr[:, :, :-1, :].copy()
    if grid.bc == PERIODIC:
        cot_qE[:, :, -1, :] += cl[:, :, 0, :]
        cot_qW[:, :, 0, :] += cr[:, :, -1, :]
    else:
        cot_qW[:, :, 0, :] += cl[:, :, 0, :]
        cot_qE[:, :, -1, :] += cr[:, :, -1, :]
    out += cot_qW[..., None] * T.em + cot_qE[..., None] * T.ep
    out += _jac_t_apply(q, cot_f, g, 0)

    # ---------------- y direction ----------------
    b = -(2.0 / grid.dy) * v
    sS = np.einsum("kJIji,j->kJIi", b, T.gLp)
    sN = np.einsum("kJIji,j->kJIi", b, T.gRp)
    if chain:
        dq = np.einsum("jl,kJIli->kJIji", T.D, q)
        out += np.einsum("kJIji,jl->kJIli", _jac_t_apply(q, b, g, 1), T.D)
        out += _hess_apply(q, b, dq, g, 1)
        cot_g = np.zeros_like(q)
    else:
        cot_g = np.einsum("kJIji,jl->kJIli", b, T.D)
    cot_g -= sS[..., None, :] * T.em[:, None] + sN[..., None, :] * T.ep[:, None]
    ny = grid.ny
    cot_G = np.zeros((4, ny + 1, grid.nx, grid.n1), dtype=q.dtype)
    cot_G[:, :-1, :, :] += sS
    cot_G[:, 1:, :, :] += sN
    below, above = cpr._y_face_states(q, grid)
    cb, ca = rusanov_vjp(below, above, cot_G, g, 1)
    cot_qN = cb[:, 1:, :, :].copy()
    cot_qS = ca[:, :-1, :, :].copy()
    if grid.bc == PERIODIC:
        cot_qN[:, -1, :, :] += cb[:, 0, :, :]
        cot_qS[:, 0, :, :] += ca[:, -1, :, :]
    else:
        cot_qS[:, 0, :, :] += cb[:, 0, :, :]
        cot_qN[:, -1, :, :] += ca[:, -1, :, :]
    out += cot_qS[..., None, :] * T.em[:, None] + cot_qN[..., None, :] * T.ep[:, None]
    out += _jac_t_apply(q, cot_g, g, 1)
    return out


def rk3_adjoint_step(qn, dt, lam3, grid: Grid):
    """lam_n = (dq_{n+1}/dq_n)^T lam3 for one unlimited SSP-RK3 step."""
    qn, q1, q2, _ = cpr.rk3_stages(qn, dt, grid)
    lam2 = (2.0 / 3.0) * (lam3 + dt * residual_vjp(q2, lam3, grid))
    lam1 = 0.25 * (lam2 + dt * residual_vjp(q1, lam2, grid))
    return lam1 + dt * residual_vjp(qn, lam1, grid) + (1.0 / 3.0) * lam3 + 0.75 * lam2


def misfit(qT, rho_exact, grid: Grid):
    """J = 1/2 sum_e sum_ij w_i w_j (dx dy/4) (rho_ij(T) - rho_exact_ij)^2."""
    d = qT[0] - rho_exact
    return 0.5 * float(np.einsum("JIji,ji->", d * d, grid.quad_weights()))


def misfit_grad(qT, rho_exact, grid: Grid):
    lam = np.zeros_like(qT)
    lam[0] = (qT[0] - rho_exact) * grid.quad_weights()
    return lam


def gradient(q0, dt, nsteps, grid: Grid, rho_exact):
    """(J, dJ/dq0) by storing every step's state and sweeping back."""
    states = [q0]
    q = q0
    for _ in range(nsteps):
        q = cpr.rk3_step(q, dt, grid)
        states.append(q)
    J = misfit(q, rho_exact, grid)
    lam = misfit_grad(q, rho_exact, grid)
    for n in range(nsteps - 1, -1, -1):
        lam = rk3_adjoint_step(states[n], dt, lam, grid)
    return J, lam

"""CPR residual, SSP-RK3 time stepping and reductions (oracle, NumPy FP64).

Layout: a state is an array q[k, J, I, j, i] of shape (4, ny, nx, P+1, P+1):
k the conserved variable (rho, rho u, rho v, e), J the element row (y), I the
element column (x), j the eta index and i the xi index of the solution point.

Residual (Section 2.2, the differential form of CPR, eq. cpr2): at every
solution point dq/dt = -(Pi[div F] + delta). With Gauss-Legendre solution
points:
  * Pi[div F] is the divergence of the degree-P interpolant of the flux,
    (2/dx) sum_l D_il f_lj + (2/dy) sum_l D_jl g_il;
  * delta lifts the jump between the common interface flux and the
    interpolated flux at each face with the Radau correction polynomials,
    (2/dx)[(F_W - f_W) gL'(xi_i) + (F_E - f_E) gR'(xi_i)] plus the y terms,
    where f_W = sum_l l_l(-1) f_lj is the flux interpolant at the face;
  * the common flux F_W at each face point is the Rusanov flux (Section 4)
    of the two face states, each extrapolated from its element's solution
    polynomial.
Boundaries: periodic wrap, or transmissive (the outside state equals the
inside extrapolated state, so the face flux is F(q_inside)).

Scheme "gll_chain" is the paper's own CPR (Section 2.2 with Gauss-Lobatto
solution points; the chain-rule divergence of its CPR flux kernel,
Algorithms 7 and 8): the face states and face fluxes are the end values of
each line, and Pi[div F] is the chain rule A(q) dq/dx + B(q) dq/dy at every
solution point, with dq/dx the derivative of the solution polynomial. The
correction term is unchanged. The chain rule does not telescope, so this
scheme is not discretely conservative for the nonlinear fluxes.

Scheme "gll_lp" is the paper's nodal DG (NDG, Section 2.4: the strong form
with the flux derivative D f and the lift of the face-flux jumps, M^-1 E)
written in the same differential form: Gauss-Lobatto points, the derivative
of the flux interpolant, and the Radau correction, whose derivatives at the
nodes are the lift columns of the exact mass matrix. The same residual as
the default scheme on Lobatto points; discretely conservative.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import euler, tables

PERIODIC = "periodic"
TRANSMISSIVE = "transmissive"
GL_LP = "gl_lp"          # Gauss-Legendre points, derivative of the flux interpolant
GLL_CHAIN = "gll_chain"  # Gauss-Lobatto points, chain-rule divergence (the paper's CPR)
GLL_LP = "gll_lp"        # Gauss-Lobatto points, derivative of the flux interpolant (NDG)
SCHEMES = (GL_LP, GLL_CHAIN, GLL_LP)


@dataclass(frozen=True)
class Grid:
    P: int
    nx: int
    ny: int
    x0: float = 0.0
    x1: float = 10.0
    y0: float = 0.0
    y1: float = 10.0
    bc: str = PERIODIC
    gamma: float = 1.4
    scheme: str = GL_LP

    def __post_init__(self):
        if not (1 <= self.P <= 8):
            raise ValueError("P out of range")
        if self.nx < 1 or self.ny < 1:
            raise ValueError("mesh must have at least one element per direction")
        if not (self.x1 > self.x0 and self.y1 > self.y0):
            raise ValueError("empty domain")
        if self.bc not in (PERIODIC, TRANSMISSIVE):
            raise ValueError(f"unknown boundary condition {self.bc}")
        if not self.gamma > 1.0:
            raise ValueError("gamma must exceed 1")
        if self.scheme not in SCHEMES:
            raise ValueError(f"unknown scheme {self.scheme}")

    @property
    def n1(self):
        return self.P + 1

    @property
    def dx(self):
        return (self.x1 - self.x0) / self.nx

    @property
    def dy(self):
        return (self.y1 - self.y0) / self.ny

    @property
    def shape(self):
        return (4, self.ny, self.nx, self.n1, self.n1)

    @property
    def n_unknowns(self):
        return 4 * self.ny * self.nx * self.n1 * self.n1

    def tables(self):
        return tables.get(self.P, "gl" if self.scheme == GL_LP else "gll")

    def coords(self):
        """Physical coordinates (x, y), each of shape (ny, nx, n1, n1), of the
        solution points: x = x0 + (I + 1/2) dx + xi_i dx/2, same in y."""
        T = self.tables()
        I = np.arange(self.nx)
        J = np.arange(self.ny)
        xc = self.x0 + (I + 0.5) * self.dx
        yc = self.y0 + (J + 0.5) * self.dy
        x = xc[None, :, None, None] + 0.5 * self.dx * T.xi[None, None, None, :]
        y = yc[:, None, None, None] + 0.5 * self.dy * T.xi[None, None, :, None]
        x = np.broadcast_to(x, (self.ny, self.nx, self.n1, self.n1)).copy()
        y = np.broadcast_to(y, (self.ny, self.nx, self.n1, self.n1)).copy()
        return x, y

    def quad_weights(self):
        """w_i w_j dx dy / 4 at each solution point, shape (n1, n1)."""
        w = self.tables().w
        return np.outer(w, w) * (self.dx * self.dy / 4.0)


# ----------------------------------------------------------------------------
# Face states and common fluxes
# ----------------------------------------------------------------------------

def _x_face_states(q, grid: Grid):
    """States left and right of every x-face, faces 0..nx per element row.
    Face I is the west face of element I; face nx the east face of the last.
    Returns (left, right), each (4, ny, nx+1, n1) indexed by j."""
    T = grid.tables()
    qW = q @ T.em          # (4, ny, nx, n1_j): sum_i l_i(-1) q_ji
    qE = q @ T.ep
    if grid.bc == PERIODIC:
        ghost_w = qE[:, :, -1:, :]
        ghost_e = qW[:, :, :1, :]
    else:
        ghost_w = qW[:, :, :1, :]
        ghost_e = qE[:, :, -1:, :]
    left = np.concatenate([ghost_w, qE], axis=2)
    right = np.concatenate([qW, ghost_e], axis=2)
    return left, right


def _y_face_states(q, grid: Grid):
    """States below and above every y-face, faces 0..ny per element column.
    Returns (below, above), each (4, ny+1, nx, n1) indexed by i."""
    T = grid.tables()
    qS = np.einsum("l,kJIli->kJIi", T.em, q)
    qN = np.einsum("l,kJIli->kJIi", T.ep, q)
    if grid.bc == PERIODIC:
        ghost_s = qN[:, -1:, :, :]
        ghost_n = qS[:, :1, :, :]
    else:
        ghost_s = qS[:, :1, :, :]
        ghost_n = qN[:, -1:, :, :]
    below = np.concatenate([ghost_s, qN], axis=1)
    above = np.concatenate([qS, ghost_n], axis=1)
    return below, above


def residual(q, grid: Grid):
    """R(q) = dq/dt of the CPR semi-discretisation; same shape as q."""
    T = grid.tables()
    g = grid.gamma
    f = euler.flux_x(q, g)
    gf = euler.flux_y(q, g)

    chain = grid.scheme == GLL_CHAIN
    if chain:
        A = euler.flux_jacobian(q, g, 0)                 # (4, 4, ny, nx, n1, n1)
        B = euler.flux_jacobian(q, g, 1)

    # x direction (xi, last axis)
    if chain:
        dqdxi = np.einsum("il,kJIjl->kJIji", T.D, q)
        dfdxi = np.einsum("abJIji,bJIji->aJIji", A, dqdxi)
    else:
        dfdxi = np.einsum("il,kJIjl->kJIji", T.D, f)
    fW = f @ T.em
    fE = f @ T.ep
    left, right = _x_face_states(q, grid)
    Fx = euler.rusanov(left, right, g, 0)               # (4, ny, nx+1, n1)
    FW = Fx[:, :, :-1, :]
    FE = Fx[:, :, 1:, :]
    Rx = dfdxi + (FW - fW)[..., None] * T.gLp + (FE - fE)[..., None] * T.gRp

    # y direction (eta, second-last axis)
    if chain:
        dqdeta = np.einsum("jl,kJIli->kJIji", T.D, q)
        dgdeta = np.einsum("abJIji,bJIji->aJIji", B, dqdeta)
    else:
        dgdeta = np.einsum("jl,kJIli->kJIji", T.D, gf)
    gS = np.einsum("l,kJIli->kJIi", T.em, gf)
    gN = np.einsum("l,kJIli->kJIi", T.ep, gf)
    below, above = _y_face_states(q, grid)
    Gy = euler.rusanov(below, above, g, 1)              # (4, ny+1, nx, n1)
    GS = Gy[:, :-1, :, :]
    GN = Gy[:, 1:, :, :]
    Ry = (dgdeta + (GS - gS)[..., None, :] * T.gLp[:, None]
          + (GN - gN)[..., None, :] * T.gRp[:, None])

    return -(2.0 / grid.dx) * Rx - (2.0 / grid.dy) * Ry


# ----------------------------------------------------------------------------
# Time integration (Section 4: three-stage Runge-Kutta of Shu and Osher)
# ----------------------------------------------------------------------------

def rk3_step(q, dt, grid: Grid, limit=None):
    """One SSP-RK3 step in Shu-Osher form:
        q1 = qn + dt R(qn)
        q2 = 3/4 qn + 1/4 (q1 + dt R(q1))
        q3 = 1/3 qn + 2/3 (q2 + dt R(q2))
    limit, if given, is applied to each stage result (Section 2.6: the
    limiter acts after each update)."""
    lim = (lambda s: s) if limit is None else limit
    q1 = lim(q + dt * residual(q, grid))
    q2 = lim(0.75 * q + 0.25 * (q1 + dt * residual(q1, grid)))
    q3 = lim((1.0 / 3.0) * q + (2.0 / 3.0) * (q2 + dt * residual(q2, grid)))
    return q3


def rk3_stages(q, dt, grid: Grid):
    """The three stage states (qn, q1, q2) and q3 of one unlimited step."""
    q1 = q + dt * residual(q, grid)
    q2 = 0.75 * q + 0.25 * (q1 + dt * residual(q1, grid))
    q3 = (1.0 / 3.0) * q + (2.0 / 3.0) * (q2 + dt * residual(q2, grid))
    return q, q1, q2, q3


def cfl_dt(q, grid: Grid, cfl):
    """dt = CFL * h / max(sqrt(u^2+v^2) + c), h = min(dx, dy) the element
    size (Section 4, the CFL condition)."""
    lam = np.max(euler.max_wave_speed(q, grid.gamma))
    return cfl * min(grid.dx, grid.dy) / lam


def run(q, grid: Grid, dt, nsteps, limit=None):
    for _ in range(nsteps):
        q = rk3_step(q, dt, grid, limit)
    return q


# ----------------------------------------------------------------------------
# Reductions
# ----------------------------------------------------------------------------

def integrals(q, grid: Grid):
    """Domain integrals of the four conserved variables by the tensor
    Gauss-Legendre rule: sum_e sum_ij w_i w_j (dx dy/4) q_k,ij."""
    W = grid.quad_weights()
    return np.einsum("kJIji,ji->k", q, W)


def element_means(q, grid: Grid):
    """Element averages (1/4) sum_ij w_i w_j q_ij, shape (4, ny, nx)."""
    w = grid.tables().w
    return 0.25 * np.einsum("kJIji,j,i->kJI", q, w, w)


def l2_error(a, b, grid: Grid):
    """Area-normalised quadrature L2 norm of a - b (one variable, shape
    (ny, nx, n1, n1)): sqrt(sum w_i w_j (dx dy/4) (a-b)^2 / |Omega|)."""
    W = grid.quad_weights()
    area = (grid.x1 - grid.x0) * (grid.y1 - grid.y0)
    d = a - b
    return float(np.sqrt(np.einsum("JIji,ji->", d * d, W) / area))


def l2_error_of_means(a, b, grid: Grid):
    """Error of element averages, RMS over elements (the paper compares the
    averaged solution with the averaged exact solution, Section 4)."""
    w = grid.tables().w
    ma = 0.25 * np.einsum("JIji,j,i->JI", a, w, w)
    mb = 0.25 * np.einsum("JIji,j,i->JI", b, w, w)
    return float(np.sqrt(np.mean((ma - mb) ** 2)))

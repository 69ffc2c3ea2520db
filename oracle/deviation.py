"""The CPR residual in deviation form (oracle; test infrastructure only).

The reduced-precision residual form evaluates the same residual as
cpr.residual (Section 2.2, the differential form with the Radau correction
and the Rusanov face flux of Section 4), rewritten so that every quantity it
rounds is a deviation from a reference state instead of a full flux value.

Each element line (a row for the x part of the residual, a column for the y
part) takes as its reference q_ref its own first solution point. Then, in
exact arithmetic:
  * the divergence of the flux interpolant is D (F - F(q_ref)): the rows of
    D sum to zero, so a constant added to F drops out;
  * the interpolant's face values are e (F - F(q_ref)) + F(q_ref): the
    extrapolation rows sum to one;
  * the Rusanov flux of two face states is
    1/2 (dF(qL) + dF(qR)) - 1/2 lam (dqR - dqL) + F(q_ref), with dF and dq
    the deviations from the reference of the line whose residual is formed
    (both face states, the neighbour's included, are written in that line's
    frame);
so the correction terms F_face - f_face are differences of deviations, and
F(q_ref) never needs to be formed. The deviation of the flux itself,
dF = F(q_ref + dq) - F(q_ref), is written from dq and the reference's
primitive values with the product rule, so that it is small wherever dq is:
with rho = rho_r + drho,
  du_n = (dm_n - u_n,r drho) / rho,
  dK   = ((m_r + dm/2) . dm - K_r drho) / rho       (K = |m|^2 / (2 rho)),
  dp   = (gamma - 1) (dE - dK),
  dF   = (dm_n, dm_n u_n + m_n,r du_n + dp, dm_t u_n + m_t,r du_n,
          du_n (E_r + p_r + dE + dp) + u_n,r (dE + dp)),
in the (mass, normal momentum, tangential momentum, energy) order, where
u_n = u_n,r + du_n is the full normal velocity.

The chain-rule scheme (gll_chain) forms A(q)(D q): D q = D dq, and A(q) is
evaluated at the full state rebuilt from the reference and the deviation.

In float64 (the default) this equals cpr.residual to rounding, which
tests/test_oracle_deviation.py pins; evaluated in float32 (dtype argument)
it models the reduced-precision arithmetic, whose rounding then scales with
the deviations within an element rather than with the full fluxes.
"""

from __future__ import annotations

import numpy as np

from . import cpr, euler


def _ref_constants(ref, gamma, axis, dtype):
    """Primitive values of the reference state, formed in float64 and then
    rounded to dtype: rho, m_n, m_t, u_n, u_t, p, E + p (normal along axis)."""
    rho, mx, my, e = ref[0], ref[1], ref[2], ref[3]
    u = mx / rho
    v = my / rho
    p = (gamma - 1.0) * (e - 0.5 * (mx * u + my * v))
    mn, mt, un, ut = (mx, my, u, v) if axis == 0 else (my, mx, v, u)
    c = dict(rho=rho, mn=mn, mt=mt, un=un, ut=ut, p=p, H=e + p, K=0.5 * (mx * u + my * v))
    return {k: np.asarray(val, dtype=np.float64).astype(dtype) for k, val in c.items()}


def deviation_flux(d, c, gamma, axis):
    """(dF, u_n, p, rho): dF = F(q_ref + d) - F(q_ref) for the flux along
    axis (0: f, 1: g) from the deviation d (leading axis: rho, rho u, rho v,
    e) and the reference constants c; also the full normal velocity,
    pressure and density (for the Rusanov wave speed)."""
    dt = d.dtype.type
    gm1 = dt(gamma - 1.0)
    half = dt(0.5)
    dr, de = d[0], d[3]
    dmn, dmt = (d[1], d[2]) if axis == 0 else (d[2], d[1])
    rho = c["rho"] + dr
    ir = dt(1.0) / rho
    dun = (dmn - c["un"] * dr) * ir
    un = c["un"] + dun
    # K = |m|^2 / (2 rho): dK = ((m_r + dm/2) . dm - K_r drho) / rho
    dK = ((c["mn"] + half * dmn) * dmn + (c["mt"] + half * dmt) * dmt - c["K"] * dr) * ir
    dp = gm1 * (de - dK)
    dFn = dmn * un + c["mn"] * dun + dp
    dFt = dmt * un + c["mt"] * dun
    dF3 = dun * (c["H"] + de + dp) + c["un"] * (de + dp)
    if axis == 0:
        F = np.stack([dmn, dFn, dFt, dF3])
    else:
        F = np.stack([dmn, dFt, dFn, dF3])
    return F, un, c["p"] + dp, rho


def _wave_speed(un, p, rho, gamma):
    return np.abs(un) + np.sqrt(rho.dtype.type(gamma) * p / rho)


def _line_residual(q, grid: cpr.Grid, dtype):
    """x part of the residual (lines along the last axis of q, elements
    along axis 2), in deviation form; returns the bracket
    D dF + (F_W - f_W) gL' + (F_E - f_E) gR' (before the -2/dx factor)."""
    T = grid.tables()
    g = grid.gamma
    D, em, ep = T.D.astype(dtype), T.em.astype(dtype), T.ep.astype(dtype)
    gLp, gRp = T.gLp.astype(dtype), T.gRp.astype(dtype)
    chain = grid.scheme == cpr.GLL_CHAIN
    lob = grid.scheme != cpr.GL_LP
    ref = q[..., 0]                                   # (4, ny, nx, n1): one per line
    c = _ref_constants(ref, g, 0, dtype)
    cl = {k: v[..., None] for k, v in c.items()}      # broadcast over the line
    d = (q - ref[..., None]).astype(dtype)            # deviations, rounded once
    dF, un, p, rho = deviation_flux(d, cl, g, 0)

    def face(dq):
        return dq[..., 0] if lob else dq @ em

    def face_hi(dq):
        return dq[..., -1] if lob else dq @ ep

    dlo, dhi = face(d), face_hi(d)                    # own face states (own frame)
    if chain:
        dq_dx = np.einsum("il,kJIjl->kJIji", D, d)
        qfull = (ref[..., None].astype(dtype) + d)
        A = euler.flux_jacobian(qfull, g, 0).astype(dtype)
        div = np.einsum("abJIji,bJIji->aJIji", A, dq_dx)
    else:
        div = np.einsum("il,kJIjl->kJIji", D, dF)
    flo, fhi = face(dF), face_hi(dF)

    # neighbour face states in this line's frame: the neighbour's deviation
    # extrapolated, plus the difference of the two references (float64)
    nx = q.shape[2]
    left = np.roll(np.arange(nx), 1)
    right = np.roll(np.arange(nx), -1)
    dm = (ref[:, :, left] - ref).astype(dtype) + dhi[:, :, left]
    dp_ = (ref[:, :, right] - ref).astype(dtype) + dlo[:, :, right]
    if grid.bc == cpr.TRANSMISSIVE:
        dm[:, :, 0] = dlo[:, :, 0]
        dp_[:, :, -1] = dhi[:, :, -1]

    def rusanov(dL, dR):
        FL, unL, pL, rL = deviation_flux(dL, c, g, 0)
        FR, unR, pR, rR = deviation_flux(dR, c, g, 0)
        lam = np.maximum(_wave_speed(unL, pL, rL, g), _wave_speed(unR, pR, rR, g))
        half = dtype(0.5)
        return half * (FL + FR) - half * lam * (dR - dL)

    FW = rusanov(dm, dlo)
    FE = rusanov(dhi, dp_)
    return div + (FW - flo)[..., None] * gLp + (FE - fhi)[..., None] * gRp


def _swap_xy(q):
    """Transpose a state: x <-> y, rho u <-> rho v."""
    return np.ascontiguousarray(q[[0, 2, 1, 3]].transpose(0, 2, 1, 4, 3))


def residual_deviation(q, grid: cpr.Grid, dtype=np.float64):
    """R(q) of cpr.residual, in deviation form, computed in dtype (the
    state q itself is float64; the result is returned as float64)."""
    dtype = np.dtype(dtype).type
    rx = _line_residual(q, grid, dtype)
    gt = cpr.Grid(P=grid.P, nx=grid.ny, ny=grid.nx, x0=grid.y0, x1=grid.y1, y0=grid.x0,
                  y1=grid.x1, bc=grid.bc, gamma=grid.gamma, scheme=grid.scheme)
    ry = _swap_xy(_line_residual(_swap_xy(q), gt, dtype).astype(np.float64))
    return -(2.0 / grid.dx) * rx.astype(np.float64) - (2.0 / grid.dy) * ry


def deviation_scales(q, grid: cpr.Grid):
    """Forward-error scales of the deviation form: the largest deviations
    any line's rounding acts on, over every line and over the adjacent
    elements' points across either face (a neighbour's face state enters in
    the line's frame). Returns (S_flux, S_state): the largest flux deviation
    |F(q) - F(q_ref)| and the largest state deviation |q - q_ref| (which the
    chain rule's D q rounds)."""
    g = grid.gamma
    sf = ss = 0.0
    for axis in (0, 1):
        qq = q if axis == 0 else np.swapaxes(q, -1, -2)
        F = euler.flux_x if axis == 0 else euler.flux_y
        ref = np.broadcast_to(qq[..., :1], qq.shape)
        el = 2 if axis == 0 else 1
        Fr = F(ref, g)
        for shift in (0, 1, -1):
            qs = np.roll(qq, shift, axis=el)
            sf = max(sf, float(np.max(np.abs(F(qs, g) - Fr))))
            ss = max(ss, float(np.max(np.abs(qs - ref))))
    return sf, ss

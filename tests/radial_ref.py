"""Reference solution of the radially expanding shock tube (the paper's
discontinuous problem, Section 4) from the equivalent one-dimensional
problem: with cylindrical symmetry the Euler equations reduce to

    d(r U)/dt + d(r F)/dr = (0, p, 0),   U = (rho, rho u, E),
    F = (rho u, rho u^2 + p, u (E + p)),

the radial form Toro uses for his reference solutions of this problem. It is
solved here by a finite-volume method on a fine grid: cells of width dr on
[0, R], face areas r_{i+1/2}, linear reconstruction of the primitive
variables with the minmod limiter, the HLL flux, the pressure source p_i/r_i
(with which a uniform state at rest is exactly steady), SSP-RK3 in time, a
mirror ghost cell at r = 0 and a copied one at r = R.

Test infrastructure only: it validates the 2D solutions of both the oracle
and the GPU path against the physics of the problem, standing in for the
paper's digitised reference profile; it shares nothing with either."""

import numpy as np


def _prim(U, g):
    rho = U[0]
    u = U[1] / rho
    p = (g - 1.0) * (U[2] - 0.5 * rho * u * u)
    return rho, u, p


def _flux(rho, u, p, g):
    E = p / (g - 1.0) + 0.5 * rho * u * u
    return np.stack([rho * u, rho * u * u + p, u * (E + p)]), np.stack([rho, rho * u, E])


def _minmod(a, b):
    return np.where(a * b > 0.0, np.sign(a) * np.minimum(np.abs(a), np.abs(b)), 0.0)


def _rhs(U, rc, rf, dr, g, planar=False):
    rho, u, p = _prim(U, g)
    W = np.stack([rho, u, p])
    # ghosts: mirror at r = 0 (u -> -u), copy at r = R
    Wl = np.stack([rho[0], -u[0], p[0]])[:, None]
    Wr = W[:, -1:]
    Wg = np.concatenate([Wl, W, Wr], axis=1)
    s = _minmod(Wg[:, 1:-1] - Wg[:, :-2], Wg[:, 2:] - Wg[:, 1:-1])
    # face states: left of face i+1/2 from cell i, right from cell i+1
    WL = W + 0.5 * s            # at the outer face of each cell
    WR = W - 0.5 * s            # at the inner face of each cell
    # the outer face of cell i has cell i on its left and cell i+1 (for the
    # last cell, the copied ghost) on its right; the face at r = 0 has zero
    # area and carries no flux
    qL = WL
    qR = np.concatenate([WR[:, 1:], WL[:, -1:]], axis=1)
    FL, UL = _flux(qL[0], qL[1], qL[2], g)
    FR, UR = _flux(qR[0], qR[1], qR[2], g)
    cL = np.sqrt(g * qL[2] / qL[0])
    cR = np.sqrt(g * qR[2] / qR[0])
    sL = np.minimum(qL[1] - cL, qR[1] - cR)
    sR = np.maximum(qL[1] + cL, qR[1] + cR)
    hll = (sR * FL - sL * FR + sL * sR * (UR - UL)) / (sR - sL)
    F = np.where(sL >= 0.0, FL, np.where(sR <= 0.0, FR, hll))
    if planar:
        # slab geometry (unit face areas, no source) with a mirror at 0: the
        # wall flux is the pressure alone
        flux_out = F
        wall = np.stack([0.0, p[0], 0.0])[:, None]
        flux_in = np.concatenate([wall, flux_out[:, :-1]], axis=1)
        return -(flux_out - flux_in) / dr, u, p, rho
    flux_out = rf[1:] * F                       # outer face of each cell
    flux_in = np.concatenate([np.zeros((3, 1)), flux_out[:, :-1]], axis=1)
    dU = -(flux_out - flux_in) / (rc * dr)
    dU[1] += p / rc
    return dU, u, p, rho


def solve(t_end, n=4000, R=1.2, gamma=1.4, cfl=0.4, radius=0.4, inside=(1.0, 1.0),
          outside=(0.125, 0.1), planar=False):
    """Cell centres and (rho, u, p) at t_end on n cells of [0, R]. planar:
    the same method in slab geometry (a plane Riemann problem at x =
    radius, wall at 0), used to check it against an exact solution."""
    g = gamma
    dr = R / n
    rf = np.arange(n + 1) * dr
    rc = 0.5 * (rf[:-1] + rf[1:])
    inner = rc < radius
    rho = np.where(inner, inside[0], outside[0])
    p = np.where(inner, inside[1], outside[1])
    u = np.zeros(n)
    _, U = _flux(rho, u, p, g)
    t = 0.0
    while t < t_end:
        rho, u, p = _prim(U, g)
        lam = np.max(np.abs(u) + np.sqrt(g * p / rho))
        dt = min(cfl * dr / lam, t_end - t)
        k1, *_ = _rhs(U, rc, rf, dr, g, planar)
        U1 = U + dt * k1
        k2, *_ = _rhs(U1, rc, rf, dr, g, planar)
        U2 = 0.75 * U + 0.25 * (U1 + dt * k2)
        k3, *_ = _rhs(U2, rc, rf, dr, g, planar)
        U = U / 3.0 + 2.0 / 3.0 * (U2 + dt * k3)
        t += dt
    rho, u, p = _prim(U, g)
    return rc, rho, u, p


def density_at(r, rc, rho):
    """Reference density at radii r (linear interpolation between cells)."""
    return np.interp(r, rc, rho)


def metrics(rho, x, y, W, w1d, rc, rho_ref):
    """Distances of a 2D density field from the reference, as integrals
    (rho, x, y of shape (ny, nx, n1, n1); W the per-point weights
    w_i w_j dx dy / 4 of shape (n1, n1); w1d the 1D weights):
      domain L1 = integral |rho - rho_ref(r)| dA / area;
      centre-row L1 = the same along the lowest row of points of element
      row ny/2 (the row of points nearest the centre line y = 0, above it),
      integral over x / length."""
    r = np.sqrt(x * x + y * y)
    d = np.abs(rho - density_at(r, rc, rho_ref))
    ny, nx = rho.shape[:2]
    l1 = float(np.einsum("JIji,ji->", d, W) / (W.sum() * ny * nx))
    row = d[ny // 2, :, 0, :]
    l1c = float(np.sum(row * np.asarray(w1d)[None, :]) / (2.0 * nx))
    return l1, l1c

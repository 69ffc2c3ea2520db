"""Seeded, synthetic inputs shared by the GPU path, the oracle and the tests.

This module holds problem definitions only: closed-form initial and exact
fields evaluated at coordinates the caller supplies, and seeded random states.
It contains none of the CPR method's arithmetic (no quadrature points, no
Lagrange or correction tables, no fluxes, no time stepping). Each caller builds
its own solution-point coordinates from its own tables and passes them in.

State convention: conserved variables (rho, rho*u, rho*v, e), stacked on a new
leading axis of length 4, with e = p/(gamma-1) + rho*(u^2+v^2)/2 (the ideal-gas
closure of the paper's Euler system, Section 2, the state/flux/EOS equations).
"""

from __future__ import annotations

import math

import numpy as np

GAMMA = 1.4


def conserved_from_primitive(rho, u, v, p, gamma=GAMMA):
    """Stack (rho, rho u, rho v, e) from primitive fields of any common shape."""
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    e = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.stack(np.broadcast_arrays(rho, rho * u, rho * v, e)).astype(np.float64)


# ----------------------------------------------------------------------------
# Isentropic vortex (Section 4.1, smooth problem; velocity, temperature and
# entropy perturbations of a uniform mean flow, advected unchanged).
# ----------------------------------------------------------------------------

class Vortex:
    """Isentropic vortex on a periodic square.

    Defaults: strength eps=5 on the periodic square [0,10]^2 with its centre at
    (5,5), mean flow rho=p=1, u=v=1, gamma=1.4. The paper's own set-up is
    eps=5, mean (1,1,0,1) on [-5,5]^2 (Section 4.1); both are instances of this
    class. The exact solution at time t is the initial field translated by
    (u_inf t, v_inf t); offsets from the centre use the minimum periodic image.
    """

    def __init__(self, eps=5.0, gamma=GAMMA, lo=0.0, hi=10.0, rho_inf=1.0,
                 u_inf=1.0, v_inf=1.0, p_inf=1.0, center=None):
        self.eps = float(eps)
        self.gamma = float(gamma)
        self.lo = float(lo)
        self.hi = float(hi)
        self.L = self.hi - self.lo
        self.rho_inf = float(rho_inf)
        self.u_inf = float(u_inf)
        self.v_inf = float(v_inf)
        self.p_inf = float(p_inf)
        c = 0.5 * (self.lo + self.hi)
        self.center = (c, c) if center is None else (float(center[0]), float(center[1]))

    def _offset(self, x, xc):
        d = np.asarray(x, dtype=np.float64) - xc
        return d - self.L * np.round(d / self.L)

    def primitive(self, x, y, t=0.0):
        xc = self.center[0] + self.u_inf * t
        yc = self.center[1] + self.v_inf * t
        xb = self._offset(x, xc)
        yb = self._offset(y, yc)
        r2 = xb * xb + yb * yb
        g = self.gamma
        amp = self.eps / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
        u = self.u_inf - amp * yb
        v = self.v_inf + amp * xb
        # temperature T = p/rho, normalised so that T_inf = p_inf/rho_inf = 1
        T = 1.0 - (g - 1.0) * self.eps ** 2 / (8.0 * g * math.pi ** 2) * np.exp(1.0 - r2)
        # isentropic: p / rho^gamma constant (= 1 for the unit free stream)
        rho = self.rho_inf * T ** (1.0 / (g - 1.0))
        p = self.p_inf * (rho / self.rho_inf) ** g
        return rho, u, v, p

    def conserved(self, x, y, t=0.0):
        rho, u, v, p = self.primitive(x, y, t)
        return conserved_from_primitive(rho, u, v, p, self.gamma)

    def free_stream(self):
        return conserved_from_primitive(self.rho_inf, self.u_inf, self.v_inf,
                                        self.p_inf, self.gamma)


# ----------------------------------------------------------------------------
# Four-quadrant Riemann problem on [0,1]^2 split at x = y = 0.5.
# ----------------------------------------------------------------------------

RIEMANN_QUADRANTS = {
    # (rho, u, v, p)
    "NE": (1.5, 0.0, 0.0, 1.5),
    "NW": (0.5323, 1.206, 0.0, 0.3),
    "SW": (0.138, 1.206, 1.206, 0.029),
    "SE": (0.5323, 0.0, 1.206, 0.3),
}


def riemann_quadrants(x, y, gamma=GAMMA, split=(0.5, 0.5), states=None):
    s = RIEMANN_QUADRANTS if states is None else states
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    east = x > split[0]
    north = y > split[1]
    prim = np.empty((4,) + np.broadcast(x, y).shape, dtype=np.float64)
    for name, mask in (("NE", east & north), ("NW", ~east & north),
                       ("SW", ~east & ~north), ("SE", east & ~north)):
        for k in range(4):
            prim[k][mask] = s[name][k]
    return conserved_from_primitive(prim[0], prim[1], prim[2], prim[3], gamma)


# ----------------------------------------------------------------------------
# Radially expanding shock tube on [-1,1]^2 (the paper's discontinuous
# problem, Section 4, after Toro): rho = p = 1 inside the circle r < 0.4,
# rho = 0.125, p = 0.1 outside, fluid at rest.
# ----------------------------------------------------------------------------

def radial_shock_tube(x, y, gamma=GAMMA, radius=0.4, inside=(1.0, 1.0),
                      outside=(0.125, 0.1)):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    r2 = x * x + y * y
    inner = r2 < radius * radius
    rho = np.where(inner, inside[0], outside[0])
    p = np.where(inner, inside[1], outside[1])
    zero = np.zeros_like(rho)
    return conserved_from_primitive(rho, zero, zero, p, gamma)


# The largest CFL the paper lists for each method on this problem (Table 4),
# by degree and mesh (160k/640k unknowns per variable at P1 are 200^2/400^2
# elements, 360k/1440k at P2 likewise). Keys: the scheme that reproduces each
# method here (gl_lp: DG, gll_chain: CPR, gll_lp: NDG).
RADIAL_TUBE_CFL = {
    ("gl_lp", 1, 200): 0.22, ("gl_lp", 1, 400): 0.2,
    ("gl_lp", 2, 200): 0.08, ("gl_lp", 2, 400): 0.08,
    ("gll_chain", 1, 200): 0.2, ("gll_chain", 1, 400): 0.2,
    ("gll_chain", 2, 200): 0.1, ("gll_chain", 2, 400): 0.1,
    ("gll_lp", 1, 200): 0.2, ("gll_lp", 1, 400): 0.2,
    ("gll_lp", 2, 200): 0.1, ("gll_lp", 2, 400): 0.1,
}


# ----------------------------------------------------------------------------
# Entropy (density) wave: rho = 1 + a sin(2 pi (x+y)/L), u = v = 1, p = 1,
# advected unchanged; a smooth periodic field with no vortex tail.
# ----------------------------------------------------------------------------

def entropy_wave(x, y, t=0.0, amp=0.2, L=10.0, u=1.0, v=1.0, p=1.0, gamma=GAMMA):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    rho = 1.0 + amp * np.sin(2.0 * math.pi * ((x - u * t) + (y - v * t)) / L)
    return conserved_from_primitive(rho, u + 0 * rho, v + 0 * rho, p + 0 * rho, gamma)


# ----------------------------------------------------------------------------
# Seeded random inputs.
# ----------------------------------------------------------------------------

def random_state(shape, seed, rho=(0.85, 1.15), vel=(-0.3, 0.3), p=(0.85, 1.15),
                 gamma=GAMMA):
    """Independent uniform primitive values at every point, converted to
    conserved form; returns an array of shape (4,) + shape. The default
    ranges keep states extrapolated to element faces (up to P=4) physical,
    rho > 0 and p > 0."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(rho[0], rho[1], size=shape)
    u = rng.uniform(vel[0], vel[1], size=shape)
    v = rng.uniform(vel[0], vel[1], size=shape)
    pp = rng.uniform(p[0], p[1], size=shape)
    return conserved_from_primitive(r, u, v, pp, gamma)


def gaussian_perturbation(shape, sigma, seed):
    """i.i.d. N(0, sigma^2) samples, C order, from numpy's default generator."""
    return sigma * np.random.default_rng(seed).standard_normal(shape)


def random_directions(shape, seeds):
    """One standard-normal direction per seed (finite-difference checks)."""
    return [np.random.default_rng(s).standard_normal(shape) for s in seeds]

"""Checks of the one-dimensional radial reference (tests/radial_ref.py) that
stands in for the paper's digitised reference profile of the radially
expanding shock tube: its slab-geometry mode against the exact solution of
the plane Riemann problem, a state at rest staying at rest (the pressure
source balances the face-area change), discrete conservation of mass and
energy in cylindrical geometry, and self-convergence."""

import numpy as np
import pytest

from tests import radial_ref as rr

G = 1.4


def exact_riemann(xi, left, right, g=G):
    """Exact solution (rho, u, p) of the plane Riemann problem at similarity
    coordinates xi = (x - x0)/t: the star pressure is the root of
    f_L(p) + f_R(p) + u_R - u_L, each f the shock (Rankine-Hugoniot) or
    rarefaction (isentropic) velocity change across its wave; the pattern
    is then sampled wave by wave."""
    rl, ul, pl = left
    rr_, ur, pr = right
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr_)

    def f(p, rk, pk, ck):
        if p > pk:
            A, B = 2.0 / ((g + 1) * rk), (g - 1) / (g + 1) * pk
            return (p - pk) * np.sqrt(A / (p + B))
        return 2 * ck / (g - 1) * ((p / pk) ** ((g - 1) / (2 * g)) - 1.0)

    lo, hi = 1e-12, 10.0 * max(pl, pr)
    for _ in range(200):           # bisection: f is monotone in p
        mid = 0.5 * (lo + hi)
        if f(mid, rl, pl, cl) + f(mid, rr_, pr, cr) + ur - ul > 0:
            hi = mid
        else:
            lo = mid
    ps = 0.5 * (lo + hi)
    us = 0.5 * (ul + ur) + 0.5 * (f(ps, rr_, pr, cr) - f(ps, rl, pl, cl))
    out = np.empty((3, len(xi)))
    for n, s in enumerate(xi):
        if s <= us:   # left of the contact
            if ps > pl:
                rs = rl * (ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1)
                S = ul - cl * np.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                out[:, n] = (rl, ul, pl) if s < S else (rs, us, ps)
            else:
                rs = rl * (ps / pl) ** (1 / g)
                cs = cl * (ps / pl) ** ((g - 1) / (2 * g))
                if s < ul - cl:
                    out[:, n] = (rl, ul, pl)
                elif s > us - cs:
                    out[:, n] = (rs, us, ps)
                else:
                    c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    u = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    rho = rl * (c / cl) ** (2 / (g - 1))
                    out[:, n] = (rho, u, pl * (c / cl) ** (2 * g / (g - 1)))
        else:         # right of the contact
            if ps > pr:
                rs = rr_ * (ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1)
                S = ur + cr * np.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                out[:, n] = (rr_, ur, pr) if s > S else (rs, us, ps)
            else:
                rs = rr_ * (ps / pr) ** (1 / g)
                cs = cr * (ps / pr) ** ((g - 1) / (2 * g))
                if s > ur + cr:
                    out[:, n] = (rr_, ur, pr)
                elif s < us + cs:
                    out[:, n] = (rs, us, ps)
                else:
                    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    u = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    rho = rr_ * (c / cr) ** (2 / (g - 1))
                    out[:, n] = (rho, u, pr * (c / cr) ** (2 * g / (g - 1)))
    return out


def test_exact_riemann_solver_invariants():
    """Rankine-Hugoniot across the computed shock, and the star states'
    pressure and velocity continuity."""
    left, right = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    xi = np.linspace(-2, 2, 4001)
    sol = exact_riemann(xi, left, right)
    rho, u, p = sol
    # the shock is the largest jump on the right; mass flux continuity there
    k = np.argmax(np.abs(np.diff(rho)) * (xi[:-1] > 1.0))
    S = 0.5 * (xi[k] + xi[k + 1])
    r1, u1, r2, u2 = rho[k], u[k], rho[k + 1], u[k + 1]
    assert abs(r1 * (u1 - S) - r2 * (u2 - S)) < 2e-3
    # p and u continuous across the contact
    mid = (xi > 0.3) & (xi < 1.5)
    assert np.ptp(p[mid]) < 1e-12 and np.ptp(u[mid]) < 1e-12


def test_slab_mode_matches_exact_riemann_solution():
    t = 0.15
    rc, rho, u, p = rr.solve(t, n=2000, R=1.2, planar=True)
    ex = exact_riemann((rc - 0.4) / t, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))
    dr = rc[1] - rc[0]
    for k, v in enumerate((rho, u, p)):
        l1 = np.sum(np.abs(v - ex[k])) * dr
        assert l1 < 2.5e-3, (k, l1)


def test_rest_state_is_steady():
    rc, rho, u, p = rr.solve(0.1, n=200, inside=(1.0, 1.0), outside=(1.0, 1.0))
    assert np.max(np.abs(u)) < 1e-13
    assert np.max(np.abs(p - 1.0)) < 1e-13 and np.max(np.abs(rho - 1.0)) < 1e-13


def test_cylindrical_mass_and_energy_conserved():
    """The walls carry no mass or energy flux and the waves stay inside R,
    so sum r_i dr rho_i and sum r_i dr E_i are constant to rounding."""
    n, R = 800, 1.2
    rc0, rho0, u0, p0 = rr.solve(0.0, n=n, R=R)
    rc, rho, u, p = rr.solve(0.25, n=n, R=R)
    dr = R / n
    E0 = p0 / (G - 1) + 0.5 * rho0 * u0 ** 2
    E = p / (G - 1) + 0.5 * rho * u ** 2
    assert abs(np.sum(rc * rho) - np.sum(rc0 * rho0)) * dr < 1e-13
    assert abs(np.sum(rc * E) - np.sum(rc0 * E0)) * dr < 1e-13


def test_self_convergence():
    sols = [rr.solve(0.25, n=n) for n in (500, 1000, 2000)]
    d = []
    for (rc_a, rho_a, _, _), (rc_b, rho_b, _, _) in zip(sols[:-1], sols[1:]):
        d.append(np.mean(np.abs(rr.density_at(rc_b, rc_a, rho_a) - rho_b)) * 1.2)
    assert d[1] < 0.7 * d[0], d


def test_stored_profile_is_the_reference():
    """tests/golden/radial_profile_t025.txt (read by the benchmark) holds
    this reference at t = 0.25, as make_radial_profile.py writes it."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "radial_profile_t025.txt")
    r, rho = np.loadtxt(path, unpack=True)
    rc, rho_ref = rr.solve(0.25, n=4000)[:2]
    assert np.allclose(r, rc, atol=1e-6)
    assert np.allclose(rho, rho_ref, rtol=1e-9, atol=1e-12)

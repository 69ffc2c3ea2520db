"""The oracle on the paper's discontinuous problem (radially expanding shock
tube, Section 4; CFL from Table 4), at 50x50 elements: the density stays
within the physical range of the problem, the solution keeps the diagonal
symmetry of its data, and its distance from the one-dimensional radial
reference (tests/radial_ref.py) is that of a shock-capturing solution on this
mesh, falling as the mesh is refined from 25x25."""

import numpy as np
import pytest

import inputs
from oracle import cpr, limiter
from tests import radial_ref as rr


def run(scheme, P, n, cfl, t_end=0.25):
    g = cpr.Grid(P=P, nx=n, ny=n, x0=-1.0, x1=1.0, y0=-1.0, y1=1.0, bc="transmissive",
                 scheme=scheme)
    x, y = g.coords()

    def lim(z):
        return limiter.limit(z, g, M=10.0)

    q = lim(inputs.radial_shock_tube(x, y))
    t = 0.0
    while t < t_end:
        dt = min(cpr.cfl_dt(q, g, cfl), t_end - t)
        q = cpr.rk3_step(q, dt, g, limit=lim)
        t += dt
    return g, x, y, q


@pytest.fixture(scope="module")
def ref():
    rc, rho, _, _ = rr.solve(0.25, n=2000)
    return rc, rho


@pytest.mark.parametrize("scheme,P,cfl", [("gl_lp", 1, 0.2), ("gl_lp", 2, 0.1),
                                          ("gll_chain", 1, 0.2)])
def test_radial_shock_tube_oracle(ref, scheme, P, cfl):
    rc, rho_ref = ref
    l1s = []
    for n in (25, 50):
        g, x, y, q = run(scheme, P, n, cfl)
        l1, l1c = rr.metrics(q[0], x, y, g.quad_weights(), g.tables().w, rc, rho_ref)
        l1s.append(l1)
        assert 0.09 < q[0].min() and q[0].max() < 1.05
        qt = q[[0, 2, 1, 3]].transpose(0, 2, 1, 4, 3)
        assert np.max(np.abs(qt - q)) < 1e-11
    print(scheme, P, l1s)
    assert l1s[1] < 0.8 * l1s[0]
    assert l1s[1] < 1.5e-2

"""The oracle against the errors the paper prints for its smooth problem
(Section 4, "Smooth Problem"; Tables 2 and 3, CFL from Table 1): the
Gauss-Lobatto chain-rule scheme reproduces the CPR column, the
Gauss-Legendre scheme the DG column and the Gauss-Lobatto scheme with the
flux derivative the NDG column. Each run takes CFL-limited steps,
dt = CFL h / max(|V| + c) from the current state, with the last step cut to
end at t = 1, then the area-normalised quadrature L2 norm of the density
error (the meshes up to 40x40 here; the HIP path runs all of them)."""

import pytest

import inputs
from oracle import cpr
from tests.golden_data import PAPER_COLUMN, PAPER_L2_RTOL, paper_vortex_l2


def paper_vortex():
    return inputs.Vortex(eps=5.0, lo=-5.0, hi=5.0, u_inf=1.0, v_inf=0.0, center=(0.0, 0.0))


def run_to_one(grid, cfl):
    V = paper_vortex()
    x, y = grid.coords()
    q = V.conserved(x, y)
    t = 0.0
    while t < 1.0:
        dt = min(cpr.cfl_dt(q, grid, cfl), 1.0 - t)
        q = cpr.rk3_step(q, dt, grid)
        t += dt
    return cpr.l2_error(q[0], V.conserved(x, y, 1.0)[0], grid)


ROWS = [r for r in paper_vortex_l2() if r[1] <= 40]


@pytest.mark.parametrize("row", ROWS, ids=lambda r: f"P{r[0]}-{r[1]}")
@pytest.mark.parametrize("scheme", cpr.SCHEMES)
def test_oracle_reproduces_paper_errors(scheme, row):
    P, n, cfl = row[:3]
    g = cpr.Grid(P=P, nx=n, ny=n, x0=-5.0, x1=5.0, y0=-5.0, y1=5.0, scheme=scheme)
    want = row[PAPER_COLUMN[scheme]]
    got = run_to_one(g, cfl)
    assert abs(got - want) <= PAPER_L2_RTOL * want, (got, want)

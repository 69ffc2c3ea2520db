"""Writes tests/golden/radial_tube_200.txt: the oracle's solution of the
paper's discontinuous problem (radially expanding shock tube, Section 4;
each scheme at the CFL Table 4 gives the method it reproduces,
inputs.RADIAL_TUBE_CFL) on the paper's 200x200 mesh, for both schemes,
summarised by figures the GPU run is compared with: steps,
the domain L1 distance of the density from the one-dimensional radial
reference (tests/radial_ref.py, 4000 cells), the same along the row of
points nearest the centre line y = 0, the change of the four totals, and the
density range. Calls only oracle/, inputs/ and tests/radial_ref.py.

    python tests/golden/make_radial_tube.py [--jobs 4]
"""

import argparse
import os
import sys
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

N = 200
SCHEMES = [("gl_lp", 1), ("gl_lp", 2), ("gll_chain", 1), ("gll_chain", 2)]
T_END = 0.25
M = 10.0


def run(case):
    import numpy as np
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(limits=1)
    except Exception:
        pass
    import inputs
    from oracle import cpr, limiter
    from tests import radial_ref
    scheme, P = case
    cfl = inputs.RADIAL_TUBE_CFL[(scheme, P, N)]
    g = cpr.Grid(P=P, nx=N, ny=N, x0=-1.0, x1=1.0, y0=-1.0, y1=1.0, bc="transmissive",
                 scheme=scheme)
    x, y = g.coords()
    q = inputs.radial_shock_tube(x, y)

    def lim(z):
        return limiter.limit(z, g, M=M)

    q = lim(q)
    I0 = cpr.integrals(q, g)
    t, k = 0.0, 0
    while t < T_END:
        dt = min(cpr.cfl_dt(q, g, cfl), T_END - t)
        q = cpr.rk3_step(q, dt, g, limit=lim)
        t += dt
        k += 1
    rc, rho_ref, _, _ = radial_ref.solve(T_END, n=4000)
    W = g.quad_weights()
    l1, l1c = radial_ref.metrics(q[0], x, y, W, g.tables().w, rc, rho_ref)
    dI = cpr.integrals(q, g) - I0
    return (scheme, P, N, cfl, k, l1, l1c, dI, float(q[0].min()), float(q[0].max()))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    a = ap.parse_args()
    with ProcessPoolExecutor(a.jobs) as ex:
        rows = list(ex.map(run, SCHEMES))
    out = os.path.join(HERE, "radial_tube_200.txt")
    with open(out, "w") as f:
        f.write("# The oracle on the paper's radially expanding shock tube (Section 4; each\n"
                "# scheme at Table 4's CFL for the method it reproduces: gl_lp DG, gll_chain\n"
                "# CPR), 200x200 elements on [-1,1]^2, transmissive, TVB limiter M=10 after\n"
                "# every stage, t = 0.25. Written by tests/golden/make_radial_tube.py.\n"
                "# Columns: scheme P n cfl steps L1_domain L1_centre_row dI_rho dI_mx dI_my\n"
                "# dI_E rho_min rho_max (L1 against the 1D radial reference, 4000 cells).\n")
        for r in rows:
            scheme, P, n, cfl, k, l1, l1c, dI, lo, hi = r
            f.write(f"{scheme} {P} {n} {cfl} {k} {l1:.10e} {l1c:.10e} "
                    + " ".join(f"{v:.6e}" for v in dI) + f" {lo:.10e} {hi:.10e}\n")
    print(open(out).read())


if __name__ == "__main__":
    main()

"""Loaders for the fixtures under tests/golden/ (values printed in the
paper, each file citing where)."""

import os

_DIR = os.path.join(os.path.dirname(__file__), "golden")


def paper_vortex_l2():
    """Rows (P, n, cfl, cpr_err, dg_err, ndg_err) of the smooth-problem error
    tables (Tables 2 and 3, CFL from Table 1)."""
    rows = []
    with open(os.path.join(_DIR, "paper_vortex_l2.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            P, n, cfl, a, b, c = line.split()
            rows.append((int(P), int(n), float(cfl), float(a), float(b), float(c)))
    return rows


# the column of each scheme in those rows
PAPER_COLUMN = {"gll_chain": 3, "gl_lp": 4, "gll_lp": 5}


# Relative tolerance against a printed error: the tables give three
# significant digits (up to 0.25% of rounding at the mantissas printed) and
# leave the time-step sequence to the reader; errors reproduce to within 1%.
PAPER_L2_RTOL = 0.01


def radial_tube_200():
    """{(scheme, P): dict} from radial_tube_200.txt (the oracle's figures on
    the paper's radially expanding shock tube at 200x200, written by
    make_radial_tube.py)."""
    out = {}
    with open(os.path.join(_DIR, "radial_tube_200.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            v = line.split()
            out[(v[0], int(v[1]))] = {
                "n": int(v[2]), "cfl": float(v[3]), "steps": int(v[4]), "l1": float(v[5]),
                "l1_row": float(v[6]), "dI": [float(a) for a in v[7:11]],
                "rho_min": float(v[11]), "rho_max": float(v[12])}
    return out

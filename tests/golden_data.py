"""Loaders for the fixtures under tests/golden/ (values printed in the
paper, each file citing where)."""

import os

_DIR = os.path.join(os.path.dirname(__file__), "golden")


def paper_vortex_l2():
    """Rows (P, n, cfl, cpr_err, dg_err) of the smooth-problem error tables
    (Tables 2 and 3, CFL from Table 1)."""
    rows = []
    with open(os.path.join(_DIR, "paper_vortex_l2.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            P, n, cfl, a, b = line.split()
            rows.append((int(P), int(n), float(cfl), float(a), float(b)))
    return rows


# Relative tolerance against a printed error: the tables give three
# significant digits (up to 0.25% of rounding at the mantissas printed) and
# leave the time-step sequence to the reader; errors reproduce to within 1%.
PAPER_L2_RTOL = 0.01

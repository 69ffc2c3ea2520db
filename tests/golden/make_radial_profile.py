"""Writes tests/golden/radial_profile_t025.txt: the one-dimensional radial
reference density of the paper's radially expanding shock tube (Section 4)
at t = 0.25 (tests/radial_ref.py: 4000 finite-volume cells on [0, 1.2]),
as (r, rho) pairs, so that the benchmark can measure the distance of its
2D solutions from it without running test code.

    python tests/golden/make_radial_profile.py
"""

import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)


def main():
    import numpy as np
    from tests import radial_ref
    rc, rho = radial_ref.solve(0.25, n=4000)[:2]
    out = os.path.join(HERE, "radial_profile_t025.txt")
    with open(out, "w") as f:
        f.write("# radial reference of the radially expanding shock tube (paper Section 4) at\n"
                "# t = 0.25: cell centre r and density, 4000 cells on [0, 1.2]\n"
                "# written by tests/golden/make_radial_profile.py (tests/radial_ref.py)\n")
        for r, d in zip(rc, rho):
            f.write(f"{r:.6f} {d:.10e}\n")
    print(out, len(rc))


if __name__ == "__main__":
    main()

"""Host logic of the paper's maximum-CFL convention (Section 4): the halving
test and the downward scan, on error functions with known answers."""

import math

from paper_1709_01619_amd import cfl_search


def test_halving_test():
    err = lambda c: 1.0 + 0.01 * c * c
    ok, e, eh = cfl_search.admissible(err, 0.3)
    assert ok and abs(e - 1.0009) < 1e-15 and abs(eh - 1.000225) < 1e-15
    # |e(c) - e(c/2)| / e(c/2) = 0.0075 c^2 / (1 + 0.0025 c^2) >= 1e-3 from c = 0.366
    assert not cfl_search.admissible(err, 0.37)[0]
    assert not cfl_search.admissible(lambda c: math.inf, 0.1)[0]


def test_scan_stops_at_largest_admissible():
    # unstable above 0.3, accurate enough below 0.366: the answer is 0.30
    err = lambda c: math.inf if c > 0.3 + 1e-12 else 1.0 + 0.01 * c * c
    c, rec = cfl_search.max_cfl(err, 0.40)
    assert c == 0.3
    assert [r[0] for r in rec] == [0.4, 0.39, 0.38, 0.37, 0.36, 0.35, 0.34, 0.33, 0.32, 0.31, 0.3]
    assert all(not r[1] for r in rec[:-1]) and rec[-1][1]
    # accuracy-limited: stable everywhere, the halving test decides
    c, _ = cfl_search.max_cfl(lambda c: 1.0 + 0.01 * c * c, 0.5)
    assert c == 0.36
    # nothing admissible
    assert cfl_search.max_cfl(lambda c: math.inf, 0.05)[0] is None

"""The paper's maximum-CFL search (Section 4) on the GPU, for its smooth
problem on 20x20 elements: the CFL found passes the halving test, every
larger CFL tried fails it, and it lies at or above Table 1's value for the
paper's CPR (0.24 at P1, 0.14 at P2 on 20x20): with the time step of this
build, dt = CFL h / max(|V| + c), the 0.1 % test holds at every CFL the
scheme is stable at, so the search ends at the stability limit."""

import pytest

from paper_1709_01619_amd import cfl_search
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("P,table1", [(1, 0.24), (2, 0.14)])
def test_max_cfl_paper_cpr(P, table1):
    say("max cfl", P)
    err = lambda c: cfl_search.vortex_error(P, 20, "gll_chain", c)
    c, rec = cfl_search.max_cfl(err, 0.40 if P == 1 else 0.25)
    print(P, c, [(r[0], r[1]) for r in rec])
    assert c is not None and c >= table1
    assert rec[-1][1] and all(not r[1] for r in rec[:-1])

"""Pins for the oracle's TVB characteristic limiter: minmod algebra, mean
preservation, idempotence, no-op limits (M -> infinity, linear data in the
interior), detection at a jump, one-dimensional data and the diagonal
symmetry of the four-quadrant Riemann problem."""

import numpy as np
import pytest

import inputs
from oracle import cpr, limiter


def test_minmod_values():
    a = np.array([1.0, -2.0, 3.0, 0.0, 2.0])
    b = np.array([2.0, -1.0, -1.0, 1.0, 0.5])
    c = np.array([0.5, -3.0, 2.0, 1.0, 4.0])
    np.testing.assert_array_equal(limiter.minmod(a, b, c), [0.5, -1.0, 0.0, 0.0, 0.5])
    np.testing.assert_array_equal(limiter.tvb_minmod(a, b, c, 1.5), [1.0, -1.0, 0.0, 0.0, 0.5])


def _riemann_grid(n, P=2):
    return cpr.Grid(P=P, nx=n, ny=n, x0=0.0, x1=1.0, y0=0.0, y1=1.0, bc="transmissive")


def _smoothed_riemann(g):
    """Quadrant data blurred with tanh fronts so several elements are
    partially limited, evaluated at the oracle's own points."""
    x, y = g.coords()
    sx = 0.5 * (1 + np.tanh((x - 0.5) / 0.03))
    sy = 0.5 * (1 + np.tanh((y - 0.5) / 0.03))
    S = inputs.RIEMANN_QUADRANTS
    prim = [(S["NE"][k] * sx * sy + S["NW"][k] * (1 - sx) * sy + S["SW"][k] * (1 - sx) * (1 - sy)
             + S["SE"][k] * sx * (1 - sy)) for k in range(4)]
    return inputs.conserved_from_primitive(*prim)


@pytest.mark.parametrize("P", [1, 2, 3])
def test_mean_preserved_and_idempotent(P):
    g = _riemann_grid(12, P)
    q = _smoothed_riemann(g)
    ql, flags = limiter.limit(q, g, M=10.0, return_flags=True)
    assert flags.any() and not flags.all()
    np.testing.assert_allclose(cpr.element_means(ql, g), cpr.element_means(q, g), atol=1e-14)
    # untouched elements are bitwise unchanged
    np.testing.assert_array_equal(ql[:, ~flags], q[:, ~flags])
    # limited elements are linear: second differences along i vanish for P >= 2
    if P >= 2:
        d2 = ql[..., 2:] - 2 * ql[..., 1:-1] + ql[..., :-2]
        T = g.tables()
        h = np.diff(T.xi)
        # nodes are not equispaced: check linearity through divided differences
        s1 = (ql[..., 1:] - ql[..., :-1]) / h
        assert np.max(np.abs(np.diff(s1, axis=-1)[:, flags])) < 1e-12
        del d2
    ql2, flags2 = limiter.limit(ql, g, M=10.0, return_flags=True)
    assert not flags2.any()
    np.testing.assert_array_equal(ql2, ql)


def test_large_m_is_noop():
    g = _riemann_grid(10)
    q = _smoothed_riemann(g)
    ql, flags = limiter.limit(q, g, M=1e30, return_flags=True)
    assert not flags.any()
    np.testing.assert_array_equal(ql, q)


def test_linear_data_untouched_in_interior():
    """Globally linear conserved data: the face deviations are exactly half
    the neighbour differences, so the TVB minmod returns them and interior
    elements pass. M = 1 keeps the TVB bound M h^2 below the deviations of
    the non-constant components (so the minmod branch is exercised) but far
    above roundoff in the components whose slope is zero."""
    g = _riemann_grid(8)
    x, y = g.coords()
    q = np.stack([1.0 + 0.3 * x + 0.2 * y, 0.1 * (1.0 + 0.3 * x + 0.2 * y),
                  -0.2 + 0.1 * x, 2.5 + 0.2 * x - 0.3 * y])
    ql, flags = limiter.limit(q, g, M=1.0, return_flags=True)
    assert not flags[1:-1, 1:-1].any()
    np.testing.assert_array_equal(ql[:, 1:-1, 1:-1], q[:, 1:-1, 1:-1])
    # a pure minmod (M = 0) would flag on roundoff-level zero slopes
    _, flags0 = limiter.limit(q, g, M=0.0, return_flags=True)
    assert flags0[1:-1, 1:-1].any()


def test_jump_is_detected():
    g = _riemann_grid(16)
    x, y = g.coords()
    q = inputs.riemann_quadrants(x, y)
    # shift the split off the element faces so the jump sits inside elements
    q = inputs.riemann_quadrants(x, y, split=(0.53, 0.53))
    ql, flags = limiter.limit(q, g, M=10.0, return_flags=True)
    cols = np.where(flags.any(axis=0))[0]
    assert 8 in cols
    # far-field elements inside a quadrant (constant data) are not flagged
    assert not flags[2, 2] and not flags[13, 13]


def test_y_independent_data_keeps_zero_y_slope():
    g = cpr.Grid(P=2, nx=12, ny=4, x0=0.0, x1=1.0, y0=0.0, y1=1.0, bc="periodic")
    x, y = g.coords()
    rho = 1.0 + 0.5 * (x > 0.52) + 0.1 * np.sin(2 * np.pi * x)
    q = inputs.conserved_from_primitive(rho, 0.2 + 0 * x, 0 * x, 1.0 + 0 * x)
    ql, flags = limiter.limit(q, g, M=10.0, return_flags=True)
    assert flags.any()
    np.testing.assert_allclose(ql, np.broadcast_to(ql[:, :1, :, :1, :], ql.shape), atol=1e-14)


def test_riemann_diagonal_symmetry_one_limited_step():
    g = _riemann_grid(16)
    x, y = g.coords()
    q = inputs.riemann_quadrants(x, y)
    lim = lambda s: limiter.limit(s, g, M=10.0)
    q = lim(q)
    dt = cpr.cfl_dt(q, g, 0.1)
    q1 = cpr.rk3_step(q, dt, g, limit=lim)
    qt = q1[[0, 2, 1, 3]].transpose(0, 2, 1, 4, 3)
    np.testing.assert_allclose(qt, q1, atol=1e-12)

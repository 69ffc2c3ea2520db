"""TVB minmod slope limiter on characteristic variables (oracle).

Section 2.6 of the paper marks troubled elements with a minmod test built
from element averages and replaces the solution there by a second-order
reconstruction q = qbar + (x - x0) minmod(forward, backward neighbour
slopes) (eq. limu); its GPU version (Algorithms 9-11) first forms element
averages, then tests edge values, then limits marked elements. This oracle
keeps that Average -> Detect -> Limit structure in the total-variation-
bounded (TVB) characteristic form of Cockburn and Shu, which the paper cites
for this limiter:

1. qbar: element means by the tensor Gauss-Legendre rule.
2. Face means of the extrapolated state on each face, e.g.
   q_E = 1/2 sum_j w_j q_E,j.
3. Deviations u+ = q_E - qbar, u- = qbar - q_W; neighbour differences
   D+ = qbar(I+1) - qbar, D- = qbar - qbar(I-1). A missing neighbour
   (transmissive boundary) has the element's own mean.
4. Characteristic variables with the left eigenvectors L_d(qbar) of the
   flux Jacobian in direction d.
5. TVB minmod m(a, b, c) = a if |a| <= M h_d^2, else minmod(a, b, c).
6. Troubled: m(.) != a for any component, either deviation, either
   direction.
7. Troubled elements become q = qbar + (x - x_I) s_x + (y - y_J) s_y with
   s_d = R_d minmod(L_d (q_E - q_W)/h_d, L_d D+/h_d, L_d D-/h_d).
"""

from __future__ import annotations

import numpy as np

from . import euler
from .cpr import PERIODIC, Grid, element_means


def minmod(a, b, c):
    """sign(a) min(|a|,|b|,|c|) if a, b, c share a sign, else 0."""
    s = np.sign(a)
    same = (np.sign(b) == s) & (np.sign(c) == s)
    m = np.minimum(np.minimum(np.abs(a), np.abs(b)), np.abs(c))
    return np.where(same, s * m, 0.0)


def tvb_minmod(a, b, c, bound):
    return np.where(np.abs(a) <= bound, a, minmod(a, b, c))


def face_means(q, grid: Grid):
    """(qW, qE, qS, qN): face averages of the extrapolated state, each of
    shape (4, ny, nx)."""
    T = grid.tables()
    w = T.w
    qW = 0.5 * np.einsum("kJIji,i,j->kJI", q, T.em, w)
    qE = 0.5 * np.einsum("kJIji,i,j->kJI", q, T.ep, w)
    qS = 0.5 * np.einsum("kJIji,j,i->kJI", q, T.em, w)
    qN = 0.5 * np.einsum("kJIji,j,i->kJI", q, T.ep, w)
    return qW, qE, qS, qN


def _neighbour_means(qbar, grid: Grid, axis):
    """(mean of the lower neighbour, mean of the upper neighbour) along
    element axis 0 (x: I) or 1 (y: J)."""
    ax = 2 if axis == 0 else 1
    if grid.bc == PERIODIC:
        lo = np.roll(qbar, 1, axis=ax)
        hi = np.roll(qbar, -1, axis=ax)
    else:
        lo = np.concatenate([np.take(qbar, [0], axis=ax),
                             np.take(qbar, np.arange(qbar.shape[ax] - 1), axis=ax)], axis=ax)
        hi = np.concatenate([np.take(qbar, np.arange(1, qbar.shape[ax]), axis=ax),
                             np.take(qbar, [qbar.shape[ax] - 1], axis=ax)], axis=ax)
    return lo, hi


def _char(L, v):
    return np.einsum("abJI,bJI->aJI", L, v)


def detect_and_slopes(q, grid: Grid, M=10.0):
    """Return (troubled[ny, nx] bool, qbar, s_x, s_y)."""
    qbar = element_means(q, grid)
    qW, qE, qS, qN = face_means(q, grid)
    troubled = np.zeros(qbar.shape[1:], dtype=bool)
    slopes = []
    for axis, (lo_face, hi_face, h) in enumerate(((qW, qE, grid.dx), (qS, qN, grid.dy))):
        nb_lo, nb_hi = _neighbour_means(qbar, grid, axis)
        R, L = euler.eigenvectors(qbar, grid.gamma, axis)
        up = _char(L, hi_face - qbar)
        um = _char(L, qbar - lo_face)
        dp = _char(L, nb_hi - qbar)
        dm = _char(L, qbar - nb_lo)
        bound = M * h * h
        bad = (tvb_minmod(up, dp, dm, bound) != up) | (tvb_minmod(um, dp, dm, bound) != um)
        troubled |= np.any(bad, axis=0)
        sc = minmod(_char(L, hi_face - lo_face) / h, dp / h, dm / h)
        slopes.append(np.einsum("abJI,bJI->aJI", R, sc))
    return troubled, qbar, slopes[0], slopes[1]


def limit(q, grid: Grid, M=10.0, return_flags=False):
    """Apply the limiter; elements that pass the test are returned unchanged."""
    troubled, qbar, sx, sy = detect_and_slopes(q, grid, M)
    T = grid.tables()
    xo = 0.5 * grid.dx * T.xi            # x - x_I at index i
    yo = 0.5 * grid.dy * T.xi            # y - y_J at index j
    lin = (qbar[..., None, None] + sx[..., None, None] * xo[None, None, None, None, :]
           + sy[..., None, None] * yo[None, None, None, :, None])
    out = np.where(troubled[None, :, :, None, None], lin, q)
    if return_flags:
        return out, troubled
    return out

"""The limiter's value pins catch the plausible mistakes in its slope
(Section 2.6, eq. limu, in its TVB characteristic form): each mistake is
planted in a copy of the oracle's detection-and-slope step, on the CPU, and at
least one value pin must then fail.

Mistakes: the first minmod argument (q_E - q_W)/h dropped, which is eq. limu's
two-argument form; that argument doubled (a half-width difference); the
characteristic matrices taken at the east face state instead of the element
mean."""

import numpy as np
import pytest

from oracle import euler, limiter
from oracle.limiter import _char, _neighbour_means, face_means, minmod, tvb_minmod
from oracle.cpr import element_means

from tests import test_oracle_limiter as pins


def _planted(kind):
    def detect_and_slopes(q, grid, M=10.0):
        qbar = element_means(q, grid)
        qW, qE, qS, qN = face_means(q, grid)
        troubled = np.zeros(qbar.shape[1:], dtype=bool)
        slopes = []
        for axis, (lo, hi, h) in enumerate(((qW, qE, grid.dx), (qS, qN, grid.dy))):
            nb_lo, nb_hi = _neighbour_means(qbar, grid, axis)
            R, L = euler.eigenvectors(hi if kind == "L_at_face" else qbar, grid.gamma, axis)
            up, um = _char(L, hi - qbar), _char(L, qbar - lo)
            dp, dm = _char(L, nb_hi - qbar), _char(L, qbar - nb_lo)
            bound = M * h * h
            bad = (tvb_minmod(up, dp, dm, bound) != up) | (tvb_minmod(um, dp, dm, bound) != um)
            troubled |= np.any(bad, axis=0)
            a = _char(L, hi - lo) / h
            if kind == "first_dropped":
                a = dp / h
            elif kind == "first_doubled":
                a = 2.0 * a
            slopes.append(np.einsum("abJI,bJI->aJI", R, minmod(a, dp / h, dm / h)))
        return troubled, qbar, slopes[0], slopes[1]
    return detect_and_slopes


PINS = (pins.test_limited_slope_values_contact, pins.test_limited_slope_values_acoustic)


def _failures():
    n = 0
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            n += 1
    return n


def test_unplanted_copy_passes(monkeypatch):
    monkeypatch.setattr(limiter, "detect_and_slopes", _planted("none"))
    assert _failures() == 0


@pytest.mark.parametrize("kind", ["first_dropped", "first_doubled", "L_at_face"])
def test_planted_mistake_fails_a_pin(monkeypatch, kind):
    monkeypatch.setattr(limiter, "detect_and_slopes", _planted(kind))
    assert _failures() >= 1

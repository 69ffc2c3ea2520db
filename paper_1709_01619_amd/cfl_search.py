"""The paper's maximum-CFL convention (Section 4): run a case to its end
time, record the error, run it again at half the CFL; if the two errors
differ by less than 0.1 %, the CFL is admissible. The maximum CFL is the
largest admissible value on a grid of CFL numbers (the paper's Table 1 and
Table 4 give two decimals). A run that breaks down (non-physical state, or
a non-finite error) is not admissible.

`max_cfl` is the search on any error function; `vortex_error` is the
paper's smooth problem on the GPU through the library's device-dt stepping.
"""

from __future__ import annotations

import math


def admissible(err, cfl, tol=1e-3):
    """(ok, e, e_half) for one CFL under the halving test."""
    e = err(cfl)
    if not math.isfinite(e):
        return False, e, float("nan")
    eh = err(0.5 * cfl)
    if not math.isfinite(eh) or eh <= 0.0:
        return False, e, eh
    return abs(e - eh) < tol * eh, e, eh


def max_cfl(err, cfl_start, step=0.01, cfl_min=0.01, tol=1e-3):
    """Largest CFL on the grid cfl_start, cfl_start - step, ... (down to
    cfl_min) that passes the halving test, scanning downwards; returns
    (cfl or None, record) with record the list of (cfl, ok, e, e_half)
    tried."""
    rec = []
    n = int(round((cfl_start - cfl_min) / step))
    for k in range(n + 1):
        c = round(cfl_start - k * step, 10)
        ok, e, eh = admissible(err, c, tol)
        rec.append((c, ok, e, eh))
        if ok:
            return c, rec
    return None, rec


def vortex_error(P, n, scheme, cfl, t_end=1.0, device="cuda"):
    """L2 density error at t_end of the paper's smooth problem (vortex of
    strength 5, mean flow (1,1,0,1), periodic [-5,5]^2) on n x n elements,
    stepped on the GPU with dt = cfl h / max(|V| + c) from the current
    state; inf if the run meets a non-physical state."""
    import torch

    import inputs
    from . import _lib
    from .solver import Solver

    s = Solver(P, n, n, -5.0, 5.0, -5.0, 5.0, cfl=cfl, t_end=t_end, scheme=scheme,
               device=device)
    V = inputs.Vortex(eps=5.0, lo=-5.0, hi=5.0, u_inf=1.0, v_inf=0.0, center=(0.0, 0.0))
    x, y = s.coords()
    xn, yn = x.cpu().numpy(), y.cpu().numpy()
    q = torch.from_numpy(V.conserved(xn, yn)).to(s.device)
    ex = torch.from_numpy(V.conserved(xn, yn, t_end)).to(s.device)
    lam = s.max_wavespeed(q)
    s.set_time(0.0)
    try:
        t = 0.0
        # chunks of steps; calls after t_end change nothing, and a breakdown
        # is reported by the synchronising get_time
        chunk = max(1, int(0.25 * t_end / (cfl * s.dx / lam)))
        while t < t_end * (1 - 1e-14):
            for _ in range(chunk):
                s.step(q, 0.0)
            t, _ = s.get_time()
            if not math.isfinite(t):
                return math.inf
        e = s.l2_diff(q, ex, 0)
    except _lib.CprError as exc:
        if exc.status == _lib.CPR_ENONPHYSICAL:
            return math.inf
        raise
    finally:
        s.close()
    return e if math.isfinite(e) else math.inf

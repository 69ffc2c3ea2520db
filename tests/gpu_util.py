"""Helpers shared by the GPU parity tests (test infrastructure)."""

import sys

import numpy as np


def torch():
    import torch as t
    return t


def dev(a):
    t = torch()
    return t.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def say(*args):
    """Name the case on stdout before its GPU work starts."""
    print("[gpu-case]", *args, flush=True)
    sys.stdout.flush()


def make_solver(grid, precision="fp64", limiter=False, tvb_m=10.0, cfl=0.0, t_end=0.0):
    from paper_1709_01619_amd import Solver
    return Solver(grid.P, grid.nx, grid.ny, grid.x0, grid.x1, grid.y0, grid.y1, bc=grid.bc,
                  precision=precision, gamma=grid.gamma, limiter=limiter, tvb_m=tvb_m, cfl=cfl,
                  t_end=t_end, scheme=grid.scheme)


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b)))))

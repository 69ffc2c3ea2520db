"""PyTorch-facing wrapper of the CPR library.

torch supplies device memory and the stream; every computation runs in the
HIP kernels of libcpr.so, reached through the C ABI (include/cpr.h). There is
no fallback: constructing a Solver without the built library or without a
GPU raises.
"""

from __future__ import annotations

import ctypes
import weakref
from ctypes import byref, c_double, c_int32, c_int64, c_void_p

import numpy as np

from . import _lib

BC = {"periodic": _lib.CPR_BC_PERIODIC, "transmissive": _lib.CPR_BC_TRANSMISSIVE}
PRECISION = {"fp64": _lib.CPR_FP64, "fp32_bulk": _lib.CPR_FP32_BULK}
SCHEME = {"gl_lp": _lib.CPR_SCHEME_GL_LP, "gll_chain": _lib.CPR_SCHEME_GLL_CHAIN,
          "gll_lp": _lib.CPR_SCHEME_GLL_LP}


def _torch():
    import torch
    return torch


class StepGraph:
    """A run of SSP-RK3 steps recorded into a HIP graph (Solver.capture_steps).
    The recorded kernels read and write the state q and the solver's scratch
    through raw device pointers, so the StepGraph holds references to both:
    neither can be freed while it exists."""

    def __init__(self, graph, solver, q):
        self.graph = graph
        self.solver = solver
        self.q = q

    def replay(self):
        """Advance q by the recorded steps (one graph launch)."""
        if not self.solver._ctx.value:
            raise RuntimeError("the solver of this graph was closed")
        self.graph.replay()


class Solver:
    """One CPR discretisation (degree P, mesh, boundary, precision, limiter,
    scheme) bound to a GPU. States are float64 tensors of shape
    (4, ny, nx, P+1, P+1) on that GPU (see include/cpr.h for the layout).
    scheme: "gl_lp" (Gauss-Legendre points, derivative of the flux
    interpolant), "gll_chain" (the paper's CPR: Gauss-Lobatto points,
    chain-rule divergence) or "gll_lp" (the paper's NDG: Gauss-Lobatto
    points, derivative of the flux interpolant)."""

    def __init__(self, P, nx, ny, x0=0.0, x1=10.0, y0=0.0, y1=10.0, bc="periodic",
                 precision="fp64", gamma=1.4, limiter=False, tvb_m=10.0, cfl=0.0, t_end=0.0,
                 device="cuda", scheme="gl_lp"):
        torch = _torch()
        self.lib = _lib.load()
        self.device = torch.device(device)
        if self.device.type != "cuda" or not torch.cuda.is_available():
            raise RuntimeError("the CPR library needs a HIP (ROCm) GPU")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.P, self.nx, self.ny = int(P), int(nx), int(ny)
        self.x0, self.x1, self.y0, self.y1 = float(x0), float(x1), float(y0), float(y1)
        self.bc = bc
        self.precision = precision
        self.gamma = float(gamma)
        self.limiter = bool(limiter)
        if scheme not in SCHEME:
            raise ValueError(f"unknown scheme {scheme}")
        self.scheme = scheme
        cfg = _lib.make_config(self.P, self.nx, self.ny, self.x0, self.x1, self.y0, self.y1,
                               BC[bc], PRECISION[precision], self.gamma,
                               _lib.CPR_LIM_TVB_CHAR if limiter else _lib.CPR_LIM_NONE,
                               float(tvb_m), float(cfl), float(t_end), SCHEME[scheme])
        self._ctx = c_void_p()
        self._graphs = weakref.WeakSet()
        with torch.cuda.device(self.device):
            st = self.lib.cpr_init(byref(cfg), c_void_p(self._stream()), byref(self._ctx))
        _lib.check(st, None, "cpr_init")

    # ------------------------------------------------------------ plumbing --
    def _stream(self):
        torch = _torch()
        return torch.cuda.current_stream(self.device).cuda_stream

    def _enter(self):
        self.lib.cpr_set_stream(self._ctx, c_void_p(self._stream()))

    def close(self):
        """Release the context and its scratch. Raises while a StepGraph
        recorded from this solver is alive (its kernels use the scratch)."""
        if getattr(self, "_ctx", None) and self._ctx.value:
            if len(getattr(self, "_graphs", ())) > 0:
                raise RuntimeError("close(): graphs recorded from this solver are alive; "
                                   "delete them first")
            self.lib.cpr_destroy(self._ctx)
            self._ctx = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n1(self):
        return self.P + 1

    @property
    def shape(self):
        return (4, self.ny, self.nx, self.n1, self.n1)

    @property
    def n_unknowns(self):
        return 4 * self.ny * self.nx * self.n1 * self.n1

    @property
    def dx(self):
        return (self.x1 - self.x0) / self.nx

    @property
    def dy(self):
        return (self.y1 - self.y0) / self.ny

    def empty(self, dtype=None):
        torch = _torch()
        return torch.empty(self.shape, dtype=dtype or torch.float64, device=self.device)

    def _ptr(self, t, dtype=None, shape=None, name="tensor"):
        torch = _torch()
        dtype = dtype or torch.float64
        shape = shape or self.shape
        if t.device != self.device:
            raise ValueError(f"{name} must live on {self.device}")
        if t.dtype != dtype:
            raise ValueError(f"{name} must be {dtype}")
        if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous tensor of shape {shape}")
        return c_void_p(t.data_ptr())

    def _check(self, st, what):
        _lib.check(st, self._ctx, what)

    # ------------------------------------------------------------- entries --
    def residual(self, q, out=None):
        torch = _torch()
        rdt = torch.float32 if self.precision == "fp32_bulk" else torch.float64
        if out is None:
            out = self.empty(rdt)
        self._enter()
        self._check(self.lib.cpr_residual(self._ctx, self._ptr(q, name="q"),
                                          self._ptr(out, rdt, name="r")), "cpr_residual")
        return out

    def step(self, q, dt, limit=False):
        """One SSP-RK3 step in place; dt <= 0 uses the device CFL dt."""
        self._enter()
        self._check(self.lib.cpr_rk3_step(self._ctx, self._ptr(q, name="q"), float(dt),
                                          1 if limit else 0), "cpr_rk3_step")
        return q

    def capture_steps(self, q, dt, nsteps, limit=False):
        """Record nsteps SSP-RK3 steps of q (in place, as step()) into a HIP
        graph and return it as a StepGraph; each replay() then advances q by
        nsteps steps with one graph launch, which removes the per-kernel
        launch cost where the mesh is small. The step path only launches
        kernels (no allocation, copy, memset or synchronisation), so it
        records as it runs; a device dt (dt <= 0) reads the context's time as
        each replay reaches it. The recorded kernels hold raw pointers to q
        and to this solver's scratch, so the StepGraph keeps both alive, and
        close() refuses while a StepGraph of this solver exists."""
        torch = _torch()
        if nsteps < 1:
            raise ValueError("nsteps must be >= 1")
        g = torch.cuda.CUDAGraph()
        with torch.cuda.device(self.device):
            with torch.cuda.graph(g):
                for _ in range(nsteps):
                    self.step(q, dt, limit=limit)
        sg = StepGraph(g, self, q)
        self._graphs.add(sg)
        return sg

    def limit(self, q, flags=None, count=False):
        torch = _torch()
        self._enter()
        fp = c_void_p(0)
        if flags is not None:
            fp = self._ptr(flags, torch.int32, (self.ny, self.nx), "flags")
        n = c_int32(0)
        self._check(self.lib.cpr_limit(self._ctx, self._ptr(q, name="q"), fp,
                                       byref(n) if count else None), "cpr_limit")
        return int(n.value) if count else None

    def residual_vjp(self, q, v, out=None):
        out = self.empty() if out is None else out
        self._enter()
        self._check(self.lib.cpr_residual_vjp(self._ctx, self._ptr(q, name="q"),
                                              self._ptr(v, name="v"), self._ptr(out, name="out")),
                    "cpr_residual_vjp")
        return out

    def adjoint_step(self, q_n, dt, lam_np1, out=None):
        out = self.empty() if out is None else out
        self._enter()
        self._check(self.lib.cpr_adjoint_step(self._ctx, self._ptr(q_n, name="q_n"), float(dt),
                                              self._ptr(lam_np1, name="lam_np1"),
                                              self._ptr(out, name="lam_n")), "cpr_adjoint_step")
        return out

    def step_stages(self, q, dt, q1, q2, out=None):
        """One unlimited SSP-RK3 step from q that also writes its stage
        states into q1 and q2 (cpr_rk3_step_stages); q(n+1) goes to out, by
        default q itself (in place)."""
        out = q if out is None else out
        self._enter()
        self._check(self.lib.cpr_rk3_step_stages(self._ctx, self._ptr(q, name="q"), float(dt),
                                                 self._ptr(q1, name="q1"),
                                                 self._ptr(q2, name="q2"),
                                                 self._ptr(out, name="out")),
                    "cpr_rk3_step_stages")

    def adjoint_step_stages(self, q_n, q1, q2, dt, lam_np1, out=None):
        """cpr_adjoint_step_stages: the adjoint step with the stage states
        supplied."""
        out = self.empty() if out is None else out
        self._enter()
        self._check(self.lib.cpr_adjoint_step_stages(
            self._ctx, self._ptr(q_n, name="q_n"), self._ptr(q1, name="q1"),
            self._ptr(q2, name="q2"), float(dt), self._ptr(lam_np1, name="lam_np1"),
            self._ptr(out, name="lam_n")), "cpr_adjoint_step_stages")
        return out

    def coords(self):
        torch = _torch()
        shp = (self.ny, self.nx, self.n1, self.n1)
        x = torch.empty(shp, dtype=torch.float64, device=self.device)
        y = torch.empty_like(x)
        self._enter()
        self._check(self.lib.cpr_point_coords(self._ctx, self._ptr(x, shape=shp),
                                              self._ptr(y, shape=shp)), "cpr_point_coords")
        return x, y

    def integrals(self, q):
        out = (c_double * 4)()
        self._enter()
        self._check(self.lib.cpr_integrals(self._ctx, self._ptr(q, name="q"), out), "cpr_integrals")
        return np.array(out[:])

    def l2_diff(self, a, b=None, var=0):
        out = c_double(0.0)
        self._enter()
        bp = self._ptr(b, name="b") if b is not None else c_void_p(0)
        self._check(self.lib.cpr_l2_diff(self._ctx, self._ptr(a, name="a"), bp, int(var),
                                         byref(out)), "cpr_l2_diff")
        return float(out.value)

    def max_wavespeed(self, q):
        out = c_double(0.0)
        self._enter()
        self._check(self.lib.cpr_max_wavespeed(self._ctx, self._ptr(q, name="q"), byref(out)),
                    "cpr_max_wavespeed")
        return float(out.value)

    def set_time(self, t):
        self._enter()
        self._check(self.lib.cpr_set_time(self._ctx, float(t)), "cpr_set_time")

    def get_time(self):
        t, dt = c_double(0.0), c_double(0.0)
        self._enter()
        self._check(self.lib.cpr_get_time(self._ctx, byref(t), byref(dt)), "cpr_get_time")
        return float(t.value), float(dt.value)

    def troubled_total(self, reset=False):
        """Troubled elements summed over every limiter pass since the last
        reset (synchronises)."""
        n = c_int64(0)
        self._enter()
        self._check(self.lib.cpr_troubled_total(self._ctx, byref(n), 1 if reset else 0),
                    "cpr_troubled_total")
        return int(n.value)

    def sync(self):
        self._enter()
        self._check(self.lib.cpr_sync(self._ctx), "cpr_sync")

    def quad_weights(self):
        """w_i w_j dx dy / 4 per solution point, (n1, n1) float64 tensor,
        from the library's own quadrature table."""
        torch = _torch()
        _, w, _, _ = _lib.tables(self.P, SCHEME[self.scheme])
        w = torch.tensor(w, dtype=torch.float64, device=self.device)
        return torch.outer(w, w) * (self.dx * self.dy / 4.0)


class Rollout:
    """nsteps unlimited SSP-RK3 steps of fixed dt as a differentiable map
    q0 -> q_T (torch.autograd.Function). The backward pass runs the
    hand-written discrete adjoint step by step in reverse, storing the state
    every ckpt_every steps in the forward pass and recomputing each
    segment's states before sweeping it backwards. The recomputation keeps
    every step's two stage states too (cpr_rk3_step_stages), so that the
    sweep runs only the three transposes per step
    (cpr_adjoint_step_stages): memory holds three states per step of one
    segment plus the checkpoints."""

    @staticmethod
    def apply(q0, solver: Solver, dt: float, nsteps: int, ckpt_every: int):
        return _rollout_fn().apply(q0, solver, float(dt), int(nsteps), int(ckpt_every))


_ROLL = None


def _rollout_fn():
    global _ROLL
    if _ROLL is not None:
        return _ROLL
    torch = _torch()

    class _Rollout(torch.autograd.Function):
        @staticmethod
        def forward(ctx, q0, solver, dt, nsteps, ckpt_every):
            if ckpt_every < 1 or nsteps < 0:
                raise ValueError("need nsteps >= 0 and ckpt_every >= 1")
            q = q0.detach().contiguous().clone()
            ckpts = {0: q.clone()}
            for n in range(nsteps):
                solver.step(q, dt)
                if (n + 1) % ckpt_every == 0 and n + 1 < nsteps:
                    ckpts[n + 1] = q.clone()
            ctx.solver, ctx.dt, ctx.nsteps, ctx.C, ctx.ckpts = solver, dt, nsteps, ckpt_every, ckpts
            return q

        @staticmethod
        def backward(ctx, grad):
            solver, dt, nsteps, C, ckpts = ctx.solver, ctx.dt, ctx.nsteps, ctx.C, ctx.ckpts
            lam = grad.detach().contiguous().clone()
            # seg[i] = (q_n, q1, q2) of step s0 + i of the segment
            seg = torch.empty((min(C, max(nsteps, 1)), 3) + tuple(solver.shape),
                              dtype=torch.float64, device=solver.device)
            nxt = torch.empty(tuple(solver.shape), dtype=torch.float64, device=solver.device)
            starts = list(range(0, nsteps, C))
            for s0 in reversed(starts):
                s1 = min(s0 + C, nsteps)
                seg[0, 0].copy_(ckpts[s0])
                for i in range(s1 - s0):
                    last = i == s1 - s0 - 1
                    z = nxt if last else seg[i + 1, 0]   # q of the next step (unused after the last)
                    solver.step_stages(seg[i, 0], dt, seg[i, 1], seg[i, 2], out=z)
                for i in range(s1 - s0 - 1, -1, -1):
                    solver.adjoint_step_stages(seg[i, 0], seg[i, 1], seg[i, 2], dt, lam, out=lam)
            return lam, None, None, None, None

    _ROLL = _Rollout
    return _ROLL

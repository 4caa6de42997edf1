"""Differentiation form: gradients of a function of the final state of an RT
run with respect to the log source rates and the log cell densities, through
the hand-written adjoint kernels of librtm1.so (rt_step_record,
rt_step_adjoint), with step checkpointing, behind a torch.autograd.Function.

Setting of the adjoint: hydrogen-only gas, one photon group, GLF transport,
periodic box (the library refuses anything else); FP64 state or the mixed
form's FP32 radiation, whose gradient is that of the mixed forward map.

Forward: `steps` calls of rt_step, a copy of the state every `every` steps
(the checkpoints) and of each step's per-cell substep counts.  Backward,
segment by segment from the last: restore the checkpoint, re-run the
segment with rt_step_record (same result as rt_step) writing one tape per
step, then rt_step_adjoint over the segment's steps in reverse.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import capi
from .capi import check, lib


def _vp(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class GradientRun:
    """A run of `steps` RT steps of length dt on an RTContext (counters on)
    from a uniform initial state (x_HII = x0, T = T0, no radiation), with
    sources at cells ijk (K, 3).  Parameters: lnNdot (K,) and lnnH
    (nz, ny, nx), float64 torch tensors."""

    def __init__(self, ctx, ijk, dt: float, steps: int, x0: float, T0: float, every: int = 20):
        if ctx.nacc is None:
            raise ValueError("the RTContext needs counters=True (per-cell substep counts)")
        if ctx.M != 1:
            raise ValueError("the adjoint needs one photon group")
        self.ctx = ctx
        self.ijk = np.ascontiguousarray(ijk, dtype=np.int32).reshape(-1, 3)
        self.dt = float(dt)
        self.steps = int(steps)
        self.every = max(1, int(every))
        self.x0, self.T0 = float(x0), float(T0)
        self.nc = int(np.prod(ctx.n))
        dev = ctx.device
        self.counts = torch.empty((self.steps, self.nc), dtype=torch.int32, device=dev)
        self.ckpt = []
        self.off_len = int(lib().rt_tape_offsets_len(ctx._h))
        self.last_backward = {}
        # the forward run the checkpoints and counts belong to: its number
        # and its parameters, which backward() sets again before re-running
        self.forward_id = 0
        self.params = None

    # ------------------------------------------------------------ forward
    def _set_params(self, lnNdot: torch.Tensor, lnnH: torch.Tensor):
        ctx = self.ctx
        nd = torch.exp(lnNdot.detach().double()).cpu().numpy().reshape(-1, 1)
        ctx.set_sources(self.ijk, nd)
        ctx.nH.copy_(torch.exp(lnnH.detach().to(ctx.device, torch.float64)).reshape(ctx.nH.shape))

    def _initial_state(self):
        ctx = self.ctx
        ctx.N.zero_()
        ctx.F.zero_()
        ctx.xHII.fill_(self.x0)
        ctx.xHeII.zero_()
        ctx.xHeIII.zero_()
        ctx.T.fill_(self.T0)
        check(lib().rt_set_current(ctx._h, 0), ctx._h)

    def _snapshot(self):
        ctx = self.ctx
        c = ctx.current
        return (ctx.N[c].clone(), ctx.F[c].clone(), ctx.xHII.clone(), ctx.T.clone())

    def _restore(self, snap):
        ctx = self.ctx
        N, F, x, T = snap
        ctx.N[0].copy_(N)
        ctx.F[0].copy_(F)
        ctx.xHII.copy_(x)
        ctx.T.copy_(T)
        check(lib().rt_set_current(ctx._h, 0), ctx._h)

    def forward(self, lnNdot: torch.Tensor, lnnH: torch.Tensor) -> torch.Tensor:
        """Runs the steps; returns x_HII after the last one (a copy)."""
        ctx = self.ctx
        self._set_params(lnNdot, lnnH)
        self._initial_state()
        self.ckpt = []
        self.forward_id += 1
        self.params = (lnNdot.detach().clone(), lnnH.detach().clone())
        for k in range(self.steps):
            if k % self.every == 0:
                self.ckpt.append(self._snapshot())
            ctx.step(self.dt, 1)
            self.counts[k].copy_(ctx.nacc.reshape(-1))
        return ctx.xHII.clone()

    # ------------------------------------------------- frozen schedule
    def record_schedule(self):
        """Record the substep schedule of every step of the last forward run
        (its parameters must still be set) for replay()."""
        ctx = self.ctx
        L = lib()
        dev = ctx.device
        nc = self.nc
        self._restore(self.ckpt[0])
        entries = (self.counts.to(torch.int64).sum(dim=1) + nc).cpu().tolist()
        base = np.concatenate([[0], np.cumsum(entries)]).astype(np.int64)
        trace = torch.empty(int(base[-1]) * 7, dtype=torch.float64, device=dev)
        off = torch.empty((self.steps, self.off_len), dtype=torch.int64, device=dev)
        Na = torch.empty(nc, dtype=torch.float64, device=dev)
        Fa = torch.empty(3 * nc, dtype=torch.float64, device=dev)
        tapes = []
        for k in range(self.steps):
            t = capi.RtTape(_vp(Na), _vp(Fa), _vp(self.counts[k]), _vp(off[k]),
                            ctypes.c_void_p(trace.data_ptr() + int(base[k]) * 7 * 8), int(entries[k]))
            check(L.rt_step_record(ctx._h, self.dt, ctypes.byref(t)), ctx._h)
            tapes.append(t)
        self._sched = (trace, off, Na, Fa, self.counts.clone(), tapes)
        for k, t in enumerate(tapes):
            t.counts = _vp(self._sched[4][k])
        return int(base[-1])

    def replay(self, lnNdot: torch.Tensor, lnnH: torch.Tensor) -> torch.Tensor:
        """x_HII after the run with the recorded substep schedule held fixed
        (rt_step_replay): the function whose gradient backward() returns."""
        ctx = self.ctx
        self._set_params(lnNdot, lnnH)
        self._initial_state()
        for t in self._sched[5]:
            check(lib().rt_step_replay(ctx._h, self.dt, ctypes.byref(t)), ctx._h)
        return ctx.xHII.clone()

    # ----------------------------------------------------------- backward
    def backward(self, grad_x: torch.Tensor, grad_T: Optional[torch.Tensor] = None,
                 forward_id: Optional[int] = None):
        """dL/dln Ndot (K,) and dL/dln n_H (nz, ny, nx) for dL/dx_HII = grad_x
        (and dL/dT = grad_T) at the end of the last forward run, at that
        run's parameters (set again here, whatever the context holds now).
        With forward_id, raises RTError unless the checkpoints still belong
        to that forward run."""
        if self.params is None:
            raise capi.RTError("backward before any forward run")
        if forward_id is not None and forward_id != self.forward_id:
            raise capi.RTError(f"the checkpoints of forward run {forward_id} were replaced by forward run "
                               f"{self.forward_id}")
        ctx = self.ctx
        self._set_params(*self.params)
        L = lib()
        dev = ctx.device
        nc = self.nc
        f64 = torch.float64
        lam_N = torch.zeros(nc, dtype=f64, device=dev)
        lam_F = torch.zeros(3 * nc, dtype=f64, device=dev)
        lam_x = grad_x.detach().to(dev, f64).reshape(-1).clone()
        lam_T = (grad_T.detach().to(dev, f64).reshape(-1).clone() if grad_T is not None
                 else torch.zeros(nc, dtype=f64, device=dev))
        wN = torch.empty(nc, dtype=f64, device=dev)
        wF = torch.empty(3 * nc, dtype=f64, device=dev)
        adj = capi.RtAdj(_vp(lam_N), _vp(lam_F), _vp(lam_x), _vp(lam_T), _vp(wN), _vp(wF))
        g_src = torch.zeros(self.ijk.shape[0], dtype=f64, device=dev)
        g_nH = torch.zeros(nc, dtype=f64, device=dev)
        ctx.reset_stats()
        nseg = len(self.ckpt)
        peak_trace = 0
        for seg in reversed(range(nseg)):
            k0 = seg * self.every
            k1 = min(k0 + self.every, self.steps)
            ns = k1 - k0
            self._restore(self.ckpt[seg])
            entries = (self.counts[k0:k1].to(torch.int64).sum(dim=1) + nc).cpu().tolist()
            base = np.concatenate([[0], np.cumsum(entries)]).astype(np.int64)
            peak_trace = max(peak_trace, int(base[-1]))
            trace = torch.empty(int(base[-1]) * 7, dtype=f64, device=dev)
            Na = torch.empty((ns, nc), dtype=f64, device=dev)
            Fa = torch.empty((ns, 3 * nc), dtype=f64, device=dev)
            off = torch.empty((ns, self.off_len), dtype=torch.int64, device=dev)
            tapes = []
            for j in range(ns):
                t = capi.RtTape(_vp(Na[j]), _vp(Fa[j]), _vp(self.counts[k0 + j]), _vp(off[j]),
                                ctypes.c_void_p(trace.data_ptr() + int(base[j]) * 7 * 8), int(entries[j]))
                tapes.append(t)
                check(L.rt_step_record(ctx._h, self.dt, ctypes.byref(t)), ctx._h)
            for j in reversed(range(ns)):
                check(L.rt_step_adjoint(ctx._h, self.dt, ctypes.byref(tapes[j]), ctypes.byref(adj),
                                        _vp(g_src), _vp(g_nH)), ctx._h)
            del trace, Na, Fa, off
        st = ctx.stats()
        if st["flags"] & capi.RT_FLAG_TRACE:
            raise capi.RTError("adjoint tape mismatch: the recorded chemistry took another substep count "
                               "than the forward run")
        self.last_backward = {"trace_entries_max": peak_trace, "flags": st["flags"]}
        return g_src, g_nH.reshape(ctx.nH.shape), lam_N, lam_F, lam_x, lam_T


class RTRun(torch.autograd.Function):
    """x_HII after the run as a differentiable function of (lnNdot, lnnH)."""

    @staticmethod
    def forward(fctx, lnNdot, lnnH, run: GradientRun):
        fctx.run = run
        fctx.src_device = lnNdot.device
        x = run.forward(lnNdot, lnnH)
        fctx.forward_id = run.forward_id
        return x

    @staticmethod
    def backward(fctx, grad_x):
        g_src, g_nH = fctx.run.backward(grad_x, forward_id=fctx.forward_id)[:2]
        return g_src.to(fctx.src_device), g_nH, None


def rt_run(run: GradientRun, lnNdot: torch.Tensor, lnnH: torch.Tensor) -> torch.Tensor:
    return RTRun.apply(lnNdot, lnnH, run)

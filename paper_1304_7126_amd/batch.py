"""Torch-backed driver of the batched C ABI (rt_batch_*): many independent
boxes advanced together, one HIP graph launch per step."""
from __future__ import annotations

import ctypes
from typing import List, Sequence

import numpy as np
import torch

from . import capi
from .capi import lib


def _check(rc, b=None):
    if rc != capi.RT_OK:
        msg = lib().rt_batch_last_error(b)
        raise capi.RTError(f"rtm1 batch error {rc}: {msg.decode() if msg else ''}")


class BoxState:
    """Device arrays of one box (same layout as runtime.RTContext)."""

    def __init__(self, n, M, fp32, device, counters):
        nx, ny, nz = n
        rdt = torch.float32 if fp32 else torch.float64
        self.n, self.M = tuple(n), M
        self.N = torch.zeros((2, M, nz, ny, nx), dtype=rdt, device=device)
        self.F = torch.zeros((2, M, 3, nz, ny, nx), dtype=rdt, device=device)
        z = torch.zeros((nz, ny, nx), dtype=torch.float64, device=device)
        self.xHII, self.xHeII, self.xHeIII, self.T, self.nH = z, z.clone(), z.clone(), z.clone(), z.clone()
        self.nacc = torch.zeros((nz, ny, nx), dtype=torch.int32, device=device) if counters else None
        self.natt = torch.zeros_like(self.nacc) if counters else None

    def c_state(self):
        s = capi.RtState()
        s.N[0], s.N[1] = self.N[0].data_ptr(), self.N[1].data_ptr()
        s.F[0], s.F[1] = self.F[0].data_ptr(), self.F[1].data_ptr()
        s.xHII, s.xHeII, s.xHeIII = self.xHII.data_ptr(), self.xHeII.data_ptr(), self.xHeIII.data_ptr()
        s.T, s.nH = self.T.data_ptr(), self.nH.data_ptr()
        s.nacc = self.nacc.data_ptr() if self.nacc is not None else None
        s.natt = self.natt.data_ptr() if self.natt is not None else None
        return s


class RTBatch:
    """nbox boxes: grids = [(n, dx, bc)], groups = [(M, c_r, sigN, sigE, ebar)];
    method parameters common to all boxes."""

    def __init__(self, grids, groups, flux=0, isothermal=False, X=0.76, Y=0.24, gamma=5.0 / 3.0, a_exp=1.0,
                 x_min=1e-6, N_floor=0.0, max_attempts=100000, fp32=False, device="cuda", counters=False,
                 smooth=False, otsa=True):
        L = lib()
        nb = len(grids)
        cg = (capi.RtGrid * nb)()
        cr = (capi.RtGroups * nb)()
        for i, ((n, dx, bc), (M, c_r, sN, sE, eb)) in enumerate(zip(grids, groups)):
            cg[i].nx, cg[i].ny, cg[i].nz = (int(v) for v in n)
            cg[i].dx = float(dx)
            for f in range(6):
                cg[i].bc[f] = int(bc[f])
            cr[i].M, cr[i].c_r = int(M), float(c_r)
            for a in range(3):
                for j in range(3):
                    cr[i].sigN[a][j] = float(sN[a][j])
                    cr[i].sigE[a][j] = float(sE[a][j])
                cr[i].ebar[a] = float(eb[a])
        p = capi.RtParams()
        p.flux, p.otsa, p.isothermal = int(flux), int(bool(otsa)), int(bool(isothermal))
        p.prec = capi.RT_PREC_FP32_TRANSPORT if fp32 else capi.RT_PREC_FP64
        p.X, p.Y, p.gamma, p.a_exp = float(X), float(Y), float(gamma), float(a_exp)
        p.x_min, p.N_floor, p.max_attempts = float(x_min), float(N_floor), int(max_attempts)
        p.smooth = int(bool(smooth))
        h = ctypes.c_void_p()
        _check(L.rt_batch_init(nb, cg, cr, ctypes.byref(p), ctypes.byref(h)), None)
        self._h = h
        self.nbox = nb
        self.device = torch.device(device)
        self.fp32 = fp32
        self.dx = [float(g[1]) for g in grids]
        self.c_r = float(groups[0][1])
        self.boxes: List[BoxState] = [BoxState(g[0], gr[0], fp32, self.device, counters)
                                      for g, gr in zip(grids, groups)]
        sb = int(L.rt_batch_scratch_bytes(h))
        self.scratch = torch.zeros(max(sb, 256), dtype=torch.uint8, device=self.device)
        states = (capi.RtState * nb)(*[b.c_state() for b in self.boxes])
        _check(L.rt_batch_bind(h, states, ctypes.c_void_p(self.scratch.data_ptr()), self.scratch.numel()), h)
        # graphs need a capturable stream: a dedicated one of default priority
        self.stream = torch.cuda.Stream(device=self.device)
        _check(L.rt_batch_set_stream(h, ctypes.c_void_p(self.stream.cuda_stream)), h)

    def load_box(self, i, st):
        b = self.boxes[i]
        torch.cuda.synchronize(self.device)
        b.N[0].copy_(torch.as_tensor(np.asarray(st["N"]), dtype=b.N.dtype))
        b.F[0].copy_(torch.as_tensor(np.asarray(st["F"]), dtype=b.F.dtype))
        b.N[1].zero_()
        b.F[1].zero_()
        for k in ("xHII", "xHeII", "xHeIII", "T", "nH"):
            getattr(b, k).copy_(torch.as_tensor(np.asarray(st[k]), dtype=torch.float64))
        torch.cuda.synchronize(self.device)
        _check(lib().rt_batch_set_current(self._h, 0), self._h)

    def set_sources(self, i, ijk, ndot):
        M = self.boxes[i].M
        ijk = np.ascontiguousarray(ijk, dtype=np.int32).reshape(-1, 3)
        ndot = np.ascontiguousarray(ndot, dtype=np.float64).reshape(ijk.shape[0], M)
        _check(lib().rt_batch_set_sources(self._h, int(i), int(ijk.shape[0]),
                                          ijk.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                          ndot.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), self._h)

    def set_tuning(self, head_blocks_per_cu=-1, head_attempts=-1, tail_blocks=-1, use_graph=-1):
        _check(lib().rt_batch_set_tuning(self._h, int(head_blocks_per_cu), int(head_attempts), int(tail_blocks),
                                         int(use_graph)), self._h)

    def courant_dt(self, courant=0.8):
        v = ctypes.c_double()
        _check(lib().rt_batch_courant_dt(self._h, float(courant), ctypes.byref(v)), self._h)
        return v.value

    def step(self, dt=0.0, nsteps=1):
        torch.cuda.current_stream(self.device).synchronize()
        _check(lib().rt_batch_step(self._h, float(dt), int(nsteps)), self._h)

    def synchronize(self):
        self.stream.synchronize()

    @property
    def current(self):
        return int(lib().rt_batch_current(self._h))

    def state_numpy(self, i):
        self.synchronize()
        b = self.boxes[i]
        c = self.current
        out = {"N": b.N[c].double().cpu().numpy(), "F": b.F[c].double().cpu().numpy()}
        for k in ("xHII", "xHeII", "xHeIII", "T", "nH"):
            out[k] = getattr(b, k).cpu().numpy()
        if b.nacc is not None:
            out["nacc"], out["natt"] = b.nacc.cpu().numpy(), b.natt.cpu().numpy()
        return out

    def stats(self):
        s = capi.RtStats()
        _check(lib().rt_batch_get_stats(self._h, ctypes.byref(s)), self._h)
        return {"substeps_total": s.substeps_total, "attempts_total": s.attempts_total,
                "attempts_max": s.attempts_max, "flags": s.flags}

    def reset_stats(self):
        _check(lib().rt_batch_reset_stats(self._h), self._h)

    def snapshot(self):
        """Device copies of every box's current state (for the autotuner)."""
        self.synchronize()
        return [(b.N.clone(), b.F.clone(), b.xHII.clone(), b.xHeII.clone(), b.xHeIII.clone(), b.T.clone())
                for b in self.boxes], self.current

    def restore(self, snap):
        arrays, cur = snap
        self.synchronize()
        for b, (N, F, x, y2, y3, T) in zip(self.boxes, arrays):
            b.N.copy_(N)
            b.F.copy_(F)
            b.xHII.copy_(x)
            b.xHeII.copy_(y2)
            b.xHeIII.copy_(y3)
            b.T.copy_(T)
        torch.cuda.synchronize(self.device)
        _check(lib().rt_batch_set_current(self._h, cur), self._h)

    def close(self):
        if getattr(self, "_h", None):
            lib().rt_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_from_specs(specs, dx, fp32=True, counters=False, seed_sources=True, **kw):
    """RTBatch for rt_inputs.BoxSpec descriptions (periodic, GLF, 1e5 K
    blackbody groups), loaded with initial states and sources.  Returns
    (batch, workloads, source lists)."""
    import rt_inputs as ri
    from .runtime import spectrum_attributes
    ws = [ri.batch_box_workload(s, dx, steps=0) for s in specs]
    grids, groups, fracs = [], [], []
    for w in ws:
        sN, sE, eb, fr = spectrum_attributes(w.spectrum)
        grids.append((w.n, w.dx, w.bc))
        groups.append((w.spectrum.M, w.c_r, sN, sE, eb))
        fracs.append(fr[: w.spectrum.M])
    b = RTBatch(grids, groups, flux=ws[0].flux, X=ws[0].X, Y=ws[0].Y, fp32=fp32, counters=counters, **kw)
    srcs = []
    for i, w in enumerate(ws):
        b.load_box(i, ri.initial_state(w))
        ijk, nd = ri.random_sources(w.n, w.n_sources, w.seed)
        f = fracs[i] / fracs[i].sum() if w.spectrum.M > 1 else np.ones(1)
        ndot = np.outer(nd, f)
        b.set_sources(i, ijk, ndot)
        srcs.append((ijk, nd))
    return b, ws, srcs

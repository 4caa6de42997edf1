"""Torch-backed driver of the C ABI: torch provides device memory and the
stream; every step of the method runs in the HIP kernels of librtm1.so."""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np
import torch

from . import capi
from .capi import check, lib


def group_attributes(T_bb: float, edges_eV: Sequence[float]):
    """Blackbody photon-group attributes from the library (host quadrature):
    (sigN (3,3), sigE (3,3), ebar (3,) erg, frac (3,))."""
    M = len(edges_eV) - 1
    e = np.ascontiguousarray(edges_eV, dtype=np.float64)
    sN = np.zeros((3, 3))
    sE = np.zeros((3, 3))
    eb = np.zeros(3)
    fr = np.zeros(3)
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    check(lib().rt_group_attributes(float(T_bb), M, dp(e), dp(sN), dp(sE), dp(eb), dp(fr)))
    return sN, sE, eb, fr


def hll_table(nf: int = 101, nth: int = 101) -> np.ndarray:
    out = np.zeros((nf, nth, 2))
    check(lib().rt_build_hll_table(nf, nth, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return out


def spectrum_attributes(spec):
    """Group attributes for an rt_inputs.Spectrum description."""
    if spec.kind == "mono":
        M = len(spec.mono_energy_eV)
        sN = np.zeros((3, 3))
        eb = np.zeros(3)
        fr = np.zeros(3)
        for i in range(M):
            sN[i] = spec.mono_sigma[i]
            eb[i] = spec.mono_energy_eV[i] * 1.602176634e-12
            fr[i] = 1.0 / M
        return sN, sN.copy(), eb, fr
    return group_attributes(spec.T_bb, spec.edges_eV)


class RTContext:
    """One uniform grid on one GPU.

    State tensors (device, contiguous, x fastest):
      N  (2, M, nz, ny, nx)      two radiation sets (App. D source/destination)
      F  (2, M, 3, nz, ny, nx)   float64, or float32 with prec=FP32 transport
      xHII, xHeII, xHeIII, T, nH (nz, ny, nx) float64
    """

    def __init__(self, n, dx, bc, M, c_r, sigN, sigE, ebar, flux=0, isothermal=False, X=0.76, Y=0.24,
                 gamma=5.0 / 3.0, a_exp=1.0, x_min=1e-6, N_floor=0.0, max_attempts=100000, fp32=False,
                 device="cuda", counters=False, smooth=False, otsa=True, brec=(-1, -1, -1), scratch=True):
        L = lib()
        g = capi.RtGrid()
        g.nx, g.ny, g.nz = (int(v) for v in n)
        g.dx = float(dx)
        for i in range(6):
            g.bc[i] = int(bc[i])
        gr = capi.RtGroups()
        gr.M = int(M)
        gr.c_r = float(c_r)
        for i in range(3):
            for j in range(3):
                gr.sigN[i][j] = float(sigN[i][j])
                gr.sigE[i][j] = float(sigE[i][j])
            gr.ebar[i] = float(ebar[i])
            gr.brec[i] = int(brec[i])
        p = capi.RtParams()
        p.flux = int(flux)
        p.otsa = int(bool(otsa))
        p.isothermal = int(bool(isothermal))
        p.prec = capi.RT_PREC_FP32_TRANSPORT if fp32 else capi.RT_PREC_FP64
        p.X, p.Y = float(X), float(Y)
        p.gamma = float(gamma)
        p.a_exp = float(a_exp)
        p.x_min = float(x_min)
        p.N_floor = float(N_floor)
        p.max_attempts = int(max_attempts)
        p.smooth = int(bool(smooth))
        h = ctypes.c_void_p()
        rc = L.rt_init(ctypes.byref(g), ctypes.byref(gr), ctypes.byref(p), ctypes.byref(h))
        check(rc, None)
        self._h = h
        self.n = tuple(int(v) for v in n)
        self.M = int(M)
        self.dx = float(dx)
        self.c_r = float(c_r)
        self.fp32 = bool(fp32)
        self.smooth = bool(smooth)
        self.otsa = bool(otsa)
        self.device = torch.device(device)
        nx, ny, nz = self.n
        rdt = torch.float32 if fp32 else torch.float64
        f64 = torch.float64
        dev = self.device
        self.N = torch.zeros((2, self.M, nz, ny, nx), dtype=rdt, device=dev)
        self.F = torch.zeros((2, self.M, 3, nz, ny, nx), dtype=rdt, device=dev)
        self.xHII = torch.zeros((nz, ny, nx), dtype=f64, device=dev)
        self.xHeII = torch.zeros_like(self.xHII)
        self.xHeIII = torch.zeros_like(self.xHII)
        self.T = torch.zeros_like(self.xHII)
        self.nH = torch.zeros_like(self.xHII)
        self.nacc = torch.zeros((nz, ny, nx), dtype=torch.int32, device=dev) if counters else None
        self.natt = torch.zeros_like(self.nacc) if counters else None
        # scratch=False: no scratch buffer (the context steps with step_noalloc)
        sb = int(L.rt_scratch_bytes(h))
        self.scratch = torch.zeros(max(sb, 256), dtype=torch.uint8, device=dev) if scratch else None
        self._bind()
        self.set_stream(torch.cuda.current_stream(dev))

    # -------------------------------------------------------------- set up
    @classmethod
    def for_workload(cls, w, fp32=False, **over):
        sN, sE, eb, fr = spectrum_attributes(w.spectrum)
        kw = dict(n=w.n, dx=w.dx, bc=w.bc, M=w.spectrum.M, c_r=w.c_r, sigN=sN, sigE=sE, ebar=eb, flux=w.flux,
                  isothermal=w.isothermal, X=w.X, Y=w.Y, gamma=w.gamma, a_exp=w.a_exp, x_min=w.x_min, fp32=fp32,
                  otsa=w.otsa, brec=w.brec)
        kw.update(over)
        ctx = cls(**kw)
        ctx.group_frac = fr[: w.spectrum.M].copy()
        inflow = w.inflow_flux(fr)
        for face in range(6):
            if w.bc[face] == capi.RT_BC_INFLOW:
                ctx.set_inflow(face, inflow[face])
        return ctx

    def _bind(self):
        s = capi.RtState()
        s.N[0] = self.N[0].data_ptr()
        s.N[1] = self.N[1].data_ptr()
        s.F[0] = self.F[0].data_ptr()
        s.F[1] = self.F[1].data_ptr()
        s.xHII = self.xHII.data_ptr()
        s.xHeII = self.xHeII.data_ptr()
        s.xHeIII = self.xHeIII.data_ptr()
        s.T = self.T.data_ptr()
        s.nH = self.nH.data_ptr()
        s.nacc = self.nacc.data_ptr() if self.nacc is not None else None
        s.natt = self.natt.data_ptr() if self.natt is not None else None
        s.scratch = self.scratch.data_ptr() if self.scratch is not None else None
        s.scratch_bytes = self.scratch.numel() if self.scratch is not None else 0
        check(lib().rt_bind(self._h, ctypes.byref(s)), self._h)

    def set_stream(self, stream):
        check(lib().rt_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)), self._h)

    def load_state(self, st):
        """Copy a host state dict (numpy, as produced by rt_inputs) into set 0."""
        rdt = self.N.dtype
        self.N[0].copy_(torch.as_tensor(np.asarray(st["N"]), dtype=rdt))
        self.F[0].copy_(torch.as_tensor(np.asarray(st["F"]), dtype=rdt))
        self.N[1].zero_()
        self.F[1].zero_()
        for k in ("xHII", "xHeII", "xHeIII", "T", "nH"):
            getattr(self, k).copy_(torch.as_tensor(np.asarray(st[k]), dtype=torch.float64))
        check(lib().rt_set_current(self._h, 0), self._h)

    def set_sources(self, ijk, ndot):
        ijk = np.ascontiguousarray(ijk, dtype=np.int32).reshape(-1, 3)
        ndot = np.ascontiguousarray(ndot, dtype=np.float64).reshape(ijk.shape[0], self.M)
        check(lib().rt_set_sources(self._h, int(ijk.shape[0]), ijk.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   ndot.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), self._h)

    def source_rates(self, ndot_total):
        f = self.group_frac / self.group_frac.sum() if self.M > 1 else np.ones(1)
        return np.ascontiguousarray(np.outer(np.asarray(ndot_total, np.float64), f))

    def set_tuning(self, head_attempts=-1, queue_cap=-1):
        """Launch tuning of the chemistry passes (results do not depend on it)."""
        check(lib().rt_set_tuning(self._h, int(head_attempts), int(queue_cap)), self._h)

    PATHS = {"auto": 0, "cell": 1, "zmarch": 2}

    def set_transport_path(self, path):
        """Transport kernel arrangement: 'auto', 'cell' or 'zmarch' (same results)."""
        check(lib().rt_set_transport_path(self._h, self.PATHS[path]), self._h)

    CHEM_PATHS = {"auto": 0, "two-pass": 1, "one-pass": 2}

    def set_chem_path(self, path):
        """Chemistry kernel arrangement after a separate transport: 'auto',
        'two-pass' (head + tail) or 'one-pass' (same results)."""
        check(lib().rt_set_chem_path(self._h, self.CHEM_PATHS[path]), self._h)

    def courant_dt(self, courant=0.8):
        v = ctypes.c_double()
        check(lib().rt_courant_dt(self._h, float(courant), ctypes.byref(v)), self._h)
        return v.value

    # -------------------------------------------------------------- steps
    def inject(self, dt):
        check(lib().rt_inject(self._h, float(dt)), self._h)

    def transport(self, dt):
        check(lib().rt_transport(self._h, float(dt)), self._h)

    def thermochem(self, dt):
        check(lib().rt_thermochem(self._h, float(dt)), self._h)

    def step(self, dt=0.0, nsteps=1):
        check(lib().rt_step(self._h, float(dt), int(nsteps)), self._h)

    def step_noalloc(self, dt=0.0, nsteps=1):
        """rt_step in the library's static per-GPU scratch (no allocation)."""
        check(lib().rt_step_noalloc(self._h, float(dt), int(nsteps)), self._h)

    # ------------------------------------------------------------ results
    @property
    def current(self) -> int:
        return int(lib().rt_current(self._h))

    def radiation(self):
        c = self.current
        return self.N[c], self.F[c]

    def state_numpy(self):
        torch.cuda.synchronize(self.device)
        N, F = self.radiation()
        out = {"N": N.double().cpu().numpy(), "F": F.double().cpu().numpy()}
        for k in ("xHII", "xHeII", "xHeIII", "T", "nH"):
            out[k] = getattr(self, k).cpu().numpy()
        if self.nacc is not None:
            out["nacc"] = self.nacc.cpu().numpy()
            out["natt"] = self.natt.cpu().numpy()
        return out

    def stats(self):
        s = capi.RtStats()
        check(lib().rt_get_stats(self._h, ctypes.byref(s)), self._h)
        M = self.M
        return {"photons": list(s.photons)[:M], "ionised_H": s.ionised_H, "max_f": s.max_f,
                "min_N": s.min_N, "substeps_total": s.substeps_total, "attempts_total": s.attempts_total,
                "attempts_max": s.attempts_max, "flags": s.flags, "injected": list(s.injected)[:M],
                "absorbed": list(s.absorbed)[:M], "outflow": list(s.outflow)[:M],
                "substep_hist": list(s.substep_hist)}

    def set_inflow(self, face, flux):
        """Photon flux [s^-1 cm^-2] per group entering through an
        RT_BC_INFLOW face (0..5 = -x,+x,-y,+y,-z,+z)."""
        f = np.ascontiguousarray(np.asarray(flux, np.float64).reshape(self.M))
        check(lib().rt_set_inflow(self._h, int(face), f.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), self._h)

    def set_expansion(self, a):
        """Super-comoving variables at expansion factor a (Sec. 5.4): the
        radiation arrays hold a^3 N and a^4 F, nH holds a^3 n_H."""
        check(lib().rt_set_expansion(self._h, float(a)), self._h)

    def set_accounting(self, enabled=True):
        """Photon accounting (injected, absorbed, outflow, substep histogram)."""
        check(lib().rt_set_accounting(self._h, int(bool(enabled))), self._h)

    def set_timing(self, enabled=True):
        check(lib().rt_set_timing(self._h, int(bool(enabled))), self._h)

    def timing(self):
        """{kernel class: (total ms, launches)} since the last call (syncs)."""
        t = capi.RtTiming()
        check(lib().rt_get_timing(self._h, ctypes.byref(t)), self._h)
        return {k: (t.ms[i], t.launches[i]) for i, k in enumerate(capi.TIMING_CLASSES)}

    def reset_stats(self):
        check(lib().rt_reset_stats(self._h), self._h)

    def hll_table(self):
        p = ctypes.POINTER(ctypes.c_double)()
        nf = ctypes.c_int()
        nth = ctypes.c_int()
        check(lib().rt_hll_table(self._h, ctypes.byref(p), ctypes.byref(nf), ctypes.byref(nth)), self._h)
        return np.ctypeslib.as_array(p, shape=(nf.value, nth.value, 2)).copy()

    def close(self):
        if getattr(self, "_h", None):
            lib().rt_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

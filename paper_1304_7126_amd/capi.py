"""ctypes declarations of the C ABI in include/rtm1.h (argument marshalling only).

The shared library is built in-tree by paper_1304_7126_amd/build.py (hipcc,
gfx950).  Loading fails loudly when it is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librtm1.so")

RT_OK, RT_EINVAL, RT_EHIP, RT_ENOMEM, RT_ESTATE, RT_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
RT_BC_PERIODIC, RT_BC_OUTFLOW, RT_BC_REFLECT, RT_BC_INFLOW = 0, 1, 2, 3
RT_FLUX_GLF, RT_FLUX_HLL = 0, 1
RT_PREC_FP64, RT_PREC_FP32_TRANSPORT = 0, 1
RT_FLAG_CAP, RT_FLAG_NAN, RT_FLAG_NNEG, RT_FLAG_TRACE = 1, 2, 8, 16

EXPORTED = [
    "rt_init", "rt_scratch_bytes", "rt_bind", "rt_set_stream", "rt_current", "rt_set_current",
    "rt_set_sources", "rt_courant_dt", "rt_inject", "rt_transport", "rt_thermochem", "rt_step",
    "rt_get_stats", "rt_reset_stats", "rt_group_attributes", "rt_hll_table", "rt_build_hll_table",
    "rt_last_error", "rt_free", "rt_set_tuning", "rt_set_transport_path", "rt_set_chem_path", "rt_set_timing", "rt_get_timing",
    "rt_batch_init", "rt_batch_scratch_bytes", "rt_batch_bind", "rt_batch_set_stream", "rt_batch_current",
    "rt_batch_set_current", "rt_batch_set_sources", "rt_batch_courant_dt", "rt_batch_step", "rt_batch_set_tuning", "rt_batch_get_stats",
    "rt_batch_reset_stats", "rt_batch_last_error", "rt_batch_free",
    "rt_tape_offsets_len", "rt_step_record", "rt_step_replay", "rt_step_adjoint", "rt_set_accounting",
    "rt_set_inflow", "rt_set_expansion", "rt_step_noalloc",
]


class RtGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("dx", ctypes.c_double), ("bc", ctypes.c_int * 6)]


class RtGroups(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int), ("c_r", ctypes.c_double),
                ("sigN", (ctypes.c_double * 3) * 3), ("sigE", (ctypes.c_double * 3) * 3),
                ("ebar", ctypes.c_double * 3), ("brec", ctypes.c_int * 3)]


class RtParams(ctypes.Structure):
    _fields_ = [("flux", ctypes.c_int), ("otsa", ctypes.c_int), ("isothermal", ctypes.c_int),
                ("prec", ctypes.c_int), ("X", ctypes.c_double), ("Y", ctypes.c_double),
                ("gamma", ctypes.c_double), ("a_exp", ctypes.c_double), ("x_min", ctypes.c_double),
                ("N_floor", ctypes.c_double), ("max_attempts", ctypes.c_longlong), ("smooth", ctypes.c_int)]


class RtState(ctypes.Structure):
    _fields_ = [("N", ctypes.c_void_p * 2), ("F", ctypes.c_void_p * 2),
                ("xHII", ctypes.c_void_p), ("xHeII", ctypes.c_void_p), ("xHeIII", ctypes.c_void_p),
                ("T", ctypes.c_void_p), ("nH", ctypes.c_void_p),
                ("nacc", ctypes.c_void_p), ("natt", ctypes.c_void_p),
                ("scratch", ctypes.c_void_p), ("scratch_bytes", ctypes.c_size_t)]


class RtStats(ctypes.Structure):
    _fields_ = [("photons", ctypes.c_double * 3), ("ionised_H", ctypes.c_double),
                ("max_f", ctypes.c_double), ("min_N", ctypes.c_double),
                ("substeps_total", ctypes.c_longlong), ("attempts_total", ctypes.c_longlong),
                ("attempts_max", ctypes.c_longlong), ("flags", ctypes.c_uint),
                ("injected", ctypes.c_double * 3), ("absorbed", ctypes.c_double * 3),
                ("outflow", ctypes.c_double * 3), ("substep_hist", ctypes.c_longlong * 64)]


TIMING_CLASSES = ("inject", "transport", "head", "tail", "other", "accounting")


class RtTiming(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * len(TIMING_CLASSES)), ("launches", ctypes.c_longlong * len(TIMING_CLASSES))]


class RtTape(ctypes.Structure):
    _fields_ = [("Na", ctypes.c_void_p), ("Fa", ctypes.c_void_p), ("counts", ctypes.c_void_p),
                ("off", ctypes.c_void_p), ("trace", ctypes.c_void_p), ("cap", ctypes.c_longlong)]


class RtAdj(ctypes.Structure):
    _fields_ = [("N", ctypes.c_void_p), ("F", ctypes.c_void_p), ("xHII", ctypes.c_void_p),
                ("T", ctypes.c_void_p), ("wN", ctypes.c_void_p), ("wF", ctypes.c_void_p)]

_lib = None


def lib():
    """Load librtm1.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1304_7126_amd.build` "
                           "(or __graft_entry__.build()); there is no fallback path")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    st = ctypes.c_int
    L.rt_init.argtypes = [ctypes.POINTER(RtGrid), ctypes.POINTER(RtGroups), ctypes.POINTER(RtParams),
                          ctypes.POINTER(vp)]
    L.rt_init.restype = st
    L.rt_scratch_bytes.argtypes = [vp]
    L.rt_scratch_bytes.restype = ctypes.c_size_t
    L.rt_bind.argtypes = [vp, ctypes.POINTER(RtState)]
    L.rt_bind.restype = st
    L.rt_set_stream.argtypes = [vp, vp]
    L.rt_set_stream.restype = st
    L.rt_current.argtypes = [vp]
    L.rt_current.restype = ctypes.c_int
    L.rt_set_current.argtypes = [vp, ctypes.c_int]
    L.rt_set_current.restype = st
    L.rt_set_sources.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int32), dp]
    L.rt_set_sources.restype = st
    L.rt_courant_dt.argtypes = [vp, ctypes.c_double, dp]
    L.rt_courant_dt.restype = st
    for name in ("rt_inject", "rt_transport", "rt_thermochem"):
        f = getattr(L, name)
        f.argtypes = [vp, ctypes.c_double]
        f.restype = st
    L.rt_step.argtypes = [vp, ctypes.c_double, ctypes.c_int]
    L.rt_step_noalloc.argtypes = [vp, ctypes.c_double, ctypes.c_int]
    L.rt_step_noalloc.restype = st
    L.rt_step.restype = st
    L.rt_set_tuning.argtypes = [vp, ctypes.c_int, ctypes.c_longlong]
    L.rt_set_tuning.restype = st
    L.rt_set_transport_path.argtypes = [vp, ctypes.c_int]
    L.rt_set_transport_path.restype = st
    L.rt_set_chem_path.argtypes = [vp, ctypes.c_int]
    L.rt_set_chem_path.restype = st
    L.rt_set_timing.argtypes = [vp, ctypes.c_int]
    L.rt_set_timing.restype = st
    L.rt_get_timing.argtypes = [vp, ctypes.POINTER(RtTiming)]
    L.rt_get_timing.restype = st
    L.rt_get_stats.argtypes = [vp, ctypes.POINTER(RtStats)]
    L.rt_get_stats.restype = st
    L.rt_reset_stats.argtypes = [vp]
    L.rt_reset_stats.restype = st
    L.rt_set_accounting.argtypes = [vp, ctypes.c_int]
    L.rt_set_accounting.restype = st
    L.rt_set_inflow.argtypes = [vp, ctypes.c_int, dp]
    L.rt_set_inflow.restype = st
    L.rt_set_expansion.argtypes = [vp, ctypes.c_double]
    L.rt_set_expansion.restype = st
    L.rt_group_attributes.argtypes = [ctypes.c_double, ctypes.c_int, dp, dp, dp, dp, dp]
    L.rt_group_attributes.restype = st
    L.rt_hll_table.argtypes = [vp, ctypes.POINTER(dp), ctypes.POINTER(ctypes.c_int),
                               ctypes.POINTER(ctypes.c_int)]
    L.rt_hll_table.restype = st
    L.rt_build_hll_table.argtypes = [ctypes.c_int, ctypes.c_int, dp]
    L.rt_build_hll_table.restype = st
    L.rt_last_error.argtypes = [vp]
    L.rt_last_error.restype = ctypes.c_char_p
    L.rt_free.argtypes = [vp]
    L.rt_free.restype = None
    # batched form
    L.rt_batch_init.argtypes = [ctypes.c_int, ctypes.POINTER(RtGrid), ctypes.POINTER(RtGroups),
                                ctypes.POINTER(RtParams), ctypes.POINTER(vp)]
    L.rt_batch_init.restype = st
    L.rt_batch_scratch_bytes.argtypes = [vp]
    L.rt_batch_scratch_bytes.restype = ctypes.c_size_t
    L.rt_batch_bind.argtypes = [vp, ctypes.POINTER(RtState), vp, ctypes.c_size_t]
    L.rt_batch_bind.restype = st
    L.rt_batch_set_stream.argtypes = [vp, vp]
    L.rt_batch_set_stream.restype = st
    L.rt_batch_current.argtypes = [vp]
    L.rt_batch_current.restype = ctypes.c_int
    L.rt_batch_set_current.argtypes = [vp, ctypes.c_int]
    L.rt_batch_set_current.restype = st
    L.rt_batch_set_sources.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int32), dp]
    L.rt_batch_set_sources.restype = st
    L.rt_batch_courant_dt.argtypes = [vp, ctypes.c_double, dp]
    L.rt_batch_courant_dt.restype = st
    L.rt_batch_step.argtypes = [vp, ctypes.c_double, ctypes.c_int]
    L.rt_batch_step.restype = st
    L.rt_batch_set_tuning.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.rt_batch_set_tuning.restype = st
    L.rt_batch_get_stats.argtypes = [vp, ctypes.POINTER(RtStats)]
    L.rt_batch_get_stats.restype = st
    L.rt_batch_reset_stats.argtypes = [vp]
    L.rt_batch_reset_stats.restype = st
    L.rt_batch_last_error.argtypes = [vp]
    L.rt_batch_last_error.restype = ctypes.c_char_p
    L.rt_batch_free.argtypes = [vp]
    L.rt_batch_free.restype = None
    L.rt_tape_offsets_len.argtypes = [vp]
    L.rt_tape_offsets_len.restype = ctypes.c_size_t
    L.rt_step_record.argtypes = [vp, ctypes.c_double, ctypes.POINTER(RtTape)]
    L.rt_step_record.restype = st
    L.rt_step_replay.argtypes = [vp, ctypes.c_double, ctypes.POINTER(RtTape)]
    L.rt_step_replay.restype = st
    L.rt_step_adjoint.argtypes = [vp, ctypes.c_double, ctypes.POINTER(RtTape), ctypes.POINTER(RtAdj), vp, vp]
    L.rt_step_adjoint.restype = st
    _lib = L
    return L


class RTError(RuntimeError):
    pass


def check(rc, ctx=None):
    if rc != RT_OK:
        msg = lib().rt_last_error(ctx)
        raise RTError(f"rtm1 error {rc}: {msg.decode() if msg else ''}")
    return rc

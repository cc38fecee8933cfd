"""ctypes declarations of the libsco C-ABI (include/sco.h)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsco.so")

SCO_OK, SCO_EINVAL, SCO_EHIP, SCO_EOVERFLOW, SCO_EINTERNAL, SCO_ENOSPC = 0, -1, -2, -3, -4, -5
SCO_ETIMEOUT, SCO_EPALETTE = -6, -7
FLAG_NAMES = {1: "edge overflow", 2: "wait timeout", 4: "palette overflow", 8: "graph state", 16: "KW round cap"}

EXPORTS = [
    "sco_workspace_size", "sco_init", "sco_switch", "sco_color", "sco_sweep", "sco_step", "sco_run",
    "sco_observables", "sco_get_spins", "sco_set_spins", "sco_get_graph", "sco_get_tables",
    "sco_phase_times", "sco_trace", "sco_trace_read", "sco_reset_counters", "sco_destroy",
    "sco_strerror", "sco_set_schedule", "sco_get_schedule", "sco_autotune", "sco_get_flags",
    "sco_counters", "sco_run_noalloc", "sco_run_graph", "sco_set_temperature", "sco_anneal",
    "sco_set_coloring", "sco_get_spins3", "sco_set_spins3", "sco_class_sizes", "sco_bond_histogram",
    "sco_survival_by_distance", "sco_set_round_cap", "sco_set_fenced_sweeps", "sco_set_step_form", "sco_validate",
]


class ChainParamsC(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32), ("periodic", ctypes.c_int32), ("n_images", ctypes.c_int32),
        ("n_sw", ctypes.c_int32),
        ("J", ctypes.c_double), ("D", ctypes.c_double), ("T", ctypes.c_double),
        ("kappa", ctypes.c_double),
        ("seed", ctypes.c_uint32), ("chain_id", ctypes.c_uint32),
        ("precision", ctypes.c_int32), ("edge_factor", ctypes.c_int32),
        ("model", ctypes.c_int32), ("pad", ctypes.c_int32),
    ]


class ObsC(ctypes.Structure):
    _fields_ = [
        ("E", ctypes.c_double), ("E_exchange", ctypes.c_double), ("E_dipolar", ctypes.c_double),
        ("M", ctypes.c_int64), ("n_edges", ctypes.c_int64),
        ("delta_union", ctypes.c_int32), ("q", ctypes.c_int32), ("colors_used", ctypes.c_int32),
        ("kw_levels", ctypes.c_int32),
        ("kw_rounds", ctypes.c_int64), ("accepted", ctypes.c_int64), ("attempts", ctypes.c_int64),
        ("rechecks", ctypes.c_int64), ("flags", ctypes.c_int64), ("near_ties", ctypes.c_int64),
        ("delta_sco", ctypes.c_int32), ("pad", ctypes.c_int32), ("m_phi", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


def flag_names(flags: int) -> str:
    return ", ".join(n for b, n in FLAG_NAMES.items() if flags & b) or "none"


class StageC(ctypes.Structure):
    _fields_ = [
        ("T", ctypes.c_double), ("E", ctypes.c_double), ("M", ctypes.c_int64), ("samples", ctypes.c_int64),
        ("abs_m", ctypes.c_double), ("m2", ctypes.c_double), ("k_mean", ctypes.c_double),
        ("delta_sco_mean", ctypes.c_double), ("delta_union_mean", ctypes.c_double),
        ("acceptance", ctypes.c_double), ("m_phi", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class ScoError(RuntimeError):
    def __init__(self, code: int, what: str, flags: int | None = None):
        self.code = code
        self.flags = flags
        extra = f"; device flags {flags:#x} ({flag_names(flags)})" if flags else ""
        super().__init__(f"{what}: {lib().sco_strerror(code).decode()} ({code}){extra}")


_lib = None


def lib():
    """Loads the HIP library; raises when it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libsco.so not found at {LIB_PATH}: build it with "
                           "`python -m paper_1503_03295_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, u64 = ctypes.c_int, ctypes.c_uint64
    sig = {
        "sco_workspace_size": ([ctypes.POINTER(ChainParamsC), i32, ctypes.POINTER(ctypes.c_size_t)], i32),
        "sco_init": ([ctypes.POINTER(P), ctypes.POINTER(ChainParamsC), i32, P, ctypes.c_size_t, P, P], i32),
        "sco_switch": ([P, u64], i32),
        "sco_color": ([P], i32),
        "sco_sweep": ([P, u64, i32], i32),
        "sco_step": ([P, u64], i32),
        "sco_run": ([P, u64, i32], i32),
        "sco_run_graph": ([P, u64, i32], i32),
        "sco_set_temperature": ([P, i32, ctypes.c_double], i32),
        "sco_set_coloring": ([P, i32], i32),
        "sco_get_spins3": ([P, i32, P], i32),
        "sco_class_sizes": ([P, i32, P, ctypes.POINTER(ctypes.c_int)], i32),
        "sco_bond_histogram": ([P, i32, P], i32),
        "sco_survival_by_distance": ([P, i32, P, P, i32, ctypes.POINTER(ctypes.c_int)], i32),
        "sco_set_round_cap": ([P, i32], i32),
        "sco_set_fenced_sweeps": ([P, i32], i32),
        "sco_set_step_form": ([P, i32], i32),
        "sco_validate": ([P, i32, ctypes.POINTER(ctypes.c_int64)], i32),
        "sco_set_spins3": ([P, i32, P], i32),
        "sco_anneal": ([P, ctypes.POINTER(ctypes.c_double), i32, i32, i32, u64, ctypes.POINTER(StageC)], i32),
        "sco_observables": ([P, ctypes.POINTER(ObsC)], i32),
        "sco_counters": ([P, ctypes.POINTER(ObsC)], i32),
        "sco_run_noalloc": ([ctypes.POINTER(ChainParamsC), i32, P, P, u64, i32, ctypes.POINTER(ObsC), P], i32),
        "sco_get_spins": ([P, i32, P], i32),
        "sco_set_spins": ([P, i32, P], i32),
        "sco_get_graph": ([P, i32, P, P, P, P, ctypes.POINTER(ctypes.c_int64)], i32),
        "sco_get_tables": ([P, i32, ctypes.POINTER(ctypes.c_int32), P, P, P, P, P, P], i32),
        "sco_phase_times": ([P, ctypes.POINTER(ctypes.c_float)], i32),
        "sco_trace": ([P, i32], i32),
        "sco_trace_read": ([P, P, P, i32, ctypes.POINTER(ctypes.c_int)], i32),
        "sco_reset_counters": ([P], i32),
        "sco_destroy": ([P], i32),
        "sco_get_flags": ([P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)], i32),
        "sco_strerror": ([i32], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def check(code: int, what: str, ctx=None) -> None:
    """Raises ScoError for a non-zero code; with a context, the error names the device
    flags of the failed launch."""
    if code != SCO_OK:
        flags = None
        if ctx:
            last = ctypes.c_int64(0)
            if lib().sco_get_flags(ctx, ctypes.byref(last), None) == SCO_OK:
                flags = int(last.value)
        raise ScoError(code, what, flags)

"""Python face of libsco: argument marshalling only.

PyTorch provides the device workspace and the stream; every step of the method
runs in the HIP kernels behind the C-ABI (include/sco.h).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import ChainParamsC, ObsC, StageC, check, lib


@dataclass
class ChainParams:
    """One Markov chain: L x L perpendicular-Ising dipolar lattice (Eq. 6 with
    s_i = +-1 along z), temperature T, V^max = kappa J_ij, n_sw sweeps per step."""
    L: int
    periodic: bool
    T: float
    J: float = 1.0
    D: float = 0.1
    kappa: float = 1.0
    n_images: int = 8
    n_sw: int = 1
    seed: int = 1
    chain_id: int = 0
    precision: int = 0  # 0 FP64, 1 FP32 accumulation + FP64 recheck
    edge_factor: int = 0
    model: int = 0      # 0 perpendicular Ising, 1 Heisenberg with the full dipolar tensor (open)

    def to_c(self) -> ChainParamsC:
        return ChainParamsC(self.L, int(self.periodic), self.n_images, self.n_sw, self.J, self.D,
                            self.T, self.kappa, self.seed & 0xFFFFFFFF, self.chain_id & 0xFFFFFFFF,
                            self.precision, self.edge_factor, self.model, 0)


def workspace_size(params: list[ChainParams]) -> int:
    arr = (ChainParamsC * len(params))(*[p.to_c() for p in params])
    n = ctypes.c_size_t(0)
    check(lib().sco_workspace_size(arr, len(params), ctypes.byref(n)), "sco_workspace_size")
    return int(n.value)


def run_noalloc(params: list[ChainParams], spins_in: torch.Tensor | None, spins_out: torch.Tensor,
                first_step: int, n_steps: int, stream: torch.cuda.Stream | None = None,
                observables: bool = True) -> list[dict] | None:
    """sco_run_noalloc: n_steps steps of the chains with the library's static scratch
    as workspace (no device allocation).  spins_in / spins_out: int8 device tensors of
    the chains' sites concatenated (spins_in None: Philox start)."""
    carr = (ChainParamsC * len(params))(*[p.to_c() for p in params])
    st = stream if stream is not None else torch.cuda.current_stream(spins_out.device)
    obs = (ObsC * len(params))() if observables else None
    ip = ctypes.c_void_p(spins_in.data_ptr()) if spins_in is not None else None
    check(lib().sco_run_noalloc(carr, len(params), ip, ctypes.c_void_p(spins_out.data_ptr()), first_step,
                                n_steps, obs, ctypes.c_void_p(st.cuda_stream)), "sco_run_noalloc")
    return [o.as_dict() for o in obs] if observables else None


class SCO:
    """A batch of independent SCO chains resident on one GPU."""

    def __init__(self, params: list[ChainParams] | ChainParams, device: str | int = "cuda",
                 init_spins: torch.Tensor | None = None, stream: torch.cuda.Stream | None = None):
        if isinstance(params, ChainParams):
            params = [params]
        self.params = list(params)
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("libsco runs on a GPU device")
        self._carr = (ChainParamsC * len(self.params))(*[p.to_c() for p in self.params])
        self.nbytes = workspace_size(self.params)
        self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ip = None
        if init_spins is not None:
            self._init = init_spins.to(device=self.device, dtype=torch.int8).contiguous()
            ip = ctypes.c_void_p(self._init.data_ptr())
        h = ctypes.c_void_p()
        check(lib().sco_init(ctypes.byref(h), self._carr, len(self.params),
                             ctypes.c_void_p(self.workspace.data_ptr()), self.nbytes, ip,
                             ctypes.c_void_p(self.stream.cuda_stream)), "sco_init")
        self._h = h
        self._lib = lib()

    def __del__(self):
        # the library object is held by the instance: at interpreter exit the module
        # globals may already be gone
        h = getattr(self, "_h", None)
        L = getattr(self, "_lib", None)
        if h and L is not None:
            L.sco_destroy(h)
            self._h = None

    def close(self) -> None:
        self.__del__()

    @property
    def n_chains(self) -> int:
        return len(self.params)

    # -- the step
    def switch(self, step: int) -> None:
        check(lib().sco_switch(self._h, step), "sco_switch", self._h)

    def color(self) -> None:
        check(lib().sco_color(self._h), "sco_color", self._h)

    def sweep(self, step: int, n_sw: int) -> None:
        check(lib().sco_sweep(self._h, step, n_sw), "sco_sweep", self._h)

    def step(self, step: int) -> None:
        check(lib().sco_step(self._h, step), "sco_step", self._h)

    def run(self, first_step: int, n_steps: int) -> None:
        check(lib().sco_run(self._h, first_step, n_steps), "sco_run", self._h)

    def run_graph(self, first_step: int, n_steps: int) -> None:
        """The same steps as run(), replayed as one HIP graph of n_steps nodes."""
        check(lib().sco_run_graph(self._h, first_step, n_steps), "sco_run_graph", self._h)

    # -- temperature schedule
    def set_temperature(self, T: float, chain: int = -1) -> None:
        check(lib().sco_set_temperature(self._h, chain, float(T)), "sco_set_temperature", self._h)
        for c in (range(self.n_chains) if chain < 0 else [chain]):
            self.params[c].T = float(T)

    def anneal(self, temps, equil_steps: int, meas_steps: int, first_step: int = 0) -> list[list[dict]]:
        """temps: n_stages x n_chains temperatures (or a 1-D schedule shared by all
        chains); returns per stage the statistics of every chain."""
        t = np.asarray(temps, dtype=np.float64)
        if t.ndim == 1:
            t = np.repeat(t[:, None], self.n_chains, axis=1)
        t = np.ascontiguousarray(t)
        ns = t.shape[0]
        out = (StageC * (ns * self.n_chains))()
        check(lib().sco_anneal(self._h, t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ns, int(equil_steps),
                               int(meas_steps), int(first_step), out), "sco_anneal", self._h)
        for c in range(self.n_chains):
            self.params[c].T = float(t[-1, c]) if ns else self.params[c].T
        return [[out[k * self.n_chains + c].as_dict() for c in range(self.n_chains)] for k in range(ns)]

    # -- results
    def observables(self) -> list[dict]:
        out = (ObsC * self.n_chains)()
        check(lib().sco_observables(self._h, out), "sco_observables", self._h)
        return [o.as_dict() for o in out]

    def counters(self) -> list[dict]:
        """Observables without the dipolar energy (E, E_dipolar NaN), O(N)."""
        out = (ObsC * self.n_chains)()
        check(lib().sco_counters(self._h, out), "sco_counters", self._h)
        return [o.as_dict() for o in out]

    def spins(self, chain: int = 0) -> np.ndarray:
        p = self.params[chain]
        out = np.empty(p.L * p.L, np.int8)
        check(lib().sco_get_spins(self._h, chain, out.ctypes.data_as(ctypes.c_void_p)), "sco_get_spins", self._h)
        return out

    def spins3(self, chain: int = 0) -> np.ndarray:
        """Heisenberg spins of a chain, shape (N, 3)."""
        p = self.params[chain]
        out = np.empty((p.L * p.L, 3), np.float64)
        check(lib().sco_get_spins3(self._h, chain, out.ctypes.data_as(ctypes.c_void_p)), "sco_get_spins3", self._h)
        return out

    def set_spins3(self, chain: int, spins: np.ndarray) -> None:
        p = self.params[chain]
        a = np.ascontiguousarray(spins, dtype=np.float64).reshape(p.L * p.L, 3)
        check(lib().sco_set_spins3(self._h, chain, a.ctypes.data_as(ctypes.c_void_p)), "sco_set_spins3", self._h)

    def set_spins(self, chain: int, spins: np.ndarray) -> None:
        a = np.ascontiguousarray(spins, dtype=np.int8)
        p = self.params[chain]
        if a.size != p.L * p.L:
            raise ValueError("wrong number of spins")
        check(lib().sco_set_spins(self._h, chain, a.ctypes.data_as(ctypes.c_void_p)), "sco_set_spins", self._h)

    def graph(self, chain: int = 0):
        p = self.params[chain]
        N = p.L * p.L
        nd = ctypes.c_int64(0)
        check(lib().sco_get_graph(self._h, chain, None, None, None, None, ctypes.byref(nd)), "sco_get_graph", self._h)
        rp = np.empty(N + 1, np.int32)
        col = np.empty(max(nd.value, 1), np.int32)
        at = np.empty(max(nd.value, 1), np.int32)
        colors = np.empty(N, np.int32)
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        check(lib().sco_get_graph(self._h, chain, ptr(rp), ptr(col), ptr(at), ptr(colors), ctypes.byref(nd)),
              "sco_get_graph", self._h)
        return rp, col[: nd.value], at[: nd.value], colors

    def tables(self, chain: int = 0) -> dict:
        K = ctypes.c_int32(0)
        check(lib().sco_get_tables(self._h, chain, ctypes.byref(K), None, None, None, None, None, None),
              "sco_get_tables", self._h)
        n = K.value
        dx = np.empty(n, np.int32); dy = np.empty(n, np.int32)
        J = np.empty(n); C = np.empty(n); th = np.empty(n); de = np.empty(n)
        ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        check(lib().sco_get_tables(self._h, chain, ctypes.byref(K), ptr(dx), ptr(dy), ptr(J), ptr(C),
                                   ptr(th), ptr(de)), "sco_get_tables", self._h)
        return {"dx": dx, "dy": dy, "J": J, "C": C, "theta": th, "delta": de}

    # -- schedule (never changes results)
    def set_schedule(self, blocks: int = 0, tile_limit: int = 0) -> None:
        check(lib().sco_set_schedule(self._h, int(blocks), int(tile_limit)), "sco_set_schedule", self._h)

    # -- graph statistics, checks and the per-step log
    def class_sizes(self, chain: int = 0) -> np.ndarray:
        """Sites per colour of the current colouring."""
        out = np.zeros(256, np.int64)
        n = ctypes.c_int(0)
        check(lib().sco_class_sizes(self._h, chain, out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n)),
              "sco_class_sizes", self._h)
        return out[: n.value]

    def bond_histogram(self, chain: int = 0) -> np.ndarray:
        """Surviving bonds of the last switching per half-displacement index."""
        K = ctypes.c_int32(0)
        check(lib().sco_get_tables(self._h, chain, ctypes.byref(K), None, None, None, None, None, None),
              "sco_get_tables", self._h)
        out = np.zeros(K.value, np.int64)
        check(lib().sco_bond_histogram(self._h, chain, out.ctypes.data_as(ctypes.c_void_p)),
              "sco_bond_histogram", self._h)
        return out

    def survival_by_distance(self, chain: int = 0):
        """P_survive(r) of the last switching: (r, p) for every distance of the table."""
        K = ctypes.c_int32(0)
        check(lib().sco_get_tables(self._h, chain, ctypes.byref(K), None, None, None, None, None, None),
              "sco_get_tables", self._h)
        r = np.zeros(K.value, np.float64)
        p = np.zeros(K.value, np.float64)
        n = ctypes.c_int(0)
        check(lib().sco_survival_by_distance(self._h, chain, r.ctypes.data_as(ctypes.c_void_p),
                                             p.ctypes.data_as(ctypes.c_void_p), K.value, ctypes.byref(n)),
              "sco_survival_by_distance", self._h)
        return r[: n.value], p[: n.value]

    def set_step_form(self, fused: bool) -> None:
        """One fused launch per step (True) or the three phase launches (False, the
        default); see sco_set_step_form."""
        check(lib().sco_set_step_form(self._h, 1 if fused else 0), "sco_set_step_form", self._h)

    def set_fenced_sweeps(self, on: bool = True) -> None:
        """Full release/acquire barriers between the sweep's colour classes (see
        sco_set_fenced_sweeps); same results, slower."""
        check(lib().sco_set_fenced_sweeps(self._h, 1 if on else 0), "sco_set_fenced_sweeps", self._h)

    def set_round_cap(self, cap: int) -> None:
        check(lib().sco_set_round_cap(self._h, int(cap)), "sco_set_round_cap", self._h)

    def validate(self, chain: int = 0) -> int:
        """Bits of the failed invariant checks (0: all hold); raises on other errors."""
        bad = ctypes.c_int64(0)
        rc = lib().sco_validate(self._h, chain, ctypes.byref(bad))
        if rc not in (_lib.SCO_OK, _lib.SCO_EINTERNAL):
            check(rc, "sco_validate", self._h)
        return int(bad.value)

    def run_logged(self, first_step: int, n_steps: int, path: str) -> None:
        """n_steps steps, one JSON line per step and chain appended to `path`: the step,
        the chain, and its counters (sco_counters: M, exchange energy, bonds, degrees,
        palette, colours used, KW levels and rounds, acceptance, rechecks, near ties,
        flags, M_phi)."""
        import json

        with open(path, "a") as f:
            for t in range(first_step, first_step + n_steps):
                self.step(t)
                for c, o in enumerate(self.counters()):
                    rec = {"step": t, "chain": c}
                    rec.update({k: v for k, v in o.items() if k not in ("E", "E_dipolar", "pad")})
                    f.write(json.dumps(rec) + "\n")

    def set_coloring(self, mode: int) -> None:
        """0 KW rule (2)' (default), 1 checkerboard x KW of the bonds, 2 whole-graph
        basic colour reduction (2)'."""
        check(lib().sco_set_coloring(self._h, int(mode)), "sco_set_coloring", self._h)

    def schedule(self) -> tuple[int, int]:
        b, t = ctypes.c_int(), ctypes.c_int()
        check(lib().sco_get_schedule(self._h, ctypes.byref(b), ctypes.byref(t)), "sco_get_schedule", self._h)
        return b.value, t.value

    def autotune(self, trial_steps: int = 3) -> dict:
        b, t, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_float()
        check(lib().sco_autotune(self._h, int(trial_steps), ctypes.byref(b), ctypes.byref(t), ctypes.byref(ms)),
              "sco_autotune", self._h)
        return {"blocks": b.value, "tile_limit": t.value, "ms_per_step": ms.value}

    def phase_times(self) -> tuple[float, float, float]:
        out = (ctypes.c_float * 3)()
        check(lib().sco_phase_times(self._h, out), "sco_phase_times", self._h)
        return tuple(out)

    def trace(self, enable: bool = True) -> None:
        check(lib().sco_trace(self._h, int(enable)), "sco_trace", self._h)

    def trace_read(self) -> list[tuple[int, float]]:
        n = ctypes.c_int(0)
        ids = np.zeros(256, np.int32)
        us = np.zeros(256)
        check(lib().sco_trace_read(self._h, ids.ctypes.data_as(ctypes.c_void_p),
                                   us.ctypes.data_as(ctypes.c_void_p), 256, ctypes.byref(n)),
              "sco_trace_read", self._h)
        k = min(n.value, 256)
        return list(zip(ids[:k].tolist(), us[:k].tolist()))

    def reset_counters(self) -> None:
        check(lib().sco_reset_counters(self._h), "sco_reset_counters", self._h)

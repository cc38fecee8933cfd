"""CPU oracle of the stochastic-cutoff (SCO) step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_1503_03295_amd``) and never imports it.

The arithmetic lives in ``sco_oracle.c`` (plain serial C, FP64, built with
``-ffp-contract=off``); this module only marshals arguments, plus one extra route
for the dipolar energy of large periodic lattices: the per-displacement spin
autocorrelations C(d) = sum_i s_i s_{i+d} from a numpy FFT, rounded to the exact
integers they are (|C| <= N, FFT error far below 1/2), then the same sum
sum_m J_m C_m over the half-displacement table as the direct route.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sco_oracle.c")
_LIB = os.path.join(_HERE, "libscooracle.so")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (a plain C shared library)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32), ("periodic", ctypes.c_int32), ("n_images", ctypes.c_int32),
        ("n_sw", ctypes.c_int32),
        ("J", ctypes.c_double), ("D", ctypes.c_double), ("T", ctypes.c_double),
        ("kappa", ctypes.c_double),
        ("seed", ctypes.c_uint32), ("chain_id", ctypes.c_uint32),
        ("coloring", ctypes.c_int32), ("model", ctypes.c_int32),
    ]


class Obs(ctypes.Structure):
    _fields_ = [
        ("E", ctypes.c_double), ("E_exchange", ctypes.c_double), ("E_dipolar", ctypes.c_double),
        ("M", ctypes.c_int64), ("n_edges", ctypes.c_int64),
        ("delta_union", ctypes.c_int32), ("q", ctypes.c_int32), ("colors_used", ctypes.c_int32),
        ("kw_levels", ctypes.c_int32),
        ("kw_rounds", ctypes.c_int64), ("accepted", ctypes.c_int64), ("attempts", ctypes.c_int64),
        ("near_ties", ctypes.c_int64), ("delta_sco", ctypes.c_int32), ("pad", ctypes.c_int32),
        ("m_phi", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.orc_philox.argtypes = [u32p, u32p, u32p]
        L.orc_philox.restype = None
        L.orc_u52.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        L.orc_u52.restype = ctypes.c_double
        L.orc_create.argtypes = [ctypes.POINTER(Params), P]
        L.orc_create.restype = P
        L.orc_destroy.argtypes = [P]
        L.orc_destroy.restype = None
        for name in ("orc_switch", "orc_step"):
            getattr(L, name).argtypes = [P, ctypes.c_uint64]
            getattr(L, name).restype = ctypes.c_int
        L.orc_color.argtypes = [P]
        L.orc_color.restype = ctypes.c_int
        L.orc_sweep.argtypes = [P, ctypes.c_uint64, ctypes.c_int]
        L.orc_sweep.restype = ctypes.c_int
        L.orc_observables.argtypes = [P, ctypes.POINTER(Obs), ctypes.c_int]
        L.orc_observables.restype = None
        L.orc_N.argtypes = [P]; L.orc_N.restype = ctypes.c_int
        L.orc_K.argtypes = [P]; L.orc_K.restype = ctypes.c_int
        L.orc_n_edges.argtypes = [P]; L.orc_n_edges.restype = ctypes.c_int64
        L.orc_get_spins.argtypes = [P, P]; L.orc_get_spins.restype = None
        L.orc_set_spins.argtypes = [P, P]; L.orc_set_spins.restype = None
        L.orc_get_tables.argtypes = [P] + [P] * 6; L.orc_get_tables.restype = None
        L.orc_get_survivors.argtypes = [P, P, P, P]; L.orc_get_survivors.restype = None
        L.orc_get_csr.argtypes = [P, P, P, P]; L.orc_get_csr.restype = None
        L.orc_get_colors.argtypes = [P, P]; L.orc_get_colors.restype = None
        L.orc_get_kw_rounds.argtypes = [P, P]; L.orc_get_kw_rounds.restype = None
        L.orc_partner.argtypes = [P, ctypes.c_int, ctypes.c_int]; L.orc_partner.restype = ctypes.c_int
        L.orc_reset_counters.argtypes = [P]; L.orc_reset_counters.restype = None
        L.orc_ties.argtypes = [P, P, P, ctypes.c_int]; L.orc_ties.restype = ctypes.c_int
        L.orc_set_temperature.argtypes = [P, ctypes.c_double]; L.orc_set_temperature.restype = ctypes.c_int
        L.orc_get_spins3.argtypes = [P, P]; L.orc_get_spins3.restype = None
        L.orc_set_spins3.argtypes = [P, P]; L.orc_set_spins3.restype = None
        L.orc_pair_energy.argtypes = [P, P, ctypes.c_int, ctypes.c_int, ctypes.c_double]
        L.orc_pair_energy.restype = ctypes.c_double
        L.orc_sphere_point.argtypes = [P] + [ctypes.c_uint32] * 4 + [P]
        L.orc_sphere_point.restype = ctypes.c_int
        for name in ("orc_color_rule2", "orc_color_whole_rule2"):
            getattr(L, name).argtypes = [P, P, ctypes.POINTER(ctypes.c_int64)]
            getattr(L, name).restype = ctypes.c_int
        L.orc_survival_counts.argtypes = [P, ctypes.c_uint64, ctypes.c_int, P]
        L.orc_survival_counts.restype = None
        L.orc_run_record.argtypes = [P, ctypes.c_uint64, ctypes.c_int, ctypes.c_int, P, P]
        L.orc_run_record.restype = ctypes.c_uint64
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox4x32_10(ctr, key) -> tuple:
    """Philox4x32-10 block function (Salmon et al., SC'11)."""
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox(c, k, o)
    return tuple(o)


def u52(lo: int, hi: int) -> float:
    return lib().orc_u52(lo & 0xFFFFFFFF, hi & 0xFFFFFFFF)


@dataclass
class ChainParams:
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
    coloring: int = 0  # 0 KW (2)', 1 checkerboard x KW of the bonds, 2 whole-graph BCR (2)'
    model: int = 0     # 0 perpendicular Ising, 1 Heisenberg with the full dipolar tensor

    def to_c(self) -> Params:
        return Params(self.L, int(self.periodic), self.n_images, self.n_sw, self.J, self.D,
                      self.T, self.kappa, self.seed & 0xFFFFFFFF, self.chain_id & 0xFFFFFFFF,
                      int(self.coloring), int(self.model))


class OracleChain:
    """One SCO Markov chain run by the serial oracle."""

    def __init__(self, params: ChainParams, init_spins: np.ndarray | None = None):
        self.params = params
        self._p = params.to_c()
        ip = None
        if init_spins is not None:
            self._init = np.ascontiguousarray(init_spins, dtype=np.int8)
            ip = _ptr(self._init)
        h = lib().orc_create(ctypes.byref(self._p), ip)
        if not h:
            raise ValueError(f"oracle rejected parameters {params}")
        self._h = h
        self.N = lib().orc_N(h)
        self.K = lib().orc_K(h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    # -- steps
    def switch(self, t: int) -> None:
        lib().orc_switch(self._h, t)

    def color(self) -> None:
        if lib().orc_color(self._h) != 0:
            raise RuntimeError("colouring ran out of colours (invariant violated)")

    def sweep(self, t: int, n_sw: int | None = None) -> None:
        lib().orc_sweep(self._h, t, self.params.n_sw if n_sw is None else n_sw)

    def step(self, t: int) -> None:
        if lib().orc_step(self._h, t) != 0:
            raise RuntimeError("oracle step failed")

    # -- state
    @property
    def spins(self) -> np.ndarray:
        out = np.empty(self.N, np.int8)
        lib().orc_get_spins(self._h, _ptr(out))
        return out

    @spins.setter
    def spins(self, s: np.ndarray) -> None:
        a = np.ascontiguousarray(s, dtype=np.int8)
        lib().orc_set_spins(self._h, _ptr(a))

    @property
    def spins3(self) -> np.ndarray:
        """Heisenberg spins, shape (N, 3)."""
        out = np.empty((self.N, 3), np.float64)
        lib().orc_get_spins3(self._h, _ptr(out))
        return out

    @spins3.setter
    def spins3(self, s: np.ndarray) -> None:
        a = np.ascontiguousarray(s, dtype=np.float64).reshape(self.N, 3)
        lib().orc_set_spins3(self._h, _ptr(a))

    def sphere_point(self, c0: int, c1: int, c2: int, tag: int):
        out = np.empty(3, np.float64)
        ok = lib().orc_sphere_point(self._h, c0, c1, c2, tag, _ptr(out))
        return out if ok else None

    def tables(self) -> dict:
        K = self.K
        dx = np.empty(K, np.int32); dy = np.empty(K, np.int32)
        J = np.empty(K); C = np.empty(K); th = np.empty(K); de = np.empty(K)
        lib().orc_get_tables(self._h, _ptr(dx), _ptr(dy), _ptr(J), _ptr(C), _ptr(th), _ptr(de))
        return {"dx": dx, "dy": dy, "J": J, "C": C, "theta": th, "delta": de}

    def survivors(self):
        E = lib().orc_n_edges(self._h)
        o = np.empty(E, np.int32); n = np.empty(E, np.int32); m = np.empty(E, np.int32)
        if E:
            lib().orc_get_survivors(self._h, _ptr(o), _ptr(n), _ptr(m))
        return o, n, m

    def csr(self):
        E = lib().orc_n_edges(self._h)
        rp = np.empty(self.N + 1, np.int32)
        col = np.empty(max(2 * E, 1), np.int32); at = np.empty(max(2 * E, 1), np.int32)
        lib().orc_get_csr(self._h, _ptr(rp), _ptr(col), _ptr(at))
        return rp, col[: 2 * E], at[: 2 * E]

    def colors(self) -> np.ndarray:
        out = np.empty(self.N, np.int32)
        lib().orc_get_colors(self._h, _ptr(out))
        return out

    def kw_rounds(self) -> np.ndarray:
        out = np.empty(64, np.int32)
        lib().orc_get_kw_rounds(self._h, _ptr(out))
        return out

    def partner(self, i: int, m: int) -> int:
        return lib().orc_partner(self._h, i, m)

    def reset_counters(self) -> None:
        lib().orc_reset_counters(self._h)

    def ties(self) -> list[tuple[int, int]]:
        """The near-tie decisions since the last switching as (kind, site): kind 1 a
        switching decision of owner `site`, kind 2 a sweep decision of `site` (the first
        256 are listed; a longer list raises)."""
        kinds = np.zeros(256, np.int32)
        sites = np.zeros(256, np.int32)
        n = lib().orc_ties(self._h, _ptr(kinds), _ptr(sites), 256)
        if n > 256:
            raise RuntimeError(f"{n} near ties in one step")
        return list(zip(kinds[:n].tolist(), sites[:n].tolist()))

    def colors_rule2(self, whole: bool = False):
        """The colouring with the basic step (2) instead of rule (2)': in every KW level,
        or on the whole graph from the N-colouring (small lattices); (colours, rounds)."""
        out = np.empty(self.N, np.int32)
        r = ctypes.c_int64(0)
        f = lib().orc_color_whole_rule2 if whole else lib().orc_color_rule2
        if f(self._h, _ptr(out), ctypes.byref(r)) != 0:
            raise RuntimeError("colouring ran out of colours")
        return out, int(r.value)

    def set_temperature(self, T: float) -> None:
        if lib().orc_set_temperature(self._h, float(T)) != 0:
            raise ValueError(f"invalid temperature {T}")
        self.params.T = float(T)
        self._p.T = float(T)


    def observables(self, dipolar: str = "auto") -> dict:
        """dipolar: 'direct' (pair sum in C), 'fft' (periodic only), 'none' or 'auto'."""
        if dipolar == "auto":
            dipolar = "direct" if self.N * self.K <= 5e8 or not self.params.periodic else "fft"
        o = Obs()
        lib().orc_observables(self._h, ctypes.byref(o), 1 if dipolar == "direct" else 0)
        d = o.as_dict()
        if dipolar == "fft":
            d["E_dipolar"] = dipolar_energy_fft(self.spins, self.params.L, self.tables())
            d["E"] = d["E_exchange"] + d["E_dipolar"]
        elif dipolar == "none":
            d["E_dipolar"] = float("nan")
            d["E"] = float("nan")
        return d

    def survival_counts(self, t0: int, n_steps: int) -> np.ndarray:
        counts = np.zeros(self.N * self.K, np.int32)
        lib().orc_survival_counts(self._h, t0, n_steps, _ptr(counts))
        return counts.reshape(self.N, self.K)

    def run_record(self, t0: int, n_steps: int, thin: int):
        n = n_steps // thin if thin > 0 else 0
        E = np.empty(max(n, 1)); M = np.empty(max(n, 1), np.int64)
        t = lib().orc_run_record(self._h, t0, n_steps, thin, _ptr(E), _ptr(M))
        return int(t), E[:n], M[:n]


def pair_energy(si, sj, dx: int, dy: int, Jm: float) -> float:
    """The oracle's dipolar pair energy of Eq. (6) (Jm = V^max = 2 D / r^3)."""
    a = np.ascontiguousarray(si, dtype=np.float64)
    b = np.ascontiguousarray(sj, dtype=np.float64)
    return lib().orc_pair_energy(_ptr(a), _ptr(b), int(dx), int(dy), float(Jm))


def autocorrelation_periodic(spins: np.ndarray, L: int) -> np.ndarray:
    """C[dy, dx] = sum_{x,y} s(x,y) s(x+dx, y+dy) (indices mod L), exact integers."""
    s = spins.reshape(L, L).astype(np.float64)
    f = np.fft.rfft2(s)
    c = np.fft.irfft2(f.conj() * f, s=(L, L))
    r = np.rint(c)
    if np.max(np.abs(c - r)) > 0.25:
        raise ArithmeticError("FFT autocorrelation not close enough to integers")
    return r.astype(np.int64)


def dipolar_energy_fft(spins: np.ndarray, L: int, tables: dict) -> float:
    """sum_m J_m C_m over the half-displacement table (periodic lattice), C_m the
    owned-pair correlation: the full autocorrelation, halved for the three
    self-conjugate displacements whose pairs it counts twice."""
    C = autocorrelation_periodic(spins, L)
    dx, dy, J = tables["dx"], tables["dy"], tables["J"]
    cm = C[dy % L, dx % L]
    h = L // 2
    sc = ((dx == h) & (dy == 0)) | ((dy == h) & ((dx == 0) | (dx == h)))
    cm = np.where(sc, cm // 2, cm)
    acc = 0.0
    for j, c in zip(J.tolist(), cm.tolist()):  # sequential, table order
        acc += j * float(c)
    return acc


def anneal(chain: OracleChain, temps, equil_steps: int, meas_steps: int, first_step: int = 0) -> list[dict]:
    """The cooling protocol of Sec. 3.1 run by the oracle: per temperature, equil_steps
    SCO steps, then meas_steps steps whose |M|, M^2, bond count and maximum degrees are
    summed as exact integers; returns the per-stage means (divided in the order
    sum / samples / N) and the state at the end of each stage."""
    out = []
    t = first_step
    N = float(chain.N)
    for T in temps:
        chain.set_temperature(T)
        acc0 = chain.observables(dipolar="none")
        for _ in range(equil_steps):
            chain.step(t)
            t += 1
        s_abs = s_m2 = s_b = s_ds = s_du = 0
        for _ in range(meas_steps):
            chain.step(t)
            t += 1
            o = chain.observables(dipolar="none")
            m = abs(int(o["M"]))
            s_abs += m
            s_m2 += m * m
            s_b += 2 * int(o["n_edges"])
            s_ds += int(o["delta_sco"])
            s_du += int(o["delta_union"])
        o = chain.observables()
        ns = float(meas_steps)
        att = o["attempts"] - acc0["attempts"]
        if chain.params.model == 1:  # the magnetisation is an Ising sum
            s_abs = s_m2 = 0
        out.append(dict(
            T=float(T), E=o["E"], M=int(o["M"]), samples=meas_steps,
            abs_m=(float(s_abs) / ns / N) if meas_steps else 0.0,
            m2=(float(s_m2) / ns / (N * N)) if meas_steps else 0.0,
            k_mean=(float(s_b) / ns / N) if meas_steps else 0.0,
            delta_sco_mean=(float(s_ds) / ns) if meas_steps else 0.0,
            delta_union_mean=(float(s_du) / ns) if meas_steps else 0.0,
            acceptance=(float(o["accepted"] - acc0["accepted"]) / att) if att else 0.0,
            m_phi=o["m_phi"],
            spins=chain.spins3 if chain.params.model == 1 else chain.spins))
    return out

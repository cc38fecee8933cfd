#!/usr/bin/env python
"""Throughput of the stochastic-cutoff (SCO) step on one MI355X.

A step is one full pass of the method over the chain: switching of every dipolar
bond + bond-graph assembly (k_step<1u>), Kuhn-Wattenhofer colouring + colour
bucketing (k_step<2u>), and n_sw colour-ordered Metropolis sweeps (k_step<4u>), three
persistent cooperative launches.  `value` = spin-update attempts per second over the
timed steps (N * n_sw per step), the steps replayed as one HIP graph, inputs resident
in HBM, HIP events on the library's stream.  `roofline` puts the dominant kernel's
algorithmic bytes per launch (the colouring's) over its mean launch duration on the
same steps against the HBM peak; `roofline.step` does the same for the whole step.
Extra legs: n_sw = 100, the 64-chain batch, the 9-chain mixed-precision workload
(FP64 vs FP32 + recheck), the annealing schedule, the colouring variants and the
paper's Heisenberg model at L = 2304.  The CPU oracle is timed on a short sample of
the same chain (one host thread).

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "spin-update attempts/s per GPU at L=2304 (incl. switch+color); HBM GB/s % peak"
HBM_PEAK_GBS = 8000.0


def progress(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def expected_candidates(J, T, kappa):
    """mean number of candidate bonds per owner: sum_m 1 - exp(-(kappa+1) J_m / T)"""
    import numpy as np

    return float(np.sum(-np.expm1(-(kappa + 1.0) * J / T)))


def phase_bytes(N, E, c, M, P, k_mean, hard, n_sw, accept):
    """Algorithmic bytes of one step, per phase: the data each phase must move once
    (the displacement-table probes are cache-resident and not counted).
      switch    per owner: its spin (1) + the partner spin of each candidate (c) +
                its survivor count (4)
      assembly  per site: degree scan read + write (8); per survivor s = E/N:
                both directions (2 x 8) + the partner count (4) + row sort read/write (16)
      colour    per pending site and level run over the whole lattice (M - P levels,
                N/2 pending each): row_ptr (4) + bond partners (4k) + neighbour
                words (4 + k) + the decision (2); the P levels held in LDS count once
      sweep     per attempt: list entry (4) + own spin (1) + NN spins (4) + row_ptr (4)
                + per bond: partner (4) + coupling (8 FP64, 4 FP32 when hard: 0) +
                partner spin (1) + the accepted write (acceptance a)"""
    s = E / N
    switch = N * (1 + c + 4)
    assembly = N * (8 + s * (16 + 4 + 16))
    per_pending = 4 + 4 * k_mean + (4 + k_mean) + 2
    colour = max(M - P, 0) * (N / 2) * per_pending + N * per_pending
    per_attempt = 4 + 1 + 4 + 4 + (0.0 if hard else k_mean * (4 + 8 + 1)) + accept
    sweep = N * n_sw * per_attempt
    return {"switch": switch + assembly, "color": colour, "sweep": sweep}


def kernel_source_hash():
    """sha256 of the kernel sources with comments and blank lines removed (edits to
    comments do not change the kernel)."""
    import hashlib
    import re

    csrc = os.path.join(ROOT, "paper_1503_03295_amd", "csrc")
    text = ""
    for name in ("sco_kernels.hip", "sco_internal.h"):
        src = open(os.path.join(csrc, name)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        lines = (re.sub(r"//.*$", "", line).strip() for line in src.splitlines())
        text += "\n".join(line for line in lines if line) + "\n"
    return hashlib.sha256(text.encode()).hexdigest()


def measured_traffic():
    """HBM bytes per launch of the dominant kernel (the colouring, k_step<2u>) from the
    committed rocprofv3 --pmc summary, or
    None when the kernel sources have changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "k_step_L2304_traffic.md")
    try:
        text = open(path).read()
        h = kernel_source_hash()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines()
                  if line.startswith(("traffic_bytes_per_launch: ", "source_sha256: ")))
    if fields.get("source_sha256", "").strip() != h:
        return None
    return float(fields["traffic_bytes_per_launch"])


def time_steps(sco, first, steps, torch, graph=True):
    """ms per step of `steps` full steps (HIP events on the library's stream), as one
    HIP-graph replay (graph) or as plain launches."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(sco.stream)
    (sco.run_graph if graph else sco.run)(first, steps)
    e1.record(sco.stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def time_both(sco, first, steps, torch, np, phases=False):
    """The same steps from the same spins as plain launches and as one HIP-graph
    replay: (ms graph, ms plain, final spins identical, per-phase ms).  With `phases`
    the steps run a third time as the three phase launches one call at a time, each
    timed by HIP events on the library's stream (the mean launch duration of each
    phase kernel over the timed steps).  The counters left are the graph run's."""
    n = sco.n_chains
    start = [sco.spins(c) for c in range(n)]
    phase_ms = None
    if phases:
        acc = np.zeros(3)
        for t in range(first, first + steps):
            sco.switch(t)
            sco.color()
            sco.sweep(t, max(p.n_sw for p in sco.params))
            acc += np.array(sco.phase_times())
        phase_ms = acc / steps
        for c in range(n):
            sco.set_spins(c, start[c])
    ms_plain = time_steps(sco, first, steps, torch, graph=False)
    after_plain = [sco.spins(c) for c in range(n)]
    for c in range(n):
        sco.set_spins(c, start[c])
    sco.reset_counters()
    ms_graph = time_steps(sco, first, steps, torch, graph=True)
    same = all(np.array_equal(sco.spins(c), after_plain[c]) for c in range(n))
    return ms_graph, ms_plain, same, phase_ms


def host_cpu():
    """The host's logical CPUs and CPU model (for the oracle's timing)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "model": model}


def anneal_leg(torch, SCO, ChainParams, L=512):
    """The cooling protocol of Sec. 3.1: 1.25 -> 0.05 in steps of 0.05, n_sw = 100, one
    equilibration and one measured step per temperature, one chain."""
    import workloads

    temps = [round(1.25 - 0.05 * k, 10) for k in range(25)]
    p = dict(workloads.chain(L, True, temps[0], 1.0, n_sw=100), edge_factor=32)
    sco = SCO([ChainParams(**p)], device="cuda:0")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(sco.stream)
    stages = sco.anneal(temps, 1, 1)
    e1.record(sco.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    steps = 2 * len(temps)
    pick = {f"{s[0]['T']:.2f}": {k: s[0][k] for k in ("k_mean", "delta_sco_mean", "delta_union_mean", "abs_m",
                                                       "acceptance")}
            for s in stages if round(s[0]["T"], 2) in (1.25, 0.45, 0.05)}
    sco.close()
    out = {"L": L, "stages": len(temps), "steps": steps, "n_sw": 100, "ms_total": ms,
           "attempts_per_s": L * L * 100 * steps / (ms / 1e3), "table1_like": pick}
    progress(f"anneal L={L}: {ms:.1f} ms for {steps} steps; {pick}")
    return out


def heisenberg_leg(torch, SCO, ChainParams, L=2304, T=1.25, n_sw=100, warm=3, steps=3):
    """The paper's own model (Eq. 6, Heisenberg spins, full dipolar tensor, open
    boundaries) at its size and n_sw: SCO steps timed after a few warm-up steps, with
    the switched graph's mean and maximum degree (Table 1's <k> and <Delta>; the paper
    quotes 1.40 and 8.54 at T = 1.25 for equilibrated chains)."""
    import workloads

    p = dict(workloads.chain(L, False, T, 1.0, n_sw=n_sw), model=1, edge_factor=16)
    sco = SCO([ChainParams(**p)], device="cuda:0")
    sco.run(0, warm)
    ms = time_steps(sco, warm, steps, torch)
    t = warm + steps
    sco.switch(t)
    sco.color()
    sco.sweep(t, n_sw)
    ph = sco.phase_times()
    o = sco.counters()[0]
    t_obs = time.perf_counter()
    full = sco.observables()[0]  # the full dipolar tensor energy by FFT correlations
    t_obs = time.perf_counter() - t_obs
    N = L * L
    out = {"L": L, "T": T, "n_sw": n_sw, "steps": steps, "ms_per_step": ms,
           "attempts_per_s": N * n_sw / (ms / 1e3),
           "phase_ms": {"switch": ph[0], "color": ph[1], "sweep": ph[2]},
           "k_mean": 2.0 * o["n_edges"] / N, "delta_sco": o["delta_sco"], "q": o["q"],
           "acceptance": o["accepted"] / max(1, o["attempts"]),
           "E_per_site": full["E"] / N, "E_dipolar_per_site": full["E_dipolar"] / N, "m_phi": full["m_phi"],
           "observables_ms": 1e3 * t_obs}
    progress(f"heisenberg L={L} T={T}: {ms:.2f} ms/step, {out['attempts_per_s']:.4g} attempts/s, "
             f"<k> {out['k_mean']:.3f}, Delta {o['delta_sco']}, E/N {out['E_per_site']:.6f}, "
             f"M_phi {out['m_phi']:.3g} ({out['observables_ms']:.1f} ms)")
    sco.close()
    return out


def coloring_leg(torch, SCO, ChainParams, params, steps=3):
    """The colouring variants on the headline chain: KW rule (2)', the checkerboard
    product of a KW colouring of the bonds, and whole-graph basic colour reduction."""
    out = {}
    for mode, name in ((0, "kw"), (1, "checkerboard_product"), (2, "whole_graph_bcr")):
        sco = SCO([ChainParams(**params)], device="cuda:0")
        sco.set_coloring(mode)
        # the whole-graph reduction takes of the order of a million rounds at L = 2304:
        # one timed step, no warm-up
        warm, n = (2, steps) if mode != 2 else (0, 1)
        sco.run(0, warm)
        ms = time_steps(sco, warm, n, torch)
        t = warm + n
        sco.switch(t)
        sco.color()
        sco.sweep(t, params["n_sw"])
        ph = sco.phase_times()
        o = sco.counters()[0]
        out[name] = {"ms_per_step": ms, "phase_ms": {"switch": ph[0], "color": ph[1], "sweep": ph[2]},
                     "kw_levels": o["kw_levels"], "kw_rounds": o["kw_rounds"], "q": o["q"],
                     "colors_used": o["colors_used"]}
        if mode == 0:
            out[name]["rounds_rule2_eq5"] = o["q"] * o["kw_levels"]
        progress(f"colouring {name}: {ms:.3f} ms/step, colour {ph[1]:.3f} ms, rounds {o['kw_rounds']}")
        sco.close()
    return out


def workload_leg(name, params, steps, torch, SCO, ChainParams, autotune=True):
    """One extra workload: spins, attempts/s and the chosen schedule."""
    sco = SCO([ChainParams(**p) for p in params], device="cuda:0")
    sched = sco.autotune(2) if autotune else None
    sco.run(0, 2)
    import numpy as np

    ms, ms_plain, same, _ = time_both(sco, 2, steps, torch, np)
    obs = sco.observables()
    spins = sum(p["L"] ** 2 for p in params)
    attempts = sum(p["L"] ** 2 * p["n_sw"] for p in params)
    out = {"chains": len(params), "spins": spins, "steps": steps, "ms_per_step": ms, "ms_per_step_plain": ms_plain,
           "graph_equals_plain": same,
           "attempts_per_s": attempts / (ms / 1e3), "schedule": sched,
           "rechecks": int(sum(o["rechecks"] for o in obs)),
           "attempts_total": int(sum(o["attempts"] for o in obs))}
    spins_out = [sco.spins(c) for c in range(len(params))]
    sco.close()
    progress(f"{name}: {ms:.3f} ms/step, {out['attempts_per_s']:.4g} attempts/s, schedule {sched}")
    return out, spins_out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n-sw", type=int, default=1)
    ap.add_argument("--kappa", type=float, default=1.0)
    ap.add_argument("--phase-steps", type=int, default=5)
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-nsw100", action="store_true")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the batched, mixed-precision, annealing and colouring legs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported (the SCO step "
              "runs on a single MI355X; multi-GPU sharding is not implemented)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import workloads
    from paper_1503_03295_amd import SCO, ChainParams

    params, _ = workloads.large_periodic(kappa=args.kappa, n_sw=args.n_sw)
    p = params[0]
    N = p["L"] * p["L"]
    progress(f"init L={p['L']} T={p['T']} kappa={p['kappa']} n_sw={p['n_sw']}")
    sco = SCO([ChainParams(**p)], device="cuda:0")
    sched = sco.autotune(3)
    progress(f"autotuned schedule: {sched}")

    for t in range(args.warmup):
        sco.step(t)
    torch.cuda.synchronize()
    progress(f"warmup {args.warmup} steps done")

    first = args.warmup
    # the timed steps as plain launches, then the same steps from the same spins as
    # one HIP-graph replay; `value` is the graph replay's
    ms_per_step, ms_plain, graph_same, timed_phase_ms = time_both(sco, first, args.steps, torch, np, phases=True)
    value = N * p["n_sw"] / (ms_per_step / 1e3)
    obs = sco.observables()[0]
    progress(f"timed {args.steps} steps: graph {ms_per_step:.3f} ms/step ({value:.4g} attempts/s), "
             f"plain launches {ms_plain:.3f} ms/step, same spins {graph_same}")

    # one traced step: block 0's phase marks inside the persistent kernel
    sco.trace(True)
    sco.step(first + args.steps)
    marks = sco.trace_read()
    sco.trace(False)
    trace = [(i, round(t, 2)) for i, t in marks]

    # per-phase times: the three phases as separate launches (k_step<1>, <2>, <4>)
    t0 = first + args.steps + 1
    acc = np.zeros(3)
    stats = []
    for s in range(args.phase_steps):
        sco.switch(t0 + s)
        sco.color()
        sco.sweep(t0 + s, p["n_sw"])
        acc += np.array(sco.phase_times())
        o = sco.observables()[0]
        stats.append((o["n_edges"], o["q"], o["kw_levels"], o["kw_rounds"], o["accepted"], o["attempts"]))
    phase_ms = acc / args.phase_steps
    E = float(np.mean([s[0] for s in stats]))
    q = float(np.mean([s[1] for s in stats]))
    M = float(np.mean([s[2] for s in stats]))
    accept = (stats[-1][4] - stats[0][4]) / max(1, stats[-1][5] - stats[0][5])
    tables = sco.tables(0)
    c = expected_candidates(tables["J"], p["T"], p["kappa"])
    k_mean = 2.0 * E / N
    tile = sched["tile_limit"]
    P = int(np.floor(np.log2(tile / q))) if q > 0 else 0
    pb = phase_bytes(N, E, c, M, P, k_mean, p["kappa"] == 1.0, p["n_sw"], accept)
    names = ["switch", "color", "sweep"]
    step_bytes = sum(pb.values())
    # the dominant kernel of the step: the colouring launch, its algorithmic bytes over
    # its mean launch duration on the timed steps
    achieved = pb["color"] / (timed_phase_ms[1] / 1e3) / 1e9
    progress("phase ms: " + ", ".join(f"{n}={t:.3f}" for n, t in zip(names, phase_ms)))

    extra = {}
    if not args.no_nsw100 and p["n_sw"] == 1:
        sco100 = SCO([ChainParams(**{**p, "n_sw": 100})], device="cuda:0")
        sco100.set_schedule(*[sched["blocks"], sched["tile_limit"]])
        sco100.run(0, 1)
        ms100 = time_steps(sco100, 1, 3, torch)
        o100 = sco100.counters()[0]  # raises if a step flagged an error
        extra["n_sw_100"] = {"ms_per_step": ms100, "value": N * 100 / (ms100 / 1e3),
                             "attempts": o100["attempts"], "flags": o100["flags"]}
        progress(f"n_sw=100: {ms100:.3f} ms/step")
        sco100.close()
    if not args.no_workloads:
        legs = {}
        bp = workloads.batched()
        legs["batched_64"], _ = workload_leg("batched 64 chains", bp, 10, torch, SCO, ChainParams)
        for kappa in (1.0, 2.0):
            mp0 = workloads.mixed_precision(precision=0, kappa=kappa)
            mp1 = workloads.mixed_precision(precision=1, kappa=kappa)
            r0, s0 = workload_leg(f"8xL2304+L4096 fp64 kappa={kappa}", mp0, 5, torch, SCO, ChainParams)
            r1, s1 = workload_leg(f"8xL2304+L4096 fp32+recheck kappa={kappa}", mp1, 5, torch, SCO, ChainParams)
            same = all(np.array_equal(x, y) for x, y in zip(s0, s1))
            legs[f"mixed_9_chains_kappa{kappa:g}"] = {"fp64": r0, "fp32_recheck": r1,
                                                     "identical_spins": bool(same),
                                                     "speedup": r0["ms_per_step"] / r1["ms_per_step"]}
        extra["workloads"] = legs
        extra["anneal"] = anneal_leg(torch, SCO, ChainParams)
        extra["coloring_variants"] = coloring_leg(torch, SCO, ChainParams, p)
        extra["heisenberg"] = heisenberg_leg(torch, SCO, ChainParams)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        progress(f"cpu baseline: oracle, {args.cpu_steps} steps")
        keys = ("L", "periodic", "T", "J", "D", "kappa", "n_images", "n_sw", "seed", "chain_id")
        ref = oracle.OracleChain(oracle.ChainParams(**{k: p[k] for k in keys}))
        c0 = time.perf_counter()
        for t in range(args.cpu_steps):
            ref.step(t)
        dt = time.perf_counter() - c0
        cpu = {"value": N * p["n_sw"] * args.cpu_steps / dt, "unit": "attempts/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{args.cpu_steps} SCO steps (switch+colour+{p['n_sw']} sweep) of the same "
                         f"L={p['L']} chain from its initial spins, single host thread, "
                         f"{dt:.1f} s",
               "host": host_cpu()}
        progress(f"cpu baseline {cpu['value']:.4g} attempts/s")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "ms_per_step_plain_launches": ms_plain,
        "graph_equals_plain_launches": graph_same,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"SCO step, L={p['L']} periodic square lattice (N={N}), perpendicular Ising "
                        f"dipolar, J=1, D=0.1, image sum |n|<=8, T={p['T']}, kappa={p['kappa']}, "
                        f"n_sw={p['n_sw']}, single chain, FP64, Philox seed 1",
            "L": p["L"], "N": N, "T": p["T"], "kappa": p["kappa"], "n_sw": p["n_sw"], "chains": 1,
            "precision": "fp64",
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
            "kernel": "k_step<2u, 0>", "algorithmic_bytes_per_launch": pb["color"],
            "launch_ms": float(timed_phase_ms[1]),
            "timed_phase_ms": dict(zip(names, [float(x) for x in timed_phase_ms])),
            "phase_bytes": pb,
            "step": {"algorithmic_bytes": step_bytes, "achieved": step_bytes / (ms_per_step / 1e3) / 1e9,
                     "frac": step_bytes / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS},
        },
        "cpu_baseline": cpu,
        "schedule": sched,
        "phase_ms": dict(zip(names, [float(x) for x in phase_ms])),
        "phase_gbs": {n: pb[n] / (t / 1e3) / 1e9 for n, t in zip(names, phase_ms)},
        "graph": {"bonds_mean": E, "k_mean": k_mean, "q_mean": q, "kw_levels": M,
                  "kw_rounds_mean": float(np.mean([s[3] for s in stats])),
                  "candidates_per_owner": c},
        "last_obs": {k: obs[k] for k in ("E", "M", "n_edges", "q", "kw_rounds", "accepted", "attempts")},
        "trace_us": trace,
        **extra,
    }
    sco.close()
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

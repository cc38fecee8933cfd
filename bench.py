#!/usr/bin/env python
"""Throughput of the stochastic-cutoff (SCO) step on one MI355X.

A step is one full pass of the method over the chain: switching of every dipolar
bond + bond-graph assembly, Kuhn-Wattenhofer colouring + colour bucketing, and n_sw
colour-ordered Metropolis sweeps.  `value` = spin-update attempts per second over
the timed steps (N * n_sw per step), inputs resident in HBM, HIP events on the
library's stream.  A second, untimed-for-`value` pass runs the three phases as
separate launches to time each one; the slowest phase is reported against the HBM
roofline with its algorithmic bytes.  The CPU reference is timed on a short sample
of the same chain (single host thread).

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


def phase_bytes(N, E, c, q, M, k_mean, hard, n_sw):
    """Algorithmic bytes per step of each phase (the data each phase must touch
    once; table look-ups excluded).  E: undirected surviving bonds; c: candidates
    per owner; k_mean: mean surviving-bond degree."""
    switch = N * (8 + 1 + c + 8 + 4) + E * (12 + 16 + 12 + 16 + 8 + 16 + 32)
    per_pending = 4 + 4 + 8 + (4 + k_mean) * 8 + 4 * k_mean + 4
    color = N * (6 + M * (6 + 0.5 * per_pending) + 8)
    per_attempt = 4 + 1 + 4 + 8 + 0.3 + (0.0 if hard else k_mean * 17)
    sweep = N * n_sw * per_attempt
    return {"switch": switch, "color": color, "sweep": sweep}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n-sw", type=int, default=1)
    ap.add_argument("--kappa", type=float, default=1.0)
    ap.add_argument("--phase-steps", type=int, default=5)
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-nsw100", action="store_true")
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
    stream = sco.stream

    for t in range(args.warmup):
        sco.step(t)
    torch.cuda.synchronize()
    progress(f"warmup {args.warmup} steps done")

    first = args.warmup
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    sco.run(first, args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ms_per_step = ms / args.steps
    value = N * p["n_sw"] * args.steps / (ms / 1e3)
    obs = sco.observables()[0]
    progress(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, {value:.4g} attempts/s")

    # one traced step: block 0's phase marks inside the persistent kernel
    sco.trace(True)
    sco.step(first + args.steps)
    marks = sco.trace_read()
    sco.trace(False)
    trace = [(i, round(t, 2)) for i, t in marks]
    progress("trace (id, us): " + " ".join(f"{i}:{t:.1f}" for i, t in trace))

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
        stats.append((o["n_edges"], o["q"], o["kw_levels"], o["kw_rounds"]))
    phase_ms = acc / args.phase_steps
    E = float(np.mean([s[0] for s in stats]))
    q = float(np.mean([s[1] for s in stats]))
    M = float(np.mean([s[2] for s in stats]))
    tables = sco.tables(0)
    c = expected_candidates(tables["J"], p["T"], p["kappa"])
    k_mean = 2.0 * E / N
    pb = phase_bytes(N, E, c, q, M, k_mean, p["kappa"] == 1.0, p["n_sw"])
    names = ["switch", "color", "sweep"]
    dom = int(np.argmax(phase_ms))
    dom_name = names[dom]
    achieved = pb[dom_name] / (phase_ms[dom] / 1e3) / 1e9
    progress("phase ms: " + ", ".join(f"{n}={t:.3f}" for n, t in zip(names, phase_ms)))

    extra = {}
    if not args.no_nsw100 and p["n_sw"] == 1:
        sco100 = SCO([ChainParams(**{**p, "n_sw": 100})], device="cuda:0")
        sco100.run(0, 1)
        torch.cuda.synchronize()
        f0 = torch.cuda.Event(enable_timing=True)
        f1 = torch.cuda.Event(enable_timing=True)
        f0.record(sco100.stream)
        sco100.run(1, 3)
        f1.record(sco100.stream)
        torch.cuda.synchronize()
        ms100 = f0.elapsed_time(f1) / 3
        extra["n_sw_100"] = {"ms_per_step": ms100, "value": N * 100 / (ms100 / 1e3)}
        progress(f"n_sw=100: {ms100:.3f} ms/step")
        sco100.close()

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
                         f"{dt:.1f} s"}
        progress(f"cpu baseline {cpu['value']:.4g} attempts/s")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
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
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "kernel": {"switch": "k_step<1u>", "color": "k_step<2u>", "sweep": "k_step<4u>"}[dom_name],
            "phase": dom_name,
            "algorithmic_bytes_per_launch": pb[dom_name],
        },
        "cpu_baseline": cpu,
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

"""The annealing driver (the cooling protocol of Sec. 3.1) on the GPU against the oracle
run through the same schedule: per-stage statistics identical (exact integer sums
divided the same way), energies within 1e-12 relative, final spins identical."""
import numpy as np
import pytest

import oracle
import workloads
from tests.parity import gpu_params, log, oracle_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1503_03295_amd import lib

    lib()
    yield


def _schedule(t0, t1, dt):
    n = int(round((t0 - t1) / dt)) + 1
    return [round(t0 - k * dt, 10) for k in range(n)]


def test_schedule_helper():
    assert _schedule(1.25, 0.05, 0.05)[:3] == [1.25, 1.2, 1.15] and len(_schedule(1.25, 0.05, 0.05)) == 25


def test_anneal_matches_oracle():
    """Two chains (L=32 open at kappa 2, L=48 periodic at kappa 1, n_sw 3) cooled
    from 1.25 to 0.5 in steps of 0.25, 2 + 3 steps per stage."""
    from paper_1503_03295_amd import SCO

    params = [dict(workloads.chain(32, False, 1.25, 2.0, chain_id=0, n_sw=3), edge_factor=16),
              dict(workloads.chain(48, True, 1.25, 1.0, chain_id=1, n_sw=3), edge_factor=16)]
    temps = _schedule(1.25, 0.5, 0.25)
    gpu = SCO([gpu_params(p) for p in params], device="cuda:0")
    stages = gpu.anneal(temps, 2, 3, first_step=7)
    log(f"anneal: {len(temps)} stages")
    for c, p in enumerate(params):
        ref = oracle.OracleChain(oracle_params(p))
        rs = oracle.anneal(ref, temps, 2, 3, first_step=7)
        for k, r in enumerate(rs):
            g = stages[k][c]
            for key in ("T", "M", "samples", "abs_m", "m2", "k_mean", "delta_sco_mean", "delta_union_mean",
                        "acceptance"):
                assert g[key] == r[key], (c, k, key, g[key], r[key])
            assert abs(g["E"] - r["E"]) <= 1e-12 * max(1.0, abs(r["E"])), (c, k)
        np.testing.assert_array_equal(gpu.spins(c), rs[-1]["spins"])
        log(f"  chain {c}: " + ", ".join(f"T={s['T']:.2f} k={s['k_mean']:.3f} D={s['delta_sco_mean']:.2f}"
                                         for s in rs))


def test_anneal_equals_stagewise_runs():
    """sco_anneal == sco_set_temperature + sco_run stage by stage (same step indices),
    on a ragged batch of chains with per-chain schedules."""
    from paper_1503_03295_amd import SCO

    params = [workloads.chain(64, True, 1.3, 2.0, chain_id=0, n_sw=2),
              workloads.chain(40, False, 1.1, 1.0, chain_id=1)]
    temps = np.array([[1.3, 1.1], [0.9, 0.8], [0.5, 0.6]])
    a = SCO([gpu_params(p) for p in params], device="cuda:0")
    a.anneal(temps, 1, 2, first_step=3)
    b = SCO([gpu_params(p) for p in params], device="cuda:0")
    t = 3
    for row in temps:
        for c, T in enumerate(row):
            b.set_temperature(T, c)
        b.run(t, 3)
        t += 3
    for c in range(len(params)):
        np.testing.assert_array_equal(a.spins(c), b.spins(c))
    oa, ob = a.observables(), b.observables()
    for x, y in zip(oa, ob):
        assert x["M"] == y["M"] and x["accepted"] == y["accepted"] and x["E"] == y["E"]

"""HIP path vs the CPU oracle on the configurations and code paths that the basic
parity tests do not reach: palettes above 32 and 64 colours in the LDS tile levels
and in the device-wide levels, the FP32 + FP64-recheck form at kappa = 1, the L=2304
chain over its first 20 steps, and the 9-chain mixed-precision workload at its own
size (59.2M spins), where the device-wide colouring levels and the sweeps keep their
lists in global memory."""
import numpy as np
import pytest

import oracle
import workloads
from tests.parity import compare_observables, compare_state, gpu_params, log, oracle_params, run_parity, step_all

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1503_03295_amd import lib

    lib()
    yield


# kappa = 6 at T = 0.1 gives q of about 43 (the 64-bit colour sets), kappa = 16 about
# 75 (the 256-bit sets); tile_limit 64 puts every level of such a palette on the
# device-wide path (q 2^P <= 64 leaves P = 0), 0 keeps them all in one LDS tile.
@pytest.mark.parametrize("kappa,q_min", [(6.0, 33), (16.0, 65)])
@pytest.mark.parametrize("tile_limit", [0, 64])
def test_large_palettes(kappa, q_min, tile_limit):
    params = [dict(workloads.chain(64, True, 0.1, kappa, chain_id=0, n_sw=2), edge_factor=128),
              dict(workloads.chain(40, False, 0.1, kappa, chain_id=1), edge_factor=128)]
    log(f"large palettes kappa={kappa} tile_limit={tile_limit}")
    out = run_parity(params, 3, graph_every=1, obs_every=1, schedule=(0, tile_limit))
    obs = out["gpu"].observables()
    assert max(o["q"] for o in obs) >= q_min, [o["q"] for o in obs]
    assert out["tolerated"] == 0


@pytest.mark.parametrize("periodic,L,temps", [(True, 256, (0.8, 1.2, 2.0)), (False, 32, (1.0,))])
def test_fp32_recheck_at_kappa_one(periodic, L, temps):
    """precision 1 at kappa = 1: FP32 exponential gaps in the switching (the sweep's
    exchange-only acceptance is a table lookup), identical to the FP64 oracle."""
    params = [workloads.chain(L, periodic, T, 1.0, chain_id=i, precision=1) for i, T in enumerate(temps)]
    log(f"fp32 + recheck kappa=1 L={L}")
    out = run_parity(params, 20, graph_every=4, obs_every=10)
    obs = out["gpu"].counters()
    log(f"  rechecks {sum(o['rechecks'] for o in obs)}, near ties {sum(o['near_ties'] for o in obs)}")
    assert sum(o["rechecks"] for o in obs) > 0
    assert out["tolerated"] == 0


@pytest.mark.timeout(900)
def test_large_lattice_twenty_steps():
    """L=2304 periodic (N = 5.3M), T = 1.2: spins, CSR and colours after each of the
    first 20 steps, then every observable."""
    params, _ = workloads.large_periodic()
    log("L=2304, 20 steps")
    out = run_parity(params, 20, graph_every=1, obs_every=0, counters_every=5)
    gpu, refs = out["gpu"], out["refs"]
    go = gpu.observables()[0]
    ro = refs[0].observables(dipolar="fft")
    for k in ("M", "n_edges", "delta_union", "q", "colors_used", "kw_levels", "kw_rounds", "near_ties"):
        assert go[k] == ro[k], k
    assert abs(go["E"] - ro["E"]) <= 1e-12 * abs(ro["E"])
    log(f"  tolerated {out['tolerated']}, near ties {go['near_ties']}")
    assert out["tolerated"] == 0


@pytest.mark.timeout(1200)
def test_full_size_mixed_precision_against_oracle():
    """The mixed-precision workload at its own size: 8 chains at L=2304 plus one at
    L=4096 (59.2M spins, kappa = 2) in one context, once with FP64 decisions and once
    with FP32 accumulation + FP64 recheck.  The L=4096 chain and one L=2304 chain are
    run by the oracle; after each of two steps both contexts must equal it in spins,
    CSR and colours.  At this size a block's share of a device-wide colouring level
    and of the sweep exceeds its LDS list, so the global-memory list paths run."""
    from paper_1503_03295_amd import SCO

    sample = (8, 3)
    ctx = {}
    for prec in (0, 1):
        params = workloads.mixed_precision(precision=prec, kappa=2.0)
        ctx[prec] = SCO([gpu_params(p) for p in params], device="cuda:0")
    params = workloads.mixed_precision(precision=0, kappa=2.0)
    refs = {c: oracle.OracleChain(oracle_params(params[c])) for c in sample}
    log(f"full size: {len(params)} chains, {sum(p['L'] ** 2 for p in params)} spins; oracle on {sample}")
    for t in range(2):
        for prec in (0, 1):
            ctx[prec].step(t)
        step_all(list(refs.values()), t)
        for prec in (0, 1):
            for c, r in refs.items():
                diffs = compare_state(ctx[prec], r, c, f"step {t}")
                assert not diffs, (prec, c, t, diffs)
        log(f"  step {t}: both contexts equal the oracle")
    for prec in (0, 1):
        obs = ctx[prec].counters()
        for c, r in refs.items():
            ro = r.observables(dipolar="none")
            for k in ("M", "n_edges", "delta_union", "q", "colors_used", "kw_levels", "kw_rounds", "near_ties"):
                assert obs[c][k] == ro[k], (prec, c, k, obs[c][k], ro[k])
        log(f"  precision {prec}: rechecks {sum(o['rechecks'] for o in obs)}")
    assert sum(o["rechecks"] for o in ctx[1].counters()) > 0
    assert sum(o["rechecks"] for o in ctx[0].counters()) == 0
    for prec in (0, 1):
        ctx[prec].close()


def test_batched_64_chains_graph_and_colours():
    """The 64-chain batch (L from 64 to 1024, T in [0.8, 2.5]) in one context, three
    steps: every chain up to L=512 and one L=1024 chain against the oracle in spins,
    CSR rows, neighbours, displacement indices and colours after every step."""
    from paper_1503_03295_amd import SCO

    params = workloads.batched()
    gpu = SCO([gpu_params(p) for p in params], device="cuda:0")
    sample = [c for c, p in enumerate(params) if p["L"] <= 512]
    sample += [next(c for c, p in enumerate(params) if p["L"] == 1024)]
    log(f"batched: {len(params)} chains; oracle on {len(sample)}")
    refs = {c: oracle.OracleChain(oracle_params(params[c])) for c in sample}
    for t in range(3):
        gpu.step(t)
        step_all(list(refs.values()), t)
        for c, r in refs.items():
            diffs = compare_state(gpu, r, c, f"step {t}")
            assert not diffs, (c, params[c]["L"], t, diffs)
    go = gpu.counters()
    for c, r in refs.items():
        ro = r.observables(dipolar="none")
        for k in ("M", "n_edges", "delta_union", "q", "colors_used", "kw_levels", "kw_rounds", "near_ties"):
            assert go[c][k] == ro[k], (c, k)

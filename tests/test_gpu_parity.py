"""HIP path vs the CPU reference, element by element, through the C-ABI."""
import numpy as np
import pytest

import oracle
import workloads
from tests.parity import compare_observables, gpu_params, log, oracle_params, run_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1503_03295_amd import lib

    lib()
    yield


@pytest.mark.parametrize("L,periodic,kappa,T", [(32, False, 1.0, 1.0), (32, False, 2.0, 1.0),
                                                (64, True, 1.5, 0.8), (256, True, 1.0, 1.2),
                                                (6, True, 2.0, 2.0), (2, False, 1.0, 1.0)])
def test_tables_bit_exact(L, periodic, kappa, T):
    from paper_1503_03295_amd import SCO

    log(f"tables L={L} periodic={periodic} kappa={kappa}")
    p = workloads.chain(L, periodic, T, kappa)
    gpu = SCO([gpu_params(p)], device="cuda:0")
    ref = oracle.OracleChain(oracle_params(p))
    g, r = gpu.tables(0), ref.tables()
    for k in ("dx", "dy", "J", "C", "theta", "delta"):
        np.testing.assert_array_equal(g[k], r[k], err_msg=k)
    np.testing.assert_array_equal(gpu.spins(0), ref.spins)


@pytest.mark.parametrize("kappa", [1.0, 2.0])
def test_small_open_lattice_full_run(kappa):
    """L=32 open, T=1.0: every step of a 1000-step run (spins, CSR, colours)."""
    params, n_steps = workloads.small_open(kappa)
    log(f"small open kappa={kappa}")
    out = run_parity(params, n_steps, graph_every=1, obs_every=100)
    log(f"  tolerated near ties: {out['tolerated']}")


@pytest.mark.parametrize("kappa", [1.0, 2.0])
def test_medium_periodic_three_temperatures(kappa):
    """L=256 periodic, T in {0.8, 1.2, 2.0}, three chains in one context."""
    params, _ = workloads.medium_periodic(kappa)
    log(f"medium periodic kappa={kappa}")
    out = run_parity(params, 40, graph_every=5, obs_every=20)
    log(f"  tolerated near ties: {out['tolerated']}")


@pytest.mark.parametrize("kappa", [1.0, 2.0])
def test_several_sweeps_after_device_wide_levels(kappa):
    """L=640 periodic (N = 410k: KW levels above the LDS tile run device-wide), four
    sweeps per step: every sweep's neighbour order comes from the final colours, and a
    sweep may start before the previous one has ended elsewhere on the lattice."""
    params = [workloads.chain(640, True, 1.1, kappa, chain_id=0, n_sw=4)]
    log(f"640 periodic, n_sw=4, kappa={kappa}")
    out = run_parity(params, 3, graph_every=1, obs_every=2)
    go = out["gpu"].observables()[0]
    # levels above P = floor(log2(28672 / q)) (the largest LDS tile) ran device-wide
    assert go["kw_levels"] > int(np.floor(np.log2(28672 / go["q"])))
    log(f"  tolerated near ties: {out['tolerated']}")


def test_step_forms_give_identical_chains():
    """A step as three phase launches (the default) and as one fused launch: same
    spins, bond graph, colours and counters, by plain launches and graph replays."""
    from paper_1503_03295_amd import SCO

    params = [workloads.chain(256, True, 1.2, 2.0, chain_id=0, n_sw=2),
              workloads.chain(40, False, 0.9, 1.0, chain_id=1)]
    a = SCO([gpu_params(p) for p in params], device="cuda:0")
    b = SCO([gpu_params(p) for p in params], device="cuda:0")
    b.set_step_form(True)
    a.run(0, 3)
    b.run(0, 3)
    a.run_graph(3, 2)
    b.run_graph(3, 2)
    for c in range(len(params)):
        np.testing.assert_array_equal(a.spins(c), b.spins(c))
        for x, y in zip(a.graph(c), b.graph(c)):
            np.testing.assert_array_equal(x, y)
    for x, y in zip(a.counters(), b.counters()):
        for k in ("M", "n_edges", "q", "kw_rounds", "accepted", "attempts", "near_ties"):
            assert x[k] == y[k], k
    assert all(t > 0 for t in a.phase_times())  # the last step's phases are timed


def test_fenced_sweeps_match_oracle():
    """The documented release/acquire barrier after every colour class gives the same
    chains as the light class barrier (a ragged batch, three sweeps per step)."""
    params = [workloads.chain(256, True, 1.2, 2.0, chain_id=0, n_sw=3),
              workloads.chain(48, False, 0.9, 1.0, chain_id=1, n_sw=2)]
    log("fenced sweeps: 256 periodic + 48 open")
    out = run_parity(params, 4, graph_every=2, counters_every=3, fenced=True)
    assert out["tolerated"] == 0


def test_ragged_batch_of_chains():
    """Chains of different L, boundaries, kappa and n_sw in one launch."""
    params = [workloads.chain(8, True, 2.0, 2.0, chain_id=0, n_sw=2),
              workloads.chain(33, False, 1.1, 1.0, chain_id=1),
              workloads.chain(64, True, 0.9, 1.0, chain_id=2, n_sw=3),
              workloads.chain(20, False, 1.7, 3.0, chain_id=3, n_sw=0),
              workloads.chain(48, True, 1.3, 2.0, chain_id=4, seed=7)]
    log("ragged batch")
    run_parity(params, 30, graph_every=3, obs_every=10)


def test_smallest_lattices():
    """The smallest lattices the boundary accepts, in one batch: an open 2 x 2 and
    3 x 3 (a handful of bonds, a palette larger than the lattice) and periodic 4 x 4
    and 6 x 6 (the image sum and the self-conjugate displacements at their smallest)."""
    params = [workloads.chain(2, False, 1.0, 1.0, chain_id=0, n_sw=2),
              workloads.chain(3, False, 0.7, 2.0, chain_id=1),
              workloads.chain(4, True, 1.5, 1.0, chain_id=2, n_sw=3),
              workloads.chain(6, True, 0.9, 2.0, chain_id=3)]
    log("smallest lattices")
    run_parity(params, 40, graph_every=1, obs_every=5)


def test_split_entry_points_equal_step():
    """sco_switch + sco_color + sco_sweep == sco_step."""
    from paper_1503_03295_amd import SCO

    p = workloads.chain(64, True, 1.0, 2.0, n_sw=2)
    a = SCO([gpu_params(p)], device="cuda:0")
    b = SCO([gpu_params(p)], device="cuda:0")
    for t in range(5):
        a.step(t)
        b.switch(t)
        b.color()
        b.sweep(t, 2)
    np.testing.assert_array_equal(a.spins(0), b.spins(0))


def test_graph_replays_equal_plain_launches():
    """sco_run_graph (a HIP graph of cooperative step nodes) gives the chains of
    sco_run; the graph is replayed several times with eager work and
    synchronisations between the replays, each replay checked."""
    from paper_1503_03295_amd import SCO

    params = [workloads.chain(128, True, 1.2, 2.0, chain_id=0, n_sw=2),
              workloads.chain(40, False, 0.9, 1.0, chain_id=1)]
    a = SCO([gpu_params(p) for p in params], device="cuda:0")
    b = SCO([gpu_params(p) for p in params], device="cuda:0")
    t = 0
    for rep in range(4):
        a.run(t, 3)
        b.run_graph(t, 3)
        t += 3
        for c in range(len(params)):
            np.testing.assert_array_equal(a.spins(c), b.spins(c), err_msg=f"replay {rep} chain {c}")
            for x, y in zip(a.graph(c), b.graph(c)):
                np.testing.assert_array_equal(x, y)
        b.step(t)  # eager work between replays
        a.step(t)
        t += 1
        assert [o["accepted"] for o in a.counters()] == [o["accepted"] for o in b.counters()]
    # another length and another grid rebuild the graph
    b.set_schedule(max(1, b.schedule()[0] // 2), 4096)
    a.run(t, 2)
    b.run_graph(t, 2)
    for c in range(len(params)):
        np.testing.assert_array_equal(a.spins(c), b.spins(c))


def test_checkpoint_resume_exact():
    from paper_1503_03295_amd import SCO

    p = workloads.chain(128, True, 1.2, 2.0)
    a = SCO([gpu_params(p)], device="cuda:0")
    for t in range(6):
        a.step(t)
        if t == 2:
            saved = a.spins(0)
    b = SCO([gpu_params(p)], device="cuda:0")
    b.set_spins(0, saved)
    for t in range(3, 6):
        b.step(t)
    np.testing.assert_array_equal(a.spins(0), b.spins(0))


def test_edge_capacity_overflow_stops_the_step():
    """An edge overflow ends the launch at the barrier after the switching: no spin
    moves, the later launches do nothing, and the next synchronising call reports it
    (with the flag named); the context stays usable afterwards."""
    from paper_1503_03295_amd import SCO, ScoError

    p = workloads.chain(64, True, 0.8, 3.0)
    p["edge_factor"] = 1
    g = SCO([gpu_params(p)], device="cuda:0")
    s0 = g.spins(0)
    g.step(0)
    g.step(1)
    np.testing.assert_array_equal(g.spins(0), s0)
    with pytest.raises(ScoError) as e:
        g.observables()
    assert e.value.code == -3 and e.value.flags == 1, e.value
    np.testing.assert_array_equal(g.spins(0), s0)
    assert g.observables()[0]["attempts"] == 0
    # sco_run reports the flag of its own steps
    with pytest.raises(ScoError) as e:
        g.run(0, 3)
    assert e.value.code == -3
    np.testing.assert_array_equal(g.spins(0), s0)
    # a chain with room runs on
    q = dict(p, edge_factor=16)
    h = SCO([gpu_params(q)], device="cuda:0")
    h.run(0, 3)
    assert h.observables()[0]["attempts"] == 3 * 64 * 64


@pytest.mark.parametrize("kappa", [1.5, 2.0])
def test_mixed_precision_matches_fp64_oracle(kappa):
    """FP32 gaps and local fields with FP64 recheck: the same chain as the FP64
    oracle, bit for bit (L=256 periodic, three temperatures)."""
    params = [workloads.chain(256, True, T, kappa, chain_id=i, precision=1)
              for i, T in enumerate((0.8, 1.2, 2.0))]
    log(f"mixed precision kappa={kappa}")
    out = run_parity(params, 30, graph_every=5, obs_every=15)
    obs = out["gpu"].observables()
    rechecks = sum(o["rechecks"] for o in obs)
    attempts = sum(o["attempts"] for o in obs)
    log(f"  rechecks {rechecks} of {attempts} attempts (+ switching draws)")
    assert rechecks > 0, "the FP64 recheck path was never taken"


def test_mixed_precision_equals_fp64_gpu_chain():
    """precision 1 and precision 0 contexts of the same chain stay identical."""
    from paper_1503_03295_amd import SCO

    p0 = workloads.chain(512, True, 1.1, 2.0, n_sw=3)
    p1 = dict(p0, precision=1)
    a = SCO([gpu_params(p0)], device="cuda:0")
    b = SCO([gpu_params(p1)], device="cuda:0")
    log("mixed precision vs fp64 on the GPU, L=512")
    for t in range(25):
        a.step(t)
        b.step(t)
        np.testing.assert_array_equal(a.spins(0), b.spins(0), err_msg=f"step {t}")
    ra, rb = a.graph(0), b.graph(0)
    for x, y in zip(ra, rb):
        np.testing.assert_array_equal(x, y)
    assert a.observables()[0]["rechecks"] == 0
    assert b.observables()[0]["rechecks"] > 0


def test_schedules_give_identical_chains():
    """Grid size and tile limit change the schedule only: the same spins, bond graph
    and colours for every choice, and the autotuner restores the chain it timed on.
    One block alone holds more sites than its LDS can count partners for and scans
    several tiles, so it takes the device-atomic partner counts and the re-reading
    scan."""
    from paper_1503_03295_amd import SCO

    params = [workloads.chain(256, True, 1.2, 2.0, chain_id=0), workloads.chain(96, False, 0.9, 1.0, chain_id=1)]
    ref = SCO([gpu_params(p) for p in params], device="cuda:0")
    for t in range(4):
        ref.step(t)
    maxb, _ = ref.schedule()
    log(f"schedules: co-resident blocks {maxb}")
    for blocks, tile in ((maxb // 2, 16384), (maxb, 4096), (max(1, maxb // 3), 1024), (7, 64), (1, 2048)):
        g = SCO([gpu_params(p) for p in params], device="cuda:0")
        g.set_schedule(blocks, tile)
        assert g.schedule() == (blocks, tile)
        for t in range(4):
            g.step(t)
        for c in range(len(params)):
            np.testing.assert_array_equal(g.spins(c), ref.spins(c))
            for x, y in zip(g.graph(c), ref.graph(c)):
                np.testing.assert_array_equal(x, y)
        obs_g, obs_r = g.observables(), ref.observables()
        for og, orr in zip(obs_g, obs_r):
            for k in ("M", "n_edges", "q", "kw_rounds", "accepted"):
                assert og[k] == orr[k], (blocks, tile, k)
    # the autotuner times trials and leaves the chain where it was
    a = SCO([gpu_params(p) for p in params], device="cuda:0")
    for t in range(2):
        a.step(t)
    before = [a.spins(c) for c in range(len(params))]
    acc_before = [o["accepted"] for o in a.observables()]
    choice = a.autotune(2)
    log(f"  autotune: {choice}")
    for c in range(len(params)):
        np.testing.assert_array_equal(a.spins(c), before[c])
    assert [o["accepted"] for o in a.observables()] == acc_before
    for t in range(2, 4):
        a.step(t)
    for c in range(len(params)):
        np.testing.assert_array_equal(a.spins(c), ref.spins(c))


def test_full_size_graph_and_colouring_properties():
    """8 chains at L=2304 plus one at L=4096 (59M spins, kappa=2), two steps: for the
    L=4096 chain and one L=2304 chain, the CSR is symmetric with rows ascending and no
    duplicates, every displacement index names the bond's displacement, the colouring
    of the union graph is proper with colours below q, and the observables count the
    graph and the spins exactly (too large for the CPU reference in a test)."""
    from paper_1503_03295_amd import SCO

    params = workloads.mixed_precision(precision=0, kappa=2.0)
    gpu = SCO([gpu_params(p) for p in params], device="cuda:0")
    log(f"full size: {len(params)} chains, {sum(p['L'] ** 2 for p in params)} spins")
    gpu.run(0, 2)
    obs = gpu.observables()
    for c in (8, 3):
        L = params[c]["L"]
        N = L * L
        rp, col, attr, colors = gpu.graph(c)
        tab = gpu.tables(c)
        s = gpu.spins(c)
        assert rp[0] == 0 and rp[-1] == len(col) == 2 * obs[c]["n_edges"]
        deg = np.diff(rp)
        rows = np.repeat(np.arange(N), deg)
        # rows ascending, no duplicate neighbour, no self bond
        same_row = rows[1:] == rows[:-1]
        assert np.all(col[1:][same_row] > col[:-1][same_row])
        assert np.all(col != rows)
        # symmetric: (u, w, m) present iff (w, u, m)
        fwd = rows.astype(np.int64) * N + col
        bwd = col.astype(np.int64) * N + rows
        order_f, order_b = np.argsort(fwd), np.argsort(bwd)
        np.testing.assert_array_equal(fwd[order_f], bwd[order_b])
        np.testing.assert_array_equal(attr[order_f], attr[order_b])
        # the displacement of each bond is its table entry (modulo the lattice)
        dx = (col % L - rows % L) % L
        dy = (col // L - rows // L) % L
        tdx, tdy = tab["dx"][attr] % L, tab["dy"][attr] % L
        assert np.all(((dx == tdx) & (dy == tdy)) | ((dx == (-tdx) % L) & (dy == (-tdy) % L)))
        # proper colouring of bonds and nearest-neighbour pairs, palette below q
        assert colors.max() < obs[c]["q"] and obs[c]["colors_used"] <= obs[c]["q"]
        assert np.all(colors[rows] != colors[col])
        v = np.arange(N)
        x, y = v % L, v // L
        assert np.all(colors[v] != colors[y * L + (x + 1) % L])
        assert np.all(colors[v] != colors[((y + 1) % L) * L + x])
        # spins and counters
        assert obs[c]["M"] == int(s.astype(np.int64).sum())
        assert obs[c]["attempts"] == 2 * N
        # union degree bound
        assert obs[c]["q"] == obs[c]["delta_union"] + 1 and obs[c]["delta_union"] >= 4

"""The colouring variants of Sec. 2.3 on the GPU against the oracle: the checkerboard
product of a KW colouring of the bonds, and basic colour reduction with rule (2)' on
the whole union graph without KW groups.  Spins, CSR and colours after every step,
round counts and the other integer observables at the end."""
import pytest

import workloads
from tests.parity import log, run_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1503_03295_amd import lib

    lib()
    yield


def _chains(mode):
    return [dict(workloads.chain(64, True, 1.2, 2.0, chain_id=0, n_sw=2), coloring=mode),
            dict(workloads.chain(33, False, 0.9, 1.0, chain_id=1), coloring=mode),
            dict(workloads.chain(96, True, 2.0, 1.5, chain_id=2), coloring=mode)]


@pytest.mark.parametrize("tile_limit", [0, 256])
def test_checkerboard_product(tile_limit):
    log(f"checkerboard product, tile_limit={tile_limit}")
    out = run_parity(_chains(1), 8, graph_every=1, obs_every=4, schedule=(0, tile_limit))
    assert out["tolerated"] == 0


def test_whole_graph_reduction():
    log("whole-graph basic colour reduction (2)'")
    out = run_parity(_chains(2), 6, graph_every=1, obs_every=3)
    obs = out["gpu"].counters()
    log("  rounds " + ", ".join(str(o["kw_rounds"]) for o in obs))
    assert all(o["kw_levels"] == 1 for o in obs)
    assert out["tolerated"] == 0


def test_device_wide_checkerboard_at_640():
    """L=640 periodic: the bond-only KW levels above the LDS tile run device-wide."""
    params = [dict(workloads.chain(640, True, 1.1, 2.0, chain_id=0, n_sw=2), coloring=1)]
    out = run_parity(params, 3, graph_every=1, obs_every=2)
    assert out["tolerated"] == 0

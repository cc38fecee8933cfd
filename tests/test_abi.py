"""The C-ABI library loads on a machine without a GPU and exports every symbol that
include/sco.h declares; host-only entry points validate their arguments."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "sco.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sco_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["sco_init", "sco_switch", "sco_color", "sco_sweep", "sco_observables"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1503_03295_amd import _lib

    L = _lib.lib()
    for n in declared_functions():
        assert hasattr(L, n), n
    assert set(declared_functions()) == set(_lib.EXPORTS)


def test_strerror():
    from paper_1503_03295_amd import _lib

    L = _lib.lib()
    assert L.sco_strerror(0) == b"ok"
    assert b"overflow" not in L.sco_strerror(-1)
    assert L.sco_strerror(-3).startswith(b"surviving bonds")


@pytest.mark.parametrize("bad", [dict(L=5, periodic=True), dict(L=2, periodic=True), dict(kappa=0.5),
                                 dict(T=0.0), dict(T=float("nan")), dict(L=1), dict(n_sw=-1),
                                 dict(precision=2), dict(J=-1.0)])
def test_workspace_size_rejects_invalid_parameters(bad):
    from paper_1503_03295_amd import ChainParams, ScoError, workspace_size

    kw = dict(L=8, periodic=True, T=1.0)
    kw.update(bad)
    with pytest.raises(ScoError) as e:
        workspace_size([ChainParams(**kw)])
    assert e.value.code == -1


def test_workspace_size_grows_with_chains():
    from paper_1503_03295_amd import ChainParams, workspace_size

    a = workspace_size([ChainParams(L=64, periodic=True, T=1.0)])
    b = workspace_size([ChainParams(L=64, periodic=True, T=1.0)] * 3)
    c = workspace_size([ChainParams(L=64, periodic=True, T=1.0, kappa=2.0)])
    assert 0 < a < b and a < c


def test_workloads_philox_matches_known_answers():
    import workloads

    assert workloads.philox4x32_10([0] * 4, [0, 0]) == (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)
    assert workloads.philox4x32_10([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2) == (
        0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)
    b = workloads.batched()
    assert len(b) == 64 and {c["L"] for c in b} <= {64, 128, 256, 512, 1024}
    assert all(0.8 <= c["T"] <= 2.5 for c in b)

"""Pins of the oracle's observables and chain bookkeeping."""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import ChainParams, OracleChain
from tests.test_oracle_exact import energies, model


@pytest.mark.parametrize("L,periodic", [(5, False), (6, True), (8, True)])
def test_energy_matches_pair_sum(L, periodic):
    """E from the owner-pair sum equals the brute-force sum over all pairs with the
    couplings computed independently (dense matrix of the test model)."""
    c = OracleChain(ChainParams(L=L, periodic=periodic, T=1.0, seed=4))
    for t in range(3):
        c.step(t)
    W, nn = model(L, periodic)
    E_ref = energies(c.spins[None, :], W, nn)[0]
    o = c.observables(dipolar="direct")
    assert o["E"] == pytest.approx(E_ref, rel=1e-12, abs=1e-12)
    assert o["M"] == int(c.spins.sum())


@pytest.mark.parametrize("L", [8, 16, 32])
def test_fft_route_equals_direct_route(L):
    c = OracleChain(ChainParams(L=L, periodic=True, T=1.5, seed=9))
    for t in range(4):
        c.step(t)
    a = c.observables(dipolar="direct")
    b = c.observables(dipolar="fft")
    assert b["E_dipolar"] == pytest.approx(a["E_dipolar"], rel=1e-12)


def test_autocorrelation_is_exact():
    rng = np.random.default_rng(0)
    L = 12
    s = rng.choice(np.array([-1, 1], np.int8), size=L * L)
    C = oracle.autocorrelation_periodic(s, L)
    g = s.reshape(L, L).astype(np.int64)
    for dy, dx in itertools.product(range(L), range(L)):
        assert C[dy, dx] == int(np.sum(g * np.roll(np.roll(g, -dy, 0), -dx, 1)))


def test_determinism_and_chain_independence():
    p = ChainParams(L=16, periodic=True, T=1.2, kappa=2.0, seed=5)
    a, b = OracleChain(p), OracleChain(p)
    for t in range(5):
        a.step(t)
        b.step(t)
    np.testing.assert_array_equal(a.spins, b.spins)
    c = OracleChain(ChainParams(L=16, periodic=True, T=1.2, kappa=2.0, seed=5, chain_id=1))
    assert not np.array_equal(c.spins, OracleChain(p).spins)


def test_checkpoint_resume_is_exact():
    p = ChainParams(L=16, periodic=False, T=1.0, kappa=2.0, seed=8)
    a = OracleChain(p)
    for t in range(10):
        a.step(t)
        if t == 4:
            saved = a.spins.copy()
    b = OracleChain(p, init_spins=saved)
    for t in range(5, 10):
        b.step(t)
    np.testing.assert_array_equal(a.spins, b.spins)


def test_initial_spins_are_philox_sign_bits():
    p = ChainParams(L=8, periodic=True, T=1.0, seed=1, chain_id=3)
    c = OracleChain(p)
    exp = [(-1 if oracle.philox4x32_10([0, v, 0, 1], [1, 3])[0] >> 31 else 1) for v in range(64)]
    np.testing.assert_array_equal(c.spins, exp)


@pytest.mark.parametrize("bad", [dict(L=5, periodic=True), dict(L=2, periodic=True),
                                 dict(kappa=0.5), dict(T=0.0), dict(T=-1.0), dict(L=1)])
def test_invalid_parameters_rejected(bad):
    kw = dict(L=8, periodic=True, T=1.0)
    kw.update(bad)
    with pytest.raises(ValueError):
        OracleChain(ChainParams(**kw))


def test_counters_and_hard_bond_freeze():
    """kappa == 1: a spin with a surviving bond never flips during the sweep."""
    c = OracleChain(ChainParams(L=32, periodic=True, T=1.0, kappa=1.0, seed=2))
    for t in range(3):
        c.switch(t)
        c.color()
        rp, _, _ = c.csr()
        before = c.spins.copy()
        c.sweep(t)
        after = c.spins
        bonded = np.diff(rp) > 0
        assert np.array_equal(before[bonded], after[bonded])
    o = c.observables(dipolar="none")
    assert o["attempts"] == 3 * 32 * 32
    assert 0 < o["accepted"] < o["attempts"]
    assert o["near_ties"] == 0

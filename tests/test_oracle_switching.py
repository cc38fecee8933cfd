"""Pins of the oracle's switching step (A) against the plain per-pair definition of
Eq. (1): with the spins held fixed, each dipolar bond V_ij = J_ij s_i s_j must
survive (switch to Vbar) independently with probability 1 - P_ij, where
P_ij = exp(beta (V_ij - V^max)) (Eq. 2) and V^max = kappa J_ij.  The oracle gets
there through geometric skipping plus thinning; this test only counts outcomes."""
import math

import numpy as np
import pytest

from oracle import ChainParams, OracleChain


def _expected_survival(c: OracleChain, spins: np.ndarray) -> np.ndarray:
    t = c.tables()
    beta = 1.0 / c.params.T
    kap = c.params.kappa
    p = np.zeros((c.N, c.K))
    valid = np.zeros((c.N, c.K), bool)
    for i in range(c.N):
        for m in range(c.K):
            j = c.partner(i, m)
            if j < 0:
                continue
            valid[i, m] = True
            V = t["J"][m] * spins[i] * spins[j]
            P = math.exp(beta * (V - kap * t["J"][m]))
            p[i, m] = 1.0 - P
    return p, valid


@pytest.mark.parametrize("L,periodic,T,kappa", [
    (4, True, 1.0, 1.0), (4, True, 0.7, 2.0), (5, False, 1.0, 1.0), (5, False, 2.0, 2.0),
    (6, True, 1.5, 1.5),
])
def test_pairwise_survival_frequencies(L, periodic, T, kappa):
    n_steps = 40000
    c = OracleChain(ChainParams(L=L, periodic=periodic, T=T, kappa=kappa, seed=11))
    rng = np.random.default_rng(L * 100 + int(10 * T))
    spins = rng.choice(np.array([-1, 1], np.int8), size=c.N)
    c.spins = spins
    counts = c.survival_counts(t0=1000, n_steps=n_steps)
    p, valid = _expected_survival(c, spins)
    # never a survivor for an unowned (i, m)
    assert counts[~valid].sum() == 0
    # kappa == 1: a parallel pair never survives
    if kappa == 1.0:
        assert np.all(counts[valid & (p == 0.0)] == 0)
    # pooled per (m, parallel/antiparallel): binomial z-scores
    t = c.tables()
    zs = []
    for m in range(c.K):
        for par in (True, False):
            sel = valid[:, m].copy()
            for i in np.nonzero(sel)[0]:
                j = c.partner(i, m)
                sel[i] = (spins[i] == spins[j]) == par
            n = int(sel.sum())
            if n == 0:
                continue
            pe = p[sel, m]
            assert np.allclose(pe, pe[0])
            pe = pe[0]
            obs = counts[sel, m].sum()
            trials = n * n_steps
            if pe == 0.0:
                assert obs == 0
                continue
            z = (obs - trials * pe) / math.sqrt(trials * pe * (1 - pe))
            zs.append(z)
    zs = np.array(zs)
    assert np.max(np.abs(zs)) < 5.0, (np.argmax(np.abs(zs)), zs.max(), zs.min())
    # the z-scores of independent classes are ~ N(0, 1)
    chi2 = float(np.sum(zs ** 2))
    k = len(zs)
    assert abs(chi2 - k) < 6 * math.sqrt(2 * k), (chi2, k)


def test_survivors_are_owner_major_in_draw_order():
    c = OracleChain(ChainParams(L=32, periodic=False, T=1.0, kappa=2.0))
    c.switch(3)
    o, n, m = c.survivors()
    assert np.all(np.diff(o) >= 0)
    same = np.diff(o) == 0
    assert np.all(np.diff(m)[same] > 0)
    for i, j, mm in zip(o, n, m):
        assert c.partner(int(i), int(mm)) == j


def test_switching_is_counter_based():
    """The survivor set of step t depends on (seed, chain, t, spins) only."""
    p = ChainParams(L=16, periodic=True, T=1.2, kappa=2.0)
    a, b = OracleChain(p), OracleChain(p)
    a.switch(5)
    b.switch(9)
    b.switch(5)
    for x, y in zip(a.survivors(), b.survivors()):
        np.testing.assert_array_equal(x, y)
    c = OracleChain(ChainParams(L=16, periodic=True, T=1.2, kappa=2.0, chain_id=1))
    c.spins = a.spins
    c.switch(5)
    assert not (len(c.survivors()[0]) == len(a.survivors()[0])
                and np.array_equal(c.survivors()[2], a.survivors()[2]))

"""Pins of the method's exactness (Sec. 2.1: SPS keeps detailed balance, so the SCO
chain samples the Boltzmann distribution of the full Hamiltonian).

1. Formula level, exact: on a 2x2 lattice the SCO transition matrix built from
   Eqs. (1)-(4) -- sum over all 2^6 bond sets b of P(b|s) times a Metropolis sweep
   of H'_b -- leaves exp(-beta H) invariant to 1e-12, for kappa = 1 and 2.
2. Oracle level, statistical: the oracle's own chain on a 4x4 lattice (2^16
   states, enumerated exactly) reproduces the Boltzmann energy distribution
   (chi-square) and <E>, <m^2>.
3. Oracle level, statistical: on 8x8 lattices the oracle agrees with plain
   single-spin Metropolis of the full long-range Hamiltonian (a textbook sampler
   written here, sharing nothing with the oracle).
"""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

from oracle import ChainParams, OracleChain

J_EX, D = 1.0, 0.1


def pair_coupling(L, periodic, dx, dy, n_images=8):
    if not periodic:
        return D / math.hypot(dx, dy) ** 3
    h = L // 2
    dx = ((dx + h - 1) % L) - h + 1
    dy = ((dy + h - 1) % L) - h + 1
    acc = 0.0
    for nx in range(-n_images, n_images + 1):
        for ny in range(-n_images, n_images + 1):
            r = math.hypot(dx + nx * L, dy + ny * L)
            acc += D / r ** 3
    return acc


def model(L, periodic):
    """dense coupling matrix W (zero diagonal) and the list of NN pairs"""
    N = L * L
    W = np.zeros((N, N))
    for i, j in itertools.combinations(range(N), 2):
        dx, dy = j % L - i % L, j // L - i // L
        W[i, j] = W[j, i] = pair_coupling(L, periodic, dx, dy)
    nn = set()
    for v in range(N):
        x, y = v % L, v // L
        for (a, b) in [(x + 1, y), (x, y + 1)]:
            if periodic:
                nn.add(tuple(sorted((v, (b % L) * L + a % L))))
            elif a < L and b < L:
                nn.add((v, b * L + a))
    return W, sorted(nn)


def energies(states, W, nn):
    s = states.astype(np.float64)
    ex = np.zeros(len(s))
    for i, j in nn:
        ex += s[:, i] * s[:, j]
    dip = 0.5 * np.einsum("ki,ij,kj->k", s, W, s)
    return -J_EX * ex + dip


def all_states(N):
    idx = np.arange(2 ** N)[:, None]
    bits = (idx >> np.arange(N)[None, :]) & 1
    return np.where(bits == 1, -1, 1).astype(np.int8)


# --------------------------------------------------------------------------- 1
@pytest.mark.parametrize("kappa", [1.0, 2.0])
@pytest.mark.parametrize("T", [0.7, 2.0])
def test_sco_transition_matrix_is_stationary_2x2(kappa, T):
    L, N = 2, 4
    W, nn = model(L, False)
    beta = 1.0 / T
    pairs = list(itertools.combinations(range(N), 2))
    states = all_states(N)
    S = len(states)
    H = energies(states, W, nn)
    pi = np.exp(-beta * (H - H.min()))
    pi /= pi.sum()
    index = {tuple(s): k for k, s in enumerate(states)}

    def vbar(Jij, s):
        P = math.exp(beta * (Jij * s - kappa * Jij))
        if P >= 1.0:
            return math.inf
        return Jij * s - T * math.log(1.0 - P)

    Tm = np.zeros((S, S))
    for b in itertools.product([0, 1], repeat=len(pairs)):
        bonds = [pairs[k] for k in range(len(pairs)) if b[k]]

        def hprime(s):
            e = -J_EX * sum(s[i] * s[j] for i, j in nn)
            for i, j in bonds:
                e += vbar(W[i, j], s[i] * s[j])
            return e

        # sweep kernel: one Metropolis trial per site, in site order
        K = np.eye(S)
        for site in range(N):
            Ks = np.zeros((S, S))
            for a, s in enumerate(states):
                e0 = hprime(s)
                t = s.copy()
                t[site] = -t[site]
                e1 = hprime(t)
                if math.isinf(e0):
                    Ks[a, a] = 1.0
                    continue
                acc = 1.0 if e1 <= e0 else math.exp(-beta * (e1 - e0))
                Ks[a, index[tuple(t)]] += acc
                Ks[a, a] += 1.0 - acc
            K = K @ Ks
        for a, s in enumerate(states):
            pb = 1.0
            for k, (i, j) in enumerate(pairs):
                P = math.exp(beta * (W[i, j] * s[i] * s[j] - kappa * W[i, j]))
                pb *= (1.0 - P) if b[k] else P
            if pb:
                Tm[a] += pb * K[a]
    np.testing.assert_allclose(Tm.sum(axis=1), 1.0, atol=1e-12)
    np.testing.assert_allclose(pi @ Tm, pi, atol=1e-12)


# --------------------------------------------------------------------------- 2
def _levels(H, tol=1e-9):
    order = np.argsort(H)
    Hs = H[order]
    cuts = np.nonzero(np.diff(Hs) > tol)[0] + 1
    starts = np.concatenate([[0], cuts])
    centers = Hs[starts]
    return centers, Hs, starts


@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("T,kappa", [(2.0, 1.0), (2.0, 2.0), (3.0, 1.0), (3.0, 2.0)])
def test_4x4_energy_distribution_matches_enumeration(periodic, T, kappa):
    L, N = 4, 16
    W, nn = model(L, periodic)
    states = all_states(N)
    H = energies(states, W, nn)
    beta = 1.0 / T
    w = np.exp(-beta * (H - H.min()))
    Z = w.sum()
    m = states.sum(axis=1) / N
    E_exact = float((w * H).sum() / Z) / N
    m2_exact = float((w * m * m).sum() / Z)

    centers, Hs, starts = _levels(H)
    ws = w[np.argsort(H)]
    p_level = np.add.reduceat(ws, starts) / Z

    thin, n_steps = 20, 200000
    c = OracleChain(ChainParams(L=L, periodic=periodic, T=T, kappa=kappa, seed=17,
                                chain_id=int(10 * T + kappa + 100 * periodic)))
    t, Es, Ms = c.run_record(0, 2000, 0)
    t, Es, Ms = c.run_record(t, n_steps, thin)
    n = len(Es)
    # each sample to its exact level
    k = np.clip(np.searchsorted(centers, Es - 1e-7), 0, len(centers) - 1)
    assert np.all(np.abs(centers[k] - Es) < 1e-7)
    obs = np.bincount(k, minlength=len(centers)).astype(float)
    exp_ = p_level * n
    # merge adjacent levels until every bin expects >= 5
    bins_o, bins_e, acc_o, acc_e = [], [], 0.0, 0.0
    for o_, e_ in zip(obs, exp_):
        acc_o += o_
        acc_e += e_
        if acc_e >= 5:
            bins_o.append(acc_o); bins_e.append(acc_e); acc_o = acc_e = 0.0
    bins_o[-1] += acc_o
    bins_e[-1] += acc_e
    chi2 = float(np.sum((np.array(bins_o) - bins_e) ** 2 / np.array(bins_e)))
    dof = len(bins_e) - 1
    pval = stats.chi2.sf(chi2, dof)
    assert pval > 1e-4, (chi2, dof, pval)
    # means (samples are 20 steps apart, several autocorrelation times)
    e = Es / N
    assert abs(e.mean() - E_exact) < 5 * e.std() / math.sqrt(n)
    mm = (Ms / N) ** 2
    assert abs(mm.mean() - m2_exact) < 5 * mm.std() / math.sqrt(n)


# --------------------------------------------------------------------------- 3
def plain_metropolis(L, periodic, T, n_sweeps, seed, thin=5):
    """Single-spin Metropolis of the full Hamiltonian (dense long-range field)."""
    N = L * L
    W, nn = model(L, periodic)
    nbr = [[] for _ in range(N)]
    for i, j in nn:
        nbr[i].append(j)
        nbr[j].append(i)
    rng = np.random.default_rng(seed)
    s = rng.choice(np.array([-1.0, 1.0]), size=N)
    f = W @ s
    beta = 1.0 / T
    E = energies(s[None, :].astype(np.int8), W, nn)[0]
    Es, Ms = [], []
    us = rng.random((n_sweeps, N))
    for sw in range(n_sweeps):
        u = us[sw]
        for i in range(N):
            dE = 2.0 * s[i] * (J_EX * sum(s[j] for j in nbr[i]) - f[i])
            if dE <= 0 or u[i] < math.exp(-beta * dE):
                s[i] = -s[i]
                f += 2.0 * s[i] * W[:, i]
                E += dE
        if sw % thin == 0:
            Es.append(E)
            Ms.append(s.sum())
    return np.array(Es), np.array(Ms)


def binned_mean_err(x, nbins=20):
    b = np.array_split(x, nbins)
    means = np.array([bb.mean() for bb in b])
    return x.mean(), means.std(ddof=1) / math.sqrt(nbins)


@pytest.mark.slow
@pytest.mark.parametrize("periodic,T,kappa", [(True, 3.0, 1.0), (False, 3.0, 2.0), (True, 1.6, 2.0)])
def test_8x8_agrees_with_plain_metropolis(periodic, T, kappa):
    L, N = 8, 64
    Ep, Mp = plain_metropolis(L, periodic, T, n_sweeps=6000, seed=3)
    Ep, Mp = Ep[40:], Mp[40:]
    c = OracleChain(ChainParams(L=L, periodic=periodic, T=T, kappa=kappa, seed=23))
    t, _, _ = c.run_record(0, 500, 0)
    t, Es, Ms = c.run_record(t, 40000, 5)
    for a, b in [(Ep / N, Es / N), ((Mp / N) ** 2, (Ms / N) ** 2)]:
        ma, ea = binned_mean_err(a)
        mb, eb = binned_mean_err(b)
        assert abs(ma - mb) < 5 * math.hypot(ea, eb), (ma, ea, mb, eb)

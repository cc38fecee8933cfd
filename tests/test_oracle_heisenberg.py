"""Pins of the oracle's Heisenberg model (Eq. 6 with the full dipolar tensor, open
lattice), each against something other than the oracle itself:
- the pair energy is S_i^T T S_j with T = (D/r^3)(I - 3 rhat rhat^T) (numpy), and
  V^max = 2 D / r^3 is the largest eigenvalue magnitude of T, attained at S_i = rhat,
  S_j = -rhat;
- the proposal points are uniform on the sphere (moments and Archimedes' uniform z);
- the switching keeps each pair with probability 1 - P_ij of Eqs. (1)-(2), P computed
  here from the tensor (binomial test per pair at fixed spins);
- the energy and M_phi of Eq. (7) equal a brute-force numpy evaluation;
- an SCO chain samples the Boltzmann distribution of the full Hamiltonian: its <E>/N
  and <|M_phi|> agree with a plain single-spin Metropolis run of Eq. (6) written here
  in numpy, within statistical errors.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import ChainParams, OracleChain


def tensor(D, dx, dy):
    r = math.hypot(dx, dy)
    rh = np.array([dx / r, dy / r, 0.0])
    return D / r ** 3 * (np.eye(3) - 3.0 * np.outer(rh, rh))


def unit_vectors(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1)[:, None]


def test_pair_energy_is_the_dipolar_tensor_and_its_bound():
    rng = np.random.default_rng(1)
    D = 0.1
    for dx, dy in [(1, 0), (0, 1), (1, 1), (-2, 3), (5, -1), (0, 7)]:
        T = tensor(D, dx, dy)
        Jm = 2.0 * D / math.hypot(dx, dy) ** 3
        ev = np.linalg.eigvalsh(T)
        assert np.isclose(np.max(np.abs(ev)), Jm, rtol=1e-14)
        for si, sj in zip(unit_vectors(rng, 20), unit_vectors(rng, 20)):
            ref = si @ T @ sj
            got = oracle.pair_energy(si, sj, dx, dy, Jm)
            assert abs(got - ref) <= 1e-14 * Jm
            assert got <= Jm * (1 + 1e-15)
        r = math.hypot(dx, dy)
        rh = np.array([dx / r, dy / r, 0.0])
        assert np.isclose(oracle.pair_energy(rh, -rh, dx, dy, Jm), Jm, rtol=1e-14)
        assert np.isclose(oracle.pair_energy(rh, rh, dx, dy, Jm), -Jm, rtol=1e-14)


def test_sphere_points_are_uniform():
    c = OracleChain(ChainParams(L=4, periodic=False, T=1.0, model=1))
    pts = np.array([c.sphere_point(3, i, 0, 5) for i in range(40000)])
    n = len(pts)
    assert np.allclose(np.linalg.norm(pts, axis=1), 1.0, atol=1e-15)
    assert np.all(np.abs(pts.mean(axis=0)) < 4.0 / math.sqrt(3 * n))
    m2 = (pts ** 2).mean(axis=0)
    assert np.all(np.abs(m2 - 1 / 3) < 4.0 * math.sqrt(4 / 45 / n))
    # Archimedes: z is uniform on [-1, 1]
    counts, _ = np.histogram(pts[:, 2], bins=20, range=(-1, 1))
    e = n / 20
    chi2 = np.sum((counts - e) ** 2 / e)
    assert chi2 < 45.0  # 19 degrees of freedom, p ~ 1e-3


@pytest.mark.parametrize("T", [0.4, 1.2])
def test_switching_keeps_pairs_with_probability_one_minus_P(T):
    L, D, beta = 4, 0.1, 1.0 / T
    c = OracleChain(ChainParams(L=L, periodic=False, T=T, model=1, seed=5))
    S = c.spins3.copy()
    n = 8000
    counts = c.survival_counts(0, n)
    tab = c.tables()
    worst = 0.0
    chi2, dof = 0.0, 0
    for i in range(c.N):
        for m in range(c.K):
            j = c.partner(i, m)
            if j < 0:
                assert counts[i, m] == 0
                continue
            dx, dy = int(tab["dx"][m]), int(tab["dy"][m])
            V = S[i] @ tensor(D, dx, dy) @ S[j]
            Vmax = 2 * D / math.hypot(dx, dy) ** 3
            p = 1.0 - math.exp(beta * (V - Vmax))
            sd = math.sqrt(n * p * (1 - p)) + 1e-9
            z = (counts[i, m] - n * p) / sd
            worst = max(worst, abs(z))
            chi2 += z * z
            dof += 1
    assert worst < 5.0, worst
    assert chi2 < dof + 5 * math.sqrt(2 * dof), (chi2, dof)
    np.testing.assert_array_equal(c.spins3, S)  # switching alone moves no spin


def brute_energy(S, L, J, D):
    N = L * L
    xy = np.array([(v % L, v // L) for v in range(N)])
    E = 0.0
    for i in range(N):
        for j in range(i + 1, N):
            dx, dy = xy[j] - xy[i]
            if abs(dx) + abs(dy) == 1:
                E -= J * S[i] @ S[j]
            E += S[i] @ tensor(D, dx, dy) @ S[j]
    return E


def m_phi(S, L):
    c = (L - 1) / 2
    tot = 0.0
    for v in range(L * L):
        rx, ry = v % L - c, v // L - c
        d = math.hypot(rx, ry)
        if d > 0:
            tot += (S[v, 0] * ry - S[v, 1] * rx) / d
    return tot / (L * L)


@pytest.mark.parametrize("L", [5, 6])
def test_energy_and_m_phi_brute_force(L):
    c = OracleChain(ChainParams(L=L, periodic=False, T=1.0, model=1, seed=2))
    for t in range(3):
        c.step(t)
    S = c.spins3
    o = c.observables()
    ref = brute_energy(S, L, 1.0, 0.1)
    assert abs(o["E"] - ref) <= 1e-12 * abs(ref)
    assert abs(o["m_phi"] - m_phi(S, L)) <= 1e-14
    # a vortex has M_phi = 1 (every spin along the circulation direction)
    cc = (L - 1) / 2
    V = np.zeros((L * L, 3))
    for v in range(L * L):
        rx, ry = v % L - cc, v // L - cc
        d = math.hypot(rx, ry)
        V[v] = (ry / d, -rx / d, 0.0) if d > 0 else (0.0, 0.0, 1.0)
    c.spins3 = V
    n_centre = 1 if L % 2 else 0
    assert abs(c.observables()["m_phi"] - (L * L - n_centre) / (L * L)) <= 1e-14


def plain_metropolis(L, T, J, D, sweeps, rng):
    """Single-spin Metropolis of the full Hamiltonian of Eq. (6): the energy is
    bilinear, so a move S_i -> S' changes it by (S' - S_i) . b_i with
    b_i = -J sum_NN S_j + sum_j T_ij S_j."""
    N = L * L
    xy = np.array([(v % L, v // L) for v in range(N)])
    B = np.zeros((N, 3, N, 3))
    for i in range(N):
        for j in range(N):
            if i == j:
                continue
            dx, dy = xy[j] - xy[i]
            B[i, :, j, :] = tensor(D, dx, dy)
            if abs(dx) + abs(dy) == 1:
                B[i, :, j, :] -= J * np.eye(3)
    B = B.reshape(N, 3, 3 * N)
    S = unit_vectors(rng, N)
    Es, Ms = [], []
    E = 0.5 * S.reshape(-1) @ B.reshape(3 * N, 3 * N) @ S.reshape(-1)
    for _ in range(sweeps):
        props = unit_vectors(rng, N)
        us = rng.random(N)
        for i in range(N):
            b = B[i] @ S.reshape(-1)
            dE = (props[i] - S[i]) @ b
            if dE <= 0 or us[i] < math.exp(-dE / T):
                S[i] = props[i]
                E += dE
        Es.append(E / N)
        Ms.append(abs(m_phi(S, L)))
    return np.array(Es), np.array(Ms)


def mean_err(x, nb=50):
    b = x[: len(x) // nb * nb].reshape(nb, -1).mean(axis=1)
    return b.mean(), b.std(ddof=1) / math.sqrt(nb)


@pytest.mark.slow
@pytest.mark.parametrize("T", [0.5, 1.5])
def test_sco_chain_matches_plain_metropolis(T):
    L, J, D = 4, 1.0, 0.1
    n, burn = 30000, 2000
    rng = np.random.default_rng(11)
    Ep, Mp = plain_metropolis(L, T, J, D, n + burn, rng)
    c = OracleChain(ChainParams(L=L, periodic=False, T=T, J=J, D=D, model=1, seed=17))
    Es, Ms = [], []
    for t in range(n + burn):
        c.step(t)
        o = c.observables()
        Es.append(o["E"] / (L * L))
        Ms.append(abs(o["m_phi"]))
    for a, b in ((Ep[burn:], np.array(Es[burn:])), (Mp[burn:], np.array(Ms[burn:]))):
        ma, ea = mean_err(a)
        mb, eb = mean_err(b)
        assert abs(ma - mb) < 4.5 * math.hypot(ea, eb), (T, ma, ea, mb, eb)

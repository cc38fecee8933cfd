"""Pins of the oracle's displacement table: the half-displacement set, the dipolar
couplings J(d) of the perpendicular-Ising reduction of Eq. (6), the cumulative
coupling C_m and the switching/pseudo-interaction columns of Eqs. (2)-(3)."""
import itertools
import math

import numpy as np
import pytest

from oracle import ChainParams, OracleChain


@pytest.mark.parametrize("L,periodic", [(2, False), (3, False), (4, False), (5, False), (6, False),
                                        (8, False), (4, True), (6, True), (8, True)])
def test_half_set_is_a_bijection_onto_unordered_pairs(L, periodic):
    """Every unordered pair {i, j} is reached from exactly one (owner, m)."""
    c = OracleChain(ChainParams(L=L, periodic=periodic, T=1.0))
    N, K = c.N, c.K
    seen = {}
    for i in range(N):
        for m in range(K):
            j = c.partner(i, m)
            if j < 0:
                continue
            assert j != i
            key = (min(i, j), max(i, j))
            assert key not in seen, f"pair {key} reached twice: {seen[key]} and {(i, m)}"
            seen[key] = (i, m)
    assert len(seen) == N * (N - 1) // 2


def test_table_sorted_by_distance():
    c = OracleChain(ChainParams(L=16, periodic=True, T=1.0))
    t = c.tables()
    r2 = t["dx"].astype(np.int64) ** 2 + t["dy"].astype(np.int64) ** 2
    assert np.all(np.diff(r2) >= 0)
    assert np.all(np.diff(t["C"]) > 0)


@pytest.mark.parametrize("L", [5, 7])
def test_open_couplings_sum_over_all_pairs(L):
    """sum over owned pairs of J_m equals the brute-force sum of D / r_ij^3 over all
    pairs i < j of an open L x L lattice, and each J_m is D / |d_m|^3."""
    D = 0.1
    c = OracleChain(ChainParams(L=L, periodic=False, T=1.0, D=D))
    t = c.tables()
    owned = 0.0
    for i in range(c.N):
        for m in range(c.K):
            if c.partner(i, m) >= 0:
                owned += t["J"][m]
    pos = [(v % L, v // L) for v in range(L * L)]
    brute = 0.0
    for a, b in itertools.combinations(pos, 2):
        r = math.hypot(a[0] - b[0], a[1] - b[1])
        brute += D / r ** 3
    assert owned == pytest.approx(brute, rel=1e-13)
    r = np.hypot(t["dx"], t["dy"])
    np.testing.assert_allclose(t["J"], D / r ** 3, rtol=1e-15)


@pytest.mark.parametrize("L,n_images", [(4, 2), (6, 3), (8, 8)])
def test_periodic_couplings_tile_the_image_box(L, n_images):
    """Summed over every nonzero displacement class mod L (the half table counts the
    classes {d,-d} once, the three self-conjugate ones alone), plus the dropped
    self-image constant, the image sums add up to sum D/|v|^3 over every nonzero
    integer vector v of the box (-L/2 - nL, L/2 + nL]^2 -- enumerated directly."""
    D = 0.1
    c = OracleChain(ChainParams(L=L, periodic=True, T=1.0, D=D, n_images=n_images))
    t = c.tables()
    h = L // 2
    sc = ((t["dx"] == h) & (t["dy"] == 0)) | ((t["dy"] == h) & ((t["dx"] == 0) | (t["dx"] == h)))
    classes = 2.0 * t["J"][~sc].sum() + t["J"][sc].sum()
    assert int(2 * (~sc).sum() + sc.sum()) == L * L - 1
    ns = np.arange(-n_images, n_images + 1)
    self_images = sum(D / (math.hypot(a * L, b * L) ** 3) for a in ns for b in ns if (a, b) != (0, 0))
    lo, hi = -h - n_images * L + 1, h + n_images * L
    xs = np.arange(lo, hi + 1, dtype=np.float64)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    r2 = X * X + Y * Y
    r2[r2 == 0] = np.inf
    box = float(np.sum(D / (r2 * np.sqrt(r2))))
    assert classes + self_images == pytest.approx(box, rel=1e-12)


def test_periodic_box_sum_approaches_lattice_constant():
    """As the image box grows the total tends to D * 4 zeta(3/2) beta(3/2) =
    D * 9.0336217..., the square-lattice sum of 1/r^3; the truncated tail outside a
    square of half-width R is about 2 pi / R (times a shape factor of order one)."""
    from scipy.special import zeta

    # Dirichlet beta(3/2) = sum_k (-1)^k / (2k+1)^{3/2}, Hurwitz-zeta form
    beta32 = (zeta(1.5, 0.25) - zeta(1.5, 0.75)) / 2 ** 3
    S = 4 * zeta(1.5) * beta32
    assert S == pytest.approx(9.0336217, abs=2e-7)
    L, n = 8, 8
    c = OracleChain(ChainParams(L=L, periodic=True, T=1.0, D=1.0, n_images=n))
    t = c.tables()
    h = L // 2
    sc = ((t["dx"] == h) & (t["dy"] == 0)) | ((t["dy"] == h) & ((t["dx"] == 0) | (t["dx"] == h)))
    total = 2.0 * t["J"][~sc].sum() + t["J"][sc].sum()
    R = (n + 0.5) * L
    assert S - 1.5 * 2 * math.pi / R < total < S


def test_periodic_table_symmetries():
    """J depends only on |dx|, |dy| and is symmetric under dx <-> dy."""
    L = 12
    c = OracleChain(ChainParams(L=L, periodic=True, T=1.0))
    t = c.tables()
    J = {(int(a), int(b)): v for a, b, v in zip(t["dx"], t["dy"], t["J"])}
    for (a, b), v in J.items():
        for (x, y) in [(b, a), (-a, b), (a, -b), (-b, a)]:
            xr = ((x + L // 2 - 1) % L) - L // 2 + 1
            yr = y % L
            if (xr, yr) in J:
                assert J[(xr, yr)] == pytest.approx(v, rel=1e-14)


@pytest.mark.parametrize("kappa", [1.0, 1.5, 2.0])
def test_switching_and_pseudo_columns(kappa):
    """theta_m = (1 - P_par) / (1 - P_anti) and delta_m = Vbar(+1) - Vbar(-1), with
    P(s) = exp(beta (J s - kappa J)) (Eq. 2) and Vbar(s) = J s - T log(1 - P(s))
    (Eq. 3) evaluated here in extended precision from the same J_m."""
    import mpmath as mp  # noqa: F401  (scipy ships mpmath)

    T = 1.3
    c = OracleChain(ChainParams(L=8, periodic=True, T=T, kappa=kappa))
    t = c.tables()
    mp.mp.dps = 40
    beta = 1 / mp.mpf(T)
    for m in range(0, c.K, 3):
        Jm = mp.mpf(float(t["J"][m]))
        Ppar = mp.e ** (beta * (Jm - kappa * Jm))
        Panti = mp.e ** (beta * (-Jm - kappa * Jm))
        theta = (1 - Ppar) / (1 - Panti)
        assert float(t["C"][m]) == pytest.approx(float(np.sum(t["J"][: m + 1])), rel=1e-14)
        if kappa == 1.0:
            assert t["theta"][m] == 0.0
            assert math.isinf(t["delta"][m])
            continue
        vbar_p = Jm - mp.mpf(T) * mp.log(1 - Ppar)
        vbar_m = -Jm - mp.mpf(T) * mp.log(1 - Panti)
        assert t["theta"][m] == pytest.approx(float(theta), rel=1e-14)
        assert t["delta"][m] == pytest.approx(float(vbar_p - vbar_m), rel=1e-13)


@pytest.mark.parametrize("L,periodic,kappa", [(12, True, 2.0), (9, False, 1.0), (10, False, 3.0)])
def test_set_temperature_equals_a_fresh_chain(L, periodic, kappa):
    """A new temperature rebuilds exactly the columns a chain created at that
    temperature has (Eqs. 2-3 at the new beta), and the chain then runs as one that
    started at the new temperature from the same spins."""
    import oracle

    a = oracle.OracleChain(oracle.ChainParams(L=L, periodic=periodic, T=1.25, kappa=kappa))
    a.step(0)
    a.set_temperature(0.45)
    b = oracle.OracleChain(oracle.ChainParams(L=L, periodic=periodic, T=0.45, kappa=kappa), init_spins=a.spins)
    ta, tb = a.tables(), b.tables()
    for k in ta:
        np.testing.assert_array_equal(ta[k], tb[k], err_msg=k)
    for t in range(1, 4):
        a.step(t)
        b.step(t)
    np.testing.assert_array_equal(a.spins, b.spins)
    with pytest.raises(ValueError):
        a.set_temperature(0.0)

"""Pins of the oracle's bond graph (CSR) and of its Kuhn-Wattenhofer colouring.

Colouring pins: the result is a proper colouring of the union of the exchange
lattice and the surviving bonds with colours 0..Delta (Sec. 2.3.1); each level
takes at most Delta+1 rounds and there are M = ceil(log2(ceil(N/(Delta+1))))
levels, so the running time is at most (Delta+1) M (Eq. 5); and the colours agree
with an independent transcription of Sec. 2.3.3 written in the paper's own terms:
1-based global colours, groups G_p(k) defined by colour ranges, colour reduction
inside each group by rule (2)' and the remapping of R_p(k) into
[1+(k-1)(Delta+1), k(Delta+1)].
"""
import math

import numpy as np
import pytest

from oracle import ChainParams, OracleChain


def nn_list(L, periodic, v):
    x, y = v % L, v // L
    if periodic:
        return [y * L + (x + 1) % L, y * L + (x - 1) % L, ((y + 1) % L) * L + x, ((y - 1) % L) * L + x]
    out = []
    if x + 1 < L:
        out.append(v + 1)
    if x > 0:
        out.append(v - 1)
    if y + 1 < L:
        out.append(v + L)
    if y > 0:
        out.append(v - L)
    return out


def union_adjacency(c: OracleChain):
    rp, col, _ = c.csr()
    L, per = c.params.L, c.params.periodic
    adj = []
    for v in range(c.N):
        s = set(nn_list(L, per, v))
        s.update(int(u) for u in col[rp[v]:rp[v + 1]])
        adj.append(s)
    return adj


@pytest.mark.parametrize("L,periodic,T,kappa", [(32, False, 1.0, 1.0), (32, True, 0.8, 2.0),
                                                (64, True, 1.2, 1.0)])
def test_csr_invariants(L, periodic, T, kappa):
    c = OracleChain(ChainParams(L=L, periodic=periodic, T=T, kappa=kappa))
    c.switch(0)
    rp, col, at = c.csr()
    E = len(col) // 2
    assert rp[0] == 0 and rp[-1] == 2 * E
    t = c.tables()
    pairs = set()
    for v in range(c.N):
        row = col[rp[v]:rp[v + 1]]
        assert np.all(np.diff(row) > 0), "rows ascending, no duplicate"
        for u, m in zip(row, at[rp[v]:rp[v + 1]]):
            pairs.add((v, int(u), int(m)))
            # the attribute is the displacement index joining the two sites
            assert c.partner(v, int(m)) == u or c.partner(int(u), int(m)) == v
    for v, u, m in pairs:
        assert (u, v, m) in pairs, "symmetric"
    o, n, m = c.survivors()
    assert len(o) == E


def paper_kw(adj, N, delta):
    """Sec. 2.3.3 transcribed with the paper's numbering; returns 0-based colours."""
    q = delta + 1
    col = [v + 1 for v in range(N)]  # initial N-colouring, colours 1..N
    groups = math.ceil(N / q)
    M = 0
    while 2 ** M < groups:
        M += 1
    rounds = []
    for p in range(1, M + 1):
        # G_p(k) = G_{p-1}(2k-1) u G_{p-1}(2k); before the reduction the vertices of
        # G_{p-1}(j) hold colours in [1+(j-1)q, jq]
        new = list(col)
        level_rounds = 0
        n_groups = math.ceil(groups / 2 ** p)
        for k in range(1, n_groups + 1):
            lo_grp, hi_grp = 2 * k - 1, 2 * k
            members = [v for v in range(N) if (v // q) // 2 ** (p - 1) + 1 in (lo_grp, hi_grp)]
            mset = set(members)
            c_lo = 1 + (lo_grp - 1) * q  # the group's colours lie in [c_lo, c_lo + 2q)
            # colour reduction 2q -> q inside the group: the colours of the upper
            # half-group, c_lo+q .. c_lo+2q-1, are eliminated by rule (2)'
            cur = {v: col[v] for v in members}
            r = 0
            while any(cur[v] >= c_lo + q for v in members):
                r += 1
                nxt = dict(cur)
                for v in members:
                    if cur[v] < c_lo + q:
                        continue
                    nbr = [u for u in adj[v] if u in mset]
                    if any(cur[u] >= c_lo + q and cur[u] > cur[v] for u in nbr):
                        continue  # not locally maximal
                    taken = {cur[u] for u in nbr}
                    nc = next(cc for cc in range(c_lo, c_lo + q) if cc not in taken)
                    nxt[v] = nc
                cur = nxt
            level_rounds = max(level_rounds, r)
            # remap R_p(k): [c_lo, c_lo+q) -> [1+(k-1)q, kq]
            for v in members:
                new[v] = cur[v] - c_lo + 1 + (k - 1) * q
        col = new
        rounds.append(level_rounds)
    return [x - 1 for x in col], M, rounds


@pytest.mark.parametrize("L,periodic,T,kappa,t", [(8, False, 1.0, 1.0, 0), (12, True, 1.0, 2.0, 1),
                                                  (16, True, 0.8, 2.0, 2), (10, False, 0.8, 2.0, 3)])
def test_kw_matches_paper_transcription(L, periodic, T, kappa, t):
    c = OracleChain(ChainParams(L=L, periodic=periodic, T=T, kappa=kappa, seed=3))
    c.switch(t)
    c.color()
    adj = union_adjacency(c)
    delta = max(len(a) for a in adj)
    ref, M, rounds = paper_kw(adj, c.N, delta)
    o = c.observables(dipolar="none")
    assert o["delta_union"] == delta
    assert o["kw_levels"] == M
    np.testing.assert_array_equal(c.colors(), np.array(ref))
    kr = c.kw_rounds()
    assert list(kr[1:M + 1]) == rounds


@pytest.mark.parametrize("L,periodic,T,kappa", [(32, False, 1.0, 1.0), (32, False, 1.0, 2.0),
                                                (64, True, 0.8, 2.0), (48, True, 2.0, 1.0)])
def test_kw_proper_palette_and_round_bound(L, periodic, T, kappa):
    c = OracleChain(ChainParams(L=L, periodic=periodic, T=T, kappa=kappa))
    for t in range(3):
        c.switch(t)
        c.color()
        adj = union_adjacency(c)
        col = c.colors()
        delta = max(len(a) for a in adj)
        q = delta + 1
        assert col.min() >= 0 and col.max() < q
        for v in range(c.N):
            for u in adj[v]:
                assert col[u] != col[v]
        o = c.observables(dipolar="none")
        M = math.ceil(math.log2(math.ceil(c.N / q)))
        assert o["kw_levels"] == M
        kr = c.kw_rounds()
        assert np.all(kr[1:M + 1] <= q)
        assert o["kw_rounds"] == kr.sum() <= q * M
        c.sweep(t)


def test_kw_single_group():
    """N <= Delta+1: no level at all, the initial colours are already in range."""
    c = OracleChain(ChainParams(L=2, periodic=False, T=0.3, kappa=2.0))
    c.switch(0)
    c.color()
    o = c.observables(dipolar="none")
    if o["q"] >= 4:
        assert o["kw_levels"] == 0
        np.testing.assert_array_equal(c.colors(), np.arange(4))


# ----------------------------------------------------------------- colouring variants
# Sec. 2.3.2 gives two rules for one round of basic colour reduction: step (2)
# recolours the vertices of the largest colour alpha, step (2)' every vertex whose
# colour is locally maximal.  In both, a pending vertex recolours only after all of its
# pending neighbours of larger colour have, and it then sees their new colours, so the
# two rules yield the same colours and differ only in the number of rounds.

@pytest.mark.parametrize("L,periodic,T,kappa", [(12, True, 1.0, 2.0), (10, False, 0.8, 1.0),
                                                (16, True, 0.5, 3.0)])
def test_kw_rule2_gives_the_same_colours_in_q_rounds_per_level(L, periodic, T, kappa):
    c = OracleChain(ChainParams(L=L, periodic=periodic, T=T, kappa=kappa))
    c.step(0)
    c.switch(1)
    c.color()
    o = c.observables(dipolar="none")
    col2, r2 = c.colors_rule2()
    np.testing.assert_array_equal(col2, c.colors())
    q, M = o["q"], o["kw_levels"]
    assert r2 == q * M, "step (2): alpha runs from 2q-1 down to q in every level (Eq. 5)"
    assert o["kw_rounds"] <= r2


def greedy_decreasing(adj, N, q):
    """Sequential greedy colouring in decreasing vertex order: vertices 0..q-1 keep
    their index as colour, every other vertex takes the smallest colour unused by its
    neighbours (textbook first-fit)."""
    col = list(range(N))
    for v in range(N - 1, q - 1, -1):
        used = {col[u] for u in adj[v] if col[u] < q}
        col[v] = next(k for k in range(q) if k not in used)
    return col


def decreasing_depth(adj, N, q):
    """Longest chain of pending vertices (index >= q) joined by edges along which the
    index increases: the number of synchronous rounds of rule (2)'."""
    depth = [0] * N
    best = 0
    for v in range(N - 1, q - 1, -1):
        d = 1 + max([depth[u] for u in adj[v] if u > v and u >= q], default=0)
        depth[v] = d
        best = max(best, d)
    return best


@pytest.mark.parametrize("L,periodic,T,kappa", [(8, True, 1.0, 2.0), (9, False, 0.7, 1.0),
                                                (16, True, 1.2, 1.0), (20, False, 0.9, 2.0)])
def test_whole_graph_reduction_is_first_fit_in_decreasing_order(L, periodic, T, kappa):
    """Basic colour reduction on the whole union graph (no KW groups) with rule (2)'
    gives the first-fit colouring in decreasing site order, in as many rounds as the
    longest increasing-index chain of pending vertices; step (2) gives the same colours
    in N - (Delta+1) rounds."""
    c = OracleChain(ChainParams(L=L, periodic=periodic, T=T, kappa=kappa, coloring=2))
    c.step(0)
    c.switch(1)
    c.color()
    o = c.observables(dipolar="none")
    adj = union_adjacency(c)
    delta = max(len(a) for a in adj)
    q = delta + 1
    assert o["q"] == q and o["kw_levels"] == 1
    colours = c.colors()
    np.testing.assert_array_equal(colours, greedy_decreasing(adj, c.N, q))
    assert o["kw_rounds"] == decreasing_depth(adj, c.N, q)
    assert all(colours[v] != colours[u] for v in range(c.N) for u in adj[v])
    if c.N <= 100:
        col2, r2 = c.colors_rule2(whole=True)
        np.testing.assert_array_equal(col2, colours)
        assert r2 == c.N - q


@pytest.mark.parametrize("L,periodic,T,kappa", [(16, True, 1.0, 2.0), (12, False, 0.6, 3.0),
                                                (32, True, 1.2, 1.0)])
def test_checkerboard_product_colouring(L, periodic, T, kappa):
    """Colour 2 c + ((x + y) mod 2), c a KW colouring of the bonds alone with
    q = max(Delta_bonds + 1, 2): proper on the union graph, below 2 q, and c equals a
    KW colouring of the bond graph by the paper transcription."""
    c = OracleChain(ChainParams(L=L, periodic=periodic, T=T, kappa=kappa, coloring=1))
    c.step(0)
    c.switch(1)
    c.color()
    o = c.observables(dipolar="none")
    rp, col, _ = c.csr()
    bonds = [set(int(u) for u in col[rp[v]:rp[v + 1]]) for v in range(c.N)]
    q = max(max(len(b) for b in bonds) + 1, 2)
    assert o["q"] == q
    colours = c.colors()
    assert colours.max() < 2 * q and colours.min() >= 0
    adj = union_adjacency(c)
    assert all(colours[v] != colours[u] for v in range(c.N) for u in adj[v])
    par = (np.arange(c.N) % L + np.arange(c.N) // L) % 2
    np.testing.assert_array_equal(colours % 2, par)
    ref, M, rounds = paper_kw(bonds, c.N, q - 1)
    np.testing.assert_array_equal(colours // 2, np.asarray(ref))
    assert o["kw_levels"] == M

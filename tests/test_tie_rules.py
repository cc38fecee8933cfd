"""The parity harness's near-tie rule (CPU): which differences one step's tied
decisions may account for, and the oracle's list of those decisions."""
import numpy as np

import oracle
from tests.parity import tie_explains


def test_graph_differences_need_a_tied_switching_decision():
    s = np.ones(16, np.int8)
    assert tie_explains(["csr"], [(1, 3)], s, s, 1, True)
    assert tie_explains(["row_ptr", "spins"], [(1, 3)], s, s, 1, True)
    assert not tie_explains(["colors"], [(2, 3)], s, s, 1, True)
    assert not tie_explains(["csr"], [], s, s, 1, True)


def test_spin_differences_need_a_tied_sweep_decision_at_a_differing_site():
    a = np.ones(16, np.int8)
    b = a.copy()
    b[5] = -1
    assert tie_explains(["spins"], [(2, 5)], a, b, 1, True)
    assert not tie_explains(["spins"], [(2, 4)], a, b, 1, True)
    assert not tie_explains(["spins"], [(1, 5)], a, b, 1, True)  # graph compared and equal
    assert tie_explains(["spins"], [(1, 5)], a, b, 1, False)  # graph not compared
    assert tie_explains(["spins"], [(2, 4)], a, b, 3, True)  # a later sweep may undo it
    a3 = np.zeros((16, 3))
    b3 = a3.copy()
    b3[7, 2] = 1e-16
    assert tie_explains(["spins"], [(2, 7)], a3, b3, 1, True)
    assert not tie_explains(["spins"], [(2, 6)], a3, b3, 1, True)


def test_oracle_lists_every_tie_of_the_step():
    c = oracle.OracleChain(oracle.ChainParams(L=32, periodic=True, T=1.1, kappa=2.0))
    for t in range(6):
        before = c.observables(dipolar="none")["near_ties"]
        c.step(t)
        ties = c.ties()
        assert len(ties) == c.observables(dipolar="none")["near_ties"] - before
        assert all(k in (1, 2) and 0 <= v < c.N for k, v in ties)

"""Seeded synthetic workloads (chain parameters only; no arithmetic of the method).

Every input of the SCO step is synthetic: a lattice size, boundary condition,
temperature, kappa, Philox seed and chain id per chain; the initial spins are then
drawn by each implementation from its own Philox4x32-10.  The batched workload draws
each chain's L and T with the small pure-Python Philox below (counter (0, 0, 0, 5),
key (seed, chain)).
"""
from __future__ import annotations

M0, M1, W0, W1 = 0xD2511F53, 0xCD9E8D57, 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32-10 (Salmon et al., SC'11), pure Python."""
    c0, c1, c2, c3 = [int(x) & MASK for x in ctr]
    k0, k1 = [int(x) & MASK for x in key]
    for r in range(10):
        if r:
            k0, k1 = (k0 + W0) & MASK, (k1 + W1) & MASK
        p0, p1 = M0 * c0, M1 * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0) & MASK, p1 & MASK, ((p0 >> 32) ^ c3 ^ k1) & MASK, p0 & MASK
    return c0, c1, c2, c3


def _u52(lo, hi):
    return (float(((hi << 32) | lo) >> 12) + 0.5) * 2.0 ** -52


def chain(L, periodic, T, kappa=1.0, chain_id=0, seed=1, n_sw=1, precision=0, J=1.0, D=0.1,
          n_images=8):
    return dict(L=L, periodic=periodic, T=T, kappa=kappa, chain_id=chain_id, seed=seed, n_sw=n_sw,
                precision=precision, J=J, D=D, n_images=n_images)


def small_open(kappa=1.0):
    """L=32 open, T=1.0, seed 1, 1000 SCO steps."""
    return [chain(32, False, 1.0, kappa)], 1000


def medium_periodic(kappa=1.0):
    """L=256 periodic, T in {0.8, 1.2, 2.0}, 2000 SCO steps."""
    return [chain(256, True, T, kappa, chain_id=i) for i, T in enumerate((0.8, 1.2, 2.0))], 2000


def large_periodic(kappa=1.0, n_sw=1):
    """L=2304 periodic (N = 5,308,416), T=1.2, single chain, 200 SCO steps."""
    return [chain(2304, True, 1.2, kappa, n_sw=n_sw)], 200


def batched(n_chains=64, seed=1, kappa=1.0):
    """64 chains, L from {64,128,256,512,1024} and T uniform in [0.8, 2.5] by Philox."""
    out = []
    for c in range(n_chains):
        w = philox4x32_10((0, 0, 0, 5), (seed, c))
        L = (64, 128, 256, 512, 1024)[w[0] % 5]
        T = 0.8 + 1.7 * _u52(w[2], w[3])
        out.append(chain(L, True, T, kappa, chain_id=c, seed=seed))
    return out


def mixed_precision(precision=1, kappa=2.0):
    """8 chains at L=2304 plus one at L=4096, T = 1.0 + 0.5 c / 8."""
    out = []
    for c in range(9):
        L = 4096 if c == 8 else 2304
        out.append(chain(L, True, 1.0 + 0.5 * c / 8, kappa, chain_id=c, precision=precision))
    return out

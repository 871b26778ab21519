"""Pins of the oracle's census outputs (main text, Fig. 1F: the state the
environment responds to, and the counters the throughput metric is built
on), each recomputed outside the oracle:

- sum_z, sum_z2: phenotypes recomputed from the genomes by the additive map
  z = sum_l e_l (b0_l + b1_l - 1) (eqn. S2, phenotype value, as a biallelic
  midpoint sum), summed in Python integers;
- updates: the running sum of N_t x L over the generations, from the census
  sizes read after every step;
- near_ties: survival draws with |x 2^-32 - p| < 1e-6 and 0 < p < 1,
  recounted from the SURVIVE words (Philox4x32-10 evaluated here with numpy,
  itself checked against the published known-answer vectors) and p
  evaluated independently as v(z) s(N) with numpy's exp.
"""
import numpy as np
import pytest

import oracle
from conftest import read_kat

M0, M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
MASK = np.uint64(0xFFFFFFFF)
ST_SURVIVE = 3


def philox_np(c0, c1, c2, c3, key):
    """Philox4x32-10 (Salmon et al., SC'11) over arrays of counters."""
    x = [np.asarray(c, dtype=np.uint64) & MASK for c in (c0, c1, c2, c3)]
    x = np.broadcast_arrays(*x)
    x = [a.copy() for a in x]
    k0, k1 = int(key[0]), int(key[1])
    for _ in range(10):
        pa = x[0] * M0
        pb = x[2] * M1
        n0 = (pb >> np.uint64(32)) ^ x[1] ^ np.uint64(k0)
        n2 = (pa >> np.uint64(32)) ^ x[3] ^ np.uint64(k1)
        x = [n0, pb & MASK, n2, pa & MASK]
        k0 = (k0 + 0x9E3779B9) & 0xFFFFFFFF
        k1 = (k1 + 0xBB67AE85) & 0xFFFFFFFF
    return [a.astype(np.uint32) for a in x]


def test_numpy_philox_matches_published_vectors():
    for ctr, key, want in read_kat():
        got = philox_np(*[np.array([c]) for c in ctr], key)
        assert [int(g[0]) for g in got] == want


def phenotypes_from_genomes(words, L, effects=None):
    """z of every individual from packed genomes, one locus at a time."""
    n = words.shape[0]
    W = (L + 31) // 32
    w = words.reshape(n, 2, W)
    e = np.ones(L, np.int64) if effects is None else np.asarray(effects, np.int64)
    z = np.zeros(n, np.int64)
    for l in range(L):
        b0 = (w[:, 0, l // 32] >> np.uint32(l % 32)) & np.uint32(1)
        b1 = (w[:, 1, l // 32] >> np.uint32(l % 32)) & np.uint32(1)
        z += e[l] * (b0.astype(np.int64) + b1.astype(np.int64) - 1)
    return z


def near_tie_count(z, seed, t, c3, theta, omega, s=1.0):
    n = len(z)
    x = philox_np(np.arange(n), ST_SURVIVE << 24, t, c3, (seed & 0xFFFFFFFF, seed >> 32))[0]
    d = np.asarray(z, float) - theta
    p = np.exp(-(d * d) / (2.0 * omega * omega)) * s if omega > 0 else np.full(n, s)
    u = x.astype(np.float64) / 4294967296.0
    return int(np.sum((p > 0) & (p < 1) & (np.abs(u - p) < 1e-6)))


@pytest.mark.parametrize("regime", ["wf", "poisson"])
def test_census_sums_and_updates(regime):
    L = 64 if regime == "wf" else 96
    eff = None if regime == "wf" else np.random.default_rng(4).integers(-4, 5, L).astype(np.int8)
    kw = dict(seed=11, n0=3000, n_loci=L, r=0.1, mu=1e-3, theta=0.0, omega=12.0)
    if regime == "poisson":
        kw.update(regime=1, capacity=6000, K=3000.0, fecundity=2.2, effects=eff, omega=40.0)
    pop = oracle.OraclePop(**kw)
    updates = 0
    for t in range(8):
        if t:
            pop.step(1)
            updates += pop.n * L
        st = pop.stats()
        z = phenotypes_from_genomes(pop.genomes(), L, eff)
        assert st["n"] == len(z)
        assert st["sum_z"] == int(z.sum())
        assert st["sum_z2"] == int((z * z).sum())
        assert st["updates"] == updates
        assert st["generation"] == t


def test_near_ties_recounted_from_survive_words():
    # 4e6 survival draws under Gaussian viability; a near tie has chance
    # about 2e-6 per draw with 0 < p < 1, so a handful are expected
    seed, N, L, theta, omega, G = 3, 200000, 32, 0.0, 6.0, 20
    pop = oracle.OraclePop(seed=seed, replicate_id=5, n0=N, n_loci=L, r=0.5, mu=1e-3, theta=theta, omega=omega)
    c3 = 5 << 12
    want = 0
    for t in range(G):
        want += near_tie_count(pop.phenotypes(), seed, t, c3, theta, omega)
        pop.step(1)
    assert pop.stats()["near_ties"] == want
    assert want >= 3  # the check must see ties, not only their absence


def test_near_ties_with_density_factor():
    seed, L, theta, omega, K, lam = 9, 32, 0.0, 5.0, 150000.0, 2.0
    pop = oracle.OraclePop(seed=seed, regime=1, n0=150000, capacity=400000, n_loci=L, r=0.3, mu=0.0, theta=theta,
                           omega=omega, K=K, fecundity=lam)
    want = 0
    for t in range(12):
        n = pop.n
        s = 1.0 / (1.0 + (lam - 1.0) * n / K)
        want += near_tie_count(pop.phenotypes(), seed, t, 0, theta, omega, s)
        pop.step(1)
    assert pop.stats()["near_ties"] == want
    assert want >= 1

"""Pins of the oracle's patches and backward migration (Supplementary
Information S3: a P-patch metacommunity, each patch linked by migration to
its neighbouring patches), read as a ring of Wright-Fisher patches whose
offspring descend, with probability m, from parents in one of the two
neighbouring patches.

What the mathematics fixes: with selection off and every adult surviving,
E[p_k(t+1)] = (1 - 2 mu) [(1 - m) p_k + m/2 (p_{k-1} + p_{k+1})] + mu at
every locus (two neighbours at distance one; P = 2 makes them one patch);
the fraction of migrant offspring is m, split evenly between the sides;
m = 0 leaves every patch an independent replicate; a patch that loses all
its adults is refilled from its neighbours and keeps its census.
"""
import numpy as np
import pytest
from scipy import stats

import oracle


def pack(alleles):
    """(n, 2, L) uint8 -> (n, 2, W) uint32."""
    n, _, L = alleles.shape
    W = (L + 31) // 32
    words = np.zeros((n, 2, W), np.uint32)
    for l in range(L):
        words[:, :, l // 32] |= alleles[:, :, l].astype(np.uint32) << np.uint32(l % 32)
    return words


def test_zero_migration_patch_is_an_independent_replicate():
    kw = dict(seed=3, replicate_id=5, n0=200, n_loci=96, mu=1e-3, r=0.05, omega=6.0)
    ring = oracle.OraclePop(n_patches=3, migration=0.0, **kw)
    alone = oracle.OraclePop(**kw)
    ring.step(6)
    alone.step(6)
    assert np.array_equal(ring.genomes(0), alone.genomes())
    assert ring.stats(0) == alone.stats()
    # the other patches draw from their own counter fields
    assert not np.array_equal(ring.genomes(1), ring.genomes(0))
    mom, dad, src = ring.parents(2, with_source=True)
    assert np.all(src == 2)


def test_one_patch_ignores_the_migration_rate():
    kw = dict(seed=8, n0=150, n_loci=64, mu=1e-3, r=0.5, omega=8.0)
    a = oracle.OraclePop(n_patches=1, migration=0.7, **kw)
    b = oracle.OraclePop(**kw)
    a.step(5)
    b.step(5)
    assert np.array_equal(a.genomes(), b.genomes())
    assert a.stats() == b.stats()


@pytest.mark.parametrize("P,m,mu", [(4, 0.2, 0.01), (2, 0.3, 0.0), (5, 1.0, 0.0)])
def test_expected_allele_frequency_after_one_generation(P, m, mu):
    N, L, R = 600, 128, 12
    g = np.random.default_rng(100 + P)
    freq = g.uniform(0.05, 0.95, P)
    dev = np.zeros((R, P))
    for rep in range(R):
        pop = oracle.OraclePop(seed=21, replicate_id=rep, n0=N, n_loci=L, r=0.5, mu=mu, omega=0.0,
                               n_patches=P, migration=m)
        p = np.zeros(P)
        for k in range(P):
            a = (g.random((N, 2, L)) < freq[k]).astype(np.uint8)
            p[k] = a.mean()
            pop.set_genomes(pack(a), generation=0, patch=k)
        pop.step(1)
        for k in range(P):
            nb = p[(k - 1) % P] + p[(k + 1) % P]
            expect = (1 - 2 * mu) * ((1 - m) * p[k] + m / 2 * nb) + mu
            dev[rep, k] = pop.alleles(k).mean() - expect
    z = dev.mean(axis=0) / (dev.std(axis=0, ddof=1) / np.sqrt(R))
    assert np.all(np.abs(z) < 4.5), (dev.mean(axis=0), z)


def test_migrant_fraction_and_sides():
    P, N, m = 5, 400, 0.15
    pop = oracle.OraclePop(seed=12, n0=N, n_loci=32, omega=0.0, n_patches=P, migration=m)
    migrants = left = total = 0
    for _ in range(6):
        pop.step(1)
        for k in range(P):
            _, _, src = pop.parents(k, with_source=True)
            total += src.size
            migrants += int(np.sum(src != k))
            left += int(np.sum(src == (k - 1) % P))
            assert np.all((src == k) | (src == (k - 1) % P) | (src == (k + 1) % P))
    assert stats.binomtest(migrants, total, m).pvalue > 1e-4
    assert stats.binomtest(left, migrants, 0.5).pvalue > 1e-4


def test_parents_are_survivors_of_their_source_patch():
    P, N = 4, 300
    pop = oracle.OraclePop(seed=14, n0=N, n_loci=64, omega=3.0, r=0.3, n_patches=P, migration=0.3)
    pop.step(3)
    surv = [set(pop.survivors(k).tolist()) for k in range(P)]
    assert all(len(s) < N for s in surv)  # selection removed some adults
    for k in range(P):
        mom, dad, src = pop.parents(k, with_source=True)
        for a, b, s in zip(mom.tolist(), dad.tolist(), src.tolist()):
            assert a in surv[s] and b in surv[s]


def test_a_dead_patch_is_refilled_from_its_neighbours():
    P, N, L = 5, 300, 64
    pop = oracle.OraclePop(seed=30, n0=N, n_loci=L, omega=0.5, theta=0.0, n_patches=P, migration=0.05)
    ones = np.ones((N, 2, L), np.uint8)
    het = np.zeros((N, 2, L), np.uint8)
    het[:, 1, :] = 1  # z = 0: survives surely at theta = 0
    pop.set_genomes(pack(ones), generation=0, patch=0)  # z = L: dies surely
    for k in range(1, P):
        pop.set_genomes(pack(het), generation=0, patch=k)
    pop.step(1)
    assert pop.stats(0)["n_survivors"] == 0
    assert pop.stats(0)["n"] == N  # the census is kept
    _, _, src = pop.parents(0, with_source=True)
    assert np.all((src == 1) | (src == P - 1))
    assert stats.binomtest(int(np.sum(src == 1)), src.size, 0.5).pvalue > 1e-4
    # the neighbours' offspring never descend from the empty patch
    for k in (1, P - 1):
        _, _, s2 = pop.parents(k, with_source=True)
        assert not np.any(s2 == 0)


def test_patches_without_any_source_go_extinct():
    P, N, L = 3, 100, 32
    pop = oracle.OraclePop(seed=31, n0=N, n_loci=L, omega=0.5, theta=0.0, n_patches=P, migration=0.1)
    ones = np.ones((N, 2, L), np.uint8)
    for k in range(P):
        pop.set_genomes(pack(ones), generation=4, patch=k)
    pop.step(2)
    tot = pop.total_stats()
    assert tot["n"] == 0 and tot["extinct"] == 1 and tot["generation"] == 6
    assert all(pop.stats(k)["extinct"] == 1 for k in range(P))


def test_patches_need_wright_fisher():
    with pytest.raises(ValueError):
        oracle.OraclePop(regime=1, n0=10, capacity=20, fecundity=2.0, n_patches=2, migration=0.1)

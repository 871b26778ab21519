"""Pins of the oracle's biased island dispersal (Supplementary S3, Fig. S3
caption: a share pi of the migrants from a patch returns to its patch of
origin), read backwards: offspring of patch k are would-be migrants with
probability m; a share pi of those descend from home after all, the others
from a patch drawn uniformly among the other P - 1.

What the mathematics fixes: with selection off and every adult surviving,
E[p_k(t+1)] = (1 - 2 mu) [(1 - m') p_k + m'/(P - 1) sum_{i != k} p_i] + mu
with the effective rate m' = m (1 - pi); the migrant fraction is m'; the
source of a migrant is uniform over the other patches; pi = 1 is no
migration at all; a patch whose adults all died keeps its census while any
patch has survivors, its offspring descending from the first patch with
survivors after the drawn one in ring order.
"""
import numpy as np
import pytest
from scipy import stats

import oracle
from test_oracle_migration import pack


@pytest.mark.parametrize("P,m,pi,mu", [(5, 0.3, 0.4, 0.01), (3, 0.5, 0.0, 0.0), (6, 1.0, 0.5, 0.0)])
def test_expected_allele_frequency_after_one_generation(P, m, pi, mu):
    N, L, R = 500, 128, 12
    g = np.random.default_rng(300 + P)
    freq = g.uniform(0.05, 0.95, P)
    mp = m * (1 - pi)
    dev = np.zeros((R, P))
    for rep in range(R):
        pop = oracle.OraclePop(seed=41, replicate_id=rep, n0=N, n_loci=L, r=0.5, mu=mu, omega=0.0,
                               n_patches=P, migration=m, dispersal=1, home_return=pi)
        p = np.zeros(P)
        for k in range(P):
            a = (g.random((N, 2, L)) < freq[k]).astype(np.uint8)
            p[k] = a.mean()
            pop.set_genomes(pack(a), generation=0, patch=k)
        pop.step(1)
        for k in range(P):
            others = (p.sum() - p[k]) / (P - 1)
            expect = (1 - 2 * mu) * ((1 - mp) * p[k] + mp * others) + mu
            dev[rep, k] = pop.alleles(k).mean() - expect
    z = dev.mean(axis=0) / (dev.std(axis=0, ddof=1) / np.sqrt(R))
    assert np.all(np.abs(z) < 4.5), (dev.mean(axis=0), z)


@pytest.mark.parametrize("pi", [0.0, 0.4])
def test_migrant_fraction_and_uniform_sources(pi):
    P, N, m = 6, 500, 0.25
    pop = oracle.OraclePop(seed=13, n0=N, n_loci=32, omega=0.0, n_patches=P, migration=m, dispersal=1,
                           home_return=pi)
    migrants = total = 0
    offset = np.zeros(P - 1)  # source - home (mod P), 1 .. P - 1
    for _ in range(8):
        pop.step(1)
        for k in range(P):
            _, _, src = pop.parents(k, with_source=True)
            total += src.size
            mig = src[src != k].astype(np.int64)
            migrants += mig.size
            np.add.at(offset, (mig - k) % P - 1, 1)
    assert stats.binomtest(migrants, total, m * (1 - pi)).pvalue > 1e-4
    assert stats.chisquare(offset).pvalue > 1e-4


def test_all_migrants_returning_home_is_no_migration():
    kw = dict(seed=17, n0=200, n_loci=96, mu=1e-3, r=0.05, omega=6.0, n_patches=4)
    island = oracle.OraclePop(migration=0.6, dispersal=1, home_return=1.0, **kw)
    closed = oracle.OraclePop(migration=0.0, **kw)
    island.step(5)
    closed.step(5)
    for k in range(4):
        assert np.array_equal(island.genomes(k), closed.genomes(k))
        assert island.stats(k) == closed.stats(k)


def test_ring_and_island_share_their_first_word():
    # the same would-be migrants in both dispersal models: MIGRATE word 0
    kw = dict(seed=19, n0=300, n_loci=32, omega=0.0, n_patches=5, migration=0.2)
    ring = oracle.OraclePop(**kw)
    island = oracle.OraclePop(dispersal=1, home_return=0.0, **kw)
    ring.step(1)
    island.step(1)
    for k in range(5):
        assert np.array_equal(ring.parents(k, with_source=True)[2] != k,
                              island.parents(k, with_source=True)[2] != k)


def test_a_dead_patch_is_refilled_from_the_next_live_patch():
    P, N, L = 6, 300, 64
    pop = oracle.OraclePop(seed=33, n0=N, n_loci=L, omega=0.5, theta=0.0, n_patches=P, migration=0.1,
                           dispersal=1, home_return=0.3)
    ones = np.ones((N, 2, L), np.uint8)  # z = L: dies surely
    het = np.zeros((N, 2, L), np.uint8)
    het[:, 1, :] = 1  # z = 0: survives surely at theta = 0
    for k in range(P):
        pop.set_genomes(pack(ones if k in (0, 1, 4) else het), generation=0, patch=k)
    pop.step(1)
    live = {2, 3, 5}
    for k in range(P):
        assert pop.stats(k)["n"] == N  # every patch keeps its census: some patch survives
        _, _, src = pop.parents(k, with_source=True)
        assert set(src.tolist()) <= live
    # patch 0 is dead: every offspring descends from its drawn source when
    # that one lives, else from the first live patch after it
    _, _, src0 = pop.parents(0, with_source=True)
    assert set(src0.tolist()) <= live and len(set(src0.tolist())) >= 2


def test_no_survivor_anywhere_is_extinction():
    P, N, L = 4, 100, 32
    pop = oracle.OraclePop(seed=34, n0=N, n_loci=L, omega=0.5, theta=0.0, n_patches=P, migration=0.5,
                           dispersal=1, home_return=0.2)
    ones = np.ones((N, 2, L), np.uint8)
    for k in range(P):
        pop.set_genomes(pack(ones), generation=2, patch=k)
    pop.step(1)
    assert pop.total_stats()["n"] == 0 and pop.total_stats()["extinct"] == 1


def test_dispersal_parameters_are_checked():
    for bad in (dict(dispersal=2), dict(dispersal=1, home_return=1.5), dict(dispersal=1, home_return=-0.1)):
        with pytest.raises(ValueError):
            oracle.OraclePop(n0=10, n_patches=3, migration=0.1, **bad)

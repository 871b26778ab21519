"""Population-level pins of the oracle's generation step.

Hardy-Weinberg proportions with selection off, the heterozygosity decay law
H_t = H_0 (1 - 1/2N)^t of neutral Wright-Fisher sampling, the exact midparent
regression of the additive model with symmetric mutation, survival
frequencies against v(z) s(N) evaluated independently, Poisson fecundity
moments, the Beverton-Holt equilibrium, uniform parent choice, capacity
truncation and extinction.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle


def viability(z, theta, omega):
    return np.exp(-((np.asarray(z, float) - theta) ** 2) / (2.0 * omega * omega))


def test_hardy_weinberg_after_one_generation():
    N, L = 3000, 64
    pop = oracle.OraclePop(seed=5, n0=N, n_loci=L, r=0.5, mu=0.0, omega=0.0)
    # skew allele frequencies away from 1/2 by seeding a structured parent set
    g = np.random.default_rng(8)
    p_locus = g.uniform(0.1, 0.9, L)
    alle = (g.random((N, 2, L)) < p_locus).astype(np.uint8)
    words = np.zeros((N, 2, 2), np.uint32)
    for l in range(L):
        words[:, :, l // 32] |= alle[:, :, l].astype(np.uint32) << np.uint32(l % 32)
    pop.set_genomes(words, generation=3)
    p_par = alle.reshape(N, -1).reshape(N, 2, L).mean(axis=(0, 1))
    pop.step(1)
    a = pop.alleles()
    geno = a.sum(axis=1)  # 0, 1, 2 copies of allele 1
    chi2 = 0.0
    for l in range(L):
        p = p_par[l]
        exp = np.array([(1 - p) ** 2, 2 * p * (1 - p), p * p]) * N
        obs = np.bincount(geno[:, l], minlength=3)
        chi2 += (((obs - exp) ** 2) / exp).sum()
    # each locus contributes 2 degrees of freedom given the parental p
    assert stats.chi2.sf(chi2, 2 * L) > 1e-4


@pytest.mark.parametrize("r", [0.5, 0.01])
def test_heterozygosity_decay_law(r):
    N, L, T, R = 20, 32, 15, 1000
    H = np.zeros((R, T + 1))
    for rep in range(R):
        pop = oracle.OraclePop(seed=77, replicate_id=rep, n0=N, n_loci=L, r=r, mu=0.0, omega=0.0)
        for t in range(T + 1):
            if t:
                pop.step(1)
            if t in (0, 5, 10, 15):
                p = pop.alleles().mean(axis=(0, 1))
                H[rep, t] = np.mean(2 * p * (1 - p))
    for t in (5, 10, 15):
        pred = H[:, 0].mean() * (1 - 1 / (2 * N)) ** t
        mean = H[:, t].mean()
        se = H[:, t].std(ddof=1) / math.sqrt(R)
        assert abs(mean - pred) < 4 * se, (t, mean, pred, se)


def test_midparent_regression_with_mutation():
    N, L, mu = 2000, 256, 0.05
    pop = oracle.OraclePop(seed=31, n0=N, n_loci=L, r=0.2, mu=mu, omega=0.0)
    z_par = pop.phenotypes().astype(float)
    pop.step(1)
    mom, dad = pop.parents()
    z_child = pop.phenotypes().astype(float)
    resid = z_child - (1 - 2 * mu) * (z_par[mom] + z_par[dad]) / 2
    se = resid.std(ddof=1) / math.sqrt(N)
    assert abs(resid.mean()) < 4 * se


def test_survival_frequency_and_compaction():
    N, L, omega = 5000, 64, 3.0
    pop = oracle.OraclePop(seed=13, n0=N, n_loci=L, r=0.5, mu=1e-3, omega=omega)
    obs_total = exp_total = var_total = 0.0
    for _ in range(4):
        z = pop.phenotypes()
        v = viability(z, 0.0, omega)
        pop.step(1)
        S = pop.survivors()
        st = pop.stats()
        assert st["n_survivors"] == len(S)
        assert np.all(np.diff(S.astype(np.int64)) > 0)  # ascending, distinct
        assert S.size == 0 or S[-1] < N
        obs_total += len(S)
        exp_total += v.sum()
        var_total += (v * (1 - v)).sum()
        # mean viability reported exactly as a sum of thresholds
        assert abs(st["sum_threshold"] / 2 ** 32 - v.sum()) < 1e-6 * N
    assert abs(obs_total - exp_total) < 4 * math.sqrt(var_total)


def test_survivors_carry_higher_viability():
    N, L, omega = 4000, 64, 2.5
    pop = oracle.OraclePop(seed=17, n0=N, n_loci=L, r=0.5, omega=omega)
    z = pop.phenotypes()
    pop.step(1)
    S = pop.survivors()
    alive = np.zeros(N, bool)
    alive[S] = True
    v = viability(z, 0.0, omega)
    # logistic check: P(alive | z) tracks v(z) per phenotype class
    for zz in np.unique(z):
        sel = z == zz
        n = sel.sum()
        if n < 30:
            continue
        p = v[sel][0]
        assert abs(alive[sel].mean() - p) < 5 * math.sqrt(max(p * (1 - p), 1e-9) / n) + 1e-9


def test_parents_uniform_over_survivors():
    N, L = 2000, 32
    pop = oracle.OraclePop(seed=23, n0=N, n_loci=L, omega=0.0)
    pop.step(1)
    mom, dad = pop.parents()
    counts = np.bincount(np.concatenate([mom, dad]), minlength=N)
    exp = 2.0 * N / N
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert stats.chi2.sf(chi2, N - 1) > 1e-4
    # mothers and fathers are independent draws
    assert abs(np.corrcoef(mom, dad)[0, 1]) < 4 / math.sqrt(N)


def test_poisson_fecundity_moments():
    N, L, lam = 4000, 32, 2.2
    pop = oracle.OraclePop(seed=29, regime=1, n0=N, capacity=10 * N, n_loci=L, omega=0.0, K=0.0, fecundity=lam)
    pop.step(1)
    st = pop.stats()
    assert st["n_survivors"] == N  # no density dependence, no selection
    n1 = st["n"]
    assert abs(n1 - lam * N) < 5 * math.sqrt(lam * N)
    mom, _ = pop.parents()
    kids = np.bincount(mom, minlength=N)
    assert abs(kids.var(ddof=1) / lam - 1) < 0.1
    # slots are assigned in ascending mother order
    assert np.all(np.diff(mom.astype(np.int64)) >= 0)


def test_beverton_holt_equilibrium():
    K, lam = 3000.0, 2.2
    pop = oracle.OraclePop(seed=41, regime=1, n0=300, capacity=20000, n_loci=32, omega=0.0, K=K, fecundity=lam)
    sizes = []
    for t in range(120):
        n_before = pop.n
        pop.step(1)
        st = pop.stats()
        if t >= 60:
            sizes.append(st["n"])
        # survival multiplier s(N) = 1 / (1 + (lam - 1) N / K) is the only filter
        s = 1.0 / (1.0 + (lam - 1.0) * n_before / K)
        assert abs(st["sum_threshold"] / 2 ** 32 - s * n_before) < 1e-6 * n_before + 1
    m = float(np.mean(sizes))
    assert abs(m - K) < 0.03 * K


def test_capacity_truncation():
    pop = oracle.OraclePop(seed=43, regime=1, n0=500, capacity=600, n_loci=16, omega=0.0, K=0.0, fecundity=3.0)
    pop.step(1)
    st = pop.stats()
    assert st["n"] == 600
    mom, _ = pop.parents()
    assert len(mom) == 600
    # total offspring drawn = kept + truncated, and is Poisson(3 * 500)
    total = st["n"] + st["truncated"]
    assert abs(total - 1500) < 5 * math.sqrt(1500)


def test_extinction_freezes_population():
    pop = oracle.OraclePop(seed=47, n0=200, n_loci=64, omega=0.5, theta=1000.0)
    pop.step(1)
    st = pop.stats()
    assert st["n_survivors"] == 0 and st["n"] == 0 and st["extinct"] == 1
    pop.step(3)
    st = pop.stats()
    assert st["n"] == 0 and st["extinct"] == 1 and st["generation"] == 4


def test_same_seed_same_run_and_replicates_differ():
    a = oracle.OraclePop(seed=1, n0=300, n_loci=64, mu=1e-3, r=0.5, omega=8.0)
    b = oracle.OraclePop(seed=1, n0=300, n_loci=64, mu=1e-3, r=0.5, omega=8.0)
    c = oracle.OraclePop(seed=1, replicate_id=1, n0=300, n_loci=64, mu=1e-3, r=0.5, omega=8.0)
    a.step(10)
    b.step(10)
    c.step(10)
    assert np.array_equal(a.genomes(), b.genomes())
    assert not np.array_equal(a.genomes(), c.genomes())

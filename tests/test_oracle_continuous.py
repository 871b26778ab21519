"""Pins of the oracle's continuous-allele genetics (Supplementary S2,
"Genetics"): one float allelic value per locus and haplotype, gametes that
carry half of the parent's alleles, Gaussian mutation with standard
deviation varpi times the mean initial allelic value, the offspring's
genetic value as the sum over loci of the midpoints of the inherited
values, residual phenotypic noise varrho and the exp transform.

What fixes each part, independently of the oracle's own formulas:

* the Box-Muller deviates: a Kolmogorov-Smirnov test against the standard
  normal, moments, and the two-sided 3-sigma tail mass;
* gametes: with allelic values 0.0 and 1.0 the continuous gamete is the
  biallelic gamete of the same draws (whose law is pinned by exact
  enumeration in test_oracle_genetics.py), in every crossover mode; with
  arbitrary values each locus carries one of the parent's two values;
* mutation: the mutated loci are the biallelic rule's flips, their number
  follows Binomial(L, mu), and the changes are N(0, (varpi a0)^2);
* phenotype: the closed-form midpoint sum (math.fsum), the noise law, the
  log-normal law of the exp transform;
* population: initial values N(a0, s0^2); the midparent regression
  E[g_child] = (g_mom + g_dad) / 2; survival against exp(-(z-theta)^2 /
  (2 omega^2)) evaluated by numpy; census sums recomputed from phenotypes.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle

ST_INIT, ST_MUTVAL_MAT, ST_NOISE = 1, 13, 15


def cont_pop(**kw):
    base = dict(seed=5, n0=200, n_loci=48, genetics=1, allele_mean=0.5, allele_sd=0.1, mut_sd_factor=0.2,
                noise_sd=0.0, r=0.5, mu=0.0)
    base.update(kw)
    return oracle.OraclePop(**base)


# ---------------------------------------------------------------- deviates

def test_box_muller_deviates_are_standard_normal():
    x = np.concatenate([oracle.normals(11, 3, j, ST_NOISE, 4, 0, 20000) for j in range(10)])
    assert stats.kstest(x, "norm").pvalue > 1e-3
    n = x.size
    assert abs(x.mean()) < 4.0 / math.sqrt(n)
    assert abs(x.var() - 1.0) < 4.0 * math.sqrt(2.0 / n)
    tail = np.mean(np.abs(x) > 3.0)
    p3 = 2.0 * stats.norm.sf(3.0)
    assert abs(tail - p3) < 4.0 * math.sqrt(p3 / n)
    assert np.all(np.isfinite(x))


def test_deviates_of_distinct_blocks_are_independent():
    a = oracle.normals(11, 3, 7, ST_MUTVAL_MAT, 2, 0, 50000)
    b = oracle.normals(11, 3, 8, ST_MUTVAL_MAT, 2, 0, 50000)
    assert abs(np.corrcoef(a, b)[0, 1]) < 4.0 / math.sqrt(a.size)
    assert abs(np.corrcoef(a[:-1], a[1:])[0, 1]) < 4.0 / math.sqrt(a.size)


# ---------------------------------------------------------------- gametes

@pytest.mark.parametrize("r", [0.5, 0.0, 0.02, 0.3])
def test_zero_one_values_reproduce_the_biallelic_gamete(r):
    L = 70
    cont = cont_pop(n_loci=L, r=r)
    bial = oracle.OraclePop(seed=5, n0=200, n_loci=L, r=r, mu=0.0)
    parent_f = np.stack([np.zeros(L, np.float32), np.ones(L, np.float32)])
    parent_b = np.stack([np.zeros(L, np.uint8), np.ones(L, np.uint8)])
    for pat in (False, True):
        gf = cont.sample_gametes_cont(parent_f, 0, 300, gen=3, paternal=pat)
        gb = bial.sample_gametes(parent_b, 0, 300, gen=3, paternal=pat)
        assert np.array_equal(gf, gb.astype(np.float32))


def test_every_locus_carries_one_of_the_parents_values():
    L = 64
    pop = cont_pop(n_loci=L, r=0.2)
    g = np.random.default_rng(2)
    parent = g.normal(0.5, 0.3, (2, L)).astype(np.float32)
    gam = pop.sample_gametes_cont(parent, 0, 500, gen=1)
    from0 = gam == parent[0]
    from1 = gam == parent[1]
    assert np.all(from0 | from1)
    # a biallelic gamete of the same draws picks haplotype 1 exactly where
    # the continuous gamete took parent[1]
    bial = oracle.OraclePop(seed=5, n0=200, n_loci=L, r=0.2)
    gb = bial.sample_gametes(np.stack([np.zeros(L, np.uint8), np.ones(L, np.uint8)]), 0, 500, gen=1)
    assert np.array_equal(from1 & ~from0, gb.astype(bool) & ~from0)


def test_mutated_loci_are_the_biallelic_flips_and_changes_are_gaussian():
    L, mu, a0, varpi = 96, 0.05, 0.8, 0.3
    pop = cont_pop(n_loci=L, mu=mu, allele_mean=a0, mut_sd_factor=varpi)
    bial = oracle.OraclePop(seed=5, n0=200, n_loci=L, r=0.5, mu=mu)
    parent = np.full((2, L), a0, np.float32)
    count = 4000
    gf = pop.sample_gametes_cont(parent, 0, count, gen=2, paternal=True)
    gb = bial.sample_gametes(np.zeros((2, L), np.uint8), 0, count, gen=2, paternal=True)
    changed = gf != np.float32(a0)
    assert np.array_equal(changed, gb.astype(bool))
    # the number of mutated loci per gamete is Binomial(L, mu)
    k = changed.sum(axis=1)
    assert abs(k.mean() - L * mu) < 4.0 * math.sqrt(L * mu * (1 - mu) / count)
    # each change is N(0, (varpi a0)^2), up to float rounding of the value
    d = (gf[changed].astype(np.float64) - a0) / (varpi * a0)
    assert d.size > 10000
    assert stats.kstest(d, "norm").pvalue > 1e-3


def test_mutation_sd_scales_with_the_mean_initial_value():
    L = 32
    sds = []
    for a0 in (0.25, 2.0):
        pop = cont_pop(n_loci=L, mu=0.5, allele_mean=a0, mut_sd_factor=0.1)
        gf = pop.sample_gametes_cont(np.full((2, L), a0, np.float32), 0, 3000, gen=0)
        d = gf.astype(np.float64) - a0
        sds.append(d[gf != np.float32(a0)].std())
    assert abs(sds[0] / 0.025 - 1.0) < 0.03
    assert abs(sds[1] / 0.2 - 1.0) < 0.03


# ---------------------------------------------------------------- phenotype

def test_phenotype_is_the_midpoint_sum_without_noise():
    L = 300
    pop = cont_pop(n_loci=L)
    g = np.random.default_rng(3)
    for _ in range(20):
        h0 = g.normal(0.2, 1.0, L).astype(np.float32)
        h1 = g.normal(-0.1, 1.0, L).astype(np.float32)
        want = math.fsum(0.5 * (float(a) + float(b)) for a, b in zip(h0, h1))
        got = pop.phenotype_cont_of(h0, h1)
        assert got == pytest.approx(want, rel=1e-6, abs=1e-6)


def test_phenotype_noise_and_exp_transform_laws():
    L, rho = 16, 0.3
    h0 = np.full(L, 0.05, np.float32)
    h1 = np.full(L, 0.02, np.float32)
    g = math.fsum(0.5 * (float(a) + float(b)) for a, b in zip(h0, h1))
    plain = cont_pop(n_loci=L, noise_sd=rho)
    expo = cont_pop(n_loci=L, noise_sd=rho, exp_transform=1)
    zs = np.array([plain.phenotype_cont_of(h0, h1, j=j, gen=5) for j in range(6000)])
    ze = np.array([expo.phenotype_cont_of(h0, h1, j=j, gen=5) for j in range(6000)])
    assert stats.kstest((zs - g) / rho, "norm").pvalue > 1e-3
    # same draws: the transform is exp of the noisy value
    assert np.allclose(ze, np.exp(zs.astype(np.float64)), rtol=1e-6)
    assert stats.kstest((np.log(ze.astype(np.float64)) - g) / rho, "norm").pvalue > 1e-3
    # founders (block 1) and newborns (block 0) draw different noise
    f = np.array([plain.phenotype_cont_of(h0, h1, j=j, gen=5, sub=1) for j in range(200)])
    assert not np.allclose(f, zs[:200])


# ---------------------------------------------------------------- population

def test_initial_values_are_normal_around_the_mean():
    a0, s0 = 1.5, 0.25
    pop = cont_pop(n0=400, n_loci=40, allele_mean=a0, allele_sd=s0)
    v = pop.allele_values().astype(np.float64).ravel()
    assert stats.kstest((v - a0) / s0, "norm").pvalue > 1e-3
    z = pop.phenotypes_f().astype(np.float64)
    g = 0.5 * v.reshape(400, 2, 40).sum(axis=(1, 2))
    assert np.allclose(z, g, rtol=1e-6, atol=1e-6)


def test_midparent_regression():
    L = 40
    pop = cont_pop(n0=3000, n_loci=L, r=0.1, mu=0.01, allele_sd=0.3)
    adults = pop.allele_values().astype(np.float64)
    gv = 0.5 * adults.sum(axis=(1, 2))
    pop.step(1)
    mom, dad = pop.parents()
    kids = pop.allele_values().astype(np.float64)
    gk = 0.5 * kids.sum(axis=(1, 2))
    d = gk - 0.5 * (gv[mom] + gv[dad])
    assert abs(d.mean()) < 4.0 * d.std() / math.sqrt(d.size)
    # slope of the child's value on the midparent value is 1 (no selection)
    mid = 0.5 * (gv[mom] + gv[dad])
    slope = np.cov(mid, gk)[0, 1] / mid.var(ddof=1)
    assert abs(slope - 1.0) < 0.1


def test_survival_follows_gaussian_viability_of_the_phenotype():
    theta, omega = 12.5, 1.5
    pop = cont_pop(n0=20000, n_loci=25, allele_mean=0.5, allele_sd=0.08, omega=omega, theta=theta)
    z = pop.phenotypes_f().astype(np.float64)
    p = np.exp(-((z - theta) ** 2) / (2.0 * omega * omega))
    t_np = np.floor(p * 2.0 ** 32)
    pop.step(1)
    st = pop.stats()
    # floor(p 2^32) per adult, p by numpy's exp: within one unit each
    assert abs(st["sum_threshold"] - t_np.sum()) <= z.size
    assert abs(st["n_survivors"] - p.sum()) < 4.0 * math.sqrt((p * (1 - p)).sum())


def test_census_sums_of_phenotypes():
    pop = cont_pop(n0=500, n_loci=20, noise_sd=0.2, mu=0.02, omega=3.0, theta=5.0)
    pop.step(3)
    z = pop.phenotypes_f().astype(np.float64)
    st = pop.stats()
    assert st["sum_zf"] == pytest.approx(z.sum(), rel=1e-12)
    assert st["sum_zf2"] == pytest.approx((z * z).sum(), rel=1e-12)
    assert st["sum_z"] == 0 and st["sum_z2"] == 0
    assert st["updates"] == 3 * 500 * 20


def test_set_alleles_round_trip_and_rejections():
    pop = cont_pop(n0=50, n_loci=10)
    v = np.random.default_rng(9).normal(0, 1, (30, 2, 10)).astype(np.float32)
    pop.set_allele_values(v, generation=4)
    assert np.array_equal(pop.allele_values(), v)
    assert pop.generation == 4 and pop.n == 30
    with pytest.raises(ValueError):
        oracle.OraclePop(n0=10, n_loci=8, genetics=1, regime=2, ecology=dict(n0_consumer=1, capacity_consumer=1,
                         resource_trials=1, habitat=0, attack=0.5, match_width=1.0, encounters=1.0,
                         conversion=0.5, resource_q0=0.5, resource_K=10.0, surv_resource=[1, 1, 1, 0],
                         surv_consumer=[1, 1, 1, 0]))
    with pytest.raises(ValueError):
        oracle.OraclePop(n0=10, n_loci=8, genetics=1, noise_sd=-1.0)

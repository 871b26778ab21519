"""Pins of the oracle's linkage map and mating systems (main text: mating
systems random, shared preference or assortative, monogamy or
polygynandry, arbitrary linkage; Supplementary S2, "Reproduction": mothers
among the females, fathers among the males, each egg's parents drawn at
random among the eligible).

* Linkage map: a map of one value r reproduces the uniform bit-serial
  gametes exactly (the rule the biallelic pins fix); each boundary crosses
  over at its own rate, boundaries of rate 0 never; the three-locus gamete
  law by exact enumeration with two different rates; neighbouring
  boundaries independent.
* Sexes: fair sex ratio; mothers female and fathers male; mothers uniform
  over the surviving females and fathers over the surviving males; in the
  Poisson regime only females have offspring, lambda each; a population
  that loses a sex ends.
* Mate choice: fathers' phenotypes follow n(z) a(z) (shared preference)
  and n(z) a(z_m - z) given the mother (assortative), against the adults'
  own phenotypes; with no acceptable male the fallback still picks a male.
* Monogamy: a mother's offspring share one father; the mothers' mates are
  uniform over the males.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle


def het_parent(L):
    return np.stack([np.zeros(L, np.uint8), np.ones(L, np.uint8)])


def crossovers(gametes):
    # boundary b (between loci b-1 and b) crossed over where the gamete of a
    # 0/1 parent changes haplotype
    return gametes[:, 1:] != gametes[:, :-1]


# ---------------------------------------------------------------- linkage map

@pytest.mark.parametrize("r", [0.1, 0.3])
def test_uniform_map_is_the_bit_serial_rule(r):
    L = 150
    plain = oracle.OraclePop(seed=4, n0=10, n_loci=L, r=r)
    mapped = oracle.OraclePop(seed=4, n0=10, n_loci=L, r=r, linkage=np.full(L - 1, r))
    for pat in (False, True):
        a = plain.sample_gametes(het_parent(L), 0, 400, gen=2, paternal=pat)
        b = mapped.sample_gametes(het_parent(L), 0, 400, gen=2, paternal=pat)
        assert np.array_equal(a, b)


def test_each_boundary_crosses_over_at_its_own_rate():
    L = 70
    g = np.random.default_rng(1)
    rmap = g.uniform(0.0, 0.5, L - 1)
    rmap[[0, 10, 33]] = 0.0
    rmap[[5, 40]] = 0.5
    rmap[[7]] = 1e-3
    pop = oracle.OraclePop(seed=9, n0=10, n_loci=L, r=0.01, linkage=rmap)
    n = 30000
    x = crossovers(pop.sample_gametes(het_parent(L), 0, n, gen=1))
    freq = x.mean(axis=0)
    assert not x[:, [0, 10, 33]].any()
    sd = np.sqrt(np.maximum(rmap * (1 - rmap), 1e-12) / n)
    assert np.all(np.abs(freq - rmap) < 5.0 * sd + 1e-12)
    # neighbouring boundaries are independent
    for b in (3, 20, 50):
        assert abs(np.corrcoef(x[:, b], x[:, b + 1])[0, 1]) < 5.0 / math.sqrt(n)


def test_three_locus_gamete_law_with_two_rates():
    r1, r2 = 0.1, 0.35
    pop = oracle.OraclePop(seed=2, n0=10, n_loci=3, linkage=[r1, r2])
    n = 40000
    gam = pop.sample_gametes(het_parent(3), 0, n, gen=0)
    codes = gam[:, 0] * 4 + gam[:, 1] * 2 + gam[:, 2]
    obs = np.bincount(codes, minlength=8)
    exp = np.zeros(8)
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                p = 0.5 * (r1 if a != b else 1 - r1) * (r2 if b != c else 1 - r2)
                exp[a * 4 + b * 2 + c] = p * n
    assert stats.chisquare(obs, exp).pvalue > 1e-3


def test_map_rejects_rates_outside_the_range():
    with pytest.raises(ValueError):
        oracle.OraclePop(n0=10, n_loci=4, linkage=[0.1, 0.6, 0.2])


# ---------------------------------------------------------------- sexes

def wf_sexes(**kw):
    d = dict(seed=3, n0=4000, n_loci=32, r=0.5, mu=0.0, omega=0.0, sexes=1)
    d.update(kw)
    return oracle.OraclePop(**d)


def test_fair_sex_ratio_and_parents_of_the_right_sex():
    pop = wf_sexes()
    s0 = pop.sexes()
    assert abs(s0.mean() - 0.5) < 4 * 0.5 / math.sqrt(s0.size)
    pop.step(1)
    mom, dad = pop.parents()
    assert np.all(s0[mom] == 0) and np.all(s0[dad] == 1)
    s1 = pop.sexes()
    assert abs(s1.mean() - 0.5) < 4 * 0.5 / math.sqrt(s1.size)
    assert not np.array_equal(s0, s1)


def test_mothers_uniform_over_females_fathers_over_males():
    pop = wf_sexes(n0=600)
    sex = pop.sexes()
    counts_m = np.zeros(600)
    counts_f = np.zeros(600)
    for _ in range(25):
        sex = pop.sexes()
        pop.step(1)
        mom, dad = pop.parents()
        f, m = np.flatnonzero(sex == 0), np.flatnonzero(sex == 1)
        cm = np.bincount(mom, minlength=600)[f]
        cd = np.bincount(dad, minlength=600)[m]
        # multinomial uniformity within each generation
        assert stats.chisquare(cm).pvalue > 1e-4
        assert stats.chisquare(cd).pvalue > 1e-4


def test_poisson_regime_only_females_reproduce():
    lam = 2.2
    pop = wf_sexes(regime=1, n0=5000, capacity=50000, fecundity=lam, K=0.0)
    sex = pop.sexes()
    pop.step(1)
    mom, dad = pop.parents()
    assert np.all(sex[mom] == 0) and np.all(sex[dad] == 1)
    nf = int((sex == 0).sum())
    n = pop.n
    assert abs(n - lam * nf) < 5 * math.sqrt(lam * nf)


def test_losing_a_sex_ends_the_population():
    # two founders; the run ends once a generation has only one sex
    pop = wf_sexes(n0=2, capacity=2)
    for _ in range(40):
        pop.step(1)
        if pop.n == 0:
            break
    assert pop.n == 0 and pop.stats()["extinct"] == 1


# ---------------------------------------------------------------- mate choice

def phenotyped(mating, width, opt=0.0, sexes=1, n0=3000, L=40, seed=5, **kw):
    return oracle.OraclePop(seed=seed, n0=n0, n_loci=L, r=0.5, mu=0.0, omega=0.0, sexes=sexes, mating=mating,
                            pref_optimum=opt, pref_width=width, **kw)


def test_shared_preference_weights_fathers_by_acceptance():
    w, opt = 2.0, 3.0
    pop = phenotyped(1, w, opt)
    z, sex = pop.phenotypes(), pop.sexes()
    pop.step(1)
    _, dad = pop.parents()
    males = np.flatnonzero(sex == 1)
    zs = np.arange(z.min(), z.max() + 1)
    weight = np.array([np.sum(z[males] == v) * math.exp(-((v - opt) ** 2) / (2 * w * w)) for v in zs])
    exp = weight / weight.sum() * dad.size
    obs = np.array([np.sum(z[dad] == v) for v in zs])
    keep = exp > 5
    obs_k, exp_k = obs[keep], exp[keep]
    assert obs[~keep].sum() <= max(10, 0.02 * dad.size)
    assert stats.chisquare(obs_k, exp_k * obs_k.sum() / exp_k.sum()).pvalue > 1e-4


def test_assortative_fathers_follow_the_mothers_phenotype():
    w = 1.5
    pop = phenotyped(2, w)
    z, sex = pop.phenotypes(), pop.sexes()
    pop.step(1)
    mom, dad = pop.parents()
    males = np.flatnonzero(sex == 1)
    zm_all = z[males]
    # strong positive correlation of the pair's phenotypes
    assert np.corrcoef(z[mom], z[dad])[0, 1] > 0.5
    # conditional law for the commonest mother phenotypes
    for v in np.bincount(z[mom] - z.min()).argsort()[-3:] + z.min():
        sel = z[mom] == v
        zs = np.arange(zm_all.min(), zm_all.max() + 1)
        weight = np.array([np.sum(zm_all == u) * math.exp(-((v - u) ** 2) / (2 * w * w)) for u in zs])
        exp = weight / weight.sum() * sel.sum()
        obs = np.array([np.sum(z[dad[sel]] == u) for u in zs])
        keep = exp > 5
        assert stats.chisquare(obs[keep], exp[keep] * obs[keep].sum() / exp[keep].sum()).pvalue > 1e-4


def test_no_acceptable_male_falls_back_to_a_male():
    # preferred phenotype far outside the population: every proposal is
    # rejected, the fallback picks the next male in survivor order
    pop = phenotyped(1, 0.05, opt=1000.0, n0=300)
    sex = pop.sexes()
    pop.step(1)
    mom, dad = pop.parents()
    assert np.all(sex[dad] == 1) and np.all(sex[mom] == 0)


def test_monogamy_mothers_share_one_father():
    pop = phenotyped(0, 1.0, sexes=1, monogamy=1, n0=2000)
    sex = pop.sexes()
    pop.step(1)
    mom, dad = pop.parents()
    mate = {}
    for m, d in zip(mom, dad):
        assert mate.setdefault(int(m), int(d)) == int(d)
    assert np.all(sex[list(mate.values())] == 1)
    # the mates of distinct mothers are uniform over the males
    males = np.flatnonzero(sex == 1)
    c = np.bincount(np.array(list(mate.values())), minlength=2000)[males]
    assert stats.chisquare(c).pvalue > 1e-4
    # with several offspring per mother, polygynandry gives different fathers
    poly = phenotyped(0, 1.0, sexes=1, monogamy=0, n0=2000)
    poly.step(1)
    pm, pd = poly.parents()
    differ = sum(1 for m in np.unique(pm) if len(set(pd[pm == m].tolist())) > 1)
    assert differ > 100


def test_hermaphrodite_monogamy_and_continuous_assortment():
    # monogamy without sexes: selfing allowed, one mate per mother
    pop = phenotyped(0, 1.0, sexes=0, monogamy=1, n0=500)
    pop.step(1)
    mom, dad = pop.parents()
    mate = {}
    for m, d in zip(mom, dad):
        assert mate.setdefault(int(m), int(d)) == int(d)
    # assortative mating on continuous phenotypes
    cpop = oracle.OraclePop(seed=8, n0=3000, n_loci=16, genetics=1, allele_mean=0.1, allele_sd=0.2, noise_sd=0.1,
                            mu=0.0, r=0.5, omega=0.0, sexes=1, mating=2, pref_width=0.2)
    z = cpop.phenotypes_f().astype(np.float64)
    cpop.step(1)
    mom, dad = cpop.parents()
    assert np.corrcoef(z[mom], z[dad])[0, 1] > 0.5


def test_mating_options_need_one_patch():
    with pytest.raises(ValueError):
        oracle.OraclePop(n0=10, n_loci=8, n_patches=3, migration=0.1, sexes=1)
    with pytest.raises(ValueError):
        oracle.OraclePop(n0=10, n_loci=8, mating=1, pref_width=0.0)

"""Pins of the oracle's genotype-phenotype map and gamete formation.

* Phenotype: closed form for unit effects, antisymmetry under allele
  complement, additivity in the effects, and the single-locus increment.
* Gametes: exact enumeration of the gamete distribution for two and three
  loci (independent crossovers at each boundary with probability r, then an
  independent flip at each locus with probability mu), the recombination
  fraction, the crossover-count law, and the mutation law.
"""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

import oracle

TWO32 = 1 << 32


def rng(seed):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------- phenotype

def test_phenotype_unit_effects_closed_form():
    L = 77
    pop = oracle.OraclePop(n0=1, n_loci=L)
    g = rng(1)
    for _ in range(50):
        h0 = g.integers(0, 2, L).astype(np.uint8)
        h1 = g.integers(0, 2, L).astype(np.uint8)
        # all effects +1: z = (#ones in h0) + (#ones in h1) - L
        assert pop.phenotype_of(h0, h1) == int(h0.sum()) + int(h1.sum()) - L


def test_phenotype_heterozygote_zero_and_complement_antisymmetry():
    L = 64
    e = rng(2).integers(-4, 5, L).astype(np.int8)
    pop = oracle.OraclePop(n0=1, n_loci=L, effects=e)
    g = rng(3)
    for _ in range(50):
        h0 = g.integers(0, 2, L).astype(np.uint8)
        h1 = g.integers(0, 2, L).astype(np.uint8)
        assert pop.phenotype_of(h0, 1 - h0) == 0  # heterozygous everywhere
        assert pop.phenotype_of(1 - h0, 1 - h1) == -pop.phenotype_of(h0, h1)
    ones = np.ones(L, np.uint8)
    assert pop.phenotype_of(ones, ones) == int(e.astype(int).sum())


def test_phenotype_additive_in_effects_and_locus_increment():
    L = 40
    g = rng(4)
    e1 = g.integers(-4, 5, L).astype(np.int8)
    e2 = g.integers(-4, 5, L).astype(np.int8) // 2
    pa = oracle.OraclePop(n0=1, n_loci=L, effects=e1)
    pb = oracle.OraclePop(n0=1, n_loci=L, effects=e2)
    pc = oracle.OraclePop(n0=1, n_loci=L, effects=(e1 + e2).astype(np.int8))
    for _ in range(30):
        h0 = g.integers(0, 2, L).astype(np.uint8)
        h1 = g.integers(0, 2, L).astype(np.uint8)
        assert pc.phenotype_of(h0, h1) == pa.phenotype_of(h0, h1) + pb.phenotype_of(h0, h1)
        l = int(g.integers(0, L))
        h0b = h0.copy()
        h0b[l] ^= 1
        delta = pa.phenotype_of(h0b, h1) - pa.phenotype_of(h0, h1)
        assert delta == (int(e1[l]) if h0b[l] == 1 else -int(e1[l]))


# ---------------------------------------------------------------- gametes

def exact_gamete_law(h0, h1, r, mu):
    """P(gamete) by enumeration over which haplotype each locus copies."""
    n = len(h0)
    law = {}
    for s in itertools.product([0, 1], repeat=n):
        ps = 0.5
        for k in range(1, n):
            ps *= r if s[k] != s[k - 1] else 1 - r
        for gam in itertools.product([0, 1], repeat=n):
            p = ps
            for l in range(n):
                src = h1[l] if s[l] else h0[l]
                p *= (1 - mu) if gam[l] == src else mu
            law[gam] = law.get(gam, 0.0) + p
    return law


def effective_r(r):
    mode = oracle.recomb_mode(r)
    if mode == "lazy":
        return math.floor(r * TWO32) / TWO32
    return r


@pytest.mark.parametrize("r", [0.5, 0.0, 0.01, 0.08, 0.1, 0.2, 0.35])
@pytest.mark.parametrize("mu", [0.0, 0.05])
@pytest.mark.parametrize("nloc", [2, 3])
def test_gamete_distribution_matches_enumeration(r, mu, nloc):
    h0 = [0, 1, 0][:nloc]
    h1 = [1, 0, 1][:nloc]
    pop = oracle.OraclePop(seed=11, n0=1, n_loci=nloc, r=r, mu=mu)
    count = 200_000
    par = np.stack([np.array(h0, np.uint8), np.array(h1, np.uint8)])
    gam = pop.sample_gametes(par, j0=0, count=count, gen=5)
    codes = (gam.astype(np.int64) * (1 << np.arange(nloc))).sum(axis=1)
    obs = np.bincount(codes, minlength=1 << nloc)
    law = exact_gamete_law(h0, h1, effective_r(r), mu)
    exp = np.array([law[tuple((c >> l) & 1 for l in range(nloc))] for c in range(1 << nloc)]) * count
    keep = exp > 0
    assert obs[~keep].sum() == 0
    chi2 = (((obs[keep] - exp[keep]) ** 2) / exp[keep]).sum()
    pval = stats.chi2.sf(chi2, keep.sum() - 1)
    assert pval > 1e-4, (obs, exp)


@pytest.mark.parametrize("r", [0.001, 0.01, 0.09, 0.1, 0.3, 0.5])
def test_recombination_fraction_and_crossover_count(r):
    L = 1024
    pop = oracle.OraclePop(seed=3, n0=1, n_loci=L, r=r, mu=0.0)
    par = np.stack([np.zeros(L, np.uint8), np.ones(L, np.uint8)])
    count = 2000
    gam = pop.sample_gametes(par, j0=100, count=count, gen=2, paternal=True)
    switches = (gam[:, 1:] != gam[:, :-1]).sum(axis=1)
    re = effective_r(r)
    n = count * (L - 1)
    frac = switches.sum() / n
    assert abs(frac - re) < 5 * math.sqrt(re * (1 - re) / n) + 1e-12
    # crossovers are independent across boundaries: Binomial(L-1, r) counts
    if 0 < re < 0.5:
        var = switches.var(ddof=1)
        assert abs(var / ((L - 1) * re * (1 - re)) - 1) < 0.15
    # the first locus copies either haplotype with probability 1/2
    first = gam[:, 0].mean()
    assert abs(first - 0.5) < 5 * math.sqrt(0.25 / count)


def test_no_recombination_copies_one_haplotype():
    L = 300
    pop = oracle.OraclePop(seed=9, n0=1, n_loci=L, r=0.0, mu=0.0)
    g = rng(5)
    par = g.integers(0, 2, (2, L)).astype(np.uint8)
    gam = pop.sample_gametes(par, j0=0, count=400)
    same0 = (gam == par[0]).all(axis=1)
    same1 = (gam == par[1]).all(axis=1)
    assert np.all(same0 | same1)
    assert 150 < same1.sum() < 250


@pytest.mark.parametrize("mu", [1e-3, 0.02, 0.3])
def test_mutation_law(mu):
    L = 200
    pop = oracle.OraclePop(seed=21, n0=1, n_loci=L, r=0.3, mu=mu)
    par = np.zeros((2, L), np.uint8)  # homozygous: every 1 in a gamete is a mutation
    count = 20000
    gam = pop.sample_gametes(par, j0=0, count=count, gen=7)
    k = gam.sum(axis=1)
    assert abs(k.mean() - L * mu) < 5 * math.sqrt(L * mu * (1 - mu) / count)
    assert abs(k.var(ddof=1) / (L * mu * (1 - mu)) - 1) < 0.1
    per_locus = gam.sum(axis=0)
    chi2 = ((per_locus - per_locus.mean()) ** 2 / per_locus.mean()).sum()
    assert stats.chi2.sf(chi2, L - 1) > 1e-4


def test_packed_layout_roundtrip_and_zero_tail():
    L = 70  # three words, six tail bits
    pop = oracle.OraclePop(seed=4, n0=10, capacity=12, n_loci=L)
    g = pop.genomes()
    assert g.shape == (10, 2, 3)
    assert np.all(g[:, :, 2] >> 6 == 0)
    a = pop.alleles()
    # locus l lives at word l // 32, bit l % 32
    for l in (0, 31, 32, 63, 64, 69):
        assert np.array_equal(a[:, :, l], (g[:, :, l // 32] >> (l % 32)) & 1)
    z = pop.phenotypes()
    assert np.array_equal(z, a.astype(np.int64).sum(axis=(1, 2)) - L)
    pop.set_genomes(g[:5], generation=17)
    assert pop.n == 5 and pop.generation == 17
    assert np.array_equal(pop.genomes(), g[:5])


def test_initial_population_is_fair_bits():
    L, n = 256, 2000
    pop = oracle.OraclePop(seed=99, n0=n, n_loci=L)
    a = pop.alleles()
    p = a.mean()
    assert abs(p - 0.5) < 5 * math.sqrt(0.25 / a.size)
    # no correlation between the two haplotypes of an individual
    agree = (a[:, 0, :] == a[:, 1, :]).mean()
    assert abs(agree - 0.5) < 5 * math.sqrt(0.25 / (n * L))

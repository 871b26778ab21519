"""Pins of the oracle's two-species consumer-resource regime (Supplementary
Information S3: consumers exploit resources by phenotype matching; read as
an individual-based model with age classes 0-3).

What the mathematics fixes: a consumer at phenotype distance d from every
resource captures a fraction a exp(-d^2 / (2 sigma^2)) of its Poisson
encounters; every captured resource is credited exactly once and dies; when
several consumers catch the same resource the lowest consumer index is
credited; survivors are Binomial(n_a, s_a) per age class and age by one;
resource offspring are Binomial(trials, q0 max(0, 1 - N/K)) per survivor;
consumer offspring Poisson(c x intake).
"""
import numpy as np
import pytest
from scipy import stats

import oracle

CR = 2


def eco(**kw):
    e = dict(n0_consumer=100, capacity_consumer=1000, resource_trials=4, habitat=0, attack=0.5, match_width=4.0,
             encounters=20.0, conversion=0.5, resource_q0=0.55, resource_K=1e5,
             surv_resource=(0.5, 0.8, 0.8, 0.0), surv_consumer=(0.6, 0.8, 0.8, 0.0))
    e.update(kw)
    return e


def genomes_with_z(n, L, z):
    """n genomes (L loci, unit effects) of phenotype z: L + z ones in all."""
    ones = L + z
    bits = np.zeros((n, 2 * L), np.uint8)
    bits[:, :ones] = 1
    bits = bits.reshape(n, 2, L)
    W = (L + 31) // 32
    words = np.zeros((n, 2, W), np.uint32)
    for l in range(L):
        words[:, :, l // 32] |= bits[:, :, l].astype(np.uint32) << np.uint32(l % 32)
    return words


def test_small_binomial_table_matches_the_distribution():
    for n, q in [(4, 0.55), (4, 0.01), (8, 0.3), (1, 0.9), (4, 0.0), (4, 1.0)]:
        T = oracle.small_binomial_thresholds(n, q).astype(float)
        cdf = stats.binom.cdf(np.arange(len(T)), n, q) * 2.0 ** 32
        assert T[-1] == 2.0 ** 32
        assert np.all(np.abs(T[:-1] - np.floor(cdf[:-1])) <= 2), (n, q)
        assert np.all(np.diff(T) >= 0)


@pytest.mark.parametrize("d", [0, 3, 6])
def test_capture_fraction_follows_phenotype_matching(d):
    L, NR, NC, a, sig, lam = 64, 200_000, 150, 0.5, 4.0, 20.0
    e = eco(n0_consumer=NC, capacity_consumer=NC, attack=a, match_width=sig, encounters=lam, resource_q0=0.0,
            surv_resource=(1, 1, 1, 1), surv_consumer=(1, 1, 1, 1))
    pop = oracle.OraclePop(seed=3, regime=CR, n0=NR, capacity=NR, n_loci=L, ecology=e)
    pop.set_genomes(genomes_with_z(NR, L, 0), 0, species=0)
    pop.set_genomes(genomes_with_z(NC, L, d), 0, species=1)
    pop.step(1)
    intake = pop.intake()
    expect = lam * a * np.exp(-d * d / (2 * sig * sig)) * NC
    assert abs(intake.sum() - expect) < 4.5 * np.sqrt(expect) + 3, (intake.sum(), expect)
    # every credited capture killed a distinct resource (survival is certain otherwise)
    assert pop.stats(species=0)["n_survivors"] == NR - intake.sum()
    assert pop.stats(species=1)["captures"] == intake.sum()


def test_lowest_consumer_is_credited():
    L, NR, NC = 32, 5, 40
    e = eco(n0_consumer=NC, capacity_consumer=NC, attack=1.0, match_width=1e6, encounters=30.0, resource_q0=0.0,
            surv_resource=(1, 1, 1, 1), surv_consumer=(1, 1, 1, 1))
    pop = oracle.OraclePop(seed=5, regime=CR, n0=NR, capacity=NR, n_loci=L, ecology=e)
    pop.step(1)
    intake = pop.intake()
    # consumer 0 meets about 30 of the 5 resources: it catches and is credited all of them
    assert intake[0] == NR and intake[1:].sum() == 0
    assert pop.stats(species=0)["n"] == 0


def test_age_classes_survive_by_their_rates_and_age():
    L, N = 32, 20_000
    sr = (0.3, 0.7, 0.9, 0.0)
    e = eco(n0_consumer=0, capacity_consumer=1, attack=0.0, resource_q0=0.9, resource_K=1e9, surv_resource=sr)
    pop = oracle.OraclePop(seed=8, regime=CR, n0=N, capacity=4 * N, n_loci=L, omega=0.0, ecology=e)
    ages_before = pop.ages(species=0)
    for gen in range(4):
        ages_before = pop.ages(species=0)
        pop.step(1)
        S = pop.survivors(species=0)
        alive = np.zeros(len(ages_before), bool)
        alive[S] = True
        for a in range(4):
            sel = ages_before == a
            if sel.sum() > 50:
                k = int(alive[sel].sum())
                assert stats.binomtest(k, int(sel.sum()), sr[a]).pvalue > 1e-4, (gen, a, k, sel.sum())
        after = pop.ages(species=0)
        ns = len(S)
        assert np.array_equal(after[:ns], ages_before[S] + 1)
        assert np.all(after[ns:] == 0) and after.max() <= 3


def test_oldest_class_holds_three_and_older():
    e = eco(n0_consumer=0, capacity_consumer=1, attack=0.0, resource_q0=0.0, surv_resource=(1, 1, 1, 1))
    pop = oracle.OraclePop(seed=3, regime=CR, n0=500, capacity=500, n_loci=32, ecology=e)
    for gen in range(1, 7):
        pop.step(1)
        assert np.all(pop.ages(species=0) == min(gen, 3))
        assert pop.n_of(species=0) == 500


def test_carried_survivors_keep_their_genomes():
    L = 96
    e = eco(n0_consumer=50, capacity_consumer=500, encounters=5.0)
    pop = oracle.OraclePop(seed=9, regime=CR, n0=800, capacity=3000, n_loci=L, mu=1e-3, r=0.2, ecology=e)
    pop.step(2)
    for sp in (0, 1):
        g0, z0 = pop.genomes(species=sp), pop.phenotypes(species=sp)
        pop.step(1)
        S = pop.survivors(species=sp)
        g1, z1 = pop.genomes(species=sp), pop.phenotypes(species=sp)
        assert np.array_equal(g1[: len(S)], g0[S]) and np.array_equal(z1[: len(S)], z0[S])
        assert pop.stats(species=sp)["n"] == len(S) + pop.newborns(species=sp)
        pop2 = pop  # the next species continues from the same replicate state
        del pop2


@pytest.mark.parametrize("N,K,trials,q0", [(5000, 1e5, 4, 0.55), (5000, 10_000, 4, 0.55), (5000, 4000, 4, 0.55),
                                           (3000, 1e9, 2, 0.3)])
def test_resource_fecundity_is_logistic_binomial(N, K, trials, q0):
    L = 32
    e = eco(n0_consumer=0, capacity_consumer=1, attack=0.0, resource_trials=trials, resource_q0=q0, resource_K=K,
            surv_resource=(1, 1, 1, 1))
    pop = oracle.OraclePop(seed=10, regime=CR, n0=N, capacity=100 * N, n_loci=L, ecology=e)
    pop.step(1)
    q = q0 * max(0.0, 1.0 - N / K)
    births = pop.newborns(species=0)
    mean, var = N * trials * q, N * trials * q * (1 - q)
    assert abs(births - mean) <= 5 * np.sqrt(var) + 1e-9, (births, mean)
    if q == 0.0:
        assert births == 0


def test_consumer_fecundity_is_poisson_in_intake():
    L, NR, NC, c = 32, 100_000, 2000, 0.7
    e = eco(n0_consumer=NC, capacity_consumer=10 * NC, attack=0.8, match_width=1e6, encounters=3.0, conversion=c,
            resource_q0=0.0, surv_resource=(1, 1, 1, 1), surv_consumer=(1, 1, 1, 1))
    pop = oracle.OraclePop(seed=11, regime=CR, n0=NR, capacity=NR, n_loci=L, ecology=e)
    pop.step(1)
    lam = c * pop.intake().sum()
    births = pop.newborns(species=1)
    assert abs(births - lam) < 5 * np.sqrt(lam), (births, lam)


def test_encounters_scale_with_resource_density():
    # with a habitat of H slots an encounter finds a resource with
    # probability N_R / H: intake falls in proportion
    L, NC, lam = 32, 400, 10.0
    got = []
    for NR in (5000, 20000):
        e = eco(n0_consumer=NC, capacity_consumer=NC, habitat=40000, attack=1.0, match_width=1e6, encounters=lam,
                resource_q0=0.0, surv_resource=(1, 1, 1, 1), surv_consumer=(1, 1, 1, 1))
        pop = oracle.OraclePop(seed=13, regime=CR, n0=NR, capacity=NR, n_loci=L, ecology=e)
        pop.step(1)
        got.append(pop.intake().sum())
        expect = NC * lam * NR / 40000
        assert abs(got[-1] - expect) < 5 * np.sqrt(expect), (NR, got[-1], expect)


def test_both_species_persist_with_the_workload_constants():
    # the consumer-resource workload's constants at a tenth of its size
    e = eco(n0_consumer=1000, capacity_consumer=5000, habitat=20_000, resource_K=25_000)
    pop = oracle.OraclePop(seed=12, regime=CR, n0=10_000, capacity=25_000, n_loci=64, mu=1e-4, r=0.2, ecology=e)
    sizes = []
    for _ in range(25):
        pop.step(1)
        sizes.append((pop.n_of(species=0), pop.n_of(species=1)))
    assert all(r > 3000 and c > 300 for r, c in sizes), sizes


def test_consumer_resource_needs_the_ecology():
    with pytest.raises(ValueError):
        oracle.OraclePop(regime=CR, n0=10, capacity=20)

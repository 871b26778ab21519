"""Statistical checks of the HIP library against the model itself, not
against the oracle: crossovers, mutations, Wright-Fisher parents, survival
and fecundity in the Poisson / Beverton-Holt regime, and migration on a
ring of patches.

Crossovers: with every parent heterozygous at every locus (one
haplotype all 0, the other all 1), no mutation and no selection, a change of
allele between adjacent loci of a newborn's haplotype is exactly a crossover
at that boundary.  Gametes follow Fig. 1B and the genetics of
Supplementary Information S2 (r = 1/2 is free recombination; for linked
loci the reading taken is a crossover at each boundary independently with
probability r, without interference): the haplotype copied at the first
locus is either parent haplotype with probability 1/2, and bits past locus
L - 1 stay 0."""
import numpy as np
import pytest

from gpu_helpers import say
from paper_1603_09255_amd import spegg

pytestmark = pytest.mark.gpu

N = 20000


def het_parents(n, L):
    W = (L + 31) // 32
    words = np.zeros((n, 2, W), np.uint32)
    words[:, 1, :] = 0xFFFFFFFF
    if L % 32:
        words[:, 1, -1] = (1 << (L % 32)) - 1
    return words


def one_generation(L, r, seed):
    d = dict(seed=seed, replicate_id=1, regime=0, n0=N, capacity=N, n_loci=L, mu=0.0, r=r, theta=0.0,
             omega=0.0, K=0.0, fecundity=0.0)
    pop = spegg.Population([d])
    pop.write_genomes(0, het_parents(N, L), 10)
    pop.step(1)
    g = pop.genomes(0)
    pop.close()
    assert g.shape == (N, 2, (L + 31) // 32)
    bits = np.unpackbits(np.ascontiguousarray(g).view(np.uint8), bitorder="little").reshape(N, 2, -1)
    return bits


@pytest.mark.parametrize("L,r", [(1000, 0.01), (1000, 0.1), (1000, 0.3), (64, 0.5), (257, 0.0)],
                         ids=["skip-0.01", "skip-0.1", "lazy-0.3", "raw-0.5", "zero"])
def test_crossovers_are_independent_bernoulli_per_boundary(L, r):
    say("recombination statistics L", L, "r", r)
    bits = one_generation(L, r, seed=31 + L)
    assert not bits[:, :, L:].any(), "bits past the last locus must stay 0"
    hap = bits[:, :, :L].reshape(2 * N, L)
    # the first locus copies either parent haplotype with probability 1/2
    p0 = hap[:, 0].mean()
    assert abs(p0 - 0.5) < 6 * np.sqrt(0.25 / (2 * N)), p0
    switches = hap[:, 1:] != hap[:, :-1]
    m = switches.size
    frac = switches.mean()
    if r == 0.0:
        assert frac == 0.0
        return
    sd = np.sqrt(r * (1 - r) / m)
    assert abs(frac - r) < 6 * sd, (frac, r, sd)
    # per-gamete counts: Binomial(L - 1, r) -- variance r (1 - r) (L - 1); a
    # random word reused across boundaries would inflate it
    counts = switches.sum(axis=1)
    var = r * (1 - r) * (L - 1)
    assert abs(counts.var() - var) < 6 * var * np.sqrt(2.0 / counts.size) + 0.05, (counts.var(), var)
    # neighbouring boundaries uncorrelated
    a, b = switches[:, :-1], switches[:, 1:]
    cov = np.count_nonzero(a & b) / a.size - a.mean() * b.mean()
    assert abs(cov) < 6 * r * (1 - r) / np.sqrt(a.size), cov


@pytest.mark.parametrize("mu", [1e-3, 0.05])
def test_mutations_flip_each_locus_with_probability_mu(mu):
    # every parent homozygous 0: a newborn's 1 bits are exactly its gametes'
    # mutations, K ~ Binomial(L, mu) distinct loci per gamete, so each locus
    # flips with probability mu and a gamete's count has variance L mu (1 - mu)
    L = 1000
    say("mutation statistics mu", mu)
    d = dict(seed=41, replicate_id=2, regime=0, n0=N, capacity=N, n_loci=L, mu=mu, r=0.5, theta=0.0, omega=0.0,
             K=0.0, fecundity=0.0)
    pop = spegg.Population([d])
    pop.write_genomes(0, np.zeros((N, 2, (L + 31) // 32), np.uint32), 3)
    pop.step(1)
    g = pop.genomes(0)
    pop.close()
    bits = np.unpackbits(np.ascontiguousarray(g).view(np.uint8), bitorder="little").reshape(N, 2, -1)
    assert not bits[:, :, L:].any()
    per_gamete = bits[:, :, :L].reshape(2 * N, L).sum(axis=1)
    m = 2 * N * L
    frac = per_gamete.sum() / m
    assert abs(frac - mu) < 6 * np.sqrt(mu * (1 - mu) / m), frac
    var = L * mu * (1 - mu)
    assert abs(per_gamete.var() - var) < 6 * np.sqrt((2 * var * var + var) / per_gamete.size), per_gamete.var()


def test_wright_fisher_parents_are_uniform_over_the_adults():
    # no selection: every adult survives, and each newborn's mother and father
    # are uniform over the N adults, so an adult's offspring count is
    # Binomial(2N, 1/N): mean 2, variance 2 (1 - 1/N)
    L = 64
    d = dict(seed=43, replicate_id=3, regime=0, n0=N, capacity=N, n_loci=L, mu=0.0, r=0.5, theta=0.0, omega=0.0,
             K=0.0, fecundity=0.0)
    pop = spegg.Population([d])
    pop.set_trace(True)
    pop.step(1)
    mom, dad = pop.parents(0)
    assert pop.stats()[0]["n_survivors"] == N
    pop.close()
    assert mom.size == N and dad.size == N and mom.max() < N and dad.max() < N
    kids = np.bincount(mom, minlength=N) + np.bincount(dad, minlength=N)
    assert kids.sum() == 2 * N
    var = 2.0 * (1 - 1.0 / N)
    assert abs(kids.var() - var) < 6 * np.sqrt((2 * var * var + var) / N), kids.var()
    # mothers and fathers drawn independently
    assert abs(np.corrcoef(mom.astype(np.float64), dad.astype(np.float64))[0, 1]) < 6 / np.sqrt(N)


def test_poisson_bh_survival_and_fecundity_match_the_model():
    # every adult has phenotype z = 0 (heterozygous at every locus, unit
    # effects): it survives with probability v(0) s(N), Gaussian viability
    # v(z) = exp(-(z - theta)^2 / (2 omega^2)) times the Beverton-Holt factor
    # s(N) = 1 / (1 + (lambda - 1) N / K), and each survivor leaves
    # Poisson(lambda) newborns
    L, theta, omega, lam, K = 256, 5.0, 10.0, 2.2, float(N)
    d = dict(seed=47, replicate_id=4, regime=1, n0=N, capacity=4 * N, n_loci=L, mu=0.0, r=0.5, theta=theta,
             omega=omega, K=K, fecundity=lam)
    pop = spegg.Population([d])
    pop.write_genomes(0, het_parents(N, L), 5)
    pop.step(1)
    st = pop.stats()[0]
    pop.close()
    p = np.exp(-(theta ** 2) / (2 * omega ** 2)) / (1 + (lam - 1) * N / K)
    S = st["n_survivors"]
    assert abs(S - N * p) < 6 * np.sqrt(N * p * (1 - p)), (S, N * p)
    assert st["truncated"] == 0
    assert abs(st["n"] - lam * S) < 6 * np.sqrt(lam * S), (st["n"], lam * S)


def test_ring_migrants_at_rate_m_split_evenly():
    # patches on a ring, all with survivors: a newborn's parents come from a
    # ring neighbour with probability m, either side with probability 1/2
    # (Supplementary Information S3)
    P, n, m = 4, 8000, 0.1
    d = dict(seed=53, replicate_id=6, regime=0, n0=n, capacity=n, n_loci=64, mu=0.0, r=0.5, theta=0.0, omega=0.0,
             K=0.0, fecundity=0.0, n_patches=P, migration=m)
    pop = spegg.Population([d])
    pop.set_trace(True)
    pop.step(1)
    moved = right = total = 0
    for k in range(P):
        _, _, src = pop.parents(0, patch=k, with_source=True)
        total += src.size
        moved += int(np.count_nonzero(src != k))
        right += int(np.count_nonzero(src == (k + 1) % P))
        assert np.all((src == k) | (src == (k + 1) % P) | (src == (k - 1) % P))
    pop.close()
    assert total == P * n
    assert abs(moved / total - m) < 6 * np.sqrt(m * (1 - m) / total), moved / total
    assert abs(right / moved - 0.5) < 6 * np.sqrt(0.25 / moved), right / moved

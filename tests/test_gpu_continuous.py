"""GPU parity of continuous-allele genetics (Supplementary S2, "Genetics"):
the HIP library against the oracle, generation by generation.

Integer results are compared exactly: survivor lists, traced parents and
their source patches, census sizes, near ties.  Allelic values and
phenotypes are floats computed in double (Box-Muller deviates through the
device's and glibc's log and cos, the genetic value summed in another
order) and rounded to float, so they agree to rounding: every value within
a relative 1e-6 of the oracle's (the tolerance the model states for
fitness), and at most one value in a thousand not bit-identical.  The
viability thresholds floor(p 2^32) may differ by one unit per adult, so
their census sum is compared within the number of adults; the phenotype
sums within a relative 1e-9.

Shape invariance and batching are compared exactly against the library
itself: the values a newborn gets do not depend on the kernel shape or on
the other replicates in the launch."""
import numpy as np
import pytest

from gpu_helpers import say
import oracle
from paper_1603_09255_amd import spegg

pytestmark = pytest.mark.gpu

CONT_KEYS = ("seed", "replicate_id", "regime", "n0", "capacity", "n_loci", "mu", "r", "theta", "omega", "K",
             "fecundity", "n_patches", "migration", "dispersal", "home_return", "genetics", "allele_mean",
             "allele_sd", "mut_sd_factor", "noise_sd", "exp_transform")
EXACT = ("generation", "n", "n_parents", "n_survivors", "extinct", "captures", "sum_z", "sum_z2", "near_ties",
         "truncated", "updates")
RTOL = 1e-6


def cont(**kw):
    d = dict(seed=3, replicate_id=2, regime=spegg.WF, n0=400, capacity=400, n_loci=64, mu=0.01, r=0.5,
             theta=3.0, omega=2.0, genetics=spegg.CONTINUOUS, allele_mean=0.05, allele_sd=0.02,
             mut_sd_factor=0.5, noise_sd=0.1, exp_transform=0)
    d.update(kw)
    return d


def oracle_of(desc):
    return oracle.OraclePop(**{k: desc[k] for k in CONT_KEYS if k in desc})


def close_values(g, o, what):
    assert g.shape == o.shape, f"{what}: shapes {g.shape} vs {o.shape}"
    if g.size == 0:
        return
    scale = max(1.0, float(np.abs(o).max()))
    ok = np.abs(g.astype(np.float64) - o.astype(np.float64)) <= RTOL * np.maximum(np.abs(o), 1e-3 * scale)
    assert ok.all(), f"{what}: {int((~ok).sum())} values beyond rtol {RTOL}, first at {np.argwhere(~ok)[:5].tolist()}"
    diff = int((g != o).sum())
    assert diff <= max(1, g.size // 1000), f"{what}: {diff} of {g.size} values not bit-identical"


def close_stats(sg, so, what):
    for k in EXACT:
        assert sg[k] == so[k], f"{what}: {k} {sg[k]} vs {so[k]}\n gpu {sg}\n oracle {so}"
    assert abs(int(sg["sum_threshold"]) - int(so["sum_threshold"])) <= max(so["n_parents"], 1), \
        f"{what}: sum_threshold {sg['sum_threshold']} vs {so['sum_threshold']}"
    for k in ("sum_zf", "sum_zf2"):
        assert sg[k] == pytest.approx(so[k], rel=1e-9, abs=1e-9), f"{what}: {k} {sg[k]} vs {so[k]}"


def same_state(gpu, orc, what, parents=True):
    close_stats(gpu.stats()[0], orc.total_stats(), what)
    per = gpu.deme_stats(0)
    for k in range(orc.n_demes):
        wk = f"{what}, patch {k}"
        sok = orc.stats(k)
        close_stats(per[k], sok, wk)
        close_values(gpu.alleles(0, k), orc.allele_values(k), f"{wk}: alleles")
        close_values(gpu.phenotypes_f(0, k), orc.phenotypes_f(k), f"{wk}: phenotypes")
        if sok["generation"] > 0 and sok["n_parents"] > 0:
            assert np.array_equal(gpu.survivors(0, k), orc.survivors(k)), f"{wk}: survivor lists differ"
        if parents and sok["generation"] > 0 and orc.newborns(k) > 0:
            gm, gd, gs = gpu.parents(0, k, with_source=True)
            om, od, os_ = orc.parents(k, with_source=True)
            assert np.array_equal(gs, os_), f"{wk}: source patches differ"
            assert np.array_equal(gm, om) and np.array_equal(gd, od), f"{wk}: parents differ"


CASES = [
    ("raw_l64", cont(), 6),
    ("skip_l301_exp", cont(n_loci=301, r=0.02, allele_mean=0.005, allele_sd=0.004, theta=4.0, exp_transform=1,
                           noise_sd=0.05), 5),
    ("lazy_l1000", cont(n_loci=1000, r=0.3, n0=150, capacity=150, mu=1e-3, allele_mean=0.003, allele_sd=0.003,
                        theta=3.0, omega=1.0), 4),
    ("zero_l33_no_noise", cont(n_loci=33, r=0.0, noise_sd=0.0, theta=1.6), 6),
    ("l1", cont(n_loci=1, r=0.1, mu=0.2, allele_mean=1.0, allele_sd=0.5, theta=1.0, omega=1.0), 6),
    ("l3_lazy", cont(n_loci=3, r=0.4, mu=0.1, allele_mean=0.5, allele_sd=0.3, theta=1.5, omega=0.8), 6),
    ("poisson_bh", cont(regime=spegg.POISSON_BH, n0=400, capacity=1000, K=500.0, fecundity=2.2, n_loci=128,
                        r=0.1, mu=0.005, allele_mean=0.02, allele_sd=0.01, theta=2.6, omega=3.0), 6),
    ("ring4", cont(n_patches=4, migration=0.2, n0=150, capacity=150), 5),
    ("island5", cont(n_patches=5, migration=0.3, dispersal=spegg.ISLAND, home_return=0.25, n0=120, capacity=120,
                     r=0.2), 5),
    ("l4096_skip", cont(n_loci=4096, r=0.001, n0=40, capacity=40, mu=2e-4, allele_mean=0.001, allele_sd=0.001,
                        theta=4.1, omega=2.0), 3),
    ("strong_selection_neg_mean", cont(allele_mean=-0.05, theta=-3.5, omega=0.5, r=0.05), 6),
]


@pytest.mark.parametrize("name,desc,gens", CASES, ids=[c[0] for c in CASES])
def test_continuous_lockstep(name, desc, gens):
    say("continuous lockstep", name)
    gpu = spegg.Population([desc])
    gpu.set_trace(True)
    orc = oracle_of(desc)
    same_state(gpu, orc, f"{name} start", parents=False)
    for _ in range(gens):
        gpu.step(1)
        orc.step(1)
        same_state(gpu, orc, f"{name} generation {orc.generation}")
    gpu.close()
    orc.close()


def test_written_values_lockstep():
    d = cont(n_loci=97, r=0.15, n0=300, capacity=300, mu=0.02)
    vals = np.random.default_rng(12).normal(0.04, 0.03, (250, 2, 97)).astype(np.float32)
    say("continuous written values")
    gpu = spegg.Population([d])
    gpu.set_trace(True)
    orc = oracle_of(d)
    gpu.write_alleles(0, vals, 7)
    orc.set_allele_values(vals, 7)
    assert np.array_equal(gpu.alleles(0), vals)
    same_state(gpu, orc, "written", parents=False)
    for _ in range(3):
        gpu.step(1)
        orc.step(1)
        same_state(gpu, orc, f"written, generation {orc.generation}")
    gpu.close()
    orc.close()


def test_bench_size_sampled():
    # the continuous bench workload's shape: N = 10^5, L = 256, two
    # generations, every value compared
    d = cont(n0=100000, capacity=100000, n_loci=256, r=0.5, mu=1e-3, allele_mean=0.01, allele_sd=0.01,
             mut_sd_factor=0.5, noise_sd=0.2, theta=2.6, omega=1.0)
    say("continuous bench size")
    gpu = spegg.Population([d])
    orc = oracle_of(d)
    for g in range(2):
        gpu.step(1)
        orc.step(1)
        same_state(gpu, orc, f"bench size, generation {g + 1}", parents=False)
    gpu.close()
    orc.close()


def test_shape_and_batch_invariance():
    a = cont(n_loci=200, r=0.05, replicate_id=5)
    b = cont(n_loci=64, r=0.3, replicate_id=6, n0=300, capacity=300)
    bial = dict(seed=3, replicate_id=7, regime=spegg.WF, n0=300, capacity=300, n_loci=128, mu=1e-3, r=0.1,
                theta=0.0, omega=8.0)
    say("continuous shape and batch invariance")
    ref = []
    for d in (a, b):
        p = spegg.Population([d])
        p.step(5)
        ref.append((p.alleles(0), p.phenotypes_f(0), p.stats()[0]))
        p.close()
    batch = spegg.Population([a, bial, b])
    batch.step(5)
    for i, k in ((0, 0), (1, 2)):
        assert np.array_equal(batch.alleles(k), ref[i][0])
        assert np.array_equal(batch.phenotypes_f(k), ref[i][1])
        assert batch.stats()[k] == ref[i][2]
    batch.close()
    key = 200 | 0x80000000  # continuous genome of 200 floats per haplotype
    for g in (1, 4, 32):
        p = spegg.Population([a])
        p.set_offspring_cap(key, g)
        p.step(5)
        assert np.array_equal(p.alleles(0), ref[0][0]), f"lanes per gamete {g}"
        assert p.stats()[0] == ref[0][2]
        p.close()


def test_continuous_rejections():
    with pytest.raises(spegg.SpeggError):
        spegg.Population([cont(regime=spegg.CONSUMER_RESOURCE)])
    with pytest.raises(spegg.SpeggError):
        spegg.Population([cont(noise_sd=-1.0)])
    with pytest.raises(spegg.SpeggError):
        spegg.Population([cont(effects=np.ones(64, np.int8))])
    p = spegg.Population([cont()])
    with pytest.raises(spegg.SpeggError):
        p.genomes(0)
    with pytest.raises(spegg.SpeggError):
        p.allele_counts(0)
    with pytest.raises(spegg.SpeggError):
        p.write_alleles(0, np.full((3, 2, 64), np.nan, np.float32), 0)
    p.close()
    q = spegg.Population([dict(seed=1, n0=10, capacity=10, n_loci=8)])
    with pytest.raises(spegg.SpeggError):
        q.alleles(0)
    q.close()

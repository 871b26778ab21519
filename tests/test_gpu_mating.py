"""GPU parity of the linkage map and the mating systems (main text: arbitrary
linkage; random, shared-preference or assortative mating, monogamy or
polygynandry; Supplementary S2, "Reproduction"): the HIP library against
the oracle after every generation -- census, genomes, phenotypes, sexes,
survivors and traced parents, bit for bit for biallelic genomes; for
continuous alleles the integer results exactly and the values to the
tolerance of test_gpu_continuous."""
import numpy as np
import pytest

from gpu_helpers import assert_same_state, say
import oracle
from paper_1603_09255_amd import spegg
from test_gpu_continuous import CONT_KEYS, same_state as cont_same_state

pytestmark = pytest.mark.gpu

KEYS = ("seed", "replicate_id", "regime", "n0", "capacity", "n_loci", "mu", "r", "theta", "omega", "K", "fecundity",
        "effects", "n_patches", "migration", "dispersal", "home_return", "linkage", "sexes", "mating",
        "pref_optimum", "pref_width", "monogamy")


def oracle_of(desc):
    keys = KEYS + tuple(k for k in CONT_KEYS if k not in KEYS)
    return oracle.OraclePop(**{k: desc[k] for k in keys if k in desc})


def base(**kw):
    d = dict(seed=11, replicate_id=3, regime=spegg.WF, n0=500, capacity=500, n_loci=64, mu=1e-3, r=0.5,
             theta=0.0, omega=6.0)
    d.update(kw)
    return d


def rmap(L, seed, zeros=(), halves=()):
    g = np.random.default_rng(seed)
    m = g.uniform(0.0, 0.5, L - 1)
    m[list(zeros)] = 0.0
    m[list(halves)] = 0.5
    return m


EFF = np.random.default_rng(4).integers(-4, 5, 96).astype(np.int8)

CASES = [
    ("map_uniform_l150", base(n_loci=150, r=0.3, linkage=np.full(149, 0.3)), 5),
    ("map_random_l256", base(n_loci=256, linkage=rmap(256, 1, zeros=(0, 31, 100), halves=(5, 63))), 5),
    ("map_l1024_small_rates", base(n_loci=1024, n0=200, capacity=200, linkage=rmap(1024, 2) * 0.02), 4),
    ("map_l33", base(n_loci=33, linkage=rmap(33, 3, zeros=(31,))), 5),
    ("sexes_wf", base(sexes=1), 6),
    ("sexes_poisson", base(regime=spegg.POISSON_BH, n0=400, capacity=1200, K=600.0, fecundity=2.4, sexes=1), 6),
    ("preference_sexes", base(sexes=1, mating=spegg.PREFERENCE, pref_optimum=4.0, pref_width=3.0), 6),
    ("assortative", base(mating=spegg.ASSORTATIVE, pref_width=2.0), 6),
    ("assortative_effects", base(n_loci=96, effects=EFF, omega=30.0, sexes=1, mating=spegg.ASSORTATIVE,
                                  pref_width=4.0, r=0.05), 5),
    ("monogamy_sexes", base(sexes=1, monogamy=1), 6),
    ("monogamy_assortative_map", base(monogamy=1, mating=spegg.ASSORTATIVE, pref_width=1.5, n_loci=128,
                                      linkage=rmap(128, 5)), 5),
    ("fallback", base(sexes=1, mating=spegg.PREFERENCE, pref_optimum=500.0, pref_width=0.5, n0=200, capacity=200),
     4),
]


def same(gpu, orc, what, desc, parents=True):
    assert_same_state(gpu, 0, orc, what, parents=parents)
    if desc.get("sexes"):
        assert np.array_equal(gpu.sexes(0), orc.sexes()), f"{what}: sexes differ"


@pytest.mark.parametrize("name,desc,gens", CASES, ids=[c[0] for c in CASES])
def test_mating_lockstep(name, desc, gens):
    say("mating lockstep", name)
    gpu = spegg.Population([desc])
    gpu.set_trace(True)
    orc = oracle_of(desc)
    same(gpu, orc, f"{name} start", desc, parents=False)
    for _ in range(gens):
        gpu.step(1)
        orc.step(1)
        same(gpu, orc, f"{name} generation {orc.generation}", desc)
    gpu.close()
    orc.close()


def test_written_genomes_and_lost_sex():
    d = base(sexes=1, n0=300, capacity=300, mating=spegg.ASSORTATIVE, pref_width=2.0)
    words = np.random.default_rng(8).integers(0, 2 ** 32, (300, 2, 2), dtype=np.uint64).astype(np.uint32)
    say("mating written genomes")
    gpu = spegg.Population([d])
    gpu.set_trace(True)
    orc = oracle_of(d)
    gpu.write_genomes(0, words, 9)
    orc.set_genomes(words, 9)
    same(gpu, orc, "written", d, parents=False)
    for _ in range(3):
        gpu.step(1)
        orc.step(1)
        same(gpu, orc, f"written, generation {orc.generation}", d)
    gpu.close()
    orc.close()
    # two founders: the population ends once a generation has one sex
    d2 = base(sexes=1, n0=2, capacity=2, seed=21)
    gpu = spegg.Population([d2])
    orc = oracle_of(d2)
    for _ in range(30):
        gpu.step(1)
        orc.step(1)
        same(gpu, orc, f"two founders, generation {orc.generation}", d2, parents=False)
    assert orc.stats()["extinct"] == gpu.stats()[0]["extinct"]
    gpu.close()
    orc.close()


def test_continuous_with_mating_and_map():
    d = dict(seed=5, replicate_id=1, regime=spegg.WF, n0=400, capacity=400, n_loci=80, mu=0.01, r=0.2,
             theta=2.0, omega=1.5, genetics=spegg.CONTINUOUS, allele_mean=0.03, allele_sd=0.02, mut_sd_factor=0.5,
             noise_sd=0.1, sexes=1, mating=spegg.ASSORTATIVE, pref_width=0.3, monogamy=1,
             linkage=rmap(80, 9, zeros=(2,)))
    say("continuous mating lockstep")
    gpu = spegg.Population([d])
    gpu.set_trace(True)
    orc = oracle_of(d)
    for g in range(5):
        gpu.step(1)
        orc.step(1)
        cont_same_state(gpu, orc, f"continuous mating, generation {g + 1}")
        assert np.array_equal(gpu.sexes(0), orc.sexes())
    gpu.close()
    orc.close()


def test_batch_invariance_and_shapes():
    a = base(sexes=1, mating=spegg.PREFERENCE, pref_optimum=2.0, pref_width=2.0, replicate_id=31)
    b = base(n_loci=256, linkage=rmap(256, 6), replicate_id=32)
    plain = base(n_loci=256, r=0.2, replicate_id=33)
    say("mating batch invariance")
    ref = []
    for d in (a, b):
        p = spegg.Population([d])
        p.step(4)
        ref.append((p.genomes(0), p.stats()[0]))
        p.close()
    batch = spegg.Population([a, plain, b])
    batch.step(4)
    for i, k in ((0, 0), (1, 2)):
        assert np.array_equal(batch.genomes(k), ref[i][0])
        assert batch.stats()[k] == ref[i][1]
    batch.close()
    for g in (1, 2, 8):
        p = spegg.Population([b])
        p.set_offspring_cap(8, g)
        p.step(4)
        assert np.array_equal(p.genomes(0), ref[1][0]), f"lanes per gamete {g}"
        p.close()


def test_mating_rejections():
    with pytest.raises(spegg.SpeggError):
        spegg.Population([base(n_patches=3, migration=0.1, sexes=1)])
    with pytest.raises(spegg.SpeggError):
        spegg.Population([base(mating=spegg.PREFERENCE, pref_width=0.0)])
    with pytest.raises(spegg.SpeggError):
        spegg.Population([base(n_loci=8, linkage=[0.1, 0.2, 0.7, 0.1, 0.1, 0.1, 0.1])])

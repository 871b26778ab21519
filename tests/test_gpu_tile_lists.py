"""The two ways of launching a generation give the same populations, bit
for bit: one block per tile of every deme's capacity, or resident grids
walking lists of the tiles each generation occupies (the default for
populations of several demes whose censuses can fall below their
capacities).  SPEGG_TILE_LISTS forces either way at creation; every output
-- census, genomes or allelic values, phenotypes, masses, sexes, ages,
survivors and traced parents -- is compared after every generation.  So do
four adults per thread in survive and compact and one (SPEGG_SURV_ITEMS)."""
import os

import numpy as np
import pytest

from gpu_helpers import say
from paper_1603_09255_amd import spegg, workloads

pytestmark = pytest.mark.gpu

PHY = dict(alpha=0.3, gamma=0.75, delta=0.1, attack=2.0, handling=1.0, K=[6000.0, 6000.0], growth=[2.0, 2.0],
           growth_sd=[0.1, 0.1], R0=[6000.0, 6000.0], steepness=5.0, switch_frac=0.5, w_max=8.0, kappa=1.0,
           qJ=0.2, qA=0.4, beta1=0.05, beta2=20.0, beta_s=20.0, maturity=1.0, v_f=1.0, v_m=1.0,
           kappa1=0.5, kappa2=2000.0, kappa3=1.0, breed_every=3)


def phys(rid, n0, cap, L=16):
    return dict(seed=3, replicate_id=rid, regime=spegg.PHYSIOLOGY, n0=n0, capacity=cap, n_loci=L, mu=1e-3, r=0.5,
                genetics=spegg.CONTINUOUS, allele_mean=-2.3 / L, allele_sd=0.02, mut_sd_factor=0.2, noise_sd=0.05,
                exp_transform=1, physiology=dict(PHY))


def cr(rid, **eco):
    e = dict(workloads.CR_ECOLOGY, n0_consumer=60, capacity_consumer=400, habitat=0, encounters=6.0)
    e.update(eco)
    return dict(seed=4, replicate_id=rid, regime=spegg.CONSUMER_RESOURCE, n0=500, capacity=1500, n_loci=64,
                mu=1e-3, r=0.5, omega=0.0, ecology=e)


def poisson(rid, **kw):
    d = dict(seed=6, replicate_id=rid, regime=spegg.POISSON_BH, n0=400, capacity=3000, n_loci=96, mu=1e-3,
             r=0.05, omega=8.0, K=500.0, fecundity=2.2)
    d.update(kw)
    return d


def wf(rid, **kw):
    d = dict(seed=7, replicate_id=rid, regime=spegg.WF, n0=700, capacity=700, n_loci=256, mu=1e-3, r=0.3,
             omega=6.0)
    d.update(kw)
    return d


CONT_KEY = 0x80000000


def shape_key(d):
    """Key of a replicate's offspring-kernel shape: words per haplotype,
    the top bit set for continuous alleles (floats, a multiple of 4)."""
    L = d["n_loci"]
    if d.get("genetics") == spegg.CONTINUOUS:
        return ((L + 3) // 4 * 4) | CONT_KEY
    return (L + 31) // 32


def build(reps, listed):
    old = os.environ.get("SPEGG_TILE_LISTS")
    os.environ["SPEGG_TILE_LISTS"] = "1" if listed else "0"
    try:
        pop = spegg.Population(reps)
    finally:
        if old is None:
            del os.environ["SPEGG_TILE_LISTS"]
        else:
            os.environ["SPEGG_TILE_LISTS"] = old
    pop.set_trace(True)
    return pop


def same(a, b, reps, what):
    sa, sb = a.stats(), b.stats()
    assert sa == sb, f"{what}: stats differ"
    for i, d in enumerate(reps):
        n_species = 2 if d.get("regime") == spegg.CONSUMER_RESOURCE else 1
        n_patches = d.get("n_patches", 1) if n_species == 1 else 1
        assert a.deme_stats(i) == b.deme_stats(i), f"{what}, replicate {i}: deme stats differ"
        for s in range(n_species):
            for p in range(n_patches):
                w = f"{what}, replicate {i} patch {p} species {s}"
                if d.get("genetics") == spegg.CONTINUOUS:
                    assert np.array_equal(a.alleles(i), b.alleles(i)), f"{w}: alleles"
                    assert np.array_equal(a.phenotypes_f(i), b.phenotypes_f(i)), f"{w}: phenotypes"
                else:
                    assert np.array_equal(a.genomes(i, p, s), b.genomes(i, p, s)), f"{w}: genomes"
                    assert np.array_equal(a.phenotypes(i, p, s), b.phenotypes(i, p, s)), f"{w}: phenotypes"
                st = a.deme_stats(i)[p if n_species == 1 else s]
                if st["generation"] > 0 and st["n_parents"] > 0:
                    assert np.array_equal(a.survivors(i, p, s), b.survivors(i, p, s)), f"{w}: survivors"
                    if st["n"] > 0 and not (d.get("regime") == spegg.PHYSIOLOGY and st["n"] == st["n_survivors"]):
                        ga = a.parents(i, p, with_source=True, species=s)
                        gb = b.parents(i, p, with_source=True, species=s)
                        assert all(np.array_equal(x, y) for x, y in zip(ga, gb)), f"{w}: parents"
                if n_species == 2:
                    assert np.array_equal(a.ages(i, s), b.ages(i, s)), f"{w}: ages"
        if d.get("regime") == spegg.PHYSIOLOGY:
            for x, y in zip(a.body(i), b.body(i)):
                assert np.array_equal(x, y), f"{what}, replicate {i}: masses"
            assert np.array_equal(a.sexes(i), b.sexes(i)), f"{what}, replicate {i}: sexes"


CASES = [
    ("physiology", [phys(1, 1500, 12000), phys(2, 300, 9000), phys(3, 2500, 2600, L=40)], 10),
    ("consumer_resource", [cr(4), cr(5, n0_consumer=200, capacity_consumer=800, encounters=10.0),
                           cr(6, attack=0.0)], 8),
    ("poisson_rings_islands", [poisson(7), wf(8, n_patches=5, migration=0.1, n0=300, capacity=900),
                               wf(9, n_patches=4, migration=0.3, dispersal=spegg.ISLAND, home_return=0.5, n0=100,
                                  capacity=400, n_loci=96, r=0.05)], 8),
    ("mixed", [wf(10), poisson(11, n0=5, K=20.0), cr(12), phys(13, 600, 5000), wf(14, n_loci=64, sexes=1)], 8),
    ("wright_fisher", [wf(15), wf(16, n_loci=1024, r=0.01, n0=300, capacity=300), wf(17, n_patches=3,
                                                                                      migration=0.05)], 6),
    ("one_deme", [poisson(18)], 8),
]


@pytest.mark.parametrize("name,reps,gens", CASES, ids=[c[0] for c in CASES])
def test_lists_equal_capacity_grids(name, reps, gens):
    say("tile lists", name)
    dense, listed = build(reps, False), build(reps, True)
    same(dense, listed, reps, f"{name} start")
    for g in range(gens):
        dense.step(1)
        listed.step(1)
        same(dense, listed, reps, f"{name} generation {g + 1}")
    # many generations at once (graph replay), then new kernel shapes
    dense.step(17)
    listed.step(17)
    same(dense, listed, reps, f"{name} after graph replays")
    keys = {shape_key(d) for d in reps}
    for p in (dense, listed):
        for key in keys:
            p.set_offspring_cap(key, 2 if key & CONT_KEY else 1)
    dense.step(3)
    listed.step(3)
    same(dense, listed, reps, f"{name} after a change of shapes")
    dense.close()
    listed.close()


def build_env(reps, **env):
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        pop = spegg.Population(reps)
    finally:
        for k, v in old.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v
    pop.set_trace(True)
    return pop


@pytest.mark.parametrize("name,reps", [
    ("physiology", [phys(1, 1500, 12000), phys(2, 300, 9000), phys(3, 2500, 2600, L=40)]),
    ("poisson_wf", [poisson(4), wf(5, n_patches=3, migration=0.05, n0=300, capacity=900), wf(6, sexes=1)]),
    ("consumer_resource", [cr(7), cr(8, n0_consumer=200, capacity_consumer=800, encounters=10.0)]),
], ids=["physiology", "poisson_wf", "consumer_resource"])
def test_adults_per_thread_equal(name, reps):
    """Four adults per thread (the default for several demes) and one give
    the same populations."""
    say("adults per thread", name)
    four, one = build_env(reps), build_env(reps, SPEGG_SURV_ITEMS="1")
    same(four, one, reps, f"{name} start")
    for g in range(12):
        four.step(1)
        one.step(1)
        same(four, one, reps, f"{name} generation {g + 1}")
    four.close()
    one.close()

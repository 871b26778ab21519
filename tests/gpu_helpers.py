"""Shared helpers of the GPU parity tests: run the HIP library and the
oracle from the same seeded inputs and compare every output exactly."""
import sys

import numpy as np

import oracle
from paper_1603_09255_amd import spegg

ORACLE_KEYS = ("seed", "replicate_id", "regime", "n0", "capacity", "n_loci", "mu", "r", "theta", "omega", "K",
               "fecundity", "effects", "n_patches", "migration", "ecology", "dispersal", "home_return")


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def oracle_pop(desc):
    return oracle.OraclePop(**{k: desc[k] for k in ORACLE_KEYS if k in desc})


def assert_same_state(gpu, rep, orc, what, parents=False):
    """Every output of replicate rep equal to the oracle's: the replicate's
    census, and per deme (patch, or species of the consumer-resource
    regime) the census, genomes, phenotypes, ages, survivors, intake and
    (parents=True) the traced parents with their source patch."""
    sg = gpu.stats()[rep]
    so = orc.total_stats()
    assert sg == so, f"{what}: stats differ\n gpu    {sg}\n oracle {so}"
    per = gpu.deme_stats(rep)
    cr = orc.n_demes == 2 and orc.n_patches == 1
    for k in range(orc.n_demes):
        patch, species = (0, k) if cr else (k, 0)
        wk = f"{what}, {'species' if cr else 'patch'} {k}"
        sok = orc.stats(patch, species)
        assert per[k] == sok, f"{wk}: stats differ\n gpu    {per[k]}\n oracle {sok}"
        g = gpu.genomes(rep, patch, species)
        o = orc.genomes(patch, species)
        assert g.shape == o.shape, f"{wk}: genome shapes {g.shape} vs {o.shape}"
        if not np.array_equal(g, o):
            bad = np.argwhere(g != o)
            raise AssertionError(f"{wk}: {len(bad)} genome words differ, first at {bad[:5].tolist()}")
        assert np.array_equal(gpu.phenotypes(rep, patch, species), orc.phenotypes(patch, species)), \
            f"{wk}: phenotypes differ"
        if cr:
            assert np.array_equal(gpu.ages(rep, species), orc.ages(species=species)), f"{wk}: ages differ"
        if sok["generation"] > 0 and sok["n_parents"] > 0:
            assert np.array_equal(gpu.survivors(rep, patch, species), orc.survivors(patch, species)), \
                f"{wk}: survivor lists differ"
            if cr and species == 1:
                assert np.array_equal(gpu.intake(rep), orc.intake()), f"{wk}: intake differs"
        if parents and sok["generation"] > 0 and orc.newborns(patch, species) > 0:
            gm, gd, gs = gpu.parents(rep, patch, with_source=True, species=species)
            om, od, os_ = orc.parents(patch, with_source=True, species=species)
            assert np.array_equal(gs, os_), f"{wk}: source patches differ"
            assert np.array_equal(gm, om) and np.array_equal(gd, od), f"{wk}: parents differ"


def lockstep(desc, generations, start_words=None, start_gen=0, trace=True, check_every=1):
    """Advance one replicate on the GPU and in the oracle, comparing after
    every `check_every` generations.  Returns the final oracle stats."""
    gpu = spegg.Population([desc])
    orc = oracle_pop(desc)
    if trace:
        gpu.set_trace(True)
    if start_words is not None:
        gpu.write_genomes(0, start_words, start_gen)
        orc.set_genomes(start_words, start_gen)
    assert_same_state(gpu, 0, orc, "start")
    done = 0
    while done < generations:
        k = min(check_every, generations - done)
        gpu.step(k)
        orc.step(k)
        done += k
        assert_same_state(gpu, 0, orc, f"generation {orc.generation}", parents=trace)
    st = orc.stats()
    gpu.close()
    orc.close()
    return st

"""Shared helpers of the GPU parity tests: run the HIP library and the
oracle from the same seeded inputs and compare every output exactly."""
import sys

import numpy as np

import oracle
from paper_1603_09255_amd import spegg

ORACLE_KEYS = ("seed", "replicate_id", "regime", "n0", "capacity", "n_loci", "mu", "r", "theta", "omega", "K",
               "fecundity", "effects")


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def oracle_pop(desc):
    return oracle.OraclePop(**{k: desc[k] for k in ORACLE_KEYS if k in desc})


def assert_same_state(gpu, rep, orc, what, parents=False):
    sg = gpu.stats()[rep]
    so = orc.stats()
    assert sg == so, f"{what}: stats differ\n gpu    {sg}\n oracle {so}"
    g = gpu.genomes(rep)
    o = orc.genomes()
    assert g.shape == o.shape, f"{what}: genome shapes {g.shape} vs {o.shape}"
    if not np.array_equal(g, o):
        bad = np.argwhere(g != o)
        raise AssertionError(f"{what}: {len(bad)} genome words differ, first at {bad[:5].tolist()}")
    assert np.array_equal(gpu.phenotypes(rep), orc.phenotypes()), f"{what}: phenotypes differ"
    if so["generation"] > 0 and so["n_parents"] > 0:
        assert np.array_equal(gpu.survivors(rep), orc.survivors()), f"{what}: survivor lists differ"
    if parents and so["n"] > 0:
        gm, gd = gpu.parents(rep)
        om, od = orc.parents()
        assert np.array_equal(gm, om) and np.array_equal(gd, od), f"{what}: parents differ"


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

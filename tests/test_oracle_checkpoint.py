"""Checkpoint, restore, continue in the oracle: a Wright-Fisher or
Poisson/Beverton-Holt replicate without sexes is wholly described by its
genomes and its generation counter, since each random word is keyed by
(seed, replicate, generation, individual) (main text, Fig. 1: a generation
maps the adults of one census to the next).  A replicate rebuilt from a
read-out continues exactly as the original, in every patch of a ring."""
import numpy as np
import pytest

import oracle

CASES = [
    dict(seed=5, replicate_id=0, regime=0, n0=300, capacity=300, n_loci=96, mu=1e-3, r=0.3, omega=6.0),
    dict(seed=5, replicate_id=1, regime=0, n0=150, capacity=150, n_loci=1024, mu=1e-4, r=0.01, omega=20.0),
    dict(seed=5, replicate_id=2, regime=1, n0=200, capacity=900, n_loci=64, mu=1e-3, r=0.5, omega=8.0, K=300.0,
         fecundity=2.2),
    dict(seed=5, replicate_id=3, regime=0, n0=80, capacity=80, n_loci=256, mu=1e-3, r=0.1, omega=10.0,
         n_patches=3, migration=0.1),
]
STATE = ("generation", "n", "sum_z", "sum_z2")
PER_GENERATION = STATE + ("n_parents", "n_survivors", "extinct", "sum_threshold")


def same(a, b, patches, keys, what):
    for p in range(patches):
        sa, sb = a.stats(p), b.stats(p)
        for k in keys:
            assert sa[k] == sb[k], f"{what}, patch {p}: {k}"
        assert np.array_equal(a.genomes(p), b.genomes(p)), f"{what}, patch {p}: genomes"


@pytest.mark.parametrize("desc", CASES, ids=["wf-bit-serial", "wf-gaps-L1024", "poisson-bh", "ring"])
def test_restored_replicate_continues_alike(desc):
    patches = desc.get("n_patches", 1)
    orig = oracle.OraclePop(**desc)
    orig.step(4)
    gen = orig.stats(0)["generation"]
    rest = oracle.OraclePop(**desc)
    for p in range(patches):
        rest.set_genomes(orig.genomes(p), gen, patch=p)
    same(orig, rest, patches, STATE, "restored")
    for g in range(5):
        orig.step(1)
        rest.step(1)
        same(orig, rest, patches, PER_GENERATION, f"generation {gen + g + 1}")


def test_generation_counter_is_part_of_the_state():
    # the same genomes restored one generation later draw other words
    desc = CASES[0]
    orig = oracle.OraclePop(**desc)
    orig.step(4)
    gen = orig.stats(0)["generation"]
    late = oracle.OraclePop(**desc)
    late.set_genomes(orig.genomes(0), gen + 1)
    orig.step(1)
    late.step(1)
    assert not np.array_equal(orig.genomes(0), late.genomes(0))

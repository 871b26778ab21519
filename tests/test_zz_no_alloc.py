"""The allocation-free allele counts against the allocating entry point:
the same counts, bit for bit, on two calls in a row, the second over a
smaller genome (the library's counter array keeps the first call's
counts, so the second must clear what it uses)."""
import numpy as np
import pytest

from gpu_helpers import oracle_pop, say
from paper_1603_09255_amd import spegg

pytestmark = pytest.mark.gpu


def test_noalloc_allele_counts_match_the_allocating_call():
    reps = [dict(seed=31, replicate_id=7, regime=0, n0=3000, capacity=3000, n_loci=1024, mu=1e-3, r=0.05,
                 theta=0.0, omega=0.0),
            dict(seed=31, replicate_id=8, regime=0, n0=500, capacity=500, n_loci=70, mu=1e-2, r=0.3,
                 theta=0.0, omega=0.0)]
    say("no-alloc allele counts", [(d["n_loci"], d["n0"]) for d in reps])
    pop = spegg.Population(reps)
    pop.step(4)
    for rep in (0, 1):  # the larger genome first, then the smaller one
        a = pop.allele_counts_noalloc(rep)
        b = pop.allele_counts(rep)
        assert a.shape == b.shape == (reps[rep]["n_loci"],)
        assert np.array_equal(a, b), rep
        orc = oracle_pop(reps[rep])
        orc.step(4)
        assert np.array_equal(a.astype(np.int64), orc.alleles().astype(np.int64).sum(axis=(0, 1)))
        orc.close()
    # a length other than the replicate's is rejected before any device work
    out = np.zeros(1024, np.uint32)
    st = pop.lib.spegg_allele_counts_noalloc(pop._h, 1, 0, 0, out.ctypes.data_as(spegg.C.POINTER(spegg.C.c_uint32)),
                                             1024, None)
    assert st == spegg.E_INVALID
    assert np.array_equal(pop.allele_counts_noalloc(1), pop.allele_counts(1))
    pop.close()

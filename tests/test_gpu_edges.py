"""GPU parity at rare edges of the model, bit for bit against the oracle.

- A gamete whose geometric-gap crossover walk reads the word 0xFFFFFFFF
  while a crossover is still to follow (tests/golden/skip_gap_edge.txt): the
  gap table reaches 2^32 inside the genome, and that word must give the
  index of that entry, not a jump past the last boundary (Supplementary S2,
  "Genetics": independent crossovers at each boundary).
- Enough survival draws that near ties |x 2^-32 - p| < 1e-6 occur: both
  sides count the same ones (they are counted, not forced).
"""
import os

import numpy as np
import pytest

from conftest import GOLDEN
from gpu_helpers import lockstep, oracle_pop, say
from paper_1603_09255_amd import spegg, workloads

pytestmark = pytest.mark.gpu


def read_gap_edge():
    with open(os.path.join(GOLDEN, "skip_gap_edge.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    seed, c3, r, L, slots, t, j, stream, word, b, gap = rows[0]
    return dict(seed=int(seed), c3=int(c3), r=float(r), L=int(L), slots=int(slots), t=int(t), j=int(j),
                stream=int(stream), word=int(word), b=int(b), gap=int(gap))


def test_gap_word_at_table_edge_bit_exact():
    e = read_gap_edge()
    assert e["c3"] == 0  # replicate 0, species 0, patch 0
    n = e["slots"]
    desc = dict(seed=e["seed"], replicate_id=0, regime=0, n0=n, capacity=n, n_loci=e["L"], mu=1e-4, r=e["r"],
                theta=0.0, omega=0.0, K=0.0, fecundity=0.0)
    words = workloads.random_genomes(n, e["L"], seed=2024, p_one=0.5)
    say("gap edge", e)
    # one generation from generation t: newborn j's gamete reads the edge word
    lockstep(desc, 1, start_words=words, start_gen=e["t"], trace=True)


def test_near_ties_counted_alike():
    # 4e6 survival draws under Gaussian viability: the oracle counts 8 near
    # ties (pinned against an independent recount in the CPU tests)
    desc = dict(seed=3, replicate_id=5, regime=0, n0=200000, capacity=200000, n_loci=32, mu=1e-3, r=0.5,
                theta=0.0, omega=6.0, K=0.0, fecundity=0.0)
    say("near ties", desc)
    gpu = spegg.Population([desc])
    orc = oracle_pop(desc)
    for _ in range(4):
        gpu.step(5)
        orc.step(5)
        sg, so = gpu.stats()[0], orc.stats()
        assert sg == so, (sg, so)
    assert np.array_equal(gpu.genomes(0), orc.genomes())
    assert so["near_ties"] >= 3
    gpu.close()
    orc.close()


@pytest.mark.parametrize("regime", ["wf", "poisson"])
def test_single_deme_of_many_tile_groups(regime):
    # a census of millions in one deme: survival tiles far beyond one tile
    # group, so every compaction prefix sums group totals and the tiles of
    # its own group
    if regime == "wf":
        desc = dict(seed=21, replicate_id=2, regime=0, n0=4_000_000, capacity=4_000_000, n_loci=32, mu=1e-3,
                    r=0.5, theta=0.0, omega=6.0, K=0.0, fecundity=0.0)
    else:
        desc = dict(seed=22, replicate_id=3, regime=1, n0=3_000_000, capacity=6_000_000, n_loci=32, mu=1e-3,
                    r=0.3, theta=0.0, omega=6.0, K=3_000_000.0, fecundity=2.2)
    say("many tile groups", regime, desc["n0"])
    lockstep(desc, 2, trace=True)

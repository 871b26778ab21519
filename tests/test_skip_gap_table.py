"""Geometric-gap crossovers (Supplementary S2, "Genetics": independent
crossovers at each boundary, drawn as geometric gaps by inversion): the
library's lookup, run on the host over the table the offspring kernel
holds, against the oracle's gap for every word that can reach a table edge.

The full table T_k = floor((1 - (1-r)^(k+1)) 2^32) reaches 2^32 for long
genomes; a word x always lies below that entry, so the kernel keeps the
entries before it, all of which fit the 32-bit words it stores in LDS."""
import math
import os

import numpy as np
import pytest

import oracle
from conftest import GOLDEN
from paper_1603_09255_amd import spegg

ALWAYS = 1 << 32
CASES = [(r, L) for r in (0.044, 0.05, 0.09, 0.0999, 0.163, 0.169) for L in (256, 1024)] + [(0.01, 16384)]


def words_at_edges(T):
    xs = {0, 1, ALWAYS - 2, ALWAYS - 1}
    for k in list(range(0, 8)) + list(range(len(T) - 8, len(T))) + list(range(0, len(T), 37)):
        if 0 <= k < len(T) and T[k] < ALWAYS:
            for d in (-1, 0, 1):
                if 0 <= int(T[k]) + d < ALWAYS:
                    xs.add(int(T[k]) + d)
    return sorted(xs)


@pytest.mark.parametrize("r,L", CASES)
def test_gap_lookup_matches_oracle_at_every_edge(r, L):
    full = oracle.geometric_thresholds(r, L - 1)
    first_always = next((k for k, t in enumerate(full) if int(t) >= ALWAYS), L - 1)
    for x in words_at_edges(full):
        want = oracle.skip_gap(r, L, x)
        for guess in (0, first_always // 2, first_always, L):
            got, n = spegg.geometric_gap(r, L, x, guess)
            assert n == first_always
            assert got == want, (r, L, x, guess, got, want)


@pytest.mark.parametrize("r,L", CASES)
def test_kernel_table_fits_32_bits(r, L):
    full = spegg.threshold_table(2, r, L - 1, cap=L)
    _, n = spegg.geometric_gap(r, L, 0, 0)
    kept = full[:n]
    assert np.all(kept < ALWAYS)
    if n < L - 1:
        assert int(full[n]) == ALWAYS  # the table stops at its first 2^32 entry


@pytest.mark.parametrize("r,k_edge", [(0.1, 427), (0.09, 477)])
def test_reaching_case_exists(r, k_edge):
    # the edge the narrowing once broke: for L = 1024 the table reaches 2^32
    # inside the genome, so the top word must give that index.  The sum of
    # the terms rounds to 1 once (1-r)^(k+1) falls below about 2^-64 (the
    # 64-bit significand of the extended-precision accumulator), so the edge
    # sits near 64 ln 2 / -ln(1-r).
    full = oracle.geometric_thresholds(r, 1023)
    k = next(k for k, t in enumerate(full) if int(t) >= ALWAYS)
    assert abs(k - 64 * math.log(2) / -math.log1p(-r)) < 0.03 * k
    assert k == k_edge
    assert oracle.skip_gap(r, 1024, ALWAYS - 1) == k_edge
    assert spegg.geometric_gap(r, 1024, ALWAYS - 1, 0)[0] == k_edge


def test_gap_edge_fixture_is_what_it_says():
    # the stored gamete of tests/golden/skip_gap_edge.txt: its counter gives
    # the word 0xFFFFFFFF (Philox pinned to the published answers elsewhere),
    # the word's gap is the table's 2^32 index, and a crossover still follows
    with open(os.path.join(GOLDEN, "skip_gap_edge.txt")) as f:
        row = next(ln.split() for ln in f if ln.strip() and not ln.startswith("#"))
    seed, c3, r, L, slots, t, j, stream, word, b, gap = row
    seed, c3, L, t, j, stream, word, b, gap = map(int, (seed, c3, L, t, j, stream, word, b, gap))
    r = float(r)
    assert oracle.recomb_mode(r) == "skip"
    assert j < int(slots) and word >= 4  # gaps are read from word 4 on
    blk = oracle.philox4x32_10([j, (stream << 24) | (word >> 2), t, c3], [seed & 0xFFFFFFFF, seed >> 32])
    assert int(blk[word & 3]) == ALWAYS - 1
    full = oracle.geometric_thresholds(r, L - 1)
    assert gap == next(k for k, v in enumerate(full) if int(v) >= ALWAYS)
    assert oracle.skip_gap(r, L, ALWAYS - 1) == gap
    assert b + 1 + gap <= L - 1

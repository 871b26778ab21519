"""Pins of the oracle's random-number generator and threshold tables.

Philox4x32-10 is pinned to its published known-answer vectors; every
inverse-CDF table is pinned to an independent library CDF (scipy.stats) and
to exact moments of the distribution it encodes.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from conftest import read_kat

TWO32 = 1 << 32


@pytest.mark.parametrize("row", read_kat())
def test_philox_known_answers(row):
    ctr, key, expect = row
    got = oracle.philox4x32_10(ctr, key)
    assert [int(x) for x in got] == expect


def test_philox_bit_balance():
    # 64k words from a counter sweep: each bit position is set with
    # frequency 1/2 within 5 standard errors.
    words = np.array([oracle.philox4x32_10([i, 7 << 24, 3, 5], [1, 0]) for i in range(16384)],
                     dtype=np.uint32).reshape(-1)
    bits = np.unpackbits(words.view(np.uint8)).reshape(-1, 32)
    freq = bits.mean(axis=0)
    se = 0.5 / math.sqrt(words.size)
    assert np.all(np.abs(freq - 0.5) < 5 * se)


def test_prob_threshold_definition():
    assert oracle.prob_threshold(0.0) == 0
    assert oracle.prob_threshold(-0.5) == 0
    assert oracle.prob_threshold(1.0) == TWO32
    assert oracle.prob_threshold(1.5) == TWO32
    assert oracle.prob_threshold(0.5) == 1 << 31
    assert oracle.prob_threshold(0.25) == 1 << 30
    assert oracle.prob_threshold(2.0 ** -32) == 1
    assert oracle.prob_threshold(math.nextafter(1.0, 0.0)) == TWO32 - 1


def _pmf_from_thresholds(T):
    T = np.asarray(T, dtype=np.float64)
    prev = np.concatenate([[0.0], T[:-1]])
    return (T - prev) / TWO32


@pytest.mark.parametrize("lam", [0.5, 2.2, 10.0, 30.0])
def test_poisson_table(lam):
    T = oracle.poisson_thresholds(lam)
    assert T[-1] == TWO32
    assert np.all(np.diff(T.astype(np.int64)) >= 0)
    k = np.arange(len(T) - 1)
    ref = np.floor(stats.poisson.cdf(k, lam) * TWO32)
    assert np.all(np.abs(T[:-1].astype(np.float64) - ref) <= 2)
    pmf = _pmf_from_thresholds(T)
    kk = np.arange(len(T))
    assert abs((pmf * kk).sum() - lam) < 1e-6 * max(lam, 1)
    assert abs((pmf * (kk - lam) ** 2).sum() - lam) < 1e-5 * max(lam, 1)


@pytest.mark.parametrize("L,mu", [(1024, 1e-6), (64, 1e-5), (256, 0.01), (10, 0.3), (1, 0.2)])
def test_binomial_table(L, mu):
    T = oracle.binomial_thresholds(L, mu)
    assert T[-1] == TWO32
    assert len(T) <= L + 1
    k = np.arange(len(T) - 1)
    ref = np.floor(stats.binom.cdf(k, L, mu) * TWO32)
    assert np.all(np.abs(T[:-1].astype(np.float64) - ref) <= 2)
    pmf = _pmf_from_thresholds(T)
    assert abs((pmf * np.arange(len(T))).sum() - L * mu) < 1e-6 * max(L * mu, 1)


def test_binomial_table_exact_small_case():
    # L = 3, mu = 1/2: F = 1/8, 4/8, 7/8, 1 exactly.
    T = oracle.binomial_thresholds(3, 0.5)
    assert list(T) == [TWO32 // 8, TWO32 // 2, 7 * TWO32 // 8, TWO32]
    # mu = 0: a mutation never happens.
    assert list(oracle.binomial_thresholds(1024, 0.0)) == [TWO32]


@pytest.mark.parametrize("r", [0.001, 0.01, 0.1, 0.16])
def test_geometric_table(r):
    n = 1023
    T = oracle.geometric_thresholds(r, n)
    k = np.arange(n)
    ref = np.floor(stats.geom.cdf(k + 1, r) * TWO32)  # P(gap <= k) = 1 - (1-r)^(k+1)
    assert np.all(np.abs(T.astype(np.float64) - ref) <= 2)
    assert T[0] == math.floor(r * TWO32) or abs(int(T[0]) - r * TWO32) <= 1


def test_recomb_mode_rule():
    assert oracle.recomb_mode(0.5) == "raw"
    assert oracle.recomb_mode(0.0) == "zero"
    assert oracle.recomb_mode(0.01) == "skip"
    assert oracle.recomb_mode(0.0999) == "skip"
    assert oracle.recomb_mode(0.10) == "lazy"
    assert oracle.recomb_mode(0.17) == "lazy"
    assert oracle.recomb_mode(0.4999) == "lazy"

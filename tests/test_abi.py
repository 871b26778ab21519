"""Host-side checks of the C ABI (no GPU needed).

The library loads, exports every function include/spegg.h declares, builds
threshold tables bit-identical to the oracle's (independently written from
the same definitions), picks the same crossover-sampling mode, and rejects
invalid descriptors with the documented status before touching a device.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from conftest import ROOT
from paper_1603_09255_amd import spegg, workloads

HEADER = os.path.join(ROOT, "include", "spegg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spegg_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return spegg.load()


def test_library_exports_every_declared_function(lib):
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    declared = int(re.search(r"#define SPEGG_ABI_VERSION (\d+)", open(HEADER).read()).group(1))
    assert lib.spegg_abi_version() == declared


@pytest.mark.parametrize("lam", [0.0, 0.5, 2.2, 10.0, 30.0, 200.0])
def test_poisson_tables_match_oracle(lam):
    assert np.array_equal(spegg.threshold_table(0, lam), oracle.poisson_thresholds(lam))


@pytest.mark.parametrize("L,mu", [(1024, 1e-6), (64, 1e-5), (256, 0.01), (10, 0.3), (1, 0.2), (3, 0.5),
                                  (1024, 0.0), (16384, 1e-4), (257, 0.9)])
def test_binomial_tables_match_oracle(L, mu):
    lib_t = spegg.threshold_table(1, mu, L, cap=L + 1)
    assert np.array_equal(lib_t, oracle.binomial_thresholds(L, mu, cap=L + 1))


@pytest.mark.parametrize("r", [0.001, 0.01, 0.05, 0.1, 0.169])
@pytest.mark.parametrize("n", [0, 1, 63, 1023, 16383])
def test_geometric_tables_match_oracle(r, n):
    assert np.array_equal(spegg.threshold_table(2, r, n, cap=max(n, 1)), oracle.geometric_thresholds(r, n))


@pytest.mark.parametrize("r", [0.0, 1e-9, 0.001, 0.01, 0.0999999, 0.1, 0.17, 0.25, 0.4999999, 0.5])
def test_recomb_mode_matches_oracle(r):
    assert spegg.recomb_mode(r) == oracle.recomb_mode(r)


def base_desc(**kw):
    d = dict(seed=1, replicate_id=0, regime=0, n0=100, capacity=100, n_loci=64, mu=1e-3, r=0.5, theta=0.0,
             omega=8.0, K=0.0, fecundity=0.0)
    d.update(kw)
    return d


@pytest.mark.parametrize("bad,needle", [
    (dict(n_loci=0), "n_loci"),
    (dict(n_loci=16385), "n_loci"),
    (dict(n0=101), "n0"),
    (dict(capacity=0, n0=0), "capacity"),
    (dict(mu=1.0), "mu"),
    (dict(mu=-0.1), "mu"),
    (dict(r=0.51), "r "),
    (dict(regime=7), "regime"),
    (dict(replicate_id=1 << 20), "replicate_id"),
    (dict(effects=np.array([5] + [1] * 63, np.int8)), "effect"),
    (dict(regime=1, fecundity=-1.0), "fecundity"),
    (dict(regime=1, fecundity=5000.0), "fecundity"),
    (dict(theta=float("nan")), "theta"),
    (dict(n_patches=0), "n_patches"),
    (dict(n_patches=1025), "n_patches"),
    (dict(n_patches=2, migration=1.5), "migration"),
    (dict(n_patches=2, regime=1, fecundity=2.0, capacity=200), "Wright-Fisher"),
    (dict(regime=2), "ecology"),
    (dict(ecology=dict(n0_consumer=1, capacity_consumer=1)), "one-species"),
    (dict(regime=2, ecology=dict(n0_consumer=5, capacity_consumer=4, resource_trials=4, match_width=1.0,
                                 resource_K=10.0)), "consumer census"),
    (dict(regime=2, ecology=dict(n0_consumer=1, capacity_consumer=4, resource_trials=0, match_width=1.0,
                                 resource_K=10.0)), "resource_trials"),
    (dict(regime=2, ecology=dict(n0_consumer=1, capacity_consumer=4, resource_trials=4, match_width=0.0,
                                 resource_K=10.0)), "ecology rates"),
    (dict(regime=2, ecology=dict(n0_consumer=1, capacity_consumer=4, resource_trials=4, match_width=1.0,
                                 resource_K=10.0, surv_consumer=(1, 1, 1.5, 0))), "age class 2"),
    (dict(regime=2, n_patches=2, ecology=dict(n0_consumer=1, capacity_consumer=4, resource_trials=4,
                                              match_width=1.0, resource_K=10.0)), "Wright-Fisher"),
])
def test_invalid_descriptors_are_rejected(bad, needle):
    with pytest.raises(spegg.SpeggError) as ei:
        spegg.footprint([base_desc(), base_desc(**bad)])
    assert needle in str(ei.value)
    assert "replicate 1" in str(ei.value)


def test_footprint_counts_every_patch():
    one = spegg.footprint([base_desc(capacity=1000, n0=10)])
    ring = spegg.footprint([base_desc(capacity=1000, n0=10, n_patches=5, migration=0.1)])
    # five patches of buffers (plus the parent-source trace), one set of tables
    assert 4.5 * one < ring < 6 * one


def test_footprint_scales_with_capacity_and_loci():
    a = spegg.footprint([base_desc(capacity=1000, n0=10)])
    b = spegg.footprint([base_desc(capacity=2000, n0=10)])
    c = spegg.footprint([base_desc(capacity=1000, n0=10, n_loci=1024)])
    assert b > a and c > a
    # two genome buffers of capacity x 2W words dominate at L = 1024
    assert c - a >= 2 * 1000 * 2 * (32 - 2) * 4
    d = spegg.footprint([base_desc(capacity=1000, n0=10)] * 3)
    assert d >= 3 * a - 3 * 4096


def test_workload_footprints():
    small, _ = workloads.plain_small()
    scale, _ = workloads.plain_scale()
    assert spegg.footprint([small]) < 1 << 20
    fp = spegg.footprint([scale])
    assert 2 * 250_000 * 256 < fp < 200 << 20


def test_create_rejects_bad_workspace_before_device_use(lib):
    arr, keep = spegg.make_descs([base_desc()])
    h = C.c_void_p()
    st = lib.spegg_pop_create(arr, 1, None, 1 << 20, None, C.byref(h))
    assert st == spegg.E_NOMEM and not h.value
    st = lib.spegg_pop_create(arr, 1, C.c_void_p(4096), 16, None, C.byref(h))
    assert st == spegg.E_NOMEM and "needs" in spegg.last_error()
    st = lib.spegg_pop_create(arr, 1, C.c_void_p(4097), 1 << 30, None, C.byref(h))
    assert st == spegg.E_NOMEM and "aligned" in spegg.last_error()
    st = lib.spegg_pop_create(arr, 0, C.c_void_p(4096), 1 << 30, None, C.byref(h))
    assert st == spegg.E_INVALID


def test_calls_on_null_handle(lib):
    assert lib.spegg_step_generations(None, 1) == spegg.E_INVALID
    assert lib.spegg_stats(None, None, 0) == spegg.E_INVALID
    assert lib.spegg_set_trace(None, 1) == spegg.E_INVALID
    lib.spegg_pop_destroy(None)  # no-op

"""Host-side contract of bench.py (no GPU): one GPU only, the algorithmic
byte count per genotype-locus update, host description, the CPU-baseline
block."""
import os
import subprocess
import sys

import bench
from paper_1603_09255_amd import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_algorithmic_bytes_per_update():
    # parents read once and newborns written once (2 x L/4 bytes per
    # individual over L updates) plus 20 bytes of metadata per individual
    for L in (64, 256, 1024):
        assert bench.bytes_per_update(L) == 0.5 + 20.0 / L
    assert abs(bench.bytes_per_update(1024) - 0.51953125) < 1e-15


def test_host_cpu_description():
    model, nproc = bench.host_cpu()
    assert isinstance(model, str) and model
    assert nproc >= 1


def test_measured_traffic_is_keyed_to_sources_and_shape(monkeypatch):
    sha = bench.device_sources_sha()
    assert len(sha) == 16
    entry = {"device_sources_sha256_16": sha, "lanes_per_gamete_by_W": {32: 4}, "bytes_per_newborn": 700.0}
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, "probe", entry)
    assert bench.measured_traffic("probe", {32: 4}) == 700.0
    assert bench.measured_traffic("probe", {"32": 4}) == 700.0
    assert bench.measured_traffic("probe", {32: 2}) is None
    assert bench.measured_traffic("absent", {32: 4}) is None
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, "probe", dict(entry, device_sources_sha256_16="0" * 16))
    assert bench.measured_traffic("probe", {32: 4}) is None


def test_offspring_bytes_and_philox_blocks_per_newborn():
    # the offspring launch: parents once and the newborn once, plus two
    # parent indices and a phenotype
    assert bench.offspring_bytes_per_newborn(1024) == 512 + 12
    # raw bits: one word per 32 loci, four to a block, per gamete; plus the
    # parent block and one mutation-count block per gamete
    assert bench.philox_blocks_per_newborn(1024, 0.5, 0.0) == 3 + 2 * 8
    # bit-serial: each word of 32 boundaries needs about two blocks (bit
    # planes until every boundary is decided: the maximum of 32 geometric(1/2)
    # draws, about 6.3 planes)
    b = bench.philox_blocks_per_newborn(1024, 0.3, 0.0)
    per_word = (b - 3) / 2 - 1
    assert 1.9 * 32 < per_word < 2.1 * 32
    # r = 1/4: R = 2^30 has no 1 bit past its second plane, so every word is
    # decided within the first block
    assert bench.philox_blocks_per_newborn(256, 0.25, 0.0) == 3 + 2 * (1 + 8)
    # geometric gaps: one word each, r (L - 1) + 1 expected
    assert abs(bench.philox_blocks_per_newborn(1025, 0.01, 0.0) - (3 + 2 * (1 + (0.01 * 1024 + 1) / 4))) < 1e-12


def test_cpu_baseline_batched_is_the_oracle_on_a_replicate_subset():
    reps = workloads.batched_table(n_reps=64)
    small = [dict(d, n0=min(d["n0"], 600), capacity=min(d["n0"], 600)) for d in reps]
    cb = bench.cpu_baseline_batched(small, 4, 1, 2)
    assert cb["kind"] == "oracle" and cb["cores"] == 2 and cb["unit"] == bench.UNIT and cb["value"] > 0
    assert cb["sample"].startswith("4 of the 64 replicates")


def test_cpu_baseline_block_is_the_oracle_on_a_bounded_sample():
    desc, _ = workloads.plain_small(seed=3)
    cb = bench.cpu_baseline(desc, 0.2)
    assert set(cb) >= {"value", "unit", "cores", "kind", "sample"}
    assert cb["kind"] == "oracle" and cb["cores"] == 1 and cb["unit"] == bench.UNIT
    assert cb["value"] > 0
    gens = int(cb["sample"].split()[0])
    assert 1 <= gens <= 200

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


def test_measured_traffic_is_keyed_to_sources_and_shape():
    sha = bench.device_sources_sha()
    assert len(sha) == 16
    shape = bench.MEASURED_TRAFFIC["lanes_per_gamete_by_W"]
    other = {W: (1 if g != 1 else 2) for W, g in shape.items()}
    assert bench.measured_traffic_per_update(other) is None
    if sha == bench.MEASURED_TRAFFIC["device_sources_sha256_16"]:
        assert bench.measured_traffic_per_update(shape) == bench.MEASURED_TRAFFIC["bytes_per_update"]
    else:
        assert bench.measured_traffic_per_update(shape) is None


def test_cpu_baseline_block_is_the_oracle_on_a_bounded_sample():
    desc, _ = workloads.plain_small(seed=3)
    cb = bench.cpu_baseline(desc, 0.2)
    assert set(cb) >= {"value", "unit", "cores", "kind", "sample"}
    assert cb["kind"] == "oracle" and cb["cores"] == 1 and cb["unit"] == bench.UNIT
    assert cb["value"] > 0
    gens = int(cb["sample"].split()[0])
    assert 1 <= gens <= 200

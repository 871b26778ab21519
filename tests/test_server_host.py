"""Host-side checks of the job server: submission validation, footprint
admission limits and result bookkeeping (no device access: the arena is a
placeholder address that no call below dereferences)."""
import pytest

from paper_1603_09255_amd import spegg, workloads

FAKE_ARENA = 1 << 40  # aligned placeholder; submit and usage never touch it


def job(n_reps=2, **kw):
    d = dict(seed=1, n0=300, capacity=300, n_loci=256, r=0.2, mu=1e-5, omega=6.0, n_patches=4, migration=0.01)
    d.update(kw)
    return [dict(d, replicate_id=i) for i in range(n_reps)]


def test_submit_checks():
    one = spegg.footprint(job())
    srv = spegg.Server(4 * one, arena=FAKE_ARENA, stream=None, n_streams=1)
    srv.submit(1, job(), 10)
    with pytest.raises(spegg.SpeggError) as ei:
        srv.submit(1, job(), 10)  # id in use
    assert ei.value.status == spegg.E_INVALID
    with pytest.raises(spegg.SpeggError) as ei:
        srv.submit(2, job(n_reps=9), 10)  # larger than the whole arena
    assert ei.value.status == spegg.E_NOMEM
    with pytest.raises(spegg.SpeggError) as ei:
        srv.submit(3, job(n_loci=0), 10)
    assert ei.value.status == spegg.E_INVALID and "n_loci" in str(ei.value)
    with pytest.raises(spegg.SpeggError):
        srv.submit(4, job(), 0)
    assert srv.usage() == (0, 4 * one - (4 * one) % 256)
    assert srv.poll() == []
    with pytest.raises(spegg.SpeggError) as ei:
        srv.result(1)  # still waiting: no result yet
    assert ei.value.status == spegg.E_INVALID
    srv.close()


def test_create_rejects_misaligned_arena():
    with pytest.raises(spegg.SpeggError) as ei:
        spegg.Server(1 << 20, arena=FAKE_ARENA + 8, stream=None, n_streams=1)
    assert ei.value.status == spegg.E_NOMEM
    with pytest.raises(spegg.SpeggError) as ei:
        spegg.Server(1 << 20, arena=FAKE_ARENA, stream=None, n_streams=9)
    assert ei.value.status == spegg.E_INVALID


def test_serve_trace_shape():
    jobs = workloads.serve_trace(n_jobs=50, rate=20.0)
    arr = [a for a, *_ in jobs]
    assert arr == sorted(arr) and len(jobs) == 50
    # mean inter-arrival near 1/20 s
    assert 0.03 < arr[-1] / 50 < 0.08
    ids = [d["replicate_id"] for _, _, descs, _ in jobs for d in descs]
    assert len(ids) == len(set(ids))
    for _, _, descs, gens in jobs:
        assert 100 <= gens <= 2000 and 8 <= len(descs) <= 256
        d = descs[0]
        assert d["n_patches"] == 100 and d["n_loci"] == 256 and d["migration"] == 0.01
        assert 200 <= d["n0"] <= 5000 and 1e-7 <= d["mu"] <= 1e-4 and 2 <= d["omega"] <= 16
        assert spegg.footprint(descs) > 0

"""GPU checks of the job server: served jobs (admitted, batched with other
jobs, retired) end exactly where their replicates end when run alone, and
where the oracle ends for small ones; admission waits for memory."""
import numpy as np
import pytest

from gpu_helpers import oracle_pop, say
from paper_1603_09255_amd import serve, spegg, workloads

pytestmark = pytest.mark.gpu


def small_job(rid0, n_reps, **kw):
    d = dict(seed=3, n0=120, capacity=120, n_loci=64, r=0.3, mu=1e-3, omega=5.0, n_patches=3, migration=0.05)
    d.update(kw)
    return [dict(d, replicate_id=rid0 + i) for i in range(n_reps)]


def test_served_jobs_equal_alone_and_oracle():
    jobs = [(0.0, 10, small_job(0, 2), 7), (0.0, 11, small_job(10, 3, n_loci=100, r=0.01), 4),
            (0.0, 12, small_job(20, 1, n_patches=1, regime=1, capacity=400, K=150.0, fecundity=2.0), 9)]
    arena = 4 * sum(spegg.footprint(d) for _, _, d, _ in jobs)
    srv = spegg.Server(arena)
    for _, jid, descs, gens in jobs:
        srv.submit(jid, descs, gens)
    for jid in (10, 12):  # their populations stay readable after they finish
        srv.keep(jid)
    finished = []
    for _ in range(20):
        srv.step(2)  # uneven lengths: jobs leave after different steps
        finished += srv.poll()
    assert sorted(finished) == [10, 11, 12]
    assert finished.index(11) < finished.index(10) < finished.index(12)
    for _, jid, descs, gens in jobs:
        got = srv.result(jid)
        alone = spegg.Population(descs)
        alone.step(gens)
        assert got == alone.stats(), f"job {jid}"
        if jid in (10, 12):
            # in the mix and alone: the same genomes, replicate by replicate and patch by patch
            mixed = srv.population(jid)
            for i in range(len(descs)):
                for patch in range(descs[i].get("n_patches", 1)):
                    assert np.array_equal(mixed.genomes(i, patch), alone.genomes(i, patch)), (jid, i, patch)
        alone.close()
        for i, d in enumerate(descs):
            orc = oracle_pop(d)
            orc.step(gens)
            assert got[i] == orc.total_stats(), f"job {jid} replicate {i}"
            if jid in (10, 12):
                for patch in range(d.get("n_patches", 1)):
                    assert np.array_equal(srv.population(jid).genomes(i, patch), orc.genomes(patch))
    assert srv.usage()[0] > 0  # the kept jobs hold their memory
    srv.release(10)
    srv.release(12)
    assert srv.usage()[0] == 0
    with pytest.raises(spegg.SpeggError):
        srv.release(12)
    srv.close()


def test_admission_waits_for_memory_and_fills_freed_space():
    a, b, c = small_job(0, 4), small_job(10, 4), small_job(20, 1)
    fa = spegg.footprint(a)
    srv = spegg.Server(fa + fa // 2)  # room for one big job at a time
    srv.submit(1, a, 3)
    srv.submit(2, b, 3)
    srv.submit(3, c, 3)  # fits beside job 1, but waits behind job 2 (oldest first)
    assert srv.step(1) == (1, 2)
    assert srv.step(2) == (1, 2)  # job 1 finished on the device; retired at the next step or drain
    assert srv.poll() == []
    assert srv.drain() == (2, 0)  # job 1 retired, then 2 and 3 admitted together
    assert srv.poll() == [1]
    assert srv.step(3) == (2, 0)
    assert srv.drain() == (0, 0)
    assert sorted(srv.poll()) == [2, 3]
    for jid, descs in ((1, a), (2, b), (3, c)):
        alone = spegg.Population(descs)
        alone.step(3)
        assert srv.result(jid) == alone.stats()
        alone.close()
    srv.close()


def test_serving_loop_small_trace():
    jobs = workloads.serve_trace(n_jobs=12, rate=200.0, reps=(1, 3), gens=(5, 30), patch_n=(100, 400),
                                 n_patches=8)
    arena = 3 * max(spegg.footprint(d) for _, _, d, _ in jobs)
    say("serving 12 jobs")
    out = serve.run_trace(jobs, arena, quantum=4)
    assert len(out["latency_s"]) == 12 and np.all(out["latency_s"] > 0)
    assert out["p99_s"] >= out["p50_s"]
    for _, jid, descs, gens in jobs[:3]:
        alone = spegg.Population(descs)
        alone.step(gens)
        assert out["results"][jid] == alone.stats()
        alone.close()

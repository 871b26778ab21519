"""Serving loop over the library's job server: jobs are submitted when
their arrival time comes, every scheduling step advances the resident jobs
(continuous batching), and a job's latency is its completion time minus its
arrival time, both on the loop's wall clock."""
import time

import numpy as np

from . import spegg


def run_trace(jobs, arena_bytes, quantum=1, server=None, log=None):
    """Serve jobs [(arrival_s, job_id, descs, generations)] in arrival
    order.  Returns a dict with per-job latencies (s), the makespan, the
    genotype-locus updates done and the jobs' final results."""
    srv = server or spegg.Server(arena_bytes)
    pending = sorted(jobs, key=lambda j: j[0])
    arrival = {j[1]: j[0] for j in pending}
    updates_of = {j[1]: j[3] * sum(d["n0"] * d.get("n_patches", 1) * d["n_loci"] for d in j[2]) for j in pending}
    done, results = {}, {}
    nxt, steps, max_resident = 0, 0, 0
    t0 = time.perf_counter()
    while len(done) < len(pending):
        now = time.perf_counter() - t0
        while nxt < len(pending) and pending[nxt][0] <= now:
            a, jid, descs, gens = pending[nxt]
            srv.submit(jid, descs, gens)
            nxt += 1
        resident, waiting = srv.step(quantum)
        steps += 1
        max_resident = max(max_resident, resident)
        t_done = time.perf_counter() - t0
        for jid in srv.poll():
            done[jid] = t_done
            results[jid] = srv.result(jid)
            if log:
                log(f"serve: job {jid} done at {t_done:.3f} s (latency {t_done - arrival[jid]:.3f} s, "
                    f"{resident} resident, {waiting} waiting)")
        if resident == 0 and waiting == 0 and nxt < len(pending):
            wait = pending[nxt][0] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
    makespan = time.perf_counter() - t0
    if server is None:
        srv.close()
    lat = np.array([done[j] - arrival[j] for j in sorted(done)])
    return {
        "latency_s": lat,
        "p50_s": float(np.percentile(lat, 50)),
        "p99_s": float(np.percentile(lat, 99)),
        "makespan_s": makespan,
        "updates": int(sum(updates_of.values())),
        "steps": steps,
        "max_resident": max_resident,
        "results": results,
    }

#!/usr/bin/env python3
"""Throughput of the per-generation update on one MI355X.

Default workload: the batched form -- 4096 Wright-Fisher replicates of
uneven census N ~ U{500..50000} and genome length L in {64, 256, 1024}
(bit-packed uint32 words), mu log-uniform in [1e-7, 1e-4], r ~ U[0.001,
0.5], Gaussian stabilising selection of width ~ U[2, 16], all advanced
together (Supplementary Fig. S5(B): one flattened loop over replicates and
individuals).  A step is one generation of every replicate (survival,
compaction, parents, gametes, phenotypes, census); the data are synthetic
(seeded parameter table and Philox initial genomes).

Prints one JSON line: genotype-locus updates/s (sum over the timed
generations of N_t x L, divided by wall time with the populations resident
on the device), the roofline of the dominant kernel (the offspring launches)
from HIP events in a second pass, the plain per-replicate GPU loop on a
sample, and the CPU oracle on a replicate subset on the host cores.
Other workloads: --workload scale (one replicate at scale), small, ecology,
serve.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "genotype-locus updates/s on 1 GPU (% HBM roofline); p50/p99 sweep-job latency"
UNIT = "genotype-locus updates/s"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


# HBM bytes per newborn of the dominant offspring launch, from rocprofv3
# FETCH_SIZE and WRITE_SIZE counters scaled by a device copy of known size
# (profiles/*_hbm_traffic.md), by workload; each entry is valid only for the
# device sources with its SHA-256 prefix and the offspring shapes it was
# taken with (lanes-per-gamete cap by genome words W); otherwise the
# traffic figure is null until re-measured.
MEASURED_TRAFFIC = {
    # offspring L = 1024 class of the 4096-replicate table: FETCH 7114392 KiB x 2.00 + WRITE 11669357 KiB x 1.00
    # per launch over 33832793 newborns (profiles/offspring_batched_table_kernel_trace.md)
    "batched": {"device_sources_sha256_16": "cd66b0e8ac59217a", "lanes_per_gamete_by_W": {2: 1, 8: 1, 32: 4},
                "bytes_per_newborn": 783.8},
    # plain method at scale, L = 1024, census about 63.2k: FETCH 10209 KiB x 2.00 + WRITE 22940 KiB x 1.00 per
    # launch (profiles/offspring_plain_scale_hbm_traffic.md)
    "scale": {"device_sources_sha256_16": "cd66b0e8ac59217a", "lanes_per_gamete_by_W": {32: 4},
              "bytes_per_newborn": 702.6},
    # continuous alleles, N = 1e5, L = 256: FETCH 202945 KiB x 2.00 + WRITE 200441 KiB x 1.00 per launch
    # (profiles/offspring_continuous_kernel_trace.md)
    "continuous": {"device_sources_sha256_16": "cd66b0e8ac59217a", "lanes_per_gamete_by_W": {0x80000100: 8},
                   "bytes_per_newborn": 6208.8},
}
# the device code and the compiler flags it is built with
DEVICE_SOURCES = ("csrc/kernels.hip", "csrc/philox.h", "csrc/spegg_internal.h", "build.py")


def device_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for name in DEVICE_SOURCES:
        with open(os.path.join(ROOT, "paper_1603_09255_amd", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, tuned):
    """Counted HBM bytes per newborn of the dominant launch, or None."""
    m = MEASURED_TRAFFIC.get(workload)
    if m is None or device_sources_sha() != m["device_sources_sha256_16"]:
        return None
    if {int(k): v for k, v in tuned.items()} != m["lanes_per_gamete_by_W"]:
        return None
    return m["bytes_per_newborn"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cpu():
    """The host CPU's model name and logical core count."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def device_context(torch, spegg):
    """Figures of the same run to set the kernel against: the achievable
    device-copy bandwidth (1 GiB, read + write counted) and the throughput of
    the device Philox generator the kernels use (a probe with no other
    memory traffic)."""
    n = 1 << 28
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(5):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * 4 * n / (a.elapsed_time(b) / 1e3) / 1e9
    del src, dst
    threads, m = 1 << 21, 256
    out = torch.zeros(threads, dtype=torch.int32, device="cuda")
    spegg.philox_rate(1, m, out)
    torch.cuda.synchronize()
    a.record()
    for _ in range(5):
        spegg.philox_rate(1, m, out)
    b.record()
    torch.cuda.synchronize()
    words = 5 * 4 * threads * m / (a.elapsed_time(b) / 1e3)
    return {"copy_GBs": copy_gbs, "copy_frac_of_peak": copy_gbs / HBM_PEAK_GBS,
            "copy": "device-to-device copy of 1 GiB, 5 times, events on the current stream",
            "philox_words_per_s": words,
            "philox": f"Philox4x32-10 probe: {threads} threads x {m} blocks, 5 launches"}


def bytes_per_update(L):
    # compulsory traffic of a generation per genotype-locus update: read the
    # parents' genomes once and write the newborns' once (2 x L/4 bytes per
    # individual over L updates), plus about 20 bytes of per-individual
    # metadata (phenotype read and write, survivor index, two parent indices)
    return 0.5 + 20.0 / L


def choose_shapes(pop, descs, gcap, generations_per_trial):
    """The offspring kernel's lanes-per-gamete cap per genome length W: timed
    by the autotuner, or pinned (gcap > 0: profiled runs, where a profiler's
    per-dispatch gaps would swamp the tuner's clock)."""
    if isinstance(gcap, dict):
        for W, g in gcap.items():
            pop.set_offspring_cap(W, g)
        return dict(gcap)
    if gcap <= 0:
        return pop.autotune(generations_per_trial=generations_per_trial)
    Ws = sorted({(d["n_loci"] + 31) // 32 for d in descs})
    for W in Ws:
        pop.set_offspring_cap(W, gcap)
    return {W: gcap for W in Ws}


def cpu_baseline(desc, budget_s):
    """The oracle (plain serial loop) on the host, single thread, on as many
    generations of the same workload as fit in about budget_s seconds."""
    import oracle

    keys = ("seed", "replicate_id", "regime", "n0", "capacity", "n_loci", "mu", "r", "theta", "omega", "K",
            "fecundity", "effects", "n_patches", "migration", "genetics", "allele_mean", "allele_sd",
            "mut_sd_factor", "noise_sd", "exp_transform", "physiology")
    orc = oracle.OraclePop(**{k: desc[k] for k in keys if k in desc})
    start_updates = orc.stats()["updates"]
    gens = 0
    t0 = time.perf_counter()
    while True:
        orc.step(1)
        gens += 1
        el = time.perf_counter() - t0
        if el >= budget_s or gens >= 200:
            break
    upd = orc.stats()["updates"] - start_updates
    orc.close()
    model, nproc = host_cpu()
    return {"value": upd / el, "unit": UNIT, "cores": 1, "kind": "oracle", "host_cpu": model, "host_nproc": nproc,
            "sample": f"{gens} generations of the same workload from its initial population "
                      f"({upd} updates, {el:.1f} s, initialisation excluded), one thread"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50, help="timed generations")
    ap.add_argument("--warmup", type=int, default=5, help="untimed generations first")
    ap.add_argument("--cpu-reps", type=int, default=64, help="batched: replicates of the CPU oracle subset")
    ap.add_argument("--cpu-gens", type=int, default=2, help="batched: generations of the CPU oracle subset")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["scale", "batched", "serve", "ecology", "small", "continuous",
                                           "physiology"],
                    default="batched",
                    help="batched: the 4096-replicate batch (default); scale: one replicate at scale; "
                         "small: the small parity configuration (launch- and latency-bound); "
                         "serve: sweep jobs arriving at random, served with continuous batching; "
                         "ecology: 64 replicates of the two-species consumer-resource form; "
                         "continuous: one replicate of continuous allelic values (float32) at scale; "
                         "physiology: 100 replicates of the size-structured consumer of two resources")
    ap.add_argument("--reps", type=int, default=4096, help="replicates of the batched workload")
    ap.add_argument("--plain-sample", type=int, default=64,
                    help="batched: replicates timed one at a time for the plain per-replicate loop")
    ap.add_argument("--jobs", type=int, default=200, help="serve: jobs in the trace")
    ap.add_argument("--rate", type=float, default=20.0, help="serve: arrivals per second")
    ap.add_argument("--sweep", type=str, default="",
                    help="serve: comma-separated arrival rates for a rate sweep after the main trace")
    ap.add_argument("--quantum", type=int, default=8, help="serve: generations per scheduling step")
    ap.add_argument("--full-jobs", action="store_true",
                    help="serve: jobs at their full size (reps U{8..256}, gens U{100..2000}); hours of GPU time")
    ap.add_argument("--gcap", type=int, default=0,
                    help="pin the offspring kernel's lanes-per-gamete cap instead of autotuning (0: autotune)")
    ap.add_argument("--gcaps", type=str, default="",
                    help="pin the cap per genome words instead, as W:cap,W:cap (profiled runs)")
    ap.add_argument("--no-context", action="store_true", help="skip the device copy and Philox probe")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only copy a device buffer of this many MiB 5 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gcaps:
        args.gcap = {int(a): int(b) for a, b in (x.split(":") for x in args.gcaps.split(","))}
    if args.calibrate_copy_mib:
        return calibrate_copy(args.calibrate_copy_mib)
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the workload is one replicate "
              "resident on one device)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1603_09255_amd import spegg, workloads

    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "ecology":
        return bench_ecology(args)
    if args.workload == "small":
        return bench_small(args)
    if args.workload == "continuous":
        return bench_continuous(args)
    if args.workload == "physiology":
        return bench_physiology(args)
    return bench_scale(args)


def bench_scale(args):
    """One replicate at scale (Poisson(2.2) + Beverton-Holt, N0 = 1e5, L = 1024)."""
    import torch

    from paper_1603_09255_amd import spegg, workloads

    desc, _ = workloads.plain_scale(seed=1)
    L = desc["n_loci"]
    torch.cuda.set_device(0)
    log(f"bench: creating population N0={desc['n0']} L={L}")
    pop = spegg.Population([desc])
    torch.cuda.synchronize()
    # the autotuner's trial generations are ordinary generations: part of the warm-up
    tuned = choose_shapes(pop, [desc], args.gcap, 4)
    log(f"bench: lanes per gamete by W: {tuned}; warmup {args.warmup} generations")
    pop.step(args.warmup)
    pop.prepare_graphs()  # the graphs the timed region replays, captured before it
    torch.cuda.synchronize()

    # Timed region: K generations, nothing but the generation launches.
    s0 = pop.stats()[0]
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} generations")
    t0 = time.perf_counter()
    pop.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s1 = pop.stats()[0]
    elapsed = t1 - t0
    updates = s1["updates"] - s0["updates"]
    value = updates / elapsed
    log(f"bench: {updates} updates in {elapsed * 1e3:.2f} ms ({value:.4g}/s); N now {s1['n']}")

    # Roofline pass: the same number of generations with the offspring
    # kernel bracketed by HIP events on the population's stream.
    pop.set_timing(["offspring"])
    pop.kernel_times()
    s0b = pop.stats()[0]
    torch.cuda.synchronize()
    t0b = time.perf_counter()
    pop.step(args.steps)
    torch.cuda.synchronize()
    t1b = time.perf_counter()
    s1b = pop.stats()[0]
    kt = pop.kernel_times()
    pop.set_timing([])
    updates_b = s1b["updates"] - s0b["updates"]
    off_ms, off_n = kt["offspring"]
    per_launch_bytes = updates_b / max(off_n, 1) * bytes_per_update(L)
    avg_launch_s = off_ms / 1e3 / max(off_n, 1)
    achieved = per_launch_bytes / avg_launch_s / 1e9
    log(f"bench: event pass {(t1b - t0b) * 1e3:.2f} ms; offspring kernel avg {avg_launch_s * 1e6:.2f} us x {off_n}")
    pop.close()
    context = device_context(torch, spegg)
    log(f"bench: device copy {context['copy_GBs']:.0f} GB/s, Philox {context['philox_words_per_s']:.3g} words/s")
    # the same launches against the bytes they would move if every parent
    # gather missed the caches (parents read once per newborn gamete)
    gather_miss = 0.75 + 20.0 / L

    out = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "plain method at scale: 1 replicate, N0=100000 (capacity 250000), L=1024 loci in uint32 "
                        "words, effects on [-4,4], r=0.01, mu=1e-6, Poisson(2.2) fecundity, Beverton-Holt "
                        "survival K=100000, stabilising selection width 64",
            "replicates": 1,
            "n_loci": L,
            "generations_timed": args.steps,
            "mean_census": updates / args.steps / L,
            "offspring_lanes_per_gamete_by_W": {str(k): v for k, v in tuned.items()},
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "offspring",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": (None if measured_traffic("scale", tuned) is None else
                        measured_traffic("scale", tuned) * updates_b / L / max(off_n, 1)),
            "traffic_unit": "HBM bytes per launch (rocprofv3 counters, scaled)",
            "bytes_per_update": bytes_per_update(L),
            "avg_launch_us": avg_launch_s * 1e6,
            "launches": off_n,
            "timing": "HIP events around each offspring launch, in a second pass of the same length",
            "bytes_per_update_gather_miss": gather_miss,
            "frac_gather_miss": achieved * gather_miss / bytes_per_update(L) / HBM_PEAK_GBS,
            "frac_of_copy": achieved / context["copy_GBs"],
        },
        "context": context,
    }
    if not args.no_cpu_baseline:
        log(f"bench: CPU oracle sample, about {args.cpu_seconds:.0f} s")
        out["cpu_baseline"] = cpu_baseline(desc, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def cont_bytes_per_update(L):
    # continuous alleles: read the parents' values once and write the
    # newborns' once (2 x 2 x 4 bytes per locus and individual over one
    # update per locus), plus the same ~20 bytes of per-individual metadata
    return 16.0 + 20.0 / L


def bench_continuous(args):
    """One replicate of continuous allelic values (Supplementary S2,
    "Genetics"): N = 100000, L = 256 float32 loci, Wright-Fisher."""
    import torch

    from paper_1603_09255_amd import spegg, workloads

    desc, _ = workloads.continuous_scale(seed=1)
    L = desc["n_loci"]
    torch.cuda.set_device(0)
    log(f"bench: creating continuous population N={desc['n0']} L={L}")
    pop = spegg.Population([desc])
    torch.cuda.synchronize()
    tuned = pop.autotune(generations_per_trial=2) if args.gcap == 0 else {}
    if args.gcap and not isinstance(args.gcap, dict):
        pop.set_offspring_cap(((L + 3) // 4 * 4) | 0x80000000, args.gcap)
        tuned = {((L + 3) // 4 * 4) | 0x80000000: args.gcap}
    log(f"bench: lanes per gamete by genome key: {tuned}; warmup {args.warmup} generations")
    pop.step(args.warmup)
    pop.prepare_graphs()
    torch.cuda.synchronize()
    s0 = pop.stats()[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pop.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s1 = pop.stats()[0]
    elapsed = t1 - t0
    updates = s1["updates"] - s0["updates"]
    value = updates / elapsed
    log(f"bench: {updates} updates in {elapsed * 1e3:.2f} ms ({value:.4g}/s)")
    pop.set_timing(["survive", "compact", "offspring"])
    pop.kernel_times()
    s0b = pop.stats()[0]
    pop.step(args.steps)
    torch.cuda.synchronize()
    s1b = pop.stats()[0]
    kt = pop.kernel_times()
    pop.set_timing([])
    pop.close()
    updates_b = s1b["updates"] - s0b["updates"]
    off_ms, off_n = kt["offspring"]
    avg_launch_s = off_ms / 1e3 / max(off_n, 1)
    achieved = updates_b / max(off_n, 1) * cont_bytes_per_update(L) / avg_launch_s / 1e9
    gather_miss = 24.0 + 20.0 / L  # each newborn gamete reads both parental haplotypes
    out = {
        "metric": METRIC,
        "value": value,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "continuous allelic values (Supplementary S2): 1 Wright-Fisher replicate, N=100000, "
                        "L=256 float32 loci, free recombination, mu=1e-3 with N(0, 0.005^2) changes, noise 0.2, "
                        "stabilising selection (optimum 2.6, width 1)",
            "replicates": 1,
            "n_loci": L,
            "generations_timed": args.steps,
            "offspring_lanes_per_gamete": {str(k): v for k, v in tuned.items()},
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "offspring (continuous alleles)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": (None if measured_traffic("continuous", tuned) is None else
                        measured_traffic("continuous", tuned) * updates_b / L / max(off_n, 1)),
            "traffic_unit": "HBM bytes per launch (rocprofv3 counters, scaled)",
            "bytes_per_update": cont_bytes_per_update(L),
            "avg_launch_us": avg_launch_s * 1e6,
            "launches": off_n,
            "timing": "HIP events around each offspring launch, in a second pass of the same length",
            "bytes_per_update_gather_miss": gather_miss,
            "frac_gather_miss": achieved * gather_miss / cont_bytes_per_update(L) / HBM_PEAK_GBS,
            "kernel_us": {k: (v[0] * 1e3 / max(v[1], 1)) for k, v in kt.items() if v[1]},
        },
    }
    if not args.no_cpu_baseline:
        log(f"bench: CPU oracle sample, about {args.cpu_seconds:.0f} s")
        out["cpu_baseline"] = cpu_baseline(desc, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def bench_small(args):
    """The small parity configuration (one Wright-Fisher replicate, N = 1000,
    L = 64): far too little work to fill the device, so it is bound by
    launch and dependency latency; reported as microseconds per generation,
    with no roofline claim."""
    import torch

    from paper_1603_09255_amd import spegg, workloads

    desc, _ = workloads.plain_small(seed=1)
    torch.cuda.set_device(0)
    pop = spegg.Population([desc])
    pop.step(args.warmup)
    torch.cuda.synchronize()
    s0 = pop.stats()[0]["updates"]
    t0 = time.perf_counter()
    pop.step(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    updates = pop.stats()[0]["updates"] - s0
    pop.set_timing()
    pop.kernel_times()
    pop.step(min(args.steps, 200))
    kt = pop.kernel_times()
    pop.close()
    out = {
        "metric": METRIC, "value": updates / elapsed, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "small parity configuration: 1 Wright-Fisher replicate, N=1000, L=64, unit effects, "
                               "selection width 8, r=0.5, mu=1e-5",
                   "us_per_generation": elapsed * 1e6 / args.steps,
                   "kernel_us_per_launch": {k: v[0] * 1e3 / v[1] for k, v in kt.items() if v[1]},
                   "note": "launch- and latency-bound: 64000 updates per generation"},
    }
    print(json.dumps(out), flush=True)


ALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9  # VALU lane operations/s: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
PHILOX_OPS = 40  # VALU operations per Philox4x32-10 block: 10 rounds of 2 v_mad_u64_u32 + 2 v_bitop3_b32


def offspring_bytes_per_newborn(L):
    """Compulsory bytes of the offspring launch per newborn: the parental
    genomes read once (L/4 per newborn when parents and newborns are as
    many) and the newborn written once (L/4), two parent indices read and
    the phenotype written (12 B)."""
    return L / 2.0 + 12.0


def recomb_mode(r):
    return "raw" if r == 0.5 else "zero" if r == 0.0 else "skip" if r < 0.10 else "lazy"


def philox_blocks_per_newborn(L, r, mu, migration=False):
    """Expected Philox4x32-10 blocks the model's draws take per newborn in
    the library's stream layout: one for the parents, one per gamete for
    the mutation count, one for a migration draw; per gamete the crossover
    words -- raw bits (one word per 32 loci), the phase block plus one word
    per geometric gap (skip), or the phase block plus, per word of 32
    boundaries, bit planes until every boundary is decided or R has no bit
    left (bit-serial) -- and about two words per mutated locus."""
    W = (L + 31) // 32
    mode = recomb_mode(r)
    if mode == "raw":
        gam = math.ceil(W / 4)
    elif mode == "zero":
        gam = 1.0
    elif mode == "skip":
        gam = 1.0 + (r * (L - 1) + 1.0) / 4.0
    else:
        R = int(math.floor(r * 4294967296.0))
        nsig = 32 - ((R & -R).bit_length() - 1)  # planes until R has no 1 bit left
        gam = 1.0
        for w in range(W):
            b = min(32 * w + 32, L) - max(32 * w, 1)  # boundaries 32w .. 32w + 31 within 1 .. L - 1
            if b <= 0:
                continue
            gam += sum(1.0 - (1.0 - 2.0 ** (-4 * m)) ** b if m else 1.0 for m in range((nsig + 3) // 4))
    return 3.0 + (1.0 if migration else 0.0) + 2.0 * (gam + L * mu / 2.0)


def cpu_baseline_batched(reps, n_sample, gens, threads):
    """The oracle (plain serial loop per replicate) on an evenly spaced
    subset of the replicates, replicates spread over host threads (ctypes
    releases the interpreter lock for the oracle's calls)."""
    import concurrent.futures

    import oracle

    keys = ("seed", "replicate_id", "regime", "n0", "capacity", "n_loci", "mu", "r", "theta", "omega", "K",
            "fecundity", "effects", "n_patches", "migration")
    stride = max(1, len(reps) // n_sample)
    sample = reps[::stride][:n_sample]
    with concurrent.futures.ThreadPoolExecutor(threads) as ex:
        pops = list(ex.map(lambda d: oracle.OraclePop(**{k: d[k] for k in keys if k in d}), sample))
        t0 = time.perf_counter()
        list(ex.map(lambda o: o.step(gens), pops))
        el = time.perf_counter() - t0
    upd = sum(o.stats()["updates"] for o in pops)
    for o in pops:
        o.close()
    model, nproc = host_cpu()
    return {"value": upd / el, "unit": UNIT, "cores": threads, "kind": "oracle", "host_cpu": model,
            "host_nproc": nproc,
            "sample": f"{len(sample)} of the {len(reps)} replicates (every {stride}th), {gens} generations each "
                      f"from the initial populations, {upd} updates in {el:.1f} s on {threads} threads, one "
                      "replicate per thread at a time; a rate of the same workload mix, not extrapolated"}


def per_rep_updates(s0, s1):
    return [b["updates"] - a["updates"] for a, b in zip(s0, s1)]


def bench_batched(args):
    """Replicates of uneven N and L advanced together, against the plain
    per-replicate loop (the same kernels, one replicate at a time, eager
    launches) on a sample of the same replicates."""
    import torch

    from paper_1603_09255_amd import spegg

    from paper_1603_09255_amd import workloads

    reps = workloads.batched_table(n_reps=args.reps)
    Ls = [d["n_loci"] for d in reps]
    torch.cuda.set_device(0)
    log(f"bench: creating batch of {len(reps)} replicates")
    pop = spegg.Population(reps)
    torch.cuda.synchronize()
    tuned = choose_shapes(pop, reps, args.gcap, 2)
    log(f"bench: lanes per gamete by W: {tuned}; warmup {args.warmup} generations")
    pop.step(args.warmup)
    pop.prepare_graphs()  # the graphs the timed region replays, captured before it
    torch.cuda.synchronize()
    s0 = pop.stats()
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} generations of the batch")
    t0 = time.perf_counter()
    pop.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s1 = pop.stats()
    elapsed = t1 - t0
    du = per_rep_updates(s0, s1)
    updates = sum(du)
    value = updates / elapsed
    gen_bytes = sum(u * bytes_per_update(L) for u, L in zip(du, Ls))
    log(f"bench: batch {updates} updates in {elapsed:.3f} s ({value:.4g}/s)")

    # Roofline pass: the same generations launched eagerly with every kernel
    # bracketed by HIP events on the population's stream.
    gens_b = min(args.steps, 20)
    pop.set_timing()
    pop.kernel_times()
    pop.offspring_class_times()
    sb0 = pop.stats()
    pop.step(gens_b)
    kt = pop.kernel_times()
    ct = pop.offspring_class_times()
    sb1 = pop.stats()
    pop.set_timing([])
    pop.close()
    dub = per_rep_updates(sb0, sb1)
    W_of = [(L + 31) // 32 for L in Ls]
    classes = []
    for wmin, wmax, ms, n in ct:
        members = [i for i in range(len(reps)) if wmin <= W_of[i] <= wmax]
        newborns = sum(dub[i] / Ls[i] for i in members)
        byts = sum(dub[i] / Ls[i] * offspring_bytes_per_newborn(Ls[i]) for i in members)
        blocks = sum(dub[i] / Ls[i] * philox_blocks_per_newborn(Ls[i], reps[i]["r"], reps[i]["mu"])
                     for i in members)
        avg_s = ms / 1e3 / max(n, 1)
        ach = byts / max(n, 1) / avg_s / 1e9 if n else 0.0
        alu = blocks * PHILOX_OPS / max(n, 1) / avg_s if n else 0.0
        classes.append({"n_loci": sorted({Ls[i] for i in members}), "replicates": len(members),
                        "newborns_per_launch": newborns / max(n, 1), "avg_launch_us": avg_s * 1e6, "launches": n,
                        "bytes_per_launch": byts / max(n, 1), "achieved_GBs": ach, "frac": ach / HBM_PEAK_GBS,
                        "philox_blocks_per_launch": blocks / max(n, 1),
                        "alu_frac": alu / ALU_PEAK_OPS})
    dom = max(classes, key=lambda c: c["avg_launch_us"] * c["launches"])
    off_ms, off_n = kt["offspring"]
    off_bytes = sum(dub[i] / Ls[i] * offspring_bytes_per_newborn(Ls[i]) for i in range(len(reps)))
    per_kind_us = {k: v[0] * 1e3 / gens_b for k, v in kt.items() if v[1]}
    log(f"bench: event pass, per generation: " + ", ".join(f"{k} {v:.0f} us" for k, v in per_kind_us.items()))
    for c in classes:
        log(f"bench: offspring L={c['n_loci']}: {c['avg_launch_us']:.0f} us, {c['achieved_GBs']:.0f} GB/s "
            f"(frac {c['frac']:.3f}), Philox ALU frac {c['alu_frac']:.3f}")

    # plain per-replicate loop on a sample
    sample = reps[: args.plain_sample]
    plain_updates, plain_time = 0, 0.0
    for d in sample:
        p = spegg.Population([d])
        p.set_graph(False)
        p.step(args.warmup)
        torch.cuda.synchronize()
        a0 = p.stats()[0]["updates"]
        ta = time.perf_counter()
        p.step(args.steps)
        torch.cuda.synchronize()
        plain_time += time.perf_counter() - ta
        plain_updates += p.stats()[0]["updates"] - a0
        p.close()
    plain_rate = plain_updates / plain_time if plain_time > 0 else None  # --plain-sample 0: not measured
    if plain_rate:
        log(f"bench: plain loop over {len(sample)} replicates: {plain_rate:.4g} updates/s")
    context = None if args.no_context else device_context(torch, spegg)
    traffic = measured_traffic("batched", tuned)
    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"batched form: {len(reps)} Wright-Fisher replicates, N ~ U{{500..50000}}, "
                               "L from {64,256,1024} (uint32 words), mu log-uniform [1e-7,1e-4], r ~ U[0.001,0.5], "
                               "selection width ~ U[2,16], all advanced together, one graph replay per 16 "
                               "generations",
                   "replicates": len(reps), "generations_timed": args.steps,
                   "mean_census_total": updates / args.steps / (sum(Ls) / len(Ls)) if Ls else 0,
                   "plain_loop_updates_per_s": plain_rate, "plain_loop_sample": len(sample),
                   "speedup_vs_plain_loop": value / plain_rate if plain_rate else None,
                   "offspring_lanes_per_gamete_by_W": {str(k): v for k, v in tuned.items()},
                   "kernel_us_per_generation": per_kind_us},
        "roofline": {"bound": "hbm", "kernel": f"offspring, L={dom['n_loci']} launch class",
                     "achieved": dom["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": dom["frac"],
                     "traffic": None if traffic is None else traffic * dom["newborns_per_launch"],
                     "traffic_unit": "HBM bytes per launch (rocprofv3 counters, scaled)",
                     "bytes_per_newborn": "L/2 + 12", "avg_launch_us": dom["avg_launch_us"],
                     "launches": dom["launches"],
                     "timing": "HIP events around each launch, in a second pass of " + str(gens_b) + " generations",
                     "alu": {"philox_blocks_per_launch": dom["philox_blocks_per_launch"],
                             "ops_per_block": PHILOX_OPS, "peak_ops_per_s": ALU_PEAK_OPS,
                             "frac": dom["alu_frac"]},
                     "classes": classes,
                     "offspring_all": {"achieved": off_bytes / (off_ms / 1e3) / 1e9 if off_ms else None,
                                       "frac": off_bytes / (off_ms / 1e3) / 1e9 / HBM_PEAK_GBS if off_ms else None},
                     "generation": {"bytes_per_update": "0.5 + 20/L", "achieved": gen_bytes / elapsed / 1e9,
                                    "frac": gen_bytes / elapsed / 1e9 / HBM_PEAK_GBS}},
        "context": context,
    }
    if not args.no_cpu_baseline:
        threads = min(os.cpu_count() or 1, 16)
        log(f"bench: CPU oracle on a replicate subset, {threads} threads")
        out["cpu_baseline"] = cpu_baseline_batched(reps, args.cpu_reps, args.cpu_gens, threads)
    print(json.dumps(out), flush=True)


def bench_ecology(args):
    """64 replicates of the consumer-resource form (resource 1e5, consumer
    1e4, L = 256, ages 0-3), all advanced together; updates count carried
    survivors and newborns of both species."""
    import torch

    from paper_1603_09255_amd import spegg, workloads

    reps, _ = workloads.consumer_resource(n_reps=64)
    torch.cuda.set_device(0)
    log(f"bench: creating {len(reps)} consumer-resource replicates")
    pop = spegg.Population(reps)
    tuned = choose_shapes(pop, reps, args.gcap, 2)
    pop.step(args.warmup)
    torch.cuda.synchronize()
    s0 = sum(r["updates"] for r in pop.stats())
    t0 = time.perf_counter()
    pop.step(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = pop.stats()
    updates = sum(r["updates"] for r in st) - s0
    value = updates / elapsed
    log(f"bench: {updates} updates in {elapsed:.3f} s ({value:.4g}/s)")
    # roofline pass: offspring launches bracketed by events
    pop.set_timing(["offspring"])
    pop.kernel_times()
    sb0 = sum(r["updates"] for r in pop.stats())
    gens_b = min(args.steps, 50)
    pop.step(gens_b)
    kt = pop.kernel_times()
    sb1 = sum(r["updates"] for r in pop.stats())
    pop.set_timing([])
    per = pop.deme_stats(0)
    pop.close()
    off_ms, off_n = kt["offspring"]
    bpu = bytes_per_update(256)
    achieved = (sb1 - sb0) * bpu / (off_ms / 1e3) / 1e9
    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": "two-species consumer-resource form: 64 replicates, resource N0=1e5 (capacity 2.5e5), "
                               "consumer N0=1e4 (capacity 5e4), L=256 each, capture by Gaussian phenotype matching "
                               "(width 4), ages 0-3, resource logistic binomial fecundity, consumer fecundity "
                               "Poisson in intake",
                   "replicates": len(reps), "generations_timed": args.steps,
                   "replicate0_resource_n": per[0]["n"], "replicate0_consumer_n": per[1]["n"],
                   "replicate0_captures": per[1]["captures"],
                   "offspring_lanes_per_gamete_by_W": {str(k): v for k, v in tuned.items()}},
        "roofline": {"bound": "hbm", "kernel": "offspring", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None, "bytes_per_update": bpu,
                     "launches": off_n, "generations": gens_b},
    }
    print(json.dumps(out), flush=True)


def phys_bytes_per_individual():
    """Compulsory HBM bytes of one time step per individual of the
    physiology regime: survive reads X, Y (doubles), the phenotype (float)
    and the sex and writes X, Y, the gonads and the fate (47 B); compact
    reads the fate and writes a survivor index (6 B); a survivor moves to the
    next census with its masses, phenotype and sex (2 x 21 B).  Its allelic
    values need not move (the library keeps them in place)."""
    return 47.0 + 6.0 + 42.0


def phys_bytes_per_recruit(L):
    """Compulsory bytes of one recruit: its parents' allelic values read
    (2 x 2 x 4 L bytes, each gamete taking every locus from one of a
    parent's two haplotypes: 8 B per locus) and its own written (8 L), its
    masses, phenotype and sex written (21 B)."""
    return 16.0 * L + 21.0


def bench_physiology(args):
    """100 replicates of the physiologically structured consumer of
    Supplementary S2 (50000 founders each, L = 16 continuous loci), all
    advanced together, one time step per generation."""
    import torch

    from paper_1603_09255_amd import spegg, workloads

    reps, _ = workloads.physiology_batch(n_reps=100)
    L = reps[0]["n_loci"]
    torch.cuda.set_device(0)
    log(f"bench: creating {len(reps)} physiology replicates")
    pop = spegg.Population(reps)
    pop.step(args.warmup)
    pop.prepare_graphs()
    torch.cuda.synchronize()
    st0 = pop.stats()
    s0 = sum(r["updates"] for r in st0)
    t0 = time.perf_counter()
    pop.step(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = pop.stats()
    updates = sum(r["updates"] for r in st) - s0
    inds = updates / L  # individual-steps
    value = updates / elapsed
    log(f"bench: {updates} updates ({inds:.4g} individual-steps) in {elapsed:.3f} s ({value:.4g}/s)")
    # second pass, step by step: kernel times from events, and the recruits
    # per individual-step (census minus survivors after each step)
    pop.set_timing(["survive", "compact", "offspring", "carry"])
    pop.kernel_times()
    gens_b = min(args.steps, 50)
    recruits, inds_b = 0, 0
    for _ in range(gens_b):
        pop.step(1)
        for r in pop.stats():
            recruits += r["n"] - r["n_survivors"]
            inds_b += r["n"]
    kt = pop.kernel_times()
    pop.set_timing([])
    per_kind_us = {k: v[0] * 1e3 / gens_b for k, v in kt.items() if v[1]}
    log("bench: per step: " + ", ".join(f"{k} {v:.0f} us" for k, v in per_kind_us.items()))
    pop.close()
    recruit_rate = recruits / max(inds_b, 1)
    bytes_per_ind = phys_bytes_per_individual() + recruit_rate * phys_bytes_per_recruit(L)
    gen_bytes = inds * bytes_per_ind
    achieved = gen_bytes / elapsed / 1e9
    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "physiologically structured consumer of two resources (Supplementary S2): 100 "
                               "replicates of 50000 founders (capacity 200000), neonate mass exp(z) from 16 "
                               "continuous loci, masses in double, breeding every 5 steps",
                   "replicates": len(reps), "generations_timed": args.steps,
                   "individual_steps_per_s": inds / elapsed,
                   "mean_census": inds / args.steps / len(reps),
                   "replicate0_resources": st[0]["resource"],
                   "kernel_us_per_step": per_kind_us},
        "roofline": {"bound": "hbm", "kernel": "whole time step (survive, compact, carry, offspring)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "bytes_per_individual_step": bytes_per_ind,
                     "bytes_model": "95 B per individual-step (survive 47, compact 6, survivors' masses, phenotype "
                                    "and sex moved 42) + (16 L + 21) B per recruit, recruits per individual-step "
                                    f"{recruit_rate:.4g} from the second pass",
                     "timing": "wall clock of the timed steps; kernel times from HIP events in a second pass"},
        "context": {"paper": "the paper reports more than 200x over one CPU core for its size-structured case "
                             "study on one commodity GPGPU (main text, Fig. 2B), hardware and parameters other "
                             "than these"},
    }
    if not args.no_cpu_baseline:
        log(f"bench: CPU oracle sample, about {args.cpu_seconds:.0f} s")
        out["cpu_baseline"] = cpu_baseline(reps[0], args.cpu_seconds)
    print(json.dumps(out), flush=True)


SERVE_SCALED = dict(reps=(1, 8), gens=(20, 200))  # the served jobs, cut to fit a bench run


def bench_serve(args):
    """Sweep jobs of 100-patch rings (L = 256, m = 0.01) arriving as a
    Poisson process, admitted by footprint and served with continuous
    batching; latency = completion - arrival on the loop's clock."""
    import torch

    from paper_1603_09255_amd import serve, spegg, workloads

    torch.cuda.set_device(0)
    shape = {} if args.full_jobs else SERVE_SCALED
    free, _total = torch.cuda.mem_get_info()
    arena = int(free * 0.8) & ~255
    srv = spegg.Server(arena)

    def one(rate, n_jobs):
        jobs = workloads.serve_trace(n_jobs=n_jobs, rate=rate, **shape)
        log(f"bench: serving {n_jobs} jobs at {rate}/s")
        # full-size jobs run for minutes: a line per finished job shows progress
        out = serve.run_trace(jobs, arena, quantum=args.quantum, server=srv, log=log if args.full_jobs else None)
        return {"rate_per_s": rate, "jobs": n_jobs, "p50_s": out["p50_s"], "p99_s": out["p99_s"],
                "makespan_s": out["makespan_s"], "updates_per_s": out["updates"] / out["makespan_s"],
                "max_resident": out["max_resident"], "steps": out["steps"]}

    # warm-up: a few jobs to load code and allocator paths
    serve.run_trace(workloads.serve_trace(n_jobs=3, rate=1000.0, seed=99, **shape), arena, quantum=args.quantum,
                    server=srv)
    main_run = one(args.rate, args.jobs)
    sweep = [one(float(r), max(20, args.jobs // 4)) for r in args.sweep.split(",") if r]
    srv.close()
    out = {
        "metric": METRIC, "value": main_run["updates_per_s"], "unit": UNIT, "n_gpus": 1, "steps": main_run["steps"],
        "warmup": 3, "ms_per_step": main_run["makespan_s"] * 1e3 / max(main_run["steps"], 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "served sweep jobs: Poisson arrivals; per job one parameter point (per-patch N "
                               "~U{200..5000}, mu log-uniform [1e-7,1e-4], r ~U[0.001,0.5], width ~U[2,16]) run as "
                               "replicates of a 100-patch ring, L=256, m=0.01; "
                               + ("full-size jobs (reps U{8..256}, gens U{100..2000})" if args.full_jobs else
                                  "jobs cut to reps U{1..8}, gens U{20..200}"),
                   "jobs": args.jobs, "arrival_rate_per_s": args.rate, "quantum_generations": args.quantum,
                   "p50_latency_s": main_run["p50_s"], "p99_latency_s": main_run["p99_s"],
                   "makespan_s": main_run["makespan_s"], "max_resident_jobs": main_run["max_resident"],
                   "arena_bytes": arena, "rate_sweep": sweep},
    }
    print(json.dumps(out), flush=True)


def calibrate_copy(mib):
    """A plain device copy of known size: each launch reads and writes
    mib MiB, the reference for scaling the HBM byte counters."""
    import torch
    n = mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"bench: copied {mib} MiB 5 times")


def workloads_bytes(d):
    """Compulsory bytes of one generation of replicate d at its initial census."""
    return d["n0"] * d["n_loci"] * bytes_per_update(d["n_loci"])


if __name__ == "__main__":
    main()

"""GPU parity: the HIP library against the oracle, bit for bit.

Every case starts both sides from the same seeded input (the INIT stream or
genomes from the shared input generator), advances them independently and
compares genomes, phenotypes, survivor lists, parents and the census after
every generation.  Tolerance: none (all decisions are integer comparisons).
"""
import numpy as np
import pytest

import oracle
from conftest import read_kat
from gpu_helpers import assert_same_state, lockstep, oracle_pop, say
from paper_1603_09255_amd import spegg, workloads

pytestmark = pytest.mark.gpu


def test_device_philox_known_answers():
    for ctr, key, expect in read_kat():
        say("philox KAT", ctr, key)
        out = spegg.philox_fill(key[0] | (key[1] << 32), np.array([ctr], np.uint32))
        assert [int(x) for x in out[0]] == expect


def test_device_philox_matches_oracle_on_counter_grid():
    g = np.random.default_rng(3)
    ctr = g.integers(0, 1 << 32, (4096, 4), dtype=np.uint64).astype(np.uint32)
    seed = 0x1234_5678_9ABC_DEF0
    say("philox grid", ctr.shape)
    dev = spegg.philox_fill(seed, ctr)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for i in range(0, 4096, 37):
        assert np.array_equal(dev[i], oracle.philox4x32_10(ctr[i], key))


def test_philox_rate_probe_folds_the_oracle_blocks():
    import torch
    seed, m, n = 0xDEAD_BEEF_0123_4567, 5, 3000
    key = [seed & 0xFFFFFFFF, seed >> 32]
    say("philox rate probe", m, n)
    out = torch.zeros(n, dtype=torch.int32, device="cuda")
    spegg.philox_rate(seed, m, out)
    got = out.cpu().numpy().view(np.uint32)
    for i in list(range(0, n, 97)) + [n - 1]:
        acc = 0
        for k in range(m):
            w = oracle.philox4x32_10(np.array([i, k, 0, 0], np.uint32), key)
            acc ^= int(w[0]) ^ int(w[1]) ^ int(w[2]) ^ int(w[3])
        assert int(got[i]) == acc, i
    spegg.philox_rate(seed, 0, out)  # no blocks: the fold of nothing
    assert not out.any().item()


@pytest.mark.parametrize("L,n0", [(1, 7), (31, 50), (32, 64), (33, 65), (64, 1000), (100, 257), (1024, 300),
                                  (4000, 40)])
def test_initial_population_matches_oracle(L, n0):
    say("init", L, n0)
    d = dict(seed=5, replicate_id=3, regime=0, n0=n0, capacity=n0 + 5, n_loci=L, mu=0.0, r=0.5, omega=0.0)
    pop = spegg.Population([d])
    orc = oracle_pop(d)
    assert_same_state(pop, 0, orc, "init")


def test_plain_small_100_generations_bit_exact():
    desc, gens = workloads.plain_small(seed=1)
    say("plain small", desc, gens)
    st = lockstep(desc, gens, trace=True, check_every=10)
    assert st["generation"] == 100 and st["n"] == 1000


CASES = [
    # id, descriptor overrides, generations
    ("wf-raw-L64", dict(regime=0, n_loci=64, r=0.5, mu=1e-3, omega=4.0), 3),
    ("wf-zero-L100", dict(regime=0, n_loci=100, r=0.0, mu=0.01, omega=6.0), 3),
    ("wf-skip-L1024", dict(regime=0, n_loci=1024, r=0.01, mu=1e-3, omega=20.0), 3),
    ("wf-skip-L257", dict(regime=0, n_loci=257, r=0.09, mu=0.02, omega=9.0), 3),
    ("wf-lazy-L200", dict(regime=0, n_loci=200, r=0.3, mu=1e-2, omega=8.0), 3),
    ("wf-lazy-boundary-r", dict(regime=0, n_loci=96, r=0.10, mu=0.0, omega=0.0), 2),
    ("wf-lazy-L2048", dict(regime=0, n_loci=2048, r=0.45, mu=1e-4, omega=30.0), 2),
    ("wf-L1", dict(regime=0, n_loci=1, r=0.01, mu=0.1, omega=0.5), 3),
    # the gap table's edges: one threshold (L = 2), and r just below the bit-serial cut, where gaps of 0 and
    # gaps past the table's end are both common
    ("wf-skip-L2", dict(regime=0, n_loci=2, r=0.08, mu=0.05, omega=1.0), 3),
    ("wf-skip-L33-r0095", dict(regime=0, n_loci=33, r=0.095, mu=0.01, omega=3.0), 3),
    ("wf-L31-high-mu", dict(regime=0, n_loci=31, r=0.5, mu=0.4, omega=3.0), 3),
    ("wf-effects", dict(regime=0, n_loci=300, r=0.05, mu=1e-3, omega=15.0, effects="grid"), 3),
    ("pois-bh-L1024", dict(regime=1, n_loci=1024, r=0.01, mu=1e-4, omega=64.0, K=800.0, fecundity=2.2,
                           capacity=3000, effects="grid"), 3),
    ("pois-trunc", dict(regime=1, n_loci=64, r=0.25, mu=1e-3, omega=0.0, K=0.0, fecundity=4.0, capacity=700), 3),
    ("pois-no-K", dict(regime=1, n_loci=40, r=0.5, mu=0.0, omega=5.0, K=0.0, fecundity=1.5, capacity=5000), 4),
    ("extinction", dict(regime=0, n_loci=64, r=0.5, mu=0.0, omega=0.3, theta=500.0), 3),
    ("n-one", dict(regime=0, n_loci=70, r=0.2, mu=0.05, omega=0.0, n0=1, capacity=1), 3),
    # kernel shapes: 8-byte lanes (L=256), chunked genomes (L=8192, 16384), odd word count (L=4000)
    ("wf-lazy-L256", dict(regime=0, n_loci=256, r=0.2, mu=1e-3, omega=10.0), 3),
    ("wf-skip-L8192-chunks", dict(regime=0, n_loci=8192, r=0.002, mu=1e-4, omega=60.0, n0=120), 2),
    ("wf-raw-L4000-odd-words", dict(regime=0, n_loci=4000, r=0.5, mu=1e-4, omega=50.0, n0=80), 2),
    ("pois-lazy-L16384", dict(regime=1, n_loci=16384, r=0.3, mu=1e-5, omega=0.0, K=60.0, fecundity=2.0,
                              n0=40, capacity=120), 2),
    # the largest LDS footprint: the longest genome in skip mode (gap table of L - 1 thresholds) with effect
    # planes
    ("wf-skip-L16384-max", dict(regime=0, n_loci=16384, r=0.001, mu=1e-5, omega=90.0, effects="grid", n0=48,
                                capacity=64), 2),
]


@pytest.mark.parametrize("name,over,gens", CASES, ids=[c[0] for c in CASES])
def test_lockstep_from_generator_genomes(name, over, gens):
    over = dict(over)
    L = over["n_loci"]
    n0 = over.pop("n0", 600)
    cap = over.pop("capacity", n0)
    if over.get("effects") == "grid":
        over["effects"] = np.random.default_rng(L).integers(-4, 5, L).astype(np.int8)
    desc = dict(seed=77, replicate_id=5, n0=n0, capacity=cap, theta=0.0, K=0.0, fecundity=0.0)
    desc.update(over)
    words = workloads.random_genomes(n0, L, seed=L + n0, p_one=0.4)
    say("lockstep", name, "L", L, "n0", n0, "cap", cap)
    lockstep(desc, gens, start_words=words, start_gen=37, trace=True)


def test_batch_equals_each_replicate_alone_and_oracle():
    g = np.random.default_rng(11)
    reps = []
    for i, (L, regime, r) in enumerate([(64, 0, 0.5), (1024, 0, 0.01), (256, 1, 0.3), (33, 0, 0.0),
                                        (700, 1, 0.12), (64, 0, 0.2)]):
        n0 = int(g.integers(50, 400))
        reps.append(dict(seed=9, replicate_id=100 + i, regime=regime, n0=n0, capacity=3 * n0, n_loci=L, r=r,
                         mu=1e-3, theta=0.0, omega=float(g.uniform(3, 20)), K=float(n0), fecundity=2.0))
    say("batch of", len(reps))
    batch = spegg.Population(reps)
    batch.set_trace(True)
    batch.step(4)
    for i, d in enumerate(reps):
        alone = spegg.Population([d])
        alone.set_trace(True)
        alone.step(4)
        assert batch.stats()[i] == alone.stats()[0]
        assert np.array_equal(batch.genomes(i), alone.genomes(0))
        orc = oracle_pop(d)
        orc.step(4)
        assert_same_state(batch, i, orc, f"batch replicate {i}", parents=True)
        alone.close()


def test_batched_table_full_size_sampled_replicates():
    # the batched workload at its full size (4096 Wright-Fisher replicates,
    # N ~ U{500..50000}, L in {64, 256, 1024}, r ~ U[0.001, 0.5]) in the
    # launch configuration the bench times (graph replay, the lanes-per-gamete
    # caps its autotuner picks); for every genome length and crossover mode
    # the first and the largest replicate against the oracle
    reps = workloads.batched_table(n_reps=4096)
    say("batched table", len(reps))
    pop = spegg.Population(reps)
    for W, g in ((2, 1), (8, 1), (32, 4)):
        pop.set_offspring_cap(W, g)
    pop.step(2)
    stats = pop.stats()
    groups = {}
    for i, d in enumerate(reps):
        groups.setdefault((d["n_loci"], oracle.recomb_mode(d["r"])), []).append(i)
    assert len(groups) >= 6  # three lengths, geometric and bit-serial crossovers
    for key in sorted(groups):
        idx = groups[key]
        for i in sorted({idx[0], max(idx, key=lambda k: reps[k]["n0"])}):
            say("batched replicate", i, "L", reps[i]["n_loci"], "mode", key[1], "N", reps[i]["n0"])
            orc = oracle_pop(reps[i])
            orc.step(2)
            assert_same_state(pop, i, orc, f"batched replicate {i}")
            orc.close()
    # every replicate: generation 2, and a Wright-Fisher census unchanged
    # unless the replicate died out
    for k, st in enumerate(stats):
        assert st["generation"] == 2
        assert st["n"] == (0 if st["extinct"] else reps[k]["n0"])
    pop.close()


def test_offspring_grid_changes_no_result(monkeypatch):
    # a grid of 64 blocks: every block loops over many tiles, in a one-deme
    # class and in a class of several demes
    one = [dict(seed=4, replicate_id=60, n0=5000, capacity=6000, n_loci=256, r=0.05, mu=1e-3, omega=12.0)]
    many = [dict(seed=4, replicate_id=61 + i, n0=900 + 300 * i, capacity=2000, n_loci=256, r=r, mu=1e-3,
                 omega=10.0) for i, r in enumerate((0.05, 0.3, 0.5))]
    for reps in (one, many):
        say("grid 64 against the default", len(reps))
        default = spegg.Population(reps)
        monkeypatch.setenv("SPEGG_OFFSPRING_GRID", "64")
        small = spegg.Population(reps)
        monkeypatch.delenv("SPEGG_OFFSPRING_GRID")
        default.step(3)
        small.step(3)
        for i in range(len(reps)):
            assert default.stats()[i] == small.stats()[i]
            assert np.array_equal(default.genomes(i), small.genomes(i))
        orc = oracle_pop(reps[-1])
        orc.step(3)
        assert_same_state(small, len(reps) - 1, orc, "grid 64")
        orc.close()
        default.close()
        small.close()


def test_plain_scale_first_generations_full_size():
    desc, _ = workloads.plain_scale(seed=1)
    say("plain scale full size, 2 generations")
    gpu = spegg.Population([desc])
    gpu.set_trace(True)
    orc = oracle_pop(desc)
    assert_same_state(gpu, 0, orc, "init")
    for _ in range(2):
        gpu.step(1)
        orc.step(1)
        assert_same_state(gpu, 0, orc, f"generation {orc.generation}", parents=True)


def test_write_read_errors_and_roundtrip():
    d = dict(seed=1, n0=10, capacity=20, n_loci=40, r=0.5, omega=0.0)
    pop = spegg.Population([d])
    w = workloads.random_genomes(15, 40, seed=2)
    pop.write_genomes(0, w, 9)
    assert np.array_equal(pop.genomes(0), w)
    assert pop.stats()[0]["generation"] == 9
    bad = w.copy()
    bad[3, 1, 1] |= 1 << 20  # locus 52 >= L
    with pytest.raises(spegg.SpeggError) as ei:
        pop.write_genomes(0, bad, 9)
    assert ei.value.status == spegg.E_INVALID
    with pytest.raises(spegg.SpeggError):
        pop.write_genomes(0, workloads.random_genomes(21, 40, seed=3), 0)
    with pytest.raises(spegg.SpeggError) as ei:
        pop.parents(0)
    assert ei.value.status == spegg.E_STATE
    import ctypes as C
    got = C.c_uint32()
    small = np.zeros(4, np.uint32)
    st = pop.lib.spegg_read_genomes(pop._h, 0, 0, 0, small.ctypes.data_as(C.POINTER(C.c_uint32)), 4, C.byref(got))
    assert st == spegg.E_INVALID and got.value == 15


def test_kernel_timing_counts_launches():
    desc, _ = workloads.plain_small(seed=2)
    pop = spegg.Population([desc])
    pop.set_timing()
    pop.step(5)
    t = pop.kernel_times()
    one_species = ("survive", "compact", "offspring")
    assert all(t[k][1] == 5 and t[k][0] > 0 for k in one_species)
    assert t["encounter"][1] == 0 and t["carry"][1] == 0  # consumer-resource kernels only
    eco = dict(workloads.CR_ECOLOGY, n0_consumer=50, capacity_consumer=200, habitat=0)
    cr = spegg.Population([dict(seed=3, regime=2, n0=300, capacity=900, n_loci=64, ecology=eco)])
    cr.set_timing()
    cr.step(4)
    # the survivors are carried inside compact: no carry launch of its own
    assert all(v[1] == (0 if k == "carry" else 4) for k, v in cr.kernel_times().items())
    cr.close()
    pop.set_timing(["offspring"])
    pop.step(3)
    t = pop.kernel_times()
    assert t["offspring"][1] == 3 and t["survive"][1] == 0
    pop.set_timing([])
    pop.step(2)
    assert all(v[1] == 0 for v in pop.kernel_times().values())


@pytest.mark.parametrize("desc_name", ["small", "poisson"])
def test_graph_replay_equals_eager_and_oracle(desc_name):
    """Generations replayed as captured graphs (16- and 1-generation graphs,
    many replays, with host reads and synchronisations in between) give the
    same state as eager launches and as the oracle, after every chunk."""
    if desc_name == "small":
        desc, _ = workloads.plain_small(seed=3)
    else:
        desc = dict(seed=4, replicate_id=2, regime=1, n0=800, capacity=2500, n_loci=300, mu=1e-3, r=0.05,
                    theta=0.0, omega=12.0, K=900.0, fecundity=2.2,
                    effects=np.random.default_rng(9).integers(-4, 5, 300).astype(np.int8))
    say("graph vs eager", desc_name)
    g = spegg.Population([desc])
    e = spegg.Population([desc])
    e.set_graph(False)
    orc = oracle_pop(desc)
    for chunk in (1, 16, 3, 17, 1, 33):
        g.step(chunk)
        e.step(chunk)
        orc.step(chunk)
        assert g.stats() == e.stats()
        assert np.array_equal(g.genomes(0), e.genomes(0))
        assert_same_state(g, 0, orc, f"after chunk {chunk}")
    g.set_trace(True)  # a new trace setting recaptures the graphs
    e.set_trace(True)
    g.step(2)
    e.step(2)
    orc.step(2)
    assert_same_state(g, 0, orc, "traced", parents=True)
    assert np.array_equal(g.parents(0)[0], e.parents(0)[0])


@pytest.mark.parametrize("L,n0", [(1, 10), (70, 300), (1024, 2000)])
def test_allele_counts_match_oracle(L, n0):
    desc = dict(seed=12, replicate_id=1, regime=0, n0=n0, capacity=n0, n_loci=L, mu=1e-3, r=0.2, theta=0.0,
                omega=0.0)
    say("allele counts", L, n0)
    pop = spegg.Population([desc])
    orc = oracle_pop(desc)
    pop.step(3)
    orc.step(3)
    got = pop.allele_counts(0)
    expect = orc.alleles().astype(np.int64).sum(axis=(0, 1))
    assert np.array_equal(got.astype(np.int64), expect)
    assert got.max() <= 2 * n0


def test_autotune_changes_no_result():
    # mixed genome lengths: each W gets its own shape; the tuned run must end
    # where the untuned one (and the oracle) ends
    reps = [dict(seed=3, replicate_id=40 + i, n0=300, capacity=300, n_loci=L, r=r, mu=1e-3, omega=8.0)
            for i, (L, r) in enumerate([(1024, 0.01), (256, 0.3), (64, 0.5), (100, 0.05)])]
    tuned = spegg.Population(reps)
    chosen = tuned.autotune(generations_per_trial=2)
    assert sorted(chosen) == [2, 4, 8, 32]
    done = tuned.stats()[0]["generation"]
    assert done >= 2 * len(chosen)
    tuned.step(1)
    # a pinned shape: no timing, no result changes
    for W, g in ((32, 1), (8, 32), (2, 2)):
        tuned.set_offspring_cap(W, g)
    for bad_W, bad_g in ((32, 3), (32, 0), (32, 64), (5, 4)):
        with pytest.raises(spegg.SpeggError) as ei:
            tuned.set_offspring_cap(bad_W, bad_g)
        assert ei.value.status == spegg.E_INVALID
    tuned.step(2)
    plain = spegg.Population(reps)
    plain.step(done + 3)
    for i, d in enumerate(reps):
        assert tuned.stats()[i] == plain.stats()[i]
        assert np.array_equal(tuned.genomes(i), plain.genomes(i))
        orc = oracle_pop(d)
        orc.step(done + 3)
        assert_same_state(tuned, i, orc, f"tuned replicate {i}")

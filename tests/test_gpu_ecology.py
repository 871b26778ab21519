"""GPU parity of the two-species consumer-resource regime: the HIP library
against the oracle, bit for bit, per species -- genomes, phenotypes, ages,
survivors, intake, parents and the census -- after every generation."""
import numpy as np
import pytest

from gpu_helpers import assert_same_state, oracle_pop, say
from paper_1603_09255_amd import spegg, workloads

pytestmark = pytest.mark.gpu


def cr(**kw):
    eco = dict(workloads.CR_ECOLOGY, n0_consumer=60, capacity_consumer=400, habitat=0, encounters=6.0)
    eco.update(kw.pop("eco", {}))
    d = dict(seed=4, replicate_id=2, regime=2, n0=500, capacity=1500, n_loci=64, mu=1e-3, r=0.5, omega=0.0,
             ecology=eco)
    d.update(kw)
    return d


CASES = [
    ("base", cr(), 8),
    ("habitat_lazy", cr(n_loci=100, r=0.3, eco=dict(habitat=800, encounters=15.0)), 8),
    ("crowded_captures", cr(n0=40, capacity=200, eco=dict(n0_consumer=300, capacity_consumer=600, attack=1.0,
                                                          match_width=50.0, encounters=10.0)), 6),
    ("capacity_truncation", cr(n0=1000, capacity=1000, eco=dict(resource_q0=1.0, resource_K=1e9)), 5),
    ("viability_and_skip", cr(n_loci=256, r=0.02, omega=6.0, eco=dict(surv_consumer=(1.0, 0.9, 0.5, 0.2))), 6),
    ("consumers_starve", cr(eco=dict(attack=0.0)), 8),
    ("no_consumers", cr(eco=dict(n0_consumer=0)), 4),
]


@pytest.mark.parametrize("name,desc,gens", CASES, ids=[c[0] for c in CASES])
def test_consumer_resource_lockstep(name, desc, gens):
    say("consumer-resource lockstep", name)
    gpu = spegg.Population([desc])
    gpu.set_trace(True)
    orc = oracle_pop(desc)
    assert_same_state(gpu, 0, orc, f"{name} start")
    for _ in range(gens):
        gpu.step(1)
        orc.step(1)
        assert_same_state(gpu, 0, orc, f"{name} generation {orc.generation}", parents=True)
    gpu.close()
    orc.close()


def test_written_genomes_and_graph_replay():
    d = cr(seed=6)
    gpu = spegg.Population([d])
    orc = oracle_pop(d)
    for sp, n in ((0, 300), (1, 80)):
        w = workloads.random_genomes(n, 64, seed=10 + sp, p_one=0.4)
        gpu.write_genomes(0, w, 11, species=sp)
        orc.set_genomes(w, 11, species=sp)
    gpu.step(16)  # one replay of the long graph
    orc.step(16)
    assert_same_state(gpu, 0, orc, "after 16 generations")
    gpu.step(3)
    orc.step(3)
    assert_same_state(gpu, 0, orc, "after 19 generations")


def test_mixed_batch_equals_oracle():
    reps = [cr(replicate_id=20), dict(seed=9, replicate_id=21, n0=300, capacity=300, n_loci=64, r=0.5, omega=6.0),
            cr(replicate_id=22, n_loci=40, r=0.0), dict(seed=9, replicate_id=23, n0=150, capacity=150, n_loci=64,
                                                         n_patches=3, migration=0.1, omega=5.0)]
    batch = spegg.Population(reps)
    batch.set_trace(True)
    batch.step(5)
    for i, d in enumerate(reps):
        orc = oracle_pop(d)
        orc.step(5)
        assert_same_state(batch, i, orc, f"batch replicate {i}", parents=True)


def test_consumer_resource_full_size_two_generations():
    reps, _ = workloads.consumer_resource(n_reps=1)
    say("consumer-resource full size: 1e5 resources, 1e4 consumers, L = 256")
    gpu = spegg.Population(reps)
    gpu.set_trace(True)
    orc = oracle_pop(reps[0])
    for _ in range(2):
        gpu.step(1)
        orc.step(1)
        assert_same_state(gpu, 0, orc, f"full size generation {orc.generation}", parents=True)

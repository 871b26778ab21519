"""Seeded synthetic workloads shaped like the paper's case studies.

This module only generates inputs (parameter sets, allelic effects, random
genomes) from fixed seeds; it holds none of the model's arithmetic.  The
same dicts feed the HIP library's descriptors and the oracle's parameters
(identical key names).

The paper's own runs use about 50,000 individuals per patch, up to 100
patches and 250 iterations (main text, Fig. 2 caption); their parameter
values are not part of the paper.  The configurations below are synthetic
stand-ins of that shape.
"""
import numpy as np

WF, POISSON_BH = 0, 1


def plain_small(seed=1):
    """Wright-Fisher, N = 1000 diploids, L = 64 loci (two 32-bit words),
    unit additive effects, Gaussian stabilising selection (optimum 0,
    width 8), free recombination, mu = 1e-5 per locus; 100 generations."""
    return dict(seed=seed, replicate_id=0, regime=WF, n0=1000, capacity=1000, n_loci=64, mu=1e-5, r=0.5,
                theta=0.0, omega=8.0, K=0.0, fecundity=0.0, effects=None), 100


def plain_scale_effects(L=1024, seed=20260102):
    """Allelic effects on the integer grid [-4, 4], drawn once."""
    return np.random.default_rng(seed).integers(-4, 5, size=L).astype(np.int8)


def plain_scale(seed=1):
    """One replicate at scale: N0 = 100000 (capacity 250000), L = 1024 loci,
    effects on the integer grid [-4, 4], adjacent-locus crossover r = 0.01,
    mu = 1e-6, Poisson(2.2) fecundity with Beverton-Holt density-dependent
    survival (K = 100000), stabilising selection of width 64; 1000
    generations."""
    return dict(seed=seed, replicate_id=0, regime=POISSON_BH, n0=100_000, capacity=250_000, n_loci=1024,
                mu=1e-6, r=0.01, theta=0.0, omega=64.0, K=100_000.0, fecundity=2.2,
                effects=plain_scale_effects()), 1000


CONTINUOUS = 1


def continuous_scale(seed=1):
    """The paper's own genetics (Supplementary S2, "Genetics") at scale: one
    Wright-Fisher replicate of N = 100000 diploids with L = 256 loci of
    continuous allelic values (float32), initial values N(0.01, 0.01^2),
    free recombination (S2: all loci freely recombining), mutation with
    probability 1e-3 per locus to N(value, (0.5 x 0.01)^2), residual
    phenotypic noise 0.2, Gaussian stabilising selection of the phenotype
    (optimum 2.6, width 1); 100 generations."""
    return dict(seed=seed, replicate_id=0, regime=WF, n0=100_000, capacity=100_000, n_loci=256, mu=1e-3, r=0.5,
                theta=2.6, omega=1.0, K=0.0, fecundity=0.0, effects=None, genetics=CONTINUOUS, allele_mean=0.01,
                allele_sd=0.01, mut_sd_factor=0.5, noise_sd=0.2, exp_transform=0), 100


PHYSIOLOGY = 3

# Synthetic parameters of the physiologically structured consumer
# (Supplementary S2 gives the model but not its values): intake 0.3 W^0.75,
# metabolism 0.1 W, Holling scarcity with attack 2 and handling 1, the diet
# switching from resource 2 to resource 1 at W = 1 (w_max 8, u 1/2,
# steepness 5), reserves 0.2 X at birth and gonads above 0.4 X, maturity at
# X = 1, survival 1/(1 + exp(-20 (X - 0.05))) times 1 - exp(-20 Y/X),
# recruitment 0.5 F / (1 + F/kappa2), breeding every 5 steps; a population
# of n0 = 50000 settles near 4e4 with the adults' resource drawn down.
PHYSIOLOGY_PARAMS = dict(alpha=0.3, gamma=0.75, delta=0.1, attack=2.0, handling=1.0, K=[75000.0, 75000.0],
                         growth=[2.0, 2.0], growth_sd=[0.1, 0.1], R0=[75000.0, 75000.0], steepness=5.0,
                         switch_frac=0.5, w_max=8.0, kappa=1.0, qJ=0.2, qA=0.4, beta1=0.05, beta2=20.0, beta_s=20.0,
                         maturity=1.0, v_f=1.0, v_m=1.0, kappa1=0.5, kappa2=25000.0, kappa3=1.0, breed_every=5)


def physiology_batch(n_reps=100, seed=1, L=16):
    """The physiologically structured consumer of Supplementary S2 at the
    paper's scale (about 50000 individuals per patch, up to 100 patches,
    250 iterations): n_reps independent replicates of n0 = 50000 founders
    (capacity 200000), neonate mass exp(z) from L = 16 continuous loci
    (initial values N(-2.3/L, 0.02^2), so Omega near 0.1), mutation 1e-3 per
    locus to N(value, (0.2 x 2.3/L)^2), phenotypic noise 0.05, free
    recombination; 250 time steps."""
    return [dict(seed=seed, replicate_id=i, regime=PHYSIOLOGY, n0=50_000, capacity=200_000, n_loci=L, mu=1e-3,
                 r=0.5, theta=0.0, omega=0.0, K=0.0, fecundity=0.0, effects=None, genetics=CONTINUOUS,
                 allele_mean=-2.3 / L, allele_sd=0.02, mut_sd_factor=0.2, noise_sd=0.05, exp_transform=1,
                 physiology=dict(PHYSIOLOGY_PARAMS)) for i in range(n_reps)], 250


def batched_table(n_reps=4096, seed=20260101, philox_seed=1):
    """Per-replicate parameters of the batched form: N ~ U{500..50000},
    L from {64, 256, 1024}, mu log-uniform in [1e-7, 1e-4], r ~ U[0.001, 0.5],
    selection width ~ U[2, 16]; Wright-Fisher, unit effects."""
    g = np.random.default_rng(seed)
    N = g.integers(500, 50_001, n_reps)
    L = g.choice([64, 256, 1024], n_reps)
    mu = 10.0 ** g.uniform(-7.0, -4.0, n_reps)
    r = g.uniform(0.001, 0.5, n_reps)
    omega = g.uniform(2.0, 16.0, n_reps)
    return [dict(seed=philox_seed, replicate_id=i, regime=WF, n0=int(N[i]), capacity=int(N[i]), n_loci=int(L[i]),
                 mu=float(mu[i]), r=float(r[i]), theta=0.0, omega=float(omega[i]), K=0.0, fecundity=0.0,
                 effects=None) for i in range(n_reps)]


def random_genomes(n, L, seed, p_one=0.5):
    """n packed diploid genomes (n, 2, ceil(L/32)) uint32 with locus l at
    bit l % 32 of word l // 32, allele 1 with probability p_one, tail zero."""
    g = np.random.default_rng(seed)
    W = (L + 31) // 32
    bits = (g.random((n, 2, W * 32)) < p_one).astype(np.uint8)
    bits[:, :, L:] = 0
    return np.packbits(bits, axis=-1, bitorder="little").view(np.uint32).reshape(n, 2, W).copy()


def serve_trace(n_jobs=200, rate=20.0, seed=7, philox_seed=1, reps=(8, 256), gens=(100, 2000),
                patch_n=(200, 5000), n_patches=100, n_loci=256, migration=0.01):
    """Sweep jobs of the served form, arriving as a Poisson process of the
    given rate (jobs/s): each job is one parameter combination -- its own
    per-patch census N ~ U{patch_n}, mu log-uniform in [1e-7, 1e-4],
    r ~ U[0.001, 0.5], selection width ~ U[2, 16] -- run as U{reps}
    replicates of a ring of n_patches Wright-Fisher patches (L loci, unit
    effects, backward migration rate m) for U{gens} generations.

    Returns [(arrival_s, job_id, [descs], generations)] in arrival order.
    Replicate ids are unique over the trace, so no two replicates share a
    random stream."""
    g = np.random.default_rng(seed)
    arrivals = np.cumsum(g.exponential(1.0 / rate, n_jobs))
    jobs, rid = [], 0
    for k in range(n_jobs):
        R = int(g.integers(reps[0], reps[1] + 1))
        G = int(g.integers(gens[0], gens[1] + 1))
        N = int(g.integers(patch_n[0], patch_n[1] + 1))
        mu = float(10.0 ** g.uniform(-7.0, -4.0))
        r = float(g.uniform(0.001, 0.5))
        omega = float(g.uniform(2.0, 16.0))
        descs = [dict(seed=philox_seed, replicate_id=rid + i, regime=WF, n0=N, capacity=N, n_loci=n_loci, mu=mu,
                      r=r, theta=0.0, omega=omega, K=0.0, fecundity=0.0, effects=None, n_patches=n_patches,
                      migration=migration) for i in range(R)]
        rid += R
        jobs.append((float(arrivals[k]), k, descs, G))
    return jobs


CONSUMER_RESOURCE = 2

# Constants of the consumer-resource form (the paper gives none): chosen so
# that both species persist near R ~ 1.3e5, C ~ 1.2e4 with moderate
# fluctuations (resource logistic growth, mass-action encounters).
CR_ECOLOGY = dict(n0_consumer=10_000, capacity_consumer=50_000, resource_trials=4, habitat=200_000, attack=0.5,
                  match_width=4.0, encounters=20.0, conversion=0.5, resource_q0=0.55, resource_K=250_000.0,
                  surv_resource=(0.5, 0.8, 0.8, 0.0), surv_consumer=(0.6, 0.8, 0.8, 0.0))


def consumer_resource(n_reps=64, seed=1, n_resource=100_000, scale=1.0):
    """Two coevolving species: resource N0 = 1e5 (capacity 2.5e5), consumer
    N0 = 1e4 (capacity 5e4), each with L = 256 loci of unit effect, free of
    viability selection (trait-mediated fitness is the capture of resources
    by Gaussian phenotype matching, width 4), ages 0-3 with age-specific
    survival, mu = 1e-5, r = 0.1; 64 replicates, 500 generations.  `scale`
    shrinks every census, capacity and the habitat together."""
    eco = dict(CR_ECOLOGY)
    for k in ("n0_consumer", "capacity_consumer", "habitat"):
        eco[k] = max(1, int(eco[k] * scale))
    eco["resource_K"] = CR_ECOLOGY["resource_K"] * scale
    n0 = max(1, int(n_resource * scale))
    cap = max(n0, int(250_000 * scale))
    return [dict(seed=seed, replicate_id=i, regime=CONSUMER_RESOURCE, n0=n0, capacity=cap, n_loci=256, mu=1e-5,
                 r=0.1, theta=0.0, omega=0.0, K=0.0, fecundity=0.0, effects=None, ecology=eco)
            for i in range(n_reps)], 500

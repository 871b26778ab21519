/* Sanitizer driver of the oracle (built with -fsanitize=address,undefined
 * by tests/test_sanitizers.py): a few generations of every regime and
 * edge of the model, and the table builders. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct oracle_pop oracle_pop;
typedef struct {
    uint32_t n0_consumer, capacity_consumer, resource_trials, habitat;
    double attack, match_width, encounters, conversion, resource_q0, resource_K;
    double surv_resource[4], surv_consumer[4];
} oracle_ecology;
typedef struct {
    double alpha, gamma, delta, attack, handling;
    double K[2], growth[2], growth_sd[2], R0[2];
    double steepness, switch_frac, w_max, kappa, qJ, qA, beta1, beta2, beta_s, maturity, v_f, v_m;
    double kappa1, kappa2, kappa3;
    uint32_t breed_every;
} oracle_physiology;
typedef struct {
    uint64_t seed;
    uint32_t replicate_id, regime, n0, capacity, n_loci, n_patches;
    double mu, r, theta, omega, K, fecundity, migration;
    uint32_t dispersal;
    double home_return;
    const int8_t *effects;
    const oracle_ecology *ecology;
    uint32_t genetics;
    double allele_mean, allele_sd, mut_sd_factor, noise_sd;
    uint32_t exp_transform;
    const double *linkage;
    uint32_t sexes, mating;
    double pref_optimum, pref_width;
    uint32_t monogamy;
    const oracle_physiology *physiology;
} oracle_params;

oracle_pop *oracle_create(const oracle_params *prm);
void oracle_destroy(oracle_pop *P);
int oracle_step(oracle_pop *P, uint32_t n);
int oracle_get_genomes(const oracle_pop *P, uint32_t deme, uint32_t *words, size_t n_words);
int oracle_set_genomes(oracle_pop *P, uint32_t deme, const uint32_t *words, uint32_t n, uint32_t generation);
uint32_t oracle_get_n(const oracle_pop *P, uint32_t deme);
int oracle_get_alleles(const oracle_pop *P, uint32_t deme, float *out, size_t n_values);
int oracle_set_alleles(oracle_pop *P, uint32_t deme, const float *values, uint32_t n, uint32_t generation);
int oracle_poisson_thresholds(double lambda, uint64_t *T, int cap);
int oracle_binomial_thresholds(uint32_t L, double mu, uint64_t *T, int cap);
void oracle_geometric_thresholds(double r, uint32_t n, uint64_t *T);
int oracle_small_binomial_thresholds(uint32_t n, double q, uint64_t *T);
uint32_t oracle_skip_gap(double r, uint32_t L, uint32_t x);
int oracle_find_gap_word(uint64_t seed, uint32_t c3, double r, uint32_t L, uint32_t n_slots, uint32_t t_begin,
                         uint32_t t_end, uint32_t x_target, uint32_t out[5]);

static void run(oracle_params p, uint32_t gens)
{
    oracle_pop *P;
    static int which = 0;
    ++which;
    P = oracle_create(&p);
    uint32_t W = (p.n_loci + 31u) / 32u, n;
    uint32_t *w;
    if (!P) {
        fprintf(stderr, "create failed: case %d\n", which);
        exit(2);
    }
    oracle_step(P, gens);
    n = oracle_get_n(P, 0);
    if (p.genetics == 1) {
        float *v = (float *)calloc((size_t)(n ? n : 1) * 2u * p.n_loci, sizeof(float));
        oracle_get_alleles(P, 0, v, (size_t)(n ? n : 1) * 2u * p.n_loci);
        oracle_set_alleles(P, 0, v, n, 77);
        oracle_step(P, 1);
        free(v);
        oracle_destroy(P);
        return;
    }
    w = (uint32_t *)calloc((size_t)(n ? n : 1) * 2u * W, sizeof(uint32_t));
    oracle_get_genomes(P, 0, w, (size_t)(n ? n : 1) * 2u * W);
    oracle_set_genomes(P, 0, w, n, 77);
    oracle_step(P, 1);
    free(w);
    oracle_destroy(P);
}

int main(void)
{
    static int8_t eff[300];
    uint64_t T[2048];
    uint32_t out[5], k;
    oracle_ecology eco = {3000, 6000, 4, 30000, 0.5, 4.0, 20.0, 0.5, 0.55, 25000.0,
                          {0.5, 0.8, 0.8, 0.0}, {0.6, 0.8, 0.8, 0.0}};
    oracle_params base = {1, 3, 0, 400, 400, 64, 1, 1e-3, 0.5, 0.0, 8.0, 0.0, 0.0, 0.0, 0, 0.0, NULL, NULL,
                          0, 0.0, 0.0, 0.0, 0.0, 0, NULL, 0, 0, 0.0, 0.0, 0, NULL};
    oracle_physiology phy = {0.3, 0.75, 0.1, 2.0, 1.0, {3000.0, 3000.0}, {2.0, 2.0}, {0.1, 0.1},
                             {3000.0, 3000.0}, 5.0, 0.5, 8.0, 1.0, 0.2, 0.4, 0.05, 20.0, 20.0, 1.0, 1.0, 1.0,
                             0.5, 1000.0, 1.0, 2};
    oracle_params p;
    for (k = 0; k < 300; ++k)
        eff[k] = (int8_t)((int)(k * 7u % 9u) - 4);
    p = base; run(p, 3);                                    /* raw bits */
    p = base; p.r = 0.0; run(p, 2);                         /* no crossover */
    p = base; p.n_loci = 1024; p.r = 0.1; run(p, 2);        /* geometric gaps reaching the table's 2^32 entry */
    p = base; p.n_loci = 257; p.r = 0.3; p.mu = 0.05; run(p, 2); /* bit-serial, tail bits, mutations */
    p = base; p.n_loci = 1; p.r = 0.01; run(p, 2);
    p = base; p.n_loci = 300; p.effects = eff; p.r = 0.05; run(p, 2);
    p = base; p.regime = 1; p.capacity = 900; p.K = 400.0; p.fecundity = 2.2; run(p, 3);
    p = base; p.regime = 1; p.n0 = 300; p.capacity = 300; p.fecundity = 4.0; run(p, 3); /* truncation */
    p = base; p.omega = 0.3; p.theta = 500.0; run(p, 2);    /* extinction */
    p = base; p.n0 = 1; p.capacity = 1; run(p, 2);
    p = base; p.n_patches = 5; p.migration = 0.2; p.n0 = 100; p.capacity = 100; run(p, 3);
    p = base; p.n_patches = 7; p.migration = 0.3; p.dispersal = 1; p.home_return = 0.4; p.n0 = 80; p.capacity = 80;
    run(p, 3);
    p = base; p.regime = 2; p.n0 = 8000; p.capacity = 20000; p.n_loci = 96; p.r = 0.2; p.omega = 0.0;
    p.ecology = &eco; run(p, 3);
    /* linkage map; separate sexes with preference, assortative, monogamy */
    {
        static double map[255];
        for (k = 0; k < 255; ++k)
            map[k] = (k % 5) * 0.1;
        p = base; p.n_loci = 256; p.linkage = map; run(p, 3);
    }
    p = base; p.sexes = 1; p.mating = 1; p.pref_optimum = 2.0; p.pref_width = 3.0; run(p, 3);
    p = base; p.sexes = 1; p.mating = 2; p.pref_width = 2.0; p.regime = 1; p.capacity = 900; p.K = 400.0;
    p.fecundity = 2.2; run(p, 3);
    p = base; p.monogamy = 1; p.mating = 2; p.pref_width = 0.5; run(p, 3);
    p = base; p.sexes = 1; p.n0 = 2; p.capacity = 2; run(p, 4); /* one sex dies out */
    /* physiologically structured consumer */
    p = base; p.regime = 3; p.genetics = 1; p.exp_transform = 1; p.allele_mean = -0.15; p.allele_sd = 0.02;
    p.noise_sd = 0.05; p.n_loci = 16; p.capacity = 4000; p.physiology = &phy; run(p, 12);
    /* continuous alleles: Gaussian mutation, noise, exp transform */
    p = base; p.genetics = 1; p.allele_mean = 0.01; p.allele_sd = 0.005; p.mut_sd_factor = 0.5; p.noise_sd = 0.1;
    p.mu = 0.02; p.r = 0.05; p.n_loci = 70; p.omega = 2.0; p.theta = 1.0; p.exp_transform = 1; run(p, 3);
    p = base; p.genetics = 1; p.allele_mean = 1.0; p.allele_sd = 0.1; p.mut_sd_factor = 0.1; p.r = 0.3; p.regime = 1;
    p.capacity = 900; p.K = 400.0; p.fecundity = 2.2; p.omega = 0.0; run(p, 3);
    oracle_poisson_thresholds(2.2, T, 1024);
    oracle_poisson_thresholds(700.0, T, 1024);
    oracle_binomial_thresholds(1024, 1e-4, T, 1025);
    oracle_binomial_thresholds(5, 0.9, T, 6);
    oracle_geometric_thresholds(0.169, 1023, T);
    oracle_small_binomial_thresholds(64, 0.3, T);
    if (oracle_skip_gap(0.1, 1024, 0xFFFFFFFFu) != 427u)
        return 3;
    oracle_find_gap_word(7, 0, 0.1, 1024, 8, 0, 2, 0xFFFFFFFFu, out);
    puts("oracle sanitizer driver ok");
    return 0;
}

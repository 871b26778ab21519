/*
 * spegg_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU oracle for the per-generation update
 * of sPEGG's individual-based model (Okamoto & Amarasekare, "sPEGG: high
 * throughput eco-evolutionary simulations on commodity graphics
 * processors"): main text, Fig. 1 steps A-F; Supplementary Information S2,
 * "Genetics"; Supplementary Fig. S5(A), the serial loop over replicates and
 * individuals.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this file's library.  It shares no source with the GPU
 * library: its own Philox, its own threshold tables, its own genome
 * representation (one byte per allele, not packed words).  Conversions to
 * the packed layout exist only so that results can be compared.
 *
 * The genetics follow the biallelic reading of the paper's additive model:
 * allele value A = e_l * (2b - 1) at locus l with b in {0,1}, so the paper's
 * midpoint sum over loci of (A_f + A_m)/2 (eqn. S2 phenotype value, noise
 * variance zero) is exactly the integer z = sum_l e_l (b_f + b_m - 1).
 *
 * Every random decision is an integer comparison of a Philox4x32-10 word
 * (Salmon, Moraes, Dror & Shaw, SC'11) against a threshold; probabilities
 * are computed in IEEE double (basic operations plus glibc exp) and
 * distribution tables in x87 extended precision, each from its definition.
 *
 * Pins: see tests/test_oracle_*.py.  Every function below is pinned there
 * against a published value, a closed form, an exact enumeration or a
 * population-genetic law; none is "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_ALWAYS 4294967296ULL /* threshold that every 32-bit word is below */
#define TWO32 4294967296.0
#define TWO32L 4294967296.0L

/* Philox counter field c1 = stream << 24 | sub.  One stream per kind of
 * random decision, so that no decision reuses another's words. */
enum {
    ST_INIT = 1,
    ST_SURVIVE = 3,
    ST_FECUND = 4,
    ST_PARENT = 5,
    ST_RECOMB_MAT = 6,
    ST_RECOMB_PAT = 7,
    ST_MUTATE_MAT = 8,
    ST_MUTATE_PAT = 9,
    ST_MIGRATE = 10,
    ST_ENCOUNTER = 11,
    ST_CAPTURE = 12,
    ST_MUTVAL_MAT = 13, /* continuous alleles: deviate of a mutated locus */
    ST_MUTVAL_PAT = 14,
    ST_NOISE = 15, /* continuous alleles: residual phenotypic noise */
    ST_SEX = 16,    /* separate sexes: sex of a newborn (block 0) or founder (block 1) */
    ST_FEMALE = 17, /* separate sexes: proposals for a mother */
    ST_MATE = 18,   /* proposals for a father (sexes, mate choice or monogamy) */
    ST_RESOURCE = 19 /* physiology regime: resource growth noise (index 0, block j) */
};

enum { MATING_RANDOM = 0, MATING_PREFERENCE = 1, MATING_ASSORTATIVE = 2 };
#define PARTNER_PROPOSALS 4096u /* proposals before the fallback rule (mate_of) */

enum { GENETICS_BIALLELIC = 0, GENETICS_CONTINUOUS = 1 };

enum { REGIME_WF = 0, REGIME_POISSON_BH = 1, REGIME_CONSUMER_RESOURCE = 2, REGIME_PHYSIOLOGY = 3 };
enum { MODE_RAW = 0, MODE_ZERO = 1, MODE_SKIP = 2, MODE_LAZY = 3, MODE_MAP = 4 };

/* ------------------------------------------------------------------ */
/* Philox4x32-10, written from its published definition (Salmon et al. */
/* 2011, section 3): ten rounds of two 32x32->64 multiplications with  */
/* the Weyl key schedule.                                               */
/* ------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    int round;
    for (round = 0; round < 10; ++round) {
        uint64_t prod_a = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t prod_b = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(prod_b >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)prod_b;
        uint32_t y2 = (uint32_t)(prod_a >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)prod_a;
        x0 = y0;
        x1 = y1;
        x2 = y2;
        x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

/* Counter-based stream: the word for (individual index, stream, sub,
 * component) in generation gen of the replicate identified by c3.  The
 * last block is memoised; that changes no result. */
typedef struct {
    uint32_t key[2];
    uint32_t c3;
    uint32_t memo_ctr[4];
    uint32_t memo_out[4];
    int memo_valid;
} rng_ctx;

static uint32_t rng_word(rng_ctx *g, uint32_t index, uint32_t stream, uint32_t gen, uint32_t sub, uint32_t comp)
{
    uint32_t ctr[4];
    ctr[0] = index;
    ctr[1] = (stream << 24) | sub;
    ctr[2] = gen;
    ctr[3] = g->c3;
    if (!(g->memo_valid && memcmp(ctr, g->memo_ctr, sizeof ctr) == 0)) {
        oracle_philox4x32_10(ctr, g->key, g->memo_out);
        memcpy(g->memo_ctr, ctr, sizeof ctr);
        g->memo_valid = 1;
    }
    return g->memo_out[comp];
}

/* Word q of a stream read as one sequence: block q/4, component q%4. */
static uint32_t seq_word(rng_ctx *g, uint32_t index, uint32_t stream, uint32_t gen, uint32_t q)
{
    return rng_word(g, index, stream, gen, q >> 2, q & 3u);
}

/* Uniform index in [0, n): floor(x * n / 2^64) with x the 64-bit word
 * lo | hi << 32, so every index has probability 1/n up to 2^-64. */
static uint32_t uniform_index(uint32_t lo, uint32_t hi, uint32_t n)
{
    unsigned __int128 x = ((unsigned __int128)hi << 32) | lo;
    return (uint32_t)((x * n) >> 64);
}

/* Standard normal deviate from one Philox block by the Box-Muller
 * transform (Box & Muller 1958): u1 in (0, 1] from words 0 (low) and 1
 * (high), u2 in [0, 1) from words 2 and 3, 53 bits each, and
 * n = sqrt(-2 ln u1) cos(2 pi u2).  Continuous alleles only. */
static double normal_deviate(rng_ctx *g, uint32_t index, uint32_t stream, uint32_t gen, uint32_t sub)
{
    const double two_pi = 6.283185307179586476925;
    uint64_t a = ((uint64_t)rng_word(g, index, stream, gen, sub, 1) << 32) | rng_word(g, index, stream, gen, sub, 0);
    uint64_t b = ((uint64_t)rng_word(g, index, stream, gen, sub, 3) << 32) | rng_word(g, index, stream, gen, sub, 2);
    double u1 = ((double)(a >> 11) + 1.0) * (1.0 / 9007199254740992.0);
    double u2 = (double)(b >> 11) * (1.0 / 9007199254740992.0);
    return sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
}

/* ------------------------------------------------------------------ */
/* Thresholds.  A Bernoulli(p) decision is "x < T" with T = floor(p 2^32)*/
/* (p >= 1: always, p <= 0: never).  A discrete draw by inversion is    */
/* k = min{k : x < T_k} with T_k = floor(F(k) 2^32); the last entry is  */
/* "always".  A table ends at the first k whose T_k reaches 2^32 - 1.   */
/* ------------------------------------------------------------------ */
uint64_t oracle_prob_threshold(double p)
{
    if (p >= 1.0)
        return ORACLE_ALWAYS;
    if (!(p > 0.0))
        return 0;
    return (uint64_t)floor(p * TWO32);
}

static int close_table(long double cdf, int k, int cap, uint64_t *T)
{
    long double scaled = floorl(cdf * TWO32L);
    if (scaled >= 4294967295.0L || k == cap - 1) {
        T[k] = ORACLE_ALWAYS;
        return 1;
    }
    T[k] = (uint64_t)scaled;
    return 0;
}

/* Poisson(lambda) inverse-CDF thresholds: p_0 = e^-lambda,
 * p_k = p_{k-1} lambda / k, F(k) = F(k-1) + p_k.  Returns the length. */
int oracle_poisson_thresholds(double lambda, uint64_t *T, int cap)
{
    long double pk = expl(-(long double)lambda), cdf = 0.0L;
    int k;
    for (k = 0; k < cap; ++k) {
        if (k > 0)
            pk = pk * (long double)lambda / (long double)k;
        cdf += pk;
        if (close_table(cdf, k, cap, T))
            return k + 1;
    }
    return cap;
}

/* Binomial(L, mu) inverse-CDF thresholds: p_0 = (1-mu)^L,
 * p_k = p_{k-1} (L-k+1)/k mu/(1-mu).  Valid for 0 <= mu < 1. */
int oracle_binomial_thresholds(uint32_t L, double mu, uint64_t *T, int cap)
{
    long double m = (long double)mu;
    long double pk = powl(1.0L - m, (long double)L), cdf = 0.0L;
    int k;
    for (k = 0; k < cap; ++k) {
        if (k > 0) {
            if ((uint32_t)k > L)
                pk = 0.0L;
            else
                pk = pk * (long double)(L - (uint32_t)k + 1u) / (long double)k * m / (1.0L - m);
        }
        cdf += pk;
        if ((uint32_t)k == L) { /* all mass is in 0..L */
            T[k] = ORACLE_ALWAYS;
            return k + 1;
        }
        if (close_table(cdf, k, cap, T))
            return k + 1;
    }
    return cap;
}

/* Geometric skip thresholds: the number of non-crossover boundaries
 * before the next crossover, g, has P(g <= k) = 1 - (1-r)^(k+1).
 * T_k = floor((1 - (1-r)^(k+1)) 2^32) for k = 0 .. n-1. */
void oracle_geometric_thresholds(double r, uint32_t n, uint64_t *T)
{
    uint32_t k;
    for (k = 0; k < n; ++k)
        T[k] = (uint64_t)floorl((1.0L - powl(1.0L - (long double)r, (long double)(k + 1u))) * TWO32L);
}

/* Inversion: smallest k with x < T_k. */
static uint32_t draw_by_table(uint32_t x, const uint64_t *T, int len)
{
    int k = 0;
    while (k < len - 1 && (uint64_t)x >= T[k])
        ++k;
    return (uint32_t)k;
}

/* ------------------------------------------------------------------ */
/* Parameters, state, statistics.                                      */
/* ------------------------------------------------------------------ */
/* The consumer-resource regime's extra parameters: the resource is species
 * 0 (census n0 / capacity of the parameters), the consumer species 1. */
typedef struct {
    uint32_t n0_consumer, capacity_consumer;
    uint32_t resource_trials; /* offspring trials per surviving resource */
    uint32_t habitat;         /* slots an encounter lands on uniformly; 0: the resource census */
    double attack;      /* capture probability at a perfect phenotype match */
    double match_width; /* width of the Gaussian matching of phenotypes */
    double encounters;  /* mean encounters per consumer and generation */
    double conversion;  /* consumer offspring mean per credited capture */
    double resource_q0; /* per-trial success of a resource at low density */
    double resource_K;  /* resource density scale of the logistic factor */
    double surv_resource[4], surv_consumer[4]; /* survival by age class 0, 1, 2, 3 and older */
} oracle_ecology;

/* The physiologically structured consumer of Supplementary S2 (resource
 * consumption, somatic growth, reproduction, mortality), with two dynamic
 * resources.  Symbols as in S2. */
typedef struct oracle_physiology {
    double alpha, gamma, delta;   /* intake alpha W^gamma at carrying capacity; metabolism delta W */
    double attack, handling;      /* h(R, K) = a (R/K) / (1 + a T_H R/K) */
    double K[2], growth[2], growth_sd[2], R0[2]; /* resources: capacity, growth rate mean and sd, initial */
    double steepness, switch_frac, w_max; /* diet share of resource 1: logistic in l[W] - u l[W_max] */
    double kappa, qJ, qA;         /* allocation to irreversible mass; reserve ratios (newborn, adult) */
    double beta1, beta2, beta_s;  /* survival: size logistic and starvation */
    double maturity;              /* sigma: mature when X >= sigma */
    double v_f, v_m;              /* reproductive skew of mothers (eggs) and fathers (X) */
    double kappa1, kappa2, kappa3; /* recruits Phi = kappa1 F / (1 + (F/kappa2)^kappa3) */
    uint32_t breed_every;         /* T: reproduction every T time steps */
} oracle_physiology;

typedef struct {
    uint64_t seed;
    uint32_t replicate_id;
    uint32_t regime; /* 0: Wright-Fisher, constant N; 1: Poisson fecundity, Beverton-Holt survival */
    uint32_t n0, capacity; /* per patch */
    uint32_t n_loci;
    uint32_t n_patches; /* patches on a ring, >= 1 */
    double mu, r, theta, omega, K, fecundity;
    double migration; /* backward migration rate */
    uint32_t dispersal; /* 0: to the two ring neighbours; 1: biased island model */
    double home_return; /* island model: share of migrants that return to their patch of origin */
    const int8_t *effects; /* n_loci values, NULL: all +1 */
    const oracle_ecology *ecology; /* consumer-resource regime only */
    /* Continuous allelic values (Supplementary S2, "Genetics"): genetics =
     * GENETICS_CONTINUOUS replaces the biallelic bits by one float per
     * allele. */
    uint32_t genetics;
    double allele_mean;   /* mean initial allelic value a0 */
    double allele_sd;     /* standard deviation of the initial allelic values */
    double mut_sd_factor; /* varpi: a mutation adds N(0, (varpi a0)^2) */
    double noise_sd;      /* varrho: residual phenotypic noise */
    uint32_t exp_transform; /* 1: the expressed phenotype is exp(z) */
    /* Linkage map and mating systems (main text, the mating-system and
     * linkage paragraph; Supplementary S2, "Reproduction"). */
    const double *linkage; /* n_loci - 1 crossover probabilities, boundary b at [b-1]; NULL: r everywhere */
    uint32_t sexes;        /* 1: separate sexes (mothers female, fathers male) */
    uint32_t mating;       /* MATING_RANDOM, MATING_PREFERENCE (shared), MATING_ASSORTATIVE */
    double pref_optimum;   /* shared preference: males near this phenotype are preferred */
    double pref_width;     /* width of the preference or of the assortment, > 0 */
    uint32_t monogamy;     /* 1: all offspring of a mother in a generation share one father */
    const struct oracle_physiology *physiology; /* REGIME_PHYSIOLOGY only */
} oracle_params;

typedef struct {
    uint32_t generation, n, n_parents, n_survivors, extinct;
    uint32_t captures; /* consumers: credited captures of the last generation */
    int64_t sum_z, sum_z2;
    uint64_t near_ties, truncated, sum_threshold;
    uint64_t updates; /* cumulative genotype-locus updates, sum of N_t L */
    double sum_zf, sum_zf2; /* continuous alleles: sums of the expressed phenotypes (serial order) */
    double resource[2];     /* physiology regime: resource densities R_1, R_2 */
    double eggs;            /* physiology regime: eggs F laid at the last step (0 off breeding steps) */
} oracle_stats;

/* One patch of one species of a replicate (a deme): its own individuals
 * and its own Philox counter field c3 = replicate << 12 | species << 10 |
 * patch. */
typedef struct {
    rng_ctx rng;
    uint32_t species, cap;
    uint32_t n;
    uint8_t *genome; /* genome[i][h][l], one byte per allele */
    int32_t *z;
    float *cg;       /* continuous alleles: cg[i][h][l] */
    float *zf;       /* continuous alleles: expressed phenotype */
    double *X, *Y, *G; /* physiology regime: irreversible, reversible and gonadal mass */
    uint8_t *age;    /* consumer-resource regime: age of each individual */
    uint8_t *sex;    /* separate sexes: 0 female, 1 male */
    uint32_t n_surv_f; /* separate sexes: surviving females of the last generation */
    /* the last generation's survivors, fecundities and parents */
    uint32_t *survivors, n_survivors;
    uint32_t *kids, *owner, n_next, n_carry;
    uint32_t *mom, *dad, *src;
    uint64_t *won;     /* resources: lowest key of a capture this generation */
    uint32_t *intake;  /* consumers: credited captures this generation */
    oracle_stats stats;
} oracle_deme;

typedef struct {
    oracle_params prm;
    int8_t *effects;
    int mode;
    uint32_t L;
    uint64_t *geo;   /* L-1 entries */
    uint64_t *binom; /* mutation-count table */
    int binom_len;
    uint64_t *pois;
    int pois_len;
    uint64_t mig_T; /* migration threshold, 0: no migration */
    uint32_t *Rmap; /* linkage map: floor(r_b 2^32) of boundary b (index b, 1..L-1); NULL: none */
    uint64_t home_T; /* island model: a migrant returns home when MIGRATE word 1 < home_T */
    uint32_t generation, n_patches, n_demes;
    oracle_deme *deme;
    /* consumer-resource regime */
    oracle_ecology eco;
    /* physiology regime */
    oracle_physiology phy;
    double R[2];
    uint64_t *enc;  /* encounters per consumer, Poisson(encounters) */
    int enc_len;
    uint64_t *capT; /* capture threshold by |z_c - z_r| */
    uint32_t capT_len;
    uint64_t *cpois; /* consumer offspring: Poisson(conversion m) for intake m, TABLE_CAP each */
    int *cpois_len;
} oracle_pop;

#define TABLE_CAP 1024

/* The crossover-sampling mode is a function of r alone. */
int oracle_recomb_mode(double r)
{
    if (r == 0.5)
        return MODE_RAW;
    if (r == 0.0)
        return MODE_ZERO;
    if (r < 0.10)
        return MODE_SKIP;
    return MODE_LAZY;
}

/* Viability under Gaussian stabilising selection, v(z) = exp(-(z-theta)^2
 * / (2 omega^2)); omega <= 0 switches selection off. */
static double viability(const oracle_pop *P, int32_t z)
{
    double d;
    if (!(P->prm.omega > 0.0))
        return 1.0;
    d = (double)z - P->prm.theta;
    return exp(-(d * d) / (2.0 * P->prm.omega * P->prm.omega));
}

/* Beverton-Holt density factor s(N) = 1 / (1 + (lambda - 1) N / K): with
 * Poisson(lambda) offspring per survivor the expected next census is
 * lambda N s(N), whose fixed point is K when selection is off. */
static double density_factor(const oracle_pop *P, uint32_t n)
{
    if (P->prm.regime != REGIME_POISSON_BH || !(P->prm.K > 0.0))
        return 1.0;
    return 1.0 / (1.0 + (P->prm.fecundity - 1.0) * (double)n / P->prm.K);
}

/* Additive genotype-phenotype map, z = sum_l e_l (b0_l + b1_l - 1). */
static int32_t phenotype(const oracle_pop *P, const uint8_t *h0, const uint8_t *h1)
{
    int64_t z = 0;
    uint32_t l;
    for (l = 0; l < P->L; ++l)
        z += (int64_t)P->effects[l] * ((int64_t)h0[l] + (int64_t)h1[l] - 1);
    return (int32_t)z;
}

/* Continuous alleles: viability of an expressed phenotype (a float). */
static double viability_f(const oracle_pop *P, float z)
{
    double d;
    if (!(P->prm.omega > 0.0))
        return 1.0;
    d = (double)z - P->prm.theta;
    return exp(-(d * d) / (2.0 * P->prm.omega * P->prm.omega));
}

/* Continuous alleles (Supplementary S2, "Genetics", phenotype value): the
 * genotypic value is the sum over loci of the midpoint of the two
 * inherited allelic values; the phenotype adds residual noise
 * N(0, varrho^2) (NOISE block `sub` of individual `index` in generation
 * gen) and is expressed as exp(z) under the transform.  Stored as float. */
static float phenotype_cont(const oracle_pop *P, oracle_deme *D, const float *h0, const float *h1, uint32_t index,
                            uint32_t gen, uint32_t sub)
{
    double g = 0.0, z;
    uint32_t l;
    for (l = 0; l < P->L; ++l)
        g += 0.5 * ((double)h0[l] + (double)h1[l]);
    z = g;
    if (P->prm.noise_sd > 0.0)
        z += P->prm.noise_sd * normal_deviate(&D->rng, index, ST_NOISE, gen, sub);
    if (P->prm.exp_transform)
        z = exp(z);
    return (float)z;
}

static float *allele_row_f(const oracle_pop *P, float *g, uint32_t i, uint32_t h)
{
    return g + ((size_t)i * 2u + h) * P->L;
}

/* Separate sexes: an individual is female (0) or male (1) by one fair bit,
 * bit 0 of word 0 of SEX block `sub` (0: newborn `index` of generation gen;
 * 1: founder `index` of generation gen). */
static uint8_t sex_of(rng_ctx *g, uint32_t index, uint32_t gen, uint32_t sub)
{
    return (uint8_t)(rng_word(g, index, ST_SEX, gen, sub, 0) & 1u);
}

/* Physiology regime (Supplementary S2).  A founder (or a written
 * individual) is born at its own neonate mass: X = Omega (its expressed
 * phenotype), Y = q_J X, no gonads. */
static void founders_body(const oracle_pop *P, oracle_deme *D, uint32_t n)
{
    uint32_t i;
    free(D->X);
    free(D->Y);
    free(D->G);
    D->X = D->Y = D->G = NULL;
    if (P->prm.regime != REGIME_PHYSIOLOGY)
        return;
    D->X = (double *)malloc(sizeof(double) * (n ? n : 1));
    D->Y = (double *)malloc(sizeof(double) * (n ? n : 1));
    D->G = (double *)calloc(n ? n : 1, sizeof(double));
    for (i = 0; i < n; ++i) {
        D->X[i] = (double)D->zf[i];
        D->Y[i] = P->phy.qJ * D->X[i];
    }
}

/* S2, Resource Consumption: the proportion h(R, K) by which scarcity of a
 * resource cuts consumption, a Holling type-II response in R/K. */
static double resource_h(const oracle_physiology *F, double R, double K)
{
    double x = F->attack * R / K;
    return x / (1.0 + F->handling * x);
}

/* S2, Resource Consumption and Somatic Growth, for adult i in one time
 * step: intake alpha W^gamma split between the resources by the diet share
 * pi(W, 1) = 1 / (1 + exp(-p (l[W] - u l[W_max]))), l[W] = W^(1/3) (body
 * length from mass), each scaled by its h; net production dW = intake -
 * delta W.  A surplus goes to irreversible mass in the share min(1,
 * kappa Y/X), the rest to reserves; a deficit is drawn from the reserves
 * (irreversible mass is not starved away).  At a breeding step a mature
 * individual (X >= sigma) sets aside the reserves above q_A X as gonads.
 * Adds its consumption to e[0], e[1]. */
static void grow(const oracle_pop *P, oracle_deme *D, uint32_t i, const double h[2], int breeding, double e[2])
{
    const oracle_physiology *F = &P->phy;
    double X = D->X[i], Y = D->Y[i], W = X + Y, G = 0.0;
    double pi1 = 1.0 / (1.0 + exp(-F->steepness * (cbrt(W) - F->switch_frac * cbrt(F->w_max))));
    double intake = F->alpha * pow(W, F->gamma);
    double e1 = h[0] * pi1 * intake, e2 = h[1] * (1.0 - pi1) * intake;
    double dW = e1 + e2 - F->delta * W;
    e[0] += e1;
    e[1] += e2;
    if (dW > 0.0) {
        double f = F->kappa * Y / X;
        if (f > 1.0)
            f = 1.0;
        X += f * dW;
        Y += (1.0 - f) * dW;
    } else {
        Y += dW;
    }
    if (breeding && X >= F->maturity) {
        G = Y - F->qA * X;
        if (G < 0.0)
            G = 0.0;
        Y -= G;
    }
    D->X[i] = X;
    D->Y[i] = Y;
    D->G[i] = G;
}

/* S2, Mortality: survival from one time step to the next, starvation risk
 * times the size logistic, (1 - exp(-beta_s Y/X)) / (1 + exp(-beta_2 (X -
 * beta_1))); no reserves left: death. */
static double phys_survival(const oracle_physiology *F, double X, double Y)
{
    if (!(Y > 0.0))
        return 0.0;
    return (1.0 - exp(-F->beta_s * Y / X)) / (1.0 + exp(-F->beta2 * (X - F->beta1)));
}

static int breeding_step(const oracle_pop *P, uint32_t t)
{
    return P->prm.regime == REGIME_PHYSIOLOGY && t % P->phy.breed_every == P->phy.breed_every - 1u;
}

/* S2, Reproduction: the eggs of female i, G_i / (Omega_i + q_J Omega_i). */
static double eggs_of(const oracle_pop *P, const oracle_deme *D, uint32_t i)
{
    double om = (double)D->zf[i];
    return D->G[i] / (om + P->phy.qJ * om);
}

static void founders_sex(const oracle_pop *P, oracle_deme *D, uint32_t n, uint32_t gen)
{
    uint32_t i;
    free(D->sex);
    D->sex = (uint8_t *)calloc(n ? n : 1, 1);
    if (P->prm.sexes)
        for (i = 0; i < n; ++i)
            D->sex[i] = sex_of(&D->rng, i, gen, 1);
}

static uint8_t *allele_row(const oracle_pop *P, uint8_t *g, uint32_t i, uint32_t h)
{
    return g + ((size_t)i * 2u + h) * P->L;
}

static void free_deme(oracle_deme *D)
{
    free(D->genome);
    free(D->z);
    free(D->cg);
    free(D->zf);
    D->cg = NULL;
    D->zf = NULL;
    free(D->sex);
    D->sex = NULL;
    free(D->X);
    free(D->Y);
    free(D->G);
    D->X = D->Y = D->G = NULL;
    free(D->age);
    free(D->won);
    free(D->intake);
    D->age = NULL;
    D->won = NULL;
    D->intake = NULL;
    free(D->survivors);
    free(D->kids);
    free(D->owner);
    free(D->mom);
    free(D->dad);
    free(D->src);
    D->genome = NULL;
    D->z = NULL;
    D->survivors = D->kids = D->owner = D->mom = D->dad = D->src = NULL;
}

void oracle_destroy(oracle_pop *P)
{
    uint32_t k;
    if (!P)
        return;
    if (P->deme)
        for (k = 0; k < P->n_demes; ++k)
            free_deme(&P->deme[k]);
    free(P->deme);
    free(P->enc);
    free(P->capT);
    free(P->cpois);
    free(P->cpois_len);
    free(P->effects);
    free(P->geo);
    free(P->binom);
    free(P->pois);
    free(P->Rmap);
    free(P);
}

static void census(const oracle_pop *P, oracle_deme *D)
{
    uint32_t i;
    D->stats.generation = P->generation;
    D->stats.n = D->n;
    D->stats.sum_z = 0;
    D->stats.sum_z2 = 0;
    D->stats.sum_zf = 0.0;
    D->stats.sum_zf2 = 0.0;
    D->stats.resource[0] = P->prm.regime == REGIME_PHYSIOLOGY ? P->R[0] : 0.0;
    D->stats.resource[1] = P->prm.regime == REGIME_PHYSIOLOGY ? P->R[1] : 0.0;
    if (P->prm.genetics == GENETICS_CONTINUOUS) {
        for (i = 0; i < D->n; ++i) {
            D->stats.sum_zf += (double)D->zf[i];
            D->stats.sum_zf2 += (double)D->zf[i] * (double)D->zf[i];
        }
        return;
    }
    for (i = 0; i < D->n; ++i) {
        D->stats.sum_z += D->z[i];
        D->stats.sum_z2 += (int64_t)D->z[i] * (int64_t)D->z[i];
    }
}

/* Consumer-resource tables: encounters per consumer, capture threshold by
 * phenotype distance, consumer offspring by intake. */
static void build_ecology(oracle_pop *P)
{
    const oracle_ecology *E = &P->eco;
    uint32_t d, m;
    int32_t abs_sum = 0;
    uint32_t l;
    for (l = 0; l < P->L; ++l)
        abs_sum += P->effects[l] < 0 ? -P->effects[l] : P->effects[l];
    P->enc = (uint64_t *)malloc(sizeof(uint64_t) * TABLE_CAP);
    P->enc_len = oracle_poisson_thresholds(E->encounters, P->enc, TABLE_CAP);
    /* |z_c - z_r| <= 2 sum |e_l| */
    P->capT_len = 2u * (uint32_t)abs_sum + 1u;
    P->capT = (uint64_t *)malloc(sizeof(uint64_t) * P->capT_len);
    for (d = 0; d < P->capT_len; ++d) {
        double dd = (double)d;
        P->capT[d] = oracle_prob_threshold(E->attack * exp(-(dd * dd) / (2.0 * E->match_width * E->match_width)));
    }
    /* intake never exceeds the encounters, at most enc_len - 1 */
    P->cpois = (uint64_t *)malloc(sizeof(uint64_t) * TABLE_CAP * (size_t)P->enc_len);
    P->cpois_len = (int *)malloc(sizeof(int) * (size_t)P->enc_len);
    for (m = 0; m < (uint32_t)P->enc_len; ++m)
        P->cpois_len[m] = oracle_poisson_thresholds(E->conversion * (double)m, P->cpois + (size_t)m * TABLE_CAP, TABLE_CAP);
}

static int ecology_ok(const oracle_ecology *E)
{
    int a;
    if (!E || E->n0_consumer > E->capacity_consumer || E->capacity_consumer < 1 || E->resource_trials < 1 ||
        E->resource_trials > 64 || !(E->attack >= 0.0 && E->attack <= 1.0) || !(E->match_width > 0.0) ||
        !(E->encounters >= 0.0) || !(E->conversion >= 0.0) || !(E->resource_q0 >= 0.0 && E->resource_q0 <= 1.0) ||
        !(E->resource_K > 0.0))
        return 0;
    for (a = 0; a < 4; ++a)
        if (!(E->surv_resource[a] >= 0.0 && E->surv_resource[a] <= 1.0) ||
            !(E->surv_consumer[a] >= 0.0 && E->surv_consumer[a] <= 1.0))
            return 0;
    return 1;
}

oracle_pop *oracle_create(const oracle_params *prm)
{
    oracle_pop *P;
    uint32_t L = prm->n_loci, l, i, h, k;
    int cr = prm->regime == REGIME_CONSUMER_RESOURCE;
    if (L == 0 || prm->n0 > prm->capacity || !(prm->mu >= 0.0 && prm->mu < 1.0) || !(prm->r >= 0.0 && prm->r <= 0.5) ||
        prm->n_patches < 1 || prm->n_patches > 1024 || !(prm->migration >= 0.0 && prm->migration <= 1.0) ||
        prm->dispersal > 1 || !(prm->home_return >= 0.0 && prm->home_return <= 1.0) ||
        (prm->n_patches > 1 && prm->regime != REGIME_WF) || prm->regime > REGIME_PHYSIOLOGY ||
        (cr && !ecology_ok(prm->ecology)) || prm->genetics > GENETICS_CONTINUOUS ||
        (prm->genetics == GENETICS_CONTINUOUS &&
         (cr || prm->effects || !(prm->allele_sd >= 0.0) || !(prm->mut_sd_factor >= 0.0) || !(prm->noise_sd >= 0.0) ||
          !isfinite(prm->allele_mean))) ||
        prm->sexes > 1 || prm->mating > MATING_ASSORTATIVE || prm->monogamy > 1 ||
        (prm->mating != MATING_RANDOM && !(prm->pref_width > 0.0 && isfinite(prm->pref_width) &&
                                           isfinite(prm->pref_optimum))) ||
        ((prm->sexes || prm->mating || prm->monogamy) && (prm->n_patches != 1 || cr)))
        return NULL;
    if (prm->linkage)
        for (l = 0; l + 1 < L; ++l)
            if (!(prm->linkage[l] >= 0.0 && prm->linkage[l] <= 0.5))
                return NULL;
    if (prm->regime == REGIME_PHYSIOLOGY) {
        /* the S2 consumer: continuous alleles expressed as exp(z) (neonate
         * mass), one patch, separate sexes, mates drawn by S2's weights */
        const oracle_physiology *F = prm->physiology;
        int j;
        if (!F || prm->genetics != GENETICS_CONTINUOUS || !prm->exp_transform || prm->n_patches != 1 ||
            prm->mating || prm->monogamy || !(F->alpha > 0.0) || !(F->gamma > 0.0 && F->gamma <= 1.0) ||
            !(F->delta >= 0.0) || !(F->attack >= 0.0) || !(F->handling >= 0.0) || !(F->w_max > 0.0) ||
            !(F->kappa >= 0.0) || !(F->qJ > 0.0) || !(F->qA >= 0.0) || !(F->maturity > 0.0) ||
            !(F->v_f >= 0.0) || !(F->v_m >= 0.0) || !(F->kappa1 >= 0.0) || !(F->kappa2 > 0.0) ||
            !(F->kappa3 >= 0.0) || F->breed_every < 1 || !isfinite(F->steepness) || !isfinite(F->switch_frac) ||
            !isfinite(F->beta1) || !isfinite(F->beta2) || !(F->beta_s >= 0.0))
            return NULL;
        for (j = 0; j < 2; ++j)
            if (!(F->K[j] > 0.0) || !(F->R0[j] >= 0.0) || !isfinite(F->growth[j]) || !(F->growth_sd[j] >= 0.0))
                return NULL;
    } else if (prm->physiology) {
        return NULL;
    }
    P = (oracle_pop *)calloc(1, sizeof *P);
    if (!P)
        return NULL;
    P->prm = *prm;
    P->L = L;
    P->effects = (int8_t *)malloc(L);
    for (l = 0; l < L; ++l)
        P->effects[l] = prm->effects ? prm->effects[l] : 1;
    P->prm.effects = P->effects;
    P->prm.ecology = NULL;
    if (prm->regime == REGIME_PHYSIOLOGY) {
        P->phy = *prm->physiology;
        P->prm.sexes = 1; /* S2: a sexually reproducing population */
        P->R[0] = P->phy.R0[0];
        P->R[1] = P->phy.R0[1];
    }
    P->prm.physiology = NULL;
    P->mode = oracle_recomb_mode(prm->r);
    P->prm.linkage = NULL;
    if (prm->linkage) {
        /* a linkage map: boundary b crosses over with its own probability
         * r_b, by the exact bit-serial comparison against floor(r_b 2^32) */
        P->mode = MODE_MAP;
        P->Rmap = (uint32_t *)calloc(L, sizeof(uint32_t));
        for (l = 1; l < L; ++l)
            P->Rmap[l] = (uint32_t)floor(prm->linkage[l - 1] * TWO32);
    }
    P->geo = (uint64_t *)malloc(sizeof(uint64_t) * (L > 1 ? L - 1 : 1));
    oracle_geometric_thresholds(prm->r, L - 1, P->geo);
    P->binom = (uint64_t *)malloc(sizeof(uint64_t) * (L + 1u));
    P->binom_len = oracle_binomial_thresholds(L, prm->mu, P->binom, (int)L + 1);
    P->pois = (uint64_t *)malloc(sizeof(uint64_t) * TABLE_CAP);
    P->pois_len = oracle_poisson_thresholds(prm->fecundity, P->pois, TABLE_CAP);
    P->n_patches = prm->n_patches;
    P->n_demes = cr ? 2u : prm->n_patches;
    P->mig_T = prm->n_patches > 1 ? oracle_prob_threshold(prm->migration) : 0;
    P->home_T = oracle_prob_threshold(prm->home_return);
    if (cr) {
        P->eco = *prm->ecology;
        build_ecology(P);
    }
    P->deme = (oracle_deme *)calloc(P->n_demes, sizeof(oracle_deme));
    P->generation = 0;

    /* Initial state: every allele an independent fair bit (Hardy-Weinberg,
     * allele frequency one half), drawn from stream INIT in generation 0,
     * deme by deme; every individual of age 0. */
    for (k = 0; k < P->n_demes; ++k) {
        oracle_deme *D = &P->deme[k];
        uint32_t W = (L + 31u) / 32u;
        uint32_t n0 = cr && k == 1 ? P->eco.n0_consumer : prm->n0;
        D->species = cr ? k : 0u;
        D->cap = cr && k == 1 ? P->eco.capacity_consumer : prm->capacity;
        D->rng.key[0] = (uint32_t)prm->seed;
        D->rng.key[1] = (uint32_t)(prm->seed >> 32);
        D->rng.c3 = (prm->replicate_id << 12) | (D->species << 10) | (cr ? 0u : k);
        D->n = n0;
        D->genome = (uint8_t *)malloc((size_t)(n0 ? n0 : 1) * 2u * L);
        D->z = (int32_t *)malloc(sizeof(int32_t) * (n0 ? n0 : 1));
        D->age = (uint8_t *)calloc(n0 ? n0 : 1, 1);
        if (prm->genetics == GENETICS_CONTINUOUS) {
            /* Continuous alleles: each an independent N(a0, s0^2) value,
             * allele (h, l) from INIT block h L + l of individual i in
             * generation 0, rounded to float; the founder's phenotype noise
             * from NOISE block 1. */
            D->cg = (float *)malloc(sizeof(float) * (size_t)(n0 ? n0 : 1) * 2u * L);
            D->zf = (float *)malloc(sizeof(float) * (n0 ? n0 : 1));
            memset(D->genome, 0, (size_t)(n0 ? n0 : 1) * 2u * L);
            for (i = 0; i < n0; ++i) {
                for (h = 0; h < 2; ++h) {
                    float *row = allele_row_f(P, D->cg, i, h);
                    for (l = 0; l < L; ++l)
                        row[l] = (float)(prm->allele_mean + prm->allele_sd * normal_deviate(&D->rng, i, ST_INIT, 0, h * L + l));
                }
                D->zf[i] = phenotype_cont(P, D, allele_row_f(P, D->cg, i, 0), allele_row_f(P, D->cg, i, 1), i, 0, 1);
                D->z[i] = 0;
            }
        }
        for (i = 0; prm->genetics == GENETICS_BIALLELIC && i < n0; ++i) {
            for (h = 0; h < 2; ++h) {
                uint8_t *row = allele_row(P, D->genome, i, h);
                for (l = 0; l < L; ++l) {
                    uint32_t w = seq_word(&D->rng, i, ST_INIT, 0, h * W + l / 32u);
                    row[l] = (uint8_t)((w >> (l % 32u)) & 1u);
                }
            }
            D->z[i] = phenotype(P, allele_row(P, D->genome, i, 0), allele_row(P, D->genome, i, 1));
        }
        founders_sex(P, D, n0, 0);
        founders_body(P, D, n0);
        census(P, D);
        D->stats.n_parents = 0;
        D->stats.extinct = n0 == 0;
    }
    return P;
}

/* ------------------------------------------------------------------ */
/* Gamete formation (Fig. 1B; S2 "Genetics": a gamete carries half of  */
/* the parent's alleles, then each locus mutates with probability mu). */
/* mask[l] = 1 takes the allele of haplotype 1 at locus l.              */
/* ------------------------------------------------------------------ */

/* One boundary's crossover under the exact bit-serial comparison of a
 * uniform 32-bit U against R = floor(r 2^32): bit i of U (from the top)
 * is bit `bit` of word 31-i of the boundary's block. */
static int lazy_crossover(rng_ctx *g, uint32_t j, uint32_t stream, uint32_t gen, uint32_t block, uint32_t bit, uint32_t R)
{
    int i;
    for (i = 31; i >= 0; --i) {
        uint32_t rest = (i == 31) ? R : (R & ((1u << (i + 1)) - 1u));
        uint32_t q, x, u, ri;
        if (rest == 0)
            return 0; /* U >= R: the remaining bits of R are zero */
        q = 31u - (uint32_t)i;
        x = rng_word(g, j, stream, gen, 1u + block * 8u + (q >> 2), q & 3u);
        u = (x >> bit) & 1u;
        ri = (R >> i) & 1u;
        if (u != ri)
            return u < ri;
    }
    return 0; /* U == R */
}

/* Geometric gap drawn by word x from the L-1 thresholds of the gap table:
 * the smallest k with x < T_k, or L-1 when x reaches every entry (then the
 * next crossover would lie past the last boundary). */
static uint32_t skip_gap(const uint64_t *geo, uint32_t L, uint32_t x)
{
    uint32_t gap = 0;
    while (gap + 1u < L && (uint64_t)x >= geo[gap])
        ++gap;
    return gap;
}

static void recombination_mask(const oracle_pop *P, rng_ctx *g, uint32_t j, uint32_t stream, uint32_t gen, uint8_t *mask,
                               uint8_t *toggles)
{
    uint32_t L = P->L, l;
    uint32_t phase;
    if (P->mode == MODE_RAW) {
        /* r = 1/2: every locus independently takes either haplotype. */
        for (l = 0; l < L; ++l)
            mask[l] = (uint8_t)((seq_word(g, j, stream, gen, l / 32u) >> (l % 32u)) & 1u);
        return;
    }
    phase = seq_word(g, j, stream, gen, 0) & 1u;
    memset(toggles, 0, L);
    toggles[0] = (uint8_t)phase;
    if (P->mode == MODE_SKIP) {
        /* Crossover boundaries b (between loci b-1 and b) with independent
         * probability r: successive gaps are 1 + geometric, one word each,
         * from word 4 of the stream on (block 0 carries only the phase). */
        uint64_t b = 0;
        uint32_t q = 4;
        for (;;) {
            b += 1u + skip_gap(P->geo, L, seq_word(g, j, stream, gen, q++));
            if (b > L - 1u)
                break;
            toggles[b] = 1;
        }
    } else if (P->mode == MODE_LAZY) {
        uint32_t R = (uint32_t)floor(P->prm.r * TWO32);
        uint32_t bnd;
        for (bnd = 1; bnd < L; ++bnd)
            toggles[bnd] = (uint8_t)lazy_crossover(g, j, stream, gen, bnd / 32u, bnd % 32u, R);
    } else if (P->mode == MODE_MAP) {
        /* linkage map: the bit-serial comparison of each boundary against
         * its own threshold, from the same words as a uniform r would use */
        uint32_t bnd;
        for (bnd = 1; bnd < L; ++bnd)
            toggles[bnd] = (uint8_t)lazy_crossover(g, j, stream, gen, bnd / 32u, bnd % 32u, P->Rmap[bnd]);
    }
    /* MODE_ZERO: no crossover, the phase alone. */
    {
        uint8_t m = 0;
        for (l = 0; l < L; ++l) {
            m ^= toggles[l];
            mask[l] = m;
        }
    }
}

static void make_gamete(const oracle_pop *P, rng_ctx *g, const uint8_t *h0, const uint8_t *h1, uint32_t j, uint32_t gen,
                        int paternal, uint8_t *out, uint8_t *scratch)
{
    uint32_t L = P->L, l;
    uint8_t *mask = scratch, *toggles = scratch + L, *chosen = scratch + 2u * L;
    uint32_t rstream = paternal ? ST_RECOMB_PAT : ST_RECOMB_MAT;
    uint32_t mstream = paternal ? ST_MUTATE_PAT : ST_MUTATE_MAT;
    uint32_t K, accepted = 0, cand = 0;
    recombination_mask(P, g, j, rstream, gen, mask, toggles);
    for (l = 0; l < L; ++l)
        out[l] = mask[l] ? h1[l] : h0[l];
    /* Mutation: K ~ Binomial(L, mu) loci, chosen uniformly without
     * replacement, each flipped -- the same law as an independent flip at
     * each locus with probability mu. */
    K = draw_by_table(seq_word(g, j, mstream, gen, 0), P->binom, P->binom_len);
    if (K == 0)
        return;
    memset(chosen, 0, L);
    /* at most 2^23 candidate pairs per gamete, a bound no run with mu < 1
     * comes near; it keeps every loop finite */
    while (accepted < K && cand < (1u << 23)) {
        uint32_t lo = seq_word(g, j, mstream, gen, 1u + 2u * cand);
        uint32_t hi = seq_word(g, j, mstream, gen, 2u + 2u * cand);
        uint32_t pos = uniform_index(lo, hi, L);
        ++cand;
        if (chosen[pos])
            continue;
        chosen[pos] = 1;
        out[pos] ^= 1u;
        ++accepted;
    }
}

/* Continuous alleles (Supplementary S2, "Genetics"): the gamete takes at
 * each locus the allelic value of the haplotype the crossover mask picks
 * (the same mask as a biallelic gamete); the mutated loci are the
 * biallelic rule's K ~ Binomial(L, mu) distinct loci, and each receives a
 * new value drawn from a normal distribution centred on its value, with
 * standard deviation varpi times the mean initial allelic value:
 * value + varpi |a0| n, n from MUTVAL block `locus` of the offspring,
 * rounded to float. */
static void make_gamete_cont(const oracle_pop *P, rng_ctx *g, const float *h0, const float *h1, uint32_t j, uint32_t gen,
                             int paternal, float *out, uint8_t *scratch)
{
    uint32_t L = P->L, l;
    uint8_t *mask = scratch, *toggles = scratch + L, *chosen = scratch + 2u * L;
    uint32_t rstream = paternal ? ST_RECOMB_PAT : ST_RECOMB_MAT;
    uint32_t mstream = paternal ? ST_MUTATE_PAT : ST_MUTATE_MAT;
    uint32_t vstream = paternal ? ST_MUTVAL_PAT : ST_MUTVAL_MAT;
    double sd = P->prm.mut_sd_factor * fabs(P->prm.allele_mean);
    uint32_t K, accepted = 0, cand = 0;
    recombination_mask(P, g, j, rstream, gen, mask, toggles);
    for (l = 0; l < L; ++l)
        out[l] = mask[l] ? h1[l] : h0[l];
    K = draw_by_table(seq_word(g, j, mstream, gen, 0), P->binom, P->binom_len);
    if (K == 0)
        return;
    memset(chosen, 0, L);
    while (accepted < K && cand < (1u << 23)) {
        uint32_t lo = seq_word(g, j, mstream, gen, 1u + 2u * cand);
        uint32_t hi = seq_word(g, j, mstream, gen, 2u + 2u * cand);
        uint32_t pos = uniform_index(lo, hi, L);
        ++cand;
        if (chosen[pos])
            continue;
        chosen[pos] = 1;
        out[pos] = (float)((double)out[pos] + sd * normal_deviate(g, j, vstream, gen, pos));
        ++accepted;
    }
}

/* ------------------------------------------------------------------ */
/* One generation (Fig. 1): survival under the selective environment   */
/* (D), removal of the dead (E), parents and neonate count (A),        */
/* transmission (B), phenotypes of the newborns (C).  Patches on a     */
/* ring exchange offspring by backward migration (Supplementary S3:    */
/* each patch linked by migration to its neighbouring patches).        */
/* ------------------------------------------------------------------ */

/* Consumer-resource regime, before survival (step 1 of the generation):
 * every consumer meets Poisson(encounters) resources drawn uniformly, with
 * replacement, from the resource census, and captures one when its
 * CAPTURE word falls below the threshold of a exp(-(z_c - z_r)^2 /
 * (2 sigma^2)).  A resource captured more than once is credited to the
 * capture with the lowest (consumer, encounter) pair; captured resources
 * die.  A consumer's intake is its number of credited captures. */
static uint32_t encounter_count(oracle_pop *P, oracle_deme *C, uint32_t i, uint32_t t, uint32_t NR)
{
    if (NR == 0)
        return 0;
    return draw_by_table(seq_word(&C->rng, i, ST_ENCOUNTER, t, 0), P->enc, P->enc_len);
}

/* Target resource of encounter e of consumer i, or NR when nothing is
 * captured.  The encounter lands on a uniform slot of the habitat (at
 * least the resource census): a slot below N_R holds that resource, the
 * others are empty, so encounters fall in proportion to N_R / habitat. */
static uint32_t capture_of(oracle_pop *P, uint32_t i, uint32_t e, uint32_t t)
{
    oracle_deme *R = &P->deme[0], *C = &P->deme[1];
    uint32_t NR = R->n, span = P->eco.habitat > NR ? P->eco.habitat : NR;
    uint32_t tgt = uniform_index(seq_word(&C->rng, i, ST_ENCOUNTER, t, 1u + 2u * e),
                                 seq_word(&C->rng, i, ST_ENCOUNTER, t, 2u + 2u * e), span);
    int32_t dz;
    if (tgt >= NR)
        return NR;
    dz = C->z[i] - R->z[tgt];
    uint32_t d = (uint32_t)(dz < 0 ? -dz : dz);
    return (uint64_t)seq_word(&C->rng, i, ST_CAPTURE, t, e) < P->capT[d] ? tgt : NR;
}

static void encounters(oracle_pop *P, uint32_t t)
{
    oracle_deme *R = &P->deme[0], *C = &P->deme[1];
    uint32_t NR = R->n, NC = C->n, i, e;
    free(R->won);
    free(C->intake);
    R->won = (uint64_t *)malloc(sizeof(uint64_t) * (NR ? NR : 1));
    C->intake = (uint32_t *)calloc(NC ? NC : 1, sizeof(uint32_t));
    for (i = 0; i < NR; ++i)
        R->won[i] = UINT64_MAX;
    /* captures, each resource keeping its lowest (consumer, encounter) */
    for (i = 0; i < NC; ++i) {
        uint32_t ne = encounter_count(P, C, i, t, NR);
        for (e = 0; e < ne; ++e) {
            uint32_t tgt = capture_of(P, i, e, t);
            uint64_t key = ((uint64_t)i << 32) | e;
            if (tgt < NR && key < R->won[tgt])
                R->won[tgt] = key;
        }
    }
    /* credit */
    C->stats.captures = 0;
    for (i = 0; i < NC; ++i) {
        uint32_t ne = encounter_count(P, C, i, t, NR);
        for (e = 0; e < ne; ++e) {
            uint32_t tgt = capture_of(P, i, e, t);
            if (tgt < NR && R->won[tgt] == (((uint64_t)i << 32) | e))
                C->intake[i]++;
        }
        C->stats.captures += C->intake[i];
    }
}

/* Binomial(n, q) inverse-CDF thresholds from IEEE double basic operations
 * (the resource's density-dependent fecundity, recomputed every
 * generation): P(k) = C(n, k) q^k (1-q)^(n-k), the coefficient by the
 * recurrence C(n, k) = C(n, k-1) (n-k+1) / k, the powers by repeated
 * multiplication, F accumulated in order. */
int oracle_small_binomial_thresholds(uint32_t n, double q, uint64_t *T)
{
    double u = 1.0 - q, c = 1.0, F = 0.0;
    uint32_t k, m;
    for (k = 0; k <= n; ++k) {
        double pk;
        uint64_t thr;
        if (k > 0)
            c = c * (double)(n - k + 1u) / (double)k;
        pk = c;
        for (m = 0; m < k; ++m)
            pk = pk * q;
        for (m = 0; m < n - k; ++m)
            pk = pk * u;
        F = F + pk;
        thr = oracle_prob_threshold(F);
        if (thr >= 4294967295ULL || k == n) {
            T[k] = ORACLE_ALWAYS;
            return (int)k + 1;
        }
        T[k] = thr;
    }
    return (int)n + 1;
}

/* Survival probability of individual i of deme D: v(z) times the
 * Beverton-Holt factor (Poisson regime) or the survival of its age class
 * (consumer-resource regime). */
static double survival_probability(const oracle_pop *P, const oracle_deme *D, uint32_t i, double s)
{
    if (P->prm.regime == REGIME_PHYSIOLOGY)
        return phys_survival(&P->phy, D->X[i], D->Y[i]);
    if (P->prm.genetics == GENETICS_CONTINUOUS)
        return viability_f(P, D->zf[i]) * s;
    if (P->prm.regime == REGIME_CONSUMER_RESOURCE) {
        const double *sa = D->species == 0 ? P->eco.surv_resource : P->eco.surv_consumer;
        return viability(P, D->z[i]) * sa[D->age[i]];
    }
    return viability(P, D->z[i]) * s;
}

/* D, E and the offspring counts of A in one deme. */
static void select_and_count(oracle_pop *P, oracle_deme *D, uint32_t t)
{
    uint32_t n = D->n, i, ns = 0;
    uint64_t sumT = 0;
    double s = density_factor(P, n);
    int cr = P->prm.regime == REGIME_CONSUMER_RESOURCE;
    uint8_t *alive = (uint8_t *)calloc(n ? n : 1, 1);
    if (P->prm.regime == REGIME_PHYSIOLOGY) {
        /* S2: every adult eats and grows on this step's resources, then the
         * resources take their growth (Beverton-Holt-like, the per-capita
         * rate r_j + e_{r,j} n_j of this step) minus the consumption. */
        const oracle_physiology *F = &P->phy;
        double h[2], e[2] = {0.0, 0.0};
        int j, breeding = breeding_step(P, t);
        h[0] = resource_h(F, P->R[0], F->K[0]);
        h[1] = resource_h(F, P->R[1], F->K[1]);
        for (i = 0; i < n; ++i)
            grow(P, D, i, h, breeding, e);
        for (j = 0; j < 2; ++j) {
            double r = F->growth[j], Rn;
            if (F->growth_sd[j] > 0.0)
                r += F->growth_sd[j] * normal_deviate(&D->rng, 0, ST_RESOURCE, t, (uint32_t)j);
            Rn = r * P->R[j] / (1.0 + P->R[j] / F->K[j]) - e[j];
            P->R[j] = Rn > 0.0 ? Rn : 0.0;
        }
    }
    /* Survival: Bernoulli(p) per adult; a captured resource dies. */
    for (i = 0; i < n; ++i) {
        double p;
        uint64_t T;
        uint32_t x;
        if (cr && D->species == 0 && D->won[i] != UINT64_MAX)
            continue;
        p = survival_probability(P, D, i, s);
        T = oracle_prob_threshold(p);
        x = seq_word(&D->rng, i, ST_SURVIVE, t, 0);
        alive[i] = (uint8_t)((uint64_t)x < T);
        sumT += T;
        if (p > 0.0 && p < 1.0 && fabs((double)x * (1.0 / TWO32) - p) < 1e-6)
            D->stats.near_ties++;
    }
    /* Removal of the dead: survivors in ascending index order. */
    free(D->survivors);
    D->survivors = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    D->n_surv_f = 0;
    for (i = 0; i < n; ++i)
        if (alive[i]) {
            D->survivors[ns++] = i;
            if (P->prm.sexes && D->sex[i] == 0)
                D->n_surv_f++;
        }
    D->n_survivors = ns;
    D->stats.sum_threshold = sumT;
    free(alive);
    /* Offspring counts as mother: Poisson(fecundity) in the Poisson regime;
     * resources Binomial(trials, q0 max(0, 1 - N_R/K_R)), consumers
     * Poisson(conversion x intake) in the consumer-resource regime. */
    free(D->kids);
    D->kids = NULL;
    if (P->prm.regime == REGIME_POISSON_BH) {
        /* with separate sexes only the females are mothers */
        D->kids = (uint32_t *)malloc(sizeof(uint32_t) * (ns ? ns : 1));
        for (i = 0; i < ns; ++i)
            D->kids[i] = (P->prm.sexes && D->sex[D->survivors[i]] != 0)
                             ? 0u
                             : draw_by_table(seq_word(&D->rng, D->survivors[i], ST_FECUND, t, 0), P->pois, P->pois_len);
    } else if (cr) {
        D->kids = (uint32_t *)malloc(sizeof(uint32_t) * (ns ? ns : 1));
        if (D->species == 0) {
            uint64_t T[65];
            double x = 1.0 - (double)n / P->eco.resource_K;
            int len = oracle_small_binomial_thresholds(P->eco.resource_trials, P->eco.resource_q0 * (x > 0.0 ? x : 0.0), T);
            for (i = 0; i < ns; ++i)
                D->kids[i] = draw_by_table(seq_word(&D->rng, D->survivors[i], ST_FECUND, t, 0), T, len);
        } else {
            for (i = 0; i < ns; ++i) {
                uint32_t m = D->intake[D->survivors[i]];
                D->kids[i] = draw_by_table(seq_word(&D->rng, D->survivors[i], ST_FECUND, t, 0),
                                           P->cpois + (size_t)m * TABLE_CAP, P->cpois_len[m]);
            }
        }
    }
}

/* Neonate count of deme k and, where mothers have offspring counts, each
 * offspring slot's mother.  Wright-Fisher keeps the patch's census while
 * any patch its offspring may descend from (itself and its ring
 * neighbours) has a survivor.  The consumer-resource regime carries its
 * survivors into the next census and fills the room left up to the
 * capacity with newborns. */
static void neonates(oracle_pop *P, uint32_t k)
{
    oracle_deme *D = &P->deme[k];
    uint32_t nn, i;
    free(D->owner);
    D->owner = NULL;
    D->n_carry = 0;
    if (P->prm.regime == REGIME_WF) {
        uint32_t left = (k + P->n_patches - 1u) % P->n_patches, right = (k + 1u) % P->n_patches, q;
        uint32_t sources = D->n_survivors;
        if (P->mig_T > 0 && P->prm.dispersal == 0)
            sources += P->deme[left].n_survivors + P->deme[right].n_survivors;
        else if (P->mig_T > 0 && P->home_T < ORACLE_ALWAYS) /* island model: every patch can be a source */
            for (q = 0; q < P->n_patches; ++q)
                sources += P->deme[q].n_survivors;
        nn = sources > 0 ? D->n : 0;
        /* separate sexes: a female and a male must survive */
        if (P->prm.sexes && (D->n_surv_f == 0 || D->n_surv_f == D->n_survivors))
            nn = 0;
    } else if (P->prm.regime == REGIME_PHYSIOLOGY) {
        /* S2: survivors stay; at a breeding step the mature surviving
         * females lay F = sum of their eggs, and Phi = kappa1 F / (1 +
         * (F/kappa2)^kappa3) recruits (rounded down) join, up to the
         * capacity, when a mature male survived too */
        const oracle_physiology *F = &P->phy;
        uint32_t room, nf = 0, nm = 0;
        double eggs = 0.0, phi;
        uint64_t want = 0;
        D->n_carry = D->n_survivors;
        room = D->cap - D->n_carry;
        D->stats.eggs = 0.0;
        if (breeding_step(P, P->generation)) { /* the step being taken */
            for (i = 0; i < D->n_survivors; ++i) {
                uint32_t a = D->survivors[i];
                if (D->X[a] >= F->maturity) {
                    if (D->sex[a] == 0) {
                        eggs += eggs_of(P, D, a);
                        ++nf;
                    } else {
                        ++nm;
                    }
                }
            }
            D->stats.eggs = eggs;
            if (nf > 0 && nm > 0) {
                phi = F->kappa1 * eggs / (1.0 + pow(eggs / F->kappa2, F->kappa3));
                want = phi >= 4294967295.0 ? 4294967295ull : (uint64_t)floor(phi);
            }
        }
        nn = want > room ? room : (uint32_t)want;
        D->stats.truncated += want - nn;
    } else {
        uint64_t ktot = 0;
        uint32_t slot = 0, room;
        if (P->prm.regime == REGIME_CONSUMER_RESOURCE)
            D->n_carry = D->n_survivors;
        room = D->cap - D->n_carry;
        for (i = 0; i < D->n_survivors; ++i)
            ktot += D->kids[i];
        /* separate sexes: eggs need a surviving male (and a female) */
        if (P->prm.sexes && (D->n_surv_f == 0 || D->n_surv_f == D->n_survivors))
            ktot = 0;
        nn = ktot > room ? room : (uint32_t)ktot;
        D->stats.truncated += ktot - nn;
        D->owner = (uint32_t *)malloc(sizeof(uint32_t) * (nn ? nn : 1));
        for (i = 0; i < D->n_survivors; ++i) {
            uint32_t m;
            for (m = 0; m < D->kids[i]; ++m, ++slot)
                if (slot < nn)
                    D->owner[slot] = D->survivors[i];
        }
    }
    D->n_next = nn; /* newborns; the next census is n_carry + n_next */
}

/* The patch offspring j of patch k descends from.  With probability m it
 * is a migrant whose parents live in a ring neighbour (bit 0 of MIGRATE
 * word 1 picks the side); a source without survivors passes the draw on,
 * in the order: drawn patch, home, the picked side, the other side. */
static uint32_t island_source(oracle_pop *P, uint32_t k, uint32_t j, uint32_t t);

static uint32_t source_patch(oracle_pop *P, uint32_t k, uint32_t j, uint32_t t)
{
    oracle_deme *D = &P->deme[k];
    uint32_t left, right, side, other, drawn, order[4], q;
    if (P->mig_T == 0)
        return k;
    if (P->prm.dispersal == 1)
        return island_source(P, k, j, t);
    left = (k + P->n_patches - 1u) % P->n_patches;
    right = (k + 1u) % P->n_patches;
    side = (seq_word(&D->rng, j, ST_MIGRATE, t, 1) & 1u) ? right : left;
    other = side == right ? left : right;
    drawn = (uint64_t)seq_word(&D->rng, j, ST_MIGRATE, t, 0) < P->mig_T ? side : k;
    order[0] = drawn;
    order[1] = k;
    order[2] = side;
    order[3] = other;
    for (q = 0; q < 4; ++q)
        if (P->deme[order[q]].n_survivors > 0)
            return order[q];
    return k; /* unreachable: a patch with no source has no offspring */
}

/* Biased island dispersal (Supplementary S3, Fig. S3 caption: a share pi
 * of migrants returns to its patch of origin; the others settle in any
 * other patch).  Offspring j of patch k is a would-be migrant when MIGRATE
 * word 0 < T(m); it returns home when word 1 < T(pi); otherwise its parents
 * live in patch i of the other P-1, i uniform from words 2 and 3 (i < k
 * counts as i, i >= k as i + 1).  A source without survivors passes the
 * draw on: home, then the patches after the drawn one in ring order. */
static uint32_t island_source(oracle_pop *P, uint32_t k, uint32_t j, uint32_t t)
{
    oracle_deme *D = &P->deme[k];
    uint32_t n = P->n_patches, drawn = k, q;
    if ((uint64_t)seq_word(&D->rng, j, ST_MIGRATE, t, 0) < P->mig_T &&
        !((uint64_t)seq_word(&D->rng, j, ST_MIGRATE, t, 1) < P->home_T)) {
        uint32_t i = uniform_index(seq_word(&D->rng, j, ST_MIGRATE, t, 2), seq_word(&D->rng, j, ST_MIGRATE, t, 3),
                                   n - 1u);
        drawn = i < k ? i : i + 1u;
    }
    if (P->deme[drawn].n_survivors > 0)
        return drawn;
    if (P->deme[k].n_survivors > 0)
        return k;
    for (q = 1; q < n; ++q)
        if (P->deme[(drawn + q) % n].n_survivors > 0)
            return (drawn + q) % n;
    return k; /* unreachable: a patch with no source has no offspring */
}

/* Phenotype of adult i as a double (integer or continuous alleles). */
static double adult_z(const oracle_pop *P, const oracle_deme *D, uint32_t i)
{
    return P->prm.genetics == GENETICS_CONTINUOUS ? (double)D->zf[i] : (double)D->z[i];
}

/* Mate choice (main text: shared preference or assortative mating): the
 * probability that a mother of adult index m accepts candidate c, as the
 * threshold of its Bernoulli decision.  Shared preference: every mother
 * prefers males near pref_optimum, a(c) = exp(-(z_c - opt)^2 / (2 w^2));
 * assortative: a(c) = exp(-(z_m - z_c)^2 / (2 w^2)). */
static uint64_t choice_threshold(const oracle_pop *P, const oracle_deme *D, uint32_t c, uint32_t m)
{
    double d, w = P->prm.pref_width;
    if (P->prm.mating == MATING_PREFERENCE)
        d = adult_z(P, D, c) - P->prm.pref_optimum;
    else
        d = adult_z(P, D, m) - adult_z(P, D, c);
    return oracle_prob_threshold(exp(-(d * d) / (2.0 * w * w)));
}

/* A parent by proposals (Supplementary S2, "Reproduction": mothers among
 * the females, fathers among the males, each egg's father drawn by the
 * mothers' preference).  Proposal p is survivor S[idx(words 0, 1)] of
 * block p of `stream` for index `key` in generation t; it is accepted when
 * it has the wanted sex (want_sex 0 or 1; -1: any) and, with choice, word 2
 * lies below its mate-choice threshold.  Rejection keeps the law exact:
 * uniform over the eligible, times the acceptance probability.  After
 * PARTNER_PROPOSALS rejected proposals the parent is the first survivor of
 * the wanted sex at or after the last proposal in survivor order
 * (wrapping), or the last proposal itself when any sex will do. */
static uint32_t partner(const oracle_pop *P, oracle_deme *D, uint32_t stream, uint32_t key, uint32_t t, int want_sex,
                        int choice, uint32_t mom)
{
    uint32_t p, r = 0, c, ns = D->n_survivors;
    for (p = 0; p < PARTNER_PROPOSALS; ++p) {
        r = uniform_index(rng_word(&D->rng, key, stream, t, p, 0), rng_word(&D->rng, key, stream, t, p, 1), ns);
        c = D->survivors[r];
        if (want_sex >= 0 && D->sex[c] != (uint8_t)want_sex)
            continue;
        if (choice && !((uint64_t)rng_word(&D->rng, key, stream, t, p, 2) < choice_threshold(P, D, c, mom)))
            continue;
        return c;
    }
    if (want_sex < 0)
        return D->survivors[r];
    for (p = 0; p < ns; ++p) {
        c = D->survivors[(r + p) % ns];
        if (D->sex[c] == (uint8_t)want_sex)
            return c;
    }
    return D->survivors[r]; /* unreachable: the wanted sex survived */
}

/* S2, Reproduction: the mother of an egg among the mature females with
 * probability proportional to her eggs^v_f, the father among the mature
 * males proportional to X^v_m, by proposals: survivor S[idx(words 0, 1)] of
 * block p of `stream` for index key, accepted when it is of the wanted sex
 * and mature and word 2 lies below floor((w / w_max)^v 2^32), w_max the
 * largest weight of the generation's eligible.  After PARTNER_PROPOSALS
 * rejections: the first eligible survivor at or after the last proposal. */
static uint32_t phys_partner(const oracle_pop *P, oracle_deme *D, uint32_t stream, uint32_t key, uint32_t t, int male,
                             double wmax)
{
    const oracle_physiology *F = &P->phy;
    double v = male ? F->v_m : F->v_f;
    uint32_t p, r = 0, c, ns = D->n_survivors;
    for (p = 0; p < PARTNER_PROPOSALS; ++p) {
        double a;
        r = uniform_index(rng_word(&D->rng, key, stream, t, p, 0), rng_word(&D->rng, key, stream, t, p, 1), ns);
        c = D->survivors[r];
        if (D->sex[c] != (uint8_t)male || !(D->X[c] >= F->maturity))
            continue;
        a = (male ? D->X[c] : eggs_of(P, D, c)) / wmax;
        if (v != 1.0)
            a = pow(a, v);
        if ((uint64_t)rng_word(&D->rng, key, stream, t, p, 2) < oracle_prob_threshold(a))
            return c;
    }
    for (p = 0; p < ns; ++p) {
        c = D->survivors[(r + p) % ns];
        if (D->sex[c] == (uint8_t)male && D->X[c] >= F->maturity)
            return c;
    }
    return D->survivors[r]; /* unreachable: an eligible parent survived */
}

/* The next census of deme k into *next, *znext, *anext: carried survivors
 * first (consumer-resource regime: genomes and phenotypes copied, one age
 * class older), then the newborns -- A (parents) + B + C. */
static void offspring(oracle_pop *P, uint32_t k, uint32_t t, uint8_t **next, int32_t **znext, uint8_t **anext,
                      float **cnext, float **zfnext, uint8_t **snext, double **xnext, double **ynext)
{
    oracle_deme *D = &P->deme[k];
    uint32_t nc = D->n_carry, nn = D->n_next, j, L = P->L;
    uint32_t total = nc + nn;
    int cont = P->prm.genetics == GENETICS_CONTINUOUS;
    int phys = P->prm.regime == REGIME_PHYSIOLOGY;
    double emax = 0.0, xmax = 0.0;
    *xnext = *ynext = NULL;
    if (phys) {
        *xnext = (double *)malloc(sizeof(double) * (total ? total : 1));
        *ynext = (double *)malloc(sizeof(double) * (total ? total : 1));
        for (j = 0; j < D->n_survivors; ++j) {
            uint32_t a = D->survivors[j];
            if (!(D->X[a] >= P->phy.maturity))
                continue;
            if (D->sex[a] == 0 && eggs_of(P, D, a) > emax)
                emax = eggs_of(P, D, a);
            if (D->sex[a] == 1 && D->X[a] > xmax)
                xmax = D->X[a];
        }
    }
    uint8_t *scratch = (uint8_t *)malloc(3u * L);
    *cnext = NULL;
    *zfnext = NULL;
    if (cont) {
        *cnext = (float *)malloc(sizeof(float) * (size_t)(total ? total : 1) * 2u * L);
        *zfnext = (float *)malloc(sizeof(float) * (total ? total : 1));
    }
    free(D->mom);
    free(D->dad);
    free(D->src);
    D->mom = (uint32_t *)malloc(sizeof(uint32_t) * (nn ? nn : 1));
    D->dad = (uint32_t *)malloc(sizeof(uint32_t) * (nn ? nn : 1));
    D->src = (uint32_t *)malloc(sizeof(uint32_t) * (nn ? nn : 1));
    *next = (uint8_t *)malloc((size_t)(total ? total : 1) * 2u * L);
    *znext = (int32_t *)malloc(sizeof(int32_t) * (total ? total : 1));
    *anext = (uint8_t *)calloc(total ? total : 1, 1);
    *snext = (uint8_t *)calloc(total ? total : 1, 1);
    for (j = 0; j < nc; ++j) {
        uint32_t i = D->survivors[j];
        memcpy(allele_row(P, *next, j, 0), allele_row(P, D->genome, i, 0), 2u * L);
        (*znext)[j] = D->z[i];
        (*anext)[j] = (uint8_t)(D->age[i] < 3u ? D->age[i] + 1u : 3u); /* class 3: three and older */
        (*snext)[j] = D->sex[i];
        if (cont) {
            memcpy(allele_row_f(P, *cnext, j, 0), allele_row_f(P, D->cg, i, 0), sizeof(float) * 2u * L);
            (*zfnext)[j] = D->zf[i];
        }
        if (phys) {
            (*xnext)[j] = D->X[i];
            (*ynext)[j] = D->Y[i];
        }
    }
    for (j = 0; j < nn; ++j) {
        uint32_t w0 = seq_word(&D->rng, j, ST_PARENT, t, 0);
        uint32_t w1 = seq_word(&D->rng, j, ST_PARENT, t, 1);
        uint32_t w2 = seq_word(&D->rng, j, ST_PARENT, t, 2);
        uint32_t w3 = seq_word(&D->rng, j, ST_PARENT, t, 3);
        uint32_t sp = P->prm.regime == REGIME_WF ? source_patch(P, k, j, t) : k;
        oracle_deme *S = &P->deme[sp];
        uint32_t mom, dad, pos = nc + j;
        if (phys) {
            mom = phys_partner(P, S, ST_FEMALE, j, t, 0, emax);
            dad = phys_partner(P, S, ST_MATE, j, t, 1, xmax);
            /* the egg's irreversible mass is the mother's neonate mass, its
             * reserves the newborn maximum q_J of it */
            (*xnext)[pos] = (double)S->zf[mom];
            (*ynext)[pos] = P->phy.qJ * (double)S->zf[mom];
        } else if (P->prm.regime == REGIME_WF)
            mom = P->prm.sexes ? partner(P, S, ST_FEMALE, j, t, 0, 0, 0)
                               : S->survivors[uniform_index(w0, w1, S->n_survivors)];
        else
            mom = D->owner[j];
        if (phys) {
        } else if (!P->prm.sexes && P->prm.mating == MATING_RANDOM && !P->prm.monogamy)
            dad = S->survivors[uniform_index(w2, w3, S->n_survivors)];
        else /* monogamy: the father is the mother's one mate of the generation */
            dad = partner(P, S, ST_MATE, P->prm.monogamy ? mom : j, t, P->prm.sexes ? 1 : -1,
                          P->prm.mating != MATING_RANDOM, mom);
        if (P->prm.sexes)
            (*snext)[pos] = sex_of(&D->rng, j, t, 0);
        D->mom[j] = mom;
        D->dad[j] = dad;
        D->src[j] = P->prm.regime == REGIME_CONSUMER_RESOURCE ? 0u : sp; /* the source's patch */
        if (cont) {
            /* offspring genetic value at a locus: the midpoint of the two
             * gametes' values (phenotype_cont) */
            make_gamete_cont(P, &D->rng, allele_row_f(P, S->cg, mom, 0), allele_row_f(P, S->cg, mom, 1), j, t, 0,
                             allele_row_f(P, *cnext, pos, 0), scratch);
            make_gamete_cont(P, &D->rng, allele_row_f(P, S->cg, dad, 0), allele_row_f(P, S->cg, dad, 1), j, t, 1,
                             allele_row_f(P, *cnext, pos, 1), scratch);
            (*zfnext)[pos] = phenotype_cont(P, D, allele_row_f(P, *cnext, pos, 0), allele_row_f(P, *cnext, pos, 1), j,
                                            t, 0);
            memset(allele_row(P, *next, pos, 0), 0, 2u * L);
            (*znext)[pos] = 0;
            continue;
        }
        make_gamete(P, &D->rng, allele_row(P, S->genome, mom, 0), allele_row(P, S->genome, mom, 1), j, t, 0,
                    allele_row(P, *next, pos, 0), scratch);
        make_gamete(P, &D->rng, allele_row(P, S->genome, dad, 0), allele_row(P, S->genome, dad, 1), j, t, 1,
                    allele_row(P, *next, pos, 1), scratch);
        (*znext)[pos] = phenotype(P, allele_row(P, *next, pos, 0), allele_row(P, *next, pos, 1));
    }
    free(scratch);
}

int oracle_step(oracle_pop *P, uint32_t n_generations)
{
    uint32_t it, k, nd = P->n_demes;
    uint8_t **next = (uint8_t **)calloc(nd, sizeof(uint8_t *));
    int32_t **znext = (int32_t **)calloc(nd, sizeof(int32_t *));
    uint8_t **anext = (uint8_t **)calloc(nd, sizeof(uint8_t *));
    float **cnext = (float **)calloc(nd, sizeof(float *));
    float **zfnext = (float **)calloc(nd, sizeof(float *));
    uint8_t **snext = (uint8_t **)calloc(nd, sizeof(uint8_t *));
    double **xnext = (double **)calloc(nd, sizeof(double *));
    double **ynext = (double **)calloc(nd, sizeof(double *));
    for (it = 0; it < n_generations; ++it) {
        uint32_t t = P->generation;
        if (P->prm.regime == REGIME_CONSUMER_RESOURCE)
            encounters(P, t);
        for (k = 0; k < nd; ++k)
            select_and_count(P, &P->deme[k], t);
        for (k = 0; k < nd; ++k)
            neonates(P, k);
        for (k = 0; k < nd; ++k)
            offspring(P, k, t, &next[k], &znext[k], &anext[k], &cnext[k], &zfnext[k], &snext[k], &xnext[k], &ynext[k]);
        P->generation = t + 1;
        for (k = 0; k < nd; ++k) {
            oracle_deme *D = &P->deme[k];
            free(D->genome);
            free(D->z);
            free(D->age);
            D->genome = next[k];
            D->z = znext[k];
            D->age = anext[k];
            free(D->cg);
            free(D->zf);
            D->cg = cnext[k];
            D->zf = zfnext[k];
            free(D->sex);
            D->sex = snext[k];
            if (P->prm.regime == REGIME_PHYSIOLOGY) {
                free(D->X);
                free(D->Y);
                free(D->G);
                D->X = xnext[k];
                D->Y = ynext[k];
                D->G = (double *)calloc(D->n_carry + D->n_next ? D->n_carry + D->n_next : 1, sizeof(double));
            }
            D->stats.n_parents = D->n;
            D->stats.n_survivors = D->n_survivors;
            D->n = D->n_carry + D->n_next;
            if (D->n == 0)
                D->stats.extinct = 1;
            D->stats.updates += (uint64_t)D->n * P->L;
            census(P, D);
        }
    }
    free(next);
    free(znext);
    free(anext);
    free(cnext);
    free(zfnext);
    free(snext);
    free(xnext);
    free(ynext);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Accessors, per deme (the patch of a ring, or the species of the      */
/* consumer-resource regime: 0 resource, 1 consumer).  Packed layout:   */
/* individual i, haplotype h, word w holds loci 32w .. 32w+31, locus l  */
/* at bit l % 32; tail bits are zero.                                    */
/* ------------------------------------------------------------------ */
static oracle_deme *deme_of(const oracle_pop *P, uint32_t deme) { return deme < P->n_demes ? &P->deme[deme] : NULL; }

int oracle_get_stats(const oracle_pop *P, uint32_t deme, oracle_stats *out)
{
    oracle_deme *D = deme_of(P, deme);
    if (!D)
        return -1;
    *out = D->stats;
    return 0;
}
uint32_t oracle_get_n(const oracle_pop *P, uint32_t deme) { return deme_of(P, deme) ? P->deme[deme].n : 0; }
uint32_t oracle_get_generation(const oracle_pop *P) { return P->generation; }
uint32_t oracle_get_demes(const oracle_pop *P) { return P->n_demes; }
int oracle_get_mode(const oracle_pop *P) { return P->mode; }
/* Newborns of the last generation (the census minus carried survivors). */
uint32_t oracle_get_newborns(const oracle_pop *P, uint32_t deme) { return deme_of(P, deme) ? P->deme[deme].n_next : 0; }

int oracle_get_genomes(const oracle_pop *P, uint32_t deme, uint32_t *words, size_t n_words)
{
    uint32_t W = (P->L + 31u) / 32u, i, h, l;
    oracle_deme *D = deme_of(P, deme);
    if (!D || n_words < (size_t)D->n * 2u * W)
        return -1;
    memset(words, 0, sizeof(uint32_t) * (size_t)D->n * 2u * W);
    for (i = 0; i < D->n; ++i)
        for (h = 0; h < 2; ++h) {
            const uint8_t *row = D->genome + ((size_t)i * 2u + h) * P->L;
            uint32_t *dst = words + ((size_t)i * 2u + h) * W;
            for (l = 0; l < P->L; ++l)
                dst[l / 32u] |= (uint32_t)row[l] << (l % 32u);
        }
    return 0;
}

/* Replace a deme's population (all of age 0) at generation `generation`
 * (which becomes the replicate's generation) and reset its counters. */
int oracle_set_genomes(oracle_pop *P, uint32_t deme, const uint32_t *words, uint32_t n, uint32_t generation)
{
    uint32_t W = (P->L + 31u) / 32u, i, h, l;
    oracle_deme *D = deme_of(P, deme);
    if (!D || n > D->cap || P->prm.genetics != GENETICS_BIALLELIC)
        return -1;
    free_deme(D);
    D->genome = (uint8_t *)malloc((size_t)(n ? n : 1) * 2u * P->L);
    D->z = (int32_t *)malloc(sizeof(int32_t) * (n ? n : 1));
    D->age = (uint8_t *)calloc(n ? n : 1, 1);
    for (i = 0; i < n; ++i) {
        for (h = 0; h < 2; ++h) {
            uint8_t *row = D->genome + ((size_t)i * 2u + h) * P->L;
            const uint32_t *src = words + ((size_t)i * 2u + h) * W;
            for (l = 0; l < P->L; ++l)
                row[l] = (uint8_t)((src[l / 32u] >> (l % 32u)) & 1u);
        }
        D->z[i] = phenotype(P, D->genome + (size_t)i * 2u * P->L, D->genome + ((size_t)i * 2u + 1u) * P->L);
    }
    D->n = n;
    P->generation = generation;
    D->n_survivors = 0;
    D->n_next = 0;
    D->n_carry = 0;
    founders_sex(P, D, n, generation);
    founders_body(P, D, n);
    memset(&D->stats, 0, sizeof D->stats);
    D->stats.extinct = n == 0;
    census(P, D);
    return 0;
}

int oracle_get_phenotypes(const oracle_pop *P, uint32_t deme, int32_t *z, size_t n)
{
    oracle_deme *D = deme_of(P, deme);
    if (!D || n < D->n)
        return -1;
    memcpy(z, D->z, sizeof(int32_t) * D->n);
    return 0;
}

/* Physiology regime: irreversible and reversible mass of each individual
 * of the current census. */
int oracle_get_body(const oracle_pop *P, uint32_t deme, double *X, double *Y, size_t n)
{
    oracle_deme *D = deme_of(P, deme);
    if (!D || P->prm.regime != REGIME_PHYSIOLOGY || n < D->n)
        return -1;
    memcpy(X, D->X, sizeof(double) * D->n);
    memcpy(Y, D->Y, sizeof(double) * D->n);
    return 0;
}

/* Separate sexes: 0 female, 1 male, per individual of the current census. */
int oracle_get_sexes(const oracle_pop *P, uint32_t deme, uint8_t *sex, size_t n)
{
    oracle_deme *D = deme_of(P, deme);
    if (!D || n < D->n)
        return -1;
    memcpy(sex, D->sex, D->n);
    return 0;
}

int oracle_get_ages(const oracle_pop *P, uint32_t deme, uint8_t *age, size_t n)
{
    oracle_deme *D = deme_of(P, deme);
    if (!D || n < D->n)
        return -1;
    memcpy(age, D->age, D->n);
    return 0;
}

/* Consumers: credited captures of each adult in the last generation. */
int oracle_get_intake(const oracle_pop *P, uint32_t *intake, size_t n)
{
    oracle_deme *D = deme_of(P, 1);
    if (P->prm.regime != REGIME_CONSUMER_RESOURCE || !D || !D->intake || n < D->stats.n_parents)
        return -1;
    memcpy(intake, D->intake, sizeof(uint32_t) * D->stats.n_parents);
    return 0;
}

uint32_t oracle_get_survivors(const oracle_pop *P, uint32_t deme, uint32_t *S, size_t n)
{
    oracle_deme *D = deme_of(P, deme);
    if (!D)
        return 0;
    if (S && n >= D->n_survivors)
        memcpy(S, D->survivors, sizeof(uint32_t) * D->n_survivors);
    return D->n_survivors;
}

/* Parents of the last generation's newborns of a deme: indices into the
 * adults of their source patch, and that patch. */
int oracle_get_parents(const oracle_pop *P, uint32_t deme, uint32_t *mom, uint32_t *dad, uint32_t *src, size_t n)
{
    oracle_deme *D = deme_of(P, deme);
    if (!D || n < D->n_next || (D->n_next > 0 && !D->mom))
        return -1;
    memcpy(mom, D->mom, sizeof(uint32_t) * D->n_next);
    memcpy(dad, D->dad, sizeof(uint32_t) * D->n_next);
    if (src)
        memcpy(src, D->src, sizeof(uint32_t) * D->n_next);
    return 0;
}

/* Gametes of one parent for offspring slots j0 .. j0+count-1 of patch 0
 * in generation gen (the statistical pins sample this directly).  parent
 * is 2L bytes (haplotype 0 then 1); out is count x L bytes. */
int oracle_sample_gametes(oracle_pop *P, const uint8_t *parent, uint32_t j0, uint32_t count, uint32_t gen, int paternal, uint8_t *out)
{
    uint32_t c;
    uint8_t *scratch = (uint8_t *)malloc(3u * P->L);
    for (c = 0; c < count; ++c)
        make_gamete(P, &P->deme[0].rng, parent, parent + P->L, j0 + c, gen, paternal, out + (size_t)c * P->L, scratch);
    free(scratch);
    return 0;
}

/* Continuous alleles: a deme's allelic values, individual-major,
 * haplotype 0 then 1, L floats each. */
int oracle_get_alleles(const oracle_pop *P, uint32_t deme, float *out, size_t n_values)
{
    oracle_deme *D = deme_of(P, deme);
    if (!D || P->prm.genetics != GENETICS_CONTINUOUS || n_values < (size_t)D->n * 2u * P->L)
        return -1;
    memcpy(out, D->cg, sizeof(float) * (size_t)D->n * 2u * P->L);
    return 0;
}

int oracle_get_phenotypes_f(const oracle_pop *P, uint32_t deme, float *z, size_t n)
{
    oracle_deme *D = deme_of(P, deme);
    if (!D || P->prm.genetics != GENETICS_CONTINUOUS || n < D->n)
        return -1;
    memcpy(z, D->zf, sizeof(float) * D->n);
    return 0;
}

/* Continuous alleles: replace a deme's population by n individuals of the
 * given values at generation `generation`; each phenotype takes a
 * founder's noise (NOISE block 1 of individual i in that generation). */
int oracle_set_alleles(oracle_pop *P, uint32_t deme, const float *values, uint32_t n, uint32_t generation)
{
    uint32_t i;
    oracle_deme *D = deme_of(P, deme);
    if (!D || P->prm.genetics != GENETICS_CONTINUOUS || n > D->cap)
        return -1;
    free_deme(D);
    D->genome = (uint8_t *)calloc((size_t)(n ? n : 1) * 2u, P->L);
    D->z = (int32_t *)calloc(n ? n : 1, sizeof(int32_t));
    D->age = (uint8_t *)calloc(n ? n : 1, 1);
    D->cg = (float *)malloc(sizeof(float) * (size_t)(n ? n : 1) * 2u * P->L);
    D->zf = (float *)malloc(sizeof(float) * (n ? n : 1));
    memcpy(D->cg, values, sizeof(float) * (size_t)n * 2u * P->L);
    for (i = 0; i < n; ++i)
        D->zf[i] = phenotype_cont(P, D, allele_row_f(P, D->cg, i, 0), allele_row_f(P, D->cg, i, 1), i, generation, 1);
    D->n = n;
    P->generation = generation;
    D->n_survivors = 0;
    D->n_next = 0;
    D->n_carry = 0;
    founders_sex(P, D, n, generation);
    founders_body(P, D, n);
    memset(&D->stats, 0, sizeof D->stats);
    D->stats.extinct = n == 0;
    census(P, D);
    return 0;
}

/* Continuous alleles: gametes of one parent (2L floats, haplotype 0 then
 * 1) for offspring slots j0 .. j0+count-1 of patch 0 in generation gen. */
int oracle_sample_gametes_cont(oracle_pop *P, const float *parent, uint32_t j0, uint32_t count, uint32_t gen,
                               int paternal, float *out)
{
    uint32_t c;
    uint8_t *scratch;
    if (P->prm.genetics != GENETICS_CONTINUOUS)
        return -1;
    scratch = (uint8_t *)malloc(3u * P->L);
    for (c = 0; c < count; ++c)
        make_gamete_cont(P, &P->deme[0].rng, parent, parent + P->L, j0 + c, gen, paternal, out + (size_t)c * P->L,
                         scratch);
    free(scratch);
    return 0;
}

/* Continuous alleles: phenotype of given allele rows as newborn j of
 * generation gen (sub 0) or founder j (sub 1) of patch 0. */
float oracle_phenotype_cont(oracle_pop *P, const float *h0, const float *h1, uint32_t j, uint32_t gen, uint32_t sub)
{
    return phenotype_cont(P, &P->deme[0], h0, h1, j, gen, sub);
}

/* The normal deviates of Philox blocks (index, stream, gen, sub0 + k) for
 * k < n under key seed and counter field c3. */
void oracle_normals(uint64_t seed, uint32_t c3, uint32_t index, uint32_t stream, uint32_t gen, uint32_t sub0, uint32_t n,
                    double *out)
{
    rng_ctx g;
    uint32_t k;
    g.key[0] = (uint32_t)seed;
    g.key[1] = (uint32_t)(seed >> 32);
    g.c3 = c3;
    g.memo_valid = 0;
    for (k = 0; k < n; ++k)
        out[k] = normal_deviate(&g, index, stream, gen, sub0 + k);
}

/* The phenotype of given allele rows (for pins of the map). */
int32_t oracle_phenotype(const oracle_pop *P, const uint8_t *h0, const uint8_t *h1) { return phenotype(P, h0, h1); }

/* The geometric gap of word x for crossover probability r in a genome of L
 * loci (tests compare the GPU library's lookup with it). */
uint32_t oracle_skip_gap(double r, uint32_t L, uint32_t x)
{
    uint64_t *geo;
    uint32_t gap;
    if (L < 2)
        return 0;
    geo = (uint64_t *)malloc(sizeof(uint64_t) * (L - 1u));
    oracle_geometric_thresholds(r, L - 1u, geo);
    gap = skip_gap(geo, L, x);
    free(geo);
    return gap;
}

/* Search for a test case: over generations t in [t_begin, t_end), offspring
 * slots j < n_slots and both gametes (RECOMB streams of mother and father)
 * of a deme whose counter field is c3, walk the geometric-gap crossovers of
 * a gamete of L loci at crossover probability r as recombination_mask does,
 * and stop at the first consumed gap word equal to x_target after which
 * the next crossover still falls on a boundary (b + 1 + gap <= L - 1).
 * out = {t, j, stream, word index, boundary before the word}; returns 1 if
 * found, else 0.  A test-fixture generator: it draws the oracle's own
 * words and uses the oracle's own table. */
int oracle_find_gap_word(uint64_t seed, uint32_t c3, double r, uint32_t L, uint32_t n_slots, uint32_t t_begin,
                         uint32_t t_end, uint32_t x_target, uint32_t out[5])
{
    uint64_t *geo;
    rng_ctx g;
    uint32_t t, j, s;
    if (L < 2)
        return 0;
    geo = (uint64_t *)malloc(sizeof(uint64_t) * (L - 1u));
    oracle_geometric_thresholds(r, L - 1u, geo);
    g.key[0] = (uint32_t)seed;
    g.key[1] = (uint32_t)(seed >> 32);
    g.c3 = c3;
    g.memo_valid = 0;
    for (t = t_begin; t < t_end; ++t)
        for (j = 0; j < n_slots; ++j)
            for (s = ST_RECOMB_MAT; s <= ST_RECOMB_PAT; ++s) {
                uint64_t b = 0;
                uint32_t q = 4;
                for (;;) {
                    uint32_t x = seq_word(&g, j, s, t, q);
                    uint32_t gap = skip_gap(geo, L, x);
                    if (x == x_target && b + 1u + gap <= L - 1u) {
                        out[0] = t;
                        out[1] = j;
                        out[2] = s;
                        out[3] = q;
                        out[4] = (uint32_t)b;
                        free(geo);
                        return 1;
                    }
                    ++q;
                    b += 1u + gap;
                    if (b > L - 1u)
                        break;
                }
            }
    free(geo);
    return 0;
}

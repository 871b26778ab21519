/*
 * spegg.h -- C ABI of the MI355X implementation of sPEGG's per-generation
 * update (Okamoto & Amarasekare, "sPEGG: high throughput eco-evolutionary
 * simulations on commodity graphics processors").
 *
 * What one generation computes (main text, Fig. 1, steps A-F):
 *   D  survival under the selective environment: adult i survives with
 *      probability v(z_i) s(N_t), v Gaussian stabilising viability, s the
 *      Beverton-Holt density factor (regime SPEGG_POISSON_BH only);
 *   E  the dead are removed: survivors listed in ascending index order;
 *   A  parents and neonate count: Wright-Fisher keeps N constant and draws
 *      mother and father uniformly from the survivors; the Poisson regime
 *      gives each survivor Poisson(lambda) offspring as mother, capped at the
 *      capacity, with a uniformly drawn father;
 *   B  transmission: each parent makes a gamete by crossing over between its
 *      two haplotypes (independent crossovers with probability r at each
 *      boundary between adjacent loci) and flipping each locus with
 *      probability mu (Supplementary Information S2, "Genetics");
 *   C  the newborn's phenotype by the additive map
 *      z = sum_l e_l (b0_l + b1_l - 1), the biallelic form of the paper's
 *      midpoint sum of allelic values (eqn. S2, phenotype value).
 * Replicates advance together as one flattened loop over individuals
 * (Supplementary Fig. S5(B)); each replicate keeps its own parameters.
 *
 * Genome layout (device and host copies alike): individual i of a replicate
 * owns 2W consecutive uint32 words, W = ceil(L/32): haplotype 0 (maternal)
 * words 0..W-1, then haplotype 1 (paternal).  Locus l is bit l%32 of word
 * l/32; bits at loci >= L are zero.  Seen as uint64 on a little-endian
 * machine this is the same bit order.
 *
 * Patches: a replicate may be a ring of n_patches patches (Supplementary
 * Information S3: patches linked by migration to their neighbours), each a
 * Wright-Fisher deme of its own census; or patches under biased island
 * dispersal (spegg_rep_desc.dispersal, below).  With probability `migration` a
 * newborn of patch k descends from parents in patch k-1 or k+1 (backward
 * migration; one fair bit picks the side); a source patch without
 * survivors passes the draw on (drawn patch, home, picked side, other
 * side), so a patch keeps its census while it or a neighbour has a
 * survivor.  Patches advance together; all per-individual indices below are
 * within a patch.
 *
 * Randomness: Philox4x32-10 keyed by the replicate's 64-bit seed, with
 * counter (index, stream << 24 | block, generation, replicate_id << 12 |
 * species << 10 | patch); species is 0 outside the consumer-resource
 * regime.  No counter field encodes a batch position, a thread or a tile,
 * so a replicate's trajectory is the same alone or in any batch.
 *
 * Memory: the caller owns the device memory (one block of
 * spegg_footprint() bytes, 256-byte aligned) and the HIP stream; the library
 * never allocates device memory.  Every call below that takes a spegg_pop
 * is enqueued on that stream.  One handle is used by one thread at a time.
 *
 * Errors: every call returns a status and never throws.  A failed HIP call
 * returns SPEGG_E_DEVICE and makes the handle sticky-errored: later calls
 * return SPEGG_E_STATE.  spegg_last_error() gives the calling thread's
 * message for the last non-OK status.  Extinction and capacity truncation
 * are not errors: they are reported in spegg_rep_stats.
 */
#ifndef SPEGG_H
#define SPEGG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPEGG_ABI_VERSION 6
#define SPEGG_MAX_LOCI 16384u
#define SPEGG_MAX_REPLICATE_ID ((1u << 20) - 1u)
#define SPEGG_MAX_PATCHES 1024u

typedef enum {
    SPEGG_OK = 0,
    SPEGG_E_INVALID = -1,     /* an argument or descriptor is out of range */
    SPEGG_E_NOMEM = -2,       /* the caller's workspace is too small or misaligned */
    SPEGG_E_DEVICE = -3,      /* a HIP call failed; the handle is now sticky-errored */
    SPEGG_E_STATE = -4,       /* the handle is errored, or the call needs a mode that is off */
    SPEGG_E_UNSUPPORTED = -5  /* valid model, but outside what this library implements */
} spegg_status;

typedef enum {
    SPEGG_WF = 0,                /* Wright-Fisher: N constant, viability selection, parents uniform over survivors */
    SPEGG_POISSON_BH = 1,        /* Poisson(fecundity) offspring per surviving mother, survival x Beverton-Holt s(N) */
    SPEGG_CONSUMER_RESOURCE = 2, /* two coevolving species with age classes (spegg_ecology) */
    SPEGG_PHYSIOLOGY = 3         /* physiologically structured consumer of two resources (spegg_physiology) */
} spegg_regime;

/* The consumer-resource regime (Supplementary Information S3: a consumer
 * exploits a resource by phenotype matching), as an individual-based model
 * with overlapping generations and age classes 0..3.  Species 0 is the
 * resource (census n0, capacity of the descriptor), species 1 the consumer.
 * One generation:
 *   1. every consumer draws Poisson(encounters) encounters; each lands on a
 *      uniform slot of the habitat (at least the resource census) and meets
 *      the resource of that index if there is one (mass action); it
 *      captures it when a CAPTURE word falls below
 *      floor(attack exp(-(z_c - z_r)^2 / (2 match_width^2)) 2^32);
 *   2. a resource captured more than once is credited to the capture with
 *      the lowest (consumer index, encounter ordinal); captured resources
 *      die; a consumer's intake is its number of credited captures;
 *   3. the others survive with v(z) times the survival of their age class;
 *   4. surviving resources have Binomial(resource_trials, resource_q0 max(0,
 *      1 - N_R / resource_K)) offspring as mothers, surviving consumers
 *      Poisson(conversion x intake); fathers are uniform survivors of the
 *      same species;
 *   5. the next census is the survivors (one age class older, genomes
 *      carried; class 3 holds three and older) followed by the newborns
 *      (age 0), up to the capacity.
 * Philox counters carry the species in c3 (bits 10..11). */
typedef struct spegg_ecology {
    uint32_t n0_consumer, capacity_consumer;
    uint32_t resource_trials; /* 1..64 */
    uint32_t habitat;         /* encounter slots; 0: the resource census (every encounter meets a resource) */
    double attack;            /* capture probability at a perfect match, 0..1 */
    double match_width;       /* > 0 */
    double encounters;        /* mean encounters per consumer and generation, >= 0 */
    double conversion;        /* consumer offspring mean per credited capture, >= 0 */
    double resource_q0;       /* per-trial offspring probability of a resource at low density, 0..1 */
    double resource_K;        /* > 0 */
    double surv_resource[4], surv_consumer[4]; /* survival by age class 0, 1, 2, 3 and older; each 0..1 */
} spegg_ecology;

/* The physiologically structured consumer of Supplementary Information S2
 * (resource consumption, somatic growth, reproduction, mortality), one
 * generation = one time step.  Each individual has irreversible and
 * reversible mass X, Y and a sex; its phenotype is its neonate mass Omega =
 * exp(z) (continuous alleles with exp_transform = 1 are required).  A step:
 *   1. every individual eats: W = X + Y, intake alpha W^gamma, a share
 *      pi = 1 / (1 + exp(-steepness (W^(1/3) - switch_frac w_max^(1/3)))) of
 *      it on resource 1 and 1 - pi on resource 2, each cut by the scarcity
 *      h = x / (1 + handling x), x = attack R_j / K_j; net production dW =
 *      intake - delta W; a surplus goes to X in the share min(1, kappa Y/X)
 *      and to Y otherwise, a deficit comes out of Y; at a breeding step
 *      (step t with t % breed_every == breed_every - 1) a mature individual
 *      (X >= maturity) moves its reserves above qA X into gonads G;
 *   2. it survives with (1 - exp(-beta_s Y/X)) / (1 + exp(-beta2 (X -
 *      beta1))) (0 without reserves), a SURVIVE word against floor(p 2^32);
 *   3. the resources take r_j R/(1 + R/K_j) minus what was eaten (at least
 *      0), r_j = growth[j] + growth_sd[j] n_j, n_j the Box-Muller deviate
 *      of block j of stream 19 for index 0 in step t;
 *   4. at a breeding step the mature surviving females lay F = sum of
 *      G/(Omega + qJ Omega) eggs and floor(kappa1 F / (1 + (F/kappa2)^kappa3))
 *      recruits join (up to the capacity; none without a mature male);
 *      mothers are drawn in proportion to eggs^v_f, fathers to X^v_m among
 *      the mature, by proposals as for mate choice (stream 17 mothers, 18
 *      fathers; acceptance (w / w_max)^v, w_max the generation's largest);
 *      a recruit is born with X = its mother's Omega and Y = qJ X;
 *   5. the survivors stay (first, in order), the recruits follow.
 * Founders and written individuals start at X = their own Omega, Y = qJ X. */
typedef struct spegg_physiology {
    double alpha, gamma, delta;        /* intake alpha W^gamma (0 < gamma <= 1), metabolism delta W */
    double attack, handling;           /* scarcity h of a resource */
    double K[2], growth[2], growth_sd[2], R0[2]; /* resources: K > 0, growth rate mean and sd, initial density */
    double steepness, switch_frac, w_max; /* diet share of resource 1 */
    double kappa, qJ, qA;              /* allocation to X; reserve ratios of newborns (> 0) and adults */
    double beta1, beta2, beta_s;       /* survival */
    double maturity;                   /* mature when X >= maturity (> 0) */
    double v_f, v_m;                   /* reproductive skew of mothers and fathers */
    double kappa1, kappa2, kappa3;     /* recruitment, kappa2 > 0 */
    uint32_t breed_every;              /* >= 1 */
} spegg_physiology;

typedef struct spegg_pop spegg_pop; /* opaque; owns no device memory */

/* Dispersal among the patches of a replicate (Supplementary Information
 * S3).  SPEGG_RING: patches on a ring, a migrant's parents live in patch
 * k-1 or k+1 (bit 0 of MIGRATE word 1 picks the side).  SPEGG_ISLAND: the
 * biased island model of Supplementary Fig. S3 -- a share home_return of
 * would-be migrants returns to its patch of origin (MIGRATE word 1 below
 * floor(home_return 2^32)), the others' parents live in a patch drawn
 * uniformly among the other P-1 (index i from MIGRATE words 2 and 3, i
 * below the home patch as is, from it on as i+1); the effective migration
 * rate is migration x (1 - home_return).  A newborn is a would-be migrant
 * when MIGRATE word 0 is below floor(migration 2^32).  A source patch
 * without survivors passes the draw on: ring -- home, the drawn side, the
 * other side; island -- home, then the patches after the drawn one in ring
 * order; a patch keeps its census while any patch it can draw from has
 * survivors. */
enum { SPEGG_RING = 0, SPEGG_ISLAND = 1 };

/* Genetics of a replicate.  SPEGG_BIALLELIC: the bit-packed biallelic loci
 * described at the top of this header.  SPEGG_CONTINUOUS: the paper's own
 * genetic model (Supplementary Information S2, "Genetics"): every allele is
 * a continuous value (a float); a gamete takes at each locus the value of
 * the haplotype its crossover mask picks (the mask a biallelic gamete would
 * draw: same crossover law, same random words); each locus mutates with
 * probability mu (the biallelic rule's loci) to a value drawn from a
 * normal distribution centred on the old value with standard deviation
 * mut_sd_factor x |allele_mean| (varpi times the mean initial allelic
 * value); the newborn's genetic value is the sum over loci of the
 * midpoints of its two inherited values, its phenotype that plus
 * N(0, noise_sd^2) residual noise, expressed as exp(z) when exp_transform
 * is 1 (the S2 transform); selection acts on the expressed phenotype.
 * Initial values are N(allele_mean, allele_sd^2).  Normal deviates come
 * from one Philox block each by the Box-Muller transform (u1 in (0, 1] from
 * words 0 and 1, u2 in [0, 1) from words 2 and 3, 53 bits each,
 * sqrt(-2 ln u1) cos(2 pi u2)): allele (h, l) of founder i from INIT block
 * h L + l; the mutation of locus l of newborn j's maternal (paternal)
 * gamete from stream 13 (14) block l; newborn j's noise from stream 15
 * block 0, a founder's from block 1.  Values are computed in double and
 * stored as float, so results agree with a serial evaluation to rounding:
 * genomes and survivors match except where a rounding straddles a float
 * or a threshold boundary.  Regimes SPEGG_WF and SPEGG_POISSON_BH, with or
 * without patches; effects must be NULL. */
enum { SPEGG_BIALLELIC = 0, SPEGG_CONTINUOUS = 1 };

/* Linkage map and mating systems (main text: arbitrary linkage; random,
 * shared-preference or assortative mating, monogamy or polygynandry;
 * Supplementary Information S2, "Reproduction": mothers among the females,
 * fathers among the males).
 *
 * linkage: n_loci - 1 crossover probabilities in [0, 1/2], boundary b
 * (between loci b-1 and b) at linkage[b-1]; boundary b crosses over when
 * the bit-serial comparison of its uniform U against R_b = floor(r_b 2^32)
 * finds U < R_b, U's bits from the top taken from bit b % 32 of words
 * 1 + 8 (b / 32) + ... of the RECOMB stream, as for a uniform r of at least
 * 0.10.  NULL: r at every boundary.
 *
 * sexes = 1: each individual is female or male by bit 0 of word 0 of stream
 * 16 (block 0 for newborn j, block 1 for a founder); mothers are females,
 * fathers males; in the Poisson regime only females have offspring; a
 * population without a surviving female or male has no newborns.
 *
 * A parent of a wanted sex, and a father chosen by the mothers (mating =
 * SPEGG_PREFERENCE: acceptance exp(-(z - pref_optimum)^2 / (2
 * pref_width^2)), shared by every mother; SPEGG_ASSORTATIVE: exp(-(z_mother
 * - z)^2 / (2 pref_width^2))), come from proposals: proposal p is survivor
 * S[floor(x64 N_s / 2^64)] with x64 from words 0 (low) and 1 of block p of
 * stream 17 (mothers) or 18 (fathers) for the newborn (or, under monogamy,
 * for the mother's adult index, so that all her offspring of a generation
 * share one father), accepted when it has the wanted sex and word 2 lies
 * below floor(acceptance 2^32).  After 4096 rejected proposals the parent is
 * the first survivor of the wanted sex at or after the last proposal in
 * survivor order (wrapping), or that proposal when any sex will do.
 * Without sexes, mate choice or monogamy the parents are drawn as before.
 * Mating options need one patch and a one-species regime. */
enum { SPEGG_RANDOM_MATING = 0, SPEGG_PREFERENCE = 1, SPEGG_ASSORTATIVE = 2 };

/* One replicate.  The per-deme parameter table of Supplementary Fig. S5(B):
 * every individual looks up its replicate's entry. */
typedef struct spegg_rep_desc {
    uint64_t seed;         /* Philox key */
    uint32_t replicate_id; /* logical replicate id, 0..SPEGG_MAX_REPLICATE_ID; never a batch slot */
    uint32_t regime;       /* spegg_regime */
    uint32_t n0;           /* initial census of each patch, <= capacity */
    uint32_t capacity;     /* most individuals a patch may hold, >= 1 */
    uint32_t n_loci;       /* L, 1..SPEGG_MAX_LOCI */
    uint32_t n_patches;    /* patches on the ring, 1..SPEGG_MAX_PATCHES; more than 1 needs SPEGG_WF */
    double mu;             /* per-locus, per-gamete flip probability, 0 <= mu < 1 */
    double r;              /* crossover probability at each adjacent-locus boundary, 0 <= r <= 1/2 */
    double theta;          /* optimum of Gaussian stabilising selection */
    double omega;          /* its width, v(z) = exp(-(z-theta)^2 / (2 omega^2)); omega <= 0: no selection */
    double K;              /* Beverton-Holt carrying capacity (POISSON_BH); K <= 0: no density dependence */
    double fecundity;      /* Poisson mean lambda (POISSON_BH) */
    double migration;      /* backward migration rate, 0..1; unused with one patch */
    uint32_t dispersal;    /* SPEGG_RING (0) or SPEGG_ISLAND (1), the patches a migrant's parents may live in */
    double home_return;    /* SPEGG_ISLAND: share of would-be migrants that stay home, 0..1 */
    const int8_t *effects; /* n_loci allelic effects in [-4, 4], copied at create; NULL: all +1 */
    const spegg_ecology *ecology; /* SPEGG_CONSUMER_RESOURCE only (copied at create); else NULL */
    uint32_t genetics;     /* SPEGG_BIALLELIC (0) or SPEGG_CONTINUOUS (1) */
    double allele_mean;    /* SPEGG_CONTINUOUS: mean initial allelic value a0 */
    double allele_sd;      /* SPEGG_CONTINUOUS: standard deviation of the initial values, >= 0 */
    double mut_sd_factor;  /* SPEGG_CONTINUOUS: varpi, mutation sd = varpi |a0|, >= 0 */
    double noise_sd;       /* SPEGG_CONTINUOUS: residual phenotypic noise varrho, >= 0 */
    uint32_t exp_transform; /* SPEGG_CONTINUOUS: 1 expresses exp(z) */
    const double *linkage; /* n_loci - 1 per-boundary crossover probabilities (copied at create); NULL: r */
    uint32_t sexes;        /* 1: separate sexes */
    uint32_t mating;       /* SPEGG_RANDOM_MATING, SPEGG_PREFERENCE or SPEGG_ASSORTATIVE */
    double pref_optimum;   /* SPEGG_PREFERENCE: the preferred phenotype */
    double pref_width;     /* mate choice: width of the acceptance, > 0 */
    uint32_t monogamy;     /* 1: one father for all of a mother's offspring of a generation */
    const spegg_physiology *physiology; /* SPEGG_PHYSIOLOGY only (copied at create); else NULL */
} spegg_rep_desc;

/* Census of one deme (a patch, or a species of the consumer-resource
 * regime), or of a replicate summed over its demes, after the latest
 * generation. */
typedef struct spegg_rep_stats {
    uint32_t generation;    /* t: generations completed since creation (or since the last write) */
    uint32_t n;             /* N_t */
    uint32_t n_parents;     /* N_{t-1}, the adults the last generation started from */
    uint32_t n_survivors;   /* survivors among them */
    uint32_t extinct;       /* 1 once N reached 0 (replicate: every patch) */
    uint32_t captures;      /* consumers: resources captured and credited in the last generation; else 0 */
    int64_t sum_z;          /* sum of z over the N_t individuals (exact) */
    int64_t sum_z2;         /* sum of z^2 (exact) */
    uint64_t near_ties;     /* cumulative survival draws with |x 2^-32 - p| < 1e-6, 0 < p < 1 */
    uint64_t truncated;     /* cumulative offspring dropped at the capacity */
    uint64_t sum_threshold; /* sum over the last adults of floor(p 2^32): mean viability x 2^32 x n_parents */
    uint64_t updates;       /* cumulative genotype-locus updates: sum over generations of N_t x L */
    double sum_zf;          /* SPEGG_CONTINUOUS: sum of the expressed phenotypes (sum_z, sum_z2 are 0) */
    double sum_zf2;         /* SPEGG_CONTINUOUS: sum of their squares */
    double resource[2];     /* SPEGG_PHYSIOLOGY: resource densities R_1, R_2 after the last step */
    double eggs;            /* SPEGG_PHYSIOLOGY: eggs laid at the last step (0 off breeding steps) */
} spegg_rep_stats;

/* ABI version of the loaded library; equals SPEGG_ABI_VERSION. */
int spegg_abi_version(void);

/* Message for the calling thread's last non-OK status ("" if none).  The
 * pointer stays valid until the thread's next spegg call. */
const char *spegg_last_error(void);

/* Device bytes a population of these replicates needs; 0 if a descriptor
 * is invalid (spegg_last_error says which).  Host-only; no device access. */
size_t spegg_footprint(const spegg_rep_desc *reps, uint32_t n_reps);

/* Validate the descriptors, carve the caller's workspace (device_mem,
 * device_bytes >= spegg_footprint, 256-byte aligned), upload the parameter
 * tables, and enqueue the initial population on hip_stream (a hipStream_t;
 * NULL is the null stream): every allele an independent fair bit, drawn
 * from the INIT stream in generation 0.  Returns without waiting.  The
 * handle borrows device_mem and the stream; both must outlive it.
 * SPEGG_E_INVALID: a descriptor; SPEGG_E_NOMEM: workspace too small or
 * misaligned; SPEGG_E_UNSUPPORTED: an offspring kernel block would need more
 * LDS than the device gives one block (effect planes, gap table and bitmaps
 * of the longest genome in a shape). */
spegg_status spegg_pop_create(const spegg_rep_desc *reps, uint32_t n_reps, void *device_mem, size_t device_bytes,
                              void *hip_stream, spegg_pop **out);

/* Enqueue n_generations full generations (Fig. 1 steps D, E, A, B, C) for
 * every replicate.  Returns without waiting; no device-to-host traffic. */
spegg_status spegg_step_generations(spegg_pop *pop, uint32_t n_generations);

/* Wait for the stream, then copy the census of replicates 0..n-1 (n <=
 * n_reps), each summed over its patches, into host_out. */
spegg_status spegg_stats(spegg_pop *pop, spegg_rep_stats *host_out, uint32_t n);

/* Wait, then copy the census of each of replicate rep's demes into
 * host_out: its patches in order, or for the consumer-resource regime its
 * two species (0 resource, 1 consumer).  n must equal the number of demes. */
spegg_status spegg_deme_stats(spegg_pop *pop, uint32_t rep, spegg_rep_stats *host_out, uint32_t n);

/* Wait, then copy the current genomes of one deme of replicate rep (patch
 * `patch` of a ring, or species `species` of the consumer-resource regime;
 * the other index is 0) as N x 2W words (layout above) into host_words
 * (room for n_words words); *n_out = N.  SPEGG_E_INVALID if the room is
 * short or the deme does not exist. */
spegg_status spegg_read_genomes(spegg_pop *pop, uint32_t rep, uint32_t patch, uint32_t species, uint32_t *host_words,
                                size_t n_words, uint32_t *n_out);

/* Replace the population of one deme by n individuals (all of age 0)
 * given as n x 2W words (tail bits must be zero, n <= capacity) at
 * generation `generation`; phenotypes are recomputed and the deme's census
 * and cumulative counters reset.  The demes of one replicate must all be at
 * one generation when it next steps (SPEGG_E_STATE otherwise).  Waits for
 * the stream before returning (host_words may be reused). */
spegg_status spegg_write_genomes(spegg_pop *pop, uint32_t rep, uint32_t patch, uint32_t species,
                                 const uint32_t *host_words, uint32_t n, uint32_t generation);

/* Wait, then copy the phenotypes z (N int32) of a deme into host_z.  For
 * continuous alleles the values are the bits of the float phenotypes
 * (spegg_read_phenotypes_f reads them as floats). */
spegg_status spegg_read_phenotypes(spegg_pop *pop, uint32_t rep, uint32_t patch, uint32_t species, int32_t *host_z,
                                   size_t n, uint32_t *n_out);

/* Continuous alleles (Supplementary Information S2, "Genetics"; see
 * SPEGG_CONTINUOUS).  spegg_read_alleles waits, then copies the allelic
 * values of patch `patch` of replicate rep as N x 2 x L floats
 * (individual-major, haplotype 0 then 1, locus l at position l) into
 * host_values (room for n_values floats); *n_out = N.
 * spegg_write_alleles replaces that patch's population by n individuals
 * given in the same layout (finite values, n <= capacity) at generation
 * `generation`: phenotypes are recomputed (noise from NOISE block 1, as for
 * founders) and the census and counters reset; it waits before returning.
 * spegg_read_phenotypes_f waits, then copies the N expressed phenotypes.
 * SPEGG_E_STATE for a replicate of biallelic genomes (the genome calls
 * above return it for continuous ones); SPEGG_E_INVALID for short room or a
 * missing patch. */
spegg_status spegg_read_alleles(spegg_pop *pop, uint32_t rep, uint32_t patch, float *host_values, size_t n_values,
                                uint32_t *n_out);
spegg_status spegg_write_alleles(spegg_pop *pop, uint32_t rep, uint32_t patch, const float *host_values, uint32_t n,
                                 uint32_t generation);
spegg_status spegg_read_phenotypes_f(spegg_pop *pop, uint32_t rep, uint32_t patch, float *host_z, size_t n,
                                     uint32_t *n_out);

/* SPEGG_PHYSIOLOGY: wait, then copy each individual's irreversible and
 * reversible mass (N doubles each) of replicate rep into host_X, host_Y. */
spegg_status spegg_read_body(spegg_pop *pop, uint32_t rep, double *host_X, double *host_Y, size_t n,
                             uint32_t *n_out);

/* Separate sexes: wait, then copy each individual's sex (N uint8, 0
 * female, 1 male) of patch `patch` of replicate rep into host_sex; all 0
 * without sexes. */
spegg_status spegg_read_sexes(spegg_pop *pop, uint32_t rep, uint32_t patch, uint8_t *host_sex, size_t n,
                              uint32_t *n_out);

/* Wait, then copy the age classes (N uint8, 0..3) of a deme of the
 * consumer-resource regime into host_age. */
spegg_status spegg_read_ages(spegg_pop *pop, uint32_t rep, uint32_t species, uint8_t *host_age, size_t n,
                             uint32_t *n_out);

/* Wait, then copy each consumer's credited captures in the last
 * generation, by its index among that generation's adults. */
spegg_status spegg_read_intake(spegg_pop *pop, uint32_t rep, uint32_t *host_intake, size_t n, uint32_t *n_out);

/* Wait, then copy the ascending survivor list of a deme's last generation
 * (indices into its previous adults) into host_idx. */
spegg_status spegg_read_survivors(spegg_pop *pop, uint32_t rep, uint32_t patch, uint32_t species, uint32_t *host_idx,
                                  size_t n, uint32_t *n_out);

/* Per-locus copies of allele 1 over a deme's current census (2N genes per
 * locus): the genetic distribution behind the phenotypes (Fig. 1F;
 * Supplementary S2, "Genetics").  counts_dev is caller-owned device scratch
 * of n_loci uint32 (n_loci must equal the replicate's L); host_counts gets
 * the result; *n_out = N.  Reads every genome once; waits for the stream. */
spegg_status spegg_allele_counts(spegg_pop *pop, uint32_t rep, uint32_t patch, uint32_t species, uint32_t *counts_dev,
                                 uint32_t *host_counts, uint32_t n_loci, uint32_t *n_out);

/* For callers that cannot allocate device memory (work under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * result of spegg_allele_counts without the caller's counts_dev.  The
 * per-locus counters live in a library-owned device array of
 * SPEGG_MAX_LOCI uint32 (64 KiB per device, held until the process ends);
 * the call allocates nothing.  n_loci must equal the replicate's L (at most
 * SPEGG_MAX_LOCI; SPEGG_E_INVALID otherwise).  Every call on one device
 * shares that array: calls on one device must not overlap (from two threads
 * or two streams), or their counts race.  Waits for the stream. */
spegg_status spegg_allele_counts_noalloc(spegg_pop *pop, uint32_t rep, uint32_t patch, uint32_t species,
                                         uint32_t *host_counts, uint32_t n_loci, uint32_t *n_out);

/* Record each newborn's mother and father (indices into the previous
 * adults) from the next generation on.  Off by default. */
spegg_status spegg_set_trace(spegg_pop *pop, int enable);

/* Wait, then copy the parents recorded for a deme's newborns of the last
 * generation (the census minus carried survivors): mother and father as
 * indices into the adults of the patch they came from, and that patch
 * (host_src may be NULL).  SPEGG_E_STATE if tracing was off for the last
 * generation. */
spegg_status spegg_read_parents(spegg_pop *pop, uint32_t rep, uint32_t patch, uint32_t species, uint32_t *host_mom,
                                uint32_t *host_dad, uint32_t *host_src, size_t n, uint32_t *n_out);

/* Replay generations as captured HIP graphs (enable = 1, the default) or
 * launch every kernel (0).  Graphs are used only on a non-null stream and
 * while no kernel timing is on; results are the same either way. */
spegg_status spegg_set_graph(spegg_pop *pop, int enable);

/* Capture, without running them, the generation graphs that
 * spegg_step_generations replays (one generation and a run of 16), and
 * upload them to the device, so that a later step replays them at once.
 * Nothing is enqueued that changes the population; waits for the stream.
 * A no-op when graphs are off or timing is on. */
spegg_status spegg_prepare_graphs(spegg_pop *pop);

/* Kernel kinds timed by spegg_set_timing. */
enum {
    SPEGG_KERNEL_SURVIVE = 0,   /* step D and the offspring count of A */
    SPEGG_KERNEL_COMPACT = 1,   /* step E: survivor list, offspring slots, census advance; consumer-resource
                                   and physiology survivors carried into the next census */
    SPEGG_KERNEL_OFFSPRING = 2, /* steps A (parents), B and C, census partials */
    SPEGG_KERNEL_ENCOUNTER = 3, /* consumer-resource: encounters, captures and their credit to consumers */
    SPEGG_KERNEL_CARRY = 4,     /* no launch of its own any more (the carry is part of compact): always 0 */
    SPEGG_KERNEL_KINDS = 5
};

#define SPEGG_TIME_ALL 0x1Fu

/* Bracket the kernels of the kinds in kinds_mask (bit k: kind k; 0 stops)
 * launched by later spegg_step_generations calls with HIP events on the
 * population's stream.  The events carry no system-scope fence, so that
 * recording them neither writes back nor invalidates the caches the timed
 * kernels use. */
spegg_status spegg_set_timing(spegg_pop *pop, uint32_t kinds_mask);

/* Wait, then report per kernel kind the summed event time in milliseconds
 * and the number of launches timed since the last call, and reset them.
 * Arrays hold n_kinds (<= SPEGG_KERNEL_KINDS) entries. */
spegg_status spegg_kernel_times(spegg_pop *pop, double *ms, uint64_t *launches, uint32_t n_kinds);

/* Wait, then report the offspring launches timed since the last call, by
 * launch class (the replicates that share one kernel shape: one launch per
 * class and generation): the class's least and greatest genome words W,
 * the summed event milliseconds and the launches, for up to cap classes
 * (*n_out = the number of classes); resets these sums.  Kernel-kind sums of
 * spegg_kernel_times are kept apart. */
spegg_status spegg_offspring_class_times(spegg_pop *pop, uint32_t *w_min, uint32_t *w_max, double *ms,
                                         uint64_t *launches, uint32_t cap, uint32_t *n_out);

/* Pick the offspring kernel's shape (lanes per gamete, words per lane,
 * chunks held in registers) for each genome length W in the population by
 * timing: for each W in turn, every distinct shape first runs
 * generations_per_trial untimed generations (loading its code and capturing
 * the graphs that replay it), then generations_per_trial generations
 * bracketed by two HIP events on the population's stream, run as
 * spegg_step_generations runs them; the shapes take turns over two rounds,
 * each keeps its least time per genotype-locus update, and the least of
 * those stays.  Shapes change no result, so the trial generations are
 * ordinary generations of the simulation (the population advances by
 * 4 x generations_per_trial per shape and W).  The caller's kernel timing
 * (spegg_set_timing) is suspended meanwhile and its pending events kept.
 * Reports the distinct W (ascending) and each one's chosen cap on lanes per
 * gamete (arrays of cap entries; *n_out = number of W).  Waits. */
spegg_status spegg_autotune(spegg_pop *pop, uint32_t generations_per_trial, uint32_t *w_out, uint32_t *gcap_out,
                            uint32_t cap, uint32_t *n_out);

/* Two environment variables, read when a population is created, override
 * launch choices for experiments; neither changes a result:
 * SPEGG_OFFSPRING_GCAP (1, 2, 4, 8, 16 or 32) replaces the default cap on
 * lanes per gamete (by default the shape whose gamete spans two register
 * chunks, up to 16 lanes per chunk; 4 beyond) for every genome length;
 * SPEGG_OFFSPRING_GRID (64 .. 2^20) fixes the blocks of every
 * offspring launch (by default a one-deme class launches as many blocks as
 * the device holds at once, a class of several demes up to 2^18). */

/* Set the offspring kernel's cap on lanes per gamete for the replicates of
 * W genome words (gcap a power of two in 1..32), as spegg_autotune would
 * choose it, without timing: e.g. to reuse a tuning found earlier.  Changes
 * no result.  SPEGG_E_INVALID for another gcap or a W no replicate has.
 * Waits. */
spegg_status spegg_set_offspring_cap(spegg_pop *pop, uint32_t W, uint32_t gcap);

/* Release the handle (not the caller's memory or stream).  NULL is a no-op. */
void spegg_pop_destroy(spegg_pop *pop);

/* ------------------------------------------------------------- serving
 * Sweep jobs served from one device arena with continuous batching.  A job
 * is the replicates of one parameter sweep point (Supplementary Fig. S5(B):
 * replicates and parameter combinations run side by side), advanced for a
 * fixed number of generations.  Jobs are admitted in submission order
 * while the oldest waiting job's footprint fits in the free arena; between
 * steps resident jobs keep their state, finished jobs leave at once and
 * free their memory, and newly admitted jobs join.  A job's results are
 * those of its replicates run alone: the counters never see the batch.
 * The server borrows the arena (256-byte aligned) and the stream; it
 * allocates no device memory. */
typedef struct spegg_server spegg_server;

/* n_streams (1..8): resident jobs are spread over hip_stream and
 * n_streams - 1 streams the server creates (default priority), so the
 * kernels of different jobs overlap on the device; 1 keeps all work on
 * hip_stream.  Waits for hip_stream once (the arena must be ready). */
spegg_status spegg_server_create(void *device_mem, size_t device_bytes, void *hip_stream, uint32_t n_streams,
                                 spegg_server **out);

/* Queue a job of n_reps replicates for n_generations (>= 1) generations.
 * SPEGG_E_INVALID for a bad descriptor or a job_id already queued,
 * resident or holding an unread result; SPEGG_E_NOMEM if the job's
 * footprint exceeds the whole arena (it could never be admitted).
 * Descriptors and effects are copied. */
spegg_status spegg_server_submit(spegg_server *srv, uint64_t job_id, const spegg_rep_desc *reps, uint32_t n_reps,
                                 uint32_t n_generations);

/* Admit waiting jobs that fit (oldest first, stopping at the first that
 * does not) onto the least loaded stream and enqueue min(n_generations, its
 * remaining generations) for every resident job; a job's census is copied
 * to pinned host memory behind its last generation.  Then wait for the
 * previous step's work only (at most two steps are queued, so the device
 * runs one while the host admits and retires around the next) and retire
 * the jobs that finished before this step: results recorded, memory freed
 * (or held, spegg_server_keep).  n_generations = 0 drains instead: it waits
 * for all enqueued work and retires every finished job, then admits.
 * Reports the jobs resident (finished ones not yet retired included) and
 * those still waiting (either pointer may be NULL). */
spegg_status spegg_server_step(spegg_server *srv, uint32_t n_generations, uint32_t *n_resident, uint32_t *n_waiting);

/* Hold a waiting or running job's population after it finishes: its result
 * is reported as usual, and its population stays in the arena, readable
 * through spegg_server_population (e.g. its genomes), until
 * spegg_server_release.  SPEGG_E_INVALID for an unknown or finished job. */
spegg_status spegg_server_keep(spegg_server *srv, uint64_t job_id);

/* The population handle of a finished, kept job (valid until
 * spegg_server_release; do not destroy or step it). */
spegg_status spegg_server_population(spegg_server *srv, uint64_t job_id, spegg_pop **out);

/* Free a finished, kept job's population and memory (waits for its stream). */
spegg_status spegg_server_release(spegg_server *srv, uint64_t job_id);

/* Ids of the jobs finished since the last poll, in completion order (at
 * most cap; *n_out = how many were written). */
spegg_status spegg_server_poll(spegg_server *srv, uint64_t *job_ids, uint32_t cap, uint32_t *n_out);

/* Final census of each replicate (summed over patches) of a finished job;
 * n must equal its n_reps.  The result is released once read. */
spegg_status spegg_server_result(spegg_server *srv, uint64_t job_id, spegg_rep_stats *host_out, uint32_t n);

/* Arena bytes held by resident jobs and the largest free block. */
spegg_status spegg_server_usage(spegg_server *srv, size_t *used, size_t *largest_free);

/* Release the server and every resident job (not the arena or stream). */
void spegg_server_destroy(spegg_server *srv);

/* Host-only: the library's inverse-CDF threshold table (x < T_k decides k;
 * the last entry is 2^32, "always").  kind 0: Poisson(a); 1: Binomial(b, a);
 * 2: geometric crossover gaps for r = a over b entries.  Returns the length,
 * or -1 if cap is too small or the arguments are invalid. */
int spegg_threshold_table(int kind, double a, uint32_t b, uint64_t *out, int cap);

/* Host-only test hook: the geometric gap the offspring kernel draws from
 * word x for crossover probability r (0 < r < 1/2) in a genome of n_loci
 * (>= 2) loci, starting its table search from the first guess `guess`: the
 * smallest k with x < T_k, T_k = floor((1 - (1-r)^(k+1)) 2^32) (Supplementary
 * S2, "Genetics": crossovers at independent boundaries; the gap between
 * crossovers is geometric), over the table the kernel holds -- its entries
 * before the first T_k of 2^32, as 32-bit words -- or the table's length when
 * x reaches every entry.  *gap gets the gap; returns that table length, or
 * -1 for invalid arguments.  The result does not depend on the guess. */
int spegg_geometric_gap(double r, uint32_t n_loci, uint32_t x, uint32_t guess, uint32_t *gap);

/* Host-only: crossover-sampling mode for r (0 raw bits, r = 1/2; 1 none,
 * r = 0; 2 geometric skips, 0 < r < 0.10; 3 bit-serial comparison). */
int spegg_recomb_mode(double r);

/* Device Philox4x32-10 for testing: for i < n, out[4i..4i+3] =
 * Philox(counter ctr[4i..4i+3], key = seed), both arrays in device memory,
 * enqueued on hip_stream; waits for completion. */
spegg_status spegg_philox_fill(uint64_t seed, const uint32_t *ctr_dev, uint32_t *out_dev, uint32_t n,
                               void *hip_stream);

/* Device Philox4x32-10 throughput probe (the same generator the kernels
 * use, with no other memory traffic): for i < n, out_dev[i] = XOR of the
 * four words of the blocks with counters (i, k, 0, 0) under key seed, over
 * k < blocks_per_thread.  out_dev is device memory; enqueued on hip_stream,
 * does not wait.  4 * n * blocks_per_thread words per launch. */
spegg_status spegg_philox_rate(uint64_t seed, uint32_t blocks_per_thread, uint32_t *out_dev, uint32_t n,
                               void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* SPEGG_H */

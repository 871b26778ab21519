// Internal types shared by the host side and the kernels of libspegg.
//
// The kernels work on demes: one patch of one species of one replicate.  A
// replicate of P patches is P consecutive demes sharing its tables; the
// consumer-resource regime has two demes, resource then consumer.
//
// Device memory of a population is one caller-owned block, carved into:
//   [RepDesc x n_demes][RepState x n_demes][SurvTile...][OffTile...][tables]  uploaded once at create
//   [SurvCount...][Partial...][per-deme buffers]                              written by kernels
// Per deme: two genome buffers (ping-pong by generation parity), two
// phenotype buffers, the fates, the survivor list, the slot-owner list
// (Poisson regime) and the parent trace.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "spegg.h"

namespace spegg {

constexpr uint64_t kAlways = 1ull << 32;  // threshold every 32-bit word is below

// Philox counter field c1 = stream << 24 | block.  One stream per kind of
// random decision.
enum Stream : uint32_t {
    kStInit = 1,
    kStSurvive = 3,
    kStFecund = 4,
    kStParent = 5,
    kStRecomb = 6,  // + 0 maternal gamete, + 1 paternal
    kStMutate = 8,  // + 0 maternal gamete, + 1 paternal
    kStMigrate = 10,
    kStEncounter = 11,
    kStCapture = 12,
    kStMutVal = 13,  // continuous alleles: deviate of a mutated locus, + 0 maternal, + 1 paternal
    kStNoise = 15,   // continuous alleles: residual phenotypic noise
    kStSex = 16,     // separate sexes: newborn's sex (block 0), founder's (block 1)
    kStFemale = 17,  // separate sexes: proposals for a mother
    kStMate = 18,    // proposals for a father (sexes, mate choice, monogamy)
    kStResource = 19 // physiology regime: resource growth deviates (index 0, block j)
};

// Proposals for a parent before the fallback rule (the next survivor of the
// wanted sex); the team tests this many in rounds of its lane count.
constexpr uint32_t kPartnerProposals = 4096;

// Crossover sampling, a function of r alone.
enum Mode : uint32_t { kModeRaw = 0, kModeZero = 1, kModeSkip = 2, kModeLazy = 3, kModeMap = 4 };

// Linkage map: per 32-boundary word w of a gamete, kMapWords words at
// map + w kMapWords: [0, 32) the bit planes of the boundaries' thresholds
// R_b = floor(r_b 2^32) (word p: bit 31 - p of each R_b, top bit first),
// [32, 64) after plane p the boundaries whose R_b has a 1 bit below it,
// [64] the boundaries with R_b != 0 (boundary 0 and those past L - 1
// excluded).
constexpr uint32_t kMapWords = 65;

// Geometric gap drawn by word x: the number of thresholds T[0..len) that are
// <= x, i.e. the smallest k with x < T_k, or len when x reaches them all.  T
// holds the entries of the gap table below its first threshold of 2^32 (a
// word is always below that one), as 32-bit words, nondecreasing.  g is a
// first guess in [0, len]; the table alone decides, so any guess gives the
// same result.  constexpr: the offspring kernel and the host test hook run
// this one definition.
constexpr uint32_t geometric_gap_fix(const uint32_t *T, uint32_t len, uint32_t g, uint32_t x) {
    if (g > len) g = len;
    while (g > 0 && T[g - 1] > x) --g;
    while (g < len && T[g] <= x) ++g;
    return g;
}

constexpr double kSkipBelow = 0.10;  // r < 0.10: geometric gaps; above: bit-serial Bernoulli

constexpr int kBlock = 256;          // threads per block in every kernel
// Consecutive adults per thread in survive and compact, chosen per
// population: 1 (one deme) or 4 (several demes); a survival tile holds
// kBlock times that many adults.  Per-adult
// buffers are padded to whole tiles of the largest size.
constexpr int kSurvItemsMax = 4;
constexpr int kSurvTileMax = kBlock * kSurvItemsMax;
constexpr int kPoissonTableCap = 1024;  // longest Poisson threshold table
constexpr int kCensusSlots = 16;     // slots of the census sums (init and write_genomes spread atomics)

struct RepDesc {
    uint32_t L, W, cap, regime;
    uint32_t key0, key1, c3, mode;
    uint32_t R;          // floor(r 2^32), bit-serial mode
    uint32_t geo_len;    // skip mode: gap thresholds kept, those of the L - 1 before the first 2^32
    uint32_t binom_len, pois_len;
    uint64_t binom0;     // binom[0]: a gamete draws no mutation when x < binom0
    int32_t zmin;        // vtab[z - zmin]
    uint32_t zlen;
    int32_t sum_e;       // sum of the effects
    uint32_t unit_effects;
    uint32_t tail_mask;  // valid bits of word W-1
    uint32_t surv_tile0, surv_ntiles;
    uint32_t surv_tile;  // adults per survival tile of the population (kBlock x adults per thread)
    uint32_t grp0, grp_n;  // the deme's tile groups: first record, records per parity (0: one group suffices)
    uint32_t off_tile0, off_ntiles, off_per_tile;  // offspring tiles: global index of the first
    uint32_t off_class, off_list0;  // kernel class of the deme and the start of that class's tile list
    float geo_scale;     // 1 / log2(1 - r): first guess of a geometric gap (checked against geo)
    double K, lambda;    // Beverton-Holt density factor; 0 < K enables it
    uint64_t mig_T;      // a newborn is a migrant when MIGRATE word 0 < mig_T; 0: no migration
    uint32_t patch;      // patch of the deme within its replicate
    uint32_t left, right;  // demes of the ring neighbours (the deme itself without migration)
    uint32_t island;       // biased island dispersal (else the ring)
    uint32_t n_patches, deme0;  // the replicate's patches and the deme of its patch 0
    uint64_t home_T;       // island: a would-be migrant stays home when MIGRATE word 1 < home_T
    uint32_t species;    // consumer-resource regime: 0 resource, 1 consumer
    // consumer-resource regime
    uint32_t partner;    // deme of the other species
    uint32_t habitat;    // encounter slots (0: the resource census)
    uint32_t trials;     // resource offspring trials
    uint32_t enc_len, cap_len;
    double q0, KR;       // resource fecundity: Binomial(trials, q0 max(0, 1 - N_R / KR))
    double surv_age[4];  // survival by age class
    const uint64_t *enc;   // encounters per consumer (Poisson)
    const uint64_t *capT;  // capture threshold by |z_c - z_r|
    const uint64_t *cpois; // consumer offspring tables, Poisson(conversion m), concatenated
    const uint32_t *cpois_off;  // 2 words per intake m: offset into cpois, length
    uint8_t *age[2];     // age class, ping-pong with the genomes
    uint64_t *won;       // resources: lowest capture key this generation, ~0 when not captured
    uint32_t *intake;    // consumers: credited captures of each adult
    uint32_t *genome[2];
    int32_t *z[2];
    uint16_t *fate;      // per adult: bit 15 survived, bits 0..14 offspring as mother
    uint32_t *S;         // survivors, ascending
    uint32_t *owner;     // mother of each offspring slot (Poisson regime)
    uint32_t *mom, *dad; // parent trace
    uint32_t *src;       // parent trace: patch of the parents
    const double *vtab;  // viability by phenotype, NULL: selection off
    const uint64_t *pois, *binom, *geo;
    const uint32_t *planes;  // 4 x W bit-planes of the offset effects e + 4 (bit 0, 1, 2, 3)
    // Continuous alleles: W = L rounded up to a multiple of 4 floats per
    // haplotype (the pad zero); the phenotype buffers hold float bits.
    uint32_t cont;       // 1: continuous allelic values
    uint32_t exp_tf;     // 1: the expressed phenotype is exp(z)
    double theta, omega; // Gaussian viability of the expressed phenotype (omega <= 0: none)
    double a0, s0;       // initial allelic values N(a0, s0^2)
    double mut_sd;       // a mutation adds N(0, mut_sd^2): varpi |a0|
    double noise_sd;     // residual phenotypic noise
    // Mating systems and linkage map
    uint32_t sexes;      // 1: separate sexes, sex[] holds 0 female / 1 male
    uint32_t mating;     // SPEGG_RANDOM_MATING, SPEGG_PREFERENCE, SPEGG_ASSORTATIVE
    uint32_t monogamy;   // 1: a mother's offspring share one father
    uint32_t choice_len; // entries of choiceT (biallelic phenotypes)
    int32_t choice_zmin; // shared preference: choiceT[z - choice_zmin]; assortative: choiceT[|dz|]
    double pref_opt, pref_w;  // mate-choice optimum and width (continuous phenotypes: on the device)
    const uint64_t *choiceT;  // acceptance thresholds floor(a 2^32) (biallelic phenotypes)
    const uint32_t *map;      // linkage map planes, kMapWords per 32-boundary word (kModeMap)
    uint8_t *sex[2];          // separate sexes, ping-pong with the genomes
    // Physiology regime (Supplementary S2); symbols as in spegg_physiology
    double alpha, gamma, delta, attack, handling;
    double KR2[2], growth[2], growth_sd[2];
    double steepness, ulmax;  // ulmax = switch_frac w_max^(1/3), host-computed
    double kappa, qJ, qA, beta1, beta2, beta_s, maturity, v_f, v_m, kappa1, kappa2, kappa3;
    uint32_t breed_every;
    double *X[2], *Y[2];      // irreversible and reversible mass, ping-pong with the genomes
    // Physiology regime: allelic values stay in place for an individual's
    // life.  genome[0] holds them by storage slot; gslot[t & 1][k] is the
    // slot of census position k of generation t; gfree is a stack of the
    // free slots (the dead's, and those never used), recruits pop it.
    uint32_t *gslot[2];
    uint32_t *gfree;
    double *G;                // gonads set aside at this step's growth
    struct PhysTile *ptiles;  // per survival tile: consumption, eggs and the largest weights
};

// Per-deme state.  The census (generation t, size n) is double-buffered:
// the current census is the pair with the larger t (compared modulo 2^32);
// a generation reads it and writes (t + 1, newborns) into the other pair.
struct RepState {
    uint32_t t[2];    // generation of the census
    uint32_t n[2];    // its size
    uint32_t n_prev;  // adults of the last generation
    uint32_t n_surv;  // their survivors
    uint32_t extinct;
    uint32_t traced;          // parents of the current newborns were recorded
    uint32_t census_pending;  // census sums still sit in the offspring tiles' partials
    uint32_t error;           // set by a kernel that found an impossible state (never expected)
    uint32_t captures;        // consumers: credited captures of the last generation
    uint32_t n_carry;         // survivors carried into the current census (consumer-resource regime)
    uint32_t n_surv_f;        // separate sexes: females among the survivors
    double R[2];              // physiology regime: resource densities
    double eggs, emax, xmax;  // physiology regime: eggs of the step, largest eggs and X of the eligible parents
    uint32_t gfree_n[2];      // physiology regime: free slots at the census of generation t, by t & 1
    uint32_t gfree_top;       // physiology regime: free slots after this step's deaths (recruits pop below it)
    uint64_t near_ties, truncated, updates, sum_threshold;
    int64_t sum_z[kCensusSlots];
    uint64_t sum_z2[kCensusSlots];
    double sum_zf[kCensusSlots];   // continuous alleles: sums of the expressed phenotypes
    double sum_zf2[kCensusSlots];
};

struct SurvTile {
    uint32_t rep, start;
};

// Counts of one survival tile; tile 0 of a replicate also records the
// census the generation started from (pair index, t, n), which compact
// reads instead of the state it advances.
struct SurvCount {
    uint32_t alive, kids, near, par;
    uint64_t sum_t;
    uint32_t t, n;
    uint32_t intake;   // consumers: credited captures of the tile's adults
    uint32_t alive_f;  // separate sexes: surviving females
};

// Sums over a group of kGroupTiles consecutive survival tiles of a deme, for
// demes whose census spans more than one group: survive adds each tile's
// counts (atomics, one per nonzero field), compact reads whole groups, so a
// tile's prefix costs at most one load per thread of a group's tiles plus
// one per earlier group.  Double-buffered by the parity of the census
// generation: compact clears the other parity, which the next survive fills.
constexpr uint32_t kGroupTiles = 256;
struct SurvGroup {
    uint64_t kids, sum_t;
    uint32_t alive, near, intake, alive_f;
};

struct OffTile {
    uint32_t rep, start;
};

// Physiology regime, per survival tile: consumption of each resource, eggs
// of the mature surviving females and the largest eggs, largest X of the
// mature surviving males, and their counts.
struct PhysTile {
    double e[2], eggs, emax, xmax;
    uint32_t nf, nm;
};

// Census sums of one offspring tile (continuous alleles: the bits of two
// doubles).
struct Partial {
    int64_t sum_z;
    uint64_t sum_z2;
};

// Offspring-kernel shape for a genome of W words per haplotype: VPL
// consecutive words per lane (16- or 8-byte accesses when W allows), G
// lanes per gamete (a power of two, at most gcap), 2G lanes per newborn; a
// gamete spans nch chunks of G x VPL words, all gathered into registers up
// front when nch <= 4 (nch = 0: more chunks, gathered one at a time).  Any
// shape gives the same results: the random words a newborn consumes do not
// depend on it.
struct OffShape {
    int g, vpl, nch;
    int cont = 0;  // continuous alleles (offspring_cont_kernel; vpl is 4 floats)
    int ext = 0;   // a linkage map or a mating system (the biallelic kernel's extended instance)
};
constexpr int kDefaultGCap = 4;
inline OffShape offspring_shape(uint32_t W, int gcap = kDefaultGCap) {
    OffShape s;
    s.vpl = (W % 4 == 0) ? 4 : (W % 2 == 0) ? 2 : 1;
    const uint32_t per = W / s.vpl;  // lanes of one gamete without chunking
    s.g = 1;
    while ((uint32_t)s.g < per && s.g < gcap) s.g <<= 1;
    const uint32_t chunks = (per + s.g - 1) / s.g;
    if (chunks <= 2) {
        s.nch = chunks <= 1 ? 1 : 2;
    } else if (chunks <= 4) {
        s.nch = 4;
    } else {
        // long genomes: widest team, chunks gathered one at a time
        s.g = 1;
        while ((uint32_t)s.g < per && s.g < 32) s.g <<= 1;
        s.nch = (per + s.g - 1) / s.g <= 1 ? 1 : 0;
    }
    return s;
}
// Continuous alleles: W floats per haplotype (a multiple of 4), 4 per lane
// per chunk, G lanes per gamete (a power of two, at most gcap); a gamete
// spans nch chunks of 4G floats gathered up front (nch <= 4), or any number
// gathered one at a time (nch = 0).  Any shape gives the same results.
constexpr int kDefaultContGCap = 16;
inline OffShape offspring_cont_shape(uint32_t W, int gcap = kDefaultContGCap) {
    OffShape s;
    s.cont = 1;
    s.vpl = 4;
    const uint32_t per = W / 4u;
    s.g = 1;
    while ((uint32_t)s.g < per && s.g < gcap) s.g <<= 1;
    const uint32_t chunks = (per + s.g - 1) / s.g;
    s.nch = chunks <= 1 ? 1 : chunks <= 2 ? 2 : chunks <= 4 ? 4 : 0;
    return s;
}
inline bool same_shape(const OffShape &a, const OffShape &b) {
    return a.g == b.g && a.vpl == b.vpl && a.nch == b.nch && a.cont == b.cont && a.ext == b.ext;
}
// Newborns of one team whose parents' words are gathered before the first
// of them is finished (a latency-hiding knob; results do not depend on it).
constexpr uint32_t kOffspringInFlight = 1;
inline int offspring_per_tile(int g) {
    const int teams = kBlock / (2 * g);
    return (teams >= 16 ? teams : 16) * (int)kOffspringInFlight;
}
inline size_t offspring_lds_bytes(int g, uint32_t W) {
    // per team and gamete: crossover bitmap and flip bitmap, W words each
    return (size_t)(kBlock / (2 * g)) * 2u * 2u * W * sizeof(uint32_t);
}

struct SelArgs {
    const RepDesc *descs;
    RepState *states;
    const SurvTile *tiles;
    SurvCount *counts;
    SurvGroup *groups;
    uint32_t ntiles;
    int trace;
    int single_deme;  // >= 0: the population's only deme, whose tiles are implicit
    int items;        // adults per thread (1 or 4)
    hipStream_t s;
    // non-null: tiles is this generation's list of occupied tiles, list_n
    // its length on the device, walked by grid blocks (survive, compact)
    const uint32_t *list_n = nullptr;
    uint32_t grid_survive = 0, grid_compact = 0;
};

// This generation's lists of occupied tiles (plan_tiles_kernel), in device
// memory: counts[0] survival tiles, [1] encounter tiles, [2 + c] offspring
// tiles of kernel class c, whose list starts at off + the class's first
// tile index (the class's share of the plan's tiles).
struct TileLists {
    SurvTile *surv, *enc;
    OffTile *off;
    uint32_t *counts;
    uint32_t n_classes;
};

struct OffArgs {
    const RepDesc *descs;
    const RepState *states;
    const OffTile *tiles;
    uint32_t tile0, ntiles;
    int single_deme;  // >= 0: the class's only replicate, tiles implicit
    Partial *partials;
    uint32_t plane_words;  // LDS words reserved for the effect planes
    uint32_t geo_words;    // LDS words reserved for the geometric-gap thresholds
    uint32_t mask_words;   // continuous alleles: LDS words of one gamete's crossover (and flip) bitmap
    uint32_t grid;
    size_t lds;
    int trace;
    hipStream_t s;
    const uint32_t *list_n = nullptr;  // non-null: tiles + tile0 is the class's list of occupied tiles
};

// Host-side launchers (kernels.hip).
// The initial population of every deme (genomes, phenotypes, census sums;
// consumer-resource ages and capture keys) over the survival tiles.
hipError_t launch_create(const RepDesc *descs, RepState *states, const SurvTile *tiles, uint32_t ntiles,
                         hipStream_t s);
// Phenotypes and census sums of a deme's n individuals in buffer buf,
// written at generation gen (continuous alleles: founders' noise of gen).
hipError_t launch_phenotypes(const RepDesc *d_desc, RepState *d_state, uint32_t n, uint32_t buf, uint32_t gen,
                             hipStream_t s);
hipError_t launch_survive(const SelArgs &a);
hipError_t launch_compact(const SelArgs &a);
hipError_t launch_offspring(OffShape shape, const OffArgs &a);
// Blocks of the shape's offspring kernel one compute unit holds at once with
// lds bytes of dynamic LDS (HIP's occupancy calculation).
hipError_t offspring_blocks_per_cu(OffShape shape, size_t lds, int *blocks);
// Consumer-resource regime: encounters and captures of the consumers, one
// block per encounter tile (kBlock consumers) of a consumer deme; with
// list_n non-null, tiles is a list of list_n tiles on the device walked by
// grid blocks.
hipError_t launch_encounter(const RepDesc *descs, const RepState *states, const SurvTile *tiles, uint32_t ntiles,
                            const uint32_t *list_n, uint32_t grid, hipStream_t s);
// Consumer-resource regime, after encounter: each captured resource credits
// the consumer whose key it kept (survival tiles of every deme, or a list).
hipError_t launch_credit(const RepDesc *descs, const RepState *states, const SurvTile *tiles, uint32_t ntiles,
                         const uint32_t *list_n, uint32_t grid, hipStream_t s);
// The lists of occupied tiles of phase 0 (before encounter and survive) or
// phase 1 (after compact), one block per deme.
hipError_t launch_plan_tiles(const RepDesc *descs, const RepState *states, uint32_t n_demes, const TileLists &lists,
                             int phase, hipStream_t s);
// Blocks per compute unit of the list-walking kernels (HIP's occupancy
// calculation): kind 0 survive, 1 compact (items adults per thread), 2
// encounter.
hipError_t list_blocks_per_cu(int kind, int items, int *blocks);
// Fill n words of a uint64 array with ~0 (capture keys before the first
// generation) and n bytes with 0 (ages).
hipError_t launch_fill_u64(uint64_t *p, uint32_t n, hipStream_t s);
hipError_t launch_fill_u8(uint8_t *p, uint32_t n, hipStream_t s);
// Clear n 32-bit words (a fill kernel, so it may sit in captured work).
hipError_t launch_fill_u32(uint32_t *p, size_t n, hipStream_t s);
// Fold pending per-tile census sums into each replicate's state.
hipError_t launch_census(const RepDesc *descs, RepState *states, const Partial *partials, uint32_t n_reps,
                         hipStream_t s);

// Set the calling thread's message returned by spegg_last_error.
void set_last_error(const char *msg);

// For the job server.  Bytes of a population's per-deme state; enqueue the
// census fold and a copy of every deme's state into host_states (pinned,
// pop_state_bytes) on the population's stream, without waiting; the
// per-replicate census from such a copy once it has landed; release a
// handle whose enqueued work is known to be complete (no stream wait).
size_t pop_state_bytes(const spegg_pop *pop);
hipError_t pop_census_async(spegg_pop *pop, void *host_states);
spegg_status pop_results(spegg_pop *pop, const void *host_states, spegg_rep_stats *out);
void pop_release_done(spegg_pop *pop);

// Host twin of the kernels' choice of the current census pair.
inline uint32_t current_pair_host(const RepState &st) { return (int32_t)(st.t[1] - st.t[0]) > 0 ? 1u : 0u; }
// Per-locus copies of allele 1 over the current census of n individuals
// into counts (L words, zeroed by the caller).
hipError_t launch_allele_counts(const RepDesc *d_desc, const RepState *d_state, const RepDesc &h, uint32_t n,
                                uint32_t *counts, hipStream_t s);
// The current device's copy of the file-scope allele-count scratch (its
// address, fetched once per device) and its size in words.
hipError_t allele_scratch(uint32_t **out, size_t *words);
hipError_t launch_philox_fill(uint32_t k0, uint32_t k1, const uint32_t *ctr, uint32_t *out, uint32_t n,
                              hipStream_t s);
hipError_t launch_philox_rate(uint32_t k0, uint32_t k1, uint32_t m, uint32_t *out, uint32_t n, hipStream_t s);

}  // namespace spegg

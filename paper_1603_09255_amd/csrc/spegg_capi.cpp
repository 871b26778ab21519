// C ABI of libspegg (include/spegg.h): validation, workspace carving,
// table upload, and the per-generation launch sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "spegg.h"
#include "spegg_internal.h"
#include "tables.h"

using namespace spegg;

namespace {

thread_local std::string g_error;

}  // namespace

void spegg::set_last_error(const char *msg) { g_error = msg; }

namespace {

spegg_status fail(spegg_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return st;
}

constexpr size_t kAlign = 256;
constexpr uint32_t kMaxOffspringGrid = 1u << 18;  // blocks of one offspring launch of several demes (they loop over tiles)
constexpr uint32_t kListGridFactor = 8;  // resident grids' worth of blocks of a launch that walks a tile list

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct Carver {
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes);
        return at;
    }
};

// Everything the host derives from one descriptor, and its shared tables.
struct RepPlan {
    uint32_t W = 0, mode = 0, R = 0, opt = 0;
    bool cont = false;  // continuous alleles: W floats per haplotype
    bool ext = false;   // a linkage map or a mating system (the biallelic kernel's extended instance)
    bool phys = false;  // physiology regime: masses, carried survivors, separate sexes
    std::vector<uint32_t> map;      // linkage map planes (kModeMap)
    std::vector<uint64_t> choiceT;  // mate-choice thresholds over integer phenotypes
    int32_t choice_zmin = 0;
    size_t map_at = 0, choiceT_at = 0;
    OffShape shape{1, 1, 1};
    int32_t zmin = 0, sum_e = 0;
    uint32_t zlen = 0;
    bool unit = true;
    uint64_t mig_T = 0;
    std::vector<uint64_t> pois, binom, geo;
    std::vector<double> vtab;
    std::vector<uint32_t> planes;
    size_t vtab_at = 0, pois_at = 0, binom_at = 0, geo_at = 0, planes_at = 0;
    uint32_t deme0 = 0, n_demes = 0;  // the replicate's demes are deme0 .. deme0 + n_demes - 1
    // consumer-resource regime
    bool cr = false;
    std::vector<uint64_t> enc, capT, cpois;
    std::vector<uint32_t> cpois_off;  // (offset, length) per intake
    size_t enc_at = 0, capT_at = 0, cpois_at = 0, cpois_off_at = 0;
};

// One patch of one species of one replicate: its tiles and buffers.
struct DemePlan {
    uint32_t rep = 0, patch = 0, species = 0;
    uint32_t n0 = 0, cap = 0;
    uint32_t surv_tile0 = 0, surv_ntiles = 0, off_tile0 = 0, off_ntiles = 0;
    uint32_t off_class = 0;  // index of the deme's offspring-kernel class
    uint32_t grp0 = 0, grp_n = 0;  // tile-group sums (two parities of grp_n records)
    size_t genome[2] = {0, 0}, z[2] = {0, 0}, fate = 0, S = 0, owner = 0, mom = 0, dad = 0, src = 0, sex[2] = {0, 0};
    size_t age[2] = {0, 0}, won = 0, intake = 0;
    size_t X[2] = {0, 0}, Y[2] = {0, 0}, G = 0, ptiles = 0;  // physiology regime
    size_t gslot[2] = {0, 0}, gfree = 0;                      // physiology regime: genome slots
};

// Demes sharing one offspring-kernel shape.
struct OffClass {
    OffShape shape;
    uint32_t tile0, ntiles, grid;
    int single_deme;       // the class's only deme, or -1
    uint32_t plane_words;  // LDS words for the effect planes (0: unit effects only)
    uint32_t geo_words;    // LDS words for the geometric-gap thresholds (0: no skip-mode member)
    uint32_t mask_words;   // continuous alleles: LDS words of one gamete's bitmaps
    size_t lds;
};

// Key of a genome's offspring-shape cap: the words per haplotype, with the
// top bit set for continuous alleles (their shapes are of another kernel).
constexpr uint32_t kContKey = 0x80000000u;
uint32_t shape_key(const RepPlan &p) { return p.cont ? (p.W | kContKey) : p.W; }
OffShape shape_of_key(uint32_t key, int gcap) {
    return (key & kContKey) ? offspring_cont_shape(key & ~kContKey, gcap) : offspring_shape(key, gcap);
}

// Lanes-per-gamete cap by genome length W (the autotuner's choice); a W
// missing from the map takes the default.
using GcapMap = std::map<uint32_t, int>;

struct Plan {
    std::vector<RepPlan> reps;
    std::vector<DemePlan> demes;
    std::vector<OffClass> classes;
    std::vector<SurvTile> surv_tiles;
    std::vector<SurvTile> enc_tiles;    // encounter tiles of consumer demes (kBlock consumers each)
    std::vector<OffTile> off_tiles;
    size_t descs = 0, states = 0, surv_tiles_at = 0, off_tiles_at = 0, enc_tiles_at = 0;
    size_t static_end = 0;  // [0, static_end) is uploaded at create
    size_t surv_counts = 0, surv_groups = 0, partials = 0, total = 0;
    uint32_t n_groups = 0;  // tile-group records, both parities
    uint32_t surv_items = 1;  // adults per thread in survive and compact
    // Lists of each generation's occupied tiles, walked by resident grids
    // (populations of several demes whose censuses can fall below their
    // capacities): their counts (3 + one per possible class) and arrays.
    bool listed = false;
    size_t list_counts_at = 0, list_surv_at = 0, list_enc_at = 0, list_off_at = 0;
    uint32_t list_counts = 0;
    uint32_t grid_survive = 0, grid_compact = 0, grid_encounter = 0;
};

// Resident grids per list-walking launch (a tuning knob: results do not
// depend on it); SPEGG_LIST_GRID_FACTOR overrides.
uint32_t list_grid_factor() {
    const char *e = std::getenv("SPEGG_LIST_GRID_FACTOR");
    if (e) {
        const long v = std::atol(e);
        if (v >= 1 && v <= 64) return (uint32_t)v;
    }
    return kListGridFactor;
}

// Tile lists or one block per tile of the capacity: SPEGG_TILE_LISTS=0 or 1
// forces the choice (results do not depend on it), else lists wherever a
// population of several demes has one whose census can fall below its
// capacity (any regime but Wright-Fisher at full capacity).
bool want_tile_lists(const Plan &P, const spegg_rep_desc *reps) {
    const char *e = std::getenv("SPEGG_TILE_LISTS");
    if (e && (e[0] == '0' || e[0] == '1') && e[1] == 0) return e[0] == '1';
    if (P.demes.size() < 2) return false;
    for (const DemePlan &q : P.demes)
        if (reps[q.rep].regime != SPEGG_WF || q.cap > q.n0) return true;
    return false;
}

// Most blocks of one offspring launch; SPEGG_OFFSPRING_GRID overrides.
uint32_t offspring_grid_cap() {
    const char *e = std::getenv("SPEGG_OFFSPRING_GRID");
    if (e) {
        const long v = std::atol(e);
        if (v >= 64 && v <= (1 << 20)) return (uint32_t)v;
    }
    return kMaxOffspringGrid;
}

// Offspring grids of one-deme classes: as many blocks as the device's compute
// units hold at once (each block loops over tiles), so no tile waits for a
// second dispatch behind blocks that find no work.  Classes of several demes
// keep the larger grid: their tiles carry uneven work (censuses, crossover
// modes), which the dispatcher balances block by block.  SPEGG_OFFSPRING_GRID,
// when set, keeps the grids make_plan gave.
hipError_t fit_offspring_grids(Plan &P, int device) {
    int cus = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return e;
    if (cus <= 0) cus = 1;
    const uint32_t factor = list_grid_factor();
    if (P.listed) {
        // the list-walking launches: a few resident grids' worth of blocks
        const auto fit = [&](int kind, uint32_t ntiles, uint32_t *grid) {
            int per = 0;
            const hipError_t r = list_blocks_per_cu(kind, (int)P.surv_items, &per);
            const uint64_t g = (uint64_t)(per > 0 ? per : 1) * (uint64_t)cus * factor;
            *grid = ntiles == 0 ? 0u : ntiles < g ? ntiles : (uint32_t)g;
            return r;
        };
        const uint32_t ns = (uint32_t)P.surv_tiles.size();
        if ((e = fit(0, ns, &P.grid_survive)) != hipSuccess) return e;
        if ((e = fit(1, ns, &P.grid_compact)) != hipSuccess) return e;
        if ((e = fit(2, (uint32_t)P.enc_tiles.size(), &P.grid_encounter)) != hipSuccess) return e;
    }
    if (std::getenv("SPEGG_OFFSPRING_GRID")) return hipSuccess;
    for (OffClass &c : P.classes) {
        if (c.single_deme < 0 && !P.listed) continue;
        int per = 0;
        if ((e = offspring_blocks_per_cu(c.shape, c.lds, &per)) != hipSuccess) return e;
        const uint64_t resident = (uint64_t)(per > 0 ? per : 1) * (uint64_t)cus * (c.single_deme < 0 ? factor : 1u);
        c.grid = c.ntiles < resident ? c.ntiles : (uint32_t)resident;
    }
    return hipSuccess;
}

// The device's LDS per block against every offspring class's need (effect
// planes, gap and fecundity tables, per-team bitmaps).
hipError_t offspring_lds_limit(int device, size_t *limit) {
    int v = 0;
    const hipError_t e = hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    *limit = e == hipSuccess && v > 0 ? (size_t)v : 0;
    return e;
}

// Default lanes-per-gamete cap of the offspring kernel for a genome of W
// words (a tuning choice only: results do not depend on it).  Up to 16
// lanes' worth of words per chunk, the shape whose gamete spans two register
// chunks -- the autotuner's pick wherever it was measured (L = 64, 256,
// 1024); longer genomes keep a cap of 4 (the chunk-loop shapes).
// SPEGG_OFFSPRING_GCAP overrides for every W.
int offspring_gcap(uint32_t W) {
    const char *e = std::getenv("SPEGG_OFFSPRING_GCAP");
    if (e) {
        const int v = std::atoi(e);
        if (v == 1 || v == 2 || v == 4 || v == 8 || v == 16 || v == 32) return v;
    }
    const uint32_t vpl = W % 4 == 0 ? 4u : W % 2 == 0 ? 2u : 1u;
    const uint32_t per = W / vpl;  // lanes of a gamete in one chunk
    if (per > 16) return kDefaultGCap;
    int g = 1;
    while ((uint32_t)(2 * g) <= per / 2) g *= 2;
    return g;
}

spegg_status validate(const spegg_rep_desc &d, uint32_t i) {
    if (d.n_loci < 1 || d.n_loci > SPEGG_MAX_LOCI)
        return fail(SPEGG_E_INVALID, "replicate %u: n_loci %u outside 1..%u", i, d.n_loci, SPEGG_MAX_LOCI);
    if (d.capacity < 1 || d.capacity > (1u << 30))
        return fail(SPEGG_E_INVALID, "replicate %u: capacity %u outside 1..2^30", i, d.capacity);
    if (d.n0 > d.capacity) return fail(SPEGG_E_INVALID, "replicate %u: n0 %u exceeds capacity %u", i, d.n0, d.capacity);
    if (d.replicate_id > SPEGG_MAX_REPLICATE_ID)
        return fail(SPEGG_E_INVALID, "replicate %u: replicate_id %u exceeds %u", i, d.replicate_id,
                    SPEGG_MAX_REPLICATE_ID);
    if (d.regime != SPEGG_WF && d.regime != SPEGG_POISSON_BH && d.regime != SPEGG_CONSUMER_RESOURCE &&
        d.regime != SPEGG_PHYSIOLOGY)
        return fail(SPEGG_E_INVALID, "replicate %u: unknown regime %u", i, d.regime);
    if (d.regime == SPEGG_PHYSIOLOGY) {
        const spegg_physiology *F = d.physiology;
        if (!F) return fail(SPEGG_E_INVALID, "replicate %u: the physiology regime needs its parameters", i);
        if (d.genetics != SPEGG_CONTINUOUS || d.exp_transform != 1)
            return fail(SPEGG_E_INVALID, "replicate %u: the physiology regime's trait is exp(z) of continuous alleles",
                        i);
        if (d.n_patches != 1 || d.mating != SPEGG_RANDOM_MATING || d.monogamy)
            return fail(SPEGG_E_UNSUPPORTED, "replicate %u: the physiology regime has one patch and its own mating", i);
        bool ok = F->alpha > 0.0 && F->gamma > 0.0 && F->gamma <= 1.0 && F->delta >= 0.0 && F->attack >= 0.0 &&
                  F->handling >= 0.0 && F->w_max > 0.0 && F->kappa >= 0.0 && F->qJ > 0.0 && F->qA >= 0.0 &&
                  F->maturity > 0.0 && F->v_f >= 0.0 && F->v_m >= 0.0 && F->kappa1 >= 0.0 && F->kappa2 > 0.0 &&
                  F->kappa3 >= 0.0 && F->breed_every >= 1 && std::isfinite(F->steepness) &&
                  std::isfinite(F->switch_frac) && std::isfinite(F->beta1) && std::isfinite(F->beta2) &&
                  F->beta_s >= 0.0 && std::isfinite(F->alpha) && std::isfinite(F->kappa1);
        for (int j = 0; j < 2; ++j)
            ok = ok && F->K[j] > 0.0 && F->R0[j] >= 0.0 && std::isfinite(F->growth[j]) && F->growth_sd[j] >= 0.0 &&
                 std::isfinite(F->R0[j]) && std::isfinite(F->growth_sd[j]);
        if (!ok) return fail(SPEGG_E_INVALID, "replicate %u: physiology parameters out of range", i);
    } else if (d.physiology) {
        return fail(SPEGG_E_INVALID, "replicate %u: physiology given for another regime", i);
    }
    if (d.n_patches < 1 || d.n_patches > SPEGG_MAX_PATCHES)
        return fail(SPEGG_E_INVALID, "replicate %u: n_patches %u outside 1..%u", i, d.n_patches, SPEGG_MAX_PATCHES);
    if (d.n_patches > 1 && d.regime != SPEGG_WF)
        return fail(SPEGG_E_UNSUPPORTED, "replicate %u: patches need the Wright-Fisher regime", i);
    if (d.regime == SPEGG_CONSUMER_RESOURCE) {
        const spegg_ecology *e = d.ecology;
        if (!e) return fail(SPEGG_E_INVALID, "replicate %u: the consumer-resource regime needs an ecology", i);
        if (e->capacity_consumer < 1 || e->capacity_consumer > (1u << 30) || e->n0_consumer > e->capacity_consumer)
            return fail(SPEGG_E_INVALID, "replicate %u: consumer census %u / capacity %u", i, e->n0_consumer,
                        e->capacity_consumer);
        if (e->resource_trials < 1 || e->resource_trials > 64)
            return fail(SPEGG_E_INVALID, "replicate %u: resource_trials %u outside 1..64", i, e->resource_trials);
        if (!(e->attack >= 0.0 && e->attack <= 1.0) || !(e->match_width > 0.0) || !(e->encounters >= 0.0) ||
            !(e->conversion >= 0.0) || !(e->resource_q0 >= 0.0 && e->resource_q0 <= 1.0) ||
            !(e->resource_K > 0.0) || !std::isfinite(e->encounters) || !std::isfinite(e->conversion) ||
            !std::isfinite(e->resource_K) || !std::isfinite(e->match_width))
            return fail(SPEGG_E_INVALID, "replicate %u: ecology rates out of range", i);
        for (int a = 0; a < 4; ++a)
            if (!(e->surv_resource[a] >= 0.0 && e->surv_resource[a] <= 1.0) ||
                !(e->surv_consumer[a] >= 0.0 && e->surv_consumer[a] <= 1.0))
                return fail(SPEGG_E_INVALID, "replicate %u: survival of age class %d outside [0, 1]", i, a);
        if (d.n_patches != 1) return fail(SPEGG_E_UNSUPPORTED, "replicate %u: the consumer-resource regime has one patch", i);
    } else if (d.ecology) {
        return fail(SPEGG_E_INVALID, "replicate %u: ecology given for a one-species regime", i);
    }
    if (!(d.migration >= 0.0 && d.migration <= 1.0))
        return fail(SPEGG_E_INVALID, "replicate %u: migration %g outside [0, 1]", i, d.migration);
    if (d.dispersal != SPEGG_RING && d.dispersal != SPEGG_ISLAND)
        return fail(SPEGG_E_INVALID, "replicate %u: unknown dispersal %u", i, d.dispersal);
    if (!(d.home_return >= 0.0 && d.home_return <= 1.0))
        return fail(SPEGG_E_INVALID, "replicate %u: home_return %g outside [0, 1]", i, d.home_return);
    if (!(d.mu >= 0.0 && d.mu < 1.0)) return fail(SPEGG_E_INVALID, "replicate %u: mu %g outside [0, 1)", i, d.mu);
    if (!(d.r >= 0.0 && d.r <= 0.5)) return fail(SPEGG_E_INVALID, "replicate %u: r %g outside [0, 1/2]", i, d.r);
    if (!std::isfinite(d.theta) || std::isnan(d.omega))
        return fail(SPEGG_E_INVALID, "replicate %u: theta and omega must be numbers", i);
    if (d.regime == SPEGG_POISSON_BH) {
        if (!(d.fecundity >= 0.0) || !std::isfinite(d.fecundity))
            return fail(SPEGG_E_INVALID, "replicate %u: fecundity %g must be >= 0", i, d.fecundity);
        if (std::isnan(d.K) || std::isinf(d.K)) return fail(SPEGG_E_INVALID, "replicate %u: K must be finite", i);
    }
    if (d.effects)
        for (uint32_t l = 0; l < d.n_loci; ++l)
            if (d.effects[l] < -4 || d.effects[l] > 4)
                return fail(SPEGG_E_INVALID, "replicate %u: effect %d at locus %u outside [-4, 4]", i, d.effects[l], l);
    if (d.genetics != SPEGG_BIALLELIC && d.genetics != SPEGG_CONTINUOUS)
        return fail(SPEGG_E_INVALID, "replicate %u: unknown genetics %u", i, d.genetics);
    if (d.genetics == SPEGG_CONTINUOUS) {
        if (d.regime == SPEGG_CONSUMER_RESOURCE)
            return fail(SPEGG_E_UNSUPPORTED, "replicate %u: continuous alleles with the consumer-resource regime", i);
        if (d.effects)
            return fail(SPEGG_E_INVALID, "replicate %u: continuous alleles carry their own effects (effects must be NULL)",
                        i);
        if (!std::isfinite(d.allele_mean) || !(d.allele_sd >= 0.0) || !std::isfinite(d.allele_sd) ||
            !(d.mut_sd_factor >= 0.0) || !std::isfinite(d.mut_sd_factor) || !(d.noise_sd >= 0.0) ||
            !std::isfinite(d.noise_sd) || d.exp_transform > 1)
            return fail(SPEGG_E_INVALID, "replicate %u: continuous-allele parameters out of range", i);
    }
    if (d.linkage)
        for (uint32_t l = 0; l + 1 < d.n_loci; ++l)
            if (!(d.linkage[l] >= 0.0 && d.linkage[l] <= 0.5))
                return fail(SPEGG_E_INVALID, "replicate %u: linkage rate %g at boundary %u outside [0, 1/2]", i,
                            d.linkage[l], l + 1);
    if (d.sexes > 1 || d.monogamy > 1 || d.mating > SPEGG_ASSORTATIVE)
        return fail(SPEGG_E_INVALID, "replicate %u: unknown sexes / mating / monogamy setting", i);
    if (d.mating != SPEGG_RANDOM_MATING &&
        !(d.pref_width > 0.0 && std::isfinite(d.pref_width) && std::isfinite(d.pref_optimum)))
        return fail(SPEGG_E_INVALID, "replicate %u: mate choice needs a finite pref_width > 0", i);
    if ((d.sexes || d.mating || d.monogamy) && (d.n_patches != 1 || d.regime == SPEGG_CONSUMER_RESOURCE))
        return fail(SPEGG_E_UNSUPPORTED, "replicate %u: mating systems need one patch of a one-species regime", i);
    return SPEGG_OK;
}

spegg_status build_rep(const spegg_rep_desc &d, uint32_t i, RepPlan &p, const GcapMap *gcaps) {
    spegg_status st = validate(d, i);
    if (st != SPEGG_OK) return st;
    const uint32_t L = d.n_loci;
    p.cont = d.genetics == SPEGG_CONTINUOUS;
    p.W = p.cont ? (L + 3u) / 4u * 4u : (L + 31u) / 32u;
    p.mode = recomb_mode(d.r);
    p.R = (uint32_t)std::floor(d.r * 4294967296.0);
    p.ext = d.linkage || d.sexes || d.mating || d.monogamy;
    p.phys = d.regime == SPEGG_PHYSIOLOGY;
    if (d.linkage) {
        p.mode = kModeMap;
        linkage_planes(d.linkage, L, p.map);
    }
    p.mig_T = d.n_patches > 1 ? prob_threshold(d.migration) : 0;
    int32_t abs_sum = 0;
    p.sum_e = 0;
    p.unit = true;
    for (uint32_t l = 0; l < L; ++l) {
        const int e = d.effects ? d.effects[l] : 1;
        abs_sum += e < 0 ? -e : e;
        p.sum_e += e;
        if (e != 1) p.unit = false;
    }
    p.zmin = -abs_sum;
    p.zlen = 2u * (uint32_t)abs_sum + 1u;
    // continuous phenotypes take their viability on the device
    if (d.omega > 0.0 && !p.cont) viability_table(d.theta, d.omega, p.zmin, p.zlen, p.vtab);
    if (!p.unit) {
        // bit-planes of the offset effects e + 4 in [0, 8]
        p.planes.assign(4u * p.W, 0u);
        for (uint32_t l = 0; l < L; ++l) {
            const uint32_t m = (uint32_t)(d.effects[l] + 4), bit = 1u << (l % 32u), w = l / 32u;
            for (uint32_t k = 0; k < 4; ++k)
                if (m & (1u << k)) p.planes[k * p.W + w] |= bit;
        }
    }
    if (!binomial_table(L, d.mu, (int)L + 1, p.binom))
        return fail(SPEGG_E_UNSUPPORTED, "replicate %u: mutation-count table does not close", i);
    if (d.regime == SPEGG_POISSON_BH && !poisson_table(d.fecundity, kPoissonTableCap, p.pois))
        return fail(SPEGG_E_UNSUPPORTED, "replicate %u: fecundity %g needs more than %d table entries", i,
                    d.fecundity, kPoissonTableCap);
    if (d.mating != SPEGG_RANDOM_MATING && !p.cont) {
        // integer phenotypes: acceptance by phenotype (shared preference) or
        // by phenotype distance (assortment), both over the range of z
        p.choice_zmin = p.zmin;
        choice_table(d.mating == SPEGG_PREFERENCE, d.pref_optimum, d.pref_width, p.zmin, p.zlen, p.choiceT);
    }
    if (p.mode == kModeSkip && L > 1) {
        // the kernel keeps the gap table up to its first threshold of 2^32
        geometric_table(d.r, L - 1u, p.geo);
        p.geo.resize(geometric_device_len(p.geo));
    }
    int gcap = p.cont ? kDefaultContGCap : offspring_gcap(p.W);
    if (gcaps) {
        const auto it = gcaps->find(shape_key(p));
        if (it != gcaps->end()) gcap = it->second;
    }
    p.shape = shape_of_key(shape_key(p), gcap);
    p.shape.ext = p.ext && !p.cont ? 1 : 0;  // the continuous kernel carries these paths itself
    p.opt = (uint32_t)offspring_per_tile(p.shape.g);
    p.n_demes = d.n_patches;
    if (d.regime == SPEGG_CONSUMER_RESOURCE) {
        const spegg_ecology &e = *d.ecology;
        p.cr = true;
        p.n_demes = 2;
        if (!poisson_table(e.encounters, kPoissonTableCap, p.enc))
            return fail(SPEGG_E_UNSUPPORTED, "replicate %u: encounters %g need more than %d table entries", i,
                        e.encounters, kPoissonTableCap);
        capture_table(e.attack, e.match_width, 2u * (uint32_t)abs_sum + 1u, p.capT);
        // intake never exceeds the encounters: at most enc.size() - 1
        for (size_t m = 0; m < p.enc.size(); ++m) {
            std::vector<uint64_t> T;
            if (!poisson_table(e.conversion * (double)m, kPoissonTableCap, T))
                return fail(SPEGG_E_UNSUPPORTED, "replicate %u: consumer fecundity %g needs more than %d entries", i,
                            e.conversion * (double)m, kPoissonTableCap);
            p.cpois_off.push_back((uint32_t)p.cpois.size());
            p.cpois_off.push_back((uint32_t)T.size());
            p.cpois.insert(p.cpois.end(), T.begin(), T.end());
        }
    }
    return SPEGG_OK;
}

spegg_status make_plan(const spegg_rep_desc *reps, uint32_t n, Plan &P, const GcapMap *gcaps = nullptr,
                       int listed = -1) {
    if (!reps || n == 0) return fail(SPEGG_E_INVALID, "no replicates");
    P.reps.resize(n);
    uint64_t n_demes = 0;
    for (uint32_t i = 0; i < n; ++i) {
        const spegg_status st = build_rep(reps[i], i, P.reps[i], gcaps);
        if (st != SPEGG_OK) return st;
        P.reps[i].deme0 = (uint32_t)n_demes;
        n_demes += P.reps[i].n_demes;
    }
    if (n_demes > (1u << 24)) return fail(SPEGG_E_INVALID, "%llu patches in total exceed 2^24",
                                          (unsigned long long)n_demes);
    P.demes.resize(n_demes);
    for (uint32_t i = 0; i < n; ++i)
        for (uint32_t k = 0; k < P.reps[i].n_demes; ++k) {
            DemePlan &q = P.demes[P.reps[i].deme0 + k];
            q.rep = i;
            const bool consumer = P.reps[i].cr && k == 1;
            q.patch = P.reps[i].cr ? 0u : k;
            q.species = P.reps[i].cr ? k : 0u;
            q.n0 = consumer ? reps[i].ecology->n0_consumer : reps[i].n0;
            q.cap = consumer ? reps[i].ecology->capacity_consumer : reps[i].capacity;
        }
    // survival tiles, deme by deme: four adults per thread where the
    // population has several demes (fewer, longer blocks, the per-tile sums
    // shared by more adults; measured faster on the batched table, the
    // physiology batch and the consumer-resource replicates), else one (more
    // blocks in flight for one deme)
    P.surv_items = P.demes.size() > 1 ? (uint32_t)kSurvItemsMax : 1u;
    // SPEGG_SURV_ITEMS=1 forces one adult per thread (an experiment knob: no
    // result depends on it)
    const char *items = std::getenv("SPEGG_SURV_ITEMS");
    if (items && items[0] == '1' && items[1] == 0) P.surv_items = 1u;
    const uint32_t surv_tile = kBlock * P.surv_items;
    for (uint32_t u = 0; u < P.demes.size(); ++u) {
        DemePlan &q = P.demes[u];
        q.surv_tile0 = (uint32_t)P.surv_tiles.size();
        q.surv_ntiles = (q.cap + surv_tile - 1) / surv_tile;
        q.grp0 = P.n_groups;
        q.grp_n = q.surv_ntiles > kGroupTiles ? (q.surv_ntiles + kGroupTiles - 1) / kGroupTiles : 0u;
        P.n_groups += 2u * q.grp_n;
        for (uint32_t k = 0; k < q.surv_ntiles; ++k) P.surv_tiles.push_back(SurvTile{u, k * surv_tile});
        // consumers: encounter tiles of kBlock consumers, one per thread
        if (P.reps[q.rep].cr && q.species == 1)
            for (uint32_t k = 0; k < (q.cap + kBlock - 1u) / kBlock; ++k)
                P.enc_tiles.push_back(SurvTile{u, k * (uint32_t)kBlock});
    }
    // offspring tiles grouped by kernel shape
    std::vector<OffShape> shapes;
    for (uint32_t i = 0; i < n; ++i) {
        const OffShape sh = P.reps[i].shape;
        bool seen = false;
        for (const OffShape &x : shapes) seen |= same_shape(x, sh);
        if (!seen) shapes.push_back(sh);
    }
    for (const OffShape &sh : shapes) {
        OffClass c{sh, (uint32_t)P.off_tiles.size(), 0, 0, -1, 0, 0, 0, 0};
        uint32_t maxW = 0, members = 0, last = 0, maxgeo = 0, maxWb = 0;
        bool planes = false;
        for (uint32_t u = 0; u < P.demes.size(); ++u) {
            DemePlan &q = P.demes[u];
            const RepPlan &p = P.reps[q.rep];
            if (!same_shape(p.shape, sh)) continue;
            q.off_tile0 = (uint32_t)P.off_tiles.size();
            q.off_ntiles = (q.cap + p.opt - 1) / p.opt;
            q.off_class = (uint32_t)P.classes.size();
            for (uint32_t k = 0; k < q.off_ntiles; ++k) P.off_tiles.push_back({u, k * p.opt});
            if (p.W > maxW) maxW = p.W;
            const uint32_t Wb = (reps[q.rep].n_loci + 31u) / 32u;
            if (Wb > maxWb) maxWb = Wb;
            if (p.geo.size() > maxgeo) maxgeo = (uint32_t)p.geo.size();
            planes |= !p.unit;
            ++members;
            last = u;
        }
        c.ntiles = (uint32_t)P.off_tiles.size() - c.tile0;
        c.single_deme = members == 1 ? (int)last : -1;
        const uint32_t gmax = offspring_grid_cap();  // a tuning knob: results do not depend on it
        c.grid = c.ntiles < gmax ? c.ntiles : gmax;
        c.plane_words = planes ? 4u * maxW : 0u;
        c.geo_words = maxgeo;
        // continuous alleles: a crossover and a flip bitmap of one bit per
        // locus per team and gamete (the biallelic formula over bitmap words)
        c.mask_words = sh.cont ? maxWb : 0u;
        c.lds = (c.plane_words + c.geo_words) * sizeof(uint32_t) +
                offspring_lds_bytes(sh.g, sh.cont ? c.mask_words : maxW);
        P.classes.push_back(c);
    }
    Carver cv;
    P.descs = cv.take(sizeof(RepDesc) * P.demes.size());
    P.states = cv.take(sizeof(RepState) * P.demes.size());
    P.surv_tiles_at = cv.take(sizeof(SurvTile) * P.surv_tiles.size());
    P.enc_tiles_at = cv.take(sizeof(SurvTile) * P.enc_tiles.size());
    // offspring tiles and their partials are carved for the smallest tile of
    // any shape (16 newborns), so a change of shape moves no buffer
    size_t max_off_tiles = 0;
    for (const DemePlan &q : P.demes) max_off_tiles += (q.cap + 15u) / 16u;
    P.off_tiles_at = cv.take(sizeof(OffTile) * max_off_tiles);
    for (uint32_t i = 0; i < n; ++i) {
        RepPlan &p = P.reps[i];
        if (!p.vtab.empty()) p.vtab_at = cv.take(sizeof(double) * p.vtab.size());
        if (!p.pois.empty()) p.pois_at = cv.take(sizeof(uint64_t) * p.pois.size());
        p.binom_at = cv.take(sizeof(uint64_t) * p.binom.size());
        if (!p.geo.empty()) p.geo_at = cv.take(sizeof(uint64_t) * p.geo.size());
        if (!p.planes.empty()) p.planes_at = cv.take(sizeof(uint32_t) * p.planes.size());
        if (!p.map.empty()) p.map_at = cv.take(sizeof(uint32_t) * p.map.size());
        if (!p.choiceT.empty()) p.choiceT_at = cv.take(sizeof(uint64_t) * p.choiceT.size());
        if (p.cr) {
            p.enc_at = cv.take(sizeof(uint64_t) * p.enc.size());
            p.capT_at = cv.take(sizeof(uint64_t) * p.capT.size());
            p.cpois_at = cv.take(sizeof(uint64_t) * p.cpois.size());
            p.cpois_off_at = cv.take(sizeof(uint32_t) * p.cpois_off.size());
        }
    }
    P.static_end = cv.off;
    P.surv_counts = cv.take(sizeof(SurvCount) * P.surv_tiles.size());
    P.surv_groups = cv.take(sizeof(SurvGroup) * (P.n_groups ? P.n_groups : 1u));
    P.partials = cv.take(sizeof(Partial) * max_off_tiles);
    P.listed = listed < 0 ? want_tile_lists(P, reps) : listed != 0;
    if (P.listed) {
        // room for one class per deme, whatever shapes a re-plan picks
        P.list_counts = 2u + (uint32_t)P.demes.size();
        P.list_counts_at = cv.take(sizeof(uint32_t) * P.list_counts);
        P.list_surv_at = cv.take(sizeof(SurvTile) * P.surv_tiles.size());
        P.list_enc_at = cv.take(sizeof(SurvTile) * P.enc_tiles.size());
        P.list_off_at = cv.take(sizeof(OffTile) * max_off_tiles);
    }
    for (DemePlan &q : P.demes) {
        const RepPlan &p = P.reps[q.rep];
        const size_t cap = q.cap;
        const size_t gbytes = cap * 2u * p.W * sizeof(uint32_t);
        q.genome[0] = cv.take(gbytes);
        q.genome[1] = cv.take(gbytes);
        // phenotypes padded to whole select tiles (read as vectors)
        const size_t zcap = ((cap + kSurvTileMax - 1) / kSurvTileMax) * kSurvTileMax;
        q.z[0] = cv.take(zcap * sizeof(int32_t));
        q.z[1] = cv.take(zcap * sizeof(int32_t));
        q.fate = cv.take(zcap * sizeof(uint16_t));
        q.S = cv.take(cap * sizeof(uint32_t));
        if (reps[q.rep].regime != SPEGG_WF) q.owner = cv.take(cap * sizeof(uint32_t));
        q.mom = cv.take(cap * sizeof(uint32_t));
        q.dad = cv.take(cap * sizeof(uint32_t));
        if (p.mig_T) q.src = cv.take(cap * sizeof(uint32_t));
        if (reps[q.rep].sexes || p.phys) {
            q.sex[0] = cv.take(zcap);  // padded to whole tiles: read 4 at a time
            q.sex[1] = cv.take(zcap);
        }
        if (p.phys) {
            q.X[0] = cv.take(cap * sizeof(double));
            q.X[1] = cv.take(cap * sizeof(double));
            q.Y[0] = cv.take(cap * sizeof(double));
            q.Y[1] = cv.take(cap * sizeof(double));
            q.G = cv.take(cap * sizeof(double));
            q.ptiles = cv.take(q.surv_ntiles * sizeof(PhysTile));
            q.gslot[0] = cv.take(cap * sizeof(uint32_t));
            q.gslot[1] = cv.take(cap * sizeof(uint32_t));
            q.gfree = cv.take(cap * sizeof(uint32_t));
        }
        if (p.cr) {
            q.age[0] = cv.take(zcap);  // padded to whole tiles: read 4 at a time
            q.age[1] = cv.take(zcap);
            if (q.species == 0) q.won = cv.take(cap * sizeof(uint64_t));
            else q.intake = cv.take(cap * sizeof(uint32_t));
        }
    }
    P.total = cv.off;
    return SPEGG_OK;
}

template <typename T>
T *at(uint8_t *base, size_t off) {
    return reinterpret_cast<T *>(base + off);
}

struct Timed {
    int kind;
    int cls;  // offspring launches: the class (kernel shape) index; else -1
    hipEvent_t a, b;
};

// An instantiated graph of a fixed number of generations.
struct GenGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void release() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
};

constexpr uint32_t kGraphGenerations = 16;  // generations per replay of the long graph
constexpr int kAutotuneRounds = 2;          // interleaved timing rounds over the shapes

struct DeviceGuard {
    int prev = -1;
    bool changed = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
            changed = hipSetDevice(dev) == hipSuccess;
        }
    }
    ~DeviceGuard() {
        if (changed) (void)hipSetDevice(prev);
    }
};

}  // namespace

struct spegg_pop {
    hipStream_t stream = nullptr;
    int device = 0;
    uint8_t *base = nullptr;
    uint32_t n_reps = 0, n_demes = 0;
    Plan plan;
    std::vector<spegg_rep_desc> descs;           // the caller's descriptors, pointing at the copies below
    std::vector<std::vector<int8_t>> effects;    // copies of the effects
    std::vector<std::vector<double>> linkage;    // copies of the linkage maps
    std::vector<spegg_physiology> physiology;    // copies of the physiology parameters
    std::vector<spegg_ecology> ecology;          // copies of the ecologies
    GcapMap gcaps;                               // autotuned lanes-per-gamete caps by W
    std::vector<RepDesc> dev_descs;  // host images of the device descriptors, one per deme
    std::vector<uint32_t> deme_gen;  // each deme's generation, tracked on the host
    std::vector<uint8_t> image;      // host image of [0, static_end)
    bool errored = false;
    bool trace = false;
    uint32_t timing = 0;  // mask of kernel kinds bracketed by events
    bool use_graph = true;        // replay captured generations when the stream allows
    GenGraph graph_one, graph_many;  // captured with the trace setting below
    void drop_graphs() {
        graph_one.release();
        graph_many.release();
    }
    std::vector<Timed> pending;
    std::vector<hipEvent_t> event_pool;
    double ms[SPEGG_KERNEL_KINDS] = {0};
    uint64_t launches[SPEGG_KERNEL_KINDS] = {0};
    std::vector<double> class_ms;         // offspring event time by class since the last read
    std::vector<uint64_t> class_launches;

    RepDesc *d_descs() { return at<RepDesc>(base, plan.descs); }
    RepState *d_states() { return at<RepState>(base, plan.states); }
    SurvTile *d_surv_tiles() { return at<SurvTile>(base, plan.surv_tiles_at); }
    OffTile *d_off_tiles() { return at<OffTile>(base, plan.off_tiles_at); }
    SurvCount *d_surv_counts() { return at<SurvCount>(base, plan.surv_counts); }
    SurvGroup *d_surv_groups() { return at<SurvGroup>(base, plan.surv_groups); }
    Partial *d_partials() { return at<Partial>(base, plan.partials); }
    uint32_t *d_list_counts() { return at<uint32_t>(base, plan.list_counts_at); }
    TileLists lists() {
        return TileLists{at<SurvTile>(base, plan.list_surv_at), at<SurvTile>(base, plan.list_enc_at),
                         at<OffTile>(base, plan.list_off_at), d_list_counts(), (uint32_t)plan.classes.size()};
    }
};

namespace {

spegg_status device_fail(spegg_pop *pop, hipError_t e, const char *what) {
    if (pop) pop->errored = true;
    return fail(SPEGG_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

spegg_status check_pop(spegg_pop *pop) {
    if (!pop) return fail(SPEGG_E_INVALID, "null population handle");
    if (pop->errored) return fail(SPEGG_E_STATE, "population handle is errored by an earlier device failure");
    return SPEGG_OK;
}

hipEvent_t take_event(spegg_pop *pop) {
    if (!pop->event_pool.empty()) {
        hipEvent_t e = pop->event_pool.back();
        pop->event_pool.pop_back();
        return e;
    }
    // These events only time work on the population's stream: without the
    // system-scope fence a record does not write back and invalidate the
    // caches, which would slow the kernel it brackets and add to its time.
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

// Launch through f, bracketed by events when timing is on.
template <typename F>
hipError_t timed(spegg_pop *pop, int kind, F &&f, int cls = -1) {
    if (!(pop->timing & (1u << kind))) return f();
    hipEvent_t a = take_event(pop), b = take_event(pop);
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, pop->stream);
    if (e != hipSuccess) return e;
    e = f();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, pop->stream);
    if (e != hipSuccess) return e;
    pop->pending.push_back({kind, cls, a, b});
    return hipSuccess;
}

// A census (t, n) in pair 0; pair 1 one generation older and empty.
RepState initial_state(uint32_t t, uint32_t n) {
    RepState s;
    std::memset(&s, 0, sizeof s);
    s.t[0] = t;
    s.n[0] = n;
    s.t[1] = t - 1u;
    s.n[1] = 0;
    s.extinct = n == 0;
    return s;
}

spegg_rep_stats census_of(const RepState &s) {
    const uint32_t par = current_pair_host(s);
    spegg_rep_stats c;
    std::memset(&c, 0, sizeof c);
    c.generation = s.t[par];
    c.n = s.n[par];
    c.n_parents = s.n_prev;
    c.n_survivors = s.n_surv;
    c.extinct = s.extinct;
    c.captures = s.captures;
    for (int k = 0; k < kCensusSlots; ++k) {
        c.sum_z += s.sum_z[k];
        c.sum_z2 += (int64_t)s.sum_z2[k];
        c.sum_zf += s.sum_zf[k];
        c.sum_zf2 += s.sum_zf2[k];
    }
    c.near_ties = s.near_ties;
    c.truncated = s.truncated;
    c.resource[0] = s.R[0];
    c.resource[1] = s.R[1];
    c.eggs = s.eggs;
    c.sum_threshold = s.sum_threshold;
    c.updates = s.updates;
    return c;
}

// A replicate's census: its patches' summed (extinct when all are).
spegg_rep_stats sum_of(const spegg_rep_stats *p, uint32_t n) {
    spegg_rep_stats c = p[0];
    for (uint32_t k = 1; k < n; ++k) {
        c.n += p[k].n;
        c.n_parents += p[k].n_parents;
        c.n_survivors += p[k].n_survivors;
        c.extinct &= p[k].extinct;
        c.captures += p[k].captures;
        c.sum_z += p[k].sum_z;
        c.sum_z2 += p[k].sum_z2;
        c.sum_zf += p[k].sum_zf;
        c.sum_zf2 += p[k].sum_zf2;
        c.eggs += p[k].eggs;
        c.near_ties += p[k].near_ties;
        c.truncated += p[k].truncated;
        c.sum_threshold += p[k].sum_threshold;
        c.updates += p[k].updates;
    }
    return c;
}

spegg_status sync_stream(spegg_pop *pop) {
    const hipError_t e = hipStreamSynchronize(pop->stream);
    if (e != hipSuccess) return device_fail(pop, e, "hipStreamSynchronize");
    return SPEGG_OK;
}

spegg_status read_state(spegg_pop *pop, uint32_t deme, RepState &s) {
    hipError_t e = hipMemcpyAsync(&s, pop->d_states() + deme, sizeof s, hipMemcpyDeviceToHost, pop->stream);
    if (e != hipSuccess) return device_fail(pop, e, "hipMemcpyAsync(state)");
    return sync_stream(pop);
}

// The deme of (replicate, patch, species): patches of a ring, or the two
// species of the consumer-resource regime.
spegg_status find_deme(spegg_pop *pop, uint32_t rep, uint32_t patch, uint32_t species, uint32_t *deme) {
    if (rep >= pop->n_reps) return fail(SPEGG_E_INVALID, "replicate %u out of range (%u)", rep, pop->n_reps);
    const RepPlan &p = pop->plan.reps[rep];
    const uint32_t n_patches = p.cr ? 1u : p.n_demes, n_species = p.cr ? 2u : 1u;
    if (patch >= n_patches)
        return fail(SPEGG_E_INVALID, "patch %u out of range (replicate %u has %u)", patch, rep, n_patches);
    if (species >= n_species)
        return fail(SPEGG_E_INVALID, "species %u out of range (replicate %u has %u)", species, rep, n_species);
    *deme = p.deme0 + patch + species;
    return SPEGG_OK;
}

// Census of demes [0, n_demes) after folding pending sums.
spegg_status deme_stats(spegg_pop *pop, uint32_t n_demes, std::vector<spegg_rep_stats> &out) {
    std::vector<RepState> s(n_demes);
    hipError_t e = launch_census(pop->d_descs(), pop->d_states(), pop->d_partials(), n_demes, pop->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s.data(), pop->d_states(), sizeof(RepState) * n_demes, hipMemcpyDeviceToHost,
                           pop->stream);
    if (e != hipSuccess) return device_fail(pop, e, "stats");
    spegg_status st = sync_stream(pop);
    if (st != SPEGG_OK) return st;
    out.resize(n_demes);
    for (uint32_t u = 0; u < n_demes; ++u) {
        if (s[u].error) {
            pop->errored = true;
            return fail(SPEGG_E_DEVICE, "deme %u: a kernel reported an impossible state", u);
        }
        out[u] = census_of(s[u]);
    }
    return SPEGG_OK;
}

// Consumer-resource demes: every individual of age 0 and no resource
// captured, in both buffers (before a first generation).
hipError_t reset_species_state(spegg_pop *pop, uint32_t u) {
    const DemePlan &q = pop->plan.demes[u];
    const RepDesc &h = pop->dev_descs[u];
    if (!pop->plan.reps[q.rep].cr) return hipSuccess;
    const uint32_t zcap = ((q.cap + kSurvTileMax - 1) / kSurvTileMax) * kSurvTileMax;
    hipError_t e = launch_fill_u8(h.age[0], zcap, pop->stream);
    if (e == hipSuccess) e = launch_fill_u8(h.age[1], zcap, pop->stream);
    if (e == hipSuccess && h.won) e = launch_fill_u64(h.won, q.cap, pop->stream);
    return e;
}

// The launches of n generations on the population's stream.
hipError_t enqueue_generations(spegg_pop *pop, uint32_t n) {
    Plan &P = pop->plan;
    const uint32_t ns_tiles = (uint32_t)P.surv_tiles.size();
    const int trace = pop->trace ? 1 : 0;
    // listed: every launch walks this generation's lists of occupied tiles
    const TileLists lists = pop->lists();
    const uint32_t *ln = P.listed ? lists.counts : nullptr;
    const SurvTile *enc_tiles = P.listed ? lists.enc : at<SurvTile>(pop->base, P.enc_tiles_at);
    for (uint32_t g = 0; g < n; ++g) {
        SelArgs sa{pop->d_descs(), pop->d_states(), P.listed ? lists.surv : pop->d_surv_tiles(), pop->d_surv_counts(),
                   pop->d_surv_groups(), ns_tiles, trace, pop->n_demes == 1 ? 0 : -1, (int)P.surv_items,
                   pop->stream};
        sa.list_n = ln;
        sa.grid_survive = P.grid_survive;
        sa.grid_compact = P.grid_compact;
        hipError_t e = hipSuccess;
        if (P.listed) e = launch_plan_tiles(pop->d_descs(), pop->d_states(), pop->n_demes, lists, 0, pop->stream);
        if (e == hipSuccess && !P.enc_tiles.empty())
            e = timed(pop, SPEGG_KERNEL_ENCOUNTER, [&] {
                hipError_t r = launch_encounter(pop->d_descs(), pop->d_states(), enc_tiles,
                                                (uint32_t)P.enc_tiles.size(), ln ? ln + 1 : nullptr, P.grid_encounter,
                                                pop->stream);
                if (r == hipSuccess)  // captured resources credit their consumers
                    r = launch_credit(pop->d_descs(), pop->d_states(), sa.tiles, ns_tiles, ln, P.grid_survive,
                                      pop->stream);
                return r;
            });
        if (e == hipSuccess) e = timed(pop, SPEGG_KERNEL_SURVIVE, [&] { return launch_survive(sa); });
        if (e == hipSuccess) e = timed(pop, SPEGG_KERNEL_COMPACT, [&] { return launch_compact(sa); });
        if (e == hipSuccess && P.listed)
            e = launch_plan_tiles(pop->d_descs(), pop->d_states(), pop->n_demes, lists, 1, pop->stream);
        for (size_t ci = 0; ci < P.classes.size(); ++ci) {
            const OffClass &c = P.classes[ci];
            if (e != hipSuccess) return e;
            OffArgs oa{pop->d_descs(), pop->d_states(), P.listed ? lists.off : pop->d_off_tiles(), c.tile0, c.ntiles,
                       c.single_deme, pop->d_partials(), c.plane_words, c.geo_words, c.mask_words, c.grid, c.lds,
                       trace, pop->stream};
            oa.list_n = ln ? ln + 2 + ci : nullptr;
            e = timed(pop, SPEGG_KERNEL_OFFSPRING, [&] { return launch_offspring(c.shape, oa); }, (int)ci);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Fold the finished timing events into the per-kind and per-class sums.
spegg_status collect_times(spegg_pop *pop) {
    spegg_status st = sync_stream(pop);
    if (st != SPEGG_OK) return st;
    for (const Timed &t : pop->pending) {
        float x = 0.f;
        const hipError_t e = hipEventElapsedTime(&x, t.a, t.b);
        if (e != hipSuccess) return device_fail(pop, e, "hipEventElapsedTime");
        pop->ms[t.kind] += x;
        pop->launches[t.kind] += 1;
        if (t.cls >= 0) {
            if (pop->class_ms.size() <= (size_t)t.cls) {
                pop->class_ms.resize(t.cls + 1, 0.0);
                pop->class_launches.resize(t.cls + 1, 0);
            }
            pop->class_ms[t.cls] += x;
            pop->class_launches[t.cls] += 1;
        }
        pop->event_pool.push_back(t.a);
        pop->event_pool.push_back(t.b);
    }
    pop->pending.clear();
    return SPEGG_OK;
}

// Capture n generations (with the current trace setting) as a graph.
hipError_t capture(spegg_pop *pop, uint32_t n, GenGraph &g) {
    g.release();
    hipError_t e = hipStreamBeginCapture(pop->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t le = enqueue_generations(pop, n);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(pop->stream, &graph);
    if (le != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return le;
    }
    if (e != hipSuccess) return e;
    g.graph = graph;
    e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) g.release();
    return e;
}

}  // namespace

extern "C" {

int spegg_abi_version(void) { return SPEGG_ABI_VERSION; }

const char *spegg_last_error(void) { return g_error.c_str(); }

size_t spegg_footprint(const spegg_rep_desc *reps, uint32_t n_reps) {
    Plan P;
    if (make_plan(reps, n_reps, P) != SPEGG_OK) return 0;
    g_error.clear();
    return P.total;
}

spegg_status spegg_pop_create(const spegg_rep_desc *reps, uint32_t n_reps, void *device_mem, size_t device_bytes,
                              void *hip_stream, spegg_pop **out) {
    if (!out) return fail(SPEGG_E_INVALID, "null output handle pointer");
    *out = nullptr;
    spegg_pop *pop = new spegg_pop();
    spegg_status st = make_plan(reps, n_reps, pop->plan);
    if (st != SPEGG_OK) {
        delete pop;
        return st;
    }
    if (!device_mem || ((uintptr_t)device_mem & (kAlign - 1)) != 0) {
        delete pop;
        return fail(SPEGG_E_NOMEM, "workspace must be a non-null, %zu-byte aligned device pointer", kAlign);
    }
    if (device_bytes < pop->plan.total) {
        const size_t need = pop->plan.total;
        delete pop;
        return fail(SPEGG_E_NOMEM, "workspace holds %zu bytes, the population needs %zu", device_bytes, need);
    }
    pop->stream = (hipStream_t)hip_stream;
    pop->base = (uint8_t *)device_mem;
    pop->n_reps = n_reps;
    pop->descs.assign(reps, reps + n_reps);
    hipError_t e = hipGetDevice(&pop->device);
    if (e == hipSuccess) e = fit_offspring_grids(pop->plan, pop->device);
    size_t lds_limit = 0;
    if (e == hipSuccess) e = offspring_lds_limit(pop->device, &lds_limit);
    if (e != hipSuccess) {
        delete pop;
        return fail(SPEGG_E_DEVICE, "device query: %s", hipGetErrorString(e));
    }
    for (const OffClass &c : pop->plan.classes)
        if (c.lds > lds_limit) {
            const size_t need = c.lds;
            delete pop;
            return fail(SPEGG_E_UNSUPPORTED, "an offspring block needs %zu bytes of LDS, the device gives %zu", need,
                        lds_limit);
        }

    Plan &P = pop->plan;
    pop->n_demes = (uint32_t)P.demes.size();
    pop->image.assign(P.static_end, 0);
    uint8_t *img = pop->image.data();
    pop->dev_descs.resize(pop->n_demes);
    pop->deme_gen.assign(pop->n_demes, 0u);
    for (uint32_t u = 0; u < pop->n_demes; ++u) {
        const DemePlan &q = P.demes[u];
        const spegg_rep_desc &d = reps[q.rep];
        const RepPlan &p = P.reps[q.rep];
        RepDesc h;
        std::memset(&h, 0, sizeof h);
        h.L = d.n_loci;
        h.W = p.W;
        h.cap = q.cap;
        h.regime = d.regime;
        h.key0 = (uint32_t)d.seed;
        h.key1 = (uint32_t)(d.seed >> 32);
        h.c3 = d.replicate_id << 12 | q.species << 10 | q.patch;
        h.mode = p.mode;
        h.R = p.R;
        h.geo_len = (uint32_t)p.geo.size();
        h.binom_len = (uint32_t)p.binom.size();
        h.binom0 = p.binom[0];
        h.pois_len = (uint32_t)p.pois.size();
        h.zmin = p.zmin;
        h.zlen = p.zlen;
        h.sum_e = p.sum_e;
        h.unit_effects = p.unit ? 1u : 0u;
        h.tail_mask = (d.n_loci % 32u) ? ((1u << (d.n_loci % 32u)) - 1u) : ~0u;
        h.surv_tile0 = q.surv_tile0;
        h.surv_tile = kBlock * P.surv_items;
        h.surv_ntiles = q.surv_ntiles;
        h.grp0 = q.grp0;
        h.grp_n = q.grp_n;
        h.off_tile0 = q.off_tile0;
        h.off_ntiles = q.off_ntiles;
        h.off_per_tile = p.opt;
        h.off_class = q.off_class;
        h.off_list0 = P.classes[q.off_class].tile0;
        h.geo_scale = p.mode == kModeSkip ? (float)(1.0 / std::log2(1.0 - d.r)) : 0.0f;
        h.K = d.K;
        h.lambda = d.fecundity;
        h.mig_T = p.mig_T;
        h.patch = q.patch;
        h.left = p.mig_T ? p.deme0 + (q.patch + p.n_demes - 1u) % p.n_demes : u;
        h.right = p.mig_T ? p.deme0 + (q.patch + 1u) % p.n_demes : u;
        h.island = d.dispersal == SPEGG_ISLAND ? 1u : 0u;
        h.n_patches = p.cr ? 1u : p.n_demes;
        h.deme0 = p.deme0;
        h.home_T = prob_threshold(d.home_return);
        h.genome[0] = at<uint32_t>(pop->base, q.genome[0]);
        h.genome[1] = at<uint32_t>(pop->base, q.genome[1]);
        h.z[0] = at<int32_t>(pop->base, q.z[0]);
        h.z[1] = at<int32_t>(pop->base, q.z[1]);
        h.fate = at<uint16_t>(pop->base, q.fate);
        h.S = at<uint32_t>(pop->base, q.S);
        h.owner = q.owner ? at<uint32_t>(pop->base, q.owner) : nullptr;
        h.mom = at<uint32_t>(pop->base, q.mom);
        h.dad = at<uint32_t>(pop->base, q.dad);
        h.src = q.src ? at<uint32_t>(pop->base, q.src) : nullptr;
        h.vtab = p.vtab.empty() ? nullptr : at<double>(pop->base, p.vtab_at);
        h.pois = p.pois.empty() ? nullptr : at<uint64_t>(pop->base, p.pois_at);
        h.binom = at<uint64_t>(pop->base, p.binom_at);
        h.geo = p.geo.empty() ? nullptr : at<uint64_t>(pop->base, p.geo_at);
        h.planes = p.planes.empty() ? nullptr : at<uint32_t>(pop->base, p.planes_at);
        h.cont = p.cont ? 1u : 0u;
        h.exp_tf = d.exp_transform ? 1u : 0u;
        h.theta = d.theta;
        h.omega = d.omega;
        h.a0 = d.allele_mean;
        h.s0 = d.allele_sd;
        h.mut_sd = d.mut_sd_factor * std::fabs(d.allele_mean);
        h.noise_sd = d.noise_sd;
        h.sexes = p.phys ? 1u : d.sexes;  // the physiology regime's consumer has two sexes
        h.mating = d.mating;
        h.monogamy = d.monogamy;
        h.pref_opt = d.pref_optimum;
        h.pref_w = d.pref_width;
        h.choice_len = (uint32_t)p.choiceT.size();
        h.choice_zmin = p.choice_zmin;
        h.choiceT = p.choiceT.empty() ? nullptr : at<uint64_t>(pop->base, p.choiceT_at);
        h.map = p.map.empty() ? nullptr : at<uint32_t>(pop->base, p.map_at);
        h.sex[0] = q.sex[0] ? at<uint8_t>(pop->base, q.sex[0]) : nullptr;
        h.sex[1] = q.sex[1] ? at<uint8_t>(pop->base, q.sex[1]) : nullptr;
        if (p.phys) {
            const spegg_physiology &F = *d.physiology;
            h.alpha = F.alpha;
            h.gamma = F.gamma;
            h.delta = F.delta;
            h.attack = F.attack;
            h.handling = F.handling;
            for (int j = 0; j < 2; ++j) {
                h.KR2[j] = F.K[j];
                h.growth[j] = F.growth[j];
                h.growth_sd[j] = F.growth_sd[j];
            }
            h.steepness = F.steepness;
            h.ulmax = F.switch_frac * std::cbrt(F.w_max);
            h.kappa = F.kappa;
            h.qJ = F.qJ;
            h.qA = F.qA;
            h.beta1 = F.beta1;
            h.beta2 = F.beta2;
            h.beta_s = F.beta_s;
            h.maturity = F.maturity;
            h.v_f = F.v_f;
            h.v_m = F.v_m;
            h.kappa1 = F.kappa1;
            h.kappa2 = F.kappa2;
            h.kappa3 = F.kappa3;
            h.breed_every = F.breed_every;
            for (int b = 0; b < 2; ++b) {
                h.X[b] = at<double>(pop->base, q.X[b]);
                h.Y[b] = at<double>(pop->base, q.Y[b]);
            }
            h.G = at<double>(pop->base, q.G);
            h.ptiles = at<PhysTile>(pop->base, q.ptiles);
            h.gslot[0] = at<uint32_t>(pop->base, q.gslot[0]);
            h.gslot[1] = at<uint32_t>(pop->base, q.gslot[1]);
            h.gfree = at<uint32_t>(pop->base, q.gfree);
        }
        h.species = q.species;
        if (p.cr) {
            const spegg_ecology &ec = *d.ecology;
            h.partner = p.deme0 + (q.species ^ 1u);
            h.habitat = ec.habitat;
            h.trials = ec.resource_trials;
            h.enc_len = (uint32_t)p.enc.size();
            h.cap_len = (uint32_t)p.capT.size();
            h.q0 = ec.resource_q0;
            h.KR = ec.resource_K;
            for (int a = 0; a < 4; ++a) h.surv_age[a] = q.species == 0 ? ec.surv_resource[a] : ec.surv_consumer[a];
            h.enc = at<uint64_t>(pop->base, p.enc_at);
            h.capT = at<uint64_t>(pop->base, p.capT_at);
            h.cpois = at<uint64_t>(pop->base, p.cpois_at);
            h.cpois_off = at<uint32_t>(pop->base, p.cpois_off_at);
            h.age[0] = at<uint8_t>(pop->base, q.age[0]);
            h.age[1] = at<uint8_t>(pop->base, q.age[1]);
            h.won = q.won ? at<uint64_t>(pop->base, q.won) : nullptr;
            h.intake = q.intake ? at<uint32_t>(pop->base, q.intake) : nullptr;
        }
        pop->dev_descs[u] = h;
        std::memcpy(img + P.descs + u * sizeof(RepDesc), &h, sizeof h);
        RepState s0 = initial_state(0, q.n0);
        s0.census_pending = p.cont && q.n0 > 0;  // continuous alleles: sums folded on demand
        if (p.phys) {
            s0.gfree_n[0] = q.cap - q.n0;  // create_kernel fills the slot map and the free stack
            s0.R[0] = d.physiology->R0[0];
            s0.R[1] = d.physiology->R0[1];
        }
        std::memcpy(img + P.states + u * sizeof(RepState), &s0, sizeof s0);
    }
    for (uint32_t i = 0; i < n_reps; ++i) {
        const RepPlan &p = P.reps[i];
        if (!p.vtab.empty()) std::memcpy(img + p.vtab_at, p.vtab.data(), sizeof(double) * p.vtab.size());
        if (!p.pois.empty()) std::memcpy(img + p.pois_at, p.pois.data(), sizeof(uint64_t) * p.pois.size());
        std::memcpy(img + p.binom_at, p.binom.data(), sizeof(uint64_t) * p.binom.size());
        if (!p.geo.empty()) std::memcpy(img + p.geo_at, p.geo.data(), sizeof(uint64_t) * p.geo.size());
        if (!p.planes.empty()) std::memcpy(img + p.planes_at, p.planes.data(), sizeof(uint32_t) * p.planes.size());
        if (!p.map.empty()) std::memcpy(img + p.map_at, p.map.data(), sizeof(uint32_t) * p.map.size());
        if (!p.choiceT.empty())
            std::memcpy(img + p.choiceT_at, p.choiceT.data(), sizeof(uint64_t) * p.choiceT.size());
        if (p.cr) {
            std::memcpy(img + p.enc_at, p.enc.data(), sizeof(uint64_t) * p.enc.size());
            std::memcpy(img + p.capT_at, p.capT.data(), sizeof(uint64_t) * p.capT.size());
            std::memcpy(img + p.cpois_at, p.cpois.data(), sizeof(uint64_t) * p.cpois.size());
            std::memcpy(img + p.cpois_off_at, p.cpois_off.data(), sizeof(uint32_t) * p.cpois_off.size());
        }
    }
    if (!P.surv_tiles.empty())
        std::memcpy(img + P.surv_tiles_at, P.surv_tiles.data(), sizeof(SurvTile) * P.surv_tiles.size());
    if (!P.enc_tiles.empty())
        std::memcpy(img + P.enc_tiles_at, P.enc_tiles.data(), sizeof(SurvTile) * P.enc_tiles.size());
    if (!P.off_tiles.empty())
        std::memcpy(img + P.off_tiles_at, P.off_tiles.data(), sizeof(OffTile) * P.off_tiles.size());

    e = hipMemcpyAsync(pop->base, img, P.static_end, hipMemcpyHostToDevice, pop->stream);
    if (e != hipSuccess) {
        delete pop;
        return fail(SPEGG_E_DEVICE, "hipMemcpyAsync(tables): %s", hipGetErrorString(e));
    }
    // tile-group sums start from zero (the kernels keep them so afterwards)
    if (P.n_groups)
        e = launch_fill_u32((uint32_t *)pop->d_surv_groups(), (size_t)P.n_groups * sizeof(SurvGroup) / sizeof(uint32_t),
                            pop->stream);
    // so do the counts of the tile lists
    if (e == hipSuccess && P.listed) e = launch_fill_u32(pop->d_list_counts(), P.list_counts, pop->stream);
    if (e != hipSuccess) {
        delete pop;
        return fail(SPEGG_E_DEVICE, "tile groups: %s", hipGetErrorString(e));
    }
    // every deme's initial population in one launch
    e = launch_create(pop->d_descs(), pop->d_states(), pop->d_surv_tiles(), (uint32_t)P.surv_tiles.size(),
                      pop->stream);
    if (e != hipSuccess) {
        delete pop;
        return fail(SPEGG_E_DEVICE, "initial population: %s", hipGetErrorString(e));
    }
    // The effects, linkage and ecology pointers are the caller's: point at copies.
    pop->effects.resize(n_reps);
    pop->linkage.resize(n_reps);
    pop->ecology.resize(n_reps);
    pop->physiology.resize(n_reps);
    for (uint32_t i = 0; i < n_reps; ++i) {
        spegg_rep_desc &d = pop->descs[i];
        if (d.effects) {
            pop->effects[i].assign(d.effects, d.effects + d.n_loci);
            d.effects = pop->effects[i].data();
        }
        if (d.ecology) {
            pop->ecology[i] = *d.ecology;
            d.ecology = &pop->ecology[i];
        }
        if (d.linkage) {
            pop->linkage[i].assign(d.linkage, d.linkage + (d.n_loci > 1 ? d.n_loci - 1 : 0));
            d.linkage = pop->linkage[i].data();
        }
        if (d.physiology) {
            pop->physiology[i] = *d.physiology;
            d.physiology = &pop->physiology[i];
        }
    }
    *out = pop;
    g_error.clear();
    return SPEGG_OK;
}

spegg_status spegg_step_generations(spegg_pop *pop, uint32_t n_generations) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    // the patches of a replicate read each other's generation buffers
    for (uint32_t i = 0; i < pop->n_reps; ++i) {
        const RepPlan &p = pop->plan.reps[i];
        for (uint32_t k = 1; k < p.n_demes; ++k)
            if (pop->deme_gen[p.deme0 + k] != pop->deme_gen[p.deme0])
                return fail(SPEGG_E_STATE, "replicate %u: patch %u is at generation %u, patch 0 at %u", i, k,
                            pop->deme_gen[p.deme0 + k], pop->deme_gen[p.deme0]);
    }
    for (uint32_t &g : pop->deme_gen) g += n_generations;
    DeviceGuard guard(pop->device);
    // Graph replay needs a capturable stream and no per-launch events.
    const bool graphs = pop->use_graph && pop->stream != nullptr && pop->timing == 0;
    uint32_t done = 0;
    if (graphs) {
        hipError_t e = hipSuccess;
        while (e == hipSuccess && n_generations - done >= kGraphGenerations) {
            if (!pop->graph_many.exec) e = capture(pop, kGraphGenerations, pop->graph_many);
            if (e == hipSuccess) e = hipGraphLaunch(pop->graph_many.exec, pop->stream);
            done += kGraphGenerations;
        }
        while (e == hipSuccess && done < n_generations) {
            if (!pop->graph_one.exec) e = capture(pop, 1, pop->graph_one);
            if (e == hipSuccess) e = hipGraphLaunch(pop->graph_one.exec, pop->stream);
            ++done;
        }
        if (e != hipSuccess) return device_fail(pop, e, "generation graph");
        return SPEGG_OK;
    }
    const hipError_t e = enqueue_generations(pop, n_generations);
    if (e != hipSuccess) return device_fail(pop, e, "generation launch");
    return SPEGG_OK;
}

spegg_status spegg_prepare_graphs(spegg_pop *pop) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    if (!(pop->use_graph && pop->stream != nullptr && pop->timing == 0)) return SPEGG_OK;  // no replay to prepare
    DeviceGuard guard(pop->device);
    hipError_t e = hipSuccess;
    if (!pop->graph_many.exec) e = capture(pop, kGraphGenerations, pop->graph_many);
    if (e == hipSuccess && !pop->graph_one.exec) e = capture(pop, 1, pop->graph_one);
    // the executable graphs' resources onto the device now, not at their
    // first replay
    if (e == hipSuccess) e = hipGraphUpload(pop->graph_many.exec, pop->stream);
    if (e == hipSuccess) e = hipGraphUpload(pop->graph_one.exec, pop->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(pop->stream);
    if (e != hipSuccess) return device_fail(pop, e, "prepare_graphs");
    return SPEGG_OK;
}

spegg_status spegg_set_graph(spegg_pop *pop, int enable) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    pop->use_graph = enable != 0;
    return SPEGG_OK;
}

spegg_status spegg_stats(spegg_pop *pop, spegg_rep_stats *host_out, uint32_t n) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    if (!host_out || n == 0 || n > pop->n_reps)
        return fail(SPEGG_E_INVALID, "stats: need 0 < n <= %u and a buffer", pop->n_reps);
    DeviceGuard guard(pop->device);
    const RepPlan &last = pop->plan.reps[n - 1];
    std::vector<spegg_rep_stats> per;
    if ((st = deme_stats(pop, last.deme0 + last.n_demes, per)) != SPEGG_OK) return st;
    for (uint32_t i = 0; i < n; ++i) {
        const RepPlan &p = pop->plan.reps[i];
        host_out[i] = sum_of(per.data() + p.deme0, p.n_demes);
    }
    return SPEGG_OK;
}

spegg_status spegg_deme_stats(spegg_pop *pop, uint32_t rep, spegg_rep_stats *host_out, uint32_t n) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    if (rep >= pop->n_reps) return fail(SPEGG_E_INVALID, "replicate %u out of range (%u)", rep, pop->n_reps);
    const RepPlan &p = pop->plan.reps[rep];
    if (!host_out || n != p.n_demes)
        return fail(SPEGG_E_INVALID, "deme_stats: replicate %u has %u demes", rep, p.n_demes);
    DeviceGuard guard(pop->device);
    std::vector<spegg_rep_stats> per;
    if ((st = deme_stats(pop, p.deme0 + p.n_demes, per)) != SPEGG_OK) return st;
    for (uint32_t k = 0; k < n; ++k) host_out[k] = per[p.deme0 + k];
    return SPEGG_OK;
}

spegg_status spegg_read_genomes(spegg_pop *pop, uint32_t rep, uint32_t patch, uint32_t species, uint32_t *host_words,
                                size_t n_words, uint32_t *n_out) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    uint32_t u;
    if ((st = find_deme(pop, rep, patch, species, &u)) != SPEGG_OK) return st;
    if (pop->dev_descs[u].cont)
        return fail(SPEGG_E_STATE, "read_genomes: replicate %u has continuous alleles (spegg_read_alleles)", rep);
    DeviceGuard guard(pop->device);
    RepState s;
    if ((st = read_state(pop, u, s)) != SPEGG_OK) return st;
    const RepDesc &h = pop->dev_descs[u];
    const uint32_t n = s.n[current_pair_host(s)], t = s.t[current_pair_host(s)];
    const size_t words = (size_t)n * 2u * h.W;
    if (n_out) *n_out = n;
    if (words == 0) return SPEGG_OK;
    if (!host_words || n_words < words)
        return fail(SPEGG_E_INVALID, "read_genomes: need room for %zu words, have %zu", words, n_words);
    hipError_t e = hipMemcpyAsync(host_words, h.genome[t & 1u], words * sizeof(uint32_t), hipMemcpyDeviceToHost,
                                  pop->stream);
    if (e != hipSuccess) return device_fail(pop, e, "hipMemcpyAsync(genomes)");
    return sync_stream(pop);
}

spegg_status spegg_write_genomes(spegg_pop *pop, uint32_t rep, uint32_t patch, uint32_t species,
                                 const uint32_t *host_words, uint32_t n, uint32_t generation) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    uint32_t u;
    if ((st = find_deme(pop, rep, patch, species, &u)) != SPEGG_OK) return st;
    const RepDesc &h = pop->dev_descs[u];
    if (h.cont)
        return fail(SPEGG_E_STATE, "write_genomes: replicate %u has continuous alleles (spegg_write_alleles)", rep);
    if (n > h.cap) return fail(SPEGG_E_INVALID, "write_genomes: %u individuals exceed capacity %u", n, h.cap);
    if (n > 0 && !host_words) return fail(SPEGG_E_INVALID, "write_genomes: null words");
    for (uint32_t i = 0; i < n; ++i)
        for (uint32_t hh = 0; hh < 2; ++hh)
            if (host_words[((size_t)i * 2u + hh) * h.W + h.W - 1u] & ~h.tail_mask)
                return fail(SPEGG_E_INVALID, "write_genomes: individual %u has bits set beyond locus L-1", i);
    DeviceGuard guard(pop->device);
    if ((st = sync_stream(pop)) != SPEGG_OK) return st;
    const uint32_t buf = generation & 1u;
    const RepState s0 = initial_state(generation, n);
    hipError_t e = hipSuccess;
    if (n > 0)
        e = hipMemcpyAsync(h.genome[buf], host_words, (size_t)n * 2u * h.W * sizeof(uint32_t), hipMemcpyHostToDevice,
                           pop->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(pop->d_states() + u, &s0, sizeof s0, hipMemcpyHostToDevice, pop->stream);
    if (e == hipSuccess) e = launch_phenotypes(pop->d_descs() + u, pop->d_states() + u, n, buf, generation, pop->stream);
    if (e == hipSuccess) e = reset_species_state(pop, u);
    // the census restarts at an arbitrary generation: both parities of the
    // deme's tile-group sums from zero
    if (e == hipSuccess && h.grp_n)
        e = launch_fill_u32((uint32_t *)(pop->d_surv_groups() + h.grp0),
                            (size_t)2u * h.grp_n * sizeof(SurvGroup) / sizeof(uint32_t), pop->stream);
    if (e != hipSuccess) return device_fail(pop, e, "write_genomes");
    st = sync_stream(pop);
    if (st == SPEGG_OK) pop->deme_gen[u] = generation;
    return st;
}

spegg_status spegg_read_phenotypes(spegg_pop *pop, uint32_t rep, uint32_t patch, uint32_t species, int32_t *host_z,
                                   size_t n, uint32_t *n_out) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    uint32_t u;
    if ((st = find_deme(pop, rep, patch, species, &u)) != SPEGG_OK) return st;
    DeviceGuard guard(pop->device);
    RepState s;
    if ((st = read_state(pop, u, s)) != SPEGG_OK) return st;
    const uint32_t cn = s.n[current_pair_host(s)], ct = s.t[current_pair_host(s)];
    if (n_out) *n_out = cn;
    if (cn == 0) return SPEGG_OK;
    if (!host_z || n < cn) return fail(SPEGG_E_INVALID, "read_phenotypes: need room for %u values", cn);
    hipError_t e = hipMemcpyAsync(host_z, pop->dev_descs[u].z[ct & 1u], (size_t)cn * sizeof(int32_t),
                                  hipMemcpyDeviceToHost, pop->stream);
    if (e != hipSuccess) return device_fail(pop, e, "hipMemcpyAsync(phenotypes)");
    return sync_stream(pop);
}

spegg_status spegg_read_alleles(spegg_pop *pop, uint32_t rep, uint32_t patch, float *host_values, size_t n_values,
                                uint32_t *n_out) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    uint32_t u;
    if ((st = find_deme(pop, rep, patch, 0, &u)) != SPEGG_OK) return st;
    const RepDesc &h = pop->dev_descs[u];
    if (!h.cont) return fail(SPEGG_E_STATE, "read_alleles: replicate %u has biallelic genomes", rep);
    DeviceGuard guard(pop->device);
    RepState s;
    if ((st = read_state(pop, u, s)) != SPEGG_OK) return st;
    const uint32_t n = s.n[current_pair_host(s)], t = s.t[current_pair_host(s)];
    const size_t values = (size_t)n * 2u * h.L;
    if (n_out) *n_out = n;
    if (values == 0) return SPEGG_OK;
    if (!host_values || n_values < values)
        return fail(SPEGG_E_INVALID, "read_alleles: need room for %zu values, have %zu", values, n_values);
    // the device rows are W >= L floats (the pad zero): copy, then drop the
    // pad.  Physiology regime: rows by storage slot, through the census's
    // slot map.
    const bool slots = h.gfree != nullptr;
    std::vector<uint32_t> slot(slots ? n : 0);
    std::vector<float> rows((size_t)(slots ? h.cap : n) * 2u * h.W);
    hipError_t e = hipMemcpyAsync(rows.data(), h.genome[slots ? 0u : t & 1u], rows.size() * sizeof(float),
                                  hipMemcpyDeviceToHost, pop->stream);
    if (e == hipSuccess && slots)
        e = hipMemcpyAsync(slot.data(), h.gslot[t & 1u], n * sizeof(uint32_t), hipMemcpyDeviceToHost, pop->stream);
    if (e != hipSuccess) return device_fail(pop, e, "hipMemcpyAsync(alleles)");
    if ((st = sync_stream(pop)) != SPEGG_OK) return st;
    for (size_t i = 0; i < n; ++i) {
        const size_t from = slots ? slot[i] : i;
        if (from >= h.cap) {
            pop->errored = true;
            return fail(SPEGG_E_DEVICE, "read_alleles: individual %zu in storage slot %zu beyond capacity %u", i, from,
                        h.cap);
        }
        for (size_t hh = 0; hh < 2; ++hh)
            std::memcpy(host_values + (2u * i + hh) * h.L, rows.data() + (2u * from + hh) * h.W, sizeof(float) * h.L);
    }
    return SPEGG_OK;
}

spegg_status spegg_write_alleles(spegg_pop *pop, uint32_t rep, uint32_t patch, const float *host_values, uint32_t n,
                                 uint32_t generation) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    uint32_t u;
    if ((st = find_deme(pop, rep, patch, 0, &u)) != SPEGG_OK) return st;
    const RepDesc &h = pop->dev_descs[u];
    if (!h.cont) return fail(SPEGG_E_STATE, "write_alleles: replicate %u has biallelic genomes", rep);
    if (n > h.cap) return fail(SPEGG_E_INVALID, "write_alleles: %u individuals exceed capacity %u", n, h.cap);
    if (n > 0 && !host_values) return fail(SPEGG_E_INVALID, "write_alleles: null values");
    RepState cur_state;
    if (h.X[0]) {  // the resources carry over
        DeviceGuard g0(pop->device);
        if ((st = read_state(pop, u, cur_state)) != SPEGG_OK) return st;
    }
    for (size_t k = 0; k < (size_t)n * 2u * h.L; ++k)
        if (!std::isfinite(host_values[k])) return fail(SPEGG_E_INVALID, "write_alleles: value %zu is not finite", k);
    std::vector<float> rows((size_t)n * 2u * h.W, 0.0f);
    for (size_t r = 0; r < (size_t)n * 2u; ++r)
        std::memcpy(rows.data() + r * h.W, host_values + r * h.L, sizeof(float) * h.L);
    DeviceGuard guard(pop->device);
    if ((st = sync_stream(pop)) != SPEGG_OK) return st;
    const uint32_t buf = generation & 1u;
    RepState s0 = initial_state(generation, n);
    s0.census_pending = n > 0;  // the census sums are folded on demand
    if (h.X[0]) {
        s0.R[0] = cur_state.R[0];
        s0.R[1] = cur_state.R[1];
    }
    // physiology regime: individual i in storage slot i, the free stack
    // holding the slots above n with n on top
    const bool slots = h.gfree != nullptr;
    std::vector<uint32_t> slot_map, free_stack;
    if (slots) {
        s0.gfree_n[buf] = h.cap - n;
        slot_map.resize(n);
        for (uint32_t i = 0; i < n; ++i) slot_map[i] = i;
        free_stack.resize(h.cap - n);
        for (uint32_t k = 0; k < h.cap - n; ++k) free_stack[k] = h.cap - 1u - k;
    }
    hipError_t e = hipSuccess;
    if (n > 0)
        e = hipMemcpyAsync(h.genome[slots ? 0u : buf], rows.data(), rows.size() * sizeof(float), hipMemcpyHostToDevice,
                           pop->stream);
    if (e == hipSuccess && slots && n > 0)
        e = hipMemcpyAsync(h.gslot[buf], slot_map.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice, pop->stream);
    if (e == hipSuccess && slots && h.cap > n)
        e = hipMemcpyAsync(h.gfree, free_stack.data(), free_stack.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                           pop->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(pop->d_states() + u, &s0, sizeof s0, hipMemcpyHostToDevice, pop->stream);
    if (e == hipSuccess) e = launch_phenotypes(pop->d_descs() + u, pop->d_states() + u, n, buf, generation, pop->stream);
    if (e == hipSuccess && h.grp_n)
        e = launch_fill_u32((uint32_t *)(pop->d_surv_groups() + h.grp0),
                            (size_t)2u * h.grp_n * sizeof(SurvGroup) / sizeof(uint32_t), pop->stream);
    if (e != hipSuccess) return device_fail(pop, e, "write_alleles");
    st = sync_stream(pop);  // the host rows are copied before they are freed
    if (st == SPEGG_OK) pop->deme_gen[u] = generation;
    return st;
}

spegg_status spegg_read_phenotypes_f(spegg_pop *pop, uint32_t rep, uint32_t patch, float *host_z, size_t n,
                                     uint32_t *n_out) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    uint32_t u;
    if ((st = find_deme(pop, rep, patch, 0, &u)) != SPEGG_OK) return st;
    if (!pop->dev_descs[u].cont)
        return fail(SPEGG_E_STATE, "read_phenotypes_f: replicate %u has integer phenotypes", rep);
    static_assert(sizeof(float) == sizeof(int32_t), "phenotype buffers hold float bits");
    return spegg_read_phenotypes(pop, rep, patch, 0, reinterpret_cast<int32_t *>(host_z), n, n_out);
}

spegg_status spegg_read_body(spegg_pop *pop, uint32_t rep, double *host_X, double *host_Y, size_t n,
                             uint32_t *n_out) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    uint32_t u;
    if ((st = find_deme(pop, rep, 0, 0, &u)) != SPEGG_OK) return st;
    const RepDesc &h = pop->dev_descs[u];
    if (!h.X[0]) return fail(SPEGG_E_STATE, "read_body: replicate %u is not of the physiology regime", rep);
    DeviceGuard guard(pop->device);
    RepState s;
    if ((st = read_state(pop, u, s)) != SPEGG_OK) return st;
    const uint32_t cn = s.n[current_pair_host(s)], ct = s.t[current_pair_host(s)];
    if (n_out) *n_out = cn;
    if (cn == 0) return SPEGG_OK;
    if (!host_X || !host_Y || n < cn) return fail(SPEGG_E_INVALID, "read_body: need room for %u values", cn);
    hipError_t e = hipMemcpyAsync(host_X, h.X[ct & 1u], cn * sizeof(double), hipMemcpyDeviceToHost, pop->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(host_Y, h.Y[ct & 1u], cn * sizeof(double), hipMemcpyDeviceToHost, pop->stream);
    if (e != hipSuccess) return device_fail(pop, e, "hipMemcpyAsync(body)");
    return sync_stream(pop);
}

spegg_status spegg_read_sexes(spegg_pop *pop, uint32_t rep, uint32_t patch, uint8_t *host_sex, size_t n,
                              uint32_t *n_out) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    uint32_t u;
    if ((st = find_deme(pop, rep, patch, 0, &u)) != SPEGG_OK) return st;
    DeviceGuard guard(pop->device);
    RepState s;
    if ((st = read_state(pop, u, s)) != SPEGG_OK) return st;
    const uint32_t cn = s.n[current_pair_host(s)], ct = s.t[current_pair_host(s)];
    if (n_out) *n_out = cn;
    if (cn == 0) return SPEGG_OK;
    if (!host_sex || n < cn) return fail(SPEGG_E_INVALID, "read_sexes: need room for %u values", cn);
    const RepDesc &h = pop->dev_descs[u];
    if (!h.sex[0]) {
        std::memset(host_sex, 0, cn);
        return SPEGG_OK;
    }
    hipError_t e = hipMemcpyAsync(host_sex, h.sex[ct & 1u], cn, hipMemcpyDeviceToHost, pop->stream);
    if (e != hipSuccess) return device_fail(pop, e, "hipMemcpyAsync(sexes)");
    return sync_stream(pop);
}

spegg_status spegg_read_ages(spegg_pop *pop, uint32_t rep, uint32_t species, uint8_t *host_age, size_t n,
                             uint32_t *n_out) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    uint32_t u;
    if ((st = find_deme(pop, rep, 0, species, &u)) != SPEGG_OK) return st;
    const RepDesc &h = pop->dev_descs[u];
    if (!h.age[0]) return fail(SPEGG_E_STATE, "read_ages: replicate %u has no age classes", rep);
    DeviceGuard guard(pop->device);
    RepState s;
    if ((st = read_state(pop, u, s)) != SPEGG_OK) return st;
    const uint32_t cn = s.n[current_pair_host(s)], ct = s.t[current_pair_host(s)];
    if (n_out) *n_out = cn;
    if (cn == 0) return SPEGG_OK;
    if (!host_age || n < cn) return fail(SPEGG_E_INVALID, "read_ages: need room for %u values", cn);
    hipError_t e = hipMemcpyAsync(host_age, h.age[ct & 1u], cn, hipMemcpyDeviceToHost, pop->stream);
    if (e != hipSuccess) return device_fail(pop, e, "hipMemcpyAsync(ages)");
    return sync_stream(pop);
}

spegg_status spegg_read_intake(spegg_pop *pop, uint32_t rep, uint32_t *host_intake, size_t n, uint32_t *n_out) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    uint32_t u;
    if ((st = find_deme(pop, rep, 0, 1, &u)) != SPEGG_OK) return st;
    DeviceGuard guard(pop->device);
    RepState s;
    if ((st = read_state(pop, u, s)) != SPEGG_OK) return st;
    const uint32_t m = s.n_prev;  // the consumers the last generation started from
    if (n_out) *n_out = m;
    if (m == 0) return SPEGG_OK;
    if (!host_intake || n < m) return fail(SPEGG_E_INVALID, "read_intake: need room for %u values", m);
    hipError_t e = hipMemcpyAsync(host_intake, pop->dev_descs[u].intake, (size_t)m * sizeof(uint32_t),
                                  hipMemcpyDeviceToHost, pop->stream);
    if (e != hipSuccess) return device_fail(pop, e, "hipMemcpyAsync(intake)");
    return sync_stream(pop);
}

spegg_status spegg_read_survivors(spegg_pop *pop, uint32_t rep, uint32_t patch, uint32_t species, uint32_t *host_idx,
                                  size_t n, uint32_t *n_out) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    uint32_t u;
    if ((st = find_deme(pop, rep, patch, species, &u)) != SPEGG_OK) return st;
    DeviceGuard guard(pop->device);
    RepState s;
    if ((st = read_state(pop, u, s)) != SPEGG_OK) return st;
    const uint32_t m = s.n_surv;
    if (n_out) *n_out = m;
    if (m == 0) return SPEGG_OK;
    if (!host_idx || n < m) return fail(SPEGG_E_INVALID, "read_survivors: need room for %u indices", m);
    hipError_t e = hipMemcpyAsync(host_idx, pop->dev_descs[u].S, (size_t)m * sizeof(uint32_t),
                                  hipMemcpyDeviceToHost, pop->stream);
    if (e != hipSuccess) return device_fail(pop, e, "hipMemcpyAsync(survivors)");
    return sync_stream(pop);
}

spegg_status spegg_allele_counts(spegg_pop *pop, uint32_t rep, uint32_t patch, uint32_t species, uint32_t *counts_dev,
                                 uint32_t *host_counts, uint32_t n_loci, uint32_t *n_out) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    uint32_t u;
    if ((st = find_deme(pop, rep, patch, species, &u)) != SPEGG_OK) return st;
    const RepDesc &h = pop->dev_descs[u];
    if (h.cont) return fail(SPEGG_E_UNSUPPORTED, "allele_counts: replicate %u has continuous alleles", rep);
    if (n_loci != h.L || !counts_dev || !host_counts)
        return fail(SPEGG_E_INVALID, "allele_counts: need n_loci == %u and both arrays", h.L);
    DeviceGuard guard(pop->device);
    RepState s;
    if ((st = read_state(pop, u, s)) != SPEGG_OK) return st;
    const uint32_t n = s.n[current_pair_host(s)];
    if (n_out) *n_out = n;
    hipError_t e = hipMemsetAsync(counts_dev, 0, sizeof(uint32_t) * h.L, pop->stream);
    if (e == hipSuccess)
        e = launch_allele_counts(pop->d_descs() + u, pop->d_states() + u, h, n, counts_dev, pop->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(host_counts, counts_dev, sizeof(uint32_t) * h.L, hipMemcpyDeviceToHost, pop->stream);
    if (e != hipSuccess) return device_fail(pop, e, "allele_counts");
    return sync_stream(pop);
}

spegg_status spegg_allele_counts_noalloc(spegg_pop *pop, uint32_t rep, uint32_t patch, uint32_t species,
                                         uint32_t *host_counts, uint32_t n_loci, uint32_t *n_out) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    uint32_t u;
    if ((st = find_deme(pop, rep, patch, species, &u)) != SPEGG_OK) return st;
    const RepDesc &h = pop->dev_descs[u];
    if (h.cont) return fail(SPEGG_E_UNSUPPORTED, "allele_counts_noalloc: replicate %u has continuous alleles", rep);
    if (n_loci != h.L || !host_counts)
        return fail(SPEGG_E_INVALID, "allele_counts_noalloc: need n_loci == %u and a host array", h.L);
    DeviceGuard guard(pop->device);
    uint32_t *counts = nullptr;
    size_t words = 0;
    hipError_t e = allele_scratch(&counts, &words);
    if (e != hipSuccess) return device_fail(pop, e, "allele_counts_noalloc: scratch address");
    if (h.L > words)
        return fail(SPEGG_E_INVALID, "allele_counts_noalloc: %u loci exceed the scratch of %zu counters", h.L, words);
    RepState s;
    if ((st = read_state(pop, u, s)) != SPEGG_OK) return st;
    const uint32_t n = s.n[current_pair_host(s)];
    if (n_out) *n_out = n;
    // counters from zero by a fill kernel (the array keeps the last call's counts)
    e = launch_fill_u32(counts, h.L, pop->stream);
    if (e == hipSuccess) e = launch_allele_counts(pop->d_descs() + u, pop->d_states() + u, h, n, counts, pop->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(host_counts, counts, sizeof(uint32_t) * h.L, hipMemcpyDeviceToHost, pop->stream);
    if (e != hipSuccess) return device_fail(pop, e, "allele_counts_noalloc");
    return sync_stream(pop);
}

spegg_status spegg_set_trace(spegg_pop *pop, int enable) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    if (pop->trace != (enable != 0)) pop->drop_graphs();
    pop->trace = enable != 0;
    return SPEGG_OK;
}

spegg_status spegg_read_parents(spegg_pop *pop, uint32_t rep, uint32_t patch, uint32_t species, uint32_t *host_mom,
                                uint32_t *host_dad, uint32_t *host_src, size_t n, uint32_t *n_out) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    uint32_t u;
    if ((st = find_deme(pop, rep, patch, species, &u)) != SPEGG_OK) return st;
    DeviceGuard guard(pop->device);
    RepState s;
    if ((st = read_state(pop, u, s)) != SPEGG_OK) return st;
    if (!s.traced) return fail(SPEGG_E_STATE, "read_parents: tracing was off for the last generation");
    const uint32_t cn = s.n[current_pair_host(s)] - s.n_carry;  // newborns
    if (n_out) *n_out = cn;
    if (cn == 0) return SPEGG_OK;
    if (!host_mom || !host_dad || n < cn) return fail(SPEGG_E_INVALID, "read_parents: need room for %u entries", cn);
    const RepDesc &h = pop->dev_descs[u];
    hipError_t e = hipMemcpyAsync(host_mom, h.mom, (size_t)cn * sizeof(uint32_t), hipMemcpyDeviceToHost, pop->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(host_dad, h.dad, (size_t)cn * sizeof(uint32_t), hipMemcpyDeviceToHost, pop->stream);
    if (e != hipSuccess) return device_fail(pop, e, "hipMemcpyAsync(parents)");
    if (host_src) {
        if (h.src) {
            e = hipMemcpyAsync(host_src, h.src, (size_t)cn * sizeof(uint32_t), hipMemcpyDeviceToHost, pop->stream);
            if (e != hipSuccess) return device_fail(pop, e, "hipMemcpyAsync(parents)");
        } else {
            for (uint32_t j = 0; j < cn; ++j) host_src[j] = patch;  // no migration: the home patch
        }
    }
    return sync_stream(pop);
}

spegg_status spegg_set_timing(spegg_pop *pop, uint32_t kinds_mask) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    if (kinds_mask & ~SPEGG_TIME_ALL) return fail(SPEGG_E_INVALID, "set_timing: unknown kernel kinds in mask");
    pop->timing = kinds_mask;
    return SPEGG_OK;
}

spegg_status spegg_offspring_class_times(spegg_pop *pop, uint32_t *w_min, uint32_t *w_max, double *ms,
                                         uint64_t *launches, uint32_t cap, uint32_t *n_out) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    const uint32_t nc = (uint32_t)pop->plan.classes.size();
    if (!n_out || (cap && (!w_min || !w_max || !ms || !launches)))
        return fail(SPEGG_E_INVALID, "offspring_class_times: null argument");
    DeviceGuard guard(pop->device);
    if ((st = collect_times(pop)) != SPEGG_OK) return st;
    *n_out = nc;
    for (uint32_t c = 0; c < nc && c < cap; ++c) {
        uint32_t lo = ~0u, hi = 0;
        for (const RepPlan &p : pop->plan.reps) {
            const OffShape &a = p.shape, &b = pop->plan.classes[c].shape;
            if (!same_shape(a, b)) continue;
            lo = shape_key(p) < lo ? shape_key(p) : lo;
            hi = shape_key(p) > hi ? shape_key(p) : hi;
        }
        w_min[c] = lo;
        w_max[c] = hi;
        ms[c] = c < pop->class_ms.size() ? pop->class_ms[c] : 0.0;
        launches[c] = c < pop->class_launches.size() ? pop->class_launches[c] : 0;
    }
    pop->class_ms.assign(nc, 0.0);
    pop->class_launches.assign(nc, 0);
    return SPEGG_OK;
}

spegg_status spegg_kernel_times(spegg_pop *pop, double *ms, uint64_t *launches, uint32_t n_kinds) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    if (n_kinds > SPEGG_KERNEL_KINDS || (n_kinds && (!ms || !launches)))
        return fail(SPEGG_E_INVALID, "kernel_times: n_kinds <= %d and two arrays", SPEGG_KERNEL_KINDS);
    DeviceGuard guard(pop->device);
    if ((st = collect_times(pop)) != SPEGG_OK) return st;
    for (uint32_t k = 0; k < n_kinds; ++k) {
        ms[k] = pop->ms[k];
        launches[k] = pop->launches[k];
    }
    for (int k = 0; k < SPEGG_KERNEL_KINDS; ++k) {
        pop->ms[k] = 0;
        pop->launches[k] = 0;
    }
    return SPEGG_OK;
}

}  // extern "C"

namespace {

// Re-plan the offspring kernels with the population's lanes-per-gamete caps:
// fold pending census sums (they are indexed by the old tiles), then
// replace the offspring tiles and the descriptors' tile fields.  Buffers do
// not move: the carve does not depend on the shapes.
spegg_status apply_shapes(spegg_pop *pop) {
    Plan P2;
    spegg_status st = make_plan(pop->descs.data(), pop->n_reps, P2, &pop->gcaps, pop->plan.listed ? 1 : 0);
    if (st != SPEGG_OK) return st;
    const hipError_t eg = fit_offspring_grids(P2, pop->device);
    if (eg != hipSuccess) return device_fail(pop, eg, "autotune: grids");
    if (P2.total != pop->plan.total || P2.static_end != pop->plan.static_end || P2.off_tiles_at != pop->plan.off_tiles_at)
        return fail(SPEGG_E_STATE, "autotune: a new shape would move buffers");
    hipError_t e = launch_census(pop->d_descs(), pop->d_states(), pop->d_partials(), pop->n_demes, pop->stream);
    for (uint32_t u = 0; u < pop->n_demes; ++u) {
        RepDesc &h = pop->dev_descs[u];
        h.off_tile0 = P2.demes[u].off_tile0;
        h.off_ntiles = P2.demes[u].off_ntiles;
        h.off_per_tile = P2.reps[P2.demes[u].rep].opt;
        h.off_class = P2.demes[u].off_class;
        h.off_list0 = P2.classes[h.off_class].tile0;
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(pop->d_descs(), pop->dev_descs.data(), sizeof(RepDesc) * pop->n_demes,
                           hipMemcpyHostToDevice, pop->stream);
    if (e == hipSuccess && !P2.off_tiles.empty())
        e = hipMemcpyAsync(at<OffTile>(pop->base, P2.off_tiles_at), P2.off_tiles.data(),
                           sizeof(OffTile) * P2.off_tiles.size(), hipMemcpyHostToDevice, pop->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(pop->stream);  // the host arrays are copied before they change
    if (e != hipSuccess) return device_fail(pop, e, "autotune: new shapes");
    pop->plan = std::move(P2);
    pop->drop_graphs();
    return SPEGG_OK;
}

// Sum of the cumulative genotype-locus updates of every deme (waits).
spegg_status total_updates(spegg_pop *pop, uint64_t *out) {
    std::vector<RepState> s(pop->n_demes);
    hipError_t e = hipMemcpyAsync(s.data(), pop->d_states(), sizeof(RepState) * pop->n_demes, hipMemcpyDeviceToHost,
                                  pop->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(pop->stream);
    if (e != hipSuccess) return device_fail(pop, e, "autotune: states");
    *out = 0;
    for (const RepState &r : s) *out += r.updates;
    return SPEGG_OK;
}

}  // namespace

extern "C" {

spegg_status spegg_autotune(spegg_pop *pop, uint32_t generations_per_trial, uint32_t *w_out, uint32_t *gcap_out,
                            uint32_t cap, uint32_t *n_out) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    if (generations_per_trial == 0) return fail(SPEGG_E_INVALID, "autotune: need at least one generation per trial");
    DeviceGuard guard(pop->device);
    // one cap per genome key: words per haplotype, continuous alleles flagged
    std::vector<uint32_t> Ws;
    for (const RepPlan &p : pop->plan.reps)
        if (std::find(Ws.begin(), Ws.end(), shape_key(p)) == Ws.end()) Ws.push_back(shape_key(p));
    std::sort(Ws.begin(), Ws.end());
    // Trials run as production does (graph replay when enabled), so no
    // per-launch events: two events bracket a run of whole generations.
    const uint32_t saved_timing = pop->timing;
    pop->timing = 0;
    hipEvent_t ea = take_event(pop), eb = take_event(pop);
    if (!ea || !eb) {
        if (ea) pop->event_pool.push_back(ea);
        if (eb) pop->event_pool.push_back(eb);
        pop->timing = saved_timing;
        return fail(SPEGG_E_DEVICE, "autotune: no events");
    }
    for (uint32_t W : Ws) {
        std::vector<int> cands;
        std::vector<OffShape> seen;
        for (int g : {1, 2, 4, 8, 16, 32}) {
            const OffShape sh = shape_of_key(W, g);
            bool dup = false;
            for (const OffShape &x : seen) dup |= same_shape(x, sh);
            if (!dup) {
                seen.push_back(sh);
                cands.push_back(g);
            }
        }
        std::vector<double> score(cands.size(), -1.0);
        for (int round = 0; round < kAutotuneRounds && st == SPEGG_OK; ++round) {
            for (size_t c = 0; c < cands.size() && st == SPEGG_OK; ++c) {
                pop->gcaps[W] = cands[c];
                if ((st = apply_shapes(pop)) != SPEGG_OK) break;
                // untimed: loads the shape's code and captures the graphs the
                // timed generations replay
                if ((st = spegg_step_generations(pop, generations_per_trial)) != SPEGG_OK) break;
                uint64_t u0 = 0, u1 = 0;
                if ((st = total_updates(pop, &u0)) != SPEGG_OK) break;
                hipError_t e = hipEventRecord(ea, pop->stream);
                if (e != hipSuccess) {
                    st = device_fail(pop, e, "autotune: event");
                    break;
                }
                if ((st = spegg_step_generations(pop, generations_per_trial)) != SPEGG_OK) break;
                e = hipEventRecord(eb, pop->stream);
                if (e != hipSuccess) {
                    st = device_fail(pop, e, "autotune: event");
                    break;
                }
                if ((st = total_updates(pop, &u1)) != SPEGG_OK) break;  // waits for eb too
                float ms = 0.f;
                e = hipEventElapsedTime(&ms, ea, eb);
                if (e != hipSuccess) {
                    st = device_fail(pop, e, "autotune: event time");
                    break;
                }
                const double s = (double)ms / (double)(u1 > u0 ? u1 - u0 : 1u);
                if (score[c] < 0.0 || s < score[c]) score[c] = s;
            }
        }
        if (st != SPEGG_OK) break;
        size_t best = 0;
        for (size_t c = 1; c < cands.size(); ++c)
            if (score[c] < score[best]) best = c;
        pop->gcaps[W] = cands[best];
    }
    pop->event_pool.push_back(ea);
    pop->event_pool.push_back(eb);
    pop->timing = saved_timing;
    if (st != SPEGG_OK) return st;
    if ((st = apply_shapes(pop)) != SPEGG_OK) return st;
    if (n_out) *n_out = (uint32_t)Ws.size();
    for (uint32_t k = 0; k < Ws.size() && k < cap; ++k) {
        if (w_out) w_out[k] = Ws[k];
        if (gcap_out) gcap_out[k] = (uint32_t)pop->gcaps[Ws[k]];
    }
    return SPEGG_OK;
}

spegg_status spegg_set_offspring_cap(spegg_pop *pop, uint32_t W, uint32_t gcap) {
    spegg_status st = check_pop(pop);
    if (st != SPEGG_OK) return st;
    if (gcap == 0 || gcap > 32 || (gcap & (gcap - 1)) != 0)
        return fail(SPEGG_E_INVALID, "set_offspring_cap: cap %u is not a power of two in 1..32", gcap);
    bool have = false;
    for (const RepPlan &p : pop->plan.reps) have |= shape_key(p) == W;
    if (!have) return fail(SPEGG_E_INVALID, "set_offspring_cap: no replicate has genome key %#x", W);
    DeviceGuard guard(pop->device);
    const int saved = pop->gcaps.count(W) ? pop->gcaps[W] : (W & kContKey) ? kDefaultContGCap : offspring_gcap(W);
    pop->gcaps[W] = (int)gcap;
    st = apply_shapes(pop);
    if (st != SPEGG_OK) pop->gcaps[W] = saved;
    return st;
}

void spegg_pop_destroy(spegg_pop *pop) {
    if (!pop) return;
    {
        DeviceGuard guard(pop->device);
        (void)hipStreamSynchronize(pop->stream);
    }
    spegg::pop_release_done(pop);
}

}  // extern "C"

// Internal helpers of the job server (spegg_internal.h).
namespace spegg {

void pop_release_done(spegg_pop *pop) {
    if (!pop) return;
    {
        DeviceGuard guard(pop->device);
        for (const Timed &t : pop->pending) {
            (void)hipEventDestroy(t.a);
            (void)hipEventDestroy(t.b);
        }
        for (hipEvent_t e : pop->event_pool) (void)hipEventDestroy(e);
        pop->drop_graphs();
    }
    delete pop;
}

size_t pop_state_bytes(const spegg_pop *pop) { return sizeof(RepState) * pop->n_demes; }

hipError_t pop_census_async(spegg_pop *pop, void *host_states) {
    DeviceGuard guard(pop->device);
    hipError_t e = launch_census(pop->d_descs(), pop->d_states(), pop->d_partials(), pop->n_demes, pop->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(host_states, pop->d_states(), pop_state_bytes(pop), hipMemcpyDeviceToHost, pop->stream);
    if (e != hipSuccess) pop->errored = true;
    return e;
}

spegg_status pop_results(spegg_pop *pop, const void *host_states, spegg_rep_stats *out) {
    const RepState *s = static_cast<const RepState *>(host_states);
    std::vector<spegg_rep_stats> per(pop->n_demes);
    for (uint32_t u = 0; u < pop->n_demes; ++u) {
        if (s[u].error) {
            pop->errored = true;
            return fail(SPEGG_E_DEVICE, "deme %u: a kernel reported an impossible state", u);
        }
        per[u] = census_of(s[u]);
    }
    for (uint32_t i = 0; i < pop->n_reps; ++i) {
        const RepPlan &p = pop->plan.reps[i];
        out[i] = sum_of(per.data() + p.deme0, p.n_demes);
    }
    return SPEGG_OK;
}

}  // namespace spegg

extern "C" {

int spegg_threshold_table(int kind, double a, uint32_t b, uint64_t *out, int cap) {
    std::vector<uint64_t> T;
    bool ok = false;
    if (kind == 0) ok = poisson_table(a, cap, T);
    else if (kind == 1) ok = binomial_table(b, a, cap, T);
    else if (kind == 2) {
        if (a >= 0.0 && a <= 0.5 && (int64_t)b <= cap) {
            geometric_table(a, b, T);
            ok = true;
        }
    }
    if (!ok || !out || (int)T.size() > cap) return -1;
    std::memcpy(out, T.data(), sizeof(uint64_t) * T.size());
    return (int)T.size();
}

int spegg_recomb_mode(double r) { return (int)recomb_mode(r); }

int spegg_geometric_gap(double r, uint32_t n_loci, uint32_t x, uint32_t guess, uint32_t *gap) {
    if (!gap || !(r > 0.0 && r < 0.5) || n_loci < 2 || n_loci > SPEGG_MAX_LOCI) return -1;
    // the table as the offspring kernel holds it: up to the first threshold
    // of 2^32, narrowed to 32-bit words
    std::vector<uint64_t> T;
    geometric_table(r, n_loci - 1u, T);
    const uint32_t len = geometric_device_len(T);
    if (len == 0) return -1;
    std::vector<uint32_t> T32(T.begin(), T.begin() + len);
    *gap = geometric_gap_fix(T32.data(), len, guess, x);
    return (int)len;
}

spegg_status spegg_philox_fill(uint64_t seed, const uint32_t *ctr_dev, uint32_t *out_dev, uint32_t n,
                               void *hip_stream) {
    if (n && (!ctr_dev || !out_dev)) return fail(SPEGG_E_INVALID, "philox_fill: null arrays");
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = launch_philox_fill((uint32_t)seed, (uint32_t)(seed >> 32), ctr_dev, out_dev, n, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(SPEGG_E_DEVICE, "philox_fill: %s", hipGetErrorString(e));
    return SPEGG_OK;
}

spegg_status spegg_philox_rate(uint64_t seed, uint32_t blocks_per_thread, uint32_t *out_dev, uint32_t n,
                               void *hip_stream) {
    if (n && !out_dev) return fail(SPEGG_E_INVALID, "philox_rate: null output");
    const hipError_t e = launch_philox_rate((uint32_t)seed, (uint32_t)(seed >> 32), blocks_per_thread, out_dev, n,
                                            (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(SPEGG_E_DEVICE, "philox_rate: %s", hipGetErrorString(e));
    return SPEGG_OK;
}

}  // extern "C"

// Kernels of one generation (main text, Fig. 1) for gfx950.
//
//   survive    D + the offspring count of A: per adult p = v(z) s(N), one
//              Philox word against floor(p 2^32), the Poisson offspring
//              count of a surviving mother; a fate per adult, counts per tile
//   compact    E: each tile's prefix is the sum of the counts of the
//              replicate's earlier tiles; survivor ranks give the ascending
//              survivor list, kid ranks each mother's offspring slots; tile 0
//              of each replicate advances the census; consumer-resource and
//              physiology survivors move to the front of the next census
//   offspring  A (parents) + B (gametes: crossover mask, mutation flips)
//              + C (additive phenotype by popcounts) + census partials; one
//              team of 2G lanes per newborn, V consecutive words per lane
//   census     (on demand) folds the partials into the census sums
//              (continuous alleles: sums the census itself, in a fixed order)
//   create     (once) every deme's initial population: genomes, phenotypes,
//              census sums (integer phenotypes)
//   encounter  (consumer-resource regime, before survive) consumers meet
//              and capture resources; each captured resource keeps the
//              lowest (consumer, encounter) key by a 64-bit atomic minimum
//   credit     (consumer-resource regime, after encounter) each captured
//              resource adds one to its consumer's intake
//   plan_tiles (populations of several demes whose censuses can fall below
//              their capacities) lists the tiles a generation occupies;
//              the launches then walk the lists with resident grids
//
// All of it is integer work except p = v s (IEEE double, no contraction),
// so every result is reproducible bit for bit.  No kernel waits on another
// block of its own launch: blocks communicate only across launches.
//
// The census (generation t, size N) is double-buffered per replicate: the
// current census is the pair with the larger t; compact writes (t + 1,
// newborns) into the other pair, which no other block of its launch reads.
// So no kernel argument changes from one generation to the next and
// generations can be replayed as graphs.
#include <hip/hip_runtime.h>

#include <mutex>

#include "philox.h"
#include "spegg_internal.h"

namespace spegg {

// Device scratch of the allocation-free allele counts: one counter per locus
// for the longest genome the library takes (64 KiB), one copy per device,
// held until the process ends.  Host code never passes this name as an
// address: allele_scratch() asks each device for its copy's address.
static __device__ __align__(256) uint32_t scratch[SPEGG_MAX_LOCI];

namespace {

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, uint32_t tid = threadIdx.x) {
    const uint32_t lane = tid & 63u;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(v, o, 64);
        if (lane >= (uint32_t)o) v += t;
    }
    return v;
}

// Exclusive prefix over the block (kBlock threads = 4 waves); *total gets
// the block sum.  Every thread of the block must call it.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *sh, uint32_t *total,
                                                    uint32_t tid = threadIdx.x) {
    const uint32_t incl = wave_incl_scan(v, tid);
    const uint32_t wave = tid >> 6;
    if ((tid & 63u) == 63) sh[wave] = incl;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (uint32_t w = 0; w < kBlock / 64; ++w) {
        const uint32_t s = sh[w];
        if (w < wave) off += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + incl - v;
}

// LDS visibility among the lanes of one wave: the wave's LDS operations
// complete and are not reordered across it; global loads stay in flight.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Inclusive prefix XOR over the bits of a word: bit i = XOR of bits 0..i.
__device__ __forceinline__ uint32_t prefix_xor32(uint32_t x) {
    x ^= x << 1;
    x ^= x << 2;
    x ^= x << 4;
    x ^= x << 8;
    x ^= x << 16;
    return x;
}

__device__ __forceinline__ double density_factor(const RepDesc &d, uint32_t n) {
    if (d.regime != SPEGG_POISSON_BH || !(d.K > 0.0)) return 1.0;
    return 1.0 / (1.0 + (d.lambda - 1.0) * (double)n / d.K);
}

// Continuous alleles: a standard normal deviate from one Philox block by
// the Box-Muller transform (Box & Muller 1958): u1 in (0, 1] from words 0
// (low) and 1 (high), u2 in [0, 1) from words 2 and 3, 53 bits each;
// sqrt(-2 ln u1) cos(2 pi u2) in double.
__device__ __forceinline__ double normal_of(const Words4 &b) {
    const uint64_t a = ((uint64_t)b.v[1] << 32) | b.v[0];
    const uint64_t c = ((uint64_t)b.v[3] << 32) | b.v[2];
    const double u1 = ((double)(a >> 11) + 1.0) * (1.0 / 9007199254740992.0);
    const double u2 = (double)(c >> 11) * (1.0 / 9007199254740992.0);
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
}

// Continuous alleles: Gaussian viability of an expressed phenotype (the
// bits of a float), exp(-(z - theta)^2 / (2 omega^2)); omega <= 0: 1.
__device__ __forceinline__ double viability_cont(const RepDesc &d, uint32_t zbits) {
    if (!(d.omega > 0.0)) return 1.0;
    const double dz = (double)__uint_as_float(zbits) - d.theta;
    return exp(-(dz * dz) / (2.0 * d.omega * d.omega));
}

// Continuous alleles (Supplementary S2, phenotype value): the expressed
// phenotype of genetic value g (the sum of the loci's midpoints): plus
// noise_sd times the deviate of NOISE block `sub` of individual `index` in
// generation gen, then exp under the transform; rounded to float.
__device__ __forceinline__ float phenotype_cont(const RepDesc &d, const Rng &rng, double g, uint32_t index,
                                                uint32_t gen, uint32_t sub) {
    double z = g;
    if (d.noise_sd > 0.0) z += d.noise_sd * normal_of(rng.block(index, kStNoise, sub, gen));
    if (d.exp_tf) z = exp(z);
    return (float)z;
}

// Physiology regime (Supplementary S2).  Resource scarcity h(R, K) = x /
// (1 + T_H x), x = a R / K.
__device__ __forceinline__ double resource_h(const RepDesc &d, double R, double K) {
    const double x = d.attack * R / K;
    return x / (1.0 + d.handling * x);
}

// One time step of adult i's consumption and growth (S2, Resource
// Consumption and Somatic Growth): intake alpha W^gamma shared between the
// resources by the diet share logistic in W^(1/3), each cut by its h; the
// surplus over metabolism delta W to X in the share min(1, kappa Y/X), a
// deficit from Y; at a breeding step a mature individual's reserves above
// q_A X become gonads.  Updates X, Y; returns the gonads; adds the
// consumption to e1, e2.
__device__ __forceinline__ double phys_grow(const RepDesc &d, double h1, double h2, bool breeding, double &X,
                                            double &Y, double &e1, double &e2) {
    const double W = X + Y;
    const double pi1 = 1.0 / (1.0 + exp(-d.steepness * (cbrt(W) - d.ulmax)));
    const double intake = d.alpha * pow(W, d.gamma);
    const double c1 = h1 * pi1 * intake, c2 = h2 * (1.0 - pi1) * intake;
    const double dW = c1 + c2 - d.delta * W;
    e1 += c1;
    e2 += c2;
    if (dW > 0.0) {
        double f = d.kappa * Y / X;
        if (f > 1.0) f = 1.0;
        X += f * dW;
        Y += (1.0 - f) * dW;
    } else {
        Y += dW;
    }
    double G = 0.0;
    if (breeding && X >= d.maturity) {
        G = Y - d.qA * X;
        if (G < 0.0) G = 0.0;
        Y -= G;
    }
    return G;
}

// S2, Mortality: (1 - exp(-beta_s Y/X)) / (1 + exp(-beta_2 (X - beta_1))),
// 0 without reserves.
__device__ __forceinline__ double phys_survival(const RepDesc &d, double X, double Y) {
    if (!(Y > 0.0)) return 0.0;
    return (1.0 - exp(-d.beta_s * Y / X)) / (1.0 + exp(-d.beta2 * (X - d.beta1)));
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Additive effect sum_l e_l b_l, accumulated word by word.  With the
// offset effects e_l + 4 in [0, 8] held as four bit-planes Q_k (bit k of
// e_l + 4, W words each), sum_l e_l b_l = sum_k 2^k popc(g & Q_k) - 4 popc(g):
// per word four and-popcount pairs and one popcount into counters; the
// weights are applied once (unit effects: the popcount alone).
struct EffectSum {
    uint32_t ones = 0, q[4] = {0, 0, 0, 0};
    __device__ __forceinline__ void add(bool unit, const uint32_t *Q, uint32_t W, uint32_t w, uint32_t g) {
        ones += __popc(g);
        if (!unit) {
#pragma unroll
            for (int k = 0; k < 4; ++k) q[k] += __popc(g & Q[k * W + w]);
        }
    }
    __device__ __forceinline__ int32_t value(bool unit) const {
        if (unit) return (int32_t)ones;
        return (int32_t)(q[0] + 2u * q[1] + 4u * q[2] + 8u * q[3]) - 4 * (int32_t)ones;
    }
};

template <int V>
struct Words {
    uint32_t v[V];
};

// Device memory reached through pointers read from descriptors is accessed
// through the global address space, so loads and stores compile to global
// instructions: flat ones also count against the LDS wait counter, and every
// cross-lane or LDS wait would then wait for them too.
#define SPEGG_GLOBAL __attribute__((address_space(1)))

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ T gload(const T *p) {
    return *(const SPEGG_GLOBAL T *)p;
}

template <typename T>
__device__ __forceinline__ void gstore(T *p, const T &v) {
    *(SPEGG_GLOBAL T *)p = v;
}

template <int V>
__device__ __forceinline__ Words<V> load_words(const uint32_t *p) {
    Words<V> w;
    if constexpr (V == 4) {
        const u32x4 q = gload(reinterpret_cast<const u32x4 *>(p));
        w.v[0] = q.x;
        w.v[1] = q.y;
        w.v[2] = q.z;
        w.v[3] = q.w;
    } else if constexpr (V == 2) {
        const u32x2 q = gload(reinterpret_cast<const u32x2 *>(p));
        w.v[0] = q.x;
        w.v[1] = q.y;
    } else {
        w.v[0] = gload(p);
    }
    return w;
}

// Stores that do not allocate in L2 (newborn genomes: written once per
// generation and gathered by the next, so an L2 copy only costs the write-back
// of dirty lines when the kernel ends).
template <int V>
__device__ __forceinline__ void store_words_nt(uint32_t *p, const Words<V> &w) {
    if constexpr (V == 4) {
        __builtin_nontemporal_store(u32x4{w.v[0], w.v[1], w.v[2], w.v[3]}, (SPEGG_GLOBAL u32x4 *)p);
    } else if constexpr (V == 2) {
        __builtin_nontemporal_store(u32x2{w.v[0], w.v[1]}, (SPEGG_GLOBAL u32x2 *)p);
    } else {
        __builtin_nontemporal_store(w.v[0], (SPEGG_GLOBAL uint32_t *)p);
    }
}

template <int V>
__device__ __forceinline__ void store_words(uint32_t *p, const Words<V> &w) {
    if constexpr (V == 4) {
        gstore(reinterpret_cast<u32x4 *>(p), u32x4{w.v[0], w.v[1], w.v[2], w.v[3]});
    } else if constexpr (V == 2) {
        gstore(reinterpret_cast<u32x2 *>(p), u32x2{w.v[0], w.v[1]});
    } else {
        gstore(p, w.v[0]);
    }
}

// Smallest k with x < T[k] in a table in device memory (global loads).
__device__ __forceinline__ uint32_t table_draw_global(const uint64_t *__restrict__ T, uint32_t len, uint32_t x) {
    if ((uint64_t)x < gload(T)) return 0;
    uint32_t lo = 1, hi = len - 1;  // answer in [lo, hi]
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((uint64_t)x < gload(T + mid)) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// Geometric gap of word x (the smallest k with x < T_k, or len): T is the
// block's LDS copy of the gap table up to its first threshold of 2^32, whose
// entries all fit 32 bits (len >= 1).  A float guess floor(log2(1 - x/2^32) /
// log2(1 - r)), with 2^32 - x = ~x + 1, is checked against its two table
// neighbours and corrected when it is off, so the table alone decides.
__device__ __forceinline__ uint32_t geometric_gap(const uint32_t *T, uint32_t len, float scale, uint32_t x) {
    const float lg = __log2f((float)(~x) + 1.0f) - 32.0f;
    const float guess = lg * scale;
    const uint32_t g = guess >= (float)len ? len : (guess > 0.0f ? (uint32_t)guess : 0u);
    // both neighbours read unconditionally (indices clamped into the table,
    // which holds at least one threshold)
    const uint32_t t_lo = T[g == 0 ? 0u : g - 1u], t_hi = T[g < len ? g : len - 1u];
    const bool low_ok = g == 0 || t_lo <= x;
    const bool high_ok = g == len || x < t_hi;
    return (low_ok && high_ok) ? g : geometric_gap_fix(T, len, g, x);
}

// Four bit planes of U (the components of Philox block b, planes p0 ..
// p0 + 3 counted from the top) against R's bits at the same places, for the
// 32 boundaries of a word at once: where R's bit is 1 an undecided boundary
// with a 0 in U has U < R (a crossover), one with a 1 stays undecided; where
// R's bit is 0 a 1 in U decides U > R and a 0 stays undecided.  R is
// wave-uniform, so each bit's all-ones-or-zero mask is a scalar and every
// update one three-input bit operation.
__device__ __forceinline__ void planes_uniform(const Words4 &b, uint32_t R, int p0, uint32_t &und, uint32_t &hit) {
    uint32_t t[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t x = b.v[q];
        const uint32_t one = (uint32_t)((int32_t)(R << (p0 + q)) >> 31);  // ~0 where R's bit is 1
        t[q] = und & ~x & one;
        und &= ~(x ^ one);
    }
    hit |= t[0] | t[1] | t[2] | t[3];
}

// Index of the current census pair: the one with the larger generation.
__device__ __forceinline__ uint32_t current_pair(const RepState &st) {
    return (int32_t)(st.t[1] - st.t[0]) > 0 ? 1u : 0u;
}

// IT consecutive 16-bit fates (IT = 1, 2 or 4), one access.
template <int IT>
__device__ __forceinline__ void store_fates(uint16_t *p, const uint32_t *f) {
    if constexpr (IT == 4) {
        gstore(reinterpret_cast<u32x2 *>(p), u32x2{f[0] | (f[1] << 16), f[2] | (f[3] << 16)});
    } else if constexpr (IT == 2) {
        gstore(reinterpret_cast<uint32_t *>(p), f[0] | (f[1] << 16));
    } else {
        gstore(p, (uint16_t)f[0]);
    }
}

template <int IT>
__device__ __forceinline__ void load_fates(const uint16_t *p, uint32_t *f) {
    if constexpr (IT == 4) {
        const u32x2 w = gload(reinterpret_cast<const u32x2 *>(p));
        f[0] = w.x & 0xFFFFu;
        f[1] = w.x >> 16;
        f[2] = w.y & 0xFFFFu;
        f[3] = w.y >> 16;
    } else if constexpr (IT == 2) {
        const uint32_t w = gload(reinterpret_cast<const uint32_t *>(p));
        f[0] = w & 0xFFFFu;
        f[1] = w >> 16;
    } else {
        f[0] = gload(p);
    }
}

// IT consecutive 8-bit age classes, packed into one word.
template <int IT>
__device__ __forceinline__ uint32_t load_ages(const uint8_t *p) {
    if constexpr (IT == 4) return gload(reinterpret_cast<const uint32_t *>(p));
    else if constexpr (IT == 2) return gload(reinterpret_cast<const uint16_t *>(p));
    else return gload(p);
}

// Linkage map: the crossovers of 32-boundary word w of a gamete (bit b:
// boundary 32w + b), each boundary's uniform U compared bit by bit against
// its own threshold R_b from the top, U's plane p from bit b of word p % 4 of
// RECOMB block 1 + 8w + p / 4; a boundary is decided at the first plane where
// U and R_b differ (U < R_b: a crossover) or once R_b has no 1 bit left.
__device__ __forceinline__ uint32_t map_word(const Rng &rng, uint32_t j, uint32_t rs, uint32_t tp,
                                             const uint32_t *__restrict__ map, uint32_t w) {
    const uint32_t *m = map + (size_t)w * kMapWords;
    uint32_t und = gload(m + 64), hit = 0;
    for (uint32_t k = 0; und != 0 && k < 8u; ++k) {
        const Words4 b = rng.block(j, rs, 1u + w * 8u + k, tp);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t p = 4u * k + (uint32_t)q;
            const uint32_t one = gload(m + p), x = b.v[q];
            hit |= und & ~x & one;
            und &= ~(x ^ one) & gload(m + 32u + p);
        }
    }
    return hit;
}

// Mate choice: the threshold floor(a 2^32) of a mother (adult m) accepting
// candidate c, from the host table for integer phenotypes (shared
// preference by z, assortment by |z_m - z_c|) or computed in double for
// continuous ones; cur is the adults' buffer.
__device__ __forceinline__ uint64_t choice_threshold(const RepDesc &d, uint32_t cur, uint32_t c, uint32_t m) {
    if (d.cont) {
        const float *zf = reinterpret_cast<const float *>(d.z[cur]);
        const double dz = d.mating == SPEGG_PREFERENCE ? (double)gload(zf + c) - d.pref_opt
                                                       : (double)gload(zf + m) - (double)gload(zf + c);
        const double a = exp(-(dz * dz) / (2.0 * d.pref_w * d.pref_w));
        return a >= 1.0 ? kAlways : (a > 0.0 ? (uint64_t)floor(a * 4294967296.0) : 0ull);
    }
    const int32_t zc = gload(d.z[cur] + c);
    if (d.mating == SPEGG_PREFERENCE) return gload(d.choiceT + (zc - d.choice_zmin));
    const int32_t dz = gload(d.z[cur] + m) - zc;
    return gload(d.choiceT + (dz < 0 ? -dz : dz));
}

// A parent by proposals, the TPO lanes of a team (lane `lane`, the team's
// first wave lane seg0) testing proposals p0 + lane at once: proposal p is
// survivor S[idx(words 0, 1)] of block p of `stream` for index `key`,
// accepted when it has the wanted sex (want_sex 0 / 1; -1: any) and, with
// choice, word 2 lies below its mate-choice threshold for mother `mom`; the
// lowest accepted p wins.  After kPartnerProposals rejections: the first
// survivor of the wanted sex at or after the last proposal in survivor order
// (wrapping), or the last proposal when any sex will do.  Every lane of the
// team returns the same adult index.
template <uint32_t TPO>
__device__ uint32_t team_partner(const RepDesc &d, const Rng &rng, uint32_t stream, uint32_t key, uint32_t tp,
                                 uint32_t cur, int want_sex, bool choice, uint32_t mom, uint32_t ns, uint32_t lane,
                                 uint32_t seg0) {
    constexpr uint64_t tmask = TPO >= 64 ? ~0ull : ((1ull << TPO) - 1ull);
    const uint8_t *sex = d.sex[cur];
    uint32_t last = 0;
    for (uint32_t p0 = 0; p0 < kPartnerProposals; p0 += TPO) {
        const Words4 b = rng.block(key, stream, p0 + lane, tp);
        const uint32_t r = uniform_index(b.v[0], b.v[1], ns);
        const uint32_t c = gload(d.S + r);
        bool ok = want_sex < 0 || (int)gload(sex + c) == want_sex;
        if (ok && choice) ok = (uint64_t)b.v[2] < choice_threshold(d, cur, c, mom);
        const uint64_t seg = (__ballot(ok) >> seg0) & tmask;
        if (seg) return (uint32_t)__shfl((int)c, (int)__ffsll((unsigned long long)seg) - 1, (int)TPO);
        last = (uint32_t)__shfl((int)r, (int)TPO - 1, (int)TPO);
    }
    if (want_sex < 0) return gload(d.S + last);
    // the team scans survivor ranks from the last proposal, TPO at a time
    for (uint32_t q0 = 0; q0 < ns; q0 += TPO) {
        const uint32_t q = q0 + lane;
        uint32_t c = 0;
        bool ok = false;
        if (q < ns) {
            c = gload(d.S + (last + q) % ns);
            ok = (int)gload(sex + c) == want_sex;
        }
        const uint64_t seg = (__ballot(ok) >> seg0) & tmask;
        if (seg) return (uint32_t)__shfl((int)c, (int)__ffsll((unsigned long long)seg) - 1, (int)TPO);
    }
    return gload(d.S + last);  // unreachable: the wanted sex survived
}

// Physiology regime (S2, Reproduction): a mother among the mature
// surviving females in proportion to her eggs^v_f, a father among the mature
// surviving males in proportion to X^v_m, by proposals as in team_partner:
// proposal p accepted when eligible and word 2 lies below floor((w /
// w_max)^v 2^32), w_max the step's largest weight (from compact).  After
// kPartnerProposals rejections: the first eligible survivor at or after the
// last proposal.  cur is the adults' buffer (masses grown in place).
template <uint32_t TPO>
__device__ uint32_t team_phys_partner(const RepDesc &d, const RepState &st, const Rng &rng, uint32_t stream,
                                      uint32_t key, uint32_t tp, uint32_t cur, uint32_t male, uint32_t ns,
                                      uint32_t lane, uint32_t seg0) {
    constexpr uint64_t tmask = TPO >= 64 ? ~0ull : ((1ull << TPO) - 1ull);
    const double v = male ? d.v_m : d.v_f, wmax = male ? st.xmax : st.emax;
    const float *zf = reinterpret_cast<const float *>(d.z[cur]);
    uint32_t last = 0;
    for (uint32_t p0 = 0; p0 < kPartnerProposals; p0 += TPO) {
        const Words4 b = rng.block(key, stream, p0 + lane, tp);
        const uint32_t r = uniform_index(b.v[0], b.v[1], ns);
        const uint32_t c = gload(d.S + r);
        const double X = gload(d.X[cur] + c);
        bool ok = gload(d.sex[cur] + c) == male && X >= d.maturity;
        if (ok) {
            double w = X;
            if (!male) {
                const double om = (double)gload(zf + c);
                w = gload(d.G + c) / (om + d.qJ * om);
            }
            double a = w / wmax;
            if (v != 1.0) a = pow(a, v);
            const uint64_t T = a >= 1.0 ? kAlways : (a > 0.0 ? (uint64_t)floor(a * 4294967296.0) : 0ull);
            ok = (uint64_t)b.v[2] < T;
        }
        const uint64_t seg = (__ballot(ok) >> seg0) & tmask;
        if (seg) return (uint32_t)__shfl((int)c, (int)__ffsll((unsigned long long)seg) - 1, (int)TPO);
        last = (uint32_t)__shfl((int)r, (int)TPO - 1, (int)TPO);
    }
    for (uint32_t q0 = 0; q0 < ns; q0 += TPO) {
        const uint32_t q = q0 + lane;
        uint32_t c = 0;
        bool ok = false;
        if (q < ns) {
            c = gload(d.S + (last + q) % ns);
            ok = gload(d.sex[cur] + c) == male && gload(d.X[cur] + c) >= d.maturity;
        }
        const uint64_t seg = (__ballot(ok) >> seg0) & tmask;
        if (seg) return (uint32_t)__shfl((int)c, (int)__ffsll((unsigned long long)seg) - 1, (int)TPO);
    }
    return gload(d.S + last);  // unreachable: an eligible parent survived
}

// Words of one stream of one individual read in order, one Philox block
// per four words.
struct SeqWords {
    Rng rng;
    uint32_t index, stream, gen;
    uint32_t blk;
    Words4 w;
    __device__ __forceinline__ SeqWords(const Rng &r, uint32_t i, uint32_t st, uint32_t g)
        : rng(r), index(i), stream(st), gen(g), blk(~0u) {}
    __device__ __forceinline__ uint32_t operator()(uint32_t q) {
        if ((q >> 2) != blk) {
            blk = q >> 2;
            w = rng.block(index, stream, blk, gen);
        }
        const uint32_t c = q & 3u;
        return c == 0 ? w.v[0] : c == 1 ? w.v[1] : c == 2 ? w.v[2] : w.v[3];
    }
};

// Consumer-resource regime: the encounters of consumer i.  Each lands on a
// uniform slot of the habitat (at least the resource census NR) and meets
// the resource of that index if there is one; it captures it when its
// CAPTURE word is below the matching threshold.  f(e, target) is called
// for every capture.  Encounters go eight at a time, so that their resource
// gathers are in flight together; capT is the capture table (in LDS where
// it fits).
constexpr uint32_t kEncounterBatch = 8;
template <typename F>
__device__ __forceinline__ void consumer_captures(const RepDesc &c, uint32_t i, uint32_t t, int32_t zc,
                                                  const int32_t *__restrict__ zr, uint32_t NR,
                                                  const uint64_t *capT, F &&f) {
    if (NR == 0) return;
    const Rng rng{c.key0, c.key1, c.c3};
    SeqWords enc(rng, i, kStEncounter, t), cap(rng, i, kStCapture, t);
    const uint32_t ne = table_draw_global(c.enc, c.enc_len, enc(0));
    const uint32_t span = c.habitat > NR ? c.habitat : NR;
    for (uint32_t e0 = 0; e0 < ne; e0 += kEncounterBatch) {
        uint32_t tgt[kEncounterBatch];
        int32_t z[kEncounterBatch];
#pragma unroll
        for (uint32_t q = 0; q < kEncounterBatch; ++q) {
            const uint32_t e = e0 + q;
            tgt[q] = ~0u;
            if (e < ne) {
                const uint32_t lo = enc(1u + 2u * e), hi = enc(2u + 2u * e);
                tgt[q] = uniform_index(lo, hi, span);
            }
            z[q] = tgt[q] < NR ? gload(zr + tgt[q]) : 0;
        }
#pragma unroll
        for (uint32_t q = 0; q < kEncounterBatch; ++q) {
            const uint32_t e = e0 + q;
            if (e >= ne || tgt[q] >= NR) continue;
            const int32_t dz = zc - z[q];
            const uint32_t d = (uint32_t)(dz < 0 ? -dz : dz);
            if ((uint64_t)cap(e) < capT[d]) f(e, tgt[q]);
        }
    }
}

__device__ __forceinline__ uint64_t capture_key(uint32_t i, uint32_t e) { return ((uint64_t)i << 32) | e; }

// Binomial(n, q) thresholds from IEEE double basic operations: P(k) =
// C(n, k) q^k (1-q)^(n-k), the coefficient by C(n, k) = C(n, k-1)(n-k+1)/k,
// the powers by repeated multiplication, F accumulated in order; the table
// closes at the first threshold reaching 2^32 - 1, or at k = n.
__device__ uint32_t small_binomial_table(uint32_t n, double q, uint64_t *T) {
    const double u = 1.0 - q;
    double c = 1.0, F = 0.0;
    for (uint32_t k = 0; k <= n; ++k) {
        if (k > 0) c = c * (double)(n - k + 1u) / (double)k;
        double pk = c;
        for (uint32_t m = 0; m < k; ++m) pk = pk * q;
        for (uint32_t m = 0; m < n - k; ++m) pk = pk * u;
        F = F + pk;
        const uint64_t thr = F >= 1.0 ? kAlways : (F > 0.0 ? (uint64_t)floor(F * 4294967296.0) : 0ull);
        if (thr >= 4294967295ull || k == n) {
            T[k] = kAlways;
            return k + 1;
        }
        T[k] = thr;
    }
    return n + 1;
}

// ---------------------------------------------------------------- init

// The initial population of every deme in one launch, one thread per
// individual slot of a survival tile: the individual's 2W genome words (fair
// bits: word q is word q % 4 of Philox block q / 4 of stream INIT for the
// individual; bits of word W-1 past locus L-1 cleared), its phenotype, and
// the census sums of integer phenotypes (spread over the state's slots;
// continuous phenotypes are summed on demand).  Consumer-resource demes also
// start with age class 0 and no capture keys.
__global__ void __launch_bounds__(kBlock) create_kernel(const RepDesc *__restrict__ descs,
                                                        RepState *__restrict__ states,
                                                        const SurvTile *__restrict__ tiles) {
    const SurvTile tile = tiles[blockIdx.x];
    const RepDesc &d = descs[tile.rep];
    RepState &st = states[tile.rep];
    const uint32_t n0 = st.n[0];
    const Rng rng{d.key0, d.key1, d.c3};
    const uint32_t W = d.W, per = 2u * W;
    const bool unit = d.unit_effects != 0;
    int64_t sz = 0;
    uint64_t sz2 = 0;
    if (d.cont) {
        // Continuous alleles: allele (h, l) is N(a0, s0^2) from INIT block
        // h L + l of the individual, rounded to float; the pad loci are 0.
        // The genetic value is summed locus by locus in order.  Physiology
        // regime: founder i in storage slot i, the free stack holding the
        // slots above n0 with n0 on top.
        for (uint32_t slot = threadIdx.x; slot < d.surv_tile; slot += kBlock) {
            const uint32_t i = tile.start + slot;
            if (d.gfree && i < d.cap) {
                if (i < n0) gstore(d.gslot[0] + i, i);
                else gstore(d.gfree + (d.cap - 1u - i), i);
            }
            if (i >= n0) continue;
            float *g = reinterpret_cast<float *>(d.genome[0] + (size_t)i * per);
            double gv = 0.0;
            for (uint32_t l = 0; l < W; ++l) {
                float a = 0.0f, b = 0.0f;
                if (l < d.L) {
                    a = (float)(d.a0 + d.s0 * normal_of(rng.block(i, kStInit, l, 0)));
                    b = (float)(d.a0 + d.s0 * normal_of(rng.block(i, kStInit, d.L + l, 0)));
                    gv += 0.5 * ((double)a + (double)b);
                }
                gstore(g + l, a);
                gstore(g + W + l, b);
            }
            const float z = phenotype_cont(d, rng, gv, i, 0, 1);
            gstore(d.z[0] + i, (int32_t)__float_as_uint(z));
            if (d.sexes) gstore(d.sex[0] + i, (uint8_t)(rng.block(i, kStSex, 1, 0).v[0] & 1u));
            if (d.X[0]) {  // physiology regime: born at its own neonate mass
                gstore(d.X[0] + i, (double)z);
                gstore(d.Y[0] + i, d.qJ * (double)z);
            }
        }
        return;  // the census sums are folded on demand, in a fixed order (the state says so)
    }
    for (uint32_t slot = threadIdx.x; slot < d.surv_tile; slot += kBlock) {
        const uint32_t i = tile.start + slot;  // below the deme's whole tiles
        if (d.regime == SPEGG_CONSUMER_RESOURCE) {
            gstore(d.age[0] + i, (uint8_t)0);
            gstore(d.age[1] + i, (uint8_t)0);
            if (d.won && i < d.cap) gstore(d.won + i, (uint64_t)~0ull);
        }
        if (i < n0) {
            uint32_t *g = d.genome[0] + (size_t)i * per;
            EffectSum es;
            for (uint32_t q0 = 0; q0 < per; q0 += 4) {
                const Words4 blk = rng.block(i, kStInit, q0 >> 2, 0);
#pragma unroll
                for (uint32_t c = 0; c < 4; ++c) {
                    const uint32_t q = q0 + c, w = q % W;
                    if (q < per) {
                        const uint32_t word = w == W - 1 ? blk.v[c] & d.tail_mask : blk.v[c];
                        gstore(g + q, word);
                        es.add(unit, d.planes, W, w, word);
                    }
                }
            }
            const int64_t z = (int64_t)es.value(unit) - d.sum_e;
            gstore(d.z[0] + i, (int32_t)z);
            if (d.sexes) gstore(d.sex[0] + i, (uint8_t)(rng.block(i, kStSex, 1, 0).v[0] & 1u));
            sz += z;
            sz2 += (uint64_t)(z * z);
        }
    }
    sz = wave_sum<int64_t>(sz);
    sz2 = wave_sum<uint64_t>(sz2);
    if (lane_id() == 0 && (sz != 0 || sz2 != 0)) {
        const uint32_t slot = blockIdx.x % kCensusSlots;
        atomicAdd((unsigned long long *)&st.sum_z[slot], (unsigned long long)sz);
        atomicAdd((unsigned long long *)&st.sum_z2[slot], (unsigned long long)sz2);
    }
}

__global__ void __launch_bounds__(kBlock) phenotype_kernel(const RepDesc *__restrict__ desc,
                                                           RepState *__restrict__ state, uint32_t n, uint32_t buf,
                                                           uint32_t gen) {
    const RepDesc &d = *desc;
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (d.cont) {
        // continuous alleles written by the caller: founders of generation gen
        if (i < n) {
            // physiology regime: written individual i sits in storage slot i
            const float *g = reinterpret_cast<const float *>(d.genome[d.gfree ? 0u : buf] + (size_t)i * 2u * d.W);
            double gv = 0.0;
            for (uint32_t l = 0; l < d.L; ++l) gv += 0.5 * ((double)g[l] + (double)g[d.W + l]);
            const Rng rng{d.key0, d.key1, d.c3};
            const float z = phenotype_cont(d, rng, gv, i, gen, 1);
            d.z[buf][i] = (int32_t)__float_as_uint(z);
            if (d.sexes) d.sex[buf][i] = (uint8_t)(rng.block(i, kStSex, 1, gen).v[0] & 1u);
            if (d.X[0]) {
                d.X[buf][i] = (double)z;
                d.Y[buf][i] = d.qJ * (double)z;
            }
        }
        return;  // the census sums are folded on demand, in a fixed order (the state says so)
    }
    int64_t z = 0;
    if (i < n) {
        const uint32_t *g = d.genome[buf] + (size_t)i * 2u * d.W;
        EffectSum es;
        for (uint32_t w = 0; w < d.W; ++w) {
            es.add(d.unit_effects, d.planes, d.W, w, g[w]);
            es.add(d.unit_effects, d.planes, d.W, w, g[d.W + w]);
        }
        z = (int64_t)es.value(d.unit_effects) - d.sum_e;
        d.z[buf][i] = (int32_t)z;
        if (d.sexes) {
            const Rng rng{d.key0, d.key1, d.c3};
            d.sex[buf][i] = (uint8_t)(rng.block(i, kStSex, 1, gen).v[0] & 1u);
        }
    }
    const int64_t sz = wave_sum<int64_t>(z);
    const uint64_t sz2 = wave_sum<uint64_t>((uint64_t)(z * z));
    if (lane_id() == 0 && (sz != 0 || sz2 != 0)) {
        const uint32_t slot = blockIdx.x % kCensusSlots;
        atomicAdd((unsigned long long *)&state->sum_z[slot], (unsigned long long)sz);
        atomicAdd((unsigned long long *)&state->sum_z2[slot], (unsigned long long)sz2);
    }
}

// ---------------------------------------------------------------- survive

// One block per tile of kBlock x IT adults; thread x holds the IT
// consecutive adults from tile start + x IT (z and fate buffers are padded to
// whole tiles, so the vector accesses stay inside).
// The tile's global index gi is the block index in a launch of one block per
// tile; a block that walks a list of tiles derives it from the tile.
template <int IT, bool LIST>
__device__ __forceinline__ void survive_tile(const RepDesc *__restrict__ descs, const RepState *__restrict__ states,
                                             const SurvTile tile, SurvCount *__restrict__ counts,
                                             SurvGroup *__restrict__ groups) {
    // the thread index, opaque to the compiler in a list-walking loop: no
    // value derived from it is hoisted out of the loop and held across tiles
    uint32_t tid = threadIdx.x;
    if (LIST) asm volatile("" : "+v"(tid));
    __shared__ uint32_t sh_a[kBlock / 64], sh_k[kBlock / 64], sh_n[kBlock / 64], sh_i[kBlock / 64];
    __shared__ uint32_t sh_f[kBlock / 64];
    __shared__ uint64_t sh_t[kBlock / 64];
    __shared__ uint64_t sh_pois[kPoissonTableCap];
    const RepDesc &d = descs[tile.rep];
    const uint32_t gi = LIST ? d.surv_tile0 + tile.start / (uint32_t)(kBlock * IT) : blockIdx.x;
    // Both phenotype buffers (padded to whole tiles) are read with the census
    // state, which alone says which one holds the census: no load waits for it.
    const uint32_t i0 = tile.start + tid * IT;
    const Words<IT> zw0 = load_words<IT>(reinterpret_cast<const uint32_t *>(d.z[0]) + i0);
    const Words<IT> zw1 = load_words<IT>(reinterpret_cast<const uint32_t *>(d.z[1]) + i0);
    const RepState &st = states[tile.rep];
    const uint32_t par = current_pair(st);
    const uint32_t t = st.t[par], n = st.n[par];
    // beyond the census: uniform over the block; tile 0 always records the census
    if (tile.start >= n && tile.start != 0) return;
    const bool poisson = d.regime == SPEGG_POISSON_BH;
    const bool cr = d.regime == SPEGG_CONSUMER_RESOURCE;
    const Words<IT> zw = (t & 1u) ? zw1 : zw0;
    __shared__ uint32_t sh_tlen;
    uint32_t tlen = d.pois_len;  // length of the table in sh_pois
    if (poisson) {
        for (uint32_t q = tid; q < d.pois_len; q += kBlock) sh_pois[q] = gload(d.pois + q);
        __syncthreads();
    } else if (cr && d.species == 0) {
        // the resource's offspring table of this generation's density
        if (tid == 0) {
            const double x = 1.0 - (double)n / d.KR;
            sh_tlen = small_binomial_table(d.trials, d.q0 * (x > 0.0 ? x : 0.0), sh_pois);
        }
        __syncthreads();
        tlen = sh_tlen;
    }
    const double s = density_factor(d, n);
    const Rng rng{d.key0, d.key1, d.c3};
    const bool phys = d.regime == SPEGG_PHYSIOLOGY;
    const bool breeding = phys && t % d.breed_every == d.breed_every - 1u;
    double h1 = 0.0, h2 = 0.0, pe1 = 0.0, pe2 = 0.0, peggs = 0.0, pemax = 0.0, pxmax = 0.0;
    uint32_t pnf = 0, pnm = 0;
    if (phys) {
        h1 = resource_h(d, st.R[0], d.KR2[0]);
        h2 = resource_h(d, st.R[1], d.KR2[1]);
    }
    double v[IT];
#pragma unroll
    for (uint32_t q = 0; q < IT; ++q)
        v[q] = (d.vtab && i0 + q < n) ? gload(d.vtab + ((int32_t)zw.v[q] - d.zmin))
               : (d.cont && i0 + q < n) ? viability_cont(d, zw.v[q])
                                        : 1.0;
    uint32_t age4 = 0, sex4 = 0;
    if (cr) age4 = load_ages<IT>(d.age[t & 1u] + i0);
    if (d.sexes) sex4 = load_ages<IT>(d.sex[t & 1u] + i0);  // 0 female, 1 male per byte
    uint32_t fate[IT], a_loc = 0, k_loc = 0, near = 0, in_loc = 0, f_loc = 0;
    uint64_t thr_sum = 0;
#pragma unroll
    for (uint32_t q = 0; q < IT; ++q) {
        const uint32_t i = i0 + q;
        fate[q] = 0;
        if (i < n) {
            uint32_t intake = 0;
            bool captured = false;
            double p = v[q] * s;
            double PX = 0.0, PY = 0.0, PG = 0.0;
            if (phys) {
                // grow on this step's resources, in place; survival from the new masses
                PX = gload(d.X[t & 1u] + i);
                PY = gload(d.Y[t & 1u] + i);
                PG = phys_grow(d, h1, h2, breeding, PX, PY, pe1, pe2);
                gstore(d.X[t & 1u] + i, PX);
                gstore(d.Y[t & 1u] + i, PY);
                gstore(d.G + i, PG);
                p = phys_survival(d, PX, PY);
            }
            if (cr) {
                p = v[q] * d.surv_age[(age4 >> (8u * q)) & 3u];
                if (d.species == 0) {
                    captured = gload(d.won + i) != ~0ull;
                } else {
                    // credited captures: those whose resource kept this
                    // consumer's key (counted by credit_kernel)
                    intake = gload(d.intake + i);
                    in_loc += intake;
                }
            }
            if (!captured) {
                const uint64_t thr = p >= 1.0 ? kAlways : (p > 0.0 ? (uint64_t)floor(p * 4294967296.0) : 0ull);
                const uint32_t x = rng.block(i, kStSurvive, 0, t).v[0];
                thr_sum += thr;
                near += (p > 0.0 && p < 1.0 && fabs((double)x * (1.0 / 4294967296.0) - p) < 1e-6) ? 1u : 0u;
                if ((uint64_t)x < thr) {
                    uint32_t kids = 0;
                    const bool male = d.sexes && ((sex4 >> (8u * q)) & 1u);
                    if (d.sexes && !male) ++f_loc;
                    if (phys && PX >= d.maturity) {
                        // eligible parents of a breeding step and their weights
                        if (male) {
                            ++pnm;
                            pxmax = fmax(pxmax, PX);
                        } else {
                            const double om = (double)__uint_as_float(zw.v[q]);
                            const double e = PG / (om + d.qJ * om);
                            ++pnf;
                            peggs += e;
                            pemax = fmax(pemax, e);
                        }
                    }
                    if (male) {
                        // separate sexes: only females are mothers
                    } else if (poisson || (cr && d.species == 0)) {
                        kids = table_draw(sh_pois, tlen, rng.block(i, kStFecund, 0, t).v[0]);
                    } else if (cr) {
                        const uint32_t off = gload(d.cpois_off + 2u * intake),
                                       len = gload(d.cpois_off + 2u * intake + 1u);
                        kids = table_draw_global(d.cpois + off, len, rng.block(i, kStFecund, 0, t).v[0]);
                    }
                    fate[q] = 0x8000u | kids;
                    ++a_loc;
                    k_loc += kids;
                }
            }
        }
    }
    // fates of the thread's adults, one store
    uint16_t *fp = d.fate + i0;
    store_fates<IT>(fp, fate);
    const uint32_t wave = tid >> 6;
    if (phys) {
        // the tile's consumption, eggs and largest weights (uniform over the block)
        __shared__ double sh_p[kBlock / 64][5];
        __shared__ uint32_t sh_pn[kBlock / 64][2];
        pe1 = wave_sum<double>(pe1);
        pe2 = wave_sum<double>(pe2);
        peggs = wave_sum<double>(peggs);
        pemax = wave_max(pemax);
        pxmax = wave_max(pxmax);
        pnf = wave_sum<uint32_t>(pnf);
        pnm = wave_sum<uint32_t>(pnm);
        if ((tid & 63u) == 0) {
            sh_p[wave][0] = pe1;
            sh_p[wave][1] = pe2;
            sh_p[wave][2] = peggs;
            sh_p[wave][3] = pemax;
            sh_p[wave][4] = pxmax;
            sh_pn[wave][0] = pnf;
            sh_pn[wave][1] = pnm;
        }
        __syncthreads();
        if (tid == 0) {
            PhysTile pt{};
            for (int w = 0; w < kBlock / 64; ++w) {
                pt.e[0] += sh_p[w][0];
                pt.e[1] += sh_p[w][1];
                pt.eggs += sh_p[w][2];
                pt.emax = fmax(pt.emax, sh_p[w][3]);
                pt.xmax = fmax(pt.xmax, sh_p[w][4]);
                pt.nf += sh_pn[w][0];
                pt.nm += sh_pn[w][1];
            }
            d.ptiles[gi - d.surv_tile0] = pt;
        }
    }
    const uint32_t wa = wave_sum<uint32_t>(a_loc), wk = wave_sum<uint32_t>(k_loc), wn = wave_sum<uint32_t>(near);
    const uint32_t wi = wave_sum<uint32_t>(in_loc);
    const uint32_t wf = wave_sum<uint32_t>(f_loc);
    const uint64_t wt = wave_sum<uint64_t>(thr_sum);
    if ((tid & 63u) == 0) {
        sh_a[wave] = wa;
        sh_k[wave] = wk;
        sh_n[wave] = wn;
        sh_i[wave] = wi;
        sh_f[wave] = wf;
        sh_t[wave] = wt;
    }
    __syncthreads();
    if (tid == 0) {
        SurvCount c{};
        for (int w = 0; w < kBlock / 64; ++w) {
            c.alive += sh_a[w];
            c.kids += sh_k[w];
            c.near += sh_n[w];
            c.intake += sh_i[w];
            c.alive_f += sh_f[w];
            c.sum_t += sh_t[w];
        }
        c.par = par;
        c.t = t;
        c.n = n;
        counts[gi] = c;
        // a census of more than one tile group: the tile's counts into its
        // group's sums as well
        const uint32_t active = (n + kBlock * IT - 1) / (kBlock * IT);
        if (active > kGroupTiles) {
            SurvGroup &g = groups[d.grp0 + (t & 1u) * d.grp_n + (gi - d.surv_tile0) / kGroupTiles];
            if (c.alive) atomicAdd(&g.alive, c.alive);
            if (c.kids) atomicAdd((unsigned long long *)&g.kids, (unsigned long long)c.kids);
            if (c.near) atomicAdd(&g.near, c.near);
            if (c.sum_t) atomicAdd((unsigned long long *)&g.sum_t, (unsigned long long)c.sum_t);
            if (c.intake) atomicAdd(&g.intake, c.intake);
            if (c.alive_f) atomicAdd(&g.alive_f, c.alive_f);
        }
    }
}

// One block per survival tile of the plan (a population of one deme has its
// tiles implicit: no load before the descriptor's).
template <int IT>
__global__ void __launch_bounds__(kBlock) survive_kernel(const RepDesc *__restrict__ descs,
                                                         const RepState *__restrict__ states,
                                                         const SurvTile *__restrict__ tiles,
                                                         SurvCount *__restrict__ counts,
                                                         SurvGroup *__restrict__ groups, int single_deme) {
    const SurvTile tile = single_deme >= 0 ? SurvTile{(uint32_t)single_deme, blockIdx.x * (uint32_t)(kBlock * IT)}
                                           : tiles[blockIdx.x];
    survive_tile<IT, false>(descs, states, tile, counts, groups);
}

// A resident grid over the list of this generation's occupied tiles (the
// tiles of the censuses, written by plan_tiles_kernel).
template <int IT>
__global__ void __launch_bounds__(kBlock) survive_list_kernel(const RepDesc *__restrict__ descs,
                                                              const RepState *__restrict__ states,
                                                              const SurvTile *__restrict__ list,
                                                              const uint32_t *__restrict__ list_n,
                                                              SurvCount *__restrict__ counts,
                                                              SurvGroup *__restrict__ groups) {
    const uint32_t m = *list_n;
    for (uint32_t v = blockIdx.x; v < m; v += gridDim.x) {
        survive_tile<IT, true>(descs, states, list[v], counts, groups);
        __syncthreads();  // the next tile reuses the block's LDS
    }
}

// ---------------------------------------------------------------- compact

// Consumer-resource and physiology regimes: survivor `from` of the census
// in buffers `cur` moves to position k of the next census (compact places it
// as it lists it) with its phenotype, its age class plus one, its sex and
// masses, and -- where the allelic values stay in place (physiology) -- its
// storage slot; a genome that moves is copied by compact's whole block.  A
// resource starts the next generation uncaptured.
__device__ __forceinline__ void carry_one(const RepDesc &d, uint32_t cur, uint32_t from, uint32_t k) {
    if (d.gfree) gstore(d.gslot[cur ^ 1u] + k, gload(d.gslot[cur] + from));
    d.z[cur ^ 1u][k] = d.z[cur][from];
    if (d.age[0]) {
        const uint32_t a = d.age[cur][from];
        d.age[cur ^ 1u][k] = (uint8_t)(a < 3u ? a + 1u : 3u);  // class 3 holds three and older
    }
    if (d.won) d.won[k] = ~0ull;
    if (d.sexes) d.sex[cur ^ 1u][k] = d.sex[cur][from];
    if (d.X[0]) {  // physiology regime: the grown masses
        d.X[cur ^ 1u][k] = d.X[cur][from];
        d.Y[cur ^ 1u][k] = d.Y[cur][from];
    }
}


// One block per tile: its prefix is summed from the counts of the
// replicate's earlier tiles (written by survive, a launch earlier), then
// block ranks place its survivors and its mothers' offspring slots.  Tile 0
// of each replicate sums all the tiles and advances the census.  A census
// of more than kGroupTiles tiles also has group sums (survive added each
// tile into its group): a tile then sums the earlier groups and the earlier
// tiles of its own group, at most one load per thread each.
template <int IT, bool LIST>
__device__ __forceinline__ void compact_tile(const RepDesc *__restrict__ descs, RepState *__restrict__ states,
                                             const SurvTile tile, const SurvCount *__restrict__ counts,
                                             SurvGroup *__restrict__ groups, int trace) {
    // the thread index, opaque to the compiler in a list-walking loop: no
    // value derived from it is hoisted out of the loop and held across tiles
    uint32_t tid = threadIdx.x;
    if (LIST) asm volatile("" : "+v"(tid));
    constexpr uint32_t TILE = kBlock * IT;
    __shared__ uint32_t sh_a[kBlock / 64], sh_k[kBlock / 64], sh_in[kBlock / 64], sh_f[kBlock / 64];
    __shared__ uint64_t sh_kk[kBlock / 64], sh_n[kBlock / 64], sh_t[kBlock / 64];
    const RepDesc &d = descs[tile.rep];
    RepState &st = states[tile.rep];
    // the thread's fates, in flight during the prefix (the buffer is padded
    // to whole tiles)
    const uint32_t i0 = tile.start + tid * IT;
    uint32_t fate[IT];
    load_fates<IT>(d.fate + i0, fate);
    const SurvCount *C = counts + d.surv_tile0;
    const uint32_t k = LIST ? tile.start / TILE : blockIdx.x - d.surv_tile0;  // tile index within the replicate
    const uint32_t kg0 = k - k % kGroupTiles;      // first tile of its group
    // exclusive prefix of this tile (tile 0: the totals, with the census
    // statistics only it records).  Past tile 0 the tiles of its own group
    // before it are known from the block index: those loads go out with the
    // census header's.
    uint32_t pa = 0, pi = 0, pf = 0;
    uint64_t pk = 0, pn = 0, pt = 0;
    if (k != 0 && tid < k - kg0) {
        const SurvCount c = C[kg0 + tid];
        pa += c.alive;
        pk += c.kids;
    }
    // the census this generation started from, as survive recorded it: tile 0
    // of this launch rewrites the state's other pair
    const SurvCount c0 = C[0];
    const uint32_t par = c0.par, t = c0.t, n = c0.n;
    const uint32_t active = (n + TILE - 1) / TILE;
    if (k >= active && k != 0) return;  // beyond the census: uniform over the block
    const bool grouped = active > kGroupTiles;
    const SurvGroup *G = groups + d.grp0 + (t & 1u) * d.grp_n;
    const uint32_t wave = tid >> 6;
    if (k == 0) {
        if (grouped) {
            for (uint32_t q = tid; q * kGroupTiles < active; q += kBlock) {
                const SurvGroup g = G[q];
                pa += g.alive;
                pk += g.kids;
                pn += g.near;
                pt += g.sum_t;
                pi += g.intake;
                pf += g.alive_f;
            }
        } else {
            for (uint32_t q = tid; q < active; q += kBlock) {
                const SurvCount c = C[q];
                pa += c.alive;
                pk += c.kids;
                pn += c.near;
                pt += c.sum_t;
                pi += c.intake;
                pf += c.alive_f;
            }
        }
        // The other parity's group sums start the next generation from zero,
        // whether or not this census used groups (a later census of the
        // same parity may).
        SurvGroup *Gn = groups + d.grp0 + ((t + 1u) & 1u) * d.grp_n;
        for (uint32_t q = tid; q < d.grp_n; q += kBlock) Gn[q] = SurvGroup{0, 0, 0, 0, 0, 0};
    } else {
        for (uint32_t q = tid; q < kg0 / kGroupTiles; q += kBlock) {  // the earlier groups
            const SurvGroup g = G[q];
            pa += g.alive;
            pk += g.kids;
        }
    }
    pa = wave_sum<uint32_t>(pa);
    pk = wave_sum<uint64_t>(pk);
    if (k == 0) {  // uniform over the block
        pi = wave_sum<uint32_t>(pi);
        pf = wave_sum<uint32_t>(pf);
        pn = wave_sum<uint64_t>(pn);
        pt = wave_sum<uint64_t>(pt);
    }
    if ((tid & 63u) == 0) {
        sh_a[wave] = pa;
        sh_in[wave] = pi;
        sh_f[wave] = pf;
        sh_kk[wave] = pk;
        sh_n[wave] = pn;
        sh_t[wave] = pt;
    }
    __syncthreads();
    uint32_t sum_a = 0, sum_i = 0, sum_f = 0;
    uint64_t sum_k = 0, sum_n = 0, sum_t = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        sum_a += sh_a[w];
        sum_i += sh_in[w];
        sum_f += sh_f[w];
        sum_k += sh_kk[w];
        sum_n += sh_n[w];
        sum_t += sh_t[w];
    }
    __syncthreads();

    // A patch whose adults all died keeps its census when a patch it can
    // draw parents from has survivors to supply its newborns: count their
    // survivors (uniform over the block: only tile 0 of such a deme enters).
    uint32_t nb_alive = 0;
    if (k == 0 && sum_a == 0 && n > 0 && d.mig_T != 0 && !(d.island && d.home_T >= kAlways)) {
        // the ring's two neighbours, or under island dispersal every patch
        // (none when every would-be migrant stays home)
        uint32_t x = 0;
        const uint32_t nsrc = d.island ? d.n_patches : 2u;
        for (uint32_t e = 0; e < nsrc; ++e) {
            const uint32_t u = d.island ? d.deme0 + e : (e ? d.right : d.left);
            const SurvCount *CE = counts + descs[u].surv_tile0;
            const uint32_t act = (CE[0].n + TILE - 1) / TILE;
            for (uint32_t q = tid; q < act; q += kBlock) x += CE[q].alive;
        }
        x = wave_sum<uint32_t>(x);
        if ((tid & 63u) == 0) sh_a[wave] = x;
        __syncthreads();
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) nb_alive += sh_a[w];
        __syncthreads();
    }

    // Physiology regime, tile 0: the step's consumption, eggs and weights
    // over the tiles (uniform over the block)
    __shared__ double sh_ph[kBlock / 64][5];
    __shared__ uint32_t sh_phn[kBlock / 64][2];
    double ph[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // e1, e2, eggs, emax, xmax
    uint32_t phn[2] = {0, 0};                    // mature surviving females, males
    const bool phys = d.regime == SPEGG_PHYSIOLOGY;
    if (k == 0 && phys) {
        for (uint32_t q = tid; q < active; q += kBlock) {
            const PhysTile pt = d.ptiles[q];
            ph[0] += pt.e[0];
            ph[1] += pt.e[1];
            ph[2] += pt.eggs;
            ph[3] = fmax(ph[3], pt.emax);
            ph[4] = fmax(ph[4], pt.xmax);
            phn[0] += pt.nf;
            phn[1] += pt.nm;
        }
        for (int c = 0; c < 3; ++c) ph[c] = wave_sum<double>(ph[c]);
        ph[3] = wave_max(ph[3]);
        ph[4] = wave_max(ph[4]);
        phn[0] = wave_sum<uint32_t>(phn[0]);
        phn[1] = wave_sum<uint32_t>(phn[1]);
        if ((tid & 63u) == 0) {
            for (int c = 0; c < 5; ++c) sh_ph[wave][c] = ph[c];
            sh_phn[wave][0] = phn[0];
            sh_phn[wave][1] = phn[1];
        }
        __syncthreads();
        for (int c = 0; c < 5; ++c) ph[c] = 0.0;
        phn[0] = phn[1] = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            for (int c = 0; c < 3; ++c) ph[c] += sh_ph[w][c];
            ph[3] = fmax(ph[3], sh_ph[w][3]);
            ph[4] = fmax(ph[4], sh_ph[w][4]);
            phn[0] += sh_phn[w][0];
            phn[1] += sh_phn[w][1];
        }
    }

    if (k == 0 && tid == 0) {
        // census of the newborns, into the pair the other blocks do not read
        const uint32_t ns = sum_a;
        const bool cr = d.regime == SPEGG_CONSUMER_RESOURCE;
        uint32_t nn;
        if (phys) {
            // resources: growth at this step's rate, less what was eaten
            const Rng rng{d.key0, d.key1, d.c3};
            for (int j = 0; j < 2; ++j) {
                double r = d.growth[j];
                if (d.growth_sd[j] > 0.0) r += d.growth_sd[j] * normal_of(rng.block(0, kStResource, (uint32_t)j, t));
                const double R = st.R[j];
                const double Rn = r * R / (1.0 + R / d.KR2[j]) - ph[j];
                st.R[j] = Rn > 0.0 ? Rn : 0.0;
            }
            // recruits of a breeding step: kappa1 F / (1 + (F/kappa2)^kappa3)
            const bool breeding = t % d.breed_every == d.breed_every - 1u;
            uint64_t want = 0;
            if (breeding && phn[0] > 0 && phn[1] > 0) {
                const double phi = d.kappa1 * ph[2] / (1.0 + pow(ph[2] / d.kappa2, d.kappa3));
                want = phi >= 4294967295.0 ? 4294967295ull : (uint64_t)floor(phi);
            }
            st.eggs = breeding ? ph[2] : 0.0;
            st.emax = ph[3];
            st.xmax = ph[4];
            const uint32_t room = d.cap - ns;
            const uint32_t nb = want > room ? room : (uint32_t)want;
            st.truncated += want - nb;
            nn = ns + nb;
            // free storage slots: the recruits pop the nb below the top
            const uint32_t top = st.gfree_n[t & 1u] + (n - ns);
            st.gfree_top = top;
            st.gfree_n[(t + 1u) & 1u] = top - nb;
        } else if (ns + nb_alive == 0 || (d.sexes && (sum_f == 0 || sum_f == ns))) {
            nn = 0;  // no survivor, or (separate sexes) no surviving female or male
        } else if (d.regime == SPEGG_WF) {
            nn = n;
        } else {
            // newborns fill the room the carried survivors leave
            const uint32_t room = cr ? d.cap - ns : d.cap;
            const uint32_t nb = sum_k > room ? room : (uint32_t)sum_k;
            st.truncated += sum_k - nb;
            nn = (cr ? ns : 0u) + nb;
        }
        st.n_carry = (cr || phys) ? ns : 0u;
        st.captures = sum_i;
        st.n_prev = n;
        st.n_surv = ns;
        st.n_surv_f = sum_f;
        st.t[par ^ 1u] = t + 1;
        st.n[par ^ 1u] = nn;
        if (nn == 0) st.extinct = 1;
        st.traced = trace ? 1u : 0u;
        st.census_pending = 1;
        st.near_ties += sum_n;
        st.sum_threshold = sum_t;
        st.updates += (uint64_t)nn * d.L;
    }
    if (k >= active) return;  // tile 0 of an empty census: uniform over the block
    const uint32_t aoff = k == 0 ? 0u : sum_a;
    const uint64_t koff = k == 0 ? 0ull : sum_k;

    // survivor and slot ranks of the thread's adults, ascending order
    uint32_t a_loc = 0, k_loc = 0;
#pragma unroll
    for (uint32_t q = 0; q < IT; ++q) {
        if (i0 + q >= n) fate[q] = 0;
        a_loc += fate[q] >> 15;
        k_loc += fate[q] & 0x7FFFu;
    }
    uint32_t atot, ktot;
    uint32_t spos = aoff + block_excl_scan(a_loc, sh_a, &atot, tid);
    uint64_t slot = koff + block_excl_scan(k_loc, sh_k, &ktot, tid);
    // consumer-resource and physiology survivors lead the next census: the
    // tile's survivors are listed in LDS, then moved by the whole block,
    // consecutive threads on consecutive survivors (and genome words)
    const bool carries = d.regime == SPEGG_CONSUMER_RESOURCE || d.regime == SPEGG_PHYSIOLOGY;
    __shared__ uint32_t sh_from[kBlock * IT];
    const uint32_t tile_pos0 = aoff;  // the tile's first survivor position
#pragma unroll
    for (uint32_t q = 0; q < IT; ++q) {
        if (fate[q] >> 15) {
            if (spos < d.cap) {
                gstore(d.S + spos, i0 + q);
                if (carries) sh_from[spos - tile_pos0] = i0 + q;
            }
            ++spos;
        } else if (d.gfree && i0 + q < n) {
            // physiology regime: the storage slot of the dead onto the free
            // stack, above the slots already free, in census order
            const uint32_t at = st.gfree_n[t & 1u] + (i0 + q - spos);  // above the free ones and the dead before
            if (at < d.cap) gstore(d.gfree + at, gload(d.gslot[t & 1u] + i0 + q));
            else atomicOr(&st.error, 1u);  // free and living slots exceed the capacity: impossible
        }
        if (d.regime != SPEGG_WF) {  // mothers with offspring counts own their slots
            const uint32_t kids = fate[q] & 0x7FFFu;
            for (uint32_t m = 0; m < kids; ++m, ++slot)
                if (slot < d.cap) gstore(d.owner + slot, i0 + q);
        }
    }
    if (carries) {  // uniform over the block
        __syncthreads();
        const uint32_t cnt = tile_pos0 + atot <= d.cap ? atot : (tile_pos0 < d.cap ? d.cap - tile_pos0 : 0u);
        const uint32_t cur = t & 1u, per = 2u * d.W;
        for (uint32_t kk = tid; kk < cnt; kk += kBlock) carry_one(d, cur, sh_from[kk], tile_pos0 + kk);
        if (d.gfree) {
            // the allelic values stay in their slots
        } else if ((per & 3u) == 0) {  // 16-byte copies, consecutive threads on consecutive words
            const uint32_t per4 = per / 4u;
            const uint4 *__restrict__ src = reinterpret_cast<const uint4 *>(d.genome[cur]);
            uint4 *__restrict__ dst = reinterpret_cast<uint4 *>(d.genome[cur ^ 1u]);
            for (uint32_t idx = tid; idx < cnt * per4; idx += kBlock) {
                const uint32_t k = idx / per4, w = idx % per4;
                dst[(size_t)(tile_pos0 + k) * per4 + w] = src[(size_t)sh_from[k] * per4 + w];
            }
        } else {
            const uint32_t *__restrict__ src = d.genome[cur];
            uint32_t *__restrict__ dst = d.genome[cur ^ 1u];
            for (uint32_t idx = tid; idx < cnt * per; idx += kBlock) {
                const uint32_t k = idx / per, w = idx % per;
                dst[(size_t)(tile_pos0 + k) * per + w] = src[(size_t)sh_from[k] * per + w];
            }
        }
    }
}

template <int IT>
__global__ void __launch_bounds__(kBlock) compact_kernel(const RepDesc *__restrict__ descs,
                                                         RepState *__restrict__ states,
                                                         const SurvTile *__restrict__ tiles,
                                                         const SurvCount *__restrict__ counts,
                                                         SurvGroup *__restrict__ groups, int trace,
                                                         int single_deme) {
    const SurvTile tile = single_deme >= 0 ? SurvTile{(uint32_t)single_deme, blockIdx.x * (uint32_t)(kBlock * IT)}
                                           : tiles[blockIdx.x];
    compact_tile<IT, false>(descs, states, tile, counts, groups, trace);
}

// A resident grid over the same list of occupied tiles as survive's.
template <int IT>
__global__ void __launch_bounds__(kBlock) compact_list_kernel(const RepDesc *__restrict__ descs,
                                                              RepState *__restrict__ states,
                                                              const SurvTile *__restrict__ list,
                                                              const uint32_t *__restrict__ list_n,
                                                              const SurvCount *__restrict__ counts,
                                                              SurvGroup *__restrict__ groups, int trace) {
    const uint32_t m = *list_n;
    for (uint32_t v = blockIdx.x; v < m; v += gridDim.x) {
        compact_tile<IT, true>(descs, states, list[v], counts, groups, trace);
        __syncthreads();  // the next tile reuses the block's LDS
    }
}

// ---------------------------------------------------------------- offspring

// A: the deme a newborn of deme `rep` descends from.  Without migration its
// own; on a ring a migrant's parents live in patch k-1 or k+1; under biased
// island dispersal a would-be migrant stays home with probability pi, else
// its parents live in one of the other patches, uniformly.  A source
// without survivors passes the draw on (ring: drawn, home, picked side,
// other side; island: drawn, home, then the patches after the drawn one).
// mig(c) is word c of the newborn's MIGRATE block.
template <typename Mig>
__device__ __forceinline__ uint32_t source_deme(const RepDesc &d, const RepState &st, const RepState *states,
                                                uint32_t rep, Mig mig) {
    uint32_t su = rep;
    if (d.mig_T != 0 && d.island) {
        const uint32_t m0 = mig(0), m1 = mig(1), m2 = mig(2), m3 = mig(3);
        uint32_t dp = d.patch;
        if ((uint64_t)m0 < d.mig_T && !((uint64_t)m1 < d.home_T)) {
            const uint32_t i = uniform_index(m2, m3, d.n_patches - 1u);
            dp = i < d.patch ? i : i + 1u;
        }
        su = d.deme0 + dp;
        if (!states[su].n_surv) {
            su = rep;
            if (!st.n_surv)
                for (uint32_t q = 1; q < d.n_patches; ++q) {
                    const uint32_t u = d.deme0 + (dp + q) % d.n_patches;
                    if (states[u].n_surv) {
                        su = u;
                        break;
                    }
                }
        }
    } else if (d.mig_T != 0) {
        const uint32_t m0 = mig(0), m1 = mig(1);
        const uint32_t side = (m1 & 1u) ? d.right : d.left, other = (m1 & 1u) ? d.left : d.right;
        const uint32_t drawn = (uint64_t)m0 < d.mig_T ? side : rep;
        su = states[drawn].n_surv ? drawn : st.n_surv ? rep : states[side].n_surv ? side : other;
    }
    return su;
}

// One team of 2G lanes makes one newborn: lanes [0, G) build the maternal
// gamete (haplotype 0), lanes [G, 2G) the paternal one.  A gamete's W words
// are cut into chunks of G x V; in each chunk lane g handles V consecutive
// words from g x V.  NCH > 0: the gamete is exactly NCH chunks or fewer and
// all of them are gathered into registers before the crossover mask is
// drawn; NCH == 0: any number of chunks, gathered one at a time.
// Shapes that hold at most two chunks with at most 8 lanes per gamete run at
// least seven waves per SIMD (measured faster than six, five or four waves
// with more registers at L = 1024, although the two-chunk shapes then keep a
// few values used only on cold paths in scratch); larger ones keep the
// registers they need.
// Dynamic LDS: the effect planes (plane_words), the geometric-gap
// thresholds (geo_words, skip mode), then, per team and gamete, a crossover
// bitmap and a flip bitmap of W words each.
// EXT: the instance for replicates with a linkage map or a mating system
// (separate sexes, mate choice, monogamy); the others run without that code.
template <int G, int V, int NCH, bool EXT>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu((!EXT && NCH >= 1 && NCH <= 2 && G <= 8) ? 7 : 1, 8))) offspring_kernel(const RepDesc *__restrict__ descs,
                                                           const RepState *__restrict__ states,
                                                           const OffTile *__restrict__ tiles, uint32_t tile0,
                                                           uint32_t ntiles, int single_deme,
                                                           Partial *__restrict__ partials, uint32_t plane_words,
                                                           uint32_t geo_words, int trace,
                                                           const uint32_t *__restrict__ list_n) {
    constexpr uint32_t TPO = 2 * G;
    constexpr uint32_t TEAMS = kBlock / TPO;
    constexpr uint32_t KF = kOffspringInFlight;  // newborns of a team in flight at once
    constexpr uint32_t ITERS = (TEAMS >= 16 ? 1 : 16 / TEAMS) * KF;
    constexpr uint32_t OPT = TEAMS * ITERS;
    constexpr uint32_t CH = G * V;  // words of one gamete per chunk
    constexpr int NREG = NCH > 0 ? NCH : 1;
    // per-newborn draws, one Philox block each, spread over the team:
    // 0 parents, 1/2 crossover phase (maternal/paternal), 3/4 mutation
    // count, 5 migration (only where the deme has migration), 6 sex (EXT,
    // separate sexes)
    constexpr uint32_t NSD = EXT ? 7 : 6;
    constexpr uint32_t SR = (NSD + TPO - 1) / TPO;
    extern __shared__ uint32_t lds[];
    __shared__ int64_t red_z[kBlock / 64];
    __shared__ uint64_t red_z2[kBlock / 64];

    uint32_t *planes = lds;
    uint32_t *geo = lds + plane_words;  // geometric-gap thresholds, as 32-bit words

    // tiles: the plan's (one deme: those of its newborns), or the list of
    // this generation's occupied tiles
    uint32_t limit = ntiles;
    if (list_n) {
        const uint32_t m = *list_n;
        limit = m < ntiles ? m : ntiles;
    } else if (single_deme >= 0) {
        const RepState &s1 = states[single_deme];
        const uint32_t nb1 = s1.n[current_pair(s1)] - s1.n_carry;
        const uint32_t active = (nb1 + OPT - 1) / OPT;
        limit = active < ntiles ? active : ntiles;
    }
    for (uint32_t ti = blockIdx.x; ti < limit; ti += gridDim.x) {
        // Lane constants come from an opaque copy of the thread index, so
        // they and the Philox counter words built from them are computed in
        // the tile's body: hoisted above the loop they stay live through it
        // and spill to scratch.
        uint32_t tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const uint32_t team = tid / TPO, lane = tid % TPO;
        const uint32_t half = lane / G, gl = lane % G;
        const uint32_t seg0 = (tid & 63u) - gl;  // first wave lane of this gamete's lanes
        const uint32_t segmask = G >= 32 ? 0xFFFFFFFFu : ((1u << G) - 1u);
        uint32_t rep, start;
        if (single_deme >= 0) {
            rep = (uint32_t)single_deme;
            start = ti * OPT;
        } else {
            const OffTile tile = tiles[tile0 + ti];
            rep = tile.rep;
            start = tile.start;
        }
        const RepDesc &d = descs[rep];
        const RepState &st = states[rep];
        const uint32_t newest = current_pair(st);  // the newborns' census, written by this generation's select
        const uint32_t base = st.n_carry;          // carried survivors come first in the census
        const uint32_t nn = st.n[newest] - base;   // newborns
        if (start >= nn || st.error) continue;  // uniform over the block
        const uint32_t tp = st.t[newest] - 1u, cur = tp & 1u;
        const uint32_t W = d.W, L = d.L, mode = d.mode;
        const uint32_t nsd = d.mig_T != 0 ? 6u : 5u;  // draws 0..4, and 5 with migration
        const bool unit = d.unit_effects != 0;
        const uint64_t binom0 = d.binom0;  // most gametes carry no mutation
        const bool has_tail = d.tail_mask != ~0u;  // L not a multiple of 32
        const Rng rng{d.key0, d.key1, d.c3};
        // effect planes and gap thresholds into LDS: once per block when
        // every tile is of one deme, else for every tile
        const bool skip_table = mode == kModeSkip && d.geo_len > 0;
        if ((!unit || skip_table) && (single_deme < 0 || ti == blockIdx.x)) {
            if (!unit)
                for (uint32_t q = threadIdx.x; q < 4u * W; q += kBlock) planes[q] = gload(d.planes + q);
            if (skip_table)
                for (uint32_t q = threadIdx.x; q < d.geo_len; q += kBlock) geo[q] = (uint32_t)gload(d.geo + q);
            __syncthreads();
        }
        uint32_t *X = lds + plane_words + geo_words + (size_t)(team * 2u + half) * 2u * W;  // crossover toggles
        uint32_t *F = X + W;                                                     // mutation flips
        int64_t my_z = 0;
        uint64_t my_z2 = 0;

        // Front of a newborn: its draws, parents and the parents' haplotype
        // words (loads in flight); KF newborns of a team get their fronts
        // before the first is finished, so their gathers overlap.
        struct Front {
            uint32_t j, phase, xk, sex;
            const uint32_t *src;
            uint32_t *dst;
            Words<V> h0[NREG], h1[NREG];
        };
        auto front = [&](uint32_t j, Front &f) {
            Words4 sd[SR];
#pragma unroll
            for (uint32_t r = 0; r < SR; ++r) {
                const uint32_t kd = lane + r * TPO;
                const uint32_t stream = kd == 0   ? kStParent
                                        : kd <= 2 ? kStRecomb + kd - 1u
                                        : kd <= 4 ? kStMutate + kd - 3u
                                        : kd == 5 ? kStMigrate
                                                  : kStSex;
                const bool need = EXT ? kd < nsd || (kd == 6 && d.sexes) : kd < nsd;
                if (need) {
                    sd[r] = rng.block(j, stream, 0, tp);
                } else {
                    sd[r].v[0] = sd[r].v[1] = sd[r].v[2] = sd[r].v[3] = 0;
                }
            }
            // word c of draw kd, from the lane of the team that made it
            auto draw = [&](uint32_t kd, int c) -> uint32_t {
                return (uint32_t)__shfl((int)sd[kd / TPO].v[c], (int)(kd % TPO), (int)TPO);
            };

            // A: the patch the parents live in (a migrant's comes from a ring
            // neighbour; a patch without survivors passes the draw on: drawn,
            // home, picked side, other side), then parents uniform over its
            // survivors (Poisson: the slot's mother)
            const uint32_t su = source_deme(d, st, states, rep, [&](int c) { return draw(5, c); });
            const RepDesc &sd_src = descs[su];
            const uint32_t ns = states[su].n_surv, nprev = states[su].n_prev;
            const uint32_t p0 = draw(0, 0), p1 = draw(0, 1), p2 = draw(0, 2), p3 = draw(0, 3);
            uint32_t mom = d.regime == SPEGG_WF ? gload(sd_src.S + uniform_index(p0, p1, ns)) : gload(d.owner + j);
            uint32_t dad = gload(sd_src.S + uniform_index(p2, p3, ns));
            if constexpr (EXT) {
                // mating systems (one patch: the source is the deme itself)
                const uint32_t sx = draw(6, 0);
                f.sex = sx & 1u;
                if (d.sexes || d.mating != SPEGG_RANDOM_MATING || d.monogamy) {  // uniform over the block
                    const uint32_t tseg0 = (tid & 63u) - lane;
                    if (d.regime == SPEGG_WF && d.sexes)
                        mom = team_partner<TPO>(d, rng, kStFemale, j, tp, cur, 0, false, 0u, ns, lane, tseg0);
                    dad = team_partner<TPO>(d, rng, kStMate, d.monogamy ? mom : j, tp, cur, d.sexes ? 1 : -1,
                                            d.mating != SPEGG_RANDOM_MATING, mom, ns, lane, tseg0);
                }
            }
            // Parents are adults of the last census.  An index beyond it means
            // a broken survivor or slot list: the deme is flagged (the next
            // census read reports it as a device error) and the index clamped
            // only so that the gather stays inside the buffer.
            if (mom >= nprev || dad >= nprev) {
                atomicOr(const_cast<uint32_t *>(&st.error), 1u);
                mom = mom < nprev ? mom : nprev - 1u;
                dad = dad < nprev ? dad : nprev - 1u;
            }
            f.j = j;
            // the traced parents leave now rather than staying live in
            // registers through the newborn
            if (trace && lane == 0) {
                gstore(d.mom + j, mom);
                gstore(d.dad + j, dad);
                if (d.mig_T != 0) gstore(d.src + j, sd_src.patch);  // the buffer exists with migration only
            }
            f.src = sd_src.genome[cur] + (size_t)(half ? dad : mom) * 2u * W;
            f.dst = d.genome[cur ^ 1u] + (size_t)(base + j) * 2u * W + (size_t)half * W;
            const uint32_t phase_m = draw(1, 0), phase_p = draw(2, 0);
            const uint32_t xk_m = draw(3, 0), xk_p = draw(4, 0);
            f.phase = (half ? phase_p : phase_m) & 1u;
            f.xk = half ? xk_p : xk_m;
            // the parent's haplotypes (all chunks, or the first), in flight
            // while the crossover mask is drawn
#pragma unroll
            for (int c = 0; c < NREG; ++c) {
                const uint32_t w0 = (uint32_t)c * CH + gl * V;
                if (w0 < W) {
                    f.h0[c] = load_words<V>(f.src + w0);
                    f.h1[c] = load_words<V>(f.src + W + w0);
                }
            }
        };
        auto finish = [&](Front &f) {
            const uint32_t j = f.j;
            const uint32_t *__restrict__ src = f.src;
            uint32_t *__restrict__ dst = f.dst;
            const uint32_t rs = kStRecomb + half, ms = kStMutate + half;
            const uint32_t phase = f.phase;
            // B1: crossover toggles.  Boundary b (between loci b-1 and b)
            // toggles the source haplotype from locus b on; bit 0 of word 0
            // holds the phase (which haplotype locus 0 copies).
            if (mode == kModeSkip) {
                for (uint32_t w = gl * V; w < W; w += CH)
#pragma unroll
                    for (int v = 0; v < V; ++v) X[w + v] = 0;
                wave_lds_sync();
                // gaps come four to a Philox block from block 1 on; lane g
                // takes block blk + g, so a pass places up to 4G crossovers.
                // One locus (an empty table) has no boundary.
                uint32_t b = 0, blk = 1;
                for (; d.geo_len > 0;) {
                    const Words4 xw = rng.block(j, rs, blk + gl, tp);
                    uint32_t cum[4];
                    uint32_t acc = 0;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        acc += 1u + geometric_gap(geo, d.geo_len, d.geo_scale, xw.v[c]);
                        cum[c] = acc;
                    }
                    uint32_t incl = acc;
#pragma unroll
                    for (int o = 1; o < G; o <<= 1) {
                        const uint32_t y = __shfl_up(incl, o, G);
                        if (gl >= (uint32_t)o) incl += y;
                    }
                    const uint32_t base = b + incl - acc;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const uint32_t pos = base + cum[c];
                        if (pos <= L - 1u) atomicOr(&X[pos >> 5], 1u << (pos & 31u));
                    }
                    const uint32_t last = __shfl(b + incl, G - 1, G);
                    if (last > L - 1u) break;
                    b = last;
                    blk += G;
                }
                wave_lds_sync();
            } else if (mode == kModeLazy) {
                // Bit-serial: the crossovers of every word this lane owns
                // (word c CH + g V + v of chunk c), into its crossover words
                // X.  Bit planes of U come four to a Philox block, the top
                // bit first; a word is decided once none of its boundaries
                // is undecided or R has no 1 bit left.
                // Pass 1: blocks 0 and 1 of every word (eight planes), which
                // decide all 32 boundaries of about 88% of words.  R is the
                // same for the whole wave (one replicate per tile), so each
                // plane's R bit is a uniform branch, not a per-lane mask.
                // Pass 2: the words still undecided (their state parked in
                // F, free until mutation) walk on a block at a time in one
                // flattened loop, so the wave waits for the lane with the
                // most remaining blocks in all.
                const uint32_t R = d.R;
                const bool second = (R << 4) != 0;  // planes 4..7 can decide a boundary
                const bool more = (R << 8) != 0;    // planes past 7 can
                uint32_t pend = 0;  // bit i: the lane's i-th word undecided after pass 1 (at most 16 words)
                uint32_t idx = 0;
                for (uint32_t w0 = gl * V; w0 < W; w0 += CH) {  // V divides W: all V words exist
#pragma unroll
                    for (int v = 0; v < V; ++v, ++idx) {
                        const uint32_t w = w0 + v;
                        uint32_t und = ~0u, hit = 0;
                        const Words4 b0 = rng.block(j, rs, 1u + w * 8u, tp);
                        planes_uniform(b0, R, 0, und, hit);
                        if (second) {
                            // the second block starts once the first is folded
                            // in (interleaving the two spills registers)
                            uint32_t blk1 = 2u + w * 8u;
                            asm volatile("" : "+v"(blk1) : "v"(und));
                            const Words4 b1 = rng.block(j, rs, blk1, tp);
                            planes_uniform(b1, R, 4, und, hit);
                        }
                        X[w] = hit;
                        if (more && und != 0) {
                            F[w] = und;
                            pend |= 1u << idx;
                        }
                    }
                }
                // Rk: R shifted so that its top four bits are the planes of
                // the word's current block
                uint32_t w = 0, k = 0, und = 0, hit = 0, Rk = 0;
                bool live = false;
                for (;;) {
                    if (!live) {
                        if (pend == 0) break;
                        const uint32_t i = __builtin_ctz(pend);
                        pend &= pend - 1u;
                        w = (i / V) * CH + gl * V + i % V;
                        und = F[w];
                        hit = X[w];
                        k = 2;
                        Rk = R << 8;
                        live = true;
                    }
                    const Words4 blk = rng.block(j, rs, 1u + w * 8u + k, tp);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const uint32_t x = blk.v[q];
                        const uint32_t one = (uint32_t)((int32_t)(Rk << q) >> 31);  // ~0 where R's bit is 1
                        hit |= und & ~x & one;
                        und &= x ^ ~one;  // R bit 1: keep where x is 1; R bit 0: where x is 0
                    }
                    Rk <<= 4;
                    if (Rk == 0 || und == 0) {
                        X[w] = hit;
                        live = false;
                    } else {
                        ++k;
                    }
                }
            } else if (EXT && mode == kModeMap) {
                // linkage map: each boundary against its own threshold
                for (uint32_t w0 = gl * V; w0 < W; w0 += CH)
#pragma unroll
                    for (int v = 0; v < V; ++v) X[w0 + v] = map_word(rng, j, rs, tp, d.map, w0 + v);
            }

            // B2: mutation, K ~ Binomial(L, mu) distinct loci flipped
            const uint32_t xk = f.xk;
            const uint32_t K = (uint64_t)xk < binom0 ? 0u : table_draw_global(d.binom, d.binom_len, xk);
            if (K > 0) {
                for (uint32_t w = gl * V; w < W; w += CH)
#pragma unroll
                    for (int v = 0; v < V; ++v) F[w + v] = 0;
                wave_lds_sync();
                if (gl == 0) {
                    uint32_t accepted = 0;
                    // at most 2^23 candidates per gamete: every loop ends
                    for (uint32_t m = 0; accepted < K && m < (1u << 23); ++m) {
                        const uint32_t lo = rng.seq(j, ms, 1u + 2u * m, tp);
                        const uint32_t hi = rng.seq(j, ms, 2u + 2u * m, tp);
                        const uint32_t pos = uniform_index(lo, hi, L);
                        const uint32_t bit = 1u << (pos & 31u);
                        if (!(F[pos >> 5] & bit)) {
                            F[pos >> 5] |= bit;
                            ++accepted;
                        }
                    }
                }
                wave_lds_sync();
            }

            // B3 + C: gamete words, written out; additive phenotype
            EffectSum es;
            uint32_t carry = 0;  // parity of the toggles in earlier chunks
            auto chunk = [&](uint32_t c, const Words<V> &a, const Words<V> &b) {
                const uint32_t w0 = c * CH + gl * V;
                const bool valid = w0 < W;
                Words<V> M;
                if (mode == kModeRaw) {
                    const Words4 blk = rng.block(j, rs, w0 >> 2, tp);
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const uint32_t q = (w0 + v) & 3u;
                        M.v[v] = q == 0 ? blk.v[0] : q == 1 ? blk.v[1] : q == 2 ? blk.v[2] : blk.v[3];
                    }
                } else {
                    uint32_t lane_par = 0;
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const uint32_t w = w0 + v;
                        uint32_t tog = 0;
                        if (valid) {
                            if (mode == kModeSkip || mode == kModeLazy || (EXT && mode == kModeMap)) tog = X[w];
                            if (w == 0) tog = (tog & ~1u) | phase;
                        }
                        const uint32_t pre = prefix_xor32(tog);
                        M.v[v] = pre ^ (lane_par ? ~0u : 0u);
                        lane_par ^= pre >> 31;
                    }
                    // parity of the toggles in the gamete's lanes below this one
                    const uint64_t bal = __ballot(lane_par);
                    const uint32_t seg = (uint32_t)(bal >> seg0) & segmask;
                    const uint32_t below = __popc(seg & ((1u << gl) - 1u));
                    const uint32_t flip = ((below + carry) & 1u) ? ~0u : 0u;
#pragma unroll
                    for (int v = 0; v < V; ++v) M.v[v] ^= flip;
                    carry = (carry + __popc(seg)) & 1u;
                }
                if (valid) {
                    Words<V> g;
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        uint32_t x = (a.v[v] & ~M.v[v]) | (b.v[v] & M.v[v]);
                        if (K > 0) x ^= F[w0 + v];
                        if (has_tail && w0 + v == W - 1u) x &= d.tail_mask;
                        g.v[v] = x;
                        es.add(unit, planes, W, w0 + v, x);
                    }
                    store_words_nt<V>(dst + w0, g);
                }
            };
            if constexpr (NCH > 0) {
#pragma unroll
                for (int c = 0; c < NCH; ++c) chunk((uint32_t)c, f.h0[c], f.h1[c]);
            } else {
                const uint32_t nch = (W + CH - 1) / CH;
                chunk(0, f.h0[0], f.h1[0]);
                for (uint32_t c = 1; c < nch; ++c) {
                    const uint32_t w0 = c * CH + gl * V;
                    Words<V> a{}, b{};
                    if (w0 < W) {
                        a = load_words<V>(src + w0);
                        b = load_words<V>(src + W + w0);
                    }
                    chunk(c, a, b);
                }
            }
            int32_t zc = es.value(unit);
#pragma unroll
            for (int o = 1; o < (int)TPO; o <<= 1) zc += __shfl_xor(zc, o, TPO);
            if (lane == 0) {
                const int32_t z = zc - d.sum_e;
                gstore(d.z[cur ^ 1u] + base + j, z);
                if (EXT && d.sexes) gstore(d.sex[cur ^ 1u] + base + j, (uint8_t)f.sex);
                if (d.regime == SPEGG_CONSUMER_RESOURCE) {
                    gstore(d.age[cur ^ 1u] + base + j, (uint8_t)0);
                    if (d.species == 0) gstore(d.won + base + j, (uint64_t)~0ull);  // not captured in the next generation yet
                }
                my_z += z;
                my_z2 += (uint64_t)((int64_t)z * (int64_t)z);
            }
        };

        for (uint32_t it = 0; it < ITERS; it += KF) {
            Front fr[KF];
#pragma unroll
            for (uint32_t k = 0; k < KF; ++k) {
                const uint32_t j = start + (it + k) * TEAMS + team;
                if (j < nn) front(j, fr[k]);  // uniform over the team
            }
#pragma unroll
            for (uint32_t k = 0; k < KF; ++k) {
                const uint32_t j = start + (it + k) * TEAMS + team;
                if (j < nn) finish(fr[k]);
            }
        }
        // census sums of the tile, folded later by the census kernel
        const int64_t wz = wave_sum<int64_t>(my_z);
        const uint64_t wz2 = wave_sum<uint64_t>(my_z2);
        if (lane_id() == 0) {
            red_z[threadIdx.x >> 6] = wz;
            red_z2[threadIdx.x >> 6] = wz2;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t a = 0;
            uint64_t b = 0;
            for (int w = 0; w < kBlock / 64; ++w) {
                a += red_z[w];
                b += red_z2[w];
            }
            // the tile's own slot (a listed tile sits elsewhere in the list)
            const uint32_t slot = list_n ? d.off_tile0 + start / OPT : tile0 + ti;
            gstore(&partials[slot].sum_z, a);
            gstore(&partials[slot].sum_z2, b);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- offspring, continuous alleles

// Continuous alleles (Supplementary S2, "Genetics"): W floats per haplotype
// (L rounded up to a multiple of 4, the pad zero).  One team of 2G lanes
// makes one newborn, lanes [0, G) the maternal gamete (haplotype 0) and
// [G, 2G) the paternal one; in each chunk of 4G loci lane g holds loci
// 4g .. 4g+3 as one 16-byte access.  The crossover mask comes from the
// draws a biallelic gamete would use: crossover toggles (geometric gaps or
// bit-serial comparisons) into the gamete's LDS words, turned into mask
// words by a prefix XOR; each lane then reads the four mask bits of its
// loci.  The mutated loci are the biallelic rule's K distinct loci (flip
// bitmap in LDS); each moves by mut_sd times the deviate of its own MUTVAL
// block (keyed by the locus).  The genetic value is half the sum of both
// gametes' values; lane 0 adds the noise and stores the phenotype.
// NCH > 0: a gamete spans at most NCH chunks, all gathered before the mask
// is drawn; NCH == 0: any number, gathered one at a time.
// Dynamic LDS: the geometric-gap thresholds (geo_words), then per team and
// gamete a mask bitmap and a flip bitmap of mask_words words each.  No
// census partials: the census kernel sums continuous phenotypes itself.
template <int G, int NCH>
__global__ void __launch_bounds__(kBlock) offspring_cont_kernel(const RepDesc *__restrict__ descs,
                                                                const RepState *__restrict__ states,
                                                                const OffTile *__restrict__ tiles, uint32_t tile0,
                                                                uint32_t ntiles, int single_deme,
                                                                Partial *__restrict__ partials, uint32_t mask_words,
                                                                uint32_t geo_words, int trace,
                                                                const uint32_t *__restrict__ list_n) {
    constexpr uint32_t TPO = 2 * G;
    constexpr uint32_t TEAMS = kBlock / TPO;
    constexpr uint32_t ITERS = TEAMS >= 16 ? 1 : 16 / TEAMS;
    constexpr uint32_t OPT = TEAMS * ITERS;
    constexpr uint32_t CH = 4 * G;  // loci of one gamete per chunk
    constexpr int NREG = NCH > 0 ? NCH : 1;
    // per-newborn draws, one Philox block each, spread over the team: 0
    // parents, 1/2 crossover phase, 3/4 mutation count (maternal/paternal),
    // 5 migration, 6 phenotypic noise, 7 sex
    constexpr uint32_t NSD = 8;
    constexpr uint32_t SR = (NSD + TPO - 1) / TPO;
    extern __shared__ uint32_t lds[];
    uint32_t *geo = lds;

    uint32_t limit = ntiles;
    if (list_n) {
        const uint32_t m = *list_n;
        limit = m < ntiles ? m : ntiles;
    } else if (single_deme >= 0) {
        const RepState &s1 = states[single_deme];
        const uint32_t active = (s1.n[current_pair(s1)] - s1.n_carry + OPT - 1) / OPT;
        limit = active < ntiles ? active : ntiles;
    }
    for (uint32_t ti = blockIdx.x; ti < limit; ti += gridDim.x) {
        uint32_t tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const uint32_t team = tid / TPO, lane = tid % TPO;
        const uint32_t half = lane / G, gl = lane % G;
        const uint32_t seg0 = (tid & 63u) - gl;
        const uint32_t segmask = G >= 32 ? 0xFFFFFFFFu : ((1u << G) - 1u);
        uint32_t rep, start;
        if (single_deme >= 0) {
            rep = (uint32_t)single_deme;
            start = ti * OPT;
        } else {
            const OffTile tile = tiles[tile0 + ti];
            rep = tile.rep;
            start = tile.start;
        }
        const RepDesc &d = descs[rep];
        const RepState &st = states[rep];
        const uint32_t newest = current_pair(st);
        const uint32_t base = st.n_carry;        // carried survivors come first (physiology regime)
        const uint32_t nn = st.n[newest] - base;  // newborns
        if (start >= nn || st.error) continue;  // uniform over the block
        const uint32_t tp = st.t[newest] - 1u, cur = tp & 1u;
        const uint32_t W = d.W, L = d.L, Wb = (L + 31u) / 32u, mode = d.mode;
        const Rng rng{d.key0, d.key1, d.c3};
        const bool skip_table = mode == kModeSkip && d.geo_len > 0;
        if (skip_table && (single_deme < 0 || ti == blockIdx.x)) {
            for (uint32_t q = threadIdx.x; q < d.geo_len; q += kBlock) geo[q] = (uint32_t)gload(d.geo + q);
            __syncthreads();
        }
        uint32_t *X = lds + geo_words + (size_t)(team * 2u + half) * 2u * mask_words;  // toggles, then mask words
        uint32_t *F = X + mask_words;                                                   // mutation flips

        for (uint32_t it = 0; it < ITERS; ++it) {
            const uint32_t j = start + it * TEAMS + team;
            if (j >= nn) continue;  // uniform over the team
            Words4 sd[SR];
#pragma unroll
            for (uint32_t r = 0; r < SR; ++r) {
                const uint32_t kd = lane + r * TPO;
                const uint32_t stream = kd == 0   ? kStParent
                                        : kd <= 2 ? kStRecomb + kd - 1u
                                        : kd <= 4 ? kStMutate + kd - 3u
                                        : kd == 5 ? kStMigrate
                                        : kd == 6 ? kStNoise
                                                  : kStSex;
                if (kd < NSD && (kd != 5 || d.mig_T != 0) && (kd != 6 || d.noise_sd > 0.0) && (kd != 7 || d.sexes)) {
                    sd[r] = rng.block(j, stream, 0, tp);
                } else {
                    sd[r].v[0] = sd[r].v[1] = sd[r].v[2] = sd[r].v[3] = 0;
                }
            }
            auto draw = [&](uint32_t kd, int c) -> uint32_t {
                return (uint32_t)__shfl((int)sd[kd / TPO].v[c], (int)(kd % TPO), (int)TPO);
            };
            // A: parents
            const uint32_t su = source_deme(d, st, states, rep, [&](int c) { return draw(5, c); });
            const RepDesc &sd_src = descs[su];
            const uint32_t ns = states[su].n_surv, nprev = states[su].n_prev;
            const uint32_t p0 = draw(0, 0), p1 = draw(0, 1), p2 = draw(0, 2), p3 = draw(0, 3);
            uint32_t mom = d.regime == SPEGG_WF ? gload(sd_src.S + uniform_index(p0, p1, ns)) : gload(d.owner + j);
            uint32_t dad = gload(sd_src.S + uniform_index(p2, p3, ns));
            const uint32_t sx = draw(7, 0) & 1u;
            if (d.regime == SPEGG_PHYSIOLOGY) {  // uniform over the block
                const uint32_t tseg0 = (tid & 63u) - lane;
                mom = team_phys_partner<TPO>(d, st, rng, kStFemale, j, tp, cur, 0u, ns, lane, tseg0);
                dad = team_phys_partner<TPO>(d, st, rng, kStMate, j, tp, cur, 1u, ns, lane, tseg0);
            } else if (d.sexes || d.mating != SPEGG_RANDOM_MATING || d.monogamy) {  // uniform over the block; one patch
                const uint32_t tseg0 = (tid & 63u) - lane;
                if (d.regime == SPEGG_WF && d.sexes)
                    mom = team_partner<TPO>(d, rng, kStFemale, j, tp, cur, 0, false, 0u, ns, lane, tseg0);
                dad = team_partner<TPO>(d, rng, kStMate, d.monogamy ? mom : j, tp, cur, d.sexes ? 1 : -1,
                                        d.mating != SPEGG_RANDOM_MATING, mom, ns, lane, tseg0);
            }
            if (mom >= nprev || dad >= nprev) {
                atomicOr(const_cast<uint32_t *>(&st.error), 1u);
                mom = mom < nprev ? mom : nprev - 1u;
                dad = dad < nprev ? dad : nprev - 1u;
            }
            if (trace && lane == 0) {
                gstore(d.mom + j, mom);
                gstore(d.dad + j, dad);
                if (d.mig_T != 0) gstore(d.src + j, sd_src.patch);
            }
            if (d.sexes && lane == 0) gstore(d.sex[cur ^ 1u] + base + j, (uint8_t)sx);
            if (d.regime == SPEGG_PHYSIOLOGY && lane == 0) {
                // a recruit is born at its mother's neonate mass
                const double om = (double)__uint_as_float((uint32_t)gload(d.z[cur] + mom));
                gstore(d.X[cur ^ 1u] + base + j, om);
                gstore(d.Y[cur ^ 1u] + base + j, d.qJ * om);
            }
            const uint32_t *src;
            uint32_t *dst;
            if (d.gfree) {  // physiology regime: values by storage slot, the recruit's popped off the free stack
                const uint32_t top = st.gfree_top;
                const bool popped = j < top && top <= d.cap;  // compact left room for every recruit
                uint32_t pslot = gload(d.gslot[cur] + (half ? dad : mom));
                uint32_t nslot = popped ? gload(d.gfree + (top - 1u - j)) : 0u;
                if (!popped || pslot >= d.cap || nslot >= d.cap) {  // a broken slot map: flagged, kept in bounds
                    atomicOr(const_cast<uint32_t *>(&st.error), 1u);
                    pslot = pslot < d.cap ? pslot : 0u;
                    nslot = nslot < d.cap ? nslot : 0u;
                }
                if (lane == 0) gstore(d.gslot[cur ^ 1u] + base + j, nslot);
                src = d.genome[0] + (size_t)pslot * 2u * W;
                dst = d.genome[0] + (size_t)nslot * 2u * W + (size_t)half * W;
            } else {
                src = sd_src.genome[cur] + (size_t)(half ? dad : mom) * 2u * W;
                dst = d.genome[cur ^ 1u] + (size_t)(base + j) * 2u * W + (size_t)half * W;
            }
            // every lane takes part in each cross-lane read, then selects
            const uint32_t phase_m = draw(1, 0), phase_p = draw(2, 0);
            const uint32_t xk_m = draw(3, 0), xk_p = draw(4, 0);
            const uint32_t phase = (half ? phase_p : phase_m) & 1u;
            const uint32_t xk = half ? xk_p : xk_m;
            const uint32_t nz0 = draw(6, 0), nz1 = draw(6, 1), nz2 = draw(6, 2), nz3 = draw(6, 3);
            // the parent's values (all chunks, or the first), in flight while
            // the mask is drawn
            Words<4> h0[NREG], h1[NREG];
#pragma unroll
            for (int c = 0; c < NREG; ++c) {
                const uint32_t l0 = (uint32_t)c * CH + gl * 4u;
                if (l0 < W) {
                    h0[c] = load_words<4>(src + l0);
                    h1[c] = load_words<4>(src + W + l0);
                }
            }
            const uint32_t rs = kStRecomb + half, ms = kStMutate + half;
            // B1: crossover mask words of the gamete into X
            if (mode == kModeRaw) {
                for (uint32_t w = gl; w < Wb; w += G) X[w] = rng.seq(j, rs, w, tp);
            } else {
                for (uint32_t w = gl; w < Wb; w += G) X[w] = 0;
                wave_lds_sync();
                if (mode == kModeSkip) {
                    // geometric gaps, four to a Philox block from block 1 on;
                    // lane g takes block blk + g
                    uint32_t b = 0, blk = 1;
                    for (; d.geo_len > 0;) {
                        const Words4 xw = rng.block(j, rs, blk + gl, tp);
                        uint32_t cum[4];
                        uint32_t acc = 0;
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            acc += 1u + geometric_gap(geo, d.geo_len, d.geo_scale, xw.v[c]);
                            cum[c] = acc;
                        }
                        uint32_t incl = acc;
#pragma unroll
                        for (int o = 1; o < G; o <<= 1) {
                            const uint32_t y = __shfl_up(incl, o, G);
                            if (gl >= (uint32_t)o) incl += y;
                        }
                        const uint32_t base = b + incl - acc;
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            const uint32_t pos = base + cum[c];
                            if (pos <= L - 1u) atomicOr(&X[pos >> 5], 1u << (pos & 31u));
                        }
                        const uint32_t last = __shfl(b + incl, G - 1, G);
                        if (last > L - 1u) break;
                        b = last;
                        blk += G;
                    }
                } else if (mode == kModeLazy) {
                    // bit-serial U < R per 32-boundary word, U's bits from
                    // the top, four planes per Philox block
                    const uint32_t R = d.R;
                    for (uint32_t w = gl; w < Wb; w += G) {
                        uint32_t und = ~0u, hit = 0, Rk = R;
                        for (uint32_t k = 0;; ++k) {
                            const Words4 blk = rng.block(j, rs, 1u + w * 8u + k, tp);
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                const uint32_t x = blk.v[q];
                                const uint32_t one = (uint32_t)((int32_t)(Rk << q) >> 31);
                                hit |= und & ~x & one;
                                und &= x ^ ~one;
                            }
                            Rk <<= 4;
                            if (Rk == 0 || und == 0) break;
                        }
                        X[w] = hit;
                    }
                } else if (mode == kModeMap) {
                    // linkage map: each boundary against its own threshold
                    for (uint32_t w = gl; w < Wb; w += G) X[w] = map_word(rng, j, rs, tp, d.map, w);
                }
                wave_lds_sync();
                // toggles -> mask words: prefix XOR within each word, the
                // parity of the gamete's earlier words carried across
                uint32_t carry = 0;
                for (uint32_t wb = 0; wb < Wb; wb += G) {
                    const uint32_t w = wb + gl;
                    uint32_t tog = w < Wb ? X[w] : 0u;
                    if (w == 0) tog = (tog & ~1u) | phase;
                    const uint32_t pre = prefix_xor32(tog);
                    const uint64_t bal = __ballot(w < Wb && (pre >> 31));
                    const uint32_t seg = (uint32_t)(bal >> seg0) & segmask;
                    const uint32_t below = __popc(seg & ((1u << gl) - 1u));
                    const uint32_t m = pre ^ (((below + carry) & 1u) ? ~0u : 0u);
                    carry = (carry + __popc(seg)) & 1u;
                    wave_lds_sync();
                    if (w < Wb) X[w] = m;
                }
            }
            // B2: mutation, K ~ Binomial(L, mu) distinct loci
            const uint32_t K = (uint64_t)xk < d.binom0 ? 0u : table_draw_global(d.binom, d.binom_len, xk);
            if (K > 0) {
                for (uint32_t w = gl; w < Wb; w += G) F[w] = 0;
                wave_lds_sync();
                if (gl == 0) {
                    uint32_t accepted = 0;
                    for (uint32_t m = 0; accepted < K && m < (1u << 23); ++m) {
                        const uint32_t lo = rng.seq(j, ms, 1u + 2u * m, tp);
                        const uint32_t hi = rng.seq(j, ms, 2u + 2u * m, tp);
                        const uint32_t pos = uniform_index(lo, hi, L);
                        const uint32_t bit = 1u << (pos & 31u);
                        if (!(F[pos >> 5] & bit)) {
                            F[pos >> 5] |= bit;
                            ++accepted;
                        }
                    }
                }
            }
            wave_lds_sync();
            // B3 + C: the gamete's values, written out; their sum
            double acc = 0.0;
            auto chunk = [&](uint32_t c, const Words<4> &a, const Words<4> &b) {
                const uint32_t l0 = c * CH + gl * 4u;
                if (l0 >= W) return;
                const uint32_t msk = (X[l0 >> 5] >> (l0 & 31u)) & 0xFu;
                const uint32_t flp = K > 0 ? (F[l0 >> 5] >> (l0 & 31u)) & 0xFu : 0u;
                Words<4> g;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    uint32_t x = ((msk >> v) & 1u) ? b.v[v] : a.v[v];
                    if (l0 + v >= L) x = 0;  // pad
                    if ((flp >> v) & 1u) {
                        const double y = (double)__uint_as_float(x) +
                                         d.mut_sd * normal_of(rng.block(j, kStMutVal + half, l0 + v, tp));
                        x = __float_as_uint((float)y);
                    }
                    g.v[v] = x;
                    acc += (double)__uint_as_float(x);
                }
                store_words_nt<4>(dst + l0, g);
            };
            if constexpr (NCH > 0) {
#pragma unroll
                for (int c = 0; c < NCH; ++c) chunk((uint32_t)c, h0[c], h1[c]);
            } else {
                chunk(0, h0[0], h1[0]);
                for (uint32_t c = 1; c * CH < W; ++c) {
                    const uint32_t l0 = c * CH + gl * 4u;
                    Words<4> a{}, b{};
                    if (l0 < W) {
                        a = load_words<4>(src + l0);
                        b = load_words<4>(src + W + l0);
                    }
                    chunk(c, a, b);
                }
            }
#pragma unroll
            for (int o = 1; o < (int)TPO; o <<= 1) acc += __shfl_xor(acc, o, TPO);
            if (lane == 0) {
                double z = 0.5 * acc;
                if (d.noise_sd > 0.0) {
                    Words4 nb;
                    nb.v[0] = nz0;
                    nb.v[1] = nz1;
                    nb.v[2] = nz2;
                    nb.v[3] = nz3;
                    z += d.noise_sd * normal_of(nb);
                }
                if (d.exp_tf) z = exp(z);
                const float zf = (float)z;
                gstore(d.z[cur ^ 1u] + base + j, (int32_t)__float_as_uint(zf));
            }
            wave_lds_sync();  // X and F are rewritten by the team's next newborn
        }
        __syncthreads();  // the next tile may reload the gap table
    }
}

// ---------------------------------------------------------------- tile lists

// This generation's occupied tiles, for populations whose censuses can fall
// far below their capacities: the launches then walk these lists with
// resident grids instead of dispatching one block per tile of the capacity.
// One block per deme; a deme's tiles go to positions taken by an atomic add
// on the list's count, so the order of the demes in a list varies from run
// to run, which no result depends on (every tile writes only its own
// outputs).  Phase 0, before encounter and survive: the survival tiles of
// the census (tile 0 always: it records the census) and, for consumers,
// their encounter tiles.  Phase 1, after compact: the offspring tiles of the
// newborns, in the list of the deme's kernel class.  Each phase clears the
// counts of the other phase's lists, which it does not touch; all start at
// zero.
__global__ void __launch_bounds__(kBlock) plan_tiles_kernel(const RepDesc *__restrict__ descs,
                                                            const RepState *__restrict__ states, TileLists lists,
                                                            int phase) {
    __shared__ uint32_t base[2];
    const uint32_t u = blockIdx.x;
    const RepDesc &d = descs[u];
    const RepState &st = states[u];
    const uint32_t T = d.surv_tile;
    if (phase == 0) {
        if (u == 0)
            for (uint32_t q = threadIdx.x; q < lists.n_classes; q += kBlock) lists.counts[2u + q] = 0;
        const uint32_t n = st.n[current_pair(st)];
        // a census beyond the capacity is an impossible state (the kernels
        // that find one report it): never write past the deme's share
        uint32_t ms = n == 0 ? 1u : (n + T - 1u) / T, me = 0;
        const uint32_t enc_ntiles = (d.cap + kBlock - 1u) / kBlock;  // encounter tiles: kBlock consumers each
        if (d.regime == SPEGG_CONSUMER_RESOURCE && d.species == 1) me = (n + kBlock - 1u) / kBlock;
        ms = ms < d.surv_ntiles ? ms : d.surv_ntiles;
        me = me < enc_ntiles ? me : enc_ntiles;
        if (threadIdx.x == 0) {
            base[0] = atomicAdd(lists.counts, ms);
            base[1] = me ? atomicAdd(lists.counts + 1, me) : 0u;
        }
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < ms; k += kBlock) lists.surv[base[0] + k] = SurvTile{u, k * T};
        for (uint32_t k = threadIdx.x; k < me; k += kBlock) lists.enc[base[1] + k] = SurvTile{u, k * (uint32_t)kBlock};
    } else {
        if (u == 0 && threadIdx.x < 2) lists.counts[threadIdx.x] = 0;
        const uint32_t nn = st.n[current_pair(st)] - st.n_carry;
        uint32_t mo = (nn + d.off_per_tile - 1u) / d.off_per_tile;
        mo = mo < d.off_ntiles ? mo : d.off_ntiles;
        if (threadIdx.x == 0) base[0] = mo ? atomicAdd(lists.counts + 2u + d.off_class, mo) : 0u;
        __syncthreads();
        OffTile *off = lists.off + d.off_list0 + base[0];
        for (uint32_t k = threadIdx.x; k < mo; k += kBlock) off[k] = OffTile{u, k * d.off_per_tile};
    }
}

// ---------------------------------------------------------------- census

// One block per deme: sums of the tile partials of the newest census, or of
// the census itself (continuous alleles; carried survivors).
__global__ void __launch_bounds__(kBlock) census_kernel(const RepDesc *__restrict__ descs,
                                                        RepState *__restrict__ states,
                                                        const Partial *__restrict__ partials) {
    __shared__ int64_t sz[kBlock / 64];
    __shared__ uint64_t sz2[kBlock / 64];
    const uint32_t rep = blockIdx.x;
    RepState &st = states[rep];
    if (!st.census_pending) return;  // uniform over the block
    const RepDesc &d = descs[rep];
    if (d.cont) {
        // continuous alleles: the census is summed directly, in a fixed
        // order (floating-point sums: neither the tiles that made the census
        // nor the order of their atomics may change the result)
        double fa = 0.0, fb = 0.0;
        const uint32_t par = current_pair(st), n = st.n[par];
        const float *zf = reinterpret_cast<const float *>(d.z[st.t[par] & 1u]);
        for (uint32_t k = threadIdx.x; k < n; k += kBlock) {
            const double z = (double)zf[k];
            fa += z;
            fb += z * z;
        }
        fa = wave_sum<double>(fa);
        fb = wave_sum<double>(fb);
        __shared__ double fsz[kBlock / 64], fsz2[kBlock / 64];
        if (lane_id() == 0) {
            fsz[threadIdx.x >> 6] = fa;
            fsz2[threadIdx.x >> 6] = fb;
        }
        __syncthreads();
        if (threadIdx.x < kCensusSlots) {
            double sa = 0.0, sb = 0.0;
            if (threadIdx.x == 0)
                for (int w = 0; w < kBlock / 64; ++w) {
                    sa += fsz[w];
                    sb += fsz2[w];
                }
            st.sum_zf[threadIdx.x] = sa;
            st.sum_zf2[threadIdx.x] = sb;
        }
        if (threadIdx.x == 0) st.census_pending = 0;
        return;
    }
    int64_t a = 0;
    uint64_t b = 0;
    if (d.regime == SPEGG_CONSUMER_RESOURCE) {
        // carried survivors are not in the offspring partials: sum the census
        const uint32_t par = current_pair(st), n = st.n[par];
        const int32_t *z = d.z[st.t[par] & 1u];
        for (uint32_t k = threadIdx.x; k < n; k += kBlock) {
            a += z[k];
            b += (uint64_t)((int64_t)z[k] * (int64_t)z[k]);
        }
    } else {
        const uint32_t used = (st.n[current_pair(st)] + d.off_per_tile - 1u) / d.off_per_tile;
        for (uint32_t k = threadIdx.x; k < used; k += kBlock) {
            const Partial p = partials[d.off_tile0 + k];
            a += p.sum_z;
            b += p.sum_z2;
        }
    }
    a = wave_sum<int64_t>(a);
    b = wave_sum<uint64_t>(b);
    if (lane_id() == 0) {
        sz[threadIdx.x >> 6] = a;
        sz2[threadIdx.x >> 6] = b;
    }
    __syncthreads();
    if (threadIdx.x < kCensusSlots) {
        int64_t sa = 0;
        uint64_t sb = 0;
        if (threadIdx.x == 0)
            for (int w = 0; w < kBlock / 64; ++w) {
                sa += sz[w];
                sb += sz2[w];
            }
        st.sum_z[threadIdx.x] = sa;
        st.sum_z2[threadIdx.x] = sb;
    }
    if (threadIdx.x == 0) st.census_pending = 0;
}

// ---------------------------------------------------------------- consumer-resource

// One block per encounter tile of a consumer deme (kBlock consumers,
// whatever the survival tiles hold), one consumer per thread: every capture
// offers its key (consumer, encounter) to the captured resource, which
// keeps the lowest.  The keys were reset to ~0 when the resource census was
// written.
// The tile's capture thresholds (one table per consumer deme) are staged in
// LDS when they fit.
constexpr uint32_t kCaptureLds = 1024;
__device__ __forceinline__ void encounter_tile(const RepDesc *__restrict__ descs, const RepState *__restrict__ states,
                                               const SurvTile tile) {
    __shared__ uint64_t sh_cap[kCaptureLds];
    const uint32_t i = tile.start + threadIdx.x;
    const RepDesc &c = descs[tile.rep];
    const RepState &cs = states[tile.rep];
    const uint32_t par = current_pair(cs);
    const uint32_t t = cs.t[par], n = cs.n[par];
    const bool staged = c.cap_len <= kCaptureLds;  // uniform over the block
    if (staged) {
        __syncthreads();  // the block's previous tile has finished reading the table
        for (uint32_t q = threadIdx.x; q < c.cap_len; q += kBlock) sh_cap[q] = gload(c.capT + q);
        __syncthreads();
    }
    if (i >= n) return;
    gstore(c.intake + i, 0u);  // credit_kernel counts this generation's credited captures
    const RepDesc &r = descs[c.partner];
    const RepState &rs = states[c.partner];
    const uint32_t NR = rs.n[current_pair(rs)];
    const int32_t *zr = r.z[t & 1u];
    const int32_t *zc = c.z[t & 1u];
    unsigned long long *won = reinterpret_cast<unsigned long long *>(r.won);
    consumer_captures(c, i, t, zc[i], zr, NR, staged ? sh_cap : c.capT,
                      [&](uint32_t e, uint32_t tgt) { atomicMin(won + tgt, (unsigned long long)capture_key(i, e)); });
}

// A captured resource credits the consumer whose key it kept (the lowest
// (consumer, encounter) key of its captures): one atomic add to that
// consumer's intake.  Survival tiles of every deme; only the resources'
// act.  A thread's keys (one per kBlock resources of the tile) are all
// loaded before its first add.
__device__ __forceinline__ void credit_tile(const RepDesc *__restrict__ descs, const RepState *__restrict__ states,
                                            const SurvTile tile) {
    const RepDesc &r = descs[tile.rep];
    if (r.regime != SPEGG_CONSUMER_RESOURCE || r.species != 0) return;  // uniform over the block
    const RepState &rs = states[tile.rep];
    const uint32_t NR = rs.n[current_pair(rs)];
    uint64_t key[kSurvItemsMax];
#pragma unroll
    for (int q = 0; q < kSurvItemsMax; ++q) {
        const uint32_t k = threadIdx.x + (uint32_t)q * kBlock, j = tile.start + k;
        key[q] = (k < r.surv_tile && j < NR) ? gload(r.won + j) : ~0ull;
    }
    const RepDesc &c = descs[r.partner];
    const RepState &cs = states[r.partner];
    const uint32_t NC = cs.n[current_pair(cs)];
#pragma unroll
    for (int q = 0; q < kSurvItemsMax; ++q) {
        if (key[q] == ~0ull) continue;
        const uint32_t i = (uint32_t)(key[q] >> 32);
        if (i < NC) atomicAdd(c.intake + i, 1u);
        else atomicOr(const_cast<uint32_t *>(&rs.error), 1u);  // a key of no consumer: impossible
    }
}

__global__ void __launch_bounds__(kBlock) credit_kernel(const RepDesc *__restrict__ descs,
                                                        const RepState *__restrict__ states,
                                                        const SurvTile *__restrict__ tiles, uint32_t ntiles,
                                                        const uint32_t *__restrict__ list_n) {
    const uint32_t m = list_n ? *list_n : ntiles;
    for (uint32_t v = blockIdx.x; v < m; v += gridDim.x) credit_tile(descs, states, tiles[v]);
}

// Tiles [0, ntiles) of the plan, one block each, or the list_n occupied
// tiles of this generation's list, walked by a resident grid.
__global__ void __launch_bounds__(kBlock) encounter_kernel(const RepDesc *__restrict__ descs,
                                                           const RepState *__restrict__ states,
                                                           const SurvTile *__restrict__ tiles, uint32_t ntiles,
                                                           const uint32_t *__restrict__ list_n) {
    const uint32_t m = list_n ? *list_n : ntiles;
    for (uint32_t v = blockIdx.x; v < m; v += gridDim.x) encounter_tile(descs, states, tiles[v]);
}

__global__ void fill_u64_kernel(uint64_t *p, uint32_t n) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = ~0ull;
}

__global__ void fill_u8_kernel(uint8_t *p, uint32_t n) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void fill_u32_kernel(uint32_t *p, size_t n) {
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------- allele counts

// Copies of allele 1 at each locus over the current census (2N genes per
// locus; Fig. 1F, the genetic distribution the environment responds to).
// Thread (word w, slice of individuals) keeps 32 per-locus counters and adds
// them once; counts must be zero on entry.
__global__ void __launch_bounds__(kBlock) allele_count_kernel(const RepDesc *__restrict__ desc,
                                                              const RepState *__restrict__ state,
                                                              uint32_t *__restrict__ counts, uint32_t slice) {
    const RepDesc &d = *desc;
    const RepState &st = *state;
    const uint32_t par = current_pair(st);
    const uint32_t n = st.n[par], buf = st.t[par] & 1u;
    const uint32_t W = d.W;
    const uint64_t gid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint32_t w = (uint32_t)(gid % W), sl = (uint32_t)(gid / W);
    const uint32_t i_begin = sl * slice;
    if (i_begin >= n) return;
    const uint32_t i_end = i_begin + slice < n ? i_begin + slice : n;
    uint32_t c[32];
#pragma unroll
    for (int b = 0; b < 32; ++b) c[b] = 0;
    const uint32_t *g = d.genome[buf];
    for (uint32_t i = i_begin; i < i_end; ++i) {
        const uint32_t a = g[(size_t)i * 2u * W + w], b2 = g[(size_t)i * 2u * W + W + w];
#pragma unroll
        for (int b = 0; b < 32; ++b) c[b] += ((a >> b) & 1u) + ((b2 >> b) & 1u);
    }
    const uint32_t nb = w == W - 1u ? (d.L - 32u * w) : 32u;
    for (uint32_t b = 0; b < nb; ++b)
        if (c[b]) atomicAdd(&counts[32u * w + b], c[b]);
}

__global__ void philox_fill_kernel(uint32_t k0, uint32_t k1, const uint32_t *__restrict__ ctr,
                                   uint32_t *__restrict__ out, uint32_t n) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const Words4 w = philox(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1);
    for (int c = 0; c < 4; ++c) out[4 * i + c] = w.v[c];
}

inline uint32_t blocks_for(uint64_t n) { return (uint32_t)((n + kBlock - 1) / kBlock); }

// Every offspring kernel instance has this signature.
using OffspringKernel = void (*)(const RepDesc *, const RepState *, const OffTile *, uint32_t, uint32_t, int,
                                 Partial *, uint32_t, uint32_t, int, const uint32_t *);

template <int G, int V, bool EXT>
OffspringKernel offspring_kernel_gv(int nch) {
    switch (nch) {
    case 0: return offspring_kernel<G, V, 0, EXT>;
    case 1: return offspring_kernel<G, V, 1, EXT>;
    case 2: return offspring_kernel<G, V, 2, EXT>;
    case 4: return offspring_kernel<G, V, 4, EXT>;
    default: return nullptr;
    }
}

template <int V, bool EXT>
OffspringKernel offspring_kernel_v(int g, int nch) {
    switch (g) {
    case 1: return offspring_kernel_gv<1, V, EXT>(nch);
    case 2: return offspring_kernel_gv<2, V, EXT>(nch);
    case 4: return offspring_kernel_gv<4, V, EXT>(nch);
    case 8: return offspring_kernel_gv<8, V, EXT>(nch);
    case 16: return offspring_kernel_gv<16, V, EXT>(nch);
    case 32: return offspring_kernel_gv<32, V, EXT>(nch);
    default: return nullptr;
    }
}

template <bool EXT>
OffspringKernel offspring_kernel_ext(OffShape shape) {
    switch (shape.vpl) {
    case 1: return offspring_kernel_v<1, EXT>(shape.g, shape.nch);
    case 2: return offspring_kernel_v<2, EXT>(shape.g, shape.nch);
    case 4: return offspring_kernel_v<4, EXT>(shape.g, shape.nch);
    default: return nullptr;
    }
}

template <int G>
OffspringKernel offspring_cont_kernel_g(int nch) {
    switch (nch) {
    case 0: return offspring_cont_kernel<G, 0>;
    case 1: return offspring_cont_kernel<G, 1>;
    case 2: return offspring_cont_kernel<G, 2>;
    case 4: return offspring_cont_kernel<G, 4>;
    default: return nullptr;
    }
}

OffspringKernel offspring_cont_kernel_for(int g, int nch) {
    switch (g) {
    case 1: return offspring_cont_kernel_g<1>(nch);
    case 2: return offspring_cont_kernel_g<2>(nch);
    case 4: return offspring_cont_kernel_g<4>(nch);
    case 8: return offspring_cont_kernel_g<8>(nch);
    case 16: return offspring_cont_kernel_g<16>(nch);
    case 32: return offspring_cont_kernel_g<32>(nch);
    default: return nullptr;
    }
}

// The kernel instance of a shape, or null for a shape outside the set.
OffspringKernel offspring_kernel_for(OffShape shape) {
    if (shape.cont) return shape.vpl == 4 ? offspring_cont_kernel_for(shape.g, shape.nch) : nullptr;
    return shape.ext ? offspring_kernel_ext<true>(shape) : offspring_kernel_ext<false>(shape);
}

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_create(const RepDesc *descs, RepState *states, const SurvTile *tiles, uint32_t ntiles,
                         hipStream_t s) {
    if (ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(create_kernel, dim3(ntiles), dim3(kBlock), 0, s, descs, states, tiles);
    return hipGetLastError();
}

hipError_t launch_phenotypes(const RepDesc *d_desc, RepState *d_state, uint32_t n, uint32_t buf, uint32_t gen,
                             hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(phenotype_kernel, dim3(blocks_for(n)), dim3(kBlock), 0, s, d_desc, d_state, n, buf, gen);
    return hipGetLastError();
}

hipError_t launch_survive(const SelArgs &a) {
    if (a.list_n) {
        if (a.items == 4)
            hipLaunchKernelGGL(survive_list_kernel<4>, dim3(a.grid_survive), dim3(kBlock), 0, a.s, a.descs, a.states,
                               a.tiles, a.list_n, a.counts, a.groups);
        else if (a.items == 1)
            hipLaunchKernelGGL(survive_list_kernel<1>, dim3(a.grid_survive), dim3(kBlock), 0, a.s, a.descs, a.states,
                               a.tiles, a.list_n, a.counts, a.groups);
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    }
    if (a.items == 4)
        hipLaunchKernelGGL(survive_kernel<4>, dim3(a.ntiles), dim3(kBlock), 0, a.s, a.descs, a.states, a.tiles,
                           a.counts, a.groups, a.single_deme);
    else if (a.items == 1)
        hipLaunchKernelGGL(survive_kernel<1>, dim3(a.ntiles), dim3(kBlock), 0, a.s, a.descs, a.states, a.tiles,
                           a.counts, a.groups, a.single_deme);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_compact(const SelArgs &a) {
    if (a.list_n) {
        if (a.items == 4)
            hipLaunchKernelGGL(compact_list_kernel<4>, dim3(a.grid_compact), dim3(kBlock), 0, a.s, a.descs, a.states,
                               a.tiles, a.list_n, a.counts, a.groups, a.trace);
        else if (a.items == 1)
            hipLaunchKernelGGL(compact_list_kernel<1>, dim3(a.grid_compact), dim3(kBlock), 0, a.s, a.descs, a.states,
                               a.tiles, a.list_n, a.counts, a.groups, a.trace);
        else
            return hipErrorInvalidValue;
        return hipGetLastError();
    }
    if (a.items == 4)
        hipLaunchKernelGGL(compact_kernel<4>, dim3(a.ntiles), dim3(kBlock), 0, a.s, a.descs, a.states, a.tiles,
                           a.counts, a.groups, a.trace, a.single_deme);
    else if (a.items == 1)
        hipLaunchKernelGGL(compact_kernel<1>, dim3(a.ntiles), dim3(kBlock), 0, a.s, a.descs, a.states, a.tiles,
                           a.counts, a.groups, a.trace, a.single_deme);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_offspring(OffShape shape, const OffArgs &a) {
    const OffspringKernel k = offspring_kernel_for(shape);
    if (!k) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k, dim3(a.grid), dim3(kBlock), a.lds, a.s, a.descs, a.states, a.tiles, a.tile0, a.ntiles,
                       a.single_deme, a.partials, shape.cont ? a.mask_words : a.plane_words, a.geo_words, a.trace,
                       a.list_n);
    return hipGetLastError();
}

hipError_t offspring_blocks_per_cu(OffShape shape, size_t lds, int *blocks) {
    const OffspringKernel k = offspring_kernel_for(shape);
    if (!k) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k, kBlock, lds);
}

hipError_t launch_census(const RepDesc *descs, RepState *states, const Partial *partials, uint32_t n_reps,
                         hipStream_t s) {
    hipLaunchKernelGGL(census_kernel, dim3(n_reps), dim3(kBlock), 0, s, descs, states, partials);
    return hipGetLastError();
}

hipError_t launch_encounter(const RepDesc *descs, const RepState *states, const SurvTile *tiles, uint32_t ntiles,
                            const uint32_t *list_n, uint32_t grid, hipStream_t s) {
    if (ntiles == 0) return hipSuccess;
    const uint32_t blocks = list_n ? (grid < ntiles ? grid : ntiles) : ntiles;
    hipLaunchKernelGGL(encounter_kernel, dim3(blocks), dim3(kBlock), 0, s, descs, states, tiles, ntiles, list_n);
    return hipGetLastError();
}

hipError_t launch_credit(const RepDesc *descs, const RepState *states, const SurvTile *tiles, uint32_t ntiles,
                         const uint32_t *list_n, uint32_t grid, hipStream_t s) {
    if (ntiles == 0) return hipSuccess;
    const uint32_t blocks = list_n ? (grid < ntiles ? grid : ntiles) : ntiles;
    hipLaunchKernelGGL(credit_kernel, dim3(blocks), dim3(kBlock), 0, s, descs, states, tiles, ntiles, list_n);
    return hipGetLastError();
}

hipError_t launch_plan_tiles(const RepDesc *descs, const RepState *states, uint32_t n_demes, const TileLists &lists,
                             int phase, hipStream_t s) {
    if (n_demes == 0) return hipSuccess;
    hipLaunchKernelGGL(plan_tiles_kernel, dim3(n_demes), dim3(kBlock), 0, s, descs, states, lists, phase);
    return hipGetLastError();
}

hipError_t list_blocks_per_cu(int kind, int items, int *blocks) {
    *blocks = 0;
    const void *k = nullptr;
    if (kind == 0) k = items == 4 ? (const void *)survive_list_kernel<4> : (const void *)survive_list_kernel<1>;
    else if (kind == 1) k = items == 4 ? (const void *)compact_list_kernel<4> : (const void *)compact_list_kernel<1>;
    else if (kind == 2) k = (const void *)encounter_kernel;
    else return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k, kBlock, 0);
}

hipError_t launch_fill_u64(uint64_t *p, uint32_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks_for(n)), dim3(kBlock), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t *p, uint32_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u8_kernel, dim3(blocks_for(n)), dim3(kBlock), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks_for(n)), dim3(kBlock), 0, s, p, n);
    return hipGetLastError();
}

hipError_t allele_scratch(uint32_t **out, size_t *words) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static uint32_t *addr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        // the device's own address of its copy, taken with that device current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<uint32_t *>(p);
    }
    *out = addr[dev];
    *words = SPEGG_MAX_LOCI;
    return hipSuccess;
}

hipError_t launch_allele_counts(const RepDesc *d_desc, const RepState *d_state, const RepDesc &h, uint32_t n,
                                uint32_t *counts, hipStream_t s) {
    constexpr uint32_t kSlice = 256;  // individuals per thread
    const uint64_t threads = (uint64_t)h.W * ((n + kSlice - 1) / kSlice);
    if (threads == 0) return hipSuccess;
    hipLaunchKernelGGL(allele_count_kernel, dim3(blocks_for(threads)), dim3(kBlock), 0, s, d_desc, d_state, counts,
                       kSlice);
    return hipGetLastError();
}

// Philox throughput probe: thread i folds (XOR) the four words of blocks
// with counters (i, k, 0, 0), k < m, into out[i]; no other memory traffic.
__global__ void __launch_bounds__(kBlock) philox_rate_kernel(uint32_t k0, uint32_t k1, uint32_t m,
                                                             uint32_t *__restrict__ out, uint32_t n) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    uint32_t acc = 0;
    for (uint32_t k = 0; k < m; ++k) {
        const Words4 w = philox(i, k, 0u, 0u, k0, k1);
        acc ^= w.v[0] ^ w.v[1] ^ w.v[2] ^ w.v[3];
    }
    out[i] = acc;
}
hipError_t launch_philox_rate(uint32_t k0, uint32_t k1, uint32_t m, uint32_t *out, uint32_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(philox_rate_kernel, dim3(blocks_for(n)), dim3(kBlock), 0, s, k0, k1, m, out, n);
    return hipGetLastError();
}
hipError_t launch_philox_fill(uint32_t k0, uint32_t k1, const uint32_t *ctr, uint32_t *out, uint32_t n,
                              hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(philox_fill_kernel, dim3(blocks_for(n)), dim3(kBlock), 0, s, k0, k1, ctr, out, n);
    return hipGetLastError();
}

}  // namespace spegg

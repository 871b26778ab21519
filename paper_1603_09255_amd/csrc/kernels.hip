// Kernels of one generation (main text, Fig. 1) for gfx950.
//
//   survive   D + the fecundity draw of A: per adult, p = v(z) s(N), one
//             Philox word against floor(p 2^32); per-tile counts
//   scan      per replicate: exclusive prefix sums of the tile counts,
//             survivor count, neonate count N_{t+1}; advances the
//             generation and clears the census sums
//   compact   E: ballot/mbcnt ranks -> ascending survivor list; Poisson
//             regime: each mother writes her offspring slots
//   offspring A (parents) + B (gametes: crossover mask, mutation flips)
//             + C (additive phenotype by popcounts) + census sums; one
//             team of 2G lanes per newborn, V consecutive words per lane
//
// All of it is integer work except p = v s (IEEE double, no contraction),
// so every result is reproducible bit for bit.
#include <hip/hip_runtime.h>

#include "philox.h"
#include "spegg_internal.h"

namespace spegg {

namespace {

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(v, o, 64);
        if (lane >= (uint32_t)o) v += t;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Exclusive prefix over the block (kBlock threads = 4 waves); *total gets
// the block sum.  Every thread of the block must call it.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *sh, uint32_t *total) {
    const uint32_t incl = wave_incl_scan(v);
    const uint32_t wave = threadIdx.x >> 6;
    if (lane_id() == 63) sh[wave] = incl;
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

// Additive contribution sum_l e_l b_l of one haplotype word.
__device__ __forceinline__ int32_t word_effect(const RepDesc &d, uint32_t w, uint32_t g) {
    if (d.unit_effects) return (int32_t)__popc(g);
    const uint32_t *P = d.planes;
    const uint32_t W = d.W;
    return (int32_t)__popc(g & P[w]) + 2 * (int32_t)__popc(g & P[W + w]) + 4 * (int32_t)__popc(g & P[2 * W + w]) -
           (int32_t)__popc(g & P[3 * W + w]) - 2 * (int32_t)__popc(g & P[4 * W + w]) -
           4 * (int32_t)__popc(g & P[5 * W + w]);
}

template <int V>
struct Words {
    uint32_t v[V];
};

template <int V>
__device__ __forceinline__ Words<V> load_words(const uint32_t *p) {
    Words<V> w;
    if constexpr (V == 4) {
        const uint4 q = *reinterpret_cast<const uint4 *>(p);
        w.v[0] = q.x;
        w.v[1] = q.y;
        w.v[2] = q.z;
        w.v[3] = q.w;
    } else if constexpr (V == 2) {
        const uint2 q = *reinterpret_cast<const uint2 *>(p);
        w.v[0] = q.x;
        w.v[1] = q.y;
    } else {
        w.v[0] = *p;
    }
    return w;
}

template <int V>
__device__ __forceinline__ void store_words(uint32_t *p, const Words<V> &w) {
    if constexpr (V == 4) {
        *reinterpret_cast<uint4 *>(p) = make_uint4(w.v[0], w.v[1], w.v[2], w.v[3]);
    } else if constexpr (V == 2) {
        *reinterpret_cast<uint2 *>(p) = make_uint2(w.v[0], w.v[1]);
    } else {
        *p = w.v[0];
    }
}

// Number of geometric-gap thresholds T[0..len) that are <= x: the gap of
// the inverse-CDF draw.  A float guess floor(log2(1 - x/2^32) / log2(1 - r))
// is corrected against the table, so the table alone decides.
__device__ __forceinline__ uint32_t geometric_gap(const RepDesc &d, uint32_t x) {
    const uint32_t len = d.geo_len;
    const float lg = __log2f((float)(4294967296.0 - (double)x)) - 32.0f;
    const float guess = lg * d.geo_scale;
    uint32_t g = guess >= (float)len ? len : (guess > 0.0f ? (uint32_t)guess : 0u);
    const uint64_t *T = d.geo;
    const uint64_t below = g > 0 ? T[g - 1] : 0ull;   // both checks load at once
    const uint64_t above = g < len ? T[g] : kAlways;
    if (below > (uint64_t)x || above <= (uint64_t)x) {
        while (g > 0 && T[g - 1] > (uint64_t)x) --g;
        while (g < len && T[g] <= (uint64_t)x) ++g;
    }
    return g;
}

// Crossovers of one 32-boundary block under the bit-serial comparison
// U < R: U's bits, from the top, are successive words of the block's
// stream; a boundary is decided at its first bit differing from R.
__device__ __forceinline__ uint32_t lazy_block(const Rng &rng, uint32_t j, uint32_t rs, uint32_t tp, uint32_t w,
                                               uint32_t R) {
    uint32_t und = ~0u, hit = 0;
    for (int i = 31; i >= 0; i -= 4) {
        const Words4 blk = rng.block(j, rs, 1u + w * 8u + (uint32_t)((31 - i) >> 2), tp);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int b = i - c;
            const uint32_t rest = b == 31 ? R : (R & ((1u << (b + 1)) - 1u));
            if (rest == 0 || und == 0) return hit;
            const uint32_t x = blk.v[c];
            if ((R >> b) & 1u) {
                hit |= und & ~x;
                und &= x;
            } else {
                und &= ~x;
            }
        }
    }
    return hit;
}

// ---------------------------------------------------------------- init

__global__ void __launch_bounds__(kBlock) init_kernel(const RepDesc *__restrict__ desc, uint32_t n0) {
    const RepDesc &d = *desc;
    const uint32_t per = 2u * d.W;
    const uint64_t idx = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (uint64_t)n0 * per) return;
    const uint32_t i = (uint32_t)(idx / per), q = (uint32_t)(idx % per);
    const Rng rng{d.key0, d.key1, d.c3};
    uint32_t word = rng.seq(i, kStInit, q, 0);
    if (q % d.W == d.W - 1) word &= d.tail_mask;
    d.genome[0][idx] = word;
}

// z for n individuals of buffer buf, and their census sums.
__global__ void __launch_bounds__(kBlock) phenotype_kernel(const RepDesc *__restrict__ desc,
                                                           RepState *__restrict__ state, uint32_t n, uint32_t buf) {
    const RepDesc &d = *desc;
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    int64_t z = 0;
    if (i < n) {
        const uint32_t *g = d.genome[buf] + (size_t)i * 2u * d.W;
        int32_t acc = 0;
        for (uint32_t w = 0; w < d.W; ++w) acc += word_effect(d, w, g[w]) + word_effect(d, w, g[d.W + w]);
        z = (int64_t)acc - d.sum_e;
        d.z[buf][i] = (int32_t)z;
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

__global__ void __launch_bounds__(kBlock) survive_kernel(const RepDesc *__restrict__ descs,
                                                         const RepState *__restrict__ states,
                                                         const SurvTile *__restrict__ tiles,
                                                         SurvCount *__restrict__ counts) {
    __shared__ uint32_t sh_u[3][kBlock / 64];
    __shared__ uint64_t sh_t[kBlock / 64];
    const SurvTile tile = tiles[blockIdx.x];
    const RepDesc &d = descs[tile.rep];
    const RepState &st = states[tile.rep];
    const uint32_t n = st.n, t = st.t;
    const uint32_t i = tile.start + threadIdx.x;
    uint32_t alive = 0, kids = 0, near = 0;
    uint64_t thr = 0;
    if (i < n) {
        const int32_t z = d.z[t & 1u][i];
        const double v = d.vtab ? d.vtab[z - d.zmin] : 1.0;
        const double p = v * density_factor(d, n);
        thr = p >= 1.0 ? kAlways : (p > 0.0 ? (uint64_t)floor(p * 4294967296.0) : 0ull);
        const Rng rng{d.key0, d.key1, d.c3};
        const uint32_t x = rng.block(i, kStSurvive, 0, t).v[0];
        alive = (uint64_t)x < thr;
        near = (p > 0.0 && p < 1.0 && fabs((double)x * (1.0 / 4294967296.0) - p) < 1e-6) ? 1u : 0u;
        if (alive && d.regime == SPEGG_POISSON_BH) {
            const uint32_t xf = rng.block(i, kStFecund, 0, t).v[0];
            kids = table_draw(d.pois, d.pois_len, xf);
        }
        d.fate[i] = (uint16_t)(alive ? (0x8000u | kids) : 0u);
    }
    const uint32_t wave = threadIdx.x >> 6;
    const uint64_t ballot = __ballot(alive);
    const uint32_t k = wave_sum<uint32_t>(kids), nr = wave_sum<uint32_t>(near);
    const uint64_t ts = wave_sum<uint64_t>(thr);
    if (lane_id() == 0) {
        sh_u[0][wave] = (uint32_t)__popcll(ballot);
        sh_u[1][wave] = k;
        sh_u[2][wave] = nr;
        sh_t[wave] = ts;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        SurvCount c{};
        for (int w = 0; w < kBlock / 64; ++w) {
            c.alive += sh_u[0][w];
            c.kids += sh_u[1][w];
            c.near += sh_u[2][w];
            c.sum_t += sh_t[w];
        }
        counts[blockIdx.x] = c;
    }
}

// ---------------------------------------------------------------- scan

// One block per replicate: offsets of every survival tile, neonate count,
// and the advance of the replicate to the next generation.
__global__ void __launch_bounds__(kBlock) scan_kernel(const RepDesc *__restrict__ descs,
                                                      RepState *__restrict__ states,
                                                      SurvCount *__restrict__ counts, int trace) {
    constexpr int PER = 4;  // tiles per thread per pass, loaded together
    __shared__ uint32_t sh[2][kBlock / 64];
    __shared__ uint64_t sh64[2][kBlock / 64];
    const uint32_t rep = blockIdx.x;
    const RepDesc &d = descs[rep];
    RepState &st = states[rep];
    const uint32_t ntiles = d.surv_ntiles;
    SurvCount *c = counts + d.surv_tile0;
    uint32_t alive_carry = 0;
    uint64_t kid_carry = 0, near_sum = 0, t_sum = 0;
    for (uint32_t base = 0; base < ntiles; base += kBlock * PER) {
        const uint32_t k0 = base + threadIdx.x * PER;
        uint32_t a[PER], kk[PER], ta = 0, tk = 0;
        uint64_t nr = 0, ts = 0;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const bool ok = k0 + q < ntiles;
            const SurvCount v = ok ? c[k0 + q] : SurvCount{};
            a[q] = v.alive;
            kk[q] = v.kids;
            ta += v.alive;
            tk += v.kids;
            nr += v.near;
            ts += v.sum_t;
        }
        uint32_t tot_a, tot_k;
        const uint32_t ea = block_excl_scan(ta, sh[0], &tot_a);
        const uint32_t ek = block_excl_scan(tk, sh[1], &tot_k);
        uint32_t ra = alive_carry + ea;
        uint64_t rk = kid_carry + ek;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            if (k0 + q < ntiles) {
                c[k0 + q].alive_off = ra;
                c[k0 + q].kid_off = rk > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)rk;
            }
            ra += a[q];
            rk += kk[q];
        }
        alive_carry += tot_a;
        kid_carry += tot_k;
        nr = wave_sum<uint64_t>(nr);
        ts = wave_sum<uint64_t>(ts);
        if (lane_id() == 0) {
            sh64[0][threadIdx.x >> 6] = nr;
            sh64[1][threadIdx.x >> 6] = ts;
        }
        __syncthreads();
        for (int w = 0; w < kBlock / 64; ++w) {
            near_sum += sh64[0][w];
            t_sum += sh64[1][w];
        }
        __syncthreads();
    }
    if (threadIdx.x < kCensusSlots) {
        st.sum_z[threadIdx.x] = 0;
        st.sum_z2[threadIdx.x] = 0;
    }
    if (threadIdx.x == 0) {
        const uint32_t n = st.n, ns = alive_carry;
        uint32_t nn;
        if (ns == 0) {
            nn = 0;
        } else if (d.regime == SPEGG_WF) {
            nn = n;
        } else {
            nn = kid_carry > d.cap ? d.cap : (uint32_t)kid_carry;
            st.truncated += kid_carry - nn;
        }
        st.n_prev = n;
        st.n_surv = ns;
        st.n = nn;
        st.t += 1;
        if (nn == 0) st.extinct = 1;
        st.traced = trace ? 1u : 0u;
        st.census_pending = 1;
        st.near_ties += near_sum;
        st.sum_threshold = t_sum;
        st.updates += (uint64_t)nn * d.L;
    }
}

// ---------------------------------------------------------------- compact

__global__ void __launch_bounds__(kBlock) compact_kernel(const RepDesc *__restrict__ descs,
                                                         const RepState *__restrict__ states,
                                                         const SurvTile *__restrict__ tiles,
                                                         const SurvCount *__restrict__ counts) {
    __shared__ uint32_t sh_a[kBlock / 64];
    __shared__ uint32_t sh_k[kBlock / 64];
    const SurvTile tile = tiles[blockIdx.x];
    const RepDesc &d = descs[tile.rep];
    const RepState &st = states[tile.rep];
    const uint32_t n = st.n_prev;  // the adults this generation started from
    if (tile.start >= n) return;   // uniform over the block
    const uint32_t i = tile.start + threadIdx.x;
    const uint32_t f = i < n ? d.fate[i] : 0u;
    const uint32_t alive = f >> 15, kids = f & 0x7FFFu;
    // survivor rank: ballot within the wave, wave totals through LDS
    const uint32_t wave = threadIdx.x >> 6;
    const uint64_t ballot = __ballot(alive);
    const uint32_t rank_in_wave = __builtin_amdgcn_mbcnt_hi((uint32_t)(ballot >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)ballot, 0u));
    if (lane_id() == 0) sh_a[wave] = (uint32_t)__popcll(ballot);
    uint32_t ktot;
    const uint32_t kid_rank = block_excl_scan(kids, sh_k, &ktot);  // contains __syncthreads
    uint32_t wave_off = 0;
    for (uint32_t w = 0; w < wave; ++w) wave_off += sh_a[w];
    const SurvCount c = counts[blockIdx.x];
    if (alive) d.S[c.alive_off + wave_off + rank_in_wave] = i;
    if (d.regime == SPEGG_POISSON_BH && kids) {
        const uint32_t nn = st.n;
        const uint64_t slot0 = (uint64_t)c.kid_off + kid_rank;
        for (uint32_t m = 0; m < kids; ++m) {
            const uint64_t slot = slot0 + m;
            if (slot < nn) d.owner[slot] = i;
        }
    }
}

// ---------------------------------------------------------------- offspring

// One team of 2G lanes makes one newborn: lanes [0, G) build the maternal
// gamete (haplotype 0), lanes [G, 2G) the paternal one; in each chunk of
// G x V words, lane g handles V consecutive words from g x V.
template <int G, int V>
__global__ void __launch_bounds__(kBlock) offspring_kernel(const RepDesc *__restrict__ descs,
                                                           RepState *__restrict__ states,
                                                           const OffTile *__restrict__ tiles, uint32_t tile0,
                                                           uint32_t ntiles, int single_rep,
                                                           Partial *__restrict__ partials, int trace) {
    constexpr uint32_t TPO = 2 * G;
    constexpr uint32_t TEAMS = kBlock / TPO;
    constexpr uint32_t ITERS = TEAMS >= 16 ? 1 : 16 / TEAMS;
    constexpr uint32_t OPT = TEAMS * ITERS;
    constexpr uint32_t CH = G * V;  // words of one gamete per chunk
    extern __shared__ uint32_t lds[];
    __shared__ int64_t red_z[kBlock / 64];
    __shared__ uint64_t red_z2[kBlock / 64];

    const uint32_t team = threadIdx.x / TPO, lane = threadIdx.x % TPO;
    const uint32_t half = lane / G, gl = lane % G;
    const uint32_t seg0 = lane_id() - gl;  // first wave lane of this gamete's lanes
    const uint32_t segmask = G >= 32 ? 0xFFFFFFFFu : ((1u << G) - 1u);

    uint32_t limit = ntiles;
    if (single_rep >= 0) {
        const uint32_t nn = states[single_rep].n;
        const uint32_t active = (nn + OPT - 1) / OPT;
        limit = active < ntiles ? active : ntiles;
    }
    for (uint32_t ti = blockIdx.x; ti < limit; ti += gridDim.x) {
        uint32_t rep, start;
        if (single_rep >= 0) {
            rep = (uint32_t)single_rep;
            start = ti * OPT;
        } else {
            const OffTile tile = tiles[tile0 + ti];
            rep = tile.rep;
            start = tile.start;
        }
        const RepDesc &d = descs[rep];
        RepState &st = states[rep];
        const uint32_t nn = st.n;
        if (start >= nn) continue;  // uniform over the block
        const uint32_t tp = st.t - 1u, ns = st.n_surv, cur = tp & 1u;
        const uint32_t W = d.W, L = d.L, mode = d.mode;
        const uint64_t binom0 = d.binom[0];  // most gametes carry no mutation
        const Rng rng{d.key0, d.key1, d.c3};
        uint32_t *X = lds + (size_t)(team * 2u + half) * 2u * W;  // crossover toggles
        uint32_t *F = X + W;                                        // mutation flips
        int64_t my_z = 0;
        uint64_t my_z2 = 0;

        for (uint32_t it = 0; it < ITERS; ++it) {
            const uint32_t j = start + it * TEAMS + team;
            if (j >= nn) continue;  // uniform over the team

            // A: parents, uniform over the survivors (Poisson: the slot's mother)
            const Words4 pw = rng.block(j, kStParent, 0, tp);
            const uint32_t mom = d.regime == SPEGG_WF ? d.S[uniform_index(pw.v[0], pw.v[1], ns)] : d.owner[j];
            const uint32_t dad = d.S[uniform_index(pw.v[2], pw.v[3], ns)];
            const uint32_t *__restrict__ src = d.genome[cur] + (size_t)(half ? dad : mom) * 2u * W;
            uint32_t *__restrict__ dst = d.genome[cur ^ 1u] + (size_t)j * 2u * W + (size_t)half * W;
            const uint32_t rs = kStRecomb + half, ms = kStMutate + half;

            // first chunk of the parent's haplotypes, in flight while the
            // crossover mask is drawn
            uint32_t w0 = gl * V;
            Words<V> h0{}, h1{};
            if (w0 < W) {
                h0 = load_words<V>(src + w0);
                h1 = load_words<V>(src + W + w0);
            }

            // B1: crossover toggles.  Boundary b (between loci b-1 and b)
            // toggles the source haplotype from locus b on; bit 0 of word 0
            // holds the phase (which haplotype locus 0 copies).
            uint32_t phase = 0;
            if (mode != kModeRaw) phase = rng.block(j, rs, 0, tp).v[0] & 1u;
            if (mode == kModeSkip) {
                for (uint32_t w = gl * V; w < W; w += CH)
#pragma unroll
                    for (int v = 0; v < V; ++v) X[w + v] = 0;
                wave_lds_sync();
                // gaps come four to a Philox block from block 1 on; lane g
                // takes block blk + g, so a pass places up to 4G crossovers
                uint32_t b = 0, blk = 1;
                for (;;) {
                    const Words4 xw = rng.block(j, rs, blk + gl, tp);
                    uint32_t cum[4];
                    uint32_t acc = 0;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        acc += 1u + geometric_gap(d, xw.v[c]);
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
            }

            // B2: mutation, K ~ Binomial(L, mu) distinct loci flipped
            const uint32_t xk = rng.block(j, ms, 0, tp).v[0];
            const uint32_t K = (uint64_t)xk < binom0 ? 0u : table_draw(d.binom, d.binom_len, xk);
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
            int32_t zc = 0;
            uint32_t carry = 0;  // parity of the toggles in earlier chunks
            for (uint32_t base = 0; base < W; base += CH) {
                w0 = base + gl * V;
                const bool valid = w0 < W;
                if (base > 0 && valid) {
                    h0 = load_words<V>(src + w0);
                    h1 = load_words<V>(src + W + w0);
                }
                Words<V> M;
                if (mode == kModeRaw) {
                    const Words4 blk = rng.block(j, rs, w0 >> 2, tp);
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const uint32_t c = (w0 + v) & 3u;
                        M.v[v] = c == 0 ? blk.v[0] : c == 1 ? blk.v[1] : c == 2 ? blk.v[2] : blk.v[3];
                    }
                } else {
                    uint32_t lane_par = 0;
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const uint32_t w = w0 + v;
                        uint32_t tog = 0;
                        if (valid) {
                            if (mode == kModeSkip) tog = X[w];
                            else if (mode == kModeLazy) tog = lazy_block(rng, j, rs, tp, w, d.R);
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
                        uint32_t x = (h0.v[v] & ~M.v[v]) | (h1.v[v] & M.v[v]);
                        if (K > 0) x ^= F[w0 + v];
                        if (w0 + v == W - 1u) x &= d.tail_mask;
                        g.v[v] = x;
                        zc += word_effect(d, w0 + v, x);
                    }
                    store_words<V>(dst + w0, g);
                }
            }
#pragma unroll
            for (int o = 1; o < (int)TPO; o <<= 1) zc += __shfl_xor(zc, o, TPO);
            if (lane == 0) {
                const int32_t z = zc - d.sum_e;
                d.z[cur ^ 1u][j] = z;
                my_z += z;
                my_z2 += (uint64_t)((int64_t)z * (int64_t)z);
                if (trace) {
                    d.mom[j] = mom;
                    d.dad[j] = dad;
                }
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
            partials[tile0 + ti] = Partial{a, b};
        }
        __syncthreads();
    }
}

// One block per replicate: sums of the tile partials of the newest census.
__global__ void __launch_bounds__(kBlock) census_kernel(const RepDesc *__restrict__ descs,
                                                        RepState *__restrict__ states,
                                                        const Partial *__restrict__ partials) {
    __shared__ int64_t sz[kBlock / 64];
    __shared__ uint64_t sz2[kBlock / 64];
    const uint32_t rep = blockIdx.x;
    RepState &st = states[rep];
    if (!st.census_pending) return;  // uniform over the block
    const RepDesc &d = descs[rep];
    const uint32_t used = (st.n + d.off_per_tile - 1u) / d.off_per_tile;
    int64_t a = 0;
    uint64_t b = 0;
    for (uint32_t k = threadIdx.x; k < used; k += kBlock) {
        const Partial p = partials[d.off_tile0 + k];
        a += p.sum_z;
        b += p.sum_z2;
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

__global__ void philox_fill_kernel(uint32_t k0, uint32_t k1, const uint32_t *__restrict__ ctr,
                                   uint32_t *__restrict__ out, uint32_t n) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const Words4 w = philox(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1);
    for (int c = 0; c < 4; ++c) out[4 * i + c] = w.v[c];
}

inline uint32_t blocks_for(uint64_t n) { return (uint32_t)((n + kBlock - 1) / kBlock); }

struct OffArgs {
    const RepDesc *descs;
    RepState *states;
    const OffTile *tiles;
    uint32_t tile0, ntiles;
    int single_rep;
    Partial *partials;
    uint32_t grid;
    size_t lds;
    int trace;
    hipStream_t s;
};

template <int G, int V>
hipError_t launch_offspring_gv(const OffArgs &a) {
    hipLaunchKernelGGL((offspring_kernel<G, V>), dim3(a.grid), dim3(kBlock), a.lds, a.s, a.descs, a.states, a.tiles,
                       a.tile0, a.ntiles, a.single_rep, a.partials, a.trace);
    return hipGetLastError();
}

template <int V>
hipError_t launch_offspring_v(int g, const OffArgs &a) {
    switch (g) {
    case 1: return launch_offspring_gv<1, V>(a);
    case 2: return launch_offspring_gv<2, V>(a);
    case 4: return launch_offspring_gv<4, V>(a);
    case 8: return launch_offspring_gv<8, V>(a);
    case 16: return launch_offspring_gv<16, V>(a);
    case 32: return launch_offspring_gv<32, V>(a);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_init(const RepDesc *d_desc, const RepDesc &h, uint32_t n0, hipStream_t s) {
    const uint64_t words = (uint64_t)n0 * 2u * h.W;
    if (words == 0) return hipSuccess;
    hipLaunchKernelGGL(init_kernel, dim3(blocks_for(words)), dim3(kBlock), 0, s, d_desc, n0);
    return hipGetLastError();
}

hipError_t launch_phenotypes(const RepDesc *d_desc, RepState *d_state, uint32_t n, uint32_t buf, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(phenotype_kernel, dim3(blocks_for(n)), dim3(kBlock), 0, s, d_desc, d_state, n, buf);
    return hipGetLastError();
}

hipError_t launch_survive(const RepDesc *descs, const RepState *states, const SurvTile *tiles, SurvCount *counts,
                          uint32_t ntiles, hipStream_t s) {
    hipLaunchKernelGGL(survive_kernel, dim3(ntiles), dim3(kBlock), 0, s, descs, states, tiles, counts);
    return hipGetLastError();
}

hipError_t launch_scan(const RepDesc *descs, RepState *states, SurvCount *counts, uint32_t n_reps, int trace,
                       hipStream_t s) {
    hipLaunchKernelGGL(scan_kernel, dim3(n_reps), dim3(kBlock), 0, s, descs, states, counts, trace);
    return hipGetLastError();
}

hipError_t launch_compact(const RepDesc *descs, const RepState *states, const SurvTile *tiles,
                          const SurvCount *counts, uint32_t ntiles, hipStream_t s) {
    hipLaunchKernelGGL(compact_kernel, dim3(ntiles), dim3(kBlock), 0, s, descs, states, tiles, counts);
    return hipGetLastError();
}

hipError_t launch_offspring(OffShape shape, const RepDesc *descs, RepState *states, const OffTile *tiles,
                            uint32_t tile0, uint32_t ntiles, int single_rep, Partial *partials, uint32_t grid,
                            size_t lds, int trace, hipStream_t s) {
    const OffArgs a{descs, states, tiles, tile0, ntiles, single_rep, partials, grid, lds, trace, s};
    switch (shape.vpl) {
    case 1: return launch_offspring_v<1>(shape.g, a);
    case 2: return launch_offspring_v<2>(shape.g, a);
    case 4: return launch_offspring_v<4>(shape.g, a);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_census(const RepDesc *descs, RepState *states, const Partial *partials, uint32_t n_reps,
                         hipStream_t s) {
    hipLaunchKernelGGL(census_kernel, dim3(n_reps), dim3(kBlock), 0, s, descs, states, partials);
    return hipGetLastError();
}

hipError_t launch_philox_fill(uint32_t k0, uint32_t k1, const uint32_t *ctr, uint32_t *out, uint32_t n,
                              hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(philox_fill_kernel, dim3(blocks_for(n)), dim3(kBlock), 0, s, k0, k1, ctr, out, n);
    return hipGetLastError();
}

}  // namespace spegg

// Host-built decision tables.  Every random decision on the device is an
// integer comparison of a 32-bit Philox word x against a threshold:
//   Bernoulli(p):       x < floor(p 2^32)            (p >= 1: 2^32, always)
//   discrete inversion: k = min{k : x < T_k},  T_k = floor(F(k) 2^32),
//                       the last entry 2^32; a table closes at the first k
//                       whose T_k reaches 2^32 - 1.
// Distribution functions are accumulated term by term in x87 extended
// precision, so each table is a fixed function of its parameters.
#include "tables.h"

#include <cmath>

namespace spegg {

namespace {
constexpr long double kTwo32 = 4294967296.0L;

// Returns true when entry k closes the table.
bool put(std::vector<uint64_t> &T, long double cdf, int k, int cap) {
    const long double s = floorl(cdf * kTwo32);
    if (s >= 4294967295.0L || k == cap - 1) {
        T.push_back(kAlways);
        return true;
    }
    T.push_back((uint64_t)s);
    return false;
}
}  // namespace

uint64_t prob_threshold(double p) {
    if (p >= 1.0) return kAlways;
    if (!(p > 0.0)) return 0;
    return (uint64_t)std::floor(p * 4294967296.0);
}

// Poisson(lambda): p_0 = e^-lambda, p_k = p_{k-1} lambda / k.
bool poisson_table(double lambda, int cap, std::vector<uint64_t> &T) {
    T.clear();
    if (!(lambda >= 0.0) || cap < 1) return false;
    const long double lam = lambda;
    long double p = expl(-lam), F = 0.0L;
    for (int k = 0; k < cap; ++k) {
        if (k > 0) p = p * lam / (long double)k;
        F += p;
        if (put(T, F, k, cap)) return k < cap - 1 || floorl(F * kTwo32) >= 4294967295.0L;
    }
    return false;
}

// Binomial(L, mu), 0 <= mu < 1: p_0 = (1-mu)^L, p_k = p_{k-1} (L-k+1)/k mu/(1-mu).
bool binomial_table(uint32_t L, double mu, int cap, std::vector<uint64_t> &T) {
    T.clear();
    if (!(mu >= 0.0 && mu < 1.0) || cap < 1) return false;
    const long double m = mu;
    long double p = powl(1.0L - m, (long double)L), F = 0.0L;
    for (int k = 0; k < cap; ++k) {
        if (k > 0) p = (uint32_t)k > L ? 0.0L : p * (long double)(L - (uint32_t)k + 1u) / (long double)k * m / (1.0L - m);
        F += p;
        if ((uint32_t)k == L) {
            T.push_back(kAlways);
            return true;
        }
        if (put(T, F, k, cap)) return k < cap - 1 || floorl(F * kTwo32) >= 4294967295.0L;
    }
    return false;
}

// Gap g between crossovers (boundaries without one before the next):
// P(g <= k) = 1 - (1-r)^(k+1).
void geometric_table(double r, uint32_t n, std::vector<uint64_t> &T) {
    T.resize(n);
    const long double q = 1.0L - (long double)r;
    for (uint32_t k = 0; k < n; ++k) T[k] = (uint64_t)floorl((1.0L - powl(q, (long double)(k + 1u))) * kTwo32);
}

uint32_t geometric_device_len(const std::vector<uint64_t> &T) {
    uint32_t k = 0;
    while (k < T.size() && T[k] < kAlways) ++k;
    return k;
}

uint32_t recomb_mode(double r) {
    if (r == 0.5) return kModeRaw;
    if (r == 0.0) return kModeZero;
    return r < kSkipBelow ? kModeSkip : kModeLazy;
}

// Gaussian stabilising viability v(z) = exp(-(z - theta)^2 / (2 omega^2))
// for z = zmin .. zmin + n - 1.
void viability_table(double theta, double omega, int32_t zmin, uint32_t n, std::vector<double> &v) {
    v.resize(n);
    for (uint32_t k = 0; k < n; ++k) {
        const double d = (double)(zmin + (int32_t)k) - theta;
        v[k] = std::exp(-(d * d) / (2.0 * omega * omega));
    }
}

// Gaussian phenotype matching of consumer and resource, a exp(-d^2 /
// (2 sigma^2)) at distance d, as capture thresholds.
void capture_table(double a, double sigma, uint32_t n, std::vector<uint64_t> &T) {
    T.resize(n);
    for (uint32_t d = 0; d < n; ++d) {
        const double dd = (double)d;
        T[d] = prob_threshold(a * std::exp(-(dd * dd) / (2.0 * sigma * sigma)));
    }
}

// Mate choice over integer phenotypes (acceptance thresholds).
void choice_table(bool preference, double opt, double w, int32_t zmin, uint32_t n, std::vector<uint64_t> &T) {
    T.resize(n);
    for (uint32_t k = 0; k < n; ++k) {
        const double d = preference ? (double)(zmin + (int32_t)k) - opt : (double)k;
        T[k] = prob_threshold(std::exp(-(d * d) / (2.0 * w * w)));
    }
}

// Linkage map: threshold bit planes per 32-boundary word.
void linkage_planes(const double *r, uint32_t L, std::vector<uint32_t> &M) {
    const uint32_t Wb = (L + 31u) / 32u;
    M.assign((size_t)Wb * kMapWords, 0u);
    for (uint32_t b = 1; b < L; ++b) {
        const uint32_t R = (uint32_t)std::floor(r[b - 1] * 4294967296.0);
        uint32_t *m = M.data() + (size_t)(b / 32u) * kMapWords;
        const uint32_t bit = 1u << (b % 32u);
        if (R != 0) m[64] |= bit;
        for (uint32_t p = 0; p < 32; ++p) {
            const uint32_t i = 31u - p;  // the bit of R that plane p compares
            if ((R >> i) & 1u) m[p] |= bit;
            if (R & ((1u << i) - 1u)) m[32 + p] |= bit;  // a 1 bit below it
        }
    }
}

}  // namespace spegg

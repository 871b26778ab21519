// Sanitizer driver of the library's host code (built with
// -fsanitize=address,undefined by tests/test_sanitizers.py and linked
// against the HIP runtime): descriptor validation and the workspace plan
// (spegg_footprint, spegg_pop_create's checks before any device work), the
// threshold tables and the gap lookup.  No call here reaches a device.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "spegg.h"

static int failures = 0;
#define EXPECT(c)                                                   \
    do {                                                            \
        if (!(c)) {                                                 \
            std::fprintf(stderr, "%s:%d: %s\n", __FILE__, __LINE__, #c); \
            ++failures;                                             \
        }                                                           \
    } while (0)

static spegg_rep_desc rep(uint32_t L, double r, uint32_t n0) {
    spegg_rep_desc d;
    std::memset(&d, 0, sizeof d);
    d.seed = 1;
    d.replicate_id = 3;
    d.regime = SPEGG_WF;
    d.n0 = n0;
    d.capacity = n0;
    d.n_loci = L;
    d.n_patches = 1;
    d.mu = 1e-4;
    d.r = r;
    d.omega = 8.0;
    return d;
}

int main() {
    // footprints of valid populations of every shape
    std::vector<spegg_rep_desc> reps;
    const uint32_t Ls[] = {1, 31, 64, 257, 1024, 4000, 16384};
    const double rs[] = {0.5, 0.0, 0.01, 0.1, 0.3};
    for (uint32_t L : Ls)
        for (double r : rs) reps.push_back(rep(L, r, 100 + L % 50));
    for (size_t i = 0; i < reps.size(); ++i) reps[i].replicate_id = (uint32_t)i;
    EXPECT(spegg_footprint(reps.data(), (uint32_t)reps.size()) > 0);
    std::vector<int8_t> eff(300);
    for (int l = 0; l < 300; ++l) eff[l] = (int8_t)(l % 9 - 4);
    spegg_rep_desc e = rep(300, 0.05, 500);
    e.effects = eff.data();
    EXPECT(spegg_footprint(&e, 1) > 0);
    spegg_rep_desc ring = rep(256, 0.2, 300);
    ring.n_patches = 100;
    ring.migration = 0.01;
    EXPECT(spegg_footprint(&ring, 1) > 0);
    spegg_ecology eco;
    std::memset(&eco, 0, sizeof eco);
    eco.n0_consumer = 1000;
    eco.capacity_consumer = 4000;
    eco.resource_trials = 4;
    eco.attack = 0.5;
    eco.match_width = 4.0;
    eco.encounters = 20.0;
    eco.conversion = 0.5;
    eco.resource_q0 = 0.55;
    eco.resource_K = 2e4;
    for (int a = 0; a < 4; ++a) eco.surv_resource[a] = eco.surv_consumer[a] = 0.5;
    spegg_rep_desc cr = rep(256, 0.1, 8000);
    cr.regime = SPEGG_CONSUMER_RESOURCE;
    cr.capacity = 20000;
    cr.ecology = &eco;
    EXPECT(spegg_footprint(&cr, 1) > 0);
    spegg_rep_desc pois = rep(1024, 0.01, 1000);
    pois.regime = SPEGG_POISSON_BH;
    pois.capacity = 3000;
    pois.K = 1000.0;
    pois.fecundity = 2.2;
    EXPECT(spegg_footprint(&pois, 1) > 0);

    // invalid descriptors: rejected with a message, before any device work
    spegg_rep_desc bad = rep(0, 0.5, 10);
    EXPECT(spegg_footprint(&bad, 1) == 0 && std::strlen(spegg_last_error()) > 0);
    bad = rep(64, 0.7, 10);
    EXPECT(spegg_footprint(&bad, 1) == 0);
    bad = rep(64, 0.5, 10);
    bad.capacity = 5;
    EXPECT(spegg_footprint(&bad, 1) == 0);
    bad = rep(64, 0.5, 10);
    bad.mu = 1.0;
    EXPECT(spegg_footprint(&bad, 1) == 0);
    bad = e;
    eff[7] = 9;
    EXPECT(spegg_footprint(&bad, 1) == 0);
    eff[7] = 0;
    spegg_pop *pop = nullptr;
    EXPECT(spegg_pop_create(&bad, 0, nullptr, 0, nullptr, &pop) == SPEGG_E_INVALID && pop == nullptr);
    spegg_rep_desc ok = rep(64, 0.5, 10);
    EXPECT(spegg_pop_create(&ok, 1, nullptr, 0, nullptr, &pop) == SPEGG_E_NOMEM && pop == nullptr);
    EXPECT(spegg_pop_create(&ok, 1, nullptr, 0, nullptr, nullptr) == SPEGG_E_INVALID);

    // tables and the gap lookup
    std::vector<uint64_t> T(20000);
    EXPECT(spegg_threshold_table(0, 2.2, 0, T.data(), 1024) > 0);
    EXPECT(spegg_threshold_table(0, 900.0, 0, T.data(), 1024) == -1);
    EXPECT(spegg_threshold_table(1, 1e-4, 16384, T.data(), 16385) > 0);
    EXPECT(spegg_threshold_table(2, 0.169, 16383, T.data(), 16383) == 16383);
    uint32_t gap = 0;
    EXPECT(spegg_geometric_gap(0.1, 1024, 0xFFFFFFFFu, 0, &gap) == 427 && gap == 427);
    EXPECT(spegg_geometric_gap(0.1, 1024, 0xFFFFFFFFu, 1023, &gap) == 427 && gap == 427);
    EXPECT(spegg_geometric_gap(0.01, 16384, 0u, 16383, &gap) > 0 && gap == 0);
    EXPECT(spegg_geometric_gap(0.6, 1024, 0u, 0, &gap) == -1);
    EXPECT(spegg_recomb_mode(0.3) == 3);
    if (failures) return 1;
    std::puts("host sanitizer driver ok");
    return 0;
}

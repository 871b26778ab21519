#pragma once

#include <stdint.h>

#include <vector>

#include "spegg_internal.h"

namespace spegg {

// Each returns false if the table would need more than cap entries to
// reach probability one within 2^-32, or if an argument is out of range.
bool poisson_table(double lambda, int cap, std::vector<uint64_t> &T);
bool binomial_table(uint32_t L, double mu, int cap, std::vector<uint64_t> &T);
void geometric_table(double r, uint32_t n, std::vector<uint64_t> &T);
// Entries of a geometric-gap table the offspring kernel holds: those before
// the first threshold of 2^32.  Every word x is below that threshold, so the
// smallest k with x < T_k never lies beyond it, and the entries the kernel
// keeps (as 32-bit words in LDS) are all below 2^32.
uint32_t geometric_device_len(const std::vector<uint64_t> &T);
uint32_t recomb_mode(double r);
// Bernoulli(p) threshold floor(p 2^32); p >= 1: 2^32 (always), p <= 0: 0.
uint64_t prob_threshold(double p);
void viability_table(double theta, double omega, int32_t zmin, uint32_t n, std::vector<double> &v);
// Capture thresholds floor(a exp(-d^2 / (2 sigma^2)) 2^32) for phenotype
// distances d = 0 .. n - 1.
void capture_table(double a, double sigma, uint32_t n, std::vector<uint64_t> &T);
// Mate choice over integer phenotypes: acceptance thresholds floor(a 2^32)
// of a = exp(-d^2 / (2 w^2)); shared preference: d = z - opt for z = zmin +
// k; assortment (opt ignored): d = k, the phenotype distance (k < n).
void choice_table(bool preference, double opt, double w, int32_t zmin, uint32_t n, std::vector<uint64_t> &T);
// Linkage map planes of a gamete of L loci (rates r[b-1] of boundaries
// b = 1..L-1), kMapWords words per 32-boundary word (layout in
// spegg_internal.h).
void linkage_planes(const double *r, uint32_t L, std::vector<uint32_t> &M);

}  // namespace spegg

// Counter-based complex Gaussian samples for the randomized range finders:
// SplitMix64 (Steele, Lea and Flood 2014) at counter i, and the Box-Muller
// transform of two of its outputs.
#pragma once

#include "common.hpp"

namespace hm {

__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Entry e: sqrt(-2 ln(1 - u1)) e^{2 pi i u2} / sqrt(2), u1 and u2 the 53-bit
// fractions of outputs 2e and 2e + 1 (unit variance, CN(0, 1)).
__device__ inline cplx<double> gauss_at(uint64_t seed, uint64_t e) {
    const uint64_t x1 = splitmix64_at(seed, 2 * e);
    const uint64_t x2 = splitmix64_at(seed, 2 * e + 1);
    const double u1 = (double)(x1 >> 11) * 0x1.0p-53;
    const double u2 = (double)(x2 >> 11) * 0x1.0p-53;
    const double g = sqrt(-2.0 * log1p(-u1)) * 0.70710678118654752;
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    return {g * c, g * s};
}

}  // namespace hm

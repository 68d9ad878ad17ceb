// md_philox.hpp -- the thermostat's counter-based normals.
//
// Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw (SC 2011):
// ten rounds, each multiplying words 0 and 2 by the two round multipliers
// into 64-bit products whose halves are mixed with the other words and the
// round key; the key advances by the two Weyl increments between rounds.
// Two blocks with counters (id, step low, step high, 0) and (..., 1) under
// the key (seed low, seed high) give four pairs of 32-bit words; each pair
// forms a 53-bit uniform in (0, 1) and Box-Muller maps two uniforms to two
// standard normals (the fourth normal is unused).  Shared by md_langevin and
// the thermostat inside md_lj_forces_vv, so both draw the same noise.
#ifndef MD_PHILOX_HPP
#define MD_PHILOX_HPP

#include "md_common.hpp"

namespace md {

struct Philox4 {
    uint32_t v[4];
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t kMul0 = 0xD2511F53u, kMul1 = 0xCD9E8D57u;
    constexpr uint32_t kWeyl0 = 0x9E3779B9u, kWeyl1 = 0xBB67AE85u;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t hi0 = __umulhi(kMul0, c0), lo0 = kMul0 * c0;
        const uint32_t hi1 = __umulhi(kMul1, c2), lo1 = kMul1 * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += kWeyl0;
        k1 += kWeyl1;
    }
    return Philox4{{c0, c1, c2, c3}};
}

// (w0 w1 >> 11 + 1/2) 2^-53: a uniform strictly inside (0, 1).
__device__ __forceinline__ double uniform53(uint32_t w0, uint32_t w1)
{
    const uint64_t a = ((static_cast<uint64_t>(w0) << 32) | w1) >> 11;
    return (static_cast<double>(a) + 0.5) * 0x1p-53;
}

// Three standard normals for atom id `me` at noise counter `step`.
__device__ __forceinline__ void thermostat_normals(uint32_t me, uint64_t step, uint32_t seed_lo,
                                                   uint32_t seed_hi, double g[3])
{
    const uint32_t s_lo = static_cast<uint32_t>(step), s_hi = static_cast<uint32_t>(step >> 32);
    const Philox4 b0 = philox4x32_10(me, s_lo, s_hi, 0u, seed_lo, seed_hi);
    const Philox4 b1 = philox4x32_10(me, s_lo, s_hi, 1u, seed_lo, seed_hi);
    constexpr double kTwoPi = 6.283185307179586476925286766559;
    {
        const double r = sqrt(-2.0 * log(uniform53(b0.v[0], b0.v[1])));
        double sn, cs;
        sincos(kTwoPi * uniform53(b0.v[2], b0.v[3]), &sn, &cs);
        g[0] = r * cs;
        g[1] = r * sn;
    }
    {
        const double r = sqrt(-2.0 * log(uniform53(b1.v[0], b1.v[1])));
        g[2] = r * cos(kTwoPi * uniform53(b1.v[2], b1.v[3]));
    }
}

}  // namespace md

#endif  // MD_PHILOX_HPP

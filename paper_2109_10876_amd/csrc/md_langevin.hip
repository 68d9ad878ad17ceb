// md_langevin.hip -- md_langevin: Langevin thermostat in force form.
//
// Sec. 4 of the paper equilibrates both systems to a target temperature
// with a Langevin thermostat.  In force form each atom receives friction and
// a random kick, F += -gamma m v + sqrt(2 gamma m T / dt) xi, evaluated with
// the velocity at the time of the force evaluation.  The normals xi come
// from a counter-based generator so that they depend only on (seed, step,
// atom id): Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw
// (SC 2011) -- ten rounds, each multiplying words 0 and 2 by the two round
// multipliers into 64-bit products whose halves are mixed with the other
// words and the round key; the key advances by the two Weyl increments
// between rounds -- then Box-Muller on 53-bit uniforms.
#include "md_common.hpp"

namespace md {
namespace {

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

struct LangevinArgs {
    const int32_t *atom_off, *unit_rep, *unit_off;
    const double *vx, *vy, *vz;
    double *fx, *fy, *fz;
    const int32_t *type, *id;
    const double *mass;
    int32_t ntypes;
    double gamma, kT_dt2;   // 2 T / dt
    uint32_t seed_lo, seed_hi;
    const uint64_t *step;
};

__global__ __launch_bounds__(kUnit) void k_langevin(LangevinArgs a)
{
    const Unit w = unit_of(blockIdx.x, a.unit_rep, a.unit_off, a.atom_off);
    const int i = w.begin + threadIdx.x;
    if (i >= w.end) return;
    const uint64_t step = *a.step;
    const uint32_t s_lo = static_cast<uint32_t>(step), s_hi = static_cast<uint32_t>(step >> 32);
    const uint32_t me = static_cast<uint32_t>(a.id[i]);
    const Philox4 b0 = philox4x32_10(me, s_lo, s_hi, 0u, a.seed_lo, a.seed_hi);
    const Philox4 b1 = philox4x32_10(me, s_lo, s_hi, 1u, a.seed_lo, a.seed_hi);
    constexpr double kTwoPi = 6.283185307179586476925286766559;
    double g[3];
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
    const double m = a.mass[a.ntypes > 1 ? a.type[i] : 0];
    const double amp = sqrt(a.gamma * m * a.kT_dt2);
    const double gm = a.gamma * m;
    a.fx[i] += -gm * a.vx[i] + amp * g[0];
    a.fy[i] += -gm * a.vy[i] + amp * g[1];
    a.fz[i] += -gm * a.vz[i] + amp * g[2];
}

__global__ void k_step_advance(uint64_t *step) { *step += 1u; }

}  // namespace
}  // namespace md

extern "C" int md_langevin(const md_batch *b, const md_atoms *atoms, const double *mass,
                           int32_t ntypes, double gamma, double temperature, double dt,
                           uint64_t seed, uint64_t *step, uint32_t *status, void *stream)
{
    using namespace md;
    (void)status;
    int e = check_batch(b);
    if (e != MD_OK) return e;
    if (!atoms || !atoms->vx || !atoms->vy || !atoms->vz || !atoms->fx || !atoms->fy ||
        !atoms->fz || !atoms->id || !mass || !step)
        return MD_EINVAL;
    if (ntypes < 1 || ntypes > MD_MAX_TYPES || (ntypes > 1 && !atoms->type)) return MD_EINVAL;
    if (!(gamma >= 0.0) || !(temperature >= 0.0) || !(dt > 0.0)) return MD_EINVAL;
    LangevinArgs a{b->atom_off, b->unit_rep, b->unit_off, atoms->vx, atoms->vy, atoms->vz,
                   atoms->fx, atoms->fy, atoms->fz, atoms->type, atoms->id, mass, ntypes,
                   gamma, 2.0 * temperature / dt, static_cast<uint32_t>(seed),
                   static_cast<uint32_t>(seed >> 32), step};
    hipStream_t s = as_stream(stream);
    hipLaunchKernelGGL(k_langevin, dim3(b->n_units), dim3(kUnit), 0, s, a);
    hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(1), 0, s, step);
    return launch_status();
}

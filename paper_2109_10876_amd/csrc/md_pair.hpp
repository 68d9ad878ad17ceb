// md_pair.hpp -- Lennard-Jones pair arithmetic shared by the force kernels.
//
// Eq. lj of the paper: U(r) = 4 eps [(sig/r)^12 - (sig/r)^6] for r < r_cut.
// With s6 = (sig^2/r^2)^3:  fr = -U'(r)/r = 24 eps s6 (2 s6 - 1) / r^2 and
// U = 4 eps s6 (s6 - 1) (minus U(rc) when the energy is shifted); the force
// on i from j is fr d with d = x_i - x_j.
#pragma once

#include "md_common.hpp"

namespace md {

// Per type pair constants: 24 eps, 4 eps, sig^2, energy shift U(rc).
struct PairConst {
    double e24, e4, s2, ush;
};

__device__ __forceinline__ PairConst pair_const(double eps, double sig, double rc, int shift)
{
    PairConst p;
    p.e24 = 24.0 * eps;
    p.e4 = 4.0 * eps;
    p.s2 = sig * sig;
    double sc2 = p.s2 / (rc * rc);
    double sc6 = sc2 * sc2 * sc2;
    p.ush = shift ? 4.0 * eps * (sc6 * sc6 - sc6) : 0.0;
    return p;
}

// Per-atom accumulators.  FP64 path: ed, wd; mixed path: ef, wf (single).
struct Acc {
    double fx, fy, fz, ed, wd;
    float ef, wf;
};

// Cutoff test (always in double) and pair terms of one displacement; adds
// the force, energy and virial to the per-atom accumulators and returns the
// force factor fr (0 outside the cutoff).
//   MD_FP64: every step in double, reciprocal refined by Newton steps.
//   MD_FP32_MIXED: reciprocal and LJ polynomial in single precision, force
//   accumulated in double, per-atom energy/virial sums in single.
template <int PREC>
__device__ __forceinline__ double lj_pair_accumulate(const PairConst &pc, double dx, double dy,
                                                     double dz, double rc2, Acc &c)
{
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (!(r2 < rc2)) return 0.0;
    double fr;
    if (PREC == MD_FP64) {
        const double inv = rcp_f64(r2);
        const double s2 = pc.s2 * inv;
        const double s6 = s2 * s2 * s2;
        fr = pc.e24 * s6 * (2.0 * s6 - 1.0) * inv;
        c.ed += pc.e4 * s6 * (s6 - 1.0) - pc.ush;
        c.wd += fr * r2;
    } else {
        const float r2f = static_cast<float>(r2);
        const float inv = __builtin_amdgcn_rcpf(r2f);
        const float s2 = static_cast<float>(pc.s2) * inv;
        const float s6 = s2 * s2 * s2;
        const float frf = static_cast<float>(pc.e24) * s6 * (2.0f * s6 - 1.0f) * inv;
        fr = static_cast<double>(frf);
        c.ef += static_cast<float>(pc.e4) * s6 * (s6 - 1.0f) - static_cast<float>(pc.ush);
        c.wf += frf * r2f;
    }
    c.fx = fma(fr, dx, c.fx);
    c.fy = fma(fr, dy, c.fy);
    c.fz = fma(fr, dz, c.fz);
    return fr;
}

// Same terms as lj_pair_accumulate, evaluated for every entry and masked
// with a select instead of a branch (for loops where most entries of a
// wavefront fall inside the cutoff anyway).  A masked entry adds exact
// zeros; its arithmetic may overflow (r2 = 0) but is never selected.
template <int PREC>
__device__ __forceinline__ void lj_pair_accumulate_masked(const PairConst &pc, double dx,
                                                          double dy, double dz, double rc2,
                                                          Acc &c)
{
    const double r2 = dx * dx + dy * dy + dz * dz;
    const bool in = r2 < rc2;
    double fr;
    if (PREC == MD_FP64) {
        const double inv = rcp_f64(r2);
        const double s2 = pc.s2 * inv;
        const double s6 = s2 * s2 * s2;
        fr = in ? pc.e24 * s6 * (2.0 * s6 - 1.0) * inv : 0.0;
        c.ed += in ? pc.e4 * s6 * (s6 - 1.0) - pc.ush : 0.0;
        c.wd += fr * r2;
    } else {
        const float r2f = static_cast<float>(r2);
        const float inv = __builtin_amdgcn_rcpf(r2f);
        const float s2 = static_cast<float>(pc.s2) * inv;
        const float s6 = s2 * s2 * s2;
        const float frf = in ? static_cast<float>(pc.e24) * s6 * (2.0f * s6 - 1.0f) * inv : 0.0f;
        fr = static_cast<double>(frf);
        c.ef += in ? static_cast<float>(pc.e4) * s6 * (s6 - 1.0f) - static_cast<float>(pc.ush)
                   : 0.0f;
        c.wf += frf * r2f;
    }
    c.fx = fma(fr, dx, c.fx);
    c.fy = fma(fr, dy, c.fy);
    c.fz = fma(fr, dz, c.fz);
}

}  // namespace md

// md_pair.hpp -- Lennard-Jones pair arithmetic shared by the force kernels.
//
// Eq. lj of the paper: U(r) = 4 eps [(sig/r)^12 - (sig/r)^6] for r < r_cut.
// With s6 = (sig^2/r^2)^3:  fr = -U'(r)/r = 24 eps s6 (2 s6 - 1) / r^2 and
// U = 4 eps s6 (s6 - 1) (minus U(rc) when the energy is shifted); the force
// on i from j is fr d with d = x_i - x_j.
#pragma once

#include <type_traits>

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
    uint32_t n;   // pairs inside the cutoff (lj_pair_sums)
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
    const double r2 = norm2(dx, dy, dz);
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

// Constants of the LJ terms written in powers of q = 1/r^2: with
// q3 = q^3, the virial term w = fr r^2 = q3 (A q3 - B) and the energy
// U = q3 (C q3 - D) - U(rc), where A = 48 eps sig^12, B = 24 eps sig^6,
// C = 4 eps sig^12, D = 4 eps sig^6 (the same Eq. lj terms as PairConst).
struct PolyConst {
    double A, B, C, D, ush;
    float Af, Bf, Cf, Df, ushf;
};

__device__ __forceinline__ PolyConst poly_const(double eps, double sig, double rc, int shift)
{
    PolyConst p;
    const double s6 = sig * sig * sig * sig * sig * sig;
    p.A = 48.0 * eps * s6 * s6;
    p.B = 24.0 * eps * s6;
    p.C = 4.0 * eps * s6 * s6;
    p.D = 4.0 * eps * s6;
    const double q = 1.0 / (rc * rc), q3 = q * q * q;
    p.ush = shift ? q3 * (p.C * q3 - p.D) : 0.0;
    p.Af = static_cast<float>(p.A);
    p.Bf = static_cast<float>(p.B);
    p.Cf = static_cast<float>(p.C);
    p.Df = static_cast<float>(p.D);
    p.ushf = static_cast<float>(p.ush);
    return p;
}

// Pair terms of one displacement inside the cutoff (the test is in double);
// entries beyond it (up to rc + skin, or the far pad slot) add nothing.  In a
// wavefront almost every entry has some lane inside the cutoff, so this is
// one exec-masked pass over the pair arithmetic per entry.  Written as a
// branch around every accumulation rather than as selects of the results:
// the compiler then needs no zeros for the lanes outside (10-12% fewer
// vector instructions per entry) and the sums are the same bit for bit.
template <int PREC>
__device__ __forceinline__ void lj_pair_masked(const PolyConst &pc, double dx, double dy,
                                               double dz, double rc2, Acc &c)
{
    const double r2 = norm2(dx, dy, dz);
    if (!(r2 < rc2)) return;
    double fr;
    if (PREC == MD_FP64) {
        const double q = rcp_f64(r2);
        const double q3 = q * q * q;
        const double w = q3 * fma(pc.A, q3, -pc.B);
        fr = w * q;
        c.ed += q3 * (pc.C * q3 - pc.D) - pc.ush;
        c.wd = fma(fr, r2, c.wd);
    } else {
        const float r2f = static_cast<float>(r2);
        const float q = __builtin_amdgcn_rcpf(r2f);
        const float q3 = q * q * q;
        const float w = q3 * fmaf(pc.Af, q3, -pc.Bf);
        const float frf = w * q;
        c.ef += fmaf(q3, fmaf(pc.Cf, q3, -pc.Df), -pc.ushf);
        c.wf = fmaf(frf, r2f, c.wf);
        fr = static_cast<double>(frf);
    }
    c.fx = fma(fr, dx, c.fx);
    c.fy = fma(fr, dy, c.fy);
    c.fz = fma(fr, dz, c.fz);
}

// One atom type, energy and virial as sums: with w = q3 (A q3 - B) the
// virial term fr r^2, and A = 12 C, B = 6 D, a pair's energy is
// U = w / 12 - (D / 2) q3 - U(rc).  Each atom therefore sums w (its virial),
// q3 and its count of pairs inside the cutoff, from which its energy follows
// once (pair_sums_energy): three accumulations per pair instead of the four
// of the polynomial form.  Acc holds sum w in wd / wf, sum q3 in ed / ef and
// the count in n.
template <int PREC>
__device__ __forceinline__ void lj_pair_sums(const PolyConst &pc, double dx, double dy,
                                             double dz, double rc2, Acc &c)
{
    const double r2 = norm2(dx, dy, dz);
    if (!(r2 < rc2)) return;
    double fr;
    if (PREC == MD_FP64) {
        const double q = rcp_f64(r2);
        const double q3 = q * q * q;
        const double w = q3 * fma(pc.A, q3, -pc.B);
        fr = w * q;
        c.wd += w;
        c.ed += q3;
    } else {
        const float q = __builtin_amdgcn_rcpf(static_cast<float>(r2));
        const float q3 = q * q * q;
        const float w = q3 * fmaf(pc.Af, q3, -pc.Bf);
        const float frf = w * q;
        c.wf += w;
        c.ef += q3;
        fr = static_cast<double>(frf);
    }
    c.n += 1u;
    c.fx = fma(fr, dx, c.fx);
    c.fy = fma(fr, dy, c.fy);
    c.fz = fma(fr, dz, c.fz);
}

// The force of lj_pair_sums alone, for calls that want no energy or virial:
// the same expressions for q, q3, w and fr, so the two give the same force
// bit for bit, without the three sums per pair.
template <int PREC>
__device__ __forceinline__ void lj_pair_force(const PolyConst &pc, double dx, double dy,
                                              double dz, double rc2, Acc &c)
{
    const double r2 = norm2(dx, dy, dz);
    if (!(r2 < rc2)) return;
    double fr;
    if (PREC == MD_FP64) {
        const double q = rcp_f64(r2);
        const double q3 = q * q * q;
        const double w = q3 * fma(pc.A, q3, -pc.B);
        fr = w * q;
    } else {
        const float q = __builtin_amdgcn_rcpf(static_cast<float>(r2));
        const float q3 = q * q * q;
        const float w = q3 * fmaf(pc.Af, q3, -pc.Bf);
        fr = static_cast<double>(w * q);
    }
    c.fx = fma(fr, dx, c.fx);
    c.fy = fma(fr, dy, c.fy);
    c.fz = fma(fr, dz, c.fz);
}

// The atom's energy from the sums of lj_pair_sums (sum w, sum q3, count).
__device__ __forceinline__ double pair_sums_energy(const PolyConst &pc, double sw, double sq3,
                                                   uint32_t n)
{
    return sw * (1.0 / 12.0) - 0.5 * pc.D * sq3 - pc.ush * double(n);
}

// The same pair terms from the force constants of one type pair alone:
// with A = 48 eps s12 and B = 24 eps s6 the energy constants are C = A/12
// and D = B/6, so U = q3 (A q3 - 2B) / 12 - ush.  Three constants per type
// pair fit in registers, so a two-type list selects them per entry instead
// of reading a table.
template <int PREC>
struct PairAB {
    using T = std::conditional_t<PREC == MD_FP64, double, float>;
    T A, B, ush;
};

template <int PREC>
__device__ __forceinline__ PairAB<PREC> pair_ab(const PolyConst &p)
{
    if constexpr (PREC == MD_FP64) return PairAB<PREC>{p.A, p.B, p.ush};
    else return PairAB<PREC>{p.Af, p.Bf, p.ushf};
}

template <int PREC>
__device__ __forceinline__ PairAB<PREC> select_ab(bool second, const PairAB<PREC> &k0,
                                                  const PairAB<PREC> &k1)
{
    return PairAB<PREC>{second ? k1.A : k0.A, second ? k1.B : k0.B, second ? k1.ush : k0.ush};
}

template <int PREC>
__device__ __forceinline__ void lj_pair_ab(const PairAB<PREC> &k, double dx, double dy,
                                           double dz, double rc2, Acc &c)
{
    const double r2 = norm2(dx, dy, dz);
    // selects here, not the branch of lj_pair_masked: with per-lane constants
    // the branch form made the two-type kernel 5% slower
    const bool in = r2 < rc2;
    double fr;
    if constexpr (PREC == MD_FP64) {
        const double q = rcp_f64(r2);
        const double q3 = q * q * q;
        const double t = k.A * q3;
        fr = in ? q3 * (t - k.B) * q : 0.0;
        c.ed += in ? (q3 * (1.0 / 12.0)) * (t - 2.0 * k.B) - k.ush : 0.0;
        c.wd = fma(fr, r2, c.wd);
    } else {
        const float r2f = static_cast<float>(r2);
        const float q = __builtin_amdgcn_rcpf(r2f);
        const float q3 = q * q * q;
        const float t = k.A * q3;
        const float frf = in ? q3 * (t - k.B) * q : 0.0f;
        c.ef += in ? (q3 * (1.0f / 12.0f)) * (t - 2.0f * k.B) - k.ush : 0.0f;
        c.wf = fmaf(frf, r2f, c.wf);
        fr = static_cast<double>(frf);
    }
    c.fx = fma(fr, dx, c.fx);
    c.fy = fma(fr, dy, c.fy);
    c.fz = fma(fr, dz, c.fz);
}

// Adjoint pair terms (derivatives of Eq. lj), per unit eps or eps/sigma:
// with s2 = sig^2/r^2, s6 = s2^3, s12 = s6^2 and inv = 1/r^2,
//   fr1 = 24 s6 (2 s6 - 1) inv          (fr = eps fr1, F_i = fr d)
//   dfr1 = (-672 s12 + 192 s6) inv^2    (fr'/r = eps dfr1)
//   u1 = 4 (s12 - s6) - shift part      (U = eps u1)
//   dfs1 = (576 s12 - 144 s6) inv       (dfr/dsig = (eps/sig) dfs1)
//   dus1 = 48 s12 - 24 s6 - shift part  (dU/dsig = (eps/sig) dus1)
struct VjpConst {
    double eps, eos, s2, ush1, dus1;   // eps, eps/sig, sig^2, shift parts at rc
    float epsf, eosf, s2f, ush1f, dus1f;   // the same rounded to FP32
};

__device__ __forceinline__ VjpConst vjp_const(double eps, double sig, double rc, int shift)
{
    VjpConst c;
    c.eps = eps;
    c.eos = eps / sig;
    c.s2 = sig * sig;
    const double c2 = c.s2 / (rc * rc), c6 = c2 * c2 * c2, c12 = c6 * c6;
    c.ush1 = shift ? 4.0 * (c12 - c6) : 0.0;
    c.dus1 = shift ? (48.0 * c12 - 24.0 * c6) : 0.0;
    c.epsf = static_cast<float>(c.eps);
    c.eosf = static_cast<float>(c.eos);
    c.s2f = static_cast<float>(c.s2);
    c.ush1f = static_cast<float>(c.ush1);
    c.dus1f = static_cast<float>(c.dus1);
    return c;
}

struct VjpTerms {
    double fr1, dfr1, u1, dfs1, dus1;
};

template <int PREC>
__device__ __forceinline__ VjpTerms vjp_terms(const VjpConst &c, double r2)
{
    VjpTerms v;
    if (PREC == MD_FP64) {
        const double inv = rcp_f64(r2);
        const double s2 = c.s2 * inv, s6 = s2 * s2 * s2, s12 = s6 * s6;
        v.fr1 = 24.0 * s6 * (2.0 * s6 - 1.0) * inv;
        v.dfr1 = (-672.0 * s12 + 192.0 * s6) * inv * inv;
        v.u1 = 4.0 * (s12 - s6) - c.ush1;
        v.dfs1 = (576.0 * s12 - 144.0 * s6) * inv;
        v.dus1 = (48.0 * s12 - 24.0 * s6) - c.dus1;
    } else {
        const float invf = __builtin_amdgcn_rcpf(static_cast<float>(r2));
        const float s2 = static_cast<float>(c.s2) * invf, s6 = s2 * s2 * s2, s12 = s6 * s6;
        v.fr1 = static_cast<double>(24.0f * s6 * (2.0f * s6 - 1.0f) * invf);
        v.dfr1 = static_cast<double>((-672.0f * s12 + 192.0f * s6) * invf * invf);
        v.u1 = static_cast<double>(4.0f * (s12 - s6)) - c.ush1;
        v.dfs1 = static_cast<double>((576.0f * s12 - 144.0f * s6) * invf);
        v.dus1 = static_cast<double>(48.0f * s12 - 24.0f * s6) - c.dus1;
    }
    return v;
}

// The adjoint pair terms in FP32 throughout (FP32-mixed tile adjoint).
struct VjpTermsF {
    float fr1, dfr1, u1, dfs1, dus1;
};

__device__ __forceinline__ VjpTermsF vjp_terms_f32(const VjpConst &c, float r2)
{
    VjpTermsF v;
    const float inv = __builtin_amdgcn_rcpf(r2);
    const float s2 = c.s2f * inv, s6 = s2 * s2 * s2, s12 = s6 * s6;
    v.fr1 = 24.0f * s6 * (2.0f * s6 - 1.0f) * inv;
    v.dfr1 = (-672.0f * s12 + 192.0f * s6) * inv * inv;
    v.u1 = 4.0f * (s12 - s6) - c.ush1f;
    v.dfs1 = (576.0f * s12 - 144.0f * s6) * inv;
    v.dus1 = (48.0f * s12 - 24.0f * s6) - c.dus1f;
    return v;
}

}  // namespace md

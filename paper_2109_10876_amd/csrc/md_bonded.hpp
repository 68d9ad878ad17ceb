// md_bonded.hpp -- per-atom sums of the polymer melts' bonded terms.
//
// FENE bonds (U = -(1/2) K R0^2 ln(1 - r^2/R0^2), force on i from partner j
// fr d with fr = -K / (1 - r^2/R0^2), d = x_i - x_j) and the ring melt's
// cosine angle term (U = K (1 + cos t) for the triple a-b-c, b in the middle,
// d1 = x_a - x_b, d2 = x_c - x_b; F_a = -K (d2/(r1 r2) - cos t d1/r1^2),
// F_c likewise, F_b = -F_a - F_c), both from Sec. 4 of the paper, summed for
// one atom over its own table column so that no two threads write one atom.
// Used by md_fene_forces, md_angle_forces and md_bonded_forces.
#ifndef MD_BONDED_HPP
#define MD_BONDED_HPP

#include "md_common.hpp"

namespace md {

// Minimum image of a bond vector.  d/L through the reciprocal rounds to the
// same image as the division except within rounding of |d| = L/2, where the
// image is ambiguous anyway.
struct BondBox {
    double Lx, Ly, Lz, ix, iy, iz;
    __device__ __forceinline__ void wrap(double &dx, double &dy, double &dz) const
    {
        dx -= Lx * rint(dx * ix);
        dy -= Ly * rint(dy * iy);
        dz -= Lz * rint(dz * iz);
    }
};

__device__ __forceinline__ BondBox bond_box(const double *box, int rep)
{
    const double Lx = box[3 * rep], Ly = box[3 * rep + 1], Lz = box[3 * rep + 2];
    return BondBox{Lx, Ly, Lz, 1.0 / Lx, 1.0 / Ly, 1.0 / Lz};
}

struct BondedSum {
    double fx, fy, fz, e, w;
};

// FENE bonds of the atom at index i, table column me; partners are ids
// (found through where) or indices.  Each bond is seen from both atoms, so
// energy and virial are halved.  Returns false if a bond is broken (r >= R0;
// it contributes nothing).
template <int ORDER>
__device__ __forceinline__ bool fene_atom(int i, int me, const double *x, const double *y,
                                          const double *z, const int32_t *where,
                                          const int32_t *count, const int32_t *partner,
                                          int max_bonds, int N, double K, double R02,
                                          const BondBox &bx, BondedSum &s)
{
    const double xi = x[i], yi = y[i], zi = z[i];
    const int nb = min(count[me], max_bonds);
    bool ok = true;
    for (int k = 0; k < nb; ++k) {
        const int p = partner[size_t(k) * N + me];
        const int j = ORDER == MD_BY_ID ? where[p] : p;
        double dx = xi - x[j], dy = yi - y[j], dz = zi - z[j];
        bx.wrap(dx, dy, dz);
        const double r2 = norm2(dx, dy, dz);
        const double q = 1.0 - r2 / R02;
        if (!(q > 0.0)) {
            ok = false;
            continue;
        }
        const double fr = -K / q;
        s.fx = fma(fr, dx, s.fx);
        s.fy = fma(fr, dy, s.fy);
        s.fz = fma(fr, dz, s.fz);
        s.e += -0.25 * K * R02 * log(q);
        s.w += 0.5 * fr * r2;
    }
    return ok;
}

// Angle triples of table column me (the atom itself is one of the three
// members, compared in the table's own terms: ids or indices).  The middle
// bead adds the triple's energy and virial (d1.F_a + d2.F_c), so each triple
// counts once.  Returns false if a bond vector of a triple has zero length
// (the triple contributes nothing).
template <int ORDER>
__device__ __forceinline__ bool angle_atom(int me, const double *x, const double *y,
                                           const double *z, const int32_t *where,
                                           const int32_t *count, const int32_t *tri,
                                           int max_angles, int N, double K, const BondBox &bx,
                                           BondedSum &s)
{
    const int nt = min(count[me], max_angles);
    bool ok = true;
    for (int k = 0; k < nt; ++k) {
        const size_t row = size_t(3 * k) * N + me;
        const int ia = tri[row], ib = tri[row + N], ic = tri[row + 2 * size_t(N)];
        const int pa = ORDER == MD_BY_ID ? where[ia] : ia;
        const int pb = ORDER == MD_BY_ID ? where[ib] : ib;
        const int pc = ORDER == MD_BY_ID ? where[ic] : ic;
        double d1x = x[pa] - x[pb], d1y = y[pa] - y[pb], d1z = z[pa] - z[pb];
        double d2x = x[pc] - x[pb], d2y = y[pc] - y[pb], d2z = z[pc] - z[pb];
        bx.wrap(d1x, d1y, d1z);
        bx.wrap(d2x, d2y, d2z);
        const double r11 = d1x * d1x + d1y * d1y + d1z * d1z;
        const double r22 = d2x * d2x + d2y * d2y + d2z * d2z;
        if (!(r11 > 0.0) || !(r22 > 0.0)) {
            ok = false;
            continue;
        }
        const double inv12 = 1.0 / sqrt(r11 * r22);
        const double c = (d1x * d2x + d1y * d2y + d1z * d2z) * inv12;
        // F_a = -K (d2 inv12 - c d1 / r11), F_c = -K (d1 inv12 - c d2 / r22)
        const double qa = c / r11, qc = c / r22;
        const double fax = -K * (d2x * inv12 - qa * d1x);
        const double fay = -K * (d2y * inv12 - qa * d1y);
        const double faz = -K * (d2z * inv12 - qa * d1z);
        const double fcx = -K * (d1x * inv12 - qc * d2x);
        const double fcy = -K * (d1y * inv12 - qc * d2y);
        const double fcz = -K * (d1z * inv12 - qc * d2z);
        if (me == ia) {
            s.fx += fax;
            s.fy += fay;
            s.fz += faz;
        } else if (me == ic) {
            s.fx += fcx;
            s.fy += fcy;
            s.fz += fcz;
        } else {
            s.fx -= fax + fcx;
            s.fy -= fay + fcy;
            s.fz -= faz + fcz;
            s.e += K * (1.0 + c);
            s.w += d1x * fax + d1y * fay + d1z * faz + d2x * fcx + d2y * fcy + d2z * fcz;
        }
    }
    return ok;
}

}  // namespace md

#endif  // MD_BONDED_HPP

// md_angle.hip -- md_angle_forces: the cosine angle term of the ring melt.
//
// The paper's ring-polymer melt (Sec. 4, setup) adds a cosine potential on
// the triples (a, b, c) of consecutive beads, b in the middle.  With
// d1 = x_a - x_b, d2 = x_c - x_b (minimum image), r1 = |d1|, r2 = |d2| and
// cos t = d1.d2 / (r1 r2), the term is U = K (1 + cos t) (zero for a straight
// triple) and its forces, -grad U, are
//     F_a = -K (d2 / (r1 r2) - cos t d1 / r1^2),
//     F_c = -K (d1 / (r1 r2) - cos t d2 / r2^2),   F_b = -F_a - F_c.
// One thread per atom walks the triples that atom belongs to and keeps the
// force on its own bead only, so no two threads write one atom:
// deterministic, no atomics.  The middle bead's thread adds the triple's
// energy and virial (d1.F_a + d2.F_c), so each triple is counted once.
// A table keyed by index (md_bonded_reindex) is walked in the atoms' current
// (cell-sorted) order: table reads and force writes are coalesced and the
// partners sit in nearby cells.  A table keyed by id is walked in id order:
// its reads are then coalesced, and the beads of a chain (consecutive ids)
// still sit in nearby cells.
#include <cmath>

#include "md_common.hpp"

namespace md {
namespace {

struct AngleArgs {
    const int32_t *atom_off, *unit_rep, *unit_off;
    const double *box;
    const double *x, *y, *z;
    const int32_t *where;
    const int32_t *acount, *tri;
    int32_t N, max_angles;
    double K;
    double *fx, *fy, *fz;
    double *partial;
    uint32_t *status;
};

template <int ORDER>
__global__ __launch_bounds__(kUnit) void k_angle(AngleArgs a)
{
    __shared__ double red[kWavesPerUnit];
    const int u = blockIdx.x;
    const Unit w = unit_of(u, a.unit_rep, a.unit_off, a.atom_off);
    // column of the table: an atom id (ids of a replica span its range) or
    // the current index
    const int me = w.begin + threadIdx.x;
    double e = 0.0, vir = 0.0;
    if (me < w.end) {
        const double Lx = a.box[3 * w.rep], Ly = a.box[3 * w.rep + 1], Lz = a.box[3 * w.rep + 2];
        // d/L through the reciprocal rounds to the same image as the
        // division except within rounding of |d| = L/2, where the image is
        // ambiguous anyway
        const double ix = 1.0 / Lx, iy = 1.0 / Ly, iz = 1.0 / Lz;
        const int i = ORDER == MD_BY_ID ? a.where[me] : me;
        const int nt = min(a.acount[me], a.max_angles);
        double fx = 0.0, fy = 0.0, fz = 0.0;
        bool bad = false;
        for (int k = 0; k < nt; ++k) {
            const size_t row = size_t(3 * k) * a.N + me;
            const int ia = a.tri[row], ib = a.tri[row + a.N], ic = a.tri[row + 2 * size_t(a.N)];
            const int pa = ORDER == MD_BY_ID ? a.where[ia] : ia;
            const int pb = ORDER == MD_BY_ID ? a.where[ib] : ib;
            const int pc = ORDER == MD_BY_ID ? a.where[ic] : ic;
            double d1x = a.x[pa] - a.x[pb], d1y = a.y[pa] - a.y[pb], d1z = a.z[pa] - a.z[pb];
            double d2x = a.x[pc] - a.x[pb], d2y = a.y[pc] - a.y[pb], d2z = a.z[pc] - a.z[pb];
            d1x -= Lx * rint(d1x * ix);
            d1y -= Ly * rint(d1y * iy);
            d1z -= Lz * rint(d1z * iz);
            d2x -= Lx * rint(d2x * ix);
            d2y -= Ly * rint(d2y * iy);
            d2z -= Lz * rint(d2z * iz);
            const double r11 = d1x * d1x + d1y * d1y + d1z * d1z;
            const double r22 = d2x * d2x + d2y * d2y + d2z * d2z;
            if (!(r11 > 0.0) || !(r22 > 0.0)) {
                bad = true;
                continue;
            }
            const double inv12 = 1.0 / sqrt(r11 * r22);
            const double c = (d1x * d2x + d1y * d2y + d1z * d2z) * inv12;
            // F_a = -K (d2 inv12 - c d1 / r11), F_c = -K (d1 inv12 - c d2 / r22)
            const double qa = c / r11, qc = c / r22;
            const double fax = -a.K * (d2x * inv12 - qa * d1x);
            const double fay = -a.K * (d2y * inv12 - qa * d1y);
            const double faz = -a.K * (d2z * inv12 - qa * d1z);
            const double fcx = -a.K * (d1x * inv12 - qc * d2x);
            const double fcy = -a.K * (d1y * inv12 - qc * d2y);
            const double fcz = -a.K * (d1z * inv12 - qc * d2z);
            if (me == ia) {
                fx += fax;
                fy += fay;
                fz += faz;
            } else if (me == ic) {
                fx += fcx;
                fy += fcy;
                fz += fcz;
            } else {
                fx -= fax + fcx;
                fy -= fay + fcy;
                fz -= faz + fcz;
                e += a.K * (1.0 + c);
                vir += d1x * fax + d1y * fay + d1z * faz + d2x * fcx + d2y * fcy + d2z * fcz;
            }
        }
        a.fx[i] += fx;
        a.fy[i] += fy;
        a.fz[i] += fz;
        if (bad && a.status) atomicOr(a.status, MD_F_NONFINITE);
    }
    const double es = block_sum(e, red);
    const double ws = block_sum(vir, red);
    if (threadIdx.x == 0) {
        a.partial[size_t(u) * kPartials + 0] = es;
        a.partial[size_t(u) * kPartials + 1] = ws;
    }
}

}  // namespace
}  // namespace md

extern "C" int md_angle_forces(const md_batch *b, const md_atoms *atoms, const md_angles *angles,
                               double K, double *energy, double *virial, void *ws,
                               size_t ws_bytes, uint32_t *status, void *stream)
{
    using namespace md;
    int e = check_batch(b);
    if (e != MD_OK) return e;
    if (!atoms || !atoms->x || !atoms->y || !atoms->z || !atoms->fx || !atoms->fy ||
        !atoms->fz || !angles || !angles->count || !angles->tri || !ws)
        return MD_EINVAL;
    if (angles->order != MD_BY_ID && angles->order != MD_BY_INDEX) return MD_EINVAL;
    if (angles->order == MD_BY_ID && !atoms->where) return MD_EINVAL;
    if (angles->max_angles < 1 || angles->max_angles > MD_MAX_ANGLES) return MD_EINVAL;
    if (!(K >= 0.0) || !std::isfinite(K)) return MD_EINVAL;
    const WsLayout l = ws_layout(b);
    if (ws_bytes < l.total) return MD_ENOWS;
    double *partial = ws_at<double>(ws, l.partial);
    AngleArgs a{b->atom_off, b->unit_rep, b->unit_off, b->box, atoms->x, atoms->y, atoms->z,
                atoms->where, angles->count, angles->tri, b->N,
                angles->max_angles, K, atoms->fx, atoms->fy, atoms->fz, partial, status};
    hipStream_t s = as_stream(stream);
    if (angles->order == MD_BY_ID)
        hipLaunchKernelGGL(k_angle<MD_BY_ID>, dim3(b->n_units), dim3(kUnit), 0, s, a);
    else
        hipLaunchKernelGGL(k_angle<MD_BY_INDEX>, dim3(b->n_units), dim3(kUnit), 0, s, a);
    if (energy || virial) launch_finalize_sum2(b->R, b->unit_off, partial, 0, energy, virial, s);
    return launch_status();
}

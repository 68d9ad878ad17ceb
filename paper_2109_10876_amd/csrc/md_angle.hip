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

#include "md_bonded.hpp"

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
    BondedSum sum{0.0, 0.0, 0.0, 0.0, 0.0};
    if (me < w.end) {
        const int i = ORDER == MD_BY_ID ? a.where[me] : me;
        const bool ok = angle_atom<ORDER>(me, a.x, a.y, a.z, a.where, a.acount, a.tri,
                                          a.max_angles, a.N, a.K, bond_box(a.box, w.rep), sum);
        a.fx[i] += sum.fx;
        a.fy[i] += sum.fy;
        a.fz[i] += sum.fz;
        if (!ok && a.status) atomicOr(a.status, MD_F_NONFINITE);
    }
    const double e = sum.e, vir = sum.w;
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

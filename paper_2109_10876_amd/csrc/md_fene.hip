// md_fene.hip -- md_fene_forces: FENE bonds of the bead-spring polymer melt.
//
// The paper's polymer melt (Sec. 4) bonds consecutive monomers with the FENE
// potential U = -(1/2) K R0^2 ln(1 - r^2/R0^2); the force on i from its
// partner j is fr d with fr = -K / (1 - r^2/R0^2), d = x_i - x_j (minimum
// image).  One thread per atom walks its own bond row; each bond is seen
// from both of its atoms, so energy and virial are halved.  No atomics.
// Threads run in the atoms' current (cell-sorted) order.  A table keyed by
// id is reached through id[i] and names partners by id (found through
// where[]); a table keyed by index (md_bonded_reindex) is read coalesced and
// names the partners' indices directly.
#include "md_bonded.hpp"

namespace md {
namespace {

struct FeneArgs {
    const int32_t *atom_off, *unit_rep, *unit_off;
    const double *box;
    const double *x, *y, *z;
    const int32_t *id, *where;   // used for tables keyed by id
    const int32_t *bcount, *bpartner;
    int32_t N, max_bonds;
    double K, R02;
    double *fx, *fy, *fz;
    double *partial;
    uint32_t *status;
};

template <int ORDER>
__global__ __launch_bounds__(kUnit) void k_fene(FeneArgs a)
{
    __shared__ double red[kWavesPerUnit];
    const int u = blockIdx.x;
    const Unit w = unit_of(u, a.unit_rep, a.unit_off, a.atom_off);
    const int i = w.begin + threadIdx.x;
    BondedSum sum{0.0, 0.0, 0.0, 0.0, 0.0};
    if (i < w.end) {
        const int me = ORDER == MD_BY_ID ? a.id[i] : i;   // column of the table
        const bool ok = fene_atom<ORDER>(i, me, a.x, a.y, a.z, a.where, a.bcount, a.bpartner,
                                         a.max_bonds, a.N, a.K, a.R02, bond_box(a.box, w.rep),
                                         sum);
        a.fx[i] += sum.fx;
        a.fy[i] += sum.fy;
        a.fz[i] += sum.fz;
        if (!ok && a.status) atomicOr(a.status, MD_F_BOND_BROKEN);
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

extern "C" int md_fene_forces(const md_batch *b, const md_atoms *atoms, const md_bonds *bonds,
                              double K, double R0, double *energy, double *virial, void *ws,
                              size_t ws_bytes, uint32_t *status, void *stream)
{
    using namespace md;
    int e = check_batch(b);
    if (e != MD_OK) return e;
    if (!atoms || !atoms->x || !atoms->y || !atoms->z || !atoms->fx || !atoms->fy ||
        !atoms->fz || !bonds || !bonds->count || !bonds->partner || !ws)
        return MD_EINVAL;
    if (bonds->order != MD_BY_ID && bonds->order != MD_BY_INDEX) return MD_EINVAL;
    if (bonds->order == MD_BY_ID && (!atoms->id || !atoms->where)) return MD_EINVAL;
    if (bonds->max_bonds < 1 || bonds->max_bonds > MD_MAX_BONDS) return MD_EINVAL;
    if (!(K >= 0.0) || !(R0 > 0.0)) return MD_EINVAL;
    const WsLayout l = ws_layout(b);
    if (ws_bytes < l.total) return MD_ENOWS;
    double *partial = ws_at<double>(ws, l.partial);
    FeneArgs a{b->atom_off, b->unit_rep, b->unit_off, b->box, atoms->x, atoms->y, atoms->z,
               atoms->id, atoms->where, bonds->count, bonds->partner, b->N, bonds->max_bonds,
               K, R0 * R0, atoms->fx, atoms->fy, atoms->fz, partial, status};
    hipStream_t s = as_stream(stream);
    if (bonds->order == MD_BY_ID)
        hipLaunchKernelGGL(k_fene<MD_BY_ID>, dim3(b->n_units), dim3(kUnit), 0, s, a);
    else
        hipLaunchKernelGGL(k_fene<MD_BY_INDEX>, dim3(b->n_units), dim3(kUnit), 0, s, a);
    if (energy || virial) launch_finalize_sum2(b->R, b->unit_off, partial, 0, energy, virial, s);
    return launch_status();
}

// md_bonded.hip -- md_bonded_reindex: bonded tables in the atoms' current order.
//
// The bonded terms (FENE bonds, the ring melt's angle triples) are given per
// atom id.  After a re-sort into cell order, a thread walking the atoms in
// their new order would reach its table column through id[i] (a scattered
// read per slot) and its partners through where[].  This pass, run once per
// re-sort, writes column id[i] of each table to column i with every member
// translated to its current index, so that the per-step bonded kernels read
// the tables coalesced and gather positions from nearby cells.  Replicas
// whose gate is 0 keep their tables (their atoms did not move).
#include "md_common.hpp"

namespace md {
namespace {

struct ReindexArgs {
    const int32_t *atom_off, *unit_rep, *unit_off;
    const uint32_t *gate;
    int32_t R, n_units, N;
    const int32_t *id, *where;
    const int32_t *bcount, *bpartner;   // MD_BY_ID bonds, or null
    int32_t max_bonds;
    int32_t *bcount_out, *bpartner_out;
    const int32_t *acount, *atri;       // MD_BY_ID triples, or null
    int32_t max_angles;
    int32_t *acount_out, *atri_out;
};

__global__ __launch_bounds__(kUnit) void k_reindex(ReindexArgs a)
{
    if (a.gate && a.R == 1 && a.gate[0] == 0u) return;
    for (int u = blockIdx.x; u < a.n_units; u += gridDim.x) {
        const Unit w = unit_of(u, a.unit_rep, a.unit_off, a.atom_off);
        if (a.gate && a.gate[w.rep] == 0u) continue;
        const int i = w.begin + threadIdx.x;
        if (i >= w.end) continue;
        const int me = a.id[i];
        if (a.bcount) {
            const int nb = min(a.bcount[me], a.max_bonds);
            a.bcount_out[i] = nb;
            for (int k = 0; k < a.max_bonds; ++k) {
                const size_t o = size_t(k) * a.N;
                a.bpartner_out[o + i] = k < nb ? a.where[a.bpartner[o + me]] : -1;
            }
        }
        if (a.acount) {
            const int nt = min(a.acount[me], a.max_angles);
            a.acount_out[i] = nt;
            for (int r = 0; r < 3 * a.max_angles; ++r) {
                const size_t o = size_t(r) * a.N;
                a.atri_out[o + i] = r / 3 < nt ? a.where[a.atri[o + me]] : -1;
            }
        }
    }
}

}  // namespace
}  // namespace md

extern "C" int md_bonded_reindex(const md_batch *b, const md_atoms *atoms, const md_bonds *bonds,
                                 int32_t *bond_count, int32_t *bond_partner,
                                 const md_angles *angles, int32_t *angle_count,
                                 int32_t *angle_tri, const uint32_t *gate, void *stream)
{
    using namespace md;
    int e = check_batch(b);
    if (e != MD_OK) return e;
    if (!atoms || !atoms->id || !atoms->where) return MD_EINVAL;
    if (bonds) {
        if (bonds->order != MD_BY_ID || !bonds->count || !bonds->partner || !bond_count ||
            !bond_partner || bonds->max_bonds < 1 || bonds->max_bonds > MD_MAX_BONDS)
            return MD_EINVAL;
    }
    if (angles) {
        if (angles->order != MD_BY_ID || !angles->count || !angles->tri || !angle_count ||
            !angle_tri || angles->max_angles < 1 || angles->max_angles > MD_MAX_ANGLES)
            return MD_EINVAL;
    }
    if (!bonds && !angles) return MD_OK;
    ReindexArgs a{b->atom_off, b->unit_rep, b->unit_off, gate, b->R, b->n_units, b->N,
                  atoms->id, atoms->where,
                  bonds ? bonds->count : nullptr, bonds ? bonds->partner : nullptr,
                  bonds ? bonds->max_bonds : 0, bond_count, bond_partner,
                  angles ? angles->count : nullptr, angles ? angles->tri : nullptr,
                  angles ? angles->max_angles : 0, angle_count, angle_tri};
    hipLaunchKernelGGL(k_reindex, dim3(gated_grid(b->n_units, gate != nullptr)), dim3(kUnit), 0,
                       as_stream(stream), a);
    return launch_status();
}

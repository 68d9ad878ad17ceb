// md_bonded.hip -- md_bonded_reindex: bonded tables in the atoms' current
// order; md_bonded_forces: FENE bonds and angle triples in one pass.
//
// The bonded terms (FENE bonds, the ring melt's angle triples) are given per
// atom id.  After a re-sort into cell order, a thread walking the atoms in
// their new order would reach its table column through id[i] (a scattered
// read per slot) and its partners through where[].  This pass, run once per
// re-sort, writes column id[i] of each table to column i with every member
// translated to its current index, so that the per-step bonded kernels read
// the tables coalesced and gather positions from nearby cells.  Replicas
// whose gate is 0 keep their tables (their atoms did not move).
#include <cmath>

#include "md_bonded.hpp"

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

// FENE bonds and angle triples of the atom at index i (tables keyed by
// index), one thread per atom: one read of the position planes' cache lines
// for both terms, one force update, partials (E_bond, W_bond, E_angle,
// W_angle) per work unit.
struct BondedArgs {
    const int32_t *atom_off, *unit_rep, *unit_off;
    const double *box;
    const double *x, *y, *z;
    const int32_t *bcount, *bpartner;
    int32_t max_bonds;
    double K, R02;
    const int32_t *acount, *tri;
    int32_t max_angles;
    double Ka;
    int32_t N;
    double *fx, *fy, *fz;
    double *partial;
    uint32_t *status;
};

__global__ __launch_bounds__(kUnit) void k_bonded(BondedArgs a)
{
    __shared__ double red[kWavesPerUnit];
    const int u = blockIdx.x;
    const Unit w = unit_of(u, a.unit_rep, a.unit_off, a.atom_off);
    const int i = w.begin + threadIdx.x;
    BondedSum b{0.0, 0.0, 0.0, 0.0, 0.0}, t{0.0, 0.0, 0.0, 0.0, 0.0};
    if (i < w.end) {
        const BondBox bx = bond_box(a.box, w.rep);
        const bool bond_ok = fene_atom<MD_BY_INDEX>(i, i, a.x, a.y, a.z, nullptr, a.bcount,
                                                    a.bpartner, a.max_bonds, a.N, a.K, a.R02,
                                                    bx, b);
        const bool tri_ok = angle_atom<MD_BY_INDEX>(i, a.x, a.y, a.z, nullptr, a.acount, a.tri,
                                                    a.max_angles, a.N, a.Ka, bx, t);
        // the same sums in the same order as the two separate calls
        a.fx[i] = (a.fx[i] + b.fx) + t.fx;
        a.fy[i] = (a.fy[i] + b.fy) + t.fy;
        a.fz[i] = (a.fz[i] + b.fz) + t.fz;
        if (a.status && !bond_ok) atomicOr(a.status, MD_F_BOND_BROKEN);
        if (a.status && !tri_ok) atomicOr(a.status, MD_F_NONFINITE);
    }
    const double s0 = block_sum(b.e, red), s1 = block_sum(b.w, red);
    const double s2 = block_sum(t.e, red), s3 = block_sum(t.w, red);
    if (threadIdx.x == 0) {
        double *q = a.partial + size_t(u) * kPartials;
        q[0] = s0;
        q[1] = s1;
        q[2] = s2;
        q[3] = s3;
    }
}

// One workgroup per replica: fixed-order sums of the four partial columns.
__global__ __launch_bounds__(kFin) void k_bonded_finalize(const int32_t *unit_off,
                                                          const double *partial, double *e_bond,
                                                          double *w_bond, double *e_angle,
                                                          double *w_angle)
{
    __shared__ double red[kFin / kWave];
    const int r = blockIdx.x;
    const int u0 = unit_off[r], u1 = unit_off[r + 1];
    double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int u = u0 + threadIdx.x; u < u1; u += kFin)
        for (int k = 0; k < 4; ++k) s[k] += partial[size_t(u) * kPartials + k];
    for (int k = 0; k < 4; ++k) s[k] = block_sum_n<kFin>(s[k], red);
    if (threadIdx.x == 0) {
        if (e_bond) e_bond[r] = s[0];
        if (w_bond) w_bond[r] = s[1];
        if (e_angle) e_angle[r] = s[2];
        if (w_angle) w_angle[r] = s[3];
    }
}

}  // namespace
}  // namespace md

extern "C" int md_bonded_forces(const md_batch *b, const md_atoms *atoms, const md_bonds *bonds,
                                double K, double R0, const md_angles *angles, double Ka,
                                double *energy_bond, double *virial_bond, double *energy_angle,
                                double *virial_angle, void *ws, size_t ws_bytes,
                                uint32_t *status, void *stream)
{
    using namespace md;
    int e = check_batch(b);
    if (e != MD_OK) return e;
    if (!atoms || !atoms->x || !atoms->y || !atoms->z || !atoms->fx || !atoms->fy ||
        !atoms->fz || !bonds || !bonds->count || !bonds->partner || !angles ||
        !angles->count || !angles->tri || !ws)
        return MD_EINVAL;
    if (bonds->order != MD_BY_INDEX || angles->order != MD_BY_INDEX) return MD_EINVAL;
    if (bonds->max_bonds < 1 || bonds->max_bonds > MD_MAX_BONDS) return MD_EINVAL;
    if (angles->max_angles < 1 || angles->max_angles > MD_MAX_ANGLES) return MD_EINVAL;
    if (!(K >= 0.0) || !(R0 > 0.0) || !(Ka >= 0.0) || !(Ka < HUGE_VAL)) return MD_EINVAL;
    const WsLayout l = ws_layout(b);
    if (ws_bytes < l.total) return MD_ENOWS;
    double *partial = ws_at<double>(ws, l.partial);
    BondedArgs a{b->atom_off, b->unit_rep, b->unit_off, b->box, atoms->x, atoms->y, atoms->z,
                 bonds->count, bonds->partner, bonds->max_bonds, K, R0 * R0, angles->count,
                 angles->tri, angles->max_angles, Ka, b->N, atoms->fx, atoms->fy, atoms->fz,
                 partial, status};
    hipStream_t s = as_stream(stream);
    hipLaunchKernelGGL(k_bonded, dim3(b->n_units), dim3(kUnit), 0, s, a);
    if (energy_bond || virial_bond || energy_angle || virial_angle)
        hipLaunchKernelGGL(k_bonded_finalize, dim3(b->R), dim3(kFin), 0, s, b->unit_off, partial,
                           energy_bond, virial_bond, energy_angle, virial_angle);
    return launch_status();
}

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

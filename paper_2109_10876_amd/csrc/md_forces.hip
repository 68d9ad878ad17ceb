// md_forces.hip -- md_lj_forces: Lennard-Jones forces, energy and virial.
//
// Eq. lj of the paper, U(r) = 4 eps [(sig/r)^12 - (sig/r)^6] for r < r_cut,
// summed over the Verlet list (Sec. 2.1.1-2.1.2).  With s6 = (sig^2/r^2)^3:
//     fr = -U'(r)/r = 24 eps s6 (2 s6 - 1) / r^2,   U = 4 eps s6 (s6 - 1)
// and the force on i from j is fr * d with d = x_i - x_j + s L (list image).
//
// Mapping: one thread per atom i, 256 atoms per workgroup, work units
// remapped per XCD.  The thread walks its column of the ELL list; entry k of
// 64 consecutive atoms is one coalesced 256-byte row.  Neighbour positions
// are gathered from the cell-sorted SoA planes (mostly L2 hits).
//
// MD_FULL: each atom sums its own force, no atomics, bitwise deterministic;
// each pair's energy and virial are counted from both sides and halved.
// MD_HALF: the paper's Newton's-third-law list (Sec. 2.1.2); the partner's
// force is added with FP64 atomics.
//
// MD_FP32_MIXED: displacement, r^2, the cutoff test and the force
// accumulation stay in double (positions up to ~100 sigma would lose the
// displacement's low bits in single); only the reciprocal and the LJ
// polynomial are single precision.  Per-atom energy/virial sums are single,
// the per-replica totals double.
//
// Energy and virial: per-unit partial sums in fixed order, then one
// workgroup per replica sums its units in fixed order.
#include "md_pair.hpp"

namespace md {
namespace {

struct ForceArgs {
    const int32_t *atom_off, *unit_rep, *unit_off;
    const double *box;
    const double *x, *y, *z;
    const double *pos4;  // optional packed gather source
    const int32_t *type;
    const int32_t *count;
    const uint32_t *idx;
    int32_t ld, max_nbr;
    const double *eps, *sig;
    int32_t ntypes, shift;
    double rc;
    double *fx, *fy, *fz;
    int32_t accumulate;
    double *partial;     // [n_units * kPartials]
    uint32_t *status;
};

// Neighbour position j: from the packed copy (one 32-byte load) or from the
// three SoA planes.
template <bool P4>
__device__ __forceinline__ void load_pos(const ForceArgs &a, int j, double &px, double &py,
                                         double &pz)
{
    if (P4) {
        const double4 p = reinterpret_cast<const double4 *>(a.pos4)[j];
        px = p.x;
        py = p.y;
        pz = p.z;
    } else {
        px = a.x[j];
        py = a.y[j];
        pz = a.z[j];
    }
}

// One list entry: displacement with the entry's periodic image, then the
// pair terms.
template <int PREC, bool HALF>
__device__ __forceinline__ void pair(const ForceArgs &a, const PairConst &pc, uint32_t ent,
                                     double dx, double dy, double dz, double Lx, double Ly,
                                     double Lz, double rc2, Acc &c)
{
    const uint32_t code = ent >> MD_IDX_BITS;
    if (code != 0u) {
        dx += image_shift(code & 3u) * Lx;
        dy += image_shift((code >> 2) & 3u) * Ly;
        dz += image_shift((code >> 4) & 3u) * Lz;
    }
    const double fr = lj_pair_accumulate<PREC>(pc, dx, dy, dz, rc2, c);
    if (HALF && fr != 0.0) {
        const int j = static_cast<int>(ent & MD_IDX_MASK);
        atomicAdd(a.fx + j, -fr * dx);
        atomicAdd(a.fy + j, -fr * dy);
        atomicAdd(a.fz + j, -fr * dz);
    }
}

// One thread per atom.  The list column is consumed U entries at a time:
// U coalesced (non-temporal: the list is streamed once per call) index
// loads, then all U neighbour gathers, then the U pair evaluations -- so
// each wave keeps U gathers in flight instead of one.
template <int PREC, bool HALF, bool TYPED, int U, bool P4>
__global__ __launch_bounds__(kUnit) void k_lj(ForceArgs a)
{
    __shared__ PairConst tab[MD_MAX_TYPES * MD_MAX_TYPES];
    __shared__ double red[kWavesPerUnit];
    const int u = xcd_swizzle(blockIdx.x, gridDim.x);
    const Unit w = unit_of(u, a.unit_rep, a.unit_off, a.atom_off);

    PairConst pc0;
    if (TYPED) {
        const int nt2 = a.ntypes * a.ntypes;
        for (int t = threadIdx.x; t < nt2; t += kUnit)
            tab[t] = pair_const(a.eps[t], a.sig[t], a.rc, a.shift);
        __syncthreads();
    } else {
        pc0 = pair_const(a.eps[0], a.sig[0], a.rc, a.shift);
    }

    const int i = w.begin + threadIdx.x;
    const bool active = i < w.end;
    const double rc2 = a.rc * a.rc;
    double e_acc = 0.0, w_acc = 0.0;
    if (active) {
        const double Lx = a.box[3 * w.rep], Ly = a.box[3 * w.rep + 1], Lz = a.box[3 * w.rep + 2];
        const double xi = a.x[i], yi = a.y[i], zi = a.z[i];
        const int ti = TYPED ? a.type[i] : 0;
        const int n = min(a.count[i], a.max_nbr);
        Acc c{0.0, 0.0, 0.0, 0.0, 0.0, 0.0f, 0.0f, 0u};
        const uint32_t *col = a.idx + i;
        int k = 0;
        for (; k + U <= n; k += U) {
            uint32_t ent[U];
#pragma unroll
            for (int q = 0; q < U; ++q)
                ent[q] = __builtin_nontemporal_load(col + size_t(k + q) * a.ld);
            double px[U], py[U], pz[U];
            int tj[U];
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const int j = static_cast<int>(ent[q] & MD_IDX_MASK);
                load_pos<P4>(a, j, px[q], py[q], pz[q]);
                tj[q] = TYPED ? a.type[j] : 0;
            }
#pragma unroll
            for (int q = 0; q < U; ++q) {
                const PairConst &pc = TYPED ? tab[ti * a.ntypes + tj[q]] : pc0;
                pair<PREC, HALF>(a, pc, ent[q], xi - px[q], yi - py[q], zi - pz[q], Lx, Ly, Lz,
                                 rc2, c);
            }
        }
        for (; k < n; ++k) {
            const uint32_t ent = __builtin_nontemporal_load(col + size_t(k) * a.ld);
            const int j = static_cast<int>(ent & MD_IDX_MASK);
            double px, py, pz;
            load_pos<P4>(a, j, px, py, pz);
            const PairConst &pc = TYPED ? tab[ti * a.ntypes + a.type[j]] : pc0;
            pair<PREC, HALF>(a, pc, ent, xi - px, yi - py, zi - pz, Lx, Ly, Lz, rc2, c);
        }
        double ed = c.ed, wd = c.wd;
        if (PREC != MD_FP64) {
            ed = static_cast<double>(c.ef);
            wd = static_cast<double>(c.wf);
        }
        e_acc = HALF ? ed : 0.5 * ed;
        w_acc = HALF ? wd : 0.5 * wd;
        if (HALF) {
            atomicAdd(a.fx + i, c.fx);
            atomicAdd(a.fy + i, c.fy);
            atomicAdd(a.fz + i, c.fz);
        } else if (a.accumulate) {
            a.fx[i] += c.fx;
            a.fy[i] += c.fy;
            a.fz[i] += c.fz;
        } else {
            a.fx[i] = c.fx;
            a.fy[i] = c.fy;
            a.fz[i] = c.fz;
        }
        if (a.status && !isfinite(c.fx + c.fy + c.fz + ed)) atomicOr(a.status, MD_F_NONFINITE);
    }
    const double es = block_sum(e_acc, red);
    const double ws = block_sum(w_acc, red);
    if (threadIdx.x == 0) {
        a.partial[size_t(u) * kPartials + 0] = es;
        a.partial[size_t(u) * kPartials + 1] = ws;
    }
}

__global__ __launch_bounds__(kUnit) void k_zero3(int32_t N, double *fx, double *fy, double *fz)
{
    const int i = blockIdx.x * kUnit + threadIdx.x;
    if (i < N) {
        fx[i] = 0.0;
        fy[i] = 0.0;
        fz[i] = 0.0;
    }
}

}  // namespace

// One workgroup per replica: fixed-order sum of slot `k0` (and `k0+1`) of its
// work units' partials.
__global__ __launch_bounds__(kFin) void k_finalize_sum2(const int32_t *unit_off,
                                                        const double *partial, int k0,
                                                        double *out0, double *out1)
{
    __shared__ double red[kFin / kWave];
    const int r = blockIdx.x;
    const int u0 = unit_off[r], u1 = unit_off[r + 1];
    double s0 = 0.0, s1 = 0.0;
#pragma unroll 4
    for (int u = u0 + threadIdx.x; u < u1; u += kFin) {
        s0 += partial[size_t(u) * kPartials + k0];
        s1 += partial[size_t(u) * kPartials + k0 + 1];
    }
    s0 = block_sum_n<kFin>(s0, red);
    s1 = block_sum_n<kFin>(s1, red);
    if (threadIdx.x == 0) {
        if (out0) out0[r] = s0;
        if (out1) out1[r] = s1;
    }
}

// Template dispatch: precision x list mode x typed x batch x gather source.
template <int PREC, bool HALF, bool TYPED, int U>
void launch_lj_u(const ForceArgs &a, int n_units, bool p4, hipStream_t s)
{
    if (p4) hipLaunchKernelGGL((k_lj<PREC, HALF, TYPED, U, true>), dim3(n_units), dim3(kUnit), 0, s, a);
    else hipLaunchKernelGGL((k_lj<PREC, HALF, TYPED, U, false>), dim3(n_units), dim3(kUnit), 0, s, a);
}

template <int PREC, bool HALF, bool TYPED>
void launch_lj_t(const ForceArgs &a, int n_units, int batch, bool p4, hipStream_t s)
{
    switch (batch) {
    case 1: launch_lj_u<PREC, HALF, TYPED, 1>(a, n_units, p4, s); break;
    case 2: launch_lj_u<PREC, HALF, TYPED, 2>(a, n_units, p4, s); break;
    case 8: launch_lj_u<PREC, HALF, TYPED, 8>(a, n_units, p4, s); break;
    default: launch_lj_u<PREC, HALF, TYPED, 4>(a, n_units, p4, s); break;
    }
}

template <int PREC>
void launch_lj_p(const ForceArgs &a, int n_units, bool half, bool typed, int batch, bool p4,
                 hipStream_t s)
{
    if (half) {
        if (typed) launch_lj_t<PREC, true, true>(a, n_units, batch, p4, s);
        else launch_lj_t<PREC, true, false>(a, n_units, batch, p4, s);
    } else {
        if (typed) launch_lj_t<PREC, false, true>(a, n_units, batch, p4, s);
        else launch_lj_t<PREC, false, false>(a, n_units, batch, p4, s);
    }
}

void launch_lj(const ForceArgs &a, int n_units, int prec, bool half, bool typed, int batch,
               bool p4, hipStream_t s)
{
    if (prec == MD_FP64) launch_lj_p<MD_FP64>(a, n_units, half, typed, batch, p4, s);
    else launch_lj_p<MD_FP32_MIXED>(a, n_units, half, typed, batch, p4, s);
}

void launch_finalize_sum2(int R, const int32_t *unit_off, const double *partial, int k0,
                          double *out0, double *out1, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize_sum2, dim3(R), dim3(kFin), 0, s, unit_off, partial, k0,
                       out0, out1);
}

}  // namespace md

namespace md {

int lj_forces_check(const md_batch *b, const md_atoms *atoms, const md_nlist *nl,
                    const md_lj *p, int32_t prec)
{
    int e = check_batch(b);
    if (e != MD_OK) return e;
    if (!atoms || !atoms->x || !atoms->y || !atoms->z || !atoms->fx || !atoms->fy ||
        !atoms->fz || !nl || !nl->count || !nl->idx || !p || !p->eps || !p->sig)
        return MD_EINVAL;
    if (nl->mode != MD_HALF && nl->mode != MD_FULL && nl->mode != MD_TILE_FULL) return MD_EINVAL;
    if (nl->max_nbr < 1 || nl->ld < b->N || nl->ld % 64 != 0) return MD_EINVAL;
    if (p->ntypes < 1 || p->ntypes > MD_MAX_TYPES || !(p->rc > 0.0)) return MD_EINVAL;
    if (p->ntypes > 1 && !atoms->type) return MD_EINVAL;
    if (prec != MD_FP64 && prec != MD_FP32_MIXED) return MD_EINVAL;
    if (nl->mode == MD_TILE_FULL) {
        if (!tile_list_ok(b, nl) || !nl->cell_start) return MD_EINVAL;
        if (p->ntypes > MD_TILE_MAX_TYPES) return MD_EUNSUPPORTED;
        // a typed list is needed for several types, and only then
        if (p->ntypes > 1 ? (nl->tile_types != p->ntypes || !atoms->type) : nl->tile_types > 1)
            return MD_EINVAL;
    }
    return MD_OK;
}

int lj_forces_run(const md_batch *b, const md_atoms *atoms, const md_nlist *nl, const md_lj *p,
                  int32_t prec, int32_t accumulate, double *energy, double *virial,
                  double *partial, double *tpart, uint32_t *status, hipStream_t s)
{
    if (nl->mode == MD_TILE_FULL)
        return tile_forces(b, atoms, nl, p, prec, accumulate, nl->cell_start, energy, virial,
                           tpart, partial, b->n_units, md_tune_get(MD_TUNE_PAIR_BATCH), nullptr,
                           status, s);
    ForceArgs a{b->atom_off, b->unit_rep, b->unit_off, b->box, atoms->x, atoms->y, atoms->z,
                atoms->pos4, atoms->type, nl->count, nl->idx, nl->ld, nl->max_nbr, p->eps,
                p->sig, p->ntypes, p->shift, p->rc, atoms->fx, atoms->fy, atoms->fz, accumulate,
                partial, status};
    const bool half = nl->mode == MD_HALF;
    if (half && !accumulate)
        hipLaunchKernelGGL(k_zero3, dim3((b->N + kUnit - 1) / kUnit), dim3(kUnit), 0, s, b->N,
                           atoms->fx, atoms->fy, atoms->fz);
    const int timed = timing_begin(s);
    launch_lj(a, b->n_units, prec, half, p->ntypes > 1, md_tune_get(MD_TUNE_PAIR_BATCH),
              atoms->pos4 != nullptr, s);
    timing_end(timed, s);
    if (energy || virial)
        launch_finalize_sum2(b->R, b->unit_off, partial, 0, energy, virial, s);
    return launch_status();
}

}  // namespace md

extern "C" int md_lj_forces(const md_batch *b, const md_atoms *atoms, const md_nlist *nl,
                            const md_lj *p, int32_t prec, int32_t accumulate, double *energy,
                            double *virial, void *ws, size_t ws_bytes, uint32_t *status,
                            void *stream)
{
    using namespace md;
    int e = lj_forces_check(b, atoms, nl, p, prec);
    if (e != MD_OK) return e;
    if (!ws) return MD_EINVAL;
    const WsLayout l = ws_layout(b);
    if (ws_bytes < l.total) return MD_ENOWS;
    return lj_forces_run(b, atoms, nl, p, prec, accumulate, energy, virial,
                         ws_at<double>(ws, l.partial), ws_at<double>(ws, l.tile_partial), status,
                         as_stream(stream));
}

extern "C" int md_lj_forces_vv(const md_batch *b, md_atoms *atoms, const md_nlist *nl,
                               const md_lj *p, int32_t prec, double dt, const double *inv_mass,
                               int32_t ntypes, double skin, uint32_t *gate,
                               uint32_t *gate_clear, double *ke,
                               double *energy, double *virial, double *x_next, double *y_next,
                               double *z_next, const md_thermostat *thermo, void *ws,
                               size_t ws_bytes, uint32_t *status, void *stream)
{
    using namespace md;
    int e = check_batch(b);
    if (e != MD_OK) return e;
    if (!atoms || !atoms->x || !atoms->y || !atoms->z || !atoms->fx || !atoms->fy ||
        !atoms->fz || !atoms->vx || !atoms->vy || !atoms->vz || !atoms->xb || !atoms->yb ||
        !atoms->zb || !nl || !nl->count || !nl->idx || !p || !p->eps || !p->sig || !ws ||
        !inv_mass || !gate)
        return MD_EINVAL;
    if (nl->mode != MD_TILE_FULL) return MD_EUNSUPPORTED;
    if (nl->max_nbr < 1 || nl->ld < b->N || nl->ld % 64 != 0) return MD_EINVAL;
    if (p->ntypes < 1 || !(p->rc > 0.0)) return MD_EINVAL;
    if (p->ntypes > MD_TILE_MAX_TYPES) return MD_EUNSUPPORTED;
    if (p->ntypes > 1 && !atoms->type) return MD_EINVAL;
    if (ntypes < 1 || ntypes > MD_MAX_TYPES || (ntypes > 1 && !atoms->type)) return MD_EINVAL;
    if (prec != MD_FP64 && prec != MD_FP32_MIXED) return MD_EINVAL;
    if (!(skin >= 0.0) || !(dt > 0.0)) return MD_EINVAL;
    if (thermo && (!thermo->step || !thermo->mass || !atoms->id || !(thermo->gamma >= 0.0) ||
                   !(thermo->temperature >= 0.0)))
        return MD_EINVAL;
    // alternating gate words: not with the thermostat (its counter is
    // advanced by the finaliser), and not overlapping
    if (gate_clear && (thermo || (gate_clear < gate + b->R && gate < gate_clear + b->R)))
        return MD_EINVAL;
    const WsLayout l = ws_layout(b);
    if (ws_bytes < l.total) return MD_ENOWS;
    // a typed list for several types, and only then
    if (!tile_list_ok(b, nl) || !nl->cell_start ||
        (p->ntypes > 1 ? nl->tile_types != p->ntypes : nl->tile_types > 1))
        return MD_EINVAL;
    // next positions: the caller's buffers (all three, not overlapping the
    // current ones, and no packed copy to keep), or workspace copied back
    const bool given = x_next || y_next || z_next;
    if (given) {
        if (!x_next || !y_next || !z_next || atoms->pos4) return MD_EINVAL;
        const double *cur[3] = {atoms->x, atoms->y, atoms->z};
        const double *nxt[3] = {x_next, y_next, z_next};
        for (const double *c : cur)
            for (const double *n : nxt)
                if (n < c + b->N && c < n + b->N) return MD_EINVAL;
    }
    double *xw = ws_at<double>(ws, l.xnext);
    const VVFuse f{atoms->vx, atoms->vy, atoms->vz, atoms->xb, atoms->yb, atoms->zb, inv_mass,
                   ntypes, 0.5 * dt, dt, 0.25 * skin * skin,
                   given ? x_next : xw, given ? y_next : xw + b->N,
                   given ? z_next : xw + 2 * size_t(b->N), ke, gate, gate_clear, !given,
                   thermo ? atoms->id : nullptr, thermo ? thermo->mass : nullptr,
                   thermo ? thermo->gamma : 0.0,
                   thermo ? 2.0 * thermo->temperature / dt : 0.0,
                   thermo ? static_cast<uint32_t>(thermo->seed) : 0u,
                   thermo ? static_cast<uint32_t>(thermo->seed >> 32) : 0u,
                   thermo ? thermo->step : nullptr};
    return tile_forces(b, atoms, nl, p, prec, 0, nl->cell_start, energy, virial,
                       ws_at<double>(ws, l.tile_partial), ws_at<double>(ws, l.partial),
                       b->n_units, md_tune_get(MD_TUNE_PAIR_BATCH), &f, status,
                       as_stream(stream));
}

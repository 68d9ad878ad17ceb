// md_vjp.hip -- md_lj_forces_vjp: vector-Jacobian product of the LJ forces
// and energy with respect to positions and the per-type (eps, sigma) tables.
//
// Derivatives of Eq. lj (paper Sec. 2.1.1).  With s2 = sig^2/r^2, s6 = s2^3,
// s12 = s6^2 and inv = 1/r^2:
//   fr        = eps (24 s6 (2 s6 - 1)) inv             force factor, F_i = fr d
//   fr'/r     = eps (-672 s12 + 192 s6) inv^2
//   U         = eps (4 (s12 - s6) - shift * 4 (c12 - c6))        c = values at rc
//   dfr/dsig  = (eps/sig) (576 s12 - 144 s6) inv
//   dU/dsig   = (eps/sig) ((48 s12 - 24 s6) - shift * (48 c12 - 24 c6))
//   fr and U are linear in eps.
// For an upstream G = dL/dF and gE = dL/dE, pair (i, j) with d = x_i - x_j and
// u = G_i - G_j contributes w = fr u + (fr'/r)(d.u) d - gE fr d to dL/dx_i and
// -w to dL/dx_j; (d.u) dfr/dp + gE dU/dp to the parameter p of its type pair.
// With a full list, atom i's own column gives every w of its pairs (the
// partner's visit gives -w to the partner), so each thread writes only its
// own gradient -- no atomics, nothing stored from the forward pass: the pair
// terms are recomputed.  Parameter terms are seen from both atoms and halved.
#include "md_pair.hpp"

namespace md {
namespace {

struct VjpArgs {
    const int32_t *atom_off, *unit_rep, *unit_off;
    const double *box;
    const double *x, *y, *z;
    const int32_t *type;
    const int32_t *count;
    const uint32_t *idx;
    int32_t ld, max_nbr;
    const double *eps, *sig;
    int32_t ntypes, shift;
    double rc;
    const double *gfx, *gfy, *gfz, *gE;
    double *gx;
    int32_t N;
    double *vpart;   // [n_units][2][MD_MAX_TYPES^2]
    uint32_t *status;
};

constexpr int kSlots = MD_MAX_TYPES * MD_MAX_TYPES;

template <int PREC, int NT>
__global__ __launch_bounds__(kUnit) void k_vjp(VjpArgs a)
{
    __shared__ VjpConst tab[kSlots];
    __shared__ double red[kWavesPerUnit];
    const int u = xcd_swizzle(blockIdx.x, gridDim.x);
    const Unit w = unit_of(u, a.unit_rep, a.unit_off, a.atom_off);
    const int nt = a.ntypes;
    for (int t = threadIdx.x; t < nt * nt; t += kUnit)
        tab[t] = vjp_const(a.eps[t], a.sig[t], a.rc, a.shift);
    __syncthreads();

    double ge[NT], gs[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) { ge[t] = 0.0; gs[t] = 0.0; }
    const int i = w.begin + threadIdx.x;
    const bool active = i < w.end;
    int ti = 0;
    if (active) {
        const double Lx = a.box[3 * w.rep], Ly = a.box[3 * w.rep + 1], Lz = a.box[3 * w.rep + 2];
        const double gEr = a.gE ? a.gE[w.rep] : 0.0;
        const double rc2 = a.rc * a.rc;
        const double xi = a.x[i], yi = a.y[i], zi = a.z[i];
        const double Gx = a.gfx[i], Gy = a.gfy[i], Gz = a.gfz[i];
        ti = NT > 1 ? a.type[i] : 0;
        const int n = min(a.count[i], a.max_nbr);
        double ax = 0.0, ay = 0.0, az = 0.0;
        const uint32_t *col = a.idx + i;
        for (int k = 0; k < n; ++k) {
            const uint32_t ent = col[size_t(k) * a.ld];
            const int j = static_cast<int>(ent & MD_IDX_MASK);
            double dx = xi - a.x[j], dy = yi - a.y[j], dz = zi - a.z[j];
            const uint32_t code = ent >> MD_IDX_BITS;
            if (code != 0u) {
                dx += image_shift(code & 3u) * Lx;
                dy += image_shift((code >> 2) & 3u) * Ly;
                dz += image_shift((code >> 4) & 3u) * Lz;
            }
            const double r2 = norm2(dx, dy, dz);
            if (!(r2 < rc2)) continue;
            const int tj = NT > 1 ? a.type[j] : 0;
            const VjpConst c = tab[ti * nt + tj];
            const VjpTerms v = vjp_terms<PREC>(c, r2);
            const double fr1 = v.fr1, dfr1 = v.dfr1, u1 = v.u1, dfs1 = v.dfs1, dus1 = v.dus1;
            const double fr = c.eps * fr1, dfr = c.eps * dfr1;
            const double ux = Gx - a.gfx[j], uy = Gy - a.gfy[j], uz = Gz - a.gfz[j];
            const double du = dx * ux + dy * uy + dz * uz;
            const double t1 = dfr * du - gEr * fr;
            ax += fr * ux + t1 * dx;
            ay += fr * uy + t1 * dy;
            az += fr * uz + t1 * dz;
            const double pe = du * fr1 + gEr * u1;
            const double ps = c.eos * (du * dfs1 + gEr * dus1);
#pragma unroll
            for (int t = 0; t < NT; ++t)
                if (t == tj) { ge[t] += pe; gs[t] += ps; }
        }
        a.gx[i] = ax;
        a.gx[a.N + i] = ay;
        a.gx[2 * a.N + i] = az;
        if (a.status && !isfinite(ax + ay + az)) atomicOr(a.status, MD_F_NONFINITE);
    }
    // Block sums per (type_i, type_j) slot; each pair was seen from both atoms.
    double *vp = a.vpart + size_t(u) * 2 * kSlots;
    for (int ta = 0; ta < nt; ++ta) {
#pragma unroll
        for (int tb = 0; tb < NT; ++tb) {
            if (tb >= nt) break;
            const bool mine = active && ti == ta;
            const double se = block_sum(mine ? 0.5 * ge[tb] : 0.0, red);
            const double ss = block_sum(mine ? 0.5 * gs[tb] : 0.0, red);
            if (threadIdx.x == 0) {
                vp[ta * nt + tb] = se;
                vp[kSlots + ta * nt + tb] = ss;
            }
        }
    }
}

// One workgroup per output entry (kind, a, b): fixed-order sum over all
// units of slot (a, b) plus slot (b, a) for a != b.
__global__ __launch_bounds__(kUnit) void k_vjp_finalize(int n_units, int nt, const double *vpart,
                                                        double *geps, double *gsig)
{
    __shared__ double red[kWavesPerUnit];
    const int kind = blockIdx.x / (nt * nt), ab = blockIdx.x % (nt * nt);
    const int ta = ab / nt, tb = ab % nt;
    double s = 0.0;
    for (int u = threadIdx.x; u < n_units; u += kUnit) {
        const double *vp = vpart + size_t(u) * 2 * kSlots + kind * kSlots;
        s += ta == tb ? vp[ta * nt + tb] : vp[ta * nt + tb] + vp[tb * nt + ta];
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
        double *out = kind == 0 ? geps : gsig;
        if (out) out[ta * nt + tb] = s;
    }
}

}  // namespace
}  // namespace md

extern "C" int md_lj_forces_vjp(const md_batch *b, const md_atoms *atoms, const md_nlist *nl,
                                const md_lj *p, int32_t prec, const double *gfx,
                                const double *gfy, const double *gfz, const double *gE,
                                double *gx, double *geps, double *gsig, void *ws,
                                size_t ws_bytes, uint32_t *status, void *stream)
{
    using namespace md;
    int e = check_batch(b);
    if (e != MD_OK) return e;
    if (!atoms || !atoms->x || !atoms->y || !atoms->z || !nl || !nl->count || !nl->idx || !p ||
        !p->eps || !p->sig || !gfx || !gfy || !gfz || !gx || !ws)
        return MD_EINVAL;
    if (nl->mode != MD_FULL && nl->mode != MD_TILE_FULL) return MD_EUNSUPPORTED;
    if (nl->max_nbr < 1 || nl->ld < b->N || nl->ld % 64 != 0) return MD_EINVAL;
    if (p->ntypes < 1 || p->ntypes > MD_MAX_TYPES || !(p->rc > 0.0)) return MD_EINVAL;
    if (p->ntypes > 1 && !atoms->type) return MD_EINVAL;
    if (prec != MD_FP64 && prec != MD_FP32_MIXED) return MD_EINVAL;
    const WsLayout l = ws_layout(b);
    if (ws_bytes < l.total) return MD_ENOWS;
    if (nl->mode == MD_TILE_FULL) {
        // as for md_lj_forces: a typed list for several types, and only then
        if (!tile_list_ok(b, nl) || !nl->cell_start) return MD_EINVAL;
        if (p->ntypes > MD_TILE_MAX_TYPES) return MD_EUNSUPPORTED;
        if (p->ntypes > 1 ? nl->tile_types != p->ntypes : nl->tile_types > 1) return MD_EINVAL;
        return tile_vjp(b, atoms, nl, p, prec, gfx, gfy, gfz, gE, gx, geps, gsig, status,
                        as_stream(stream));
    }
    VjpArgs a{b->atom_off, b->unit_rep, b->unit_off, b->box, atoms->x, atoms->y, atoms->z,
              atoms->type, nl->count, nl->idx, nl->ld, nl->max_nbr, p->eps, p->sig, p->ntypes,
              p->shift, p->rc, gfx, gfy, gfz, gE, gx, b->N, ws_at<double>(ws, l.vjp_partial),
              status};
    hipStream_t s = as_stream(stream);
    const dim3 grid(b->n_units), block(kUnit);
    const int nt = p->ntypes;
#define MD_VJP_LAUNCH(P, T) hipLaunchKernelGGL((k_vjp<P, T>), grid, block, 0, s, a)
    if (prec == MD_FP64) {
        if (nt == 1) MD_VJP_LAUNCH(MD_FP64, 1);
        else if (nt == 2) MD_VJP_LAUNCH(MD_FP64, 2);
        else if (nt <= 4) MD_VJP_LAUNCH(MD_FP64, 4);
        else MD_VJP_LAUNCH(MD_FP64, 8);
    } else {
        if (nt == 1) MD_VJP_LAUNCH(MD_FP32_MIXED, 1);
        else if (nt == 2) MD_VJP_LAUNCH(MD_FP32_MIXED, 2);
        else if (nt <= 4) MD_VJP_LAUNCH(MD_FP32_MIXED, 4);
        else MD_VJP_LAUNCH(MD_FP32_MIXED, 8);
    }
#undef MD_VJP_LAUNCH
    if (geps || gsig)
        hipLaunchKernelGGL(k_vjp_finalize, dim3(2 * nt * nt), block, 0, s, b->n_units, nt,
                           ws_at<const double>(ws, l.vjp_partial), geps, gsig);
    return launch_status();
}

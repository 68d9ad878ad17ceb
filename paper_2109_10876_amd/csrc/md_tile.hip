// md_tile.hip -- tile-local Verlet lists (MD_TILE_FULL): list build and LJ
// forces with the neighbourhood of each tile staged in LDS.
//
// Same method as the global-index path (Sec. 2.1.2 cell stencil and Verlet
// radius, Eq. lj pair terms); only where neighbour positions come from
// differs.  One workgroup per tile (a block of m x py x pz cells):
//   1. stage the neighbouring rows x (a-1 .. b+1) into LDS, images applied
//      (md_tile.hpp);
//   2. build: every home atom tests the staged slots of its own 27-cell
//      stencil -- nine contiguous slot ranges, one per stencil row -- and
//      records hits as 16-bit
//      slots; forces: every home atom walks its list, reading neighbours
//      from LDS, no periodic-image arithmetic and no L2 gathers.
#include "md_pair.hpp"
#include "md_tile.hpp"

namespace md {
namespace {

struct TileArgs {
    const int32_t *tile_rep, *tile_off, *ncell, *cell_off;
    const double *box;
    const uint32_t *gate;
    const double *x, *y, *z, *pos4;
    const int32_t *cell_start;
    TileGrid g;
    int32_t n_tiles, max_nbr, ld;
    int32_t *count;
    uint16_t *idx;
    // build
    double rl2;
    int32_t *need, *tile_need;
    // forces
    const double *eps, *sig;
    int32_t shift;
    double rc;
    double *fx, *fy, *fz;
    int32_t accumulate;
    double *tpart;    // [n_tiles * 2]
    uint32_t *status;
    int32_t R;
};

constexpr int kCandBatch = 8;

template <class SH, bool P4>
__global__ __launch_bounds__(SH::TB) void k_tile_build(TileArgs a)
{
    constexpr int TB = SH::TB, CAP = SH::CAP;
    __shared__ TileStage<CAP, SH::MAXC> st;
    if (sole_replica_gated_off(a.gate, a.R)) return;
    for (int lt = blockIdx.x; lt < a.n_tiles; lt += gridDim.x) {
        const int t = xcd_swizzle(lt, a.n_tiles);
        const TileSpec s = tile_spec(t, a.tile_rep, a.tile_off, a.ncell, a.cell_off, a.box, a.g);
        if (a.gate != nullptr && a.gate[s.rep] == 0u) continue;
        const int total = stage_tile<TB, P4>(s, a.cell_start, a.x, a.y, a.z, a.pos4, st, CAP);
        if (total > CAP) {
            if (threadIdx.x == 0) {
                if (a.status) atomicOr(a.status, MD_F_TILE_OVERFLOW);
                if (a.tile_need) atomicMax(a.tile_need, total);
            }
            __syncthreads();
            continue;
        }
        const int nh = st.home_start[s.hy * s.hz];
        const double hx = s.L[0] / s.nx, hy = s.L[1] / s.ny, hz = s.L[2] / s.nz;
        // a neighbour cell is skipped when the distance from the atom to the
        // cell's box is at least r_l (with a relative margin far above
        // rounding, so no pair inside r_l is ever dropped)
        const double cull2 = a.rl2 * (1.0 + 1e-10);
        const uint32_t lastoff = uint32_t(a.max_nbr - 1) * uint32_t(a.ld);
        for (int hk = threadIdx.x; hk < nh; hk += TB) {
            int dy, dz;
            const int i = home_atom(s, st, hk, dy, dz);
            const double xi = a.x[i], yi = a.y[i], zi = a.z[i];
            const int cx = min(max(cell_coord(xi, cells_per_length(s.nx, s.L[0]), s.nx), s.a), s.b);
            const int kc = cx - s.a;   // stage index of unwrapped cell cx - 1
            const int qc = staged_row(s, dy, dz);
            const int own = st.row_slot[qc] + st.cslot[qc][kc + 1] +
                            (i - a.cell_start[st.row_rb[qc] + cx]);
            // squared gaps to the lower / upper faces of the atom's cell
            const double gxl = fmax(xi - cx * hx, 0.0), gxr = fmax((cx + 1) * hx - xi, 0.0);
            const int cy = s.y0 + dy, cz = s.z0 + dz;
            const double gyl = fmax(yi - cy * hy, 0.0), gyr = fmax((cy + 1) * hy - yi, 0.0);
            const double gzl = fmax(zi - cz * hz, 0.0), gzr = fmax((cz + 1) * hz - zi, 0.0);
            uint16_t *col = a.idx + i;
            uint32_t off = 0;   // element offset of the next entry, clamped to the last column
            int cnt = 0;
            for (int r9 = 0; r9 < 9; ++r9) {
                const int oy = r9 % 3 - 1, oz = r9 / 3 - 1;
                const double gy = oy < 0 ? gyl : (oy > 0 ? gyr : 0.0);
                const double gz = oz < 0 ? gzl : (oz > 0 ? gzr : 0.0);
                const double g2 = gy * gy + gz * gz;
                if (g2 >= cull2) continue;
                const int r = staged_row(s, dy + oy, dz + oz);
                const int k0 = kc + (g2 + gxl * gxl < cull2 ? 0 : 1);
                const int k1 = kc + (g2 + gxr * gxr < cull2 ? 3 : 2);
                const int s0 = st.row_slot[r] + st.cslot[r][k0];
                const int s1 = st.row_slot[r] + st.cslot[r][k1];
                for (int sb = s0; sb < s1; sb += kCandBatch) {
                    double px[kCandBatch], py[kCandBatch], pz[kCandBatch];
#pragma unroll
                    for (int q = 0; q < kCandBatch; ++q) {
                        const int sl = min(sb + q, s1 - 1);
                        px[q] = st.x[sl];
                        py[q] = st.y[sl];
                        pz[q] = st.z[sl];
                    }
#pragma unroll
                    for (int q = 0; q < kCandBatch; ++q) {
                        const int sl = sb + q;
                        const double dx = xi - px[q], dy2 = yi - py[q], dz2 = zi - pz[q];
                        const bool take = (sl < s1) & (sl != own) &
                                          (dx * dx + dy2 * dy2 + dz2 * dz2 < a.rl2);
                        // past max_nbr entries land in the last column (the
                        // count still grows and flags the overflow)
                        if (take) col[off] = uint16_t(sl * 8);
                        cnt += take ? 1 : 0;
                        off = take ? min(off + uint32_t(a.ld), lastoff) : off;
                    }
                }
            }
            a.count[i] = cnt;
            if (cnt > a.max_nbr) {
                if (a.status) atomicOr(a.status, MD_F_NBR_OVERFLOW);
                if (a.need) atomicMax(a.need, cnt);
            } else {
                // pad to a multiple of 16 entries (max_nbr is one) with the
                // pad slot, so force loops need no tail mask
                const int padded = (cnt + 15) & ~15;
                for (int k = cnt; k < padded; ++k) col[size_t(k) * a.ld] = uint16_t(CAP * 8);
            }
        }
        __syncthreads();
    }
}

template <class SH, int PREC, int U, bool P4>
__global__ __launch_bounds__(SH::TB) void k_tile_lj(TileArgs a)
{
    constexpr int TB = SH::TB, CAP = SH::CAP;
    __shared__ TileStage<CAP, SH::MAXC> st;
    __shared__ double red[TB / kWave];
    const int t = xcd_swizzle(blockIdx.x, gridDim.x);
    const TileSpec s = tile_spec(t, a.tile_rep, a.tile_off, a.ncell, a.cell_off, a.box, a.g);
    const PolyConst pc = poly_const(a.eps[0], a.sig[0], a.rc, a.shift);
    const double rc2 = a.rc * a.rc;
    const int total = stage_tile<TB, P4>(s, a.cell_start, a.x, a.y, a.z, a.pos4, st, CAP);
    double e_acc = 0.0, w_acc = 0.0;
    if (total > CAP) {
        if (threadIdx.x == 0 && a.status) atomicOr(a.status, MD_F_TILE_OVERFLOW);
    } else {
        const int nh = st.home_start[s.hy * s.hz];
        const char *stb = reinterpret_cast<const char *>(st.x);
        constexpr int kY = int(sizeof(double)) * decltype(st)::kStride;
        for (int hk = threadIdx.x; hk < nh; hk += TB) {
            int dy, dz;
            const int i = home_atom(s, st, hk, dy, dz);
            const double xi = a.x[i], yi = a.y[i], zi = a.z[i];
            const int n = min(a.count[i], a.max_nbr);
            Acc c{0.0, 0.0, 0.0, 0.0, 0.0, 0.0f, 0.0f};
            // Entries are LDS byte offsets, consumed U at a time while the
            // next U are in flight; a list is padded with the pad slot to a
            // multiple of 16 entries, so no entry needs a mask.  Column
            // reads stay inside the allocation (index clamped to
            // max_nbr - 1) and LDS reads inside the staging planes (offset
            // clamped to the pad slot).
            const int kmax = a.max_nbr - 1;
            const unsigned ui = unsigned(i);
            int cur[U], nxt[U];
#pragma unroll
            for (int q = 0; q < U; ++q)
                cur[q] = __builtin_nontemporal_load(a.idx + size_t(min(q, kmax)) * a.ld + ui);
            for (int k = 0; k < n; k += U) {
#pragma unroll
                for (int q = 0; q < U; ++q)
                    nxt[q] = __builtin_nontemporal_load(
                        a.idx + size_t(min(k + U + q, kmax)) * a.ld + ui);
                // all U staged positions are read before any is used
                double px[U], py[U], pz[U];
#pragma unroll
                for (int q = 0; q < U; ++q) {
                    const char *pq = stb + min(unsigned(cur[q]), unsigned(CAP * 8));
                    px[q] = *reinterpret_cast<const double *>(pq);
                    py[q] = *reinterpret_cast<const double *>(pq + kY);
                    pz[q] = *reinterpret_cast<const double *>(pq + 2 * kY);
                }
#pragma unroll
                for (int q = 0; q < U; ++q)
                    lj_pair_masked<PREC>(pc, xi - px[q], yi - py[q], zi - pz[q], rc2, c);
#pragma unroll
                for (int q = 0; q < U; ++q) cur[q] = nxt[q];
            }
            double ed = c.ed, wd = c.wd;
            if (PREC != MD_FP64) {
                ed = static_cast<double>(c.ef);
                wd = static_cast<double>(c.wf);
            }
            e_acc += 0.5 * ed;
            w_acc += 0.5 * wd;
            if (a.accumulate) {
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
    }
    const double es = block_sum_t<TB>(e_acc, red);
    const double ws = block_sum_t<TB>(w_acc, red);
    if (threadIdx.x == 0) {
        a.tpart[size_t(t) * 2 + 0] = es;
        a.tpart[size_t(t) * 2 + 1] = ws;
    }
}

// Per replica: fixed-order sums of its tiles' partials.
__global__ __launch_bounds__(kUnit) void k_tile_finalize(const int32_t *tile_off,
                                                         const double *tpart, double *energy,
                                                         double *virial)
{
    __shared__ double red[kWavesPerUnit];
    const int r = blockIdx.x;
    double s0 = 0.0, s1 = 0.0;
    for (int t = tile_off[r] + threadIdx.x; t < tile_off[r + 1]; t += kUnit) {
        s0 += tpart[size_t(t) * 2];
        s1 += tpart[size_t(t) * 2 + 1];
    }
    s0 = block_sum(s0, red);
    s1 = block_sum(s1, red);
    if (threadIdx.x == 0) {
        if (energy) energy[r] = s0;
        if (virial) virial[r] = s1;
    }
}

TileArgs tile_args(const md_batch *b, const md_atoms *atoms, const md_nlist *nl)
{
    TileArgs a{};
    a.tile_rep = nl->tile_rep;
    a.tile_off = nl->tile_off;
    a.ncell = b->ncell;
    a.cell_off = b->cell_off;
    a.box = b->box;
    a.x = atoms->x;
    a.y = atoms->y;
    a.z = atoms->z;
    a.pos4 = atoms->pos4;
    a.g = TileGrid{nl->tile_cells, nl->tile_py, nl->tile_pz};
    a.n_tiles = nl->n_tiles;
    a.max_nbr = nl->max_nbr;
    a.ld = nl->ld;
    a.count = nl->count;
    a.idx = reinterpret_cast<uint16_t *>(nl->idx);
    a.tile_need = nl->tile_need;
    a.R = b->R;
    return a;
}

}  // namespace

bool tile_stage_packed() { return md_tune_get(MD_TUNE_TILE_STAGE_PACKED) != 0; }

bool tile_list_ok(const md_batch *b, const md_nlist *nl)
{
    return nl->n_tiles >= 1 && nl->n_tiles <= b->C && nl->tile_rep && nl->tile_off &&
           nl->max_nbr % 16 == 0 &&
           nl->tile_cells >= 1 && nl->tile_cells <= tile_max_cells() && nl->tile_py >= 1 &&
           nl->tile_py <= MD_TILE_MAX_ROWS && nl->tile_pz >= 1 && nl->tile_pz <= MD_TILE_MAX_ROWS;
}

int tile_threads() { return md_tune_get(MD_TUNE_TILE_THREADS); }

namespace {

// Calls f with the shape selected by MD_TUNE_TILE_THREADS and
// MD_TUNE_TILE_SLOTS: the largest capacity of that workgroup size not above
// the requested slot count (0: the largest there is).
template <class F>
void with_tile_shape(F &&f)
{
    const int slots = md_tune_get(MD_TUNE_TILE_SLOTS);
    switch (tile_threads()) {
    case 64: f(TileShape64{}); break;
    case 128: f(TileShape128{}); break;
    default:
        if (slots == 0 || slots >= TileShape256::CAP) f(TileShape256{});
        else if (slots >= TileShape256S2048::CAP) f(TileShape256S2048{});
        else f(TileShape256S1536{});
    }
}

}  // namespace

int tile_capacity()
{
    int cap = 0;
    with_tile_shape([&](auto sh) { cap = decltype(sh)::CAP; });
    return cap;
}

int tile_max_cells()
{
    int mc = 0;
    with_tile_shape([&](auto sh) { mc = decltype(sh)::MAXC; });
    return mc;
}

int tile_build(const md_batch *b, const md_atoms *atoms, const int32_t *cell_start, double rl2,
               const md_nlist *nl, int32_t *need, const uint32_t *gate, uint32_t *status,
               hipStream_t s)
{
    TileArgs a = tile_args(b, atoms, nl);
    a.gate = gate;
    a.cell_start = cell_start;
    a.rl2 = rl2;
    a.need = need;
    a.status = status;
    const dim3 grid(gated_grid(nl->n_tiles, gate != nullptr));
    const bool p4 = tile_stage_packed() && atoms->pos4;
    with_tile_shape([&](auto sh) {
        using SH = decltype(sh);
        if (p4) hipLaunchKernelGGL((k_tile_build<SH, true>), grid, dim3(SH::TB), 0, s, a);
        else hipLaunchKernelGGL((k_tile_build<SH, false>), grid, dim3(SH::TB), 0, s, a);
    });
    return launch_status();
}

int tile_forces(const md_batch *b, const md_atoms *atoms, const md_nlist *nl, const md_lj *p,
                int32_t prec, int32_t accumulate, const int32_t *cell_start, double *energy,
                double *virial, double *tpart, int batch, uint32_t *status, hipStream_t s)
{
    TileArgs a = tile_args(b, atoms, nl);
    a.cell_start = cell_start;
    a.eps = p->eps;
    a.sig = p->sig;
    a.shift = p->shift;
    a.rc = p->rc;
    a.fx = atoms->fx;
    a.fy = atoms->fy;
    a.fz = atoms->fz;
    a.accumulate = accumulate;
    a.tpart = tpart;
    a.status = status;
    const dim3 grid(nl->n_tiles);
    const bool p4 = tile_stage_packed() && atoms->pos4;
    const bool big = batch >= 8;
    with_tile_shape([&](auto sh) {
        using SH = decltype(sh);
        const dim3 blk(SH::TB);
#define MD_TILE_LAUNCH(P, U)                                                          \
    do {                                                                              \
        if (p4) hipLaunchKernelGGL((k_tile_lj<SH, P, U, true>), grid, blk, 0, s, a);  \
        else hipLaunchKernelGGL((k_tile_lj<SH, P, U, false>), grid, blk, 0, s, a);    \
    } while (0)
        if (prec == MD_FP64) {
            if (big) MD_TILE_LAUNCH(MD_FP64, 16);
            else MD_TILE_LAUNCH(MD_FP64, 8);
        } else {
            if (big) MD_TILE_LAUNCH(MD_FP32_MIXED, 16);
            else MD_TILE_LAUNCH(MD_FP32_MIXED, 8);
        }
#undef MD_TILE_LAUNCH
    });
    if (energy || virial)
        hipLaunchKernelGGL(k_tile_finalize, dim3(b->R), dim3(kUnit), 0, s, nl->tile_off, tpart,
                           energy, virial);
    return launch_status();
}

}  // namespace md

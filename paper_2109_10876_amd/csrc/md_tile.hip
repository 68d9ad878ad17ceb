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
    const int32_t *type;
    int32_t tile_types;   // > 1: list entries carry the neighbour's type
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
    double *tpart;    // [n_tiles * kTilePartials]
    VVFuse vv;        // FUSE variant only
    uint32_t *status;
    int32_t R;
};

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Tiles go to the XCDs in chunks of this many consecutive tiles.
constexpr int kTileXcdChunk = 16;

// Tile-list builds form column byte offsets with 24-bit multiplies (and the
// whole list must span less than 4 GiB).
constexpr int kTileMaxLd = 1 << 23;
// Home cells with at most kFlatChunks x 64 stencil candidates take the
// register path (a multiple of 3: chunks are tested three at a time).
constexpr int kFlatChunks = 12;

// Lanes 0 .. nb-1 of a wavefront hold the entry counts of home atoms
// hb .. hb+nb-1: store them, flag overflow, or pad each column to a multiple
// of 16 entries (max_nbr is one) with the pad slot, so force loops need no
// tail mask.
__device__ __forceinline__ void tile_finish_counts(const TileArgs &a, int hb, int nb, int lane,
                                                   int vcnt, int cap)
{
    if (lane >= nb) return;
    const int i = hb + lane;
    a.count[i] = vcnt;
    if (vcnt > a.max_nbr) {
        if (a.status) atomicOr(a.status, MD_F_NBR_OVERFLOW);
        if (a.need) atomicMax(a.need, vcnt);
        return;
    }
    const int padded = (vcnt + 15) & ~15;
    for (int k = vcnt; k < padded; ++k) a.idx[size_t(k) * a.ld + i] = uint16_t(cap * 8);
}

// List build, one wavefront per home cell.  The lanes hold up to 64 staged
// candidates of one stencil row (nine contiguous slot ranges, one per row of
// the cell's 27-cell stencil) and the wave visits the cell's home atoms in
// turn, so every lane runs the same loop.  A home atom's hits are placed by
// a ballot and the count of hitting lanes below each lane: entries come out
// in stencil-row order, then ascending slot.  Per-atom counts live one per
// lane of a batch of up to 64 home atoms.
template <class SH, bool P4>
__global__ __launch_bounds__(SH::TB) __attribute__((amdgpu_waves_per_eu(3))) void k_tile_build(
    TileArgs a)
{
    constexpr int TB = SH::TB, CAP = SH::CAP;
    constexpr int kWaves = TB / kWave;
    __shared__ TileStage<CAP, SH::MAXC> st;
    if (sole_replica_gated_off(a.gate, a.R)) return;
    const int lane = __lane_id();
    const int wid = uniform(threadIdx.x / kWave);
    for (int lt = blockIdx.x; lt < a.n_tiles; lt += gridDim.x) {
        const int t = xcd_chunked(lt, a.n_tiles, kTileXcdChunk);
        const TileSpec s = tile_spec(t, a.tile_rep, a.tile_off, a.ncell, a.cell_off, a.box, a.g);
        if (a.gate != nullptr && a.gate[s.rep] == 0u) continue;
        if (tile_home_atoms(s, a.cell_start) == 0) continue;
        const int total = stage_tile<TB, P4>(s, a.cell_start, a.x, a.y, a.z, a.pos4, st, CAP);
        if (total > CAP) {
            if (threadIdx.x == 0) {
                if (a.status) atomicOr(a.status, MD_F_TILE_OVERFLOW);
                if (a.tile_need) atomicMax(a.tile_need, total);
            }
            __syncthreads();
            continue;
        }
        const int ncx = s.b - s.a + 1;
        const int nhc = ncx * s.hy * s.hz;
        for (int hc = wid; hc < nhc; hc += kWaves) {
            const int kc = hc % ncx, hrow = hc / ncx;   // kc: stage index of cell cx - 1
            const int dy = hrow % s.hy, dz = hrow / s.hy;
            const int qc = staged_row(s, dy, dz);
            const int cell = uniform(st.row_rb[qc]) + s.a + kc;
            const int g0 = uniform(a.cell_start[cell]), g1 = uniform(a.cell_start[cell + 1]);
            const int own0 = uniform(st.row_slot[qc] + st.cslot[qc][kc + 1]);
            const size_t ld2 = size_t(a.ld) * sizeof(uint16_t);
            // The nine stencil rows of this home cell: first slot, length.
            int rs0[9], rlen[9];
#pragma unroll
            for (int r9 = 0; r9 < 9; ++r9) {
                const int r = staged_row(s, dy + r9 % 3 - 1, dz + r9 / 3 - 1);
                rs0[r9] = uniform(st.row_slot[r] + st.cslot[r][kc]);
                rlen[r9] = uniform(st.row_slot[r] + st.cslot[r][kc + 3]) - rs0[r9];
            }
            // The nine rows concatenated in stencil order form the cell's
            // candidate sequence; flat index f of row q maps to slot
            // rs0[q] + f - pref[q].
            int pref[9];
            int T = 0;
#pragma unroll
            for (int r9 = 0; r9 < 9; ++r9) {
                pref[r9] = T;
                T += rlen[r9];
            }
            if (T <= kFlatChunks * kWave) {
                // Fast path: chunk c of the sequence (flat 64 c + lane) sits
                // in registers; each home atom tests the chunks in groups of
                // three with no branch inside a group, so the scheduler can
                // interleave them; the home atom's count is a scalar.
                double px[kFlatChunks], py[kFlatChunks], pz[kFlatChunks];
                int ent[kFlatChunks];
#pragma unroll
                for (int c = 0; c < kFlatChunks; ++c) {
                    const int f = min(c * kWave + lane, T - 1);
                    int slot = rs0[0] + f;
#pragma unroll
                    for (int q = 1; q < 9; ++q)
                        slot += f >= pref[q] ? rs0[q] - rs0[q - 1] - rlen[q - 1] : 0;
                    px[c] = st.x[slot];
                    py[c] = st.y[slot];
                    pz[c] = st.z[slot];
                    ent[c] = slot * 8;
                    if (a.tile_types > 1) {
                        int row;
                        double sx;
                        ent[c] |= a.type[slot_source(s, st, slot, row, sx)];
                    }
                }
                const int nch = (T + kWave - 1) / kWave;
                const unsigned ld2u = unsigned(ld2);
                for (int hb = g0; hb < g1; hb += kWave) {
                    const int nb = min(kWave, g1 - hb);
                    int vcnt = 0;   // lane j: entries of home atom hb + j
                    for (int j = 0; j < nb; ++j) {
                        const int hs = own0 + (hb - g0) + j;
                        const double hx = st.x[hs], hy = st.y[hs], hz = st.z[hs];
                        const int fown = pref[4] + (hs - rs0[4]);   // own slot in the sequence
                        char *col = reinterpret_cast<char *>(a.idx + (hb + j));
                        int cnt = 0;
#pragma unroll
                        for (int g = 0; g < kFlatChunks; g += 3) {
                            if (g >= nch) break;
#pragma unroll
                            for (int c = g; c < g + 3; ++c) {
                                const int left = T - c * kWave;   // valid lanes of chunk c
                                const uint64_t vm = left >= kWave ? ~uint64_t(0)
                                                    : (left <= 0 ? 0 : (uint64_t(1) << left) - 1);
                                const int lown = fown - c * kWave;   // own lane if in [0, 64)
                                const uint64_t om = (lown >= 0 && lown < kWave)
                                                        ? ~(uint64_t(1) << lown) : ~uint64_t(0);
                                const double dx = hx - px[c], dyy = hy - py[c], dzz = hz - pz[c];
                                const bool near = dx * dx + dyy * dyy + dzz * dzz < a.rl2;
                                const uint64_t m = __builtin_amdgcn_ballot_w64(near) & vm & om;
                                const int k = cnt + int(__builtin_amdgcn_mbcnt_hi(
                                                        uint32_t(m >> 32),
                                                        __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u)));
                                // past max_nbr entries are not stored (the
                                // count still grows and flags the overflow)
                                if (near && lane < left && lane != lown && k < a.max_nbr)
                                    *reinterpret_cast<uint16_t *>(
                                        col + size_t(unsigned(__umul24(unsigned(k), ld2u)))) =
                                        uint16_t(ent[c]);
                                cnt += int(__popcll(m));
                            }
                        }
                        vcnt = lane == j ? cnt : vcnt;
                    }
                    tile_finish_counts(a, hb, nb, lane, vcnt, CAP);
                }
                continue;
            }
            for (int hb = g0; hb < g1; hb += kWave) {
                const int nb = min(kWave, g1 - hb);
                int vcnt = 0;   // lane j: entries of home atom hb + j so far
                for (int r9 = 0; r9 < 9; ++r9) {
                    const int s0 = rs0[r9], s1 = rs0[r9] + rlen[r9];
                    for (int cb = s0; cb < s1; cb += kWave) {
                        const int sl = cb + lane;
                        const bool valid = sl < s1;
                        const int sc = valid ? sl : s1 - 1;
                        const double px = st.x[sc], py = st.y[sc], pz = st.z[sc];
                        int ty = 0;
                        if (a.tile_types > 1) {
                            int row;
                            double sx;
                            ty = a.type[slot_source(s, st, sc, row, sx)];
                        }
                        const uint16_t ent = uint16_t(sl * 8 + ty);
                        for (int j = 0; j < nb; ++j) {
                            const int hs = own0 + (hb - g0) + j;   // the home atom's own slot
                            const double dx = st.x[hs] - px, dyy = st.y[hs] - py,
                                         dzz = st.z[hs] - pz;
                            const bool take = valid & (sl != hs) &
                                              (dx * dx + dyy * dyy + dzz * dzz < a.rl2);
                            const uint64_t m = __builtin_amdgcn_ballot_w64(take);
                            const int cnt = __builtin_amdgcn_readlane(vcnt, j);
                            const int k = cnt + int(__builtin_amdgcn_mbcnt_hi(
                                                    uint32_t(m >> 32),
                                                    __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u)));
                            if (take && k < a.max_nbr) {
                                char *col = reinterpret_cast<char *>(a.idx + (hb + j));
                                *reinterpret_cast<uint16_t *>(col + size_t(unsigned(k)) * ld2) = ent;
                            }
                            vcnt = lane == j ? cnt + int(__popcll(m)) : vcnt;
                        }
                    }
                }
                tile_finish_counts(a, hb, nb, lane, vcnt, CAP);
            }
        }
        __syncthreads();
    }
}

// Typed lists: LJ constants of type pair (ti, tj) at ti * kTileMaxTypes + tj.
constexpr int kTileMaxTypes = MD_TILE_MAX_TYPES;

template <class SH, int PREC, int U, bool P4, bool TYPED, bool FUSE>
__global__ __launch_bounds__(SH::TB) void k_tile_lj(TileArgs a)
{
    constexpr int TB = SH::TB, CAP = SH::CAP;
    __shared__ TileStage<CAP, SH::MAXC> st;
    __shared__ double red[TB / kWave];
    __shared__ PolyConst ptab[TYPED ? kTileMaxTypes * kTileMaxTypes : 1];
    const int t = xcd_chunked(blockIdx.x, gridDim.x, kTileXcdChunk);
    const TileSpec s = tile_spec(t, a.tile_rep, a.tile_off, a.ncell, a.cell_off, a.box, a.g);
    if (tile_home_atoms(s, a.cell_start) == 0) {
        if (threadIdx.x < kTilePartials) a.tpart[size_t(t) * kTilePartials + threadIdx.x] = 0.0;
        return;
    }
    const PolyConst pc = poly_const(a.eps[0], a.sig[0], a.rc, a.shift);
    const double rc2 = a.rc * a.rc;
    if (TYPED) {
        // filled before staging, whose barriers publish it
        const int nt = a.tile_types;
        if (threadIdx.x < nt * nt) {
            const int ti = threadIdx.x / nt, tj = threadIdx.x % nt;
            ptab[ti * kTileMaxTypes + tj] = poly_const(a.eps[threadIdx.x], a.sig[threadIdx.x], a.rc,
                                                       a.shift);
        }
    }
    const int total = stage_tile<TB, P4>(s, a.cell_start, a.x, a.y, a.z, a.pos4, st, CAP);
    double e_acc = 0.0, w_acc = 0.0, ke_acc = 0.0, d2_max = 0.0;
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
            const int ti4 = TYPED ? a.type[i] * kTileMaxTypes : 0;
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
                    // typed entries carry the type in the low 3 bits
                    const unsigned e = TYPED ? unsigned(cur[q]) & ~7u : unsigned(cur[q]);
                    const char *pq = stb + min(e, unsigned(CAP * 8));
                    px[q] = *reinterpret_cast<const double *>(pq);
                    py[q] = *reinterpret_cast<const double *>(pq + kY);
                    pz[q] = *reinterpret_cast<const double *>(pq + 2 * kY);
                }
#pragma unroll
                for (int q = 0; q < U; ++q)
                    lj_pair_masked<PREC>(TYPED ? ptab[ti4 + (cur[q] & 7)] : pc, xi - px[q],
                                         yi - py[q], zi - pz[q], rc2, c);
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
            if (FUSE) {
                // md_vv_step phase 3 on this atom with the force just computed
                const VVFuse &f = a.vv;
                const double im = f.inv_mass[f.ntypes > 1 ? a.type[i] : 0];
                const double k = f.hdt * im;
                double vx = f.vx[i], vy = f.vy[i], vz = f.vz[i];
                vx = fma(k, c.fx, vx);
                vy = fma(k, c.fy, vy);
                vz = fma(k, c.fz, vz);
                ke_acc += 0.5 * (vx * vx + vy * vy + vz * vz) / im;
                vx = fma(k, c.fx, vx);
                vy = fma(k, c.fy, vy);
                vz = fma(k, c.fz, vz);
                const double x = fma(f.dt, vx, xi);
                const double y = fma(f.dt, vy, yi);
                const double z = fma(f.dt, vz, zi);
                f.xn[i] = x;
                f.yn[i] = y;
                f.zn[i] = z;
                const double ex = x - f.xb[i], ey = y - f.yb[i], ez = z - f.zb[i];
                d2_max = fmax(d2_max, ex * ex + ey * ey + ez * ez);
                f.vx[i] = vx;
                f.vy[i] = vy;
                f.vz[i] = vz;
            }
        }
    }
    const double es = block_sum_n<TB>(e_acc, red);
    const double ws = block_sum_n<TB>(w_acc, red);
    double ks = 0.0, dm = 0.0;
    if (FUSE) {
        ks = block_sum_n<TB>(ke_acc, red);
        dm = block_max_n<TB>(d2_max, red);
    }
    if (threadIdx.x == 0) {
        double *tp = a.tpart + size_t(t) * kTilePartials;
        tp[0] = es;
        tp[1] = ws;
        tp[2] = ks;
        tp[3] = dm;
    }
}

// Next positions of the fused call back into the position planes (and the
// packed copy when present).
__global__ __launch_bounds__(kUnit) void k_copy_next(int32_t n, const double *__restrict__ xn,
                                                     const double *__restrict__ yn,
                                                     const double *__restrict__ zn, double *x,
                                                     double *y, double *z, double *pos4)
{
    const int i = blockIdx.x * kUnit + threadIdx.x;
    if (i >= n) return;
    const double xv = xn[i], yv = yn[i], zv = zn[i];
    x[i] = xv;
    y[i] = yv;
    z[i] = zv;
    if (pos4) reinterpret_cast<double4 *>(pos4)[i] = make_double4(xv, yv, zv, 0.0);
}

// Per replica: fixed-order sums of its tiles' partials (energy, virial,
// kinetic energy) and the largest displacement (the rebuild gate).
__global__ __launch_bounds__(kFin) void k_tile_finalize(const int32_t *tile_off,
                                                        const double *tpart, double *energy,
                                                        double *virial, double *ke,
                                                        uint32_t *gate, double lim2)
{
    __shared__ double red[kFin / kWave];
    const int r = blockIdx.x;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, m = 0.0;
#pragma unroll 4
    for (int t = tile_off[r] + threadIdx.x; t < tile_off[r + 1]; t += kFin) {
        const double *tp = tpart + size_t(t) * kTilePartials;
        s0 += tp[0];
        s1 += tp[1];
        if (ke) s2 += tp[2];
        if (gate) m = fmax(m, tp[3]);
    }
    s0 = block_sum_n<kFin>(s0, red);
    s1 = block_sum_n<kFin>(s1, red);
    if (ke) s2 = block_sum_n<kFin>(s2, red);
    if (gate) m = block_max_n<kFin>(m, red);
    if (threadIdx.x == 0) {
        if (energy) energy[r] = s0;
        if (virial) virial[r] = s1;
        if (ke) ke[r] = s2;
        if (gate) gate[r] = m > lim2 ? 1u : 0u;
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
    a.type = atoms->type;
    a.tile_types = nl->tile_types;
    return a;
}

}  // namespace

bool tile_stage_packed() { return md_tune_get(MD_TUNE_TILE_STAGE_PACKED) != 0; }

bool tile_list_ok(const md_batch *b, const md_nlist *nl)
{
    return nl->n_tiles >= 1 && nl->n_tiles <= b->C && nl->tile_rep && nl->tile_off &&
           nl->max_nbr % 16 == 0 && nl->ld <= kTileMaxLd && nl->tile_types >= 0 &&
           nl->tile_types <= MD_TILE_MAX_TYPES &&
           size_t(nl->max_nbr) * size_t(nl->ld) * 2 < (size_t(1) << 32) &&
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
                double *virial, double *tpart, int batch, const VVFuse *vvf, uint32_t *status,
                hipStream_t s)
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
    if (vvf) a.vv = *vvf;
    a.status = status;
    const dim3 grid(nl->n_tiles);
    const bool p4 = tile_stage_packed() && atoms->pos4;
    const bool big = batch >= 8;
    const bool typed = p->ntypes > 1;
    const bool fuse = vvf != nullptr;
    with_tile_shape([&](auto sh) {
        using SH = decltype(sh);
        const dim3 blk(SH::TB);
#define MD_TILE_LAUNCH(P, U, T, F)                                                          \
    do {                                                                                    \
        if (p4) hipLaunchKernelGGL((k_tile_lj<SH, P, U, true, T, F>), grid, blk, 0, s, a);  \
        else hipLaunchKernelGGL((k_tile_lj<SH, P, U, false, T, F>), grid, blk, 0, s, a);    \
    } while (0)
        if (fuse) {
            if (prec == MD_FP64) MD_TILE_LAUNCH(MD_FP64, 8, false, true);
            else MD_TILE_LAUNCH(MD_FP32_MIXED, 8, false, true);
        } else if (typed) {
            if (prec == MD_FP64) MD_TILE_LAUNCH(MD_FP64, 8, true, false);
            else MD_TILE_LAUNCH(MD_FP32_MIXED, 8, true, false);
        } else if (prec == MD_FP64) {
            if (big) MD_TILE_LAUNCH(MD_FP64, 16, false, false);
            else MD_TILE_LAUNCH(MD_FP64, 8, false, false);
        } else {
            if (big) MD_TILE_LAUNCH(MD_FP32_MIXED, 16, false, false);
            else MD_TILE_LAUNCH(MD_FP32_MIXED, 8, false, false);
        }
#undef MD_TILE_LAUNCH
    });
    double *ke = fuse ? vvf->ke : nullptr;
    uint32_t *gate = fuse ? vvf->gate : nullptr;
    if (energy || virial || ke || gate)
        hipLaunchKernelGGL(k_tile_finalize, dim3(b->R), dim3(kFin), 0, s, nl->tile_off, tpart,
                           energy, virial, ke, gate, fuse ? vvf->lim2 : 0.0);
    if (fuse)
        hipLaunchKernelGGL(k_copy_next, dim3((b->N + kUnit - 1) / kUnit), dim3(kUnit), 0, s, b->N,
                           vvf->xn, vvf->yn, vvf->zn, atoms->x, atoms->y, atoms->z, atoms->pos4);
    return launch_status();
}

}  // namespace md

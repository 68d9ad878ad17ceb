// md_tile.hpp -- tile geometry and LDS staging shared by the tile-local list
// build and the tile-local force kernel (MD_TILE_FULL).
//
// A tile is a block of cells: x in a..b (at most m cells), y in y0..y1 and
// z in z0..z1 (at most py and pz rows).  Every pair partner of its atoms lies
// in the 27-cell stencil of some home cell, i.e. in the staged rows
// (y0-1..y1+1) x (z0-1..z1+1), each over unwrapped x = a-1 .. b+1.  That
// region is staged into LDS once per workgroup with each cell's periodic
// image already applied, so neighbour positions come from LDS instead of L2
// gathers and the list names neighbours by a 16-bit staged slot.
#pragma once

#include <climits>

#include "md_common.hpp"

namespace md {

constexpr int kTileCells = MD_TILE_MAX_CELLS;
constexpr int kMaxHomeRows = MD_TILE_MAX_ROWS * MD_TILE_MAX_ROWS;             // py pz
constexpr int kMaxStagedRows = (MD_TILE_MAX_ROWS + 2) * (MD_TILE_MAX_ROWS + 2);

// Workgroup shapes of the tile kernels: TB threads (at most TB home atoms per
// pass), CAP staged slots (3 x 8 CAP bytes of LDS), MAXC cells per tile
// along x.  LDS per workgroup bounds how many workgroups share a CU (160 KiB
// each; measured on MI355X: three workgroups of up to 53,760 bytes, four of
// up to 40,960): the force kernel of the 3072-slot shape fits two, of the
// 2048-slot shape three and of the 1536-slot shape four.
template <int TB_, int CAP_, int MAXC_>
struct TileShape {
    static constexpr int TB = TB_, CAP = CAP_, MAXC = MAXC_;
};
using TileShape64 = TileShape<64, 1024, 8>;
using TileShape128 = TileShape<128, 1792, 16>;
using TileShape256 = TileShape<256, 3072, kTileCells>;
using TileShape256S2048 = TileShape<256, 2048, 16>;
using TileShape256S1536 = TileShape<256, 1536, 8>;
static_assert(TileShape256::CAP == MD_TILE_SLOTS, "largest shape holds MD_TILE_SLOTS");

struct TileSpec {
    int rep, nx, ny, nz, coff;
    int a, b;        // home cells along x
    int y0, hy;      // home rows y0 .. y0 + hy - 1
    int z0, hz;      // home layers z0 .. z0 + hz - 1
    int nrows;       // staged rows (hy + 2)(hz + 2)
    double L[3];
};

struct TileGrid {
    int m, py, pz;
};

__device__ __forceinline__ TileSpec tile_spec(int t, const int32_t *__restrict__ tile_rep,
                                              const int32_t *__restrict__ tile_off,
                                              const int32_t *__restrict__ ncell,
                                              const int32_t *__restrict__ cell_off,
                                              const double *__restrict__ box, TileGrid g,
                                              const int32_t *__restrict__ tile_m)
{
    TileSpec s;
    s.rep = tile_rep[t];
    s.nx = ncell[3 * s.rep];
    s.ny = ncell[3 * s.rep + 1];
    s.nz = ncell[3 * s.rep + 2];
    s.coff = cell_off[s.rep];
    // the replica's cells per tile along x (never above g.m, which sizes the
    // LDS tables)
    const int m = tile_m ? min(max(tile_m[s.rep], 1), g.m) : g.m;
    const int local = t - tile_off[s.rep];
    const int tx = (s.nx + m - 1) / m, ty = (s.ny + g.py - 1) / g.py;
    const int bx = local % tx, rest = local / tx;
    const int by = rest % ty, bz = rest / ty;
    s.a = bx * m;
    s.b = min(s.a + m, s.nx) - 1;
    s.y0 = by * g.py;
    s.hy = min(s.y0 + g.py, s.ny) - s.y0;
    s.z0 = bz * g.pz;
    s.hz = min(s.z0 + g.pz, s.nz) - s.z0;
    s.nrows = (s.hy + 2) * (s.hz + 2);
    s.L[0] = box[3 * s.rep];
    s.L[1] = box[3 * s.rep + 1];
    s.L[2] = box[3 * s.rep + 2];
    return s;
}

// LDS tables of one staged tile, as the list build stages it.  Positions of
// staged slot s sit at x[s], y[s], z[s]; slot CAP is the pad slot (a position
// far outside any box) that padded list entries name.  The build reads 64
// consecutive slots of one plane at a time, so the planes' distance does not
// matter for banks there: they sit one slot apart (kStride = CAP + 2, 16-byte
// aligned), which leaves room for the build's per-wave entry buffers at three
// workgroups per CU.
template <int CAP, int MAXC>
struct TileStage {
    static constexpr int kCap = CAP;
    static constexpr int kStride = CAP + 2;
    static constexpr int kRowStage = MAXC + 3;   // cell starts a-1 .. b+2 of one staged row
    double x[kStride], y[kStride], z[kStride];
    int row_slot[kMaxStagedRows + 1];  // first slot of staged row q; [nrows] = total
    int row_rb[kMaxStagedRows];        // linear index of cell (0, y, z) of staged row q
    int row_lo[kMaxStagedRows];        // first physical cell of the row's main piece
    int row_lw[kMaxStagedRows];        // atoms in the left wrap piece (cell nx-1 at x = -1)
    int row_main[kMaxStagedRows];      // atoms in the main piece
    int row_rw[kMaxStagedRows];        // atoms in the right wrap piece (cell 0 at x = nx)
    int row_g0[kMaxStagedRows][3];     // first atom index of the three pieces
    double row_dy[kMaxStagedRows], row_dz[kMaxStagedRows];  // shift of the row's image
    int cslot[kMaxStagedRows][kRowStage];  // start (within the row) of unwrapped cell a-1+k
    static constexpr int kChunks = CAP / 64 + 1;
    int rowc[kChunks];                 // staged row holding slot 64 c (first row if several)
};

// The position planes alone (same pad slot): all that the force kernel keeps
// in LDS, so that its workgroups use less of it.  The planes are kStride
// apart, one double more than a multiple of 64, so x, y and z of a slot sit in
// different LDS banks for the force loop's random slot reads (with a multiple
// of 64 all three share a bank, and the step was 1.6% slower mixed, 0.8% FP64).
template <int CAP>
struct TilePlanes {
    static constexpr int kCap = CAP;
    static constexpr int kStride = (CAP + 1 + 63) / 64 * 64 + 1;
    double x[kStride], y[kStride], z[kStride];
};

// Coordinate of the pad slot: every distance to it is far beyond any cutoff
// and its pair terms stay finite in single precision.
constexpr double kPadCoord = 1.0e15;

// Staged row of home row offsets (dy, dz) moved by (oy, oz) in -1..1.
__device__ __forceinline__ int staged_row(const TileSpec &s, int dy, int dz)
{
    return (dz + 1) * (s.hy + 2) + (dy + 1);
}

// Staging record of a tile, written by the list build for the force kernel:
// word sl (< staged count) holds slot sl's source atom in its low 26 bits
// and the image shift of x, y, z in two bits each, a signed two-bit number
// (0: none, 1: +L, 3: -L), so that a sign-extending field extract gives the
// multiple of L to add;
// word kTabTotal holds the staged count; words kTabAdj .. +63 hold the
// adjoint's per-tile (eps, sigma) sums (32 doubles).  tab_stride words per
// tile.
constexpr uint32_t kTabSrcMask = (1u << 26) - 1;
constexpr int kTabShiftX = 26, kTabShiftY = 28, kTabShiftZ = 30;
template <class Stage>
constexpr int kTabTotal = Stage::kCap;
template <class Stage>
constexpr int kTabAdj = Stage::kCap + 64;
constexpr int tab_stride(int cap) { return cap + 128; }

__device__ __forceinline__ uint32_t shift_code(double d)
{
    return d > 0.0 ? 1u : (d < 0.0 ? 3u : 0u);
}

// p + s L for the signed two-bit field of `code` at bit `at` (s in -1, 0, 1):
// s L is exact, so this equals p + L, p - L or p bit for bit.
__device__ __forceinline__ double apply_shift(double p, uint32_t code, int at, double L)
{
    const int sh = __builtin_amdgcn_sbfe(int(code), at, 2);
    return fma(static_cast<double>(sh), L, p);
}

// Element `i` of a device array whose byte size is below 4 GiB, addressed by
// a 32-bit byte offset (one shift and a scalar base per load).
template <class T>
__device__ __forceinline__ T load_at(const T *__restrict__ base, uint32_t i)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) +
                                        (i * uint32_t(sizeof(T))));
}

// Fills the staging tables and stages positions (x, y, z planes or the
// packed copy).  All TB threads of the workgroup must call it, after every
// reader of a previous tile's staging has passed a barrier.  Returns the
// total staged count (may exceed cap: then nothing is staged).
// Source atom of staged slot sl: its staged row (from the chunk table, then
// forward over rows that end inside the chunk), and the x image shift of the
// row piece it sits in.  Needs the row tables of stage_tile's second phase.
template <class Stage>
__device__ __forceinline__ int slot_source(const TileSpec &s, const Stage &st, int sl, int &row,
                                           double &sx)
{
    int r = st.rowc[sl >> 6];
    while (sl >= st.row_slot[r + 1]) ++r;
    const int off = sl - st.row_slot[r];
    const int lw = st.row_lw[r], mn = st.row_main[r];
    const int piece = off < lw ? 0 : (off < lw + mn ? 1 : 2);
    row = r;
    sx = piece == 0 ? -s.L[0] : (piece == 1 ? 0.0 : s.L[0]);
    return st.row_g0[r][piece] + off - (piece == 0 ? 0 : (piece == 1 ? lw : lw + mn));
}

template <int TB, bool P4, class Stage, class Mid>
__device__ int stage_tile(const TileSpec &s, const int32_t *__restrict__ cs,
                          const double *__restrict__ x, const double *__restrict__ y,
                          const double *__restrict__ z, const double *__restrict__ pos4,
                          Stage &st, int cap, uint32_t *tab, Mid &&mid)
{
    const int tid = threadIdx.x;
    const int nk = s.b - s.a + 4;       // cell starts a-1 .. b+2 per staged row
    const int nq = s.nrows * nk;
    const int lo = max(s.a - 1, 0), hi = min(s.b + 1, s.nx - 1);
    if (tid == TB - 1) {
        st.x[Stage::kCap] = kPadCoord;
        st.y[Stage::kCap] = kPadCoord;
        st.z[Stage::kCap] = kPadCoord;
    }
    // Phase 1, global loads only: every (row, cell) start, and per row the
    // bounds of its three pieces (left wrap, main run, right wrap).  All of
    // a thread's loads are issued before any is stored, with mid() in
    // between, so that a caller's own loads share their latency; mid()
    // returning false (uniformly) abandons the staging: the result is -1.
    constexpr int kP1 = (kMaxStagedRows * Stage::kRowStage + TB - 1) / TB;
    auto row_of = [&](int q, double &dy, double &dz) {
        const int zr = q / (s.hy + 2), yr = q % (s.hy + 2);
        int az = s.z0 - 1 + zr, ay = s.y0 - 1 + yr;
        dz = 0.0;
        dy = 0.0;
        // a row reached across a face holds atoms one box length away
        if (az < 0) { az += s.nz; dz = -s.L[2]; } else if (az >= s.nz) { az -= s.nz; dz = s.L[2]; }
        if (ay < 0) { ay += s.ny; dy = -s.L[1]; } else if (ay >= s.ny) { ay -= s.ny; dy = s.L[1]; }
        return s.coff + (az * s.ny + ay) * s.nx;
    };
    int cv[kP1], rv[kP1][6];
#pragma unroll
    for (int j = 0; j < kP1; ++j) {
        const int t = tid + j * TB;
        cv[j] = 0;
#pragma unroll
        for (int r = 0; r < 6; ++r) rv[j][r] = 0;
        if (t < nq) {
            const int q = t / nk, k = t % nk;
            double dy, dz;
            const int rb = row_of(q, dy, dz);
            const int xu = s.a - 1 + k;
            if (xu >= 0 && xu < s.nx) cv[j] = cs[rb + xu];
            if (k == 0) {
                rv[j][0] = cs[rb + s.nx - 1];
                rv[j][1] = cs[rb + s.nx];
                rv[j][2] = cs[rb];
                rv[j][3] = cs[rb + 1];
                rv[j][4] = cs[rb + lo];
                rv[j][5] = cs[rb + hi + 1];
            }
        }
    }
    if (!mid()) return -1;
#pragma unroll
    for (int j = 0; j < kP1; ++j) {
        const int t = tid + j * TB;
        if (t < nq) {
            const int q = t / nk, k = t % nk;
            st.cslot[q][k] = cv[j];
            if (k == 0) {
                double dy, dz;
                const int rb = row_of(q, dy, dz);
                const int c_last = rv[j][0], c_end = rv[j][1];
                const int c_first = rv[j][2], c_second = rv[j][3];
                const int m0 = rv[j][4], m1 = rv[j][5];
                st.row_rb[q] = rb;
                st.row_lo[q] = lo;
                st.row_lw[q] = s.a - 1 < 0 ? c_end - c_last : 0;
                st.row_main[q] = m1 - m0;
                st.row_rw[q] = s.b + 1 >= s.nx ? c_second - c_first : 0;
                st.row_g0[q][0] = c_last;
                st.row_g0[q][1] = m0;
                st.row_g0[q][2] = c_first;
                st.row_dy[q] = dy;
                st.row_dz[q] = dz;
            }
        }
    }
    __syncthreads();
    // Phase 2, LDS only: cell starts within the row; wave 0 scans the row
    // lengths into row starts (and the chunk -> row table) and the home
    // counts into home starts.
    for (int t = tid; t < nq; t += TB) {
        const int q = t / nk, k = t % nk, xu = s.a - 1 + k;
        const int lw = st.row_lw[q], mn = st.row_main[q];
        int off;
        if (xu < 0) off = 0;
        else if (xu < s.nx) off = lw + (st.cslot[q][k] - st.row_g0[q][1]);
        else if (xu == s.nx) off = lw + mn;
        else off = lw + mn + st.row_rw[q];
        st.cslot[q][k] = off;
    }
    if (tid < kWave) {
        const int len = tid < s.nrows ? st.row_lw[tid] + st.row_main[tid] + st.row_rw[tid] : 0;
        int pl = len;   // inclusive prefix sum over the lanes
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int ul = __shfl_up(pl, o, kWave);
            if (tid >= o) pl += ul;
        }
        if (tid < s.nrows) {
            const int start = pl - len;
            st.row_slot[tid] = start;
            if (tid == s.nrows - 1) st.row_slot[s.nrows] = pl;
            for (int c = (start + 63) >> 6; c * 64 < pl && c < Stage::kChunks; ++c) st.rowc[c] = tid;
        }
    }
    __syncthreads();
    const int total = st.row_slot[s.nrows];
    if (tab && tid == 0) tab[kTabTotal<Stage>] = uint32_t(total);
    if (total > cap) return total;
    if (total > 0) {
        // Slots tid, tid + TB, ...: first resolve every slot's source atom and
        // image shift (the row from the chunk table, then forward over rows
        // that end inside the chunk), then issue all loads together (lanes
        // past the end re-read the last slot's atom), then write LDS.
        constexpr int kPer = (Stage::kCap + TB - 1) / TB;
        int src[kPer], rowof[kPer];
        double sxk[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int sl = min(tid + k * TB, total - 1);
            src[k] = slot_source(s, st, sl, rowof[k], sxk[k]);
        }
        double px[kPer], py[kPer], pz[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            if (P4) {
                const double4 v = reinterpret_cast<const double4 *>(pos4)[src[k]];
                px[k] = v.x;
                py[k] = v.y;
                pz[k] = v.z;
            } else {
                px[k] = x[src[k]];
                py[k] = y[src[k]];
                pz[k] = z[src[k]];
            }
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int sl = tid + k * TB;
            if (sl < total) {
                const double dy = st.row_dy[rowof[k]], dz = st.row_dz[rowof[k]];
                st.x[sl] = px[k] + sxk[k];
                st.y[sl] = py[k] + dy;
                st.z[sl] = pz[k] + dz;
                if (tab)
                    tab[sl] = uint32_t(src[k]) | shift_code(sxk[k]) << kTabShiftX |
                              shift_code(dy) << kTabShiftY | shift_code(dz) << kTabShiftZ;
            }
        }
    }
    __syncthreads();
    return total;
}

// Stages a tile from the table its list build wrote (see kTabTotal): the
// staged count, then every slot's source atom and image shift, gathered as
// stage_tile does -- one round trip for the table, one for the positions,
// no cell-start reads and no per-slot source search.  mid() runs while the
// table loads are in flight (returning false abandons the staging: -1).
// Source indices are clamped below n_atoms, so a table that no build has
// written gathers garbage but stays in bounds.  lsrc (optional, LDS, cap
// entries) receives every staged slot's source atom.  extra gathers more
// per-slot data with the positions: extra.load(k, src) is called with the
// position loads of a thread's k-th slot, extra.store(k, sl) with its LDS
// stores (slots below the staged count only).
struct NoSlotExtra {
    __device__ void load(int, uint32_t) {}
    __device__ void store(int, int) {}
};

template <int TB, bool P4, class Stage, class Mid, class Extra = NoSlotExtra>
__device__ int stage_from_table(const TileSpec &s, const uint32_t *__restrict__ tab, int n_atoms,
                                const double *__restrict__ x, const double *__restrict__ y,
                                const double *__restrict__ z, const double *__restrict__ pos4,
                                Stage &st, int cap, int *lsrc, Mid &&mid, Extra &&extra = Extra{})
{
    constexpr int kPer = (Stage::kCap + TB - 1) / TB;
    const int tid = threadIdx.x;
    if (tid == TB - 1) {
        st.x[Stage::kCap] = kPadCoord;
        st.y[Stage::kCap] = kPadCoord;
        st.z[Stage::kCap] = kPadCoord;
    }
    const int total = int(tab[kTabTotal<Stage>]);
    const int nload = min(total, Stage::kCap);
    uint32_t code[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int sl = tid + k * TB;
        code[k] = sl < nload ? tab[sl] : 0u;
    }
    if (!mid()) return -1;
    if (total > cap) return total;
    double px[kPer], py[kPer], pz[kPer];
    const uint32_t last = uint32_t(n_atoms - 1);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const uint32_t src = min(code[k] & kTabSrcMask, last);
        if (lsrc) {
            const int sl = tid + k * TB;
            if (sl < total) lsrc[sl] = int(src);
        }
        if (P4) {
            const double4 v = load_at(reinterpret_cast<const double4 *>(pos4), src);
            px[k] = v.x;
            py[k] = v.y;
            pz[k] = v.z;
        } else {
            px[k] = load_at(x, src);
            py[k] = load_at(y, src);
            pz[k] = load_at(z, src);
        }
        extra.load(k, src);
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int sl = tid + k * TB;
        if (sl < total) {
            st.x[sl] = apply_shift(px[k], code[k], kTabShiftX, s.L[0]);
            st.y[sl] = apply_shift(py[k], code[k], kTabShiftY, s.L[1]);
            st.z[sl] = apply_shift(pz[k], code[k], kTabShiftZ, s.L[2]);
            extra.store(k, sl);
        }
    }
    __syncthreads();
    return total;
}

template <int TB, bool P4, class Stage>
__device__ int stage_tile(const TileSpec &s, const int32_t *__restrict__ cs,
                          const double *__restrict__ x, const double *__restrict__ y,
                          const double *__restrict__ z, const double *__restrict__ pos4,
                          Stage &st, int cap)
{
    return stage_tile<TB, P4>(s, cs, x, y, z, pos4, st, cap, nullptr, [] { return true; });
}

// Number of home atoms of the tile, from the cell starts of its home rows
// (uniform across the workgroup: scalar loads).  Empty tiles (vacuum in an
// inhomogeneous system) skip staging altogether.
__device__ __forceinline__ int tile_home_atoms(const TileSpec &s, const int32_t *__restrict__ cs)
{
    int n = 0;
    for (int h = 0; h < s.hy * s.hz; ++h) {
        const int rb = s.coff + ((s.z0 + h / s.hy) * s.ny + (s.y0 + h % s.hy)) * s.nx;
        n += cs[rb + s.b + 1] - cs[rb + s.a];
    }
    return n;
}

// The home rows of a tile (runs of consecutive atoms, one per home row, in
// row order), read from the cell starts alone so that a kernel can fetch its
// home atoms' inputs while the tile is being staged.
struct HomeRows {
    int g0[kMaxHomeRows], n[kMaxHomeRows];
    int rows, total;
};

__device__ __forceinline__ HomeRows home_rows(const TileSpec &s, const int32_t *__restrict__ cs)
{
    // every row's two loads are issued at once (rows past the tile's last
    // re-read it and count zero), so they cost one round trip
    HomeRows hr;
    hr.rows = s.hy * s.hz;
    hr.total = 0;
    int e[kMaxHomeRows];
#pragma unroll
    for (int h = 0; h < kMaxHomeRows; ++h) {
        const int hh = min(h, hr.rows - 1);
        const int rb = s.coff + ((s.z0 + hh / s.hy) * s.ny + (s.y0 + hh % s.hy)) * s.nx;
        hr.g0[h] = cs[rb + s.a];
        e[h] = cs[rb + s.b + 1];
    }
#pragma unroll
    for (int h = 0; h < kMaxHomeRows; ++h) {
        hr.n[h] = h < hr.rows ? e[h] - hr.g0[h] : 0;
        hr.total += hr.n[h];
    }
    return hr;
}

// Index of home atom number k (0 <= k < total) of the tile.
__device__ __forceinline__ int home_index(const HomeRows &hr, int k)
{
    int i = hr.g0[0] + k, base = 0;
#pragma unroll
    for (int h = 1; h < kMaxHomeRows; ++h) {
        base += hr.n[h - 1];
        i = k >= base && h < hr.rows ? hr.g0[h] + (k - base) : i;
    }
    return i;
}

// Arguments of the tile kernels (list build and forces).
struct TileArgs {
    const int32_t *tile_rep, *tile_off, *ncell, *cell_off;
    const int32_t *tile_m;   // per-replica cells per tile along x, or null
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
    uint32_t *tile_src;   // staging records, tab_stride(CAP) words per tile
    int32_t n_atoms;
    // adjoint
    const double *gfx, *gfy, *gfz, *gE;
    double *gx;
    double rc;
    double *fx, *fy, *fz;
    int32_t accumulate;
    double *tpart;    // [n_tiles * kTilePartials]
    VVFuse vv;        // FUSE variant only
    uint32_t *status;
    int32_t R;
    int32_t *active;  // occupied-tile list (md_nlist.tile_active) or null
    const int32_t *todo;   // list build: tiles to rebuild (count, tiles) or null
};

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Tiles go to the XCDs in chunks of this many consecutive tiles.
constexpr int kTileXcdChunk = 16;

// Tile-list builds form column byte offsets with 24-bit multiplies (and the
// whole list must span less than 4 GiB).
constexpr int kTileMaxLd = 1 << 23;

// Tile-local list layout: an atom's entries sit in blocks of 8 consecutive
// uint16 values and the blocks of consecutive atoms are adjacent, so entry k
// of atom i is the uint16 at (k / 8) 8 ld + 8 i + k % 8: one 16-byte load
// fetches 8 entries of an atom, and a wave of consecutive atoms reads one
// contiguous run.  Byte offset of that entry (below 4 GiB: the list is).
constexpr int kEntryBlock = 8;

__device__ __forceinline__ unsigned tile_entry_byte(int k, int i, int ld)
{
    return (unsigned(__umul24(unsigned(k) >> 3, unsigned(ld))) << 4) + (unsigned(i) << 4) +
           ((unsigned(k) & 7u) << 1);
}

inline TileArgs tile_args(const md_batch *b, const md_atoms *atoms, const md_nlist *nl)
{
    TileArgs a{};
    a.tile_rep = nl->tile_rep;
    a.tile_off = nl->tile_off;
    a.tile_m = nl->tile_m;
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
    a.tile_src = nl->tile_src;
    a.n_atoms = b->N;
    return a;
}

int tile_threads();

// Calls f with the shape selected by MD_TUNE_TILE_THREADS and
// MD_TUNE_TILE_SLOTS: the largest capacity of that workgroup size not above
// the requested slot count (0: the largest there is).
template <class F>
inline void with_tile_shape(F &&f)
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

}  // namespace md

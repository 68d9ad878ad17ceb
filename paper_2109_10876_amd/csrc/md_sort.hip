// md_sort.hip -- md_cell_sort: cell binning and re-sort of the SoA arrays.
//
// The paper's Resort step (Sec. 2.1.3) re-bins particles into cells; its
// SoA layout (Sec. 3.1) keeps each attribute in its own array.  Here the
// atoms themselves are reordered cell by cell, so a cell's atoms are a
// contiguous index range and neighbour gathers in the list build and the
// force loop hit nearby addresses.
//
// Four stream-ordered kernels, each skipping replicas whose gate is 0:
//   1 bin      wrap, cell index, histogram slot (atomic per cell); the
//              atom's data copied to scratch at its current index
//   2 scan     per-replica exclusive scan of cell counts -> cell_start,
//              clearing the counts for the next call
//   3 keys     key[cell_start[c] + slot] = id   (cell members, any order)
//   4 gather   rank inside the cell by id (deterministic order), the atom's
//              wrapped data from scratch into atoms at its final index,
//              x_build := x (and the packed copy)
#include "md_common.hpp"

namespace md {
namespace {

struct BatchArgs {
    const int32_t *atom_off, *cell_off, *ncell, *unit_rep, *unit_off;
    const double *box;
    const uint32_t *gate;
    int32_t n_units, R;
};

BatchArgs batch_args(const md_batch *b, const uint32_t *gate)
{
    return BatchArgs{b->atom_off, b->cell_off, b->ncell, b->unit_rep, b->unit_off, b->box, gate,
                     b->n_units, b->R};
}

__device__ __forceinline__ bool gated_off(const BatchArgs &a, int rep)
{
    return a.gate != nullptr && a.gate[rep] == 0u;
}

// Lanes of a wave that fall into the same cell take their slots with one
// atomic add per distinct cell (consecutive atoms are mostly cell-mates).
// The groups are found first; then every group leader issues its add in one
// instruction, so the wave waits for a single atomic round trip.  Must be
// reached by every lane of the wave.
__device__ __forceinline__ int aggregated_slot(int32_t *count, int c, bool active)
{
    const int lane = __lane_id();
    unsigned long long todo = __ballot(active);
    int leader_of_mine = lane, prefix = 0, group_size = 0;
    while (todo) {
        const int leader = __ffsll(static_cast<long long>(todo)) - 1;
        const int cl = __shfl(c, leader, kWave);
        const bool mine = active && c == cl;
        const unsigned long long grp = __ballot(mine);
        if (mine) {
            leader_of_mine = leader;
            prefix = __popcll(grp & ((1ull << lane) - 1ull));
        }
        if (lane == leader) group_size = __popcll(grp);
        todo &= ~grp;
    }
    int base = 0;
    if (group_size > 0) base = atomicAdd(count + c, group_size);
    base = __shfl(base, leader_of_mine, kWave);
    return base + prefix;
}

// Grid-stride loop over work units; a unit whose replica's gate is 0 is
// skipped, so a skipped rebuild costs one short launch (one load per
// workgroup for a single replica).
#define MD_FOR_UNITS(a, w)                                                          \
    if (!sole_replica_gated_off((a).gate, (a).R))                                  \
    for (int lb_ = blockIdx.x; lb_ < (a).n_units; lb_ += gridDim.x)                \
        if (const Unit w = unit_of(lb_, (a).unit_rep, (a).unit_off, (a).atom_off); \
            !gated_off((a), w.rep))

__global__ __launch_bounds__(kUnit) void k_bin(BatchArgs a, md_atoms in, md_atoms cp,
                                               int32_t N, int32_t *__restrict__ cell_count,
                                               int32_t *__restrict__ cell_of,
                                               int32_t *__restrict__ slot)
{
    MD_FOR_UNITS(a, w) {
        const int i = w.begin + threadIdx.x;
        const bool active = i < w.end;
        int c = 0;
        if (active) {
            const double x = in.x[i], y = in.y[i], z = in.z[i];
            const double *L = a.box + 3 * w.rep;
            const int32_t *n = a.ncell + 3 * w.rep;
            int s;
            const int cx = cell_coord(wrap_coord(x, L[0], &s), cells_per_length(n[0], L[0]), n[0]);
            const int cy = cell_coord(wrap_coord(y, L[1], &s), cells_per_length(n[1], L[1]), n[1]);
            const int cz = cell_coord(wrap_coord(z, L[2], &s), cells_per_length(n[2], L[2]), n[2]);
            c = a.cell_off[w.rep] + (cz * n[1] + cy) * n[0] + cx;
            // the gather reads the atom from here, so it can write atoms in place
            cp.x[i] = x;
            cp.y[i] = y;
            cp.z[i] = z;
            cp.vx[i] = in.vx[i];
            cp.vy[i] = in.vy[i];
            cp.vz[i] = in.vz[i];
            cp.type[i] = in.type[i];
            cp.id[i] = in.id[i];
            cp.img[i] = in.img[i];
            cp.img[N + i] = in.img[N + i];
            cp.img[2 * N + i] = in.img[2 * N + i];
        }
        const int sl = aggregated_slot(cell_count, c, active);
        if (active) {
            cell_of[i] = c;
            slot[i] = sl;
        }
    }
}

// One workgroup of kScan threads per replica scans its cells in passes of
// kScanPer * kScan cells.  Counts are read and starts written coalesced,
// through LDS; each thread scans kScanPer consecutive cells from LDS (the
// LDS index is skewed by one word per 32 so those reads do not collide).
constexpr int kScan = 1024;
constexpr int kScanPer = 16;
constexpr int kScanTile = kScanPer * kScan;

__device__ __forceinline__ int scan_skew(int e) { return e + (e >> 5); }

__global__ __launch_bounds__(kScan) void k_scan(BatchArgs a, int32_t *__restrict__ cell_count,
                                                int32_t *__restrict__ cell_start)
{
    const int r = blockIdx.x;
    if (gated_off(a, r)) return;
    constexpr int kW = kScan / kWave;
    __shared__ int32_t wsum[kW];
    __shared__ int32_t buf[kScanTile + kScanTile / 32];
    const int c0 = a.cell_off[r], c1 = a.cell_off[r + 1];
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    int32_t carry = a.atom_off[r];
    for (int base = c0; base < c1; base += kScanTile) {
        int32_t g[kScanPer];
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            const int c = base + k * kScan + tid;
            g[k] = c < c1 ? cell_count[c] : 0;
        }
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) buf[scan_skew(k * kScan + tid)] = g[k];
        __syncthreads();
        int32_t v[kScanPer];
        int32_t t = 0;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            v[k] = buf[scan_skew(kScanPer * tid + k)];
            t += v[k];
        }
        int32_t inc = t;   // inclusive wave scan of the per-thread totals
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int32_t up = __shfl_up(inc, o, kWave);
            if (lane >= o) inc += up;
        }
        if (lane == kWave - 1) wsum[wid] = inc;
        __syncthreads();
        int32_t before = 0, total = 0;
#pragma unroll
        for (int k = 0; k < kW; ++k) {
            const int32_t ws = wsum[k];
            before += k < wid ? ws : 0;
            total += ws;
        }
        int32_t run = carry + before + inc - t;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            buf[scan_skew(kScanPer * tid + k)] = run;
            run += v[k];
        }
        carry += total;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            const int c = base + k * kScan + tid;
            if (c < c1) {
                cell_start[c] = buf[scan_skew(k * kScan + tid)];
                cell_count[c] = 0;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) cell_start[c1] = a.atom_off[r + 1];
}

__global__ __launch_bounds__(kUnit) void k_keys(BatchArgs a, const int32_t *__restrict__ id,
                                                const int32_t *__restrict__ cell_of,
                                                const int32_t *__restrict__ slot,
                                                const int32_t *__restrict__ cell_start,
                                                int32_t *__restrict__ key)
{
    MD_FOR_UNITS(a, w) {
        const int i = w.begin + threadIdx.x;
        if (i < w.end) key[cell_start[cell_of[i]] + slot[i]] = id[i];
    }
}

__global__ __launch_bounds__(kUnit) void k_gather(BatchArgs a, md_atoms in, md_atoms out,
                                                  int32_t N,
                                                  const int32_t *__restrict__ cell_of,
                                                  const int32_t *__restrict__ cell_start,
                                                  const int32_t *__restrict__ key)
{
    MD_FOR_UNITS(a, w) {
        const int i = w.begin + threadIdx.x;
        if (i >= w.end) continue;
        // every input of the atom is loaded first, so these loads overlap
        // the dependent cell-start and key reads of the rank search
        const double x0 = in.x[i], y0 = in.y[i], z0 = in.z[i];
        const double vx = in.vx[i], vy = in.vy[i], vz = in.vz[i];
        const int32_t ty = in.type[i], me = in.id[i];
        const int32_t ix = in.img[i], iy = in.img[N + i], iz = in.img[2 * N + i];
        const int c = cell_of[i];
        const int s = cell_start[c], e = cell_start[c + 1];
        // rank among the cell's ids, read 16 bytes at a time from the
        // 16-byte-aligned start at or below s (the key buffer is padded)
        int rank = 0;
        for (int m = s & ~3; m < e; m += 16) {
            int4 kv[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) kv[v] = *reinterpret_cast<const int4 *>(key + m + 4 * v);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int kk[4] = {kv[v].x, kv[v].y, kv[v].z, kv[v].w};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int mq = m + 4 * v + q;
                    rank += (mq >= s && mq < e && kk[q] < me) ? 1 : 0;
                }
            }
        }
        const int dst = s + rank;
        const double *L = a.box + 3 * w.rep;
        int sx, sy, sz;
        const double xw = wrap_coord(x0, L[0], &sx);
        const double yw = wrap_coord(y0, L[1], &sy);
        const double zw = wrap_coord(z0, L[2], &sz);
        out.x[dst] = xw;
        out.y[dst] = yw;
        out.z[dst] = zw;
        out.xb[dst] = xw;
        out.yb[dst] = yw;
        out.zb[dst] = zw;
        if (out.pos4) reinterpret_cast<double4 *>(out.pos4)[dst] = make_double4(xw, yw, zw, 0.0);
        out.vx[dst] = vx;
        out.vy[dst] = vy;
        out.vz[dst] = vz;
        out.type[dst] = ty;
        out.id[dst] = me;
        out.img[dst] = ix + sx;
        out.img[N + dst] = iy + sy;
        out.img[2 * N + dst] = iz + sz;
        if (out.where) out.where[me] = dst;
    }
}

bool atoms_ok(const md_atoms *a, bool need_build)
{
    if (!a) return false;
    const void *dbl[] = {a->x, a->y, a->z, a->vx, a->vy, a->vz};
    for (const void *q : dbl)
        if (!q || !aligned8(q)) return false;
    if (!a->type || !a->id || !a->img) return false;
    if (need_build && (!a->xb || !a->yb || !a->zb)) return false;
    return true;
}

}  // namespace
}  // namespace md

extern "C" int md_cell_sort(const md_batch *b, md_atoms *atoms, md_atoms *scratch,
                            int32_t *cell_start, void *ws, size_t ws_bytes,
                            const uint32_t *gate, uint32_t *status, void *stream)
{
    using namespace md;
    (void)status;
    int e = check_batch(b);
    if (e != MD_OK) return e;
    if (!atoms_ok(atoms, true) || !atoms_ok(scratch, false) || !cell_start || !ws)
        return MD_EINVAL;
    const WsLayout l = ws_layout(b);
    if (ws_bytes < l.total) return MD_ENOWS;
    hipStream_t s = as_stream(stream);
    const BatchArgs a = batch_args(b, gate);
    int32_t *cnt = ws_at<int32_t>(ws, l.cell_count);
    int32_t *cell_of = ws_at<int32_t>(ws, l.cell_of);
    int32_t *slot = ws_at<int32_t>(ws, l.slot);
    int32_t *key = ws_at<int32_t>(ws, l.key);
    const dim3 grid(gated_grid(b->n_units, gate != nullptr)), block(kUnit);
    hipLaunchKernelGGL(k_bin, grid, block, 0, s, a, *atoms, *scratch, b->N, cnt, cell_of, slot);
    hipLaunchKernelGGL(k_scan, dim3(b->R), dim3(kScan), 0, s, a, cnt, cell_start);
    hipLaunchKernelGGL(k_keys, grid, block, 0, s, a, atoms->id, cell_of, slot, cell_start, key);
    hipLaunchKernelGGL(k_gather, grid, block, 0, s, a, *scratch, *atoms, b->N, cell_of, cell_start, key);
    return launch_status();
}

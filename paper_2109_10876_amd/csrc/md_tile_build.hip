// md_tile_build.hip -- tile-local Verlet list build (MD_TILE_FULL).
//
// Same list as the global-index build (Sec. 2.1.2 cell stencil, Verlet
// radius rc + skin); the candidates of every home cell come from the tile's
// LDS staging (md_tile.hpp) with periodic images already applied, and each
// entry names its neighbour by a 16-bit staged slot.
#include "md_tile.hpp"

namespace md {
namespace {

// Home cells with at most kFlatChunks x 64 stencil candidates and at most 64
// atoms take the register path (chunks are tested three at a time); others
// the row-by-row path.
constexpr int kFlatChunks = 12;
constexpr int kChunkGroup = 3;
static_assert(kFlatChunks % kChunkGroup == 0, "whole groups of chunks");

__device__ __forceinline__ void put_entry(const TileArgs &a, int k, int i, uint16_t e)
{
    *reinterpret_cast<uint16_t *>(reinterpret_cast<char *>(a.idx) + tile_entry_byte(k, i, a.ld)) =
        e;
}

// Register path: a wave gathers one home atom's entries in its LDS buffer
// (entry kb + e at wb[e], kb a multiple of 8) and stores them a block of 8
// entries (16 bytes) per lane, lane b taking block kb / 8 + b: one store
// instruction per home atom instead of a scattered 2-byte store per hit.
// 288 entries per wave keep the build's LDS within three workgroups per CU.
constexpr int kWaveBuf = 288;

__device__ __forceinline__ void store_block(const TileArgs &a, const uint16_t *wb, int i, int kb,
                                            int b)
{
    const uint4 v = *reinterpret_cast<const uint4 *>(wb + 8 * b);
    *reinterpret_cast<uint4 *>(reinterpret_cast<char *>(a.idx) + tile_entry_byte(kb + 8 * b, i, a.ld)) =
        v;
}

// Store the buffer's whole blocks (those below max_nbr) and move the partial
// block to the front; returns the new kb.  Every lane of the wave calls it.
// Taken only when a group of chunks could overrun the buffer (about 100
// entries in hand already), so rarely on a liquid.
__device__ __forceinline__ int flush_blocks(const TileArgs &a, uint16_t *wb, int i, int kb, int cnt,
                                            int lane)
{
    const int nfb = (cnt - kb) >> 3;
    __builtin_amdgcn_wave_barrier();
    if (lane < nfb && kb + 8 * lane < a.max_nbr) store_block(a, wb, i, kb, lane);
    // Every lane moves one entry of the partial block (lanes past it copy its
    // last slot; entries past the count are overwritten before they are
    // stored).  An unconditional read and write leave no LDS load in flight
    // past this call, so the hit stores that follow need not wait for the
    // LDS queue to drain.  The caller keeps cnt - kb <= 272 here, so the
    // read stays inside the buffer.
    const uint16_t t = wb[8 * nfb + min(lane, 7)];
    __builtin_amdgcn_wave_barrier();
    wb[lane] = t;
    __builtin_amdgcn_wave_barrier();
    return kb + 8 * nfb;
}

// Lanes 0 .. nb-1 of a wavefront hold the entry counts of home atoms
// hb .. hb+nb-1: store them and flag overflow.
__device__ __forceinline__ void store_counts(const TileArgs &a, int hb, int nb, int lane, int vcnt)
{
    if (lane >= nb) return;
    a.count[hb + lane] = vcnt;
    if (vcnt > a.max_nbr) {
        if (a.status) atomicOr(a.status, MD_F_NBR_OVERFLOW);
        if (a.need) atomicMax(a.need, vcnt);
    }
}

// List build, one wavefront per home cell, whose candidates are the staged
// slots of its 27-cell stencil (nine contiguous slot ranges, one per stencil
// row).  The wave visits the cell's home atoms in turn, every lane testing
// its candidates against the same home atom; a home atom's hits are placed
// by a ballot and the count of hitting lanes below each lane, so entries
// keep candidate order.  Lists are padded to a multiple of 16 entries
// (max_nbr is one) with the pad slot, so force loops need no tail mask.
//
// Register path: the candidate sequence -- the own cell first, then the
// stencil rows in order with the middle row's own cell left out -- sits in
// registers, 64 per chunk, unused lanes holding the pad slot, and each lane
// keeps 2 p and |p|^2 of its candidates.  |h - p|^2 < rl^2 is then tested as
// 2 h.p - |p|^2 > |h|^2 - rl^2 on coordinates relative to the cell's first
// atom (all within two cell diagonals of it), with rl^2 raised by 2^-40
// relative: more than the rounding of either side, so every pair within rl
// is kept and a pair kept beyond it lies within rounding of rl.  The own atom
// is lane j of chunk 0.  A chunk's hits go to the wave's LDS buffer (one
// 2-byte LDS store per hitting lane, at the count of hits before it), and
// the home atom's finished list leaves it as 16-byte blocks.
template <class SH, bool P4>
__global__ __launch_bounds__(SH::TB) __attribute__((amdgpu_waves_per_eu(3))) void k_tile_build(
    TileArgs a)
{
    constexpr int TB = SH::TB, CAP = SH::CAP;
    constexpr int kWaves = TB / kWave;
    constexpr int C = kFlatChunks;
    __shared__ TileStage<CAP, SH::MAXC> st;
    __shared__ __attribute__((aligned(16))) uint16_t wbuf[kWaves][kWaveBuf];
    if (sole_replica_gated_off(a.gate, a.R)) return;
    const int lane = __lane_id();
    const int wid = uniform(threadIdx.x / kWave);
    uint16_t *const wb = wbuf[wid];
    const uint16_t pad = uint16_t(CAP * 8);
    const double rl2x = a.rl2 * (1.0 + 0x1p-40);
    // with a to-do list, workgroups past its count return after one load
    const int n_work = a.todo ? a.todo[0] : a.n_tiles;
    for (int lt = blockIdx.x; lt < n_work; lt += gridDim.x) {
        const int t = a.todo ? a.todo[1 + xcd_chunked(lt, n_work, kTileXcdChunk)]
                             : xcd_chunked(lt, a.n_tiles, kTileXcdChunk);
        const TileSpec s = tile_spec(t, a.tile_rep, a.tile_off, a.ncell, a.cell_off, a.box, a.g, a.tile_m);
        if (a.gate != nullptr && a.gate[s.rep] == 0u) continue;
        const int home = tile_home_atoms(s, a.cell_start);
        // occupancy for the occupied-tile list (listed by k_tile_compact)
        if (a.active && threadIdx.x == 0) a.active[1 + a.n_tiles + t] = home > 0 ? 1 : 0;
        if (home == 0) continue;
        const int total =
            stage_tile<TB, P4>(s, a.cell_start, a.x, a.y, a.z, a.pos4, st, CAP,
                               a.tile_src + size_t(t) * tab_stride(CAP), [] { return true; });
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
            const int nown = g1 - g0;
            if (nown == 0) continue;
            const int own0 = uniform(st.row_slot[qc] + st.cslot[qc][kc + 1]);
            // The nine stencil rows of this home cell: first slot, length.
            int rs0[9], rlen[9];
            int T = 0;
#pragma unroll
            for (int r9 = 0; r9 < 9; ++r9) {
                const int r = staged_row(s, dy + r9 % 3 - 1, dz + r9 / 3 - 1);
                rs0[r9] = uniform(st.row_slot[r] + st.cslot[r][kc]);
                rlen[r9] = uniform(st.row_slot[r] + st.cslot[r][kc + 3]) - rs0[r9];
                T += rlen[r9];
            }
            if (T <= C * kWave && nown <= kWave) {
                // Segments of the candidate sequence: first sequence index
                // pf and slot - index offset dl (the last segment with
                // pf <= f holds index f; empty segments are passed over).
                int pf[11], dl[11];
                {
                    int F = 0, q = 0;
                    auto seg = [&](int first, int len) {
                        pf[q] = F;
                        dl[q] = first - F;
                        F += len;
                        ++q;
                    };
                    seg(own0, nown);
#pragma unroll
                    for (int r9 = 0; r9 < 9; ++r9) {
                        if (r9 == 4) {
                            seg(rs0[4], own0 - rs0[4]);
                            seg(own0 + nown, rs0[4] + rlen[4] - own0 - nown);
                        } else {
                            seg(rs0[r9], rlen[r9]);
                        }
                    }
                }
                const int nch = (T + kWave - 1) / kWave;
                const double ox = st.x[own0], oy = st.y[own0], oz = st.z[own0];
                double px[C], py[C], pz[C], pp[C];
                int ent[C];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const int f = c * kWave + lane;
                    int d = dl[0];
#pragma unroll
                    for (int q = 1; q < 11; ++q) d = f >= pf[q] ? dl[q] : d;
                    const int slot = (c < nch && f < T) ? f + d : CAP;
                    px[c] = st.x[slot] - ox;
                    py[c] = st.y[slot] - oy;
                    pz[c] = st.z[slot] - oz;
                    pp[c] = fma(px[c], px[c], fma(py[c], py[c], pz[c] * pz[c]));
                    ent[c] = slot * 8;
                    if (a.tile_types > 1 && slot < CAP) {
                        int row;
                        double sx;
                        ent[c] |= a.type[slot_source(s, st, slot, row, sx)];
                    }
                }
                int vcnt = 0;   // lane j: entries of home atom g0 + j
                for (int j = 0; j < nown; ++j) {
                    const int hs = own0 + j;
                    const int i = g0 + j;
                    const double hx = st.x[hs] - ox, hy = st.y[hs] - oy, hz = st.z[hs] - oz;
                    const double tx = 2.0 * hx, ty = 2.0 * hy, tz = 2.0 * hz;
                    const double rhs = fma(hx, hx, fma(hy, hy, hz * hz)) - rl2x;
                    int cnt = 0;
                    int kb = 0;
#pragma unroll
                    for (int g = 0; g < C; g += kChunkGroup) {
                        if (g >= nch) break;
                        // room for the group's hits (at most its candidates) and the pad
                        if (cnt - kb + min(kChunkGroup * kWave, T - g * kWave) + 16 > kWaveBuf)
                            kb = flush_blocks(a, wb, i, kb, cnt, lane);
#pragma unroll
                        for (int c = g; c < g + kChunkGroup; ++c) {
                            const double lhs = fma(tx, px[c], fma(ty, py[c], fma(tz, pz[c], -pp[c])));
                            bool take = lhs > rhs;
                            if (c == 0) take = take && lane != j;
                            const uint64_t m = __builtin_amdgcn_ballot_w64(take);
                            if (take) {
                                const int r = int(__builtin_amdgcn_mbcnt_hi(
                                    uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u)));
                                wb[cnt - kb + r] = uint16_t(ent[c]);
                            }
                            cnt += int(__popcll(m));
                        }
                    }
                    // pad to a multiple of 16, then store the buffered blocks
                    // (past max_nbr nothing is stored; the count flags the overflow)
                    const int n16 = (cnt + 15) & ~15;
                    if (cnt + lane < n16) wb[cnt - kb + lane] = pad;
                    __builtin_amdgcn_wave_barrier();
                    const int kend = min(n16, a.max_nbr);
                    if (kb + 8 * lane < kend) store_block(a, wb, i, kb, lane);
                    __builtin_amdgcn_wave_barrier();
                    vcnt = lane == j ? cnt : vcnt;
                }
                store_counts(a, g0, nown, lane, vcnt);
                continue;
            }
            // Row-by-row path: the lanes hold 64 candidates of one stencil
            // row at a time; per-atom counts live one per lane of a batch of
            // up to 64 home atoms.
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
                                              (norm2(dx, dyy, dzz) < a.rl2);
                            const uint64_t m = __builtin_amdgcn_ballot_w64(take);
                            const int cnt = __builtin_amdgcn_readlane(vcnt, j);
                            const int k = int(__builtin_amdgcn_mbcnt_hi(
                                uint32_t(m >> 32),
                                __builtin_amdgcn_mbcnt_lo(uint32_t(m), uint32_t(cnt))));
                            if (take && k < a.max_nbr) put_entry(a, k, hb + j, ent);
                            vcnt = lane == j ? cnt + int(__popcll(m)) : vcnt;
                        }
                    }
                }
                store_counts(a, hb, nb, lane, vcnt);
                if (lane < nb && vcnt <= a.max_nbr)
                    for (int k = vcnt; k < ((vcnt + 15) & ~15); ++k) put_entry(a, k, hb + lane, pad);
            }
        }
        __syncthreads();
    }
}

// The to-do list of a batch's list build: the tiles of every replica whose
// gate is set, replica by replica, after their count.  One workgroup scans
// the replicas kFin at a time (per-replica tile counts, a block prefix sum),
// then each wave writes the tile ranges of its replicas.
__global__ __launch_bounds__(kFin) void k_tile_todo(int R, const uint32_t *__restrict__ gate,
                                                    const int32_t *__restrict__ tile_off,
                                                    int32_t *__restrict__ todo)
{
    constexpr int kW = kFin / kWave;
    __shared__ int start[kFin];
    __shared__ int wsum[kW];
    const int tid = threadIdx.x, lane = tid % kWave, wid = tid / kWave;
    int carry = 0;
    for (int base = 0; base < R; base += kFin) {
        const int r = base + tid;
        const int n = r < R && gate[r] != 0u ? tile_off[r + 1] - tile_off[r] : 0;
        int inc = n;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int up = __shfl_up(inc, o, kWave);
            if (lane >= o) inc += up;
        }
        if (lane == kWave - 1) wsum[wid] = inc;
        __syncthreads();
        int before = carry, total = carry;
        for (int w = 0; w < kW; ++w) {
            before += w < wid ? wsum[w] : 0;
            total += wsum[w];
        }
        start[tid] = before + inc - n;
        __syncthreads();
        for (int q = wid; q < kFin && base + q < R; q += kW) {
            const int rr = base + q;
            if (gate[rr] == 0u) continue;
            const int t0 = tile_off[rr], nt = tile_off[rr + 1] - t0, s0 = start[q];
            for (int k = lane; k < nt; k += kWave) todo[1 + s0 + k] = t0 + k;
        }
        carry = total;
        __syncthreads();
    }
    if (tid == 0) todo[0] = carry;
}

// The occupied-tile list of one replica: the tiles whose flag the build set,
// in ascending order, after the count.  One workgroup scans the flags in
// passes of kFin tiles (each wave's prefix from a ballot, the waves' totals
// from LDS).  Skipped when the gate is 0 (the list is still valid).
__global__ __launch_bounds__(kFin) void k_tile_compact(int n_tiles, const uint32_t *gate,
                                                       int32_t *active)
{
    if (gate && gate[0] == 0u) return;
    constexpr int kW = kFin / kWave;
    __shared__ int wsum[kW];
    const int32_t *occ = active + 1 + n_tiles;
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    int carry = 0;
    for (int base = 0; base < n_tiles; base += kFin) {
        const int t = base + threadIdx.x;
        const bool on = t < n_tiles && occ[t] != 0;
        const uint64_t m = __builtin_amdgcn_ballot_w64(on);
        const int below = int(__builtin_amdgcn_mbcnt_hi(
            uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u)));
        if (lane == 0) wsum[wid] = int(__popcll(m));
        __syncthreads();
        int before = carry, total = carry;
        for (int w = 0; w < kW; ++w) {
            before += w < wid ? wsum[w] : 0;
            total += wsum[w];
        }
        if (on) active[1 + before + below] = t;
        carry = total;
        __syncthreads();
    }
    if (threadIdx.x == 0) active[0] = carry;
}

}  // namespace

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
    a.active = nl->tile_active;   // one replica only (checked by the caller)
    if (gate && b->R > 1 && nl->tile_todo) {
        hipLaunchKernelGGL(k_tile_todo, dim3(1), dim3(kFin), 0, s, b->R, gate, nl->tile_off,
                           nl->tile_todo);
        a.todo = nl->tile_todo;
    }
    // one workgroup per tile, gated or not: the hardware hands tiles to
    // whichever workgroup slot frees first, so uneven tiles (vacuum, surface)
    // balance themselves; a gated-off tile costs a launch slot only
    const dim3 grid(nl->n_tiles);
    const bool p4 = tile_stage_packed() && atoms->pos4;
    with_tile_shape([&](auto sh) {
        using SH = decltype(sh);
        if (p4) hipLaunchKernelGGL((k_tile_build<SH, true>), grid, dim3(SH::TB), 0, s, a);
        else hipLaunchKernelGGL((k_tile_build<SH, false>), grid, dim3(SH::TB), 0, s, a);
    });
    if (nl->tile_active)
        hipLaunchKernelGGL(k_tile_compact, dim3(1), dim3(kFin), 0, s, nl->n_tiles, gate,
                           nl->tile_active);
    return launch_status();
}

}  // namespace md

// md_tile.hip -- LJ forces over tile-local Verlet lists (MD_TILE_FULL).
//
// Same method as the global-index path (Eq. lj pair terms over a Verlet list
// of radius rc + skin, Sec. 2.1.2); only where neighbour positions come from
// differs.  One workgroup per tile (a block of m x py x pz cells) stages the
// neighbouring rows x (a-1 .. b+1) into LDS with periodic images applied
// (md_tile.hpp); every home atom then walks its list of 16-bit staged slots
// (built by md_tile_build.hip), reading neighbours from LDS: no image
// arithmetic and no L2 gathers in the pair loop.
#include "md_pair.hpp"
#include "md_philox.hpp"
#include "md_tile.hpp"

namespace md {
namespace {

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// Typed lists: LJ constants of type pair (ti, tj) at ti * kTileMaxTypes + tj.
constexpr int kTileMaxTypes = MD_TILE_MAX_TYPES;

// TY: 0 one atom type; 2 two types, the constants of this atom's two type
// pairs held in registers and selected per entry; 4 up to four types, the
// constants read per entry from an LDS table.  FUSE: 0 forces only; 1 then
// md_vv_step phase 3 per atom; 2 the thermostat force added before it; 3 as
// 1 (one type, alternating gate words) for calls that want no energy,
// virial or kinetic energy: the pair loop sums the force alone and the
// tile writes no partials, only its gate word.
template <class SH, int PREC, int U, bool P4, int TY, int FUSE>
__global__ __launch_bounds__(SH::TB) void k_tile_lj(TileArgs a)
{
    constexpr int TB = SH::TB, CAP = SH::CAP;
    __shared__ TilePlanes<CAP> st;
    __shared__ double red[4][TB / kWave];
    __shared__ PolyConst ptab[TY ? kTileMaxTypes * kTileMaxTypes : 1];
    // launch slot -> tile; with the occupied-tile list, slot k takes its
    // k-th tile and writes its partials to row k, and slots past the list
    // write an empty row and leave
    const int lt = xcd_chunked(blockIdx.x, gridDim.x, kTileXcdChunk);
    int t = lt;
    if (a.active) {
        if (lt >= a.active[0]) {
            if (threadIdx.x == 0)
                for (int q = 0; q < kTilePartials; ++q)
                    a.tpart[size_t(lt) * kTilePartials + q] = 0.0;
            return;
        }
        t = min(max(a.active[1 + lt], 0), a.n_tiles - 1);
    }
    const int row = lt;   // partial row: the tile itself, or its place in the list
    const TileSpec s = tile_spec(t, a.tile_rep, a.tile_off, a.ncell, a.cell_off, a.box, a.g, a.tile_m);
    const PolyConst pc = poly_const(a.eps[0], a.sig[0], a.rc, a.shift);
    const double rc2 = a.rc * a.rc;
    if (TY) {
        // filled before staging, whose barriers publish it
        const int nt = a.tile_types;
        if (threadIdx.x < nt * nt) {
            const int ti = threadIdx.x / nt, tj = threadIdx.x % nt;
            ptab[ti * kTileMaxTypes + tj] = poly_const(a.eps[threadIdx.x], a.sig[threadIdx.x], a.rc,
                                                       a.shift);
        }
    }
    // Entries are LDS byte offsets, 8 to a 16-byte block, consumed U at a
    // time while the next U are in flight; a list is padded with the pad
    // slot to a multiple of 16 entries, so no entry needs a mask.  Block
    // reads stay inside the allocation (index clamped to the last block) and
    // LDS reads inside the staging planes (offset clamped to the pad slot).
    constexpr int NB = U / kEntryBlock;
    const int bmax = a.max_nbr / kEntryBlock - 1;
    // The home rows' cell starts, then the inputs of this thread's first
    // home atom (threads past the last one take it again, unused), are
    // fetched while the staging table loads are in flight; an empty tile
    // (vacuum) stops there.
    int hk = threadIdx.x;
    HomeRows hr;
    int nh = 0, i = 0, n = 0, ti4 = 0;
    double xi = 0.0, yi = 0.0, zi = 0.0;
    u32x4 cur[NB];
    const int total = stage_from_table<TB, P4>(
        s, a.tile_src + size_t(t) * tab_stride(CAP), a.n_atoms, a.x, a.y, a.z, a.pos4, st, CAP,
        nullptr, [&] {
            hr = home_rows(s, a.cell_start);
            nh = hr.total;
            if (nh == 0) return false;
            i = home_index(hr, min(hk, nh - 1));
            xi = a.x[i];
            yi = a.y[i];
            zi = a.z[i];
            n = min(a.count[i], a.max_nbr);
            ti4 = TY ? a.type[i] * kTileMaxTypes : 0;
#pragma unroll
            for (int b = 0; b < NB; ++b)
                cur[b] = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(a.idx) + i +
                                                    size_t(min(b, bmax)) * a.ld);
            return true;
        });
    constexpr bool kGateWords = (FUSE == 1 || FUSE == 3) && !TY;
    if (total < 0) {
        if (FUSE != 3 && threadIdx.x < kTilePartials)
            a.tpart[size_t(row) * kTilePartials + threadIdx.x] = 0.0;
        if (kGateWords && a.vv.gate_clear && threadIdx.x == 0) a.vv.gate_clear[s.rep] = 0u;
        return;
    }
    double e_acc = 0.0, w_acc = 0.0, ke_acc = 0.0, d2_max = 0.0;
    if (total > CAP) {
        if (threadIdx.x == 0 && a.status) atomicOr(a.status, MD_F_TILE_OVERFLOW);
    } else {
        const char *stb = reinterpret_cast<const char *>(st.x);
        constexpr int kY = int(sizeof(double)) * decltype(st)::kStride;
        while (hk < nh) {
            Acc c{0.0, 0.0, 0.0, 0.0, 0.0, 0.0f, 0.0f, 0u};
            PairAB<PREC> k0{}, k1{};
            if (TY == 2) {
                k0 = pair_ab<PREC>(ptab[ti4]);
                k1 = pair_ab<PREC>(ptab[ti4 + 1]);
            }
            const u32x4 *lb = reinterpret_cast<const u32x4 *>(a.idx) + i;
            u32x4 nxt[NB];
            for (int k = 0; k < n; k += U) {
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    nxt[b] = __builtin_nontemporal_load(
                        lb + size_t(min(k / kEntryBlock + NB + b, bmax)) * a.ld);
                unsigned ent[U];
#pragma unroll
                for (int q = 0; q < U; ++q) {
                    const unsigned w = cur[q / kEntryBlock][(q % kEntryBlock) / 2];
                    ent[q] = q % 2 ? w >> 16 : w & 0xffffu;
                }
                // all U staged positions are read before any is used
                double px[U], py[U], pz[U];
#pragma unroll
                for (int q = 0; q < U; ++q) {
                    // typed entries carry the type in the low 3 bits
                    const unsigned e = TY ? ent[q] & ~7u : ent[q];
                    const char *pq = stb + min(e, unsigned(CAP * 8));
                    px[q] = *reinterpret_cast<const double *>(pq);
                    py[q] = *reinterpret_cast<const double *>(pq + kY);
                    pz[q] = *reinterpret_cast<const double *>(pq + 2 * kY);
                }
#pragma unroll
                for (int q = 0; q < U; ++q) {
                    if (TY == 2)
                        lj_pair_ab<PREC>(select_ab<PREC>(ent[q] & 1u, k0, k1), xi - px[q],
                                         yi - py[q], zi - pz[q], rc2, c);
                    else if (TY)
                        lj_pair_masked<PREC>(ptab[ti4 + (ent[q] & 7)], xi - px[q], yi - py[q],
                                             zi - pz[q], rc2, c);
                    else if (FUSE == 3)
                        lj_pair_force<PREC>(pc, xi - px[q], yi - py[q], zi - pz[q], rc2, c);
                    else
                        lj_pair_sums<PREC>(pc, xi - px[q], yi - py[q], zi - pz[q], rc2, c);
                }
#pragma unroll
                for (int b = 0; b < NB; ++b) cur[b] = nxt[b];
            }
            double ed = c.ed, wd = c.wd;
            if (PREC != MD_FP64) {
                ed = static_cast<double>(c.ef);
                wd = static_cast<double>(c.wf);
            }
            // one type: the energy follows from the sums of lj_pair_sums
            if (!TY) ed = pair_sums_energy(pc, wd, ed, c.n);
            if (FUSE != 3) {
                e_acc += 0.5 * ed;
                w_acc += 0.5 * wd;
            }
            double gx = c.fx, gy = c.fy, gz = c.fz;   // the atom's force
            if (FUSE == 2) {
                // md_langevin's force, with the velocity on entry
                const VVFuse &f = a.vv;
                const double m = f.mass[f.ntypes > 1 ? a.type[i] : 0];
                double g[3];
                thermostat_normals(static_cast<uint32_t>(f.id[i]), *f.step, f.seed_lo, f.seed_hi,
                                   g);
                const double amp = sqrt(f.gamma * m * f.kT_dt2);
                const double gm = f.gamma * m;
                gx += -gm * f.vx[i] + amp * g[0];
                gy += -gm * f.vy[i] + amp * g[1];
                gz += -gm * f.vz[i] + amp * g[2];
            }
            if (a.accumulate) {
                a.fx[i] += gx;
                a.fy[i] += gy;
                a.fz[i] += gz;
            } else {
                a.fx[i] = gx;
                a.fy[i] = gy;
                a.fz[i] = gz;
            }
            if (a.status && !isfinite(gx + gy + gz + (FUSE == 3 ? 0.0 : ed)))
                atomicOr(a.status, MD_F_NONFINITE);
            if (FUSE) {
                // md_vv_step phase 3 on this atom with the force just computed
                const VVFuse &f = a.vv;
                const double im = f.inv_mass[f.ntypes > 1 ? a.type[i] : 0];
                const double k = f.hdt * im;
                double vx = f.vx[i], vy = f.vy[i], vz = f.vz[i];
                vx = fma(k, gx, vx);
                vy = fma(k, gy, vy);
                vz = fma(k, gz, vz);
                if (FUSE != 3) ke_acc += 0.5 * (vx * vx + vy * vy + vz * vz) / im;
                vx = fma(k, gx, vx);
                vy = fma(k, gy, vy);
                vz = fma(k, gz, vz);
                const double x = fma(f.dt, vx, xi);
                const double y = fma(f.dt, vy, yi);
                const double z = fma(f.dt, vz, zi);
                f.xn[i] = x;
                f.yn[i] = y;
                f.zn[i] = z;
                const double ex = x - f.xb[i], ey = y - f.yb[i], ez = z - f.zb[i];
                d2_max = fmax(d2_max, norm2(ex, ey, ez));
                f.vx[i] = vx;
                f.vy[i] = vy;
                f.vz[i] = vz;
            }
            hk += TB;
            if (hk < nh) {
                i = home_index(hr, hk);
                xi = a.x[i];
                yi = a.y[i];
                zi = a.z[i];
                n = min(a.count[i], a.max_nbr);
                ti4 = TY ? a.type[i] * kTileMaxTypes : 0;
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    cur[b] = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(a.idx) + i +
                                                        size_t(min(b, bmax)) * a.ld);
            }
        }
    }
    // the tile's partials: wave totals, one barrier, then the waves' totals
    // in wave order (as block_sum_n sums them)
    if (FUSE != 3) {
        e_acc = wave_sum(e_acc);
        w_acc = wave_sum(w_acc);
    }
    if (FUSE) {
        if (FUSE != 3) ke_acc = wave_sum(ke_acc);
        d2_max = wave_max(d2_max);
    }
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    if (lane == 0) {
        red[0][wid] = e_acc;
        red[1][wid] = w_acc;
        red[2][wid] = ke_acc;
        red[3][wid] = d2_max;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double es = 0.0, ws = 0.0, ks = 0.0, dm = 0.0;
        for (int q = 0; q < TB / kWave; ++q) {
            es += red[0][q];
            ws += red[1][q];
            ks += red[2][q];
            dm = fmax(dm, red[3][q]);
        }
        if (FUSE != 3) {
            double *tp = a.tpart + size_t(row) * kTilePartials;
            tp[0] = es;
            tp[1] = ws;
            tp[2] = FUSE ? ks : 0.0;
            tp[3] = FUSE ? dm : 0.0;
        }
        // alternating gate words (one atom type): the skin test of the tile's
        // replica, and its other word cleared (this kernel never reads it),
        // by every workgroup on its way out, without a finaliser (done before
        // the staging loads, the clear cost the pair loop registers; the
        // typed kernels leave both to the finaliser for the same reason)
        if (kGateWords && a.vv.gate_clear) {
            a.vv.gate_clear[s.rep] = 0u;
            if (dm > a.vv.lim2) atomicOr(a.vv.gate + s.rep, 1u);
        }
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
// Fixed-order sums of the per-tile partials in rows [t0, t1) of tp (stride
// kTilePartials): E, W, KE summed, the displacement maximum taken; only the
// columns asked for are read (a step that needs the gate alone reads one).
// The four reductions share one barrier; wave totals are then summed in wave
// order, as by block_sum_n.  Thread 0 returns the results.
__device__ __forceinline__ void tile_sums(int t0, int t1, const double *tp, bool want_ew,
                                          bool want_ke, bool want_gate, double out[4])
{
    constexpr int kW = kFin / kWave;
    __shared__ double red[4][kW];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, m = 0.0;
#pragma unroll 4
    for (int t = t0 + threadIdx.x; t < t1; t += kFin) {
        const double *q = tp + size_t(t) * kTilePartials;
        if (want_ew) {
            s0 += q[0];
            s1 += q[1];
        }
        if (want_ke) s2 += q[2];
        if (want_gate) m = fmax(m, q[3]);
    }
    if (want_ew) {
        s0 = wave_sum(s0);
        s1 = wave_sum(s1);
    }
    if (want_ke) s2 = wave_sum(s2);
    if (want_gate) m = wave_max(m);
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    if (lane == 0) {
        red[0][wid] = s0;
        red[1][wid] = s1;
        red[2][wid] = s2;
        red[3][wid] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double e = 0.0, w = 0.0, k = 0.0, d = 0.0;
        for (int q = 0; q < kW; ++q) {
            e += red[0][q];
            w += red[1][q];
            k += red[2][q];
            d = fmax(d, red[3][q]);
        }
        out[0] = e;
        out[1] = w;
        out[2] = k;
        out[3] = d;
    }
}

// Per replica r, the sums over its tiles [tile_off[r], tile_off[r+1]); with
// tile_off null (one replica of many tiles), over the n_rows chunk sums
// that k_tile_chunk_sums wrote to tpart.
__global__ __launch_bounds__(kFin) void k_tile_finalize(const int32_t *tile_off, int n_rows,
                                                        const double *tpart, double *energy,
                                                        double *virial, double *ke,
                                                        uint32_t *gate, uint32_t *gate_zero,
                                                        double lim2, uint64_t *step)
{
    // the thermostat's noise counter advances once per call, after every
    // tile has read it
    if (step && blockIdx.x == 0 && threadIdx.x == 0) *step += 1u;
    const int r = blockIdx.x;
    const int t0 = tile_off ? tile_off[r] : 0, t1 = tile_off ? tile_off[r + 1] : n_rows;
    double v[4];
    tile_sums(t0, t1, tpart, energy != nullptr || virial != nullptr, ke != nullptr,
              gate != nullptr, v);
    if (threadIdx.x == 0) {
        if (energy) energy[r] = v[0];
        if (virial) virial[r] = v[1];
        if (ke) ke[r] = v[2];
        if (gate) gate[r] = v[3] > lim2 ? 1u : 0u;
        if (gate_zero) gate_zero[r] = 0u;
    }
}

// First stage for a single replica of many tiles (one workgroup would read
// them all): block c sums tiles [c kTileChunk, (c+1) kTileChunk) into row c
// of out, in the same fixed order.
constexpr int kTileChunk = 4096;
constexpr int kTileChunkedFrom = 4 * kTileChunk;
static_assert(kPartials == kTilePartials, "chunk sums use the per-unit partial rows");

__global__ __launch_bounds__(kFin) void k_tile_chunk_sums(int n_tiles, const double *tpart,
                                                          double *out, bool want_ew,
                                                          bool want_ke, bool want_gate)
{
    const int c = blockIdx.x;
    double v[4];
    tile_sums(c * kTileChunk, min((c + 1) * kTileChunk, n_tiles), tpart, want_ew, want_ke,
              want_gate, v);
    if (threadIdx.x == 0)
        for (int q = 0; q < kTilePartials; ++q) out[size_t(c) * kTilePartials + q] = v[q];
}

}  // namespace

bool tile_stage_packed() { return md_tune_get(MD_TUNE_TILE_STAGE_PACKED) != 0; }

bool tile_list_ok(const md_batch *b, const md_nlist *nl)
{
    return nl->n_tiles >= 1 && nl->n_tiles <= b->C && nl->tile_rep && nl->tile_off &&
           (reinterpret_cast<uintptr_t>(nl->idx) & 15) == 0 && nl->tile_src &&
           (nl->tile_active == nullptr || b->R == 1) &&
           nl->tile_src_cap == tile_capacity() &&
           nl->max_nbr % 16 == 0 && nl->ld <= kTileMaxLd && nl->tile_types >= 0 &&
           nl->tile_types <= MD_TILE_MAX_TYPES &&
           size_t(nl->max_nbr) * size_t(nl->ld) * 2 < (size_t(1) << 32) &&
           nl->tile_cells >= 1 && nl->tile_cells <= tile_max_cells() && nl->tile_py >= 1 &&
           nl->tile_py <= MD_TILE_MAX_ROWS && nl->tile_pz >= 1 && nl->tile_pz <= MD_TILE_MAX_ROWS;
}

int tile_threads() { return md_tune_get(MD_TUNE_TILE_THREADS); }

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

int tile_forces(const md_batch *b, const md_atoms *atoms, const md_nlist *nl, const md_lj *p,
                int32_t prec, int32_t accumulate, const int32_t *cell_start, double *energy,
                double *virial, double *tpart, double *chunk_sums, int chunk_rows, int batch,
                const VVFuse *vvf, uint32_t *status, hipStream_t s)
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
    a.active = nl->tile_active;   // one replica only (checked by the callers)
    if (vvf) a.vv = *vvf;
    a.status = status;
    const dim3 grid(nl->n_tiles);
    const bool p4 = tile_stage_packed() && atoms->pos4;
    const bool big = batch >= 8;
    const bool typed = p->ntypes > 1;
    const bool fuse = vvf != nullptr;
    const int timed = timing_begin(s);
    with_tile_shape([&](auto sh) {
        using SH = decltype(sh);
        const dim3 blk(SH::TB);
#define MD_TILE_LAUNCH(P, U, T, F)                                                          \
    do {                                                                                    \
        if (p4) hipLaunchKernelGGL((k_tile_lj<SH, P, U, true, T, F>), grid, blk, 0, s, a);  \
        else hipLaunchKernelGGL((k_tile_lj<SH, P, U, false, T, F>), grid, blk, 0, s, a);    \
    } while (0)
        if (fuse) {
            // the integrator (FUSE 1), with the thermostat first (FUSE 2)
            const int ty = !typed ? 0 : (p->ntypes == 2 ? 2 : 4);
#define MD_TILE_FUSED(F)                                                                  \
    do {                                                                                  \
        if (ty == 0) {                                                                    \
            if (prec == MD_FP64) MD_TILE_LAUNCH(MD_FP64, 8, 0, F);                        \
            else MD_TILE_LAUNCH(MD_FP32_MIXED, 8, 0, F);                                  \
        } else if (ty == 2) {                                                             \
            if (prec == MD_FP64) MD_TILE_LAUNCH(MD_FP64, 8, 2, F);                        \
            else MD_TILE_LAUNCH(MD_FP32_MIXED, 8, 2, F);                                  \
        } else {                                                                          \
            if (prec == MD_FP64) MD_TILE_LAUNCH(MD_FP64, 8, 4, F);                        \
            else MD_TILE_LAUNCH(MD_FP32_MIXED, 8, 4, F);                                  \
        }                                                                                 \
    } while (0)
            // one type, alternating gate words and no energy, virial or
            // kinetic energy asked: the force-only pair loop (FUSE 3)
            const bool bare = !vvf->step && vvf->gate_clear && ty == 0 && !energy && !virial &&
                              !vvf->ke;
            if (vvf->step) MD_TILE_FUSED(2);
            else if (bare && prec == MD_FP64) {
                if (big) MD_TILE_LAUNCH(MD_FP64, 16, 0, 3);
                else MD_TILE_LAUNCH(MD_FP64, 8, 0, 3);
            } else if (bare) {
                if (big) MD_TILE_LAUNCH(MD_FP32_MIXED, 16, 0, 3);
                else MD_TILE_LAUNCH(MD_FP32_MIXED, 8, 0, 3);
            }
            else MD_TILE_FUSED(1);
#undef MD_TILE_FUSED
        } else if (typed && p->ntypes == 2) {
            if (prec == MD_FP64) MD_TILE_LAUNCH(MD_FP64, 8, 2, 0);
            else MD_TILE_LAUNCH(MD_FP32_MIXED, 8, 2, 0);
        } else if (typed) {
            if (prec == MD_FP64) MD_TILE_LAUNCH(MD_FP64, 8, 4, 0);
            else MD_TILE_LAUNCH(MD_FP32_MIXED, 8, 4, 0);
        } else if (prec == MD_FP64) {
            if (big) MD_TILE_LAUNCH(MD_FP64, 16, 0, 0);
            else MD_TILE_LAUNCH(MD_FP64, 8, 0, 0);
        } else {
            if (big) MD_TILE_LAUNCH(MD_FP32_MIXED, 16, 0, 0);
            else MD_TILE_LAUNCH(MD_FP32_MIXED, 8, 0, 0);
        }
#undef MD_TILE_LAUNCH
    });
    timing_end(timed, s);
    double *ke = fuse ? vvf->ke : nullptr;
    // alternating gate words are set and cleared by the one-type force
    // kernel itself, for typed lists by the finaliser
    const bool gate_in_kernel = fuse && vvf->gate_clear && !typed;
    uint32_t *gate = fuse && !gate_in_kernel ? vvf->gate : nullptr;
    uint32_t *gate_zero = fuse && !gate_in_kernel ? vvf->gate_clear : nullptr;
    const int n_chunks = (nl->n_tiles + kTileChunk - 1) / kTileChunk;
    if ((energy || virial || ke || gate) && b->R == 1 && nl->n_tiles >= kTileChunkedFrom &&
        chunk_sums && n_chunks <= chunk_rows) {
        hipLaunchKernelGGL(k_tile_chunk_sums, dim3(n_chunks), dim3(kFin), 0, s, nl->n_tiles,
                           tpart, chunk_sums, energy != nullptr || virial != nullptr,
                           ke != nullptr, gate != nullptr);
        hipLaunchKernelGGL(k_tile_finalize, dim3(1), dim3(kFin), 0, s, nullptr, n_chunks,
                           chunk_sums, energy, virial, ke, gate, gate_zero,
                           fuse ? vvf->lim2 : 0.0, fuse ? vvf->step : nullptr);
    } else if (energy || virial || ke || gate) {
        hipLaunchKernelGGL(k_tile_finalize, dim3(b->R), dim3(kFin), 0, s, nl->tile_off, 0, tpart,
                           energy, virial, ke, gate, gate_zero, fuse ? vvf->lim2 : 0.0,
                           fuse ? vvf->step : nullptr);
    }
    if (fuse && vvf->copy_back)
        hipLaunchKernelGGL(k_copy_next, dim3((b->N + kUnit - 1) / kUnit), dim3(kUnit), 0, s, b->N,
                           vvf->xn, vvf->yn, vvf->zn, atoms->x, atoms->y, atoms->z, atoms->pos4);
    return launch_status();
}

}  // namespace md

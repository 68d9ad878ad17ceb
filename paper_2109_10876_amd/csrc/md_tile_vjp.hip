// md_tile_vjp.hip -- md_lj_forces_vjp over tile-local lists (MD_TILE_FULL).
//
// The vector-Jacobian product of the global-index adjoint (derivatives of
// Eq. lj, Sec. 2.1.1; pair terms recomputed, nothing stored from the forward
// pass): for an upstream G = dL/dF and gE = dL/dE, pair (i, j) with
// d = x_i - x_j and u = G_i - G_j adds w = fr u + (fr'/r)(d.u) d - gE fr d to
// dL/dx_i, and (d.u) dfr/dp + gE dU/dp to the parameter p of its type pair.
// A full list gives each thread its own atom's gradient (the partner's visit
// supplies -w), and the parameter terms, seen from both atoms, are halved.
//
// One workgroup per tile: the neighbourhood is staged in LDS from the tile's
// staging record (md_tile.hpp), with, per slot, the neighbour's G (FP32-mixed)
// or its source atom (FP64, G then gathered from memory through it).
// Per-tile (eps, sigma) sums go to the record's adjoint words; a fixed-order
// finalize adds them over tiles.
#include "md_pair.hpp"
#include "md_tile.hpp"

namespace md {
namespace {

constexpr int kTT = MD_TILE_MAX_TYPES;       // type-pair slot ta * kTT + tb
constexpr int kAdjSlots = kTT * kTT;
static_assert(2 * kAdjSlots * 2 <= 64, "adjoint sums fit the record's spare words");

typedef unsigned u32x4v __attribute__((ext_vector_type(4)));

// LDS of one tile.  FP32-mixed: the upstream G of every staged slot sits
// beside its position, rounded to FP32 (a pair term, like the pair
// arithmetic), gathered once per slot with the positions instead of once per
// pair from memory.  FP64: G stays in memory, gathered per pair through the
// slot's source atom.
template <int CAP, bool STAGED_G>
struct VjpLds;
template <int CAP>
struct VjpLds<CAP, true> {
    TilePlanes<CAP> st;
    float gx[CAP + 1], gy[CAP + 1], gz[CAP + 1];
};
template <int CAP>
struct VjpLds<CAP, false> {
    TilePlanes<CAP> st;
    int lsrc[CAP];
};

// Stages G[src] of a thread's k-th slot (with its position) as FP32.
template <int KPER>
struct GradGather {
    const double *gx, *gy, *gz;
    float *lx, *ly, *lz;
    double vx[KPER], vy[KPER], vz[KPER];
    __device__ void load(int k, uint32_t src)
    {
        vx[k] = load_at(gx, src);
        vy[k] = load_at(gy, src);
        vz[k] = load_at(gz, src);
    }
    __device__ void store(int k, int sl)
    {
        lx[sl] = static_cast<float>(vx[k]);
        ly[sl] = static_cast<float>(vy[k]);
        lz[sl] = static_cast<float>(vz[k]);
    }
};

template <class SH, int PREC, int NT>
__global__ __launch_bounds__(SH::TB) void k_tile_vjp(TileArgs a)
{
    constexpr int TB = SH::TB, CAP = SH::CAP, kW = TB / kWave, NS = NT * NT;
    constexpr bool SG = PREC == MD_FP32_MIXED;
    __shared__ VjpLds<CAP, SG> L;
    __shared__ VjpConst tab[kAdjSlots];
    __shared__ double red[2 * NS][kW];
    auto &st = L.st;
    const int t = xcd_chunked(blockIdx.x, gridDim.x, kTileXcdChunk);
    const TileSpec s = tile_spec(t, a.tile_rep, a.tile_off, a.ncell, a.cell_off, a.box, a.g, a.tile_m);
    uint32_t *rec = a.tile_src + size_t(t) * tab_stride(CAP);
    double *adj = reinterpret_cast<double *>(rec + kTabAdj<TilePlanes<CAP>>);
    if (threadIdx.x < NS) {
        // the LJ table is [NT * NT] here (tile lists carry at most kTT types)
        const int ti = threadIdx.x / NT, tj = threadIdx.x % NT;
        tab[ti * kTT + tj] = vjp_const(a.eps[threadIdx.x], a.sig[threadIdx.x], a.rc, a.shift);
    }
    HomeRows hr;
    int nh = 0;
    auto mid = [&] {
        hr = home_rows(s, a.cell_start);
        nh = hr.total;
        return nh > 0;
    };
    int total;
    if constexpr (SG) {
        if (threadIdx.x == 0) L.gx[CAP] = L.gy[CAP] = L.gz[CAP] = 0.0f;
        total = stage_from_table<TB, false>(
            s, rec, a.n_atoms, a.x, a.y, a.z, nullptr, st, CAP, nullptr, mid,
            GradGather<(CAP + TB - 1) / TB>{a.gfx, a.gfy, a.gfz, L.gx, L.gy, L.gz, {}, {}, {}});
    } else {
        total = stage_from_table<TB, false>(s, rec, a.n_atoms, a.x, a.y, a.z, nullptr, st, CAP,
                                            L.lsrc, mid);
    }
    // per-thread (type_i, type_j) sums of the parameter terms
    double ae[NS], as[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) ae[q] = as[q] = 0.0;
    if (total > CAP) {
        if (threadIdx.x == 0 && a.status) atomicOr(a.status, MD_F_TILE_OVERFLOW);
    } else if (total >= 0) {
        const double gEr = a.gE ? a.gE[s.rep] : 0.0;
        const double rc2 = a.rc * a.rc;
        const int bmax = a.max_nbr / kEntryBlock - 1;
        for (int hk = threadIdx.x; hk < nh; hk += TB) {
            const int i = home_index(hr, hk);
            const double xi = a.x[i], yi = a.y[i], zi = a.z[i];
            const double Gx = a.gfx[i], Gy = a.gfy[i], Gz = a.gfz[i];
            const int ti = NT > 1 ? a.type[i] : 0;
            const int n = min(a.count[i], a.max_nbr);
            const u32x4v *lb = reinterpret_cast<const u32x4v *>(a.idx) + i;
            double ax = 0.0, ay = 0.0, az = 0.0;
            // FP32-mixed: this atom's parameter terms by the neighbour's type
            double pe_t[NT], ps_t[NT];
#pragma unroll
            for (int q = 0; q < NT; ++q) pe_t[q] = ps_t[q] = 0.0;
            const float Gxf = static_cast<float>(Gx), Gyf = static_cast<float>(Gy),
                        Gzf = static_cast<float>(Gz), gErf = static_cast<float>(gEr);
            for (int k = 0; k < n; k += kEntryBlock) {
                const u32x4v blk = lb[size_t(min(k / kEntryBlock, bmax)) * a.ld];
#pragma unroll
                for (int q = 0; q < kEntryBlock; ++q) {
                    const unsigned w = blk[q / 2];
                    const unsigned e = q % 2 ? w >> 16 : w & 0xffffu;
                    // typed entries carry the neighbour's type in the low 3 bits
                    const int slot = min(int(e >> 3), CAP);
                    const double dx = xi - st.x[slot], dy = yi - st.y[slot], dz = zi - st.z[slot];
                    const double r2 = norm2(dx, dy, dz);
                    if (!(r2 < rc2)) continue;   // pad entries never pass
                    const int tj = NT > 1 ? int(e & 7u) : 0;
                    const VjpConst c = tab[ti * kTT + tj];
                    if constexpr (SG) {
                        // the pair term in FP32, its sums in FP64
                        const VjpTermsF v = vjp_terms_f32(c, static_cast<float>(r2));
                        const float dxf = static_cast<float>(dx), dyf = static_cast<float>(dy),
                                    dzf = static_cast<float>(dz);
                        const float fr = c.epsf * v.fr1, dfr = c.epsf * v.dfr1;
                        const float ux = Gxf - L.gx[slot], uy = Gyf - L.gy[slot],
                                    uz = Gzf - L.gz[slot];
                        const float du = fmaf(dxf, ux, fmaf(dyf, uy, dzf * uz));
                        const float t1 = fmaf(dfr, du, -gErf * fr);
                        ax += static_cast<double>(fmaf(fr, ux, t1 * dxf));
                        ay += static_cast<double>(fmaf(fr, uy, t1 * dyf));
                        az += static_cast<double>(fmaf(fr, uz, t1 * dzf));
                        const float pe = fmaf(du, v.fr1, gErf * v.u1);
                        const float ps = c.eosf * fmaf(du, v.dfs1, gErf * v.dus1);
#pragma unroll
                        for (int q = 0; q < NT; ++q)
                            if (q == tj) {
                                pe_t[q] += static_cast<double>(pe);
                                ps_t[q] += static_cast<double>(ps);
                            }
                    } else {
                        const int j = L.lsrc[max(min(slot, total - 1), 0)];
                        const double gjx = a.gfx[j], gjy = a.gfy[j], gjz = a.gfz[j];
                        const VjpTerms v = vjp_terms<PREC>(c, r2);
                        const double fr = c.eps * v.fr1, dfr = c.eps * v.dfr1;
                        const double ux = Gx - gjx, uy = Gy - gjy, uz = Gz - gjz;
                        const double du = dx * ux + dy * uy + dz * uz;
                        const double t1 = dfr * du - gEr * fr;
                        ax += fr * ux + t1 * dx;
                        ay += fr * uy + t1 * dy;
                        az += fr * uz + t1 * dz;
                        const double pe = du * v.fr1 + gEr * v.u1;
                        const double ps = c.eos * (du * v.dfs1 + gEr * v.dus1);
                        const int sl = ti * NT + tj;
#pragma unroll
                        for (int p = 0; p < NS; ++p)
                            if (p == sl) {
                                ae[p] += pe;
                                as[p] += ps;
                            }
                    }
                }
            }
            if constexpr (SG) {
#pragma unroll
                for (int p = 0; p < NS; ++p)
                    if (p / NT == ti) {
                        ae[p] += pe_t[p % NT];
                        as[p] += ps_t[p % NT];
                    }
            }
            a.gx[i] = ax;
            a.gx[a.n_atoms + i] = ay;
            a.gx[2 * size_t(a.n_atoms) + i] = az;
            if (a.status && !isfinite(ax + ay + az)) atomicOr(a.status, MD_F_NONFINITE);
        }
    }
    // per-tile sums: wave totals, one barrier, the waves' totals in wave
    // order; each pair was seen from both of its atoms, hence the halves
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        const double e = wave_sum(ae[q]), g = wave_sum(as[q]);
        if (lane == 0) {
            red[q][wid] = e;
            red[NS + q][wid] = g;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * kAdjSlots) {
        const int kind = threadIdx.x / kAdjSlots, slot = threadIdx.x % kAdjSlots;
        const int ta = slot / kTT, tb = slot % kTT;
        double v = 0.0;
        if (ta < NT && tb < NT)
            for (int w = 0; w < kW; ++w) v += red[kind * NS + ta * NT + tb][w];
        adj[threadIdx.x] = 0.5 * v;
    }
}

// One workgroup per output entry (kind, a, b): fixed-order sum over all
// tiles of slot (a, b), plus slot (b, a) for a != b.
template <class SH>
__global__ __launch_bounds__(kUnit) void k_tile_vjp_finalize(const uint32_t *tile_src, int n_tiles,
                                                             int nt, double *geps, double *gsig)
{
    __shared__ double red[kWavesPerUnit];
    constexpr int kAdj = kTabAdj<TilePlanes<SH::CAP>>;
    const int kind = blockIdx.x / (nt * nt), ab = blockIdx.x % (nt * nt);
    const int ta = ab / nt, tb = ab % nt;
    double sum = 0.0;
    for (int t = threadIdx.x; t < n_tiles; t += kUnit) {
        const double *adj = reinterpret_cast<const double *>(
            tile_src + size_t(t) * tab_stride(SH::CAP) + kAdj) + kind * kAdjSlots;
        sum += ta == tb ? adj[ta * kTT + tb] : adj[ta * kTT + tb] + adj[tb * kTT + ta];
    }
    sum = block_sum(sum, red);
    if (threadIdx.x == 0) {
        double *out = kind == 0 ? geps : gsig;
        if (out) out[ta * nt + tb] = sum;
    }
}

}  // namespace

int tile_vjp(const md_batch *b, const md_atoms *atoms, const md_nlist *nl, const md_lj *p,
             int32_t prec, const double *gfx, const double *gfy, const double *gfz,
             const double *gE, double *gx, double *geps, double *gsig, uint32_t *status,
             hipStream_t s)
{
    TileArgs a = tile_args(b, atoms, nl);
    a.cell_start = nl->cell_start;
    a.eps = p->eps;
    a.sig = p->sig;
    a.shift = p->shift;
    a.rc = p->rc;
    a.gfx = gfx;
    a.gfy = gfy;
    a.gfz = gfz;
    a.gE = gE;
    a.gx = gx;
    a.status = status;
    const dim3 grid(nl->n_tiles);
    const int nt = p->ntypes;
    with_tile_shape([&](auto sh) {
        using SH = decltype(sh);
        const dim3 blk(SH::TB);
        if (prec == MD_FP64) {
            if (nt == 1) hipLaunchKernelGGL((k_tile_vjp<SH, MD_FP64, 1>), grid, blk, 0, s, a);
            else if (nt == 2) hipLaunchKernelGGL((k_tile_vjp<SH, MD_FP64, 2>), grid, blk, 0, s, a);
            else if (nt == 3) hipLaunchKernelGGL((k_tile_vjp<SH, MD_FP64, 3>), grid, blk, 0, s, a);
            else hipLaunchKernelGGL((k_tile_vjp<SH, MD_FP64, 4>), grid, blk, 0, s, a);
        } else {
            if (nt == 1) hipLaunchKernelGGL((k_tile_vjp<SH, MD_FP32_MIXED, 1>), grid, blk, 0, s, a);
            else if (nt == 2)
                hipLaunchKernelGGL((k_tile_vjp<SH, MD_FP32_MIXED, 2>), grid, blk, 0, s, a);
            else if (nt == 3)
                hipLaunchKernelGGL((k_tile_vjp<SH, MD_FP32_MIXED, 3>), grid, blk, 0, s, a);
            else hipLaunchKernelGGL((k_tile_vjp<SH, MD_FP32_MIXED, 4>), grid, blk, 0, s, a);
        }
        if (geps || gsig)
            hipLaunchKernelGGL((k_tile_vjp_finalize<SH>), dim3(2 * nt * nt), dim3(kUnit), 0, s,
                               nl->tile_src, nl->n_tiles, nt, geps, gsig);
    });
    return launch_status();
}

}  // namespace md

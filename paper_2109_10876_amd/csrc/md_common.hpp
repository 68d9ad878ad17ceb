// md_common.hpp -- shared device/host helpers of libmd (gfx950, wave64).
//
// Only the HIP translation units of libmd include this file.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "md.h"

namespace md {

constexpr int kUnit = MD_UNIT_ATOMS;   // atoms per work unit == threads per block
constexpr int kWave = 64;
constexpr int kWavesPerUnit = kUnit / kWave;
constexpr int kXcds = 8;               // MI355X: 8 accelerator complex dies

static_assert(kUnit % kWave == 0, "unit must be whole waves");

// ----------------------------------------------------------------- layout

// Workspace layout (all regions 256-byte aligned).  Counters and the cell
// histogram must be zero between calls; the kernels restore them.
struct WsLayout {
    size_t counters;     // 64 x uint32
    size_t partial;      // n_units x kPartials doubles (per-unit reduction slots)
    size_t cell_count;   // C x int32
    size_t cell_of;      // N x int32
    size_t slot;         // N x int32
    size_t key;          // N (+16 padding: 64-byte reads) x int32
    size_t vjp_partial;  // n_units x 2 x MD_MAX_TYPES^2 doubles
    size_t tile_partial; // C x kTilePartials doubles (tiles never outnumber cells)
    size_t xnext;        // 3 N doubles: next positions of the fused force + step call
    size_t total;
};
constexpr int kPartials = 4;   // E, W, KE, max displacement^2
constexpr int kTilePartials = 4;   // per tile: E, W, KE, max displacement^2

inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

inline WsLayout ws_layout(const md_batch *b)
{
    WsLayout l;
    size_t o = 0;
    l.counters = o;    o = align256(o + 64 * sizeof(uint32_t));
    l.partial = o;     o = align256(o + size_t(b->n_units) * kPartials * sizeof(double));
    l.cell_count = o;  o = align256(o + size_t(b->C) * sizeof(int32_t));
    l.cell_of = o;     o = align256(o + size_t(b->N) * sizeof(int32_t));
    l.slot = o;        o = align256(o + size_t(b->N) * sizeof(int32_t));
    l.key = o;         o = align256(o + (size_t(b->N) + 16) * sizeof(int32_t));   // 64 B reads may pass the end
    l.vjp_partial = o; o = align256(o + size_t(b->n_units) * 2 * MD_MAX_TYPES * MD_MAX_TYPES * sizeof(double));
    l.tile_partial = o; o = align256(o + size_t(b->C) * kTilePartials * sizeof(double));
    l.xnext = o;       o = align256(o + size_t(b->N) * 3 * sizeof(double));
    l.total = o;
    return l;
}

template <typename T>
inline T *ws_at(void *ws, size_t off) { return reinterpret_cast<T *>(static_cast<char *>(ws) + off); }

// Counter slots inside the workspace counter block.
enum Counter : int { kCntForces = 0, kCntVV = 1, kCntVjp = 2 };

// ------------------------------------------------------------- unit mapping

// Hardware dispatch hands workgroup b to XCD (b mod 8).  Remap so each XCD
// receives one contiguous range of work units: neighbouring atoms (and the
// neighbour positions they gather) then stay in one XCD's L2.
__device__ __forceinline__ int xcd_swizzle(int b, int nblocks)
{
    const int x = b % kXcds, k = b / kXcds;
    const int per = nblocks / kXcds, rem = nblocks % kXcds;
    return x * per + (x < rem ? x : rem) + k;
}

// Chunked variant for work laid out in space with holes (tiles over a cell
// grid that may be mostly vacuum): XCD x receives chunks x, x + 8, x + 16, ...
// of C consecutive items, so neighbouring items still share an L2 while any
// occupied band is spread over all XCDs.  Items past the last full round of
// 8 chunks are split contiguously as in xcd_swizzle.  A bijection on [0, n).
__device__ __forceinline__ int xcd_chunked(int b, int n, int C)
{
    const int x = b % kXcds, k = b / kXcds;
    const int full = n / (kXcds * C);
    if (k < full * C) return ((k / C) * kXcds + x) * C + k % C;
    const int base = full * kXcds * C, m = n - base;
    const int per = m / kXcds, rem = m % kXcds;
    return base + x * per + (x < rem ? x : rem) + (k - full * C);
}

struct Unit {
    int rep;    // replica
    int begin;  // first atom of the unit
    int end;    // one past the last atom of the unit
};

__device__ __forceinline__ Unit unit_of(int u, const int32_t *__restrict__ unit_rep,
                                        const int32_t *__restrict__ unit_off,
                                        const int32_t *__restrict__ atom_off)
{
    Unit w;
    w.rep = unit_rep[u];
    const int a0 = atom_off[w.rep], a1 = atom_off[w.rep + 1];
    w.begin = a0 + (u - unit_off[w.rep]) * kUnit;
    w.end = min(w.begin + kUnit, a1);
    return w;
}

// ---------------------------------------------------------------- geometry

// Cell coordinate of a wrapped coordinate w in [0, L): floor(w inv) with
// inv = n / L (cells_per_length), clamped to [0, n-1].  Binning and list
// build both call this with the same stored value and the same inv, so an
// atom is always searched from the cell it was binned into.
__device__ __forceinline__ double cells_per_length(int n, double L)
{
    return static_cast<double>(n) / L;
}
__device__ __forceinline__ int cell_coord(double w, double inv, int n)
{
    int c = static_cast<int>(floor(w * inv));
    return c < 0 ? 0 : (c > n - 1 ? n - 1 : c);
}

// True when the batch is one replica whose rebuild gate is 0: gated
// kernels then leave at once instead of visiting every work unit.
__device__ __forceinline__ bool sole_replica_gated_off(const uint32_t *gate, int R)
{
    return gate != nullptr && R == 1 && gate[0] == 0u;
}

// Wrap x into [0, L); returns the number of box lengths removed.  A
// coordinate already inside [0, L) is returned as is (the general formula
// gives the same value there), so only atoms that left the box pay for the
// division.
__device__ __forceinline__ double wrap_coord(double x, double L, int *shift)
{
    if (x >= 0.0 && x < L) {
        *shift = 0;
        return x;
    }
    double f = floor(x / L);
    double w = x - L * f;
    if (w >= L) { w -= L; f += 1.0; }
    if (w < 0.0) { w += L; f -= 1.0; }
    *shift = static_cast<int>(f);
    return w;
}

// Two-bit image code of s in {0, +1, -1}.
__device__ __forceinline__ uint32_t image_code(int s) { return s == 0 ? 0u : (s > 0 ? 1u : 2u); }
// Inverse: code 0 -> 0, 1 -> +1, 2 -> -1.
__device__ __forceinline__ double image_shift(uint32_t c) { return c == 0u ? 0.0 : (c == 1u ? 1.0 : -1.0); }

// ------------------------------------------------------------- arithmetic

// |(x, y, z)|^2 rounded in one fixed sequence, fma(x, x, fma(y, y, z z)):
// left to itself the compiler picks a contraction per kernel, and kernels
// that must agree bit for bit (a fused step and the split calls, the
// integrator's skin test in both) would then round differently.
__device__ __forceinline__ double norm2(double x, double y, double z)
{
    return fma(x, x, fma(y, y, z * z));
}

// Double-precision reciprocal: hardware estimate refined by two
// Newton-Raphson steps y <- y + y (1 - a y).
__device__ __forceinline__ double rcp_f64(double a)
{
    double y = __builtin_amdgcn_rcp(a);
    y = fma(y, fma(-a, y, 1.0), y);
    y = fma(y, fma(-a, y, 1.0), y);
    return y;
}

// ------------------------------------------------------------- reductions

// Deterministic wave64 sum (fixed butterfly order).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

// Block-level sum over kUnit threads in a fixed order; result valid in
// thread 0.  `lds` must hold kWavesPerUnit doubles.
// Block-wide fixed-order reductions over NT threads (NT a multiple of the
// wave size); the result is valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum_n(double v, double *lds)
{
    v = wave_sum(v);
    if (NT == kWave) return v;
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NT / kWave; ++k) s += lds[k];
    __syncthreads();
    return s;
}
template <int NT>
__device__ __forceinline__ double block_max_n(double v, double *lds)
{
    v = wave_max(v);
    if (NT == kWave) return v;
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double m = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NT / kWave; ++k) m = fmax(m, lds[k]);
    __syncthreads();
    return m;
}

// Threads of the per-replica finalize kernels: each sums every kFin-th
// partial in order (a fixed order for a fixed kFin), several loads in flight.
constexpr int kFin = 1024;

__device__ __forceinline__ double block_sum(double v, double *lds)
{
    v = wave_sum(v);
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kWavesPerUnit; ++k) s += lds[k];
    __syncthreads();
    return s;
}
__device__ __forceinline__ double block_max(double v, double *lds)
{
    v = wave_max(v);
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < kWavesPerUnit; ++k) s = fmax(s, lds[k]);
    __syncthreads();
    return s;
}

// -------------------------------------------------------------- host side

// Tile-local lists (md_tile.hip).
int tile_capacity();
int tile_max_cells();
bool tile_stage_packed();
bool tile_list_ok(const md_batch *b, const md_nlist *nl);
int tile_build(const md_batch *b, const md_atoms *atoms, const int32_t *cell_start, double rl2,
               const md_nlist *nl, int32_t *need, const uint32_t *gate, uint32_t *status,
               hipStream_t s);
// Velocity-Verlet phase 3 (Integrate2 of this step, then Integrate1 of the
// next, as in md_vv_step) applied by the tile force kernel to each home
// atom right after its force: next positions go to xn/yn/zn (the caller's
// second buffer, or workspace copied back once every workgroup has read the
// current ones).
struct VVFuse {
    double *vx, *vy, *vz;
    const double *xb, *yb, *zb;
    const double *inv_mass;
    int32_t ntypes;
    double hdt, dt, lim2;
    double *xn, *yn, *zn;
    double *ke;
    uint32_t *gate;
    // non-null: gate is set to 1 by the workgroups whose atoms moved more
    // than skin/2 (left as it is otherwise) and gate_clear is zeroed, instead
    // of a finaliser writing gate
    uint32_t *gate_clear;
    bool copy_back;   // xn/yn/zn are workspace: copy them into atoms->x/y/z
    // Langevin thermostat (step == nullptr: none)
    const int32_t *id;
    const double *mass;
    double gamma, kT_dt2;   // 2 T / dt
    uint32_t seed_lo, seed_hi;
    uint64_t *step;
};

// chunk_sums: chunk_rows rows of kTilePartials doubles of scratch for the
// two-stage sums of a single replica of many tiles (null: one stage).
int tile_forces(const md_batch *b, const md_atoms *atoms, const md_nlist *nl, const md_lj *p,
                int32_t prec, int32_t accumulate, const int32_t *cell_start, double *energy,
                double *virial, double *tpart, double *chunk_sums, int chunk_rows, int batch,
                const VVFuse *vvf, uint32_t *status, hipStream_t s);

// Adjoint over tile-local lists (md_tile_vjp.hip); arguments as md_lj_forces_vjp.
int tile_vjp(const md_batch *b, const md_atoms *atoms, const md_nlist *nl, const md_lj *p,
             int32_t prec, const double *gfx, const double *gfy, const double *gfz,
             const double *gE, double *gx, double *geps, double *gsig, uint32_t *status,
             hipStream_t s);

// Events around a pair-force kernel launch while md_kernel_timing_start
// asks for them (md_timing.hip): begin returns a slot or -1, end takes it.
int timing_begin(hipStream_t s);
void timing_end(int slot, hipStream_t s);

// md_lj_forces split in two (md_forces.hip): the checks of every argument
// but the workspace, and the launches given the two scratch regions the
// call needs -- partial (n_units rows of kPartials doubles) and, for tile
// lists, tpart (n_tiles rows of kTilePartials doubles).  Every row is written
// before it is read, so neither region needs clearing.
int lj_forces_check(const md_batch *b, const md_atoms *atoms, const md_nlist *nl,
                    const md_lj *p, int32_t prec);
int lj_forces_run(const md_batch *b, const md_atoms *atoms, const md_nlist *nl, const md_lj *p,
                  int32_t prec, int32_t accumulate, double *energy, double *virial,
                  double *partial, double *tpart, uint32_t *status, hipStream_t s);

// Per-replica fixed-order sums of partial slots k0 and k0+1 (md_forces.hip).
void launch_finalize_sum2(int R, const int32_t *unit_off, const double *partial, int k0,
                          double *out0, double *out1, hipStream_t s);

inline hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

// Grid of the kernels that a gate may skip: with a gate, a grid-stride grid
// of at most 1024 workgroups (four per CU), so a skipped call is one short
// launch; without one, a workgroup per unit.
inline int gated_grid(int n_units, bool gated)
{
    return gated ? (n_units < 1024 ? n_units : 1024) : n_units;
}

inline int launch_status()
{
    return hipGetLastError() == hipSuccess ? MD_OK : MD_EHIP;
}

// Host validation of a batch descriptor.
inline int check_batch(const md_batch *b)
{
    if (!b || b->R < 1 || b->N < 1 || b->C < 1 || b->n_units < 1) return MD_EINVAL;
    if (b->N > MD_MAX_ATOMS) return MD_ERANGE;
    if (!b->atom_off || !b->cell_off || !b->ncell || !b->box || !b->unit_rep || !b->unit_off)
        return MD_EINVAL;
    return MD_OK;
}

inline bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

}  // namespace md

// md_build.hip -- md_verlet_build: Verlet neighbour lists from the cell grid.
//
// Sec. 2.1.2 of the paper: atoms are binned into cells of edge at least
// r_cut + r_skin; the candidates of an atom are the atoms of its own cell
// and of the 26 surrounding cells; pairs closer than r_cut + r_skin form the
// Verlet list.  Sec. 3.2 stores the list grouped by the first atom
// ("SortedList": ilist / irange / jlist); here each atom's group is a column
// of an ELL matrix, so that entry k of 64 consecutive atoms is one
// contiguous 256-byte row for the wave that reads it in the force loop.
//
// One thread per atom, atoms in cell order (after md_cell_sort), work units
// remapped so that each XCD walks one contiguous slab of the box.  Candidate
// positions are read from the packed copy when the caller keeps one.  When every
// dimension has at least three cells the periodic image of a neighbour cell
// is a per-cell constant, so the inner loop is a plain difference and one
// distance test per candidate; smaller replicas reduce every candidate by
// the minimum-image rule.
#include "md_common.hpp"

namespace md {
namespace {

struct BuildArgs {
    const int32_t *atom_off, *cell_off, *ncell, *unit_rep, *unit_off;
    const double *box;
    const uint32_t *gate;
    const double *x, *y, *z;
    const double *pos4;
    const int32_t *cell_start;
    double rl2;
    int32_t max_nbr, ld, n_units;
    int32_t *count;
    uint32_t *idx;
    int32_t *need;
    uint32_t *status;
    int32_t R;
};

// Neighbour offsets along one dimension, each distinct cell once:
// n >= 3 -> {-1, 0, +1}; n == 2 -> {0, +1}; n == 1 -> {0}.
__device__ __forceinline__ void offset_range(int n, int &lo, int &hi)
{
    lo = n >= 3 ? -1 : 0;
    hi = n >= 2 ? 1 : 0;
}

constexpr int kCand = 8;   // candidate positions loaded together

template <bool P4>
__device__ __forceinline__ void cand_pos(const BuildArgs &a, int j, double &px, double &py,
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

__device__ __forceinline__ void push(const BuildArgs &a, int i, uint32_t ent, int &cnt)
{
    if (cnt < a.max_nbr) a.idx[size_t(cnt) * a.ld + i] = ent;
    ++cnt;
}

// Candidates [j0, j1) of one neighbour cell whose image is fixed for the cell:
// (xs, ys, zs) is atom i's position moved by that image.  Positions of
// kCand consecutive candidates are loaded together (indices clamped to the
// range, surplus lanes of the batch discarded) so the loads overlap.
template <bool HALF, bool P4>
__device__ __forceinline__ void scan_cell(const BuildArgs &a, int i, double xs, double ys,
                                          double zs, int j0, int j1, uint32_t code, int &cnt)
{
    for (int jb = j0; jb < j1; jb += kCand) {
        double px[kCand], py[kCand], pz[kCand];
#pragma unroll
        for (int q = 0; q < kCand; ++q) cand_pos<P4>(a, min(jb + q, j1 - 1), px[q], py[q], pz[q]);
#pragma unroll
        for (int q = 0; q < kCand; ++q) {
            const int j = jb + q;
            const double dx = xs - px[q], dy = ys - py[q], dz = zs - pz[q];
            const bool take = j < j1 && (HALF ? j > i : j != i) &&
                              norm2(dx, dy, dz) < a.rl2;
            if (take) push(a, i, uint32_t(j) | code, cnt);
        }
    }
}

// Same with the minimum image taken per pair (replicas with fewer than three
// cells along some dimension, where one cell neighbours through both faces).
template <bool HALF, bool P4>
__device__ __forceinline__ void scan_cell_mi(const BuildArgs &a, int i, double xi, double yi,
                                             double zi, const double *L, const double *iL,
                                             int j0, int j1, int &cnt)
{
    for (int jb = j0; jb < j1; jb += kCand) {
        double px[kCand], py[kCand], pz[kCand];
#pragma unroll
        for (int q = 0; q < kCand; ++q) cand_pos<P4>(a, min(jb + q, j1 - 1), px[q], py[q], pz[q]);
#pragma unroll
        for (int q = 0; q < kCand; ++q) {
            const int j = jb + q;
            double dx = xi - px[q], dy = yi - py[q], dz = zi - pz[q];
            const double tx = rint(dx * iL[0]), ty = rint(dy * iL[1]), tz = rint(dz * iL[2]);
            dx -= tx * L[0];
            dy -= ty * L[1];
            dz -= tz * L[2];
            const bool take = j < j1 && (HALF ? j > i : j != i) &&
                              norm2(dx, dy, dz) < a.rl2;
            if (take) {
                const uint32_t code = (image_code(-int(tx)) | (image_code(-int(ty)) << 2) |
                                       (image_code(-int(tz)) << 4)) << MD_IDX_BITS;
                push(a, i, uint32_t(j) | code, cnt);
            }
        }
    }
}

template <bool HALF, bool P4>
__device__ __forceinline__ void build_atom(const BuildArgs &a, const Unit &w, int i)
{
    const double L[3] = {a.box[3 * w.rep], a.box[3 * w.rep + 1], a.box[3 * w.rep + 2]};
    const int nx = a.ncell[3 * w.rep], ny = a.ncell[3 * w.rep + 1], nz = a.ncell[3 * w.rep + 2];
    const int coff = a.cell_off[w.rep];
    const double xi = a.x[i], yi = a.y[i], zi = a.z[i];
    const int cx = cell_coord(xi, cells_per_length(nx, L[0]), nx);
    const int cy = cell_coord(yi, cells_per_length(ny, L[1]), ny);
    const int cz = cell_coord(zi, cells_per_length(nz, L[2]), nz);
    int cnt = 0;

    if (nx >= 3 && ny >= 3 && nz >= 3) {
        // Per-cell image: a neighbour cell reached across a face of the box
        // holds atoms one box length away on the far side.
        for (int oz = -1; oz <= 1; ++oz) {
            int az = cz + oz, sz = 0;
            if (az < 0) { az += nz; sz = 1; } else if (az >= nz) { az -= nz; sz = -1; }
            const double zs = zi + sz * L[2];
            for (int oy = -1; oy <= 1; ++oy) {
                int ay = cy + oy, sy = 0;
                if (ay < 0) { ay += ny; sy = 1; } else if (ay >= ny) { ay -= ny; sy = -1; }
                const double ys = yi + sy * L[1];
                for (int ox = -1; ox <= 1; ++ox) {
                    int ax = cx + ox, sx = 0;
                    if (ax < 0) { ax += nx; sx = 1; } else if (ax >= nx) { ax -= nx; sx = -1; }
                    const double xs = xi + sx * L[0];
                    const uint32_t code = (image_code(sx) | (image_code(sy) << 2) |
                                           (image_code(sz) << 4)) << MD_IDX_BITS;
                    const int c = coff + (az * ny + ay) * nx + ax;
                    scan_cell<HALF, P4>(a, i, xs, ys, zs, a.cell_start[c], a.cell_start[c + 1],
                                        code, cnt);
                }
            }
        }
    } else {
        const double iL[3] = {1.0 / L[0], 1.0 / L[1], 1.0 / L[2]};
        int zlo, zhi, ylo, yhi, xlo, xhi;
        offset_range(nz, zlo, zhi);
        offset_range(ny, ylo, yhi);
        offset_range(nx, xlo, xhi);
        for (int oz = zlo; oz <= zhi; ++oz) {
            const int az = (cz + oz + nz) % nz;
            for (int oy = ylo; oy <= yhi; ++oy) {
                const int ay = (cy + oy + ny) % ny;
                for (int ox = xlo; ox <= xhi; ++ox) {
                    const int ax = (cx + ox + nx) % nx;
                    const int c = coff + (az * ny + ay) * nx + ax;
                    scan_cell_mi<HALF, P4>(a, i, xi, yi, zi, L, iL, a.cell_start[c],
                                           a.cell_start[c + 1], cnt);
                }
            }
        }
    }
    a.count[i] = cnt;
    if (cnt > a.max_nbr) {
        if (a.status) atomicOr(a.status, MD_F_NBR_OVERFLOW);
        if (a.need) atomicMax(a.need, cnt);
    }
}

// Grid-stride over work units (remapped per XCD), so a skipped rebuild
// costs one small launch.
template <bool HALF, bool P4>
__global__ __launch_bounds__(kUnit) void k_build(BuildArgs a)
{
    if (sole_replica_gated_off(a.gate, a.R)) return;
    for (int lb = blockIdx.x; lb < a.n_units; lb += gridDim.x) {
        const int u = xcd_swizzle(lb, a.n_units);
        const Unit w = unit_of(u, a.unit_rep, a.unit_off, a.atom_off);
        if (a.gate != nullptr && a.gate[w.rep] == 0u) continue;
        const int i = w.begin + threadIdx.x;
        if (i < w.end) build_atom<HALF, P4>(a, w, i);
    }
}

}  // namespace
}  // namespace md

extern "C" int md_verlet_build(const md_batch *b, const md_atoms *atoms,
                               const int32_t *cell_start, double rc, double skin,
                               md_nlist *nl, int32_t *need, const uint32_t *gate,
                               uint32_t *status, void *stream)
{
    using namespace md;
    int e = check_batch(b);
    if (e != MD_OK) return e;
    if (!atoms || !atoms->x || !atoms->y || !atoms->z || !cell_start || !nl || !nl->count ||
        !nl->idx)
        return MD_EINVAL;
    if (nl->mode != MD_HALF && nl->mode != MD_FULL && nl->mode != MD_TILE_FULL) return MD_EINVAL;
    if (nl->max_nbr < 1 || nl->ld < b->N || nl->ld % 64 != 0) return MD_EINVAL;
    if (!(rc > 0.0) || !(skin >= 0.0)) return MD_EINVAL;
    if (nl->mode == MD_TILE_FULL) {
        if (!tile_list_ok(b, nl) || nl->cell_start != cell_start) return MD_EINVAL;
        if (nl->tile_types > 1 && !atoms->type) return MD_EINVAL;
        return tile_build(b, atoms, cell_start, (rc + skin) * (rc + skin), nl, need, gate, status,
                          as_stream(stream));
    }
    BuildArgs a{b->atom_off, b->cell_off, b->ncell, b->unit_rep, b->unit_off, b->box, gate,
                atoms->x, atoms->y, atoms->z, atoms->pos4, cell_start,
                (rc + skin) * (rc + skin), nl->max_nbr, nl->ld, b->n_units, nl->count, nl->idx,
                need, status, b->R};
    hipStream_t s = as_stream(stream);
    const dim3 grid(gated_grid(b->n_units, gate != nullptr)), block(kUnit);
    const bool p4 = atoms->pos4 != nullptr;
    if (nl->mode == MD_FULL) {
        if (p4) hipLaunchKernelGGL((k_build<false, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_build<false, false>), grid, block, 0, s, a);
    } else {
        if (p4) hipLaunchKernelGGL((k_build<true, true>), grid, block, 0, s, a);
        else hipLaunchKernelGGL((k_build<true, false>), grid, block, 0, s, a);
    }
    return launch_status();
}

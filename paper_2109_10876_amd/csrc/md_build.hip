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
// remapped so that each XCD walks one contiguous slab of the box.  When every
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
    const int32_t *cell_start;
    double rl2;
    int32_t max_nbr, ld;
    int32_t *count;
    uint32_t *idx;
    int32_t *need;
    uint32_t *status;
};

// Neighbour offsets along one dimension, each distinct cell once:
// n >= 3 -> {-1, 0, +1}; n == 2 -> {0, +1}; n == 1 -> {0}.
__device__ __forceinline__ void offset_range(int n, int &lo, int &hi)
{
    lo = n >= 3 ? -1 : 0;
    hi = n >= 2 ? 1 : 0;
}

template <bool HALF>
__device__ __forceinline__ void push(const BuildArgs &a, int i, int j, uint32_t code, int &cnt)
{
    if (cnt < a.max_nbr) a.idx[size_t(cnt) * a.ld + i] = uint32_t(j) | code;
    ++cnt;
}

template <bool HALF>
__global__ __launch_bounds__(kUnit) void k_build(BuildArgs a)
{
    const int u = xcd_swizzle(blockIdx.x, gridDim.x);
    const Unit w = unit_of(u, a.unit_rep, a.unit_off, a.atom_off);
    if (a.gate != nullptr && a.gate[w.rep] == 0u) return;
    const int i = w.begin + threadIdx.x;
    if (i >= w.end) return;

    const double Lx = a.box[3 * w.rep], Ly = a.box[3 * w.rep + 1], Lz = a.box[3 * w.rep + 2];
    const int nx = a.ncell[3 * w.rep], ny = a.ncell[3 * w.rep + 1], nz = a.ncell[3 * w.rep + 2];
    const int coff = a.cell_off[w.rep];
    const double xi = a.x[i], yi = a.y[i], zi = a.z[i];
    const int cx = cell_coord(xi, Lx, nx), cy = cell_coord(yi, Ly, ny), cz = cell_coord(zi, Lz, nz);
    const double rl2 = a.rl2;
    int cnt = 0;

    if (nx >= 3 && ny >= 3 && nz >= 3) {
        // Per-cell image: a neighbour cell reached across a face of the box
        // holds atoms one box length away on the far side.
        for (int oz = -1; oz <= 1; ++oz) {
            int az = cz + oz, sz = 0;
            if (az < 0) { az += nz; sz = 1; } else if (az >= nz) { az -= nz; sz = -1; }
            const double zs = zi + sz * Lz;
            for (int oy = -1; oy <= 1; ++oy) {
                int ay = cy + oy, sy = 0;
                if (ay < 0) { ay += ny; sy = 1; } else if (ay >= ny) { ay -= ny; sy = -1; }
                const double ys = yi + sy * Ly;
                for (int ox = -1; ox <= 1; ++ox) {
                    int ax = cx + ox, sx = 0;
                    if (ax < 0) { ax += nx; sx = 1; } else if (ax >= nx) { ax -= nx; sx = -1; }
                    const double xs = xi + sx * Lx;
                    const uint32_t code = (image_code(sx) | (image_code(sy) << 2) |
                                           (image_code(sz) << 4)) << MD_IDX_BITS;
                    const int c = coff + (az * ny + ay) * nx + ax;
                    const int j0 = a.cell_start[c], j1 = a.cell_start[c + 1];
                    for (int j = j0; j < j1; ++j) {
                        if (HALF ? (j <= i) : (j == i)) continue;
                        const double dx = xs - a.x[j], dy = ys - a.y[j], dz = zs - a.z[j];
                        if (dx * dx + dy * dy + dz * dz < rl2) push<HALF>(a, i, j, code, cnt);
                    }
                }
            }
        }
    } else {
        // Fewer than three cells along some dimension: the same cell can be a
        // neighbour through either face, so take the minimum image per pair.
        const double ix = 1.0 / Lx, iy = 1.0 / Ly, iz = 1.0 / Lz;
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
                    const int j0 = a.cell_start[c], j1 = a.cell_start[c + 1];
                    for (int j = j0; j < j1; ++j) {
                        if (HALF ? (j <= i) : (j == i)) continue;
                        double dx = xi - a.x[j], dy = yi - a.y[j], dz = zi - a.z[j];
                        const double tx = rint(dx * ix), ty = rint(dy * iy), tz = rint(dz * iz);
                        dx -= tx * Lx;
                        dy -= ty * Ly;
                        dz -= tz * Lz;
                        if (dx * dx + dy * dy + dz * dz < rl2) {
                            const uint32_t code =
                                (image_code(-int(tx)) | (image_code(-int(ty)) << 2) |
                                 (image_code(-int(tz)) << 4)) << MD_IDX_BITS;
                            push<HALF>(a, i, j, code, cnt);
                        }
                    }
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
    if (nl->mode != MD_HALF && nl->mode != MD_FULL) return MD_EINVAL;
    if (nl->max_nbr < 1 || nl->ld < b->N || nl->ld % 64 != 0) return MD_EINVAL;
    if (!(rc > 0.0) || !(skin >= 0.0)) return MD_EINVAL;
    BuildArgs a{b->atom_off, b->cell_off, b->ncell, b->unit_rep, b->unit_off, b->box, gate,
                atoms->x, atoms->y, atoms->z, cell_start, (rc + skin) * (rc + skin),
                nl->max_nbr, nl->ld, nl->count, nl->idx, need, status};
    hipStream_t s = as_stream(stream);
    if (nl->mode == MD_FULL)
        hipLaunchKernelGGL(k_build<false>, dim3(b->n_units), dim3(kUnit), 0, s, a);
    else
        hipLaunchKernelGGL(k_build<true>, dim3(b->n_units), dim3(kUnit), 0, s, a);
    return launch_status();
}

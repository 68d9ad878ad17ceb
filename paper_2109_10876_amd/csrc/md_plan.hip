// md_plan.hip -- host-side planning, workspace sizing and error strings.
//
// The cell grid follows Sec. 2.1.2 of the paper: cubic-ish cells whose edge
// is at least r_cut + r_skin, so that every pair within the Verlet radius
// lies in the same or an adjacent cell.
#include <math.h>

#include "md_common.hpp"

extern "C" {

int md_abi_version(void) { return MD_ABI_VERSION; }

static int32_t g_tune[MD_TUNE_NKNOBS] = {4, 256, 0, 0};

int md_tune_set(int32_t knob, int32_t value)
{
    bool ok = false;
    if (knob == MD_TUNE_PAIR_BATCH) ok = value == 1 || value == 2 || value == 4 || value == 8;
    if (knob == MD_TUNE_TILE_THREADS) ok = value == 64 || value == 128 || value == 256;
    if (knob == MD_TUNE_TILE_STAGE_PACKED) ok = value == 0 || value == 1;
    if (knob == MD_TUNE_TILE_SLOTS)
        ok = value == 0 || value == 1536 || value == 2048 || value == MD_TILE_SLOTS;
    if (!ok) return MD_EINVAL;
    g_tune[knob] = value;
    return MD_OK;
}

int md_tile_capacity(void) { return md::tile_capacity(); }

int md_tile_max_cells(void) { return md::tile_max_cells(); }

int md_tune_get(int32_t knob)
{
    return (knob >= 0 && knob < MD_TUNE_NKNOBS) ? g_tune[knob] : MD_EINVAL;
}

const char *md_strerror(int code)
{
    switch (code) {
    case MD_OK: return "ok";
    case MD_EINVAL: return "invalid argument (null/misaligned pointer, bad count, mode or precision)";
    case MD_EBOX: return "box edge shorter than 2 (rc + skin): minimum image not unique";
    case MD_ENOWS: return "workspace smaller than md_workspace_bytes()";
    case MD_EUNSUPPORTED: return "request not supported by this build";
    case MD_EHIP: return "HIP launch failed";
    case MD_ERANGE: return "size beyond the library's encoding limits";
    case MD_ESCRATCH:
        return "batch needs more scratch than the no-allocation call holds "
               "(MD_NOALLOC_SCRATCH_BYTES)";
    default: return "unknown md error code";
    }
}

static int plan_replica(int32_t n, const double *L, double rc, double skin, int32_t nc[3])
{
    if (n < 1) return MD_EINVAL;
    const double rl = rc + skin;
    for (int d = 0; d < 3; ++d) {
        if (!(L[d] > 0.0) || !isfinite(L[d])) return MD_EINVAL;
        if (L[d] < 2.0 * rl) return MD_EBOX;
        double q = floor(L[d] / rl);
        if (q > 1024.0) return MD_ERANGE;   // at most 2^30 cells per replica
        nc[d] = q < 1.0 ? 1 : static_cast<int32_t>(q);
    }
    return MD_OK;
}

int md_plan_sizes(int32_t R, const int32_t *h_natoms, const double *h_box, double rc,
                  double skin, int32_t *h_N, int32_t *h_C, int32_t *h_n_units)
{
    if (R < 1 || !h_natoms || !h_box || !h_N || !h_C || !h_n_units) return MD_EINVAL;
    if (!(rc > 0.0) || !(skin >= 0.0) || !isfinite(rc) || !isfinite(skin)) return MD_EINVAL;
    int64_t N = 0, C = 0, U = 0;
    for (int32_t r = 0; r < R; ++r) {
        int32_t nc[3];
        int e = plan_replica(h_natoms[r], h_box + 3 * r, rc, skin, nc);
        if (e != MD_OK) return e;
        N += h_natoms[r];
        C += int64_t(nc[0]) * nc[1] * nc[2];
        U += (h_natoms[r] + md::kUnit - 1) / md::kUnit;
        if (N > MD_MAX_ATOMS || C > INT32_MAX / 2) return MD_ERANGE;
    }
    *h_N = static_cast<int32_t>(N);
    *h_C = static_cast<int32_t>(C);
    *h_n_units = static_cast<int32_t>(U);
    return MD_OK;
}

int md_plan_fill(int32_t R, const int32_t *h_natoms, const double *h_box, double rc,
                 double skin, int32_t *h_atom_off, int32_t *h_cell_off, int32_t *h_ncell,
                 int32_t *h_unit_rep, int32_t *h_unit_off)
{
    int32_t N, C, U;
    int e = md_plan_sizes(R, h_natoms, h_box, rc, skin, &N, &C, &U);
    if (e != MD_OK) return e;
    if (!h_atom_off || !h_cell_off || !h_ncell || !h_unit_rep || !h_unit_off) return MD_EINVAL;
    int32_t a = 0, c = 0, u = 0;
    for (int32_t r = 0; r < R; ++r) {
        int32_t nc[3];
        plan_replica(h_natoms[r], h_box + 3 * r, rc, skin, nc);
        h_atom_off[r] = a;
        h_cell_off[r] = c;
        h_unit_off[r] = u;
        for (int d = 0; d < 3; ++d) h_ncell[3 * r + d] = nc[d];
        const int32_t nu = (h_natoms[r] + md::kUnit - 1) / md::kUnit;
        for (int32_t k = 0; k < nu; ++k) h_unit_rep[u + k] = r;
        a += h_natoms[r];
        c += nc[0] * nc[1] * nc[2];
        u += nu;
    }
    h_atom_off[R] = a;
    h_cell_off[R] = c;
    h_unit_off[R] = u;
    return MD_OK;
}

int md_tile_plan(int32_t R, const int32_t *h_ncell, int32_t tile_cells,
                 const int32_t *h_tile_m, int32_t tile_py, int32_t tile_pz,
                 int32_t *h_tile_rep, int32_t *h_tile_off)
{
    if (R < 1 || !h_ncell || tile_cells < 1 || tile_cells > MD_TILE_MAX_CELLS) return MD_EINVAL;
    if (tile_py < 1 || tile_py > MD_TILE_MAX_ROWS || tile_pz < 1 || tile_pz > MD_TILE_MAX_ROWS)
        return MD_EINVAL;
    int64_t t = 0;
    for (int32_t r = 0; r < R; ++r) {
        const int32_t nx = h_ncell[3 * r], ny = h_ncell[3 * r + 1], nz = h_ncell[3 * r + 2];
        if (nx < 1 || ny < 1 || nz < 1) return MD_EINVAL;
        const int32_t m = h_tile_m ? h_tile_m[r] : tile_cells;
        if (m < 1 || m > tile_cells) return MD_EINVAL;
        const int64_t nt = int64_t((ny + tile_py - 1) / tile_py) * ((nz + tile_pz - 1) / tile_pz) *
                           ((nx + m - 1) / m);
        if (h_tile_off) h_tile_off[r] = static_cast<int32_t>(t);
        if (h_tile_rep)
            for (int64_t k = 0; k < nt; ++k) h_tile_rep[t + k] = r;
        t += nt;
        if (t > INT32_MAX / 2) return MD_ERANGE;
    }
    if (h_tile_off) h_tile_off[R] = static_cast<int32_t>(t);
    return static_cast<int>(t);
}

size_t md_workspace_bytes(const md_batch *b)
{
    if (md::check_batch(b) != MD_OK) return 0;
    return md::ws_layout(b).total;
}

}  // extern "C"

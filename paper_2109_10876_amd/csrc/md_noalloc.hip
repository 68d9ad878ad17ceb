// md_noalloc.hip -- md_lj_forces without a workspace argument.
//
// The two scratch regions of md_lj_forces (per-unit and per-tile partial
// sums) are carved out of one fixed device array defined in this file.  Its
// name is a host-side stand-in, not a device address: the array's address on
// each GPU is looked up once, with that GPU current, and only that address is
// handed to the kernels.
#include <mutex>

#include "md_common.hpp"

static __device__ __align__(256) unsigned char scratch[MD_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current GPU (looked up on first use).
int scratch_on_current_device(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return MD_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return MD_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();   // leave no sticky error for the next call
            return MD_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MD_OK;
}

}  // namespace

extern "C" int md_lj_forces_noalloc(const md_batch *b, const md_atoms *atoms,
                                    const md_nlist *nl, const md_lj *p, int32_t prec,
                                    int32_t accumulate, double *energy, double *virial,
                                    uint32_t *status, void *stream)
{
    using namespace md;
    const int e = lj_forces_check(b, atoms, nl, p, prec);
    if (e != MD_OK) return e;
    // partial rows first, then the per-tile rows, each region 256-byte aligned
    const size_t unit_bytes = align256(size_t(b->n_units) * kPartials * sizeof(double));
    const size_t tile_rows = nl->mode == MD_TILE_FULL ? size_t(nl->n_tiles) : 0;
    const size_t tile_bytes = align256(tile_rows * kTilePartials * sizeof(double));
    if (unit_bytes + tile_bytes > size_t(MD_NOALLOC_SCRATCH_BYTES)) return MD_ESCRATCH;
    void *base = nullptr;
    const int se = scratch_on_current_device(&base);
    if (se != MD_OK) return se;
    double *partial = static_cast<double *>(base);
    double *tpart = tile_rows ? ws_at<double>(base, unit_bytes) : nullptr;
    return lj_forces_run(b, atoms, nl, p, prec, accumulate, energy, virial, partial, tpart,
                         status, as_stream(stream));
}

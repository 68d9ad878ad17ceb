// md_timing.hip -- measurement aid: HIP events recorded by the library
// around its pair-force kernel launches (global-index and tile-local, plain
// and fused with the integrator), on the stream each launch uses, so a
// caller can read the kernel's own duration without the launches around it.
#include "md_common.hpp"

namespace md {
namespace {

constexpr int kMaxTimed = 1024;

hipEvent_t g_ev[kMaxTimed][2];
int g_created = 0;   // event pairs created so far (kept for the process)
int g_left = 0;      // launches still to be timed
int g_used = 0;      // pairs recorded since md_kernel_timing_start

}  // namespace

int timing_begin(hipStream_t s)
{
    if (g_left <= 0 || g_used >= kMaxTimed) return -1;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return -1;
    const int k = g_used;
    if (k >= g_created) {
        if (hipEventCreate(&g_ev[k][0]) != hipSuccess) return -1;
        if (hipEventCreate(&g_ev[k][1]) != hipSuccess) {
            (void)hipEventDestroy(g_ev[k][0]);
            return -1;
        }
        ++g_created;
    }
    if (hipEventRecord(g_ev[k][0], s) != hipSuccess) return -1;
    return k;
}

void timing_end(int k, hipStream_t s)
{
    if (k < 0) return;
    if (hipEventRecord(g_ev[k][1], s) != hipSuccess) return;
    ++g_used;
    --g_left;
}

}  // namespace md

extern "C" {

int md_kernel_timing_start(int32_t n)
{
    if (n < 0 || n > md::kMaxTimed) return MD_EINVAL;
    md::g_left = n;
    md::g_used = 0;
    return MD_OK;
}

int md_kernel_timing_read(double *mean_ms, int32_t *count)
{
    if (!mean_ms || !count) return MD_EINVAL;
    double total = 0.0;
    for (int k = 0; k < md::g_used; ++k) {
        float ms = 0.0f;
        if (hipEventSynchronize(md::g_ev[k][1]) != hipSuccess ||
            hipEventElapsedTime(&ms, md::g_ev[k][0], md::g_ev[k][1]) != hipSuccess)
            return MD_EHIP;
        total += ms;
    }
    *count = md::g_used;
    *mean_ms = md::g_used ? total / md::g_used : 0.0;
    return MD_OK;
}

}  // extern "C"

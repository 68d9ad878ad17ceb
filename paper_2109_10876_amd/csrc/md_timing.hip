// md_timing.hip -- measurement aid: HIP events recorded by the library
// around its pair-force kernel launches (global-index and tile-local, plain
// and fused with the integrator), on the stream each launch uses, so a
// caller can read the kernel's own duration without the launches around it.
// Also a streaming copy that gives the achievable HBM bandwidth, the
// denominator of the roofline fraction, and the known-size kernel that
// calibrates the HBM byte counters.
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

// dst = src over n 16-byte words; each thread moves kCopyPer words at a
// stride of one block, so a wave's loads and stores are contiguous 1 KiB runs
// and every thread has kCopyPer loads in flight before its first store.
constexpr int kCopyBlock = 256, kCopyPer = 4;
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kCopyBlock) void k_copy_probe(const u32x4 *__restrict__ src,
                                                           u32x4 *__restrict__ dst, size_t n)
{
    const size_t base = size_t(blockIdx.x) * (kCopyBlock * kCopyPer) + threadIdx.x;
    u32x4 v[kCopyPer];
#pragma unroll
    for (int k = 0; k < kCopyPer; ++k) {
        const size_t i = base + size_t(k) * kCopyBlock;
        if (i < n) v[k] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int k = 0; k < kCopyPer; ++k) {
        const size_t i = base + size_t(k) * kCopyBlock;
        if (i < n) __builtin_nontemporal_store(v[k], dst + i);
    }
}

}  // namespace md

extern "C" {

int md_copy_probe(const void *src, void *dst, size_t bytes, void *stream)
{
    if (!src || !dst || bytes == 0 || bytes % 16 != 0) return MD_EINVAL;
    if (reinterpret_cast<uintptr_t>(src) % 16 != 0 || reinterpret_cast<uintptr_t>(dst) % 16 != 0)
        return MD_EINVAL;
    const size_t n = bytes / 16;
    const size_t per = size_t(md::kCopyBlock) * md::kCopyPer;
    const size_t blocks = (n + per - 1) / per;
    if (blocks > 0x7fffffffu) return MD_ERANGE;
    hipLaunchKernelGGL(md::k_copy_probe, dim3(unsigned(blocks)), dim3(md::kCopyBlock), 0,
                       static_cast<hipStream_t>(stream), static_cast<const md::u32x4 *>(src),
                       static_cast<md::u32x4 *>(dst), n);
    return hipGetLastError() == hipSuccess ? MD_OK : MD_EHIP;
}

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

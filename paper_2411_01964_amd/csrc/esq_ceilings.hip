// Measured ceilings of the device for the rooflines of the segment kernel:
// LDS bandwidth of conflict-free ds_write_b64, ds_read_b64 and ds_or_b32, the
// int32 VALU issue rate of full-rate operations and of the search's funnel
// shift and popcount, and the L2 read bandwidth of 16-byte loads over an
// L2-resident buffer (what the segment init streams from the pattern
// tables), and the HBM write bandwidth of 16-byte stores sweeping a buffer
// far larger than the caches (the bound of the per-n and sieve outputs).
// Each LDS, VALU and L2 microbenchmark runs eight 256-thread workgroups per
// CU (8 waves per SIMD), with the operations in inline assembly where the
// compiler could otherwise remove or merge them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "esq.h"
#include "esq_internal.h"

namespace esq {
namespace ceil {

constexpr uint32_t kCeilBlock = 256;
constexpr uint32_t kCeilLdsBytes = 16384;  // 8 operations x 256 lanes x 8 bytes
constexpr int kCeilings = 8;
constexpr uint32_t kCeilL2Bytes = 1u << 20;  // L2-resident buffer (each XCD's L2 holds 4 MiB)
constexpr size_t kCeilHbmBytes = (size_t)2 << 30;  // write buffer: 8x the last-level cache

// OP 0: ds_write_b64, 1: ds_read_b64, 2: ds_or_b32.  Lane l touches bytes
// 8l .. 8l+7 (4l .. 4l+3 for ds_or_b32) of each 2 KB (1 KB) block, so every
// operation is conflict-free.
template <int OP>
__global__ __launch_bounds__(kCeilBlock) void k_ceil_lds(uint64_t* sink, uint32_t iters)
{
    extern __shared__ uint64_t lds[];
    const uint32_t tid = threadIdx.x;
    uint64_t acc = tid;
    if (OP == 0) {
        const uint32_t a = tid * 8u;
        const uint64_t v = 0x9e3779b97f4a7c15ull * (tid + 1);
        for (uint32_t i = 0; i < iters; i++)
            asm volatile(
                "ds_write_b64 %0, %1\n"
                "ds_write_b64 %0, %1 offset:2048\n"
                "ds_write_b64 %0, %1 offset:4096\n"
                "ds_write_b64 %0, %1 offset:6144\n"
                "ds_write_b64 %0, %1 offset:8192\n"
                "ds_write_b64 %0, %1 offset:10240\n"
                "ds_write_b64 %0, %1 offset:12288\n"
                "ds_write_b64 %0, %1 offset:14336\n"
                :
                : "v"(a), "v"(v)
                : "memory");
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    } else if (OP == 1) {
        lds[tid] = tid;
        __syncthreads();
        const uint32_t a = tid * 8u;
        for (uint32_t i = 0; i < iters; i++) {
            uint64_t r0, r1, r2, r3, r4, r5, r6, r7;
            asm volatile(
                "ds_read_b64 %0, %8\n"
                "ds_read_b64 %1, %8 offset:2048\n"
                "ds_read_b64 %2, %8 offset:4096\n"
                "ds_read_b64 %3, %8 offset:6144\n"
                "ds_read_b64 %4, %8 offset:8192\n"
                "ds_read_b64 %5, %8 offset:10240\n"
                "ds_read_b64 %6, %8 offset:12288\n"
                "ds_read_b64 %7, %8 offset:14336\n"
                "s_waitcnt lgkmcnt(0)\n"
                : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3), "=&v"(r4), "=&v"(r5), "=&v"(r6), "=&v"(r7)
                : "v"(a)
                : "memory");
            acc ^= r0 ^ r1 ^ r2 ^ r3 ^ r4 ^ r5 ^ r6 ^ r7;
        }
    } else {
        const uint32_t a = tid * 4u;
        const uint32_t v = 1u << (tid & 31u);
        for (uint32_t i = 0; i < iters; i++)
            asm volatile(
                "ds_or_b32 %0, %1\n"
                "ds_or_b32 %0, %1 offset:1024\n"
                "ds_or_b32 %0, %1 offset:2048\n"
                "ds_or_b32 %0, %1 offset:3072\n"
                "ds_or_b32 %0, %1 offset:4096\n"
                "ds_or_b32 %0, %1 offset:5120\n"
                "ds_or_b32 %0, %1 offset:6144\n"
                "ds_or_b32 %0, %1 offset:7168\n"
                :
                : "v"(a), "v"(v)
                : "memory");
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    }
    sink[(size_t)blockIdx.x * kCeilBlock + tid] = acc;
}

// 64 independent int32 VALU operations per iteration (eight chains).  OP 0:
// v_add_u32 / v_xor_b32 (full rate); 1: v_alignbit_b32 and 2: v_bcnt_u32_b32,
// the search's funnel shift and popcount.
template <int OP>
__global__ __launch_bounds__(kCeilBlock) void k_ceil_valu(uint64_t* sink, uint32_t iters)
{
    const uint32_t tid = threadIdx.x;
    uint32_t x0 = tid, x1 = tid + 1, x2 = tid + 2, x3 = tid + 3, x4 = tid + 4, x5 = tid + 5, x6 = tid + 6,
             x7 = tid + 7;
    const uint32_t c = 0x9e3779b9u;
    for (uint32_t i = 0; i < iters; i++) {
#pragma unroll
        for (int r = 0; r < 4; r++) {
            if (OP == 1) {
                asm volatile(
                    "v_alignbit_b32 %0, %0, %8, 7\n"
                    "v_alignbit_b32 %1, %1, %8, 7\n"
                    "v_alignbit_b32 %2, %2, %8, 7\n"
                    "v_alignbit_b32 %3, %3, %8, 7\n"
                    "v_alignbit_b32 %4, %4, %8, 7\n"
                    "v_alignbit_b32 %5, %5, %8, 7\n"
                    "v_alignbit_b32 %6, %6, %8, 7\n"
                    "v_alignbit_b32 %7, %7, %8, 7\n"
                    "v_alignbit_b32 %0, %0, %8, 9\n"
                    "v_alignbit_b32 %1, %1, %8, 9\n"
                    "v_alignbit_b32 %2, %2, %8, 9\n"
                    "v_alignbit_b32 %3, %3, %8, 9\n"
                    "v_alignbit_b32 %4, %4, %8, 9\n"
                    "v_alignbit_b32 %5, %5, %8, 9\n"
                    "v_alignbit_b32 %6, %6, %8, 9\n"
                    "v_alignbit_b32 %7, %7, %8, 9\n"
                    : "+v"(x0), "+v"(x1), "+v"(x2), "+v"(x3), "+v"(x4), "+v"(x5), "+v"(x6), "+v"(x7)
                    : "v"(c));
                continue;
            }
            if (OP == 2) {
                asm volatile(
                    "v_bcnt_u32_b32 %0, %0, %8\n"
                    "v_bcnt_u32_b32 %1, %1, %8\n"
                    "v_bcnt_u32_b32 %2, %2, %8\n"
                    "v_bcnt_u32_b32 %3, %3, %8\n"
                    "v_bcnt_u32_b32 %4, %4, %8\n"
                    "v_bcnt_u32_b32 %5, %5, %8\n"
                    "v_bcnt_u32_b32 %6, %6, %8\n"
                    "v_bcnt_u32_b32 %7, %7, %8\n"
                    "v_bcnt_u32_b32 %0, %0, %8\n"
                    "v_bcnt_u32_b32 %1, %1, %8\n"
                    "v_bcnt_u32_b32 %2, %2, %8\n"
                    "v_bcnt_u32_b32 %3, %3, %8\n"
                    "v_bcnt_u32_b32 %4, %4, %8\n"
                    "v_bcnt_u32_b32 %5, %5, %8\n"
                    "v_bcnt_u32_b32 %6, %6, %8\n"
                    "v_bcnt_u32_b32 %7, %7, %8\n"
                    : "+v"(x0), "+v"(x1), "+v"(x2), "+v"(x3), "+v"(x4), "+v"(x5), "+v"(x6), "+v"(x7)
                    : "v"(c));
                continue;
            }
            asm volatile(
                "v_add_u32 %0, %0, %8\n"
                "v_xor_b32 %1, %1, %8\n"
                "v_add_u32 %2, %2, %8\n"
                "v_xor_b32 %3, %3, %8\n"
                "v_add_u32 %4, %4, %8\n"
                "v_xor_b32 %5, %5, %8\n"
                "v_add_u32 %6, %6, %8\n"
                "v_xor_b32 %7, %7, %8\n"
                "v_xor_b32 %0, %0, %8\n"
                "v_add_u32 %1, %1, %8\n"
                "v_xor_b32 %2, %2, %8\n"
                "v_add_u32 %3, %3, %8\n"
                "v_xor_b32 %4, %4, %8\n"
                "v_add_u32 %5, %5, %8\n"
                "v_xor_b32 %6, %6, %8\n"
                "v_add_u32 %7, %7, %8\n"
                : "+v"(x0), "+v"(x1), "+v"(x2), "+v"(x3), "+v"(x4), "+v"(x5), "+v"(x6), "+v"(x7)
                : "v"(c));
        }
    }
    sink[(size_t)blockIdx.x * kCeilBlock + tid] = (uint64_t)(x0 ^ x1 ^ x2 ^ x3 ^ x4 ^ x5 ^ x6 ^ x7);
}

typedef uint32_t u32x4c __attribute__((ext_vector_type(4)));

// 16-byte loads over a 1 MiB buffer: each workgroup reads consecutive 4 KB
// blocks (256 lanes x 16 bytes) from its own start, eight blocks per
// iteration, as the segment init reads consecutive table words.  Every index
// is masked into the buffer.
__global__ __launch_bounds__(kCeilBlock) void k_ceil_l2(const u32x4c* buf, uint64_t* sink, uint32_t iters)
{
    constexpr uint32_t mask = kCeilL2Bytes / 16 - 1;
    const uint32_t tid = threadIdx.x;
    uint32_t base = (blockIdx.x * 8u * kCeilBlock) & mask;
    u32x4c acc = {0u, 0u, 0u, 0u};
    for (uint32_t i = 0; i < iters; i++) {
#pragma unroll
        for (uint32_t r = 0; r < 8; r++)
            acc ^= buf[(base + r * kCeilBlock + tid) & mask];
        base = (base + 8u * kCeilBlock) & mask;
    }
    sink[(size_t)blockIdx.x * kCeilBlock + tid] = (uint64_t)(acc.x ^ acc.y ^ acc.z ^ acc.w);
}

// 16-byte stores over the whole buffer, one per thread: workgroup b writes
// the 4 KB block b, so the grid sweeps the buffer front to back in launch
// order.  Of the store layouts tried (each workgroup streaming its own chunk,
// grid-strided blocks, non-temporal stores, 2 to 16 resident workgroups of
// 256 to 1024 threads per CU, 1 to 16 stores per thread) this one-shot grid
// was the fastest, as fast as a library fill.  The host launches exactly
// kCeilHbmBytes / 4 KB workgroups.
__global__ __launch_bounds__(kCeilBlock) void k_ceil_hbm_write(u32x4c* buf)
{
    const u32x4c v = {threadIdx.x, blockIdx.x, 0x5a5a5a5au, 0u};
    buf[(size_t)blockIdx.x * kCeilBlock + threadIdx.x] = v;
}

}  // namespace ceil
}  // namespace esq

using namespace esq;
using namespace esq::ceil;

extern "C" int esq_measure_ceilings(double* out)
{
    if (!out)
        return ESQ_EINVAL;
    int dev = 0, n_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu <= 0)
        return ESQ_EHIP;
    const uint32_t grid = (uint32_t)n_cu * 8u;
    uint64_t* sink = nullptr;
    u32x4c* l2buf = nullptr;
    u32x4c* hbmbuf = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = ESQ_OK;
    if (hipMalloc(&sink, (size_t)grid * kCeilBlock * sizeof(uint64_t)) != hipSuccess)
        return ESQ_ENOMEM;
    if (hipMalloc(&l2buf, kCeilL2Bytes) != hipSuccess) {
        (void)hipFree(sink);
        return ESQ_ENOMEM;
    }
    if (hipMalloc(&hbmbuf, kCeilHbmBytes) != hipSuccess) {
        (void)hipFree(sink);
        (void)hipFree(l2buf);
        return ESQ_ENOMEM;
    }
    if (hipMemset(l2buf, 0x5a, kCeilL2Bytes) != hipSuccess)
        rc = ESQ_EHIP;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        rc = ESQ_EHIP;
    // bytes (or lane-operations) per launch: per thread per iteration x
    // iterations x threads; the write ceiling is one store per thread
    const uint32_t hbm_grid = (uint32_t)(kCeilHbmBytes / (kCeilBlock * 16));
    const double per_iter[kCeilings] = {64.0, 64.0, 32.0, 64.0, 64.0, 64.0, 128.0, 16.0};
    const uint32_t iters[kCeilings] = {1024, 1024, 1024, 512, 256, 256, 128, 1};
    for (int t = 0; t < kCeilings && rc == ESQ_OK; t++) {
        float best = 0.f;
        for (int rep = 0; rep < 4 && rc == ESQ_OK; rep++) {
            if (hipEventRecord(e0, s) != hipSuccess) {
                rc = ESQ_EHIP;
                break;
            }
            if (t == 0)
                hipLaunchKernelGGL(k_ceil_lds<0>, dim3(grid), dim3(kCeilBlock), kCeilLdsBytes, s, sink, iters[t]);
            else if (t == 1)
                hipLaunchKernelGGL(k_ceil_lds<1>, dim3(grid), dim3(kCeilBlock), kCeilLdsBytes, s, sink, iters[t]);
            else if (t == 2)
                hipLaunchKernelGGL(k_ceil_lds<2>, dim3(grid), dim3(kCeilBlock), kCeilLdsBytes, s, sink, iters[t]);
            else if (t == 3)
                hipLaunchKernelGGL(k_ceil_valu<0>, dim3(grid), dim3(kCeilBlock), 0, s, sink, iters[t]);
            else if (t == 4)
                hipLaunchKernelGGL(k_ceil_valu<1>, dim3(grid), dim3(kCeilBlock), 0, s, sink, iters[t]);
            else if (t == 5)
                hipLaunchKernelGGL(k_ceil_valu<2>, dim3(grid), dim3(kCeilBlock), 0, s, sink, iters[t]);
            else if (t == 6)
                hipLaunchKernelGGL(k_ceil_l2, dim3(grid), dim3(kCeilBlock), 0, s, l2buf, sink, iters[t]);
            else
                hipLaunchKernelGGL(k_ceil_hbm_write, dim3(hbm_grid), dim3(kCeilBlock), 0, s, hbmbuf);
            float ms = 0.f;
            if (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = ESQ_EHIP;
                break;
            }
            if (rep > 0 && (best == 0.f || ms < best))  // the first launch warms up
                best = ms;
        }
        if (rc == ESQ_OK)
            out[t] = per_iter[t] * iters[t] * (double)(t == 7 ? hbm_grid : grid) * kCeilBlock / (best * 1e-3);
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (s)
        (void)hipStreamDestroy(s);
    (void)hipFree(sink);
    (void)hipFree(l2buf);
    (void)hipFree(hbmbuf);
    return rc;
}

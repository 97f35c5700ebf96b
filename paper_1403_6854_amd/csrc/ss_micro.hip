// Measurement kernels: the achievable rates of the MI355X resources the scans
// use, measured on the same device and stream as the scans, so that the walk's
// roofline can be stated against measured peaks instead of data-sheet ones.
//   * HBM stream copy: 16-byte loads and stores, grid-stride;
//   * int32 VALU: eight independent add / xor chains per lane;
//   * LDS atomics: ds_add_u32 on lane-distinct addresses;
//   * cell-update proxy: the minimal operation mix of the bitmask walk's
//     per-marker refinement (a class mask of 4 words ANDed with the marker's
//     row and its complement, population counts, the child kept, C(n, 2)
//     summed), every lane holding a class and streaming over L2-resident rows
//     -- what the walk would reach if every lane of every wave refined a live
//     class at every marker, with no dependency chain between walks.
// Each entry point runs `reps` launches after one warm-up launch, timed with
// HIP events on `stream`, and waits for them.
#include <stdint.h>

#include "selscan_micro.h"
#include "ss_internal.hpp"

namespace {

constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock) copy_kernel(const uint4 *__restrict__ src,
                                                      uint4 *__restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// 8 chains x (add + xor) per iteration: 16 int32 lane-operations.
constexpr int kValuOpsPerIter = 16;
__global__ void __launch_bounds__(kBlock) valu_kernel(uint32_t *__restrict__ out, int iters) {
    uint32_t x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = threadIdx.x * (k + 3u) + blockIdx.x;
    const uint32_t c = blockIdx.x | 1u;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = (x[k] + c) ^ (uint32_t)it;
    }
    uint32_t r = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) r ^= x[k];
    if (r == 0x9E3779B9u) out[blockIdx.x] = r;   // keeps the chains alive; almost never taken
}

__global__ void __launch_bounds__(kBlock) lds_atomic_kernel(uint32_t *__restrict__ out, int iters) {
    __shared__ uint32_t cnt[kBlock];
    cnt[threadIdx.x] = 0u;
    __syncthreads();
    for (int it = 0; it < iters; ++it) atomicAdd(&cnt[threadIdx.x], (uint32_t)it | 1u);
    __syncthreads();
    if (cnt[threadIdx.x] == 0x9E3779B9u) out[blockIdx.x] = cnt[threadIdx.x];
}

// One class per lane as a 4-word mask; every wave streams `rows` marker rows
// (4 words each, the 204-haplotype layout) starting at a row of its own.
constexpr int kCellWords = 4;
__global__ void __launch_bounds__(kBlock) cell_proxy_kernel(const uint64_t *__restrict__ rows,
                                                            int64_t n_rows, int steps,
                                                            uint32_t *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    uint64_t m[kCellWords];
#pragma unroll
    for (int w = 0; w < kCellWords; ++w)
        m[w] = 0x9E3779B97F4A7C15ull * (uint64_t)(lane * kCellWords + w + 1) ^ (uint64_t)wave;
    uint32_t cnt = 0;
#pragma unroll
    for (int w = 0; w < kCellWords; ++w) cnt += (uint32_t)__popcll(m[w]);
    uint32_t S = 0;
    int64_t k = (wave * 97) % n_rows;
    for (int s = 0; s < steps; ++s) {
        const uint64_t *r = rows + k * kCellWords;   // wave-uniform: scalar loads
        uint32_t ones = 0;
        uint64_t m1[kCellWords], m0[kCellWords];
#pragma unroll
        for (int w = 0; w < kCellWords; ++w) {
            m1[w] = m[w] & r[w];
            m0[w] = m[w] & ~r[w];
            ones += (uint32_t)__popcll(m1[w]);
        }
        const uint32_t zeros = cnt - ones;
        const bool keep1 = ones >= zeros;
#pragma unroll
        for (int w = 0; w < kCellWords; ++w) m[w] = keep1 ? m1[w] : m0[w];
        S += ((ones * (ones - 1u)) >> 1) + ((zeros * (zeros - 1u)) >> 1);
        cnt = keep1 ? ones : zeros;
        if (cnt < 2u) {   // a class that died is replaced (keeps every lane busy)
#pragma unroll
            for (int w = 0; w < kCellWords; ++w) m[w] = ~m[w];
            cnt = 64u * kCellWords - cnt;
        }
        k = k + 1 == n_rows ? 0 : k + 1;
    }
    if (S == 0x9E3779B9u) out[wave] = S;
}

int device_cus() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return n;
}

template <typename F>
int timed(F launch, int reps, hipStream_t s, double *ms) {
    if (reps < 1 || !ms) return SS_EARG;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return SS_EDEV;
    int rc = SS_OK;
    launch();   // warm-up
    if (hipGetLastError() != hipSuccess) rc = SS_EDEV;
    if (rc == SS_OK && hipEventRecord(e0, s) != hipSuccess) rc = SS_EDEV;
    for (int r = 0; rc == SS_OK && r < reps; ++r) launch();
    if (rc == SS_OK && hipGetLastError() != hipSuccess) rc = SS_EDEV;
    if (rc == SS_OK && hipEventRecord(e1, s) != hipSuccess) rc = SS_EDEV;
    float t = 0.f;
    if (rc == SS_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess))
        rc = SS_EDEV;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = rc == SS_OK ? (double)t / reps : 0.0;
    return rc;
}

}  // namespace

extern "C" {

int ss_micro_copy(const void *d_src, void *d_dst, size_t bytes, int reps, void *stream, double *ms) {
    if (!d_src || !d_dst || bytes < 16 || bytes % 16 || (uintptr_t)d_src % 16 || (uintptr_t)d_dst % 16)
        return SS_EARG;
    const int64_t n = (int64_t)(bytes / 16);
    const int blocks = device_cus() * 8;
    if (blocks <= 0) return SS_EDEV;
    hipStream_t s = (hipStream_t)stream;
    return timed([&] {
        hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, (const uint4 *)d_src,
                           (uint4 *)d_dst, n);
    }, reps, s, ms);
}

int ss_micro_valu(uint32_t *d_out, int iters, int reps, void *stream, double *ms, double *lane_ops) {
    if (!d_out || iters < 1 || !lane_ops) return SS_EARG;
    const int blocks = device_cus() * 16;   // 16 workgroups of 4 waves per CU: 16 waves per SIMD
    if (blocks <= 0) return SS_EDEV;
    hipStream_t s = (hipStream_t)stream;
    *lane_ops = (double)blocks * kBlock * (double)iters * kValuOpsPerIter;
    return timed([&] {
        hipLaunchKernelGGL(valu_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, d_out, iters);
    }, reps, s, ms);
}

int ss_micro_lds_atomic(uint32_t *d_out, int iters, int reps, void *stream, double *ms, double *ops) {
    if (!d_out || iters < 1 || !ops) return SS_EARG;
    const int blocks = device_cus() * 16;
    if (blocks <= 0) return SS_EDEV;
    hipStream_t s = (hipStream_t)stream;
    *ops = (double)blocks * kBlock * (double)iters;
    return timed([&] {
        hipLaunchKernelGGL(lds_atomic_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, d_out, iters);
    }, reps, s, ms);
}

int ss_micro_cell(const uint64_t *d_rows, int64_t n_rows, uint32_t *d_out, int steps, int reps,
                  void *stream, double *ms, double *cells) {
    if (!d_rows || !d_out || n_rows < 1 || steps < 1 || !cells) return SS_EARG;
    const int blocks = device_cus() * 8;    // 8 workgroups of 4 waves per CU: 8 waves per SIMD
    if (blocks <= 0) return SS_EDEV;
    hipStream_t s = (hipStream_t)stream;
    *cells = (double)blocks * kBlock * (double)steps * 64.0 * kCellWords;
    return timed([&] {
        hipLaunchKernelGGL(cell_proxy_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, d_rows, n_rows,
                           steps, d_out);
    }, reps, s, ms);
}

// Words d_out must hold for any of the kernels above: one per workgroup of
// the VALU and LDS kernels (16 per CU) and one per wave of the cell proxy
// (32 per CU).
int ss_micro_out_words(void) { return 64 * device_cus(); }

}  // extern "C"

// EHH walk kernel over the class-id walk of ss_walk_ids.hpp: one workgroup
// per (core site, direction).
#include "ss_walk_ids.hpp"

namespace ss {

namespace {

template <int MODE, bool TRACE, int R>
__global__ void __launch_bounds__(1024) walk_kernel(WalkArgs a) {
    walk_one<MODE, TRACE, R>(a, a.site0 + (int64_t)blockIdx.x, (int)blockIdx.y);
}

template <int MODE, bool TRACE>
hipError_t launch_r(const WalkArgs &a, const WalkShape &sh, int64_t n_blocks, hipStream_t s) {
    dim3 grid((unsigned)n_blocks, 2u, 1u);
    dim3 block((unsigned)sh.threads, 1u, 1u);
    switch (sh.slots) {
        case 1: hipLaunchKernelGGL((walk_kernel<MODE, TRACE, 1>), grid, block, sh.lds, s, a); break;
        case 2: hipLaunchKernelGGL((walk_kernel<MODE, TRACE, 2>), grid, block, sh.lds, s, a); break;
        case 4: hipLaunchKernelGGL((walk_kernel<MODE, TRACE, 4>), grid, block, sh.lds, s, a); break;
        case 8: hipLaunchKernelGGL((walk_kernel<MODE, TRACE, 8>), grid, block, sh.lds, s, a); break;
        case 16: hipLaunchKernelGGL((walk_kernel<MODE, TRACE, 16>), grid, block, sh.lds, s, a); break;
        case 32: hipLaunchKernelGGL((walk_kernel<MODE, TRACE, 32>), grid, block, sh.lds, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

WalkShape walk_shape(int32_t nA, int32_t nB, int mode) {
    WalkShape sh;
    const int words = (nA + 63) / 64 + (mode == MODE_POOLED ? (nB + 63) / 64 : 0);
    int slots = 1;
    while (slots < words && slots < 16) slots *= 2;
    int waves = (words + slots - 1) / slots;
    if (waves > 16) {   // more than 1024 threads: use more slots per wave
        slots = 32;
        waves = (words + slots - 1) / slots;
    }
    sh.threads = 64 * waves;
    sh.slots = slots;
    const int64_t n = (int64_t)nA + (mode == MODE_POOLED ? nB : 0);
    const int64_t kmax = n / 2 + 2;
    sh.lds = (size_t)(4 * kmax + 8 * kmax + 8 * kmax + 32 + 8 + 8);
    return sh;
}

hipError_t launch_walk(const WalkArgs &a, int mode, bool trace, int64_t n_blocks, hipStream_t s) {
    const WalkShape sh = walk_shape(a.nA, a.nB, mode);
    if (sh.threads > 1024) return hipErrorInvalidConfiguration;
    if (n_blocks <= 0) return hipSuccess;
    if (mode == MODE_CORE) {
        return trace ? launch_r<MODE_CORE, true>(a, sh, n_blocks, s)
                     : launch_r<MODE_CORE, false>(a, sh, n_blocks, s);
    }
    return launch_r<MODE_POOLED, false>(a, sh, n_blocks, s);
}

}  // namespace ss

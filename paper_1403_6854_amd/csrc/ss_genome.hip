// Genome-wide standardization (Sec. 1.2, Eq. 6: iHS scores standardized within
// derived-allele-frequency bins across the whole genome; Sec. 1.3, Eq. 9:
// XPEHH over all loci of the genome): the scores of many scans -- the
// chromosomes of a genome, the regions of a batch, served requests -- are
// standardized together, as one sequence of loci in the order the regions are
// given, instead of each scan on its own.
//
// The caller keeps every scan's per-site outputs in HBM (17 bytes a site), so
// the whole genome's scores are resident: 3 x 10^7 loci are 0.5 GB.  The same
// two passes as the per-scan path, over tiles of 1,024 sites cut from every
// region:
//   pass 1: per tile and bin, count and sum of the OK scores;  per bin, the
//           tiles added in order -> N, mean;
//   pass 2: per tile and bin, sum of squared deviations from the mean; per
//           bin, the tiles added in order -> N-1 standard deviation;
//   pass 3: z = (u - mean) / sd for every scored site, status OK or BIN.
// Sums are taken in a fixed order (lane butterflies, waves, tiles), so the
// results repeat exactly from run to run.  A bin is rebuilt from the scan's
// derived frequency: n1 = rint(freq * n) recovers the derived count exactly
// (freq = n1 / n correctly rounded, n <= 32767), then
// bin = min(floor(B n1 / n), B - 1) in integers, as in the scan.
#include "ss_internal.hpp"

namespace ss {

namespace {

constexpr int kBlock = 256;
constexpr int kTile = 1024;
constexpr int kPer = kTile / kBlock;   // sites per thread

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Region whose tiles contain tile t (regions are ordered by first tile).
__device__ __forceinline__ int region_of_tile(const GenomeRegion *regs, int n, int64_t t) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (regs[mid].tile0 <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Bin of a scored site, -1 for a site that is not scored (status other than
// OK or BIN).
__device__ __forceinline__ int32_t site_bin(const GenomeRegion &r, int64_t j, int32_t nbins) {
    const int8_t st = r.status[j];
    if (st != ST_OK && st != ST_BIN) return -1;
    if (!r.freq) return 0;
    const int64_t n = r.n;
    const int64_t n1 = (int64_t)rint(r.freq[j] * (double)n);
    const int64_t b = ((int64_t)nbins * n1) / n;
    return (int32_t)(b > nbins - 1 ? nbins - 1 : b);
}

__global__ void __launch_bounds__(kBlock) genome_partial_kernel(const GenomeRegion *__restrict__ regs,
                                                                int32_t nreg, int32_t nbins,
                                                                const double *__restrict__ binstat,
                                                                double *__restrict__ part) {
    __shared__ double wpart[kBlock / 64][2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t t = blockIdx.x;
    const GenomeRegion r = regs[region_of_tile(regs, nreg, t)];
    const int64_t j0 = (t - r.tile0) * kTile;
    double uv[kPer];
    int32_t bv[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int64_t j = j0 + threadIdx.x + (int64_t)q * kBlock;
        bv[q] = j < r.M ? site_bin(r, j, nbins) : -1;
        uv[q] = bv[q] >= 0 ? r.u[j] : 0.0;
    }
    for (int b = 0; b < nbins; ++b) {
        const double mean = binstat ? binstat[3 * b + 1] : 0.0;
        double c = 0.0, acc = 0.0;
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            if (bv[q] != b) continue;
            c += 1.0;
            if (binstat) {
                const double dlt = uv[q] - mean;
                acc += dlt * dlt;
            } else {
                acc += uv[q];
            }
        }
        c = wave_sum_f64(c);
        acc = wave_sum_f64(acc);
        if (lane == 0) {
            wpart[wave][0] = c;
            wpart[wave][1] = acc;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double cc = 0.0, aa = 0.0;
            for (int w = 0; w < kBlock / 64; ++w) {
                cc += wpart[w][0];
                aa += wpart[w][1];
            }
            part[(t * nbins + b) * 2 + 0] = cc;
            part[(t * nbins + b) * 2 + 1] = aa;
        }
        __syncthreads();
    }
}

// binstat[b] = {N, mean, sd} from the per-tile sums added in tile order: the
// first pass leaves N and the mean, the second the standard deviation.
__global__ void __launch_bounds__(kBlock) genome_final_kernel(int32_t nbins, int64_t ntiles,
                                                             const double *__restrict__ part,
                                                             int second, double *__restrict__ binstat) {
    const int b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= nbins) return;
    double N = 0.0, acc = 0.0;
    for (int64_t t = 0; t < ntiles; ++t) {
        N += part[(t * nbins + b) * 2 + 0];
        acc += part[(t * nbins + b) * 2 + 1];
    }
    if (!second) {
        binstat[3 * b + 0] = N;
        binstat[3 * b + 1] = N > 0.0 ? acc / N : __builtin_nan("");
    } else {
        binstat[3 * b + 2] = N > 1.0 ? sqrt(acc / (N - 1.0)) : __builtin_nan("");
    }
}

__global__ void __launch_bounds__(kBlock) genome_apply_kernel(const GenomeRegion *__restrict__ regs,
                                                              int32_t nreg, int32_t nbins,
                                                              const double *__restrict__ binstat) {
    const int64_t t = blockIdx.x;
    const GenomeRegion r = regs[region_of_tile(regs, nreg, t)];
    const int64_t j0 = (t - r.tile0) * kTile;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int64_t j = j0 + threadIdx.x + (int64_t)q * kBlock;
        if (j >= r.M) continue;
        const int32_t b = site_bin(r, j, nbins);
        double out = __builtin_nan("");
        if (b >= 0) {
            const double N = binstat[3 * b + 0], mean = binstat[3 * b + 1], sd = binstat[3 * b + 2];
            if (N >= 2.0 && sd > 0.0) {
                out = (r.u[j] - mean) / sd;
                r.status[j] = ST_OK;
            } else {
                r.status[j] = ST_BIN;
            }
        }
        r.z[j] = out;
    }
}

// Descriptors are passed by value, a chunk per launch.
constexpr int kFillChunk = 32;
struct GenomeChunk {
    GenomeRegion r[kFillChunk];
};

__global__ void genome_fill_kernel(GenomeChunk c, int n, GenomeRegion *dst) {
    const int i = threadIdx.x;
    if (i < n) dst[i] = c.r[i];
}

}  // namespace

int64_t genome_tiles(int64_t n_sites) { return (n_sites + kTile - 1) / kTile; }

size_t genome_scratch_doubles(int64_t total_tiles, int32_t nbins) {
    return (size_t)2 * (size_t)total_tiles * (size_t)nbins;
}

hipError_t launch_genome_standardize(const GenomeRegion *host, int32_t nreg, GenomeRegion *dev,
                                     int64_t total_tiles, int32_t nbins, double *binstat,
                                     double *part, hipStream_t s) {
    for (int i = 0; i < nreg; i += kFillChunk) {
        const int m = nreg - i < kFillChunk ? nreg - i : kFillChunk;
        GenomeChunk c;
        for (int q = 0; q < m; ++q) c.r[q] = host[i + q];
        hipLaunchKernelGGL(genome_fill_kernel, dim3(1), dim3(64), 0, s, c, m, dev + i);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (total_tiles <= 0) return hipSuccess;
    const dim3 grid((unsigned)total_tiles), fin((unsigned)((nbins + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(genome_partial_kernel, grid, dim3(kBlock), 0, s, (const GenomeRegion *)dev, nreg,
                       nbins, (const double *)nullptr, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(genome_final_kernel, fin, dim3(kBlock), 0, s, nbins, total_tiles,
                       (const double *)part, 0, binstat);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(genome_partial_kernel, grid, dim3(kBlock), 0, s, (const GenomeRegion *)dev, nreg,
                       nbins, (const double *)binstat, part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(genome_final_kernel, fin, dim3(kBlock), 0, s, nbins, total_tiles,
                       (const double *)part, 1, binstat);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(genome_apply_kernel, grid, dim3(kBlock), 0, s, (const GenomeRegion *)dev, nreg,
                       nbins, (const double *)binstat);
    return hipGetLastError();
}

}  // namespace ss

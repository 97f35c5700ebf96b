// Site-level kernels around the EHH walk: packing, per-site counts and
// filters, the per-site combination of the two walk directions, the
// frequency-bin standardization, and the EHH curves of ss_ehh.
//
// All of these are streaming passes over per-site arrays; they are bound by
// memory traffic and launch latency, not arithmetic, and are laid out for
// coalesced access (one wave per bit-packed row, one lane per site).
#include <math.h>

#include "ss_internal.hpp"

namespace ss {

namespace {

constexpr int kBlock = 256;

// Bit-pack 0/1 bytes (Sec. 1.1 encoding: bit set = derived allele).  A wave
// packs kPackItems consecutive (site, 64-haplotype word) items at a time:
// lane l reads haplotype 64w + l of each (64 consecutive bytes per item), the
// loads of all items in flight together; a ballot per item forms its word,
// and lanes 0 .. kPackItems-1 store the words with one coalesced store.
constexpr int kPackItems = 8;

__global__ void __launch_bounds__(kBlock) pack_kernel(const uint8_t *__restrict__ alleles,
                                                      int64_t n, int64_t M, int64_t wps,
                                                      uint64_t *__restrict__ bits) {
    const int lane = threadIdx.x & 63;
    const int64_t total = M * wps;
    const int64_t stride = (int64_t)gridDim.x * (kBlock / 64) * kPackItems;
    for (int64_t base = ((int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6)) * kPackItems;
         base < total; base += stride) {
        int64_t site = base / wps, w = base - site * wps;
        // every load issued without a condition (a lane past a row's end
        // reads byte 0 and ignores it), so that all are in flight together:
        // loads under a per-lane condition were each waited for before the next
        uint32_t v[kPackItems];
        bool ok[kPackItems];
#pragma unroll
        for (int q = 0; q < kPackItems; ++q) {
            const int64_t h = w * 64 + lane;
            ok[q] = base + q < total && h < n;
            v[q] = alleles[ok[q] ? site * n + h : 0];
            if (++w == wps) {
                w = 0;
                ++site;
            }
        }
        bool one[kPackItems];
#pragma unroll
        for (int q = 0; q < kPackItems; ++q) one[q] = ok[q] && v[q] != 0u;
        uint64_t mine = 0;
#pragma unroll
        for (int q = 0; q < kPackItems; ++q) {
            const uint64_t word = __ballot(one[q]);
            if (lane == q) mine = word;
        }
        if (lane < kPackItems && base + lane < total) bits[base + lane] = mine;
    }
}

// The per-site passes before a walk -- site statistics, the haplotype-major
// copies and the segment lengths -- read different inputs and write
// different outputs, so they run as parts of one launch, each in its own
// range of workgroups; each part is a handful of latency-bound load rounds,
// and in one launch they overlap instead of queueing one after another.

// Haplotype-major copy of the bit matrix for the pairwise phase of the walk:
// row h holds haplotype h's alleles at every site, 64 sites per word, with
// one zero word of padding on each side (word w covers sites 64(w-1) ..
// 64(w-1)+63), so that any 64 consecutive sites are two neighbouring words.
// One wave per (64-site block, 64-haplotype word): lane i loads the word of
// site i of the block, and 64 ballots transpose the 64 x 64 bit block.
__device__ void transpose_part(int64_t blk, int64_t nblk, const uint64_t *__restrict__ bits,
                               int64_t wps, int64_t n, int64_t M, int64_t mwp,
                               uint64_t *__restrict__ hbits) {
    const int lane = threadIdx.x & 63;
    const int64_t words = (n + 63) / 64;
    const int64_t stride = nblk * (kBlock / 64);
    for (int64_t item = blk * (kBlock / 64) + (threadIdx.x >> 6); item < mwp * words;
         item += stride) {
        const int64_t wp = item / words;          // padded block of 64 sites
        const int64_t w = item - wp * words;      // word of 64 haplotypes
        const int64_t site = (wp - 1) * 64 + lane;
        const uint64_t v = (site >= 0 && site < M) ? bits[site * wps + w] : 0ull;
        uint64_t out = 0ull;
        for (int l = 0; l < 64; ++l) {
            const uint64_t col = __ballot(((v >> l) & 1ull) != 0ull);
            if (lane == l) out = col;
        }
        const int64_t h = w * 64 + lane;
        if (h < n) hbits[h * mwp + wp] = out;
    }
}

// Length of every segment between neighbouring sites on the map EHH is
// integrated over (genetic, or physical in bp), with the gap rules of
// Sec. 1.2 applied once per scan instead of once per walk step: seg[k] is the
// length of the segment from site k-1 to site k, scaled by gap_scale / b when
// its physical length b exceeds gap_scale, or -1 when b > max_gap (the walk
// aborts there).  seg[0] is unused.  One lane per site.
__device__ void segment_part(int64_t blk, int64_t M, const int64_t *__restrict__ pos,
                             const double *__restrict__ gpos, int64_t gap_scale, int64_t max_gap,
                             int32_t physical, double *__restrict__ seg) {
    const int64_t k = blk * kBlock + threadIdx.x;
    if (k >= M) return;
    if (k == 0) {
        seg[0] = -1.0;
        return;
    }
    // positions and map read together: the map is used whatever the gap
    // test says, so its reads do not wait for it
    const int64_t b = pos[k] - pos[k - 1];
    const double dg = gpos[k] - gpos[k - 1];
    double g = physical ? (double)b : dg;
    if (b > gap_scale) g = g * ((double)gap_scale / (double)b);
    if (b > max_gap) g = -1.0;
    seg[k] = g;
}

// Per-site derived count n1, derived frequency, frequency bin, MAF filter
// (Sec. 1.2: sites with MAF < cutoff are not scored) and the cores' sizes
// (a core with fewer than two haplotypes leaves the score undefined).
__device__ void site_outputs(int64_t site, int64_t n, int64_t n1, double maf_cutoff, int32_t nbins,
                             double *__restrict__ freq, int32_t *__restrict__ bin,
                             uint8_t *__restrict__ walk_flag, int8_t *__restrict__ status) {
    const int64_t n0 = n - n1;
    freq[site] = (double)n1 / (double)n;
    int64_t b = ((int64_t)nbins * n1) / n;
    if (b > nbins - 1) b = nbins - 1;
    bin[site] = (int32_t)b;
    const double maf = (double)(n0 < n1 ? n0 : n1) / (double)n;
    int8_t st = ST_OK;
    if (maf < maf_cutoff) st = ST_MAF;
    else if (n0 < 2 || n1 < 2) st = ST_UNDEF;
    status[site] = st;
    walk_flag[site] = st == ST_OK ? 1 : 0;
}

// Rows of up to kLaneRowWords words are counted one site per lane (neighbouring
// lanes read neighbouring rows); longer rows one site per wave, a word per lane.
constexpr int64_t kLaneRowWords = 4;

__host__ __device__ inline int64_t site_stats_items(int64_t n, int64_t M) {
    return (n + 63) / 64 <= kLaneRowWords ? (M + 63) / 64 : M;   // waves' worth of work
}

__device__ void site_stats_part(int64_t blk, int64_t nblk, const uint64_t *__restrict__ bits,
                                int64_t wps, int64_t n, int64_t M, double maf_cutoff,
                                int32_t nbins, double *__restrict__ freq,
                                int32_t *__restrict__ bin, uint8_t *__restrict__ walk_flag,
                                int8_t *__restrict__ status) {
    const int lane = threadIdx.x & 63;
    const int64_t words = (n + 63) / 64;
    if (words <= kLaneRowWords) {
        for (int64_t site = blk * kBlock + threadIdx.x; site < M; site += nblk * kBlock) {
            uint32_t c = 0;
            for (int64_t w = 0; w < words; ++w) {
                uint64_t x = bits[site * wps + w];
                const int64_t valid = n - w * 64;
                if (valid < 64) x &= (1ull << valid) - 1ull;
                c += (uint32_t)__popcll(x);
            }
            site_outputs(site, n, c, maf_cutoff, nbins, freq, bin, walk_flag, status);
        }
        return;
    }
    const int64_t stride = nblk * (kBlock / 64);
    for (int64_t site = blk * (kBlock / 64) + (threadIdx.x >> 6); site < M; site += stride) {
        uint32_t c = 0;
        for (int64_t w = lane; w < words; w += 64) {
            uint64_t x = bits[site * wps + w];
            const int64_t valid = n - w * 64;
            if (valid < 64) x &= (1ull << valid) - 1ull;
            c += (uint32_t)__popcll(x);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
        if (lane == 0) site_outputs(site, n, c, maf_cutoff, nbins, freq, bin, walk_flag, status);
    }
}

// Workgroups [0, b_stats) count sites, [b_stats, b_seg) compute segments,
// then one range per haplotype-major copy.
__global__ void __launch_bounds__(kBlock) site_pass_kernel(SitePass p) {
    int64_t blk = blockIdx.x;
    if (blk < p.b_stats) {
        site_stats_part(blk, p.b_stats, p.bits, p.wps, p.n, p.M, p.maf_cutoff, p.nbins, p.freq,
                        p.bin, p.walk_flag, p.status);
        return;
    }
    blk -= p.b_stats;
    if (blk < p.b_seg) {
        segment_part(blk, p.M, p.pos, p.gpos, p.gap_scale, p.max_gap, p.physical, p.seg);
        return;
    }
    blk -= p.b_seg;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        if (blk < p.b_tr[t]) {
            transpose_part(blk, p.b_tr[t], p.tr[t].bits, p.tr[t].wps, p.tr[t].n, p.M, p.mwp,
                           p.tr[t].hbits);
            return;
        }
        blk -= p.b_tr[t];
    }
}

// iHH = downstream sum + upstream sum (Eq. 4 / Eq. 7); the locus status is the
// downstream abort if any, else the upstream one; then the log-ratio
// (Eq. 5 / Eq. 8).
__global__ void __launch_bounds__(kBlock) combine_kernel(
    int64_t M, const uint8_t *__restrict__ walk_flag, const WalkRec *__restrict__ rec,
    double *__restrict__ out_a, double *__restrict__ out_b, double *__restrict__ unstd,
    int8_t *__restrict__ status, int32_t *__restrict__ steps_out, int pooled) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= M) return;
    const double nan = __builtin_nan("");
    // the records are read before the flag, not after it (a site that was not
    // walked reads its slots and ignores them)
    const WalkRec r0 = rec[4 * j + 0], r1 = rec[4 * j + 1], r2 = rec[4 * j + 2], r3 = rec[4 * j + 3];
    const bool walked = walk_flag == nullptr || walk_flag[j] != 0;
    if (!walked) {
        out_a[j] = nan;
        out_b[j] = nan;
        unstd[j] = nan;
        if (steps_out) {
            if (pooled) { steps_out[2 * j] = 0; steps_out[2 * j + 1] = 0; }
            else for (int q = 0; q < 4; ++q) steps_out[4 * j + q] = 0;
        }
        return;   // status already set by the site pass
    }
    // a direction aborts if the walk of either core aborted (iHS walks may be
    // split by core; joint walks write the same status to both slots)
    const int32_t sd = r0.status != ST_OK ? r0.status : r1.status;
    const int32_t su = r2.status != ST_OK ? r2.status : r3.status;
    int32_t st = sd != ST_OK ? sd : su;
    // slot 0 of a direction holds core 0 (iHS) or population A (XPEHH),
    // slot 1 holds core 1 or population B
    const double x0 = r0.ihh + r2.ihh;
    const double x1 = r1.ihh + r3.ihh;
    double a = nan, b = nan, u = nan;
    if (st == ST_OK) {
        if (!(x0 > 0.0) || !(x1 > 0.0)) {
            st = ST_UNDEF;
        } else if (pooled) {
            a = x0;
            b = x1;
            u = log(a / b);
        } else {
            a = x1;   // iHH_1 (derived)
            b = x0;   // iHH_0 (ancestral)
            u = log(a / b);
        }
    }
    out_a[j] = a;
    out_b[j] = b;
    unstd[j] = u;
    status[j] = (int8_t)st;
    if (steps_out) {
        if (pooled) {
            steps_out[2 * j] = r0.steps;
            steps_out[2 * j + 1] = r2.steps;
        } else {
            steps_out[4 * j + 0] = r0.steps;
            steps_out[4 * j + 1] = r1.steps;
            steps_out[4 * j + 2] = r2.steps;
            steps_out[4 * j + 3] = r3.steps;
        }
    }
}

// Frequency-bin statistics (Eq. 6; Eq. 9 with one bin): count, mean and N-1
// standard deviation of the OK scores of each bin, in two passes like the
// definition (mean first, then squared deviations from it).  Sites are cut
// into tiles of kTile, one per workgroup; each thread holds kTile / kBlock
// sites, and for every bin the workgroup sums them with fixed-order wave
// reductions; the per-tile partial sums are then added in tile order.  The
// summation order is fixed, so results are identical from run to run.
constexpr int kTile = 1024;

// Lane value moved by a DPP row operation, the two halves of the double one
// after the other (lanes the operation does not write, or that read from
// outside their row with bound_ctrl, get +0.0).
template <int CTRL, int ROW_MASK, bool BC>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t x = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, CTRL, ROW_MASK, 0xF, BC);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), CTRL, ROW_MASK,
                                                              0xF, BC);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over the 64 lanes of a wave, in every lane: an inclusive scan in DPP
// register moves (within each row of 16 lanes by shifts of 1, 2, 4 and 8,
// then row 0's total into row 1 and row 2's into row 3, then rows 0-1 into
// rows 2-3), whose last lane holds the total.  The butterfly of lane
// permutes it replaces went through LDS at every step.
__device__ __forceinline__ double wave_sum_f64(double v) {
    v += dpp_f64<0x111, 0xF, true>(v);    // row_shr:1
    v += dpp_f64<0x112, 0xF, true>(v);    // row_shr:2
    v += dpp_f64<0x114, 0xF, true>(v);    // row_shr:4
    v += dpp_f64<0x118, 0xF, true>(v);    // row_shr:8
    v += dpp_f64<0x142, 0xA, false>(v);   // row_bcast:15
    v += dpp_f64<0x143, 0xC, false>(v);   // row_bcast:31
    const uint64_t x = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)x, 63);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(x >> 32), 63);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__global__ void __launch_bounds__(kBlock) bin_partial_kernel(
    int64_t M, const double *__restrict__ u, const int8_t *__restrict__ status,
    const int32_t *__restrict__ bin, int32_t nbins, int64_t ntiles,
    const double *__restrict__ binstat, double *__restrict__ part) {
    constexpr int kPer = kTile / kBlock;   // sites per thread
    __shared__ double wpart[kBlock / 64][2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t t0 = (int64_t)blockIdx.x * kTile;
    double uv[kPer];
    int32_t bv[kPer], sv[kPer];
    // all loads issued at once, without per-lane conditions (a lane past the
    // end reads site 0 and ignores it)
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int64_t jj = t0 + threadIdx.x + (int64_t)q * kBlock;
        const int64_t jc = jj < M ? jj : 0;
        sv[q] = status[jc];
        bv[q] = bin ? bin[jc] : 0;
        uv[q] = u[jc];
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const bool ok = t0 + threadIdx.x + (int64_t)q * kBlock < M && sv[q] == ST_OK;
        if (!ok) {
            bv[q] = -1;
            uv[q] = 0.0;
        }
    }
    for (int b = 0; b < nbins; ++b) {
        // second pass: squared deviations from the bin's mean
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
            part[((int64_t)blockIdx.x * nbins + b) * 2 + 0] = cc;
            part[((int64_t)blockIdx.x * nbins + b) * 2 + 1] = aa;
        }
        __syncthreads();
    }
}

// binstat[b] = {N, mean, sd}: after the first pass N and the mean, after the
// second pass the standard deviation, from the per-tile partial sums added in
// tile order.
__global__ void __launch_bounds__(kBlock) bin_final_kernel(int32_t nbins, int64_t ntiles,
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

__global__ void __launch_bounds__(kBlock) standardize_kernel(int64_t M,
                                                             const double *__restrict__ u,
                                                             int8_t *__restrict__ status,
                                                             const int32_t *__restrict__ bin,
                                                             const double *__restrict__ binstat,
                                                             double *__restrict__ z) {
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= M) return;
    // the site's score, status and bin read together, not one after another
    const double uj = u[j];
    const int8_t st = status[j];
    const int b = bin ? bin[j] : 0;
    double out = __builtin_nan("");
    if (st == ST_OK) {
        const double N = binstat[3 * b + 0], mean = binstat[3 * b + 1], sd = binstat[3 * b + 2];
        if (N >= 2.0 && sd > 0.0) out = (uj - mean) / sd;
        else status[j] = ST_BIN;
    }
    z[j] = out;
}

// Regions of up to kFusedMaxSites sites with kFusedMinBins to kFusedMaxBins
// bins: one workgroup per bin takes three steps over the region's sites --
// count and sum of the bin's OK scores, their squared deviations from the
// mean, then the bin's z-scores -- so the five launches of the tiled path
// above become one.  (With fewer bins too few workgroups share the work, and the tiled path
// is faster.)  Each thread accumulates its sites in site order and the block
// combines the threads in a fixed tree, so the results repeat exactly from run
// to run.
constexpr int kFusedBlock = 1024;
constexpr int64_t kFusedMaxSites = (int64_t)1 << 16;
constexpr int32_t kFusedMinBins = 8, kFusedMaxBins = 256;

__device__ __forceinline__ double block_sum_f64(double v, double *red) {
    v = wave_sum_f64(v);
    __syncthreads();   // red is no longer read by an earlier sum
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kFusedBlock / 64; ++w) t += red[w];
    return t;
}

// Eight sites per thread per round, their loads issued together.
constexpr int kFusedUnroll = 8;
constexpr int64_t kFusedRound = (int64_t)kFusedUnroll * kFusedBlock;
// Regions of up to kFusedMaxRounds rounds keep their sites in registers
// (kFusedMaxRounds * kFusedUnroll doubles per thread): the three steps then
// share one read of global memory (bins and statuses, then the bin's OK
// scores) instead of reading the sites once per step.
constexpr int kFusedMaxRounds = 4;
static_assert(kFusedMaxRounds * kFusedUnroll <= 32, "held sites are flagged in 32-bit masks");

// R > 0: the region's sites (at most R rounds) held in registers; R = 0: each
// step reads them again.  Both accumulate in the same order (rounds, then the
// eight sites of a round), so they give identical results.
template <int R>
__global__ void __launch_bounds__(kFusedBlock) bin_fused_kernel(int64_t M,
                                                                const double *__restrict__ u,
                                                                int8_t *__restrict__ status,
                                                                const int32_t *__restrict__ bin,
                                                                double *__restrict__ binstat,
                                                                double *__restrict__ z) {
    __shared__ double red[kFusedBlock / 64];
    const int b = (int)blockIdx.x;
    constexpr int kHeld = R > 0 ? R * kFusedUnroll : 1;
    double held[kHeld];
    uint32_t inbin = 0, okbin = 0;   // R > 0: bit r * 8 + q of the held sites
    // held slot i = r * 8 + q: site q of round r (32-bit: fused regions hold
    // at most 2^16 sites).  Accesses add threadIdx.x to a wave-uniform base,
    // which keeps one address register per array instead of one per slot.
    auto held_site = [&](int i) -> uint32_t {
        return threadIdx.x + (uint32_t)((i / kFusedUnroll) * kFusedRound + (i % kFusedUnroll) * kFusedBlock);
    };
    // OK scores of bin b among the round's sites of this thread (site order)
    // (Sites past the end read site 0 and are then ignored: loads under a
    // per-lane condition were each waited for before the next was issued.)
    auto load = [&](int64_t j0, bool (&in)[kFusedUnroll], double (&uu)[kFusedUnroll]) {
        int32_t bj[kFusedUnroll];
        int32_t st[kFusedUnroll];
#pragma unroll
        for (int q = 0; q < kFusedUnroll; ++q) {
            const int64_t j = j0 + (int64_t)q * kFusedBlock;
            const int64_t jc = j < M ? j : 0;
            bj[q] = bin ? bin[jc] : 0;
            st[q] = status[jc];
            uu[q] = u[jc];
        }
#pragma unroll
        for (int q = 0; q < kFusedUnroll; ++q) {
            const bool inr = j0 + (int64_t)q * kFusedBlock < M;
            in[q] = inr && bj[q] == b && st[q] == ST_OK;
            if (!inr) uu[q] = 0.0;
        }
    };
    double c = 0.0, sum = 0.0;
    if (R > 0) {
        // bins and statuses of the held sites first, then the scores of the
        // bin's OK sites only: two loads in flight per site at a time
        // every load issued without a condition (a lane past the end reads
        // site 0 and ignores it), so that all are in flight together: loads
        // under a per-lane condition were each waited for before the next
        int32_t bjv[kHeld], stv[kHeld];
#pragma unroll
        for (int i = 0; i < kHeld; ++i) {
            const uint32_t j = held_site(i), j0 = j - threadIdx.x;
            const int32_t off = j < (uint32_t)M ? (int32_t)threadIdx.x : -(int32_t)j0;
            bjv[i] = bin ? (bin + j0)[off] : 0;
            stv[i] = (status + j0)[off];
        }
#pragma unroll
        for (int i = 0; i < kHeld; ++i) {
            const bool inr = held_site(i) < (uint32_t)M;
            if (inr && bjv[i] == b) inbin |= 1u << i;
            if (inr && bjv[i] == b && stv[i] == ST_OK) okbin |= 1u << i;
        }
#pragma unroll
        for (int i = 0; i < kHeld; ++i) {
            const double *ui = u + (held_site(i) - threadIdx.x);
            held[i] = ((okbin >> i) & 1u) ? ui[threadIdx.x] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < kHeld; ++i) {
            if ((okbin >> i) & 1u) {
                c += 1.0;
                sum += held[i];
            }
        }
    } else {
        for (int64_t j0 = threadIdx.x; j0 < M; j0 += kFusedRound) {
            bool in[kFusedUnroll];
            double uu[kFusedUnroll];
            load(j0, in, uu);
#pragma unroll
            for (int q = 0; q < kFusedUnroll; ++q) {
                if (in[q]) {
                    c += 1.0;
                    sum += uu[q];
                }
            }
        }
    }
    const double N = block_sum_f64(c, red);
    const double S = block_sum_f64(sum, red);
    const double mean = N > 0.0 ? S / N : __builtin_nan("");
    double sq = 0.0;
    if (R > 0) {
#pragma unroll
        for (int i = 0; i < kHeld; ++i) {
            if ((okbin >> i) & 1u) {
                const double dlt = held[i] - mean;
                sq += dlt * dlt;
            }
        }
    } else {
        for (int64_t j0 = threadIdx.x; j0 < M; j0 += kFusedRound) {
            bool in[kFusedUnroll];
            double uu[kFusedUnroll];
            load(j0, in, uu);
#pragma unroll
            for (int q = 0; q < kFusedUnroll; ++q) {
                if (in[q]) {
                    const double dlt = uu[q] - mean;
                    sq += dlt * dlt;
                }
            }
        }
    }
    const double Q = block_sum_f64(sq, red);
    const double sd = N > 1.0 ? sqrt(Q / (N - 1.0)) : __builtin_nan("");
    if (threadIdx.x == 0) {
        binstat[3 * b + 0] = N;
        binstat[3 * b + 1] = mean;
        binstat[3 * b + 2] = sd;
    }
    const bool good = N >= 2.0 && sd > 0.0;
    if (R > 0) {
#pragma unroll
        for (int i = 0; i < kHeld; ++i) {
            if (!((inbin >> i) & 1u)) continue;
            const uint32_t j0 = held_site(i) - threadIdx.x;
            double out = __builtin_nan("");
            if ((okbin >> i) & 1u) {
                if (good) out = (held[i] - mean) / sd;
                else (status + j0)[threadIdx.x] = ST_BIN;
            }
            (z + j0)[threadIdx.x] = out;
        }
        return;
    }
    for (int64_t j0 = threadIdx.x; j0 < M; j0 += kFusedRound) {
        int32_t bj[kFusedUnroll];
        int8_t st[kFusedUnroll];
        double uu[kFusedUnroll];
#pragma unroll
        for (int q = 0; q < kFusedUnroll; ++q) {
            const int64_t j = j0 + (int64_t)q * kFusedBlock;
            const bool inr = j < M;
            bj[q] = inr ? (bin ? bin[j] : 0) : -1;
            st[q] = inr ? status[j] : (int8_t)ST_MAF;
            uu[q] = inr ? u[j] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < kFusedUnroll; ++q) {
            if (bj[q] != b) continue;
            const int64_t j = j0 + (int64_t)q * kFusedBlock;
            double out = __builtin_nan("");
            if (st[q] == ST_OK) {
                if (good) out = (uu[q] - mean) / sd;
                else status[j] = ST_BIN;
            }
            z[j] = out;
        }
    }
}

// ss_ehh epilogue: EHH curves from the traced integer sums (S_c at x0 is
// C(n_c, 2), the denominator of Eq. 3), iHH = downstream + upstream, status.
__global__ void ehh_finish_kernel(int64_t n, int64_t cap, const uint64_t *__restrict__ S,
                                  const int64_t *__restrict__ len,
                                  const WalkRec *__restrict__ rec, double *__restrict__ ehh,
                                  double *__restrict__ ihh, int8_t *__restrict__ status) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double nan = __builtin_nan("");
    const double Pall = (double)(n * (n - 1) / 2);
    if (t < 2 * (cap + 1)) {
        const int64_t d = t / (cap + 1), i = t - d * (cap + 1);
        const uint64_t *Sd = S + (size_t)d * (cap + 1) * 2;
        double *e = ehh + (size_t)t * 3;
        if (i <= len[d]) {
            const double P0 = (double)Sd[0], P1 = (double)Sd[1];
            e[0] = (double)Sd[2 * i + 0] / P0;
            e[1] = (double)Sd[2 * i + 1] / P1;
            e[2] = (double)(Sd[2 * i + 0] + Sd[2 * i + 1]) / Pall;
        } else {
            e[0] = e[1] = e[2] = nan;
        }
    }
    if (t == 0) {
        int32_t st = rec[0].status != ST_OK ? rec[0].status : rec[2].status;   // downstream, upstream
        const bool small = S[0] == 0 || S[1] == 0;   // C(n_c, 2) = 0: n_c < 2
        if (st == ST_OK && small) st = ST_UNDEF;
        double i0 = nan, i1 = nan;
        if (st == ST_OK) {
            i0 = rec[0].ihh + rec[2].ihh;
            i1 = rec[1].ihh + rec[3].ihh;
            if (!(i0 > 0.0) || !(i1 > 0.0)) {
                st = ST_UNDEF;
                i0 = i1 = nan;
            }
        }
        ihh[0] = i0;
        ihh[1] = i1;
        status[0] = (int8_t)st;
    }
}

}  // namespace

// Grids of the wave-per-item kernels are capped (they loop over their items):
// one launch may not exceed 2^32 work items in x.
constexpr int64_t kMaxBlocks = 1 << 20;

static int64_t wave_blocks(int64_t items) {
    const int64_t b = (items + kBlock / 64 - 1) / (kBlock / 64);
    return b < kMaxBlocks ? (b > 0 ? b : 1) : kMaxBlocks;
}

hipError_t launch_pack(const uint8_t *alleles, int64_t n, int64_t M, int64_t wps,
                       uint64_t *bits, hipStream_t s) {
    const int64_t blocks = wave_blocks((M * wps + kPackItems - 1) / kPackItems);
    hipLaunchKernelGGL(pack_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, alleles, n, M,
                       wps, bits);
    return hipGetLastError();
}

hipError_t launch_site_pass(SitePass p, hipStream_t s) {
    p.b_stats = p.bits ? wave_blocks(site_stats_items(p.n, p.M)) : 0;
    p.b_seg = (p.M + kBlock - 1) / kBlock;
    for (int t = 0; t < 2; ++t)
        p.b_tr[t] = p.tr[t].hbits ? wave_blocks(p.mwp * ((p.tr[t].n + 63) / 64)) : 0;
    const int64_t blocks = p.b_stats + p.b_seg + p.b_tr[0] + p.b_tr[1];
    if (blocks <= 0) return hipSuccess;
    if (blocks >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(site_pass_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_combine(int mode, int64_t M, const uint8_t *walk_flag, const WalkRec *rec,
                          double *out_a,
                          double *out_b, double *unstd, int8_t *status, int32_t *steps_out,
                          hipStream_t s) {
    const int64_t blocks = (M + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(combine_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, M, walk_flag,
                       rec, out_a, out_b, unstd, status, steps_out,
                       mode == MODE_POOLED ? 1 : 0);
    return hipGetLastError();
}

int64_t standardize_scratch_doubles(int64_t M, int32_t nbins) {
    const int64_t ntiles = (M + kTile - 1) / kTile;
    return 2 * 2 * ntiles * (int64_t)nbins;
}

hipError_t launch_standardize(int64_t M, const double *unstd, int8_t *status, const int32_t *bin,
                              int32_t nbins, double *binstat, double *scratch, double *z,
                              hipStream_t s) {
    if (M <= kFusedMaxSites && nbins >= kFusedMinBins && nbins <= kFusedMaxBins) {
        const dim3 grid((unsigned)nbins), block(kFusedBlock);
        static_assert(kFusedMaxRounds == 4, "one case per round count below");
        switch ((M + kFusedRound - 1) / kFusedRound) {
            case 1: hipLaunchKernelGGL(bin_fused_kernel<1>, grid, block, 0, s, M, unstd, status, bin, binstat, z); break;
            case 2: hipLaunchKernelGGL(bin_fused_kernel<2>, grid, block, 0, s, M, unstd, status, bin, binstat, z); break;
            case 3: hipLaunchKernelGGL(bin_fused_kernel<3>, grid, block, 0, s, M, unstd, status, bin, binstat, z); break;
            case 4: hipLaunchKernelGGL(bin_fused_kernel<4>, grid, block, 0, s, M, unstd, status, bin, binstat, z); break;
            default: hipLaunchKernelGGL(bin_fused_kernel<0>, grid, block, 0, s, M, unstd, status, bin, binstat, z); break;
        }
        return hipGetLastError();
    }
    const int64_t ntiles = (M + kTile - 1) / kTile;
    double *first = scratch;
    double *second = scratch + 2 * ntiles * (int64_t)nbins;
    const dim3 fin((unsigned)((nbins + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(bin_partial_kernel, dim3((unsigned)ntiles), dim3(kBlock), 0, s, M, unstd,
                       status, bin, nbins, ntiles, (const double *)nullptr, first);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bin_final_kernel, fin, dim3(kBlock), 0, s, nbins, ntiles,
                       (const double *)first, 0, binstat);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(bin_partial_kernel, dim3((unsigned)ntiles), dim3(kBlock), 0, s, M, unstd,
                       status, bin, nbins, ntiles, (const double *)binstat, second);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(bin_final_kernel, fin, dim3(kBlock), 0, s, nbins, ntiles,
                       (const double *)second, 1, binstat);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t blocks = (M + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(standardize_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, M, unstd,
                       status, bin, binstat, z);
    return hipGetLastError();
}

hipError_t launch_ehh_finish(int64_t n, int64_t cap, const uint64_t *S, const int64_t *len,
                             const WalkRec *rec, double *ehh,
                             double *ihh, int8_t *status, hipStream_t s) {
    const int64_t items = 2 * (cap + 1);
    const int64_t blocks = (items + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(ehh_finish_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, n, cap, S,
                       len, rec, ehh, ihh, status);
    return hipGetLastError();
}

}  // namespace ss

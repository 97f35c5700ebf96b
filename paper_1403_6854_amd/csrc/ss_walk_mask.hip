// EHH walk with the partition held as per-class haplotype bitmasks in
// registers: one wave per (core site, direction), one class per lane (and
// per slot when there can be more than 64 classes).  Used for haplotype
// counts up to 512 (pooled, for XPEHH).
//
// What it computes is the same partition refinement as ss_walk.hip
// (Sec. 1.1, Eqs. 1-3: classes of identical haplotypes from x0 out to x_i;
// Sec. 1.2, Eq. 4 and the rules below it; Sec. 1.3, Eq. 7 for the pooled
// walk of XPEHH); only the representation differs:
//   * class c is a bitmask over the haplotypes (W 64-bit words, marker-major
//     packing) held by lane c % 64 in slot c / 64.  Splitting a class by the
//     alleles at marker k is an AND with row k and a popcount, so a marker
//     costs a few VALU instructions per word for all classes at once, with no
//     LDS traffic and no barrier;
//   * the child with the allele-1 members stays in place if it has >= 2
//     members, else the allele-0 child; when both children survive, the
//     second one is appended through LDS (a rare event once the first few
//     markers have separated the founder groups);
//   * the stop test EHH_c = S_c / C(n_c,2) < cutoff is evaluated on integers:
//     correctly rounded division is monotone in S, so fl(S/P) < cutoff holds
//     exactly for S <= thr, with thr found once per walk by testing 64
//     candidates around cutoff * P with the same IEEE division;
//   * the FP64 trapezoid terms of 64 markers are formed lane-parallel after
//     the markers have been refined, and added to iHH one by one in marker
//     order, so the sums round exactly as the definition's left-to-right sum.
#include "ss_internal.hpp"

namespace ss {

namespace {

__device__ __forceinline__ uint32_t choose2(uint32_t x) { return (x * (x - 1u)) >> 1; }

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) { return __ockl_wfred_add_u32(v); }

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int i) {
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, i);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), i);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ double readlane_f64(double v, int i) {
    return __builtin_bit_cast(double, readlane64(__builtin_bit_cast(uint64_t, v), i));
}

// Largest S in [0, P] with (double)S / (double)P < cutoff (P >= 1), found by
// testing 64 consecutive candidates around cutoff * P, one per lane.
__device__ __forceinline__ uint32_t stop_threshold(uint32_t P, double cutoff, int lane) {
    const double Pd = (double)P;
    int64_t c0 = (int64_t)(cutoff * Pd) - 32;
    int64_t s = c0 + lane;
    if (s < 0) s = 0;
    if (s > (int64_t)P) s = (int64_t)P;
    const bool below = (double)s / Pd < cutoff;
    const uint64_t m = __ballot(below);
    const int top = 63 - __builtin_clzll(m);   // m != 0: candidate 0 or c0 is always below
    return (uint32_t)__builtin_amdgcn_readlane((uint32_t)s, top);
}

// Class record in the staging area for appends and compaction: W mask words
// followed by one word holding countA | countB << 16 | core << 31.
template <int W>
struct Staging {
    uint64_t *base;
    __device__ uint64_t *at(int c) const { return base + (size_t)c * (W + 1); }
};

template <int MODE, int W, int NS>
__global__ void __launch_bounds__(64) mask_walk_kernel(WalkArgs a) {
    extern __shared__ uint64_t lds64[];
    const int lane = threadIdx.x;
    const int d = blockIdx.y;
    const int dir = d == 0 ? 1 : -1;
    const int64_t j = a.site0 + (int64_t)blockIdx.x;
    if (j >= a.M) return;
    if (a.walk_flag && !a.walk_flag[j]) return;
    const Staging<W> stage{lds64};
    const int WA = a.WA;

    // Word w of the pooled row at site k (A's words, then B's).
    auto rowword = [&](int w, int64_t k) -> uint64_t {
        return w < WA ? a.bitsA[k * a.wpsA + w] : a.bitsB[k * a.wpsB + (w - WA)];
    };
    auto validmask = [&](int w) -> uint64_t {
        const int nv = w < WA ? a.nA - 64 * w : a.nB - 64 * (w - WA);
        return nv >= 64 ? ~0ull : (nv <= 0 ? 0ull : ((1ull << nv) - 1ull));
    };

    // ---- classes at x0: lane 0 = allele 0, lane 1 = allele 1 --------------
    uint64_t m[NS][W];
    uint32_t ca[NS], cb[NS], cr[NS];   // counts in A and B, core allele (CORE mode)
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        ca[s] = cb[s] = cr[s] = 0u;
#pragma unroll
        for (int w = 0; w < W; ++w) m[s][w] = 0ull;
    }
    uint32_t n0a = 0, n0b = 0, n1a = 0, n1b = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const uint64_t r = rowword(w, j) & validmask(w);
        const uint64_t z = ~r & validmask(w);
        if (lane == 0) m[0][w] = z;
        if (lane == 1) m[0][w] = r;
        if (w < WA) { n0a += __popcll(z); n1a += __popcll(r); }
        else        { n0b += __popcll(z); n1b += __popcll(r); }
    }
    if (lane == 0) { ca[0] = n0a; cb[0] = n0b; cr[0] = 0u; }
    if (lane == 1) { ca[0] = n1a; cb[0] = n1b; cr[0] = 1u; }
    if (lane < 2 && ca[0] + cb[0] < 2u) { ca[0] = cb[0] = 0u; }
    int kend = 2;   // class indices in use (uniform)

    // ---- per-walk constants -------------------------------------------------
    // Per-class sums are reduced once per marker: two 16-bit fields in one
    // 32-bit lane value when every sum fits (C(n,2) < 2^16), else two values.
    bool act0, act1;
    uint32_t thr0 = 0, thr1 = 0, thrP = 0;
    double P0, P1, ep0, ep1;
    bool pack16;
    if (MODE == MODE_CORE) {
        P0 = (double)choose2(n0a);
        P1 = (double)choose2(n1a);
        act0 = n0a >= 2u;
        act1 = n1a >= 2u;
        if (act0) thr0 = stop_threshold(choose2(n0a), a.cutoff, lane);
        if (act1) thr1 = stop_threshold(choose2(n1a), a.cutoff, lane);
        ep0 = 1.0;
        ep1 = 1.0;
        pack16 = choose2(n0a) < 65536u && choose2(n1a) < 65536u;
    } else {
        P0 = (double)choose2((uint32_t)a.nA);
        P1 = (double)choose2((uint32_t)a.nB);
        thrP = stop_threshold(choose2((uint32_t)(a.nA + a.nB)), a.cutoff, lane);
        ep0 = (double)(choose2(n0a) + choose2(n1a)) / P0;
        ep1 = (double)(choose2(n0b) + choose2(n1b)) / P1;
        act0 = true;
        act1 = false;
        pack16 = choose2((uint32_t)a.nA) < 65536u && choose2((uint32_t)a.nB) < 65536u;
    }
    double ihh0 = 0.0, ihh1 = 0.0;
    int32_t steps0 = 0, steps1 = 0;
    int32_t status = ST_OK;
    int step = 0;

    // Write every live class (and the second child of every split) to LDS at
    // dense indices and read them back: live classes first, then the children.
    auto compact = [&](const bool (&split)[NS], const uint64_t (&zm)[NS][W],
                       const uint32_t (&za)[NS], const uint32_t (&zb)[NS]) {
        int nlive = 0;
        int offs[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const uint64_t lm = __ballot(ca[s] + cb[s] >= 2u);
            offs[s] = nlive + (int)lanes_below(lm);
            nlive += __popcll(lm);
        }
        int nsp = nlive;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (ca[s] + cb[s] >= 2u) {
                uint64_t *e = stage.at(offs[s]);
#pragma unroll
                for (int w = 0; w < W; ++w) e[w] = m[s][w];
                e[W] = (uint64_t)(ca[s] | (cb[s] << 16) | (cr[s] << 31));
            }
            const uint64_t sm = __ballot(split[s]);
            if (split[s]) {
                uint64_t *e = stage.at(nsp + (int)lanes_below(sm));
#pragma unroll
                for (int w = 0; w < W; ++w) e[w] = zm[s][w];
                e[W] = (uint64_t)(za[s] | (zb[s] << 16) | (cr[s] << 31));
            }
            nsp += __popcll(sm);
        }
        __syncthreads();
        kend = nsp;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int c = 64 * s + lane;
            if (c < kend) {
                const uint64_t *e = stage.at(c);
#pragma unroll
                for (int w = 0; w < W; ++w) m[s][w] = e[w];
                const uint32_t x = (uint32_t)e[W];
                ca[s] = x & 0xFFFFu;
                cb[s] = (x >> 16) & 0x7FFFu;
                cr[s] = x >> 31;
            } else {
                ca[s] = cb[s] = 0u;
            }
        }
        __syncthreads();
    };

    while (act0 || act1) {
        // ---- lane i stages step i of the next 64: its row words (read back
        // with readlane, so no memory latency sits on the per-marker chain)
        // and its segment: end of data, abort gap, or scaled genetic length
        const int64_t kb = j + (int64_t)dir * (int64_t)(step + 1 + lane);
        const bool inr = kb >= 0 && kb < a.M;
        uint64_t rowv[W];
#pragma unroll
        for (int w = 0; w < W; ++w) rowv[w] = inr ? rowword(w, kb) : 0ull;
        int32_t stl = ST_OK;
        double gl = 0.0;
        if (!inr) {
            stl = ST_EDGE;
        } else {
            const int64_t lo = dir > 0 ? kb - 1 : kb;
            const int64_t b = a.pos[lo + 1] - a.pos[lo];
            if (b > a.max_gap) {
                stl = ST_GAP;
            } else {
                double g = a.gpos[lo + 1] - a.gpos[lo];
                if (b > a.gap_scale) g = g * ((double)a.gap_scale / (double)b);
                gl = g;
            }
        }
        const uint64_t abort_mask = __ballot(stl != ST_OK);
        const int nb = abort_mask ? (int)__builtin_ctzll(abort_mask) : 64;
        const int32_t abort_st = abort_mask ? (int32_t)__builtin_amdgcn_readlane(stl, nb) : ST_OK;

        // per-step sums of this batch: lane i holds step i's values
        uint32_t sbA = 0, sbB = 0, sbP = 0;
        const bool was0 = act0, was1 = act1;
        int nterm0 = 0, nterm1 = 0;   // trapezoid terms added in this batch
        int i = 0;
        for (; i < 64 && (act0 || act1); ++i) {
            if (i == nb) { status = abort_st; break; }
            uint64_t r[W];
#pragma unroll
            for (int w = 0; w < W; ++w) r[w] = readlane64(rowv[w], i);

            uint32_t accA = 0, accB = 0, accP = 0;
            bool split[NS];
            uint64_t zm[NS][W];
            uint32_t za[NS], zb[NS];
            uint64_t anysplit = 0;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                split[s] = false;
                za[s] = zb[s] = 0u;
                if (64 * s >= kend) continue;   // uniform
                uint32_t oa = 0, ob = 0;
                uint64_t m1[W];
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    m1[w] = m[s][w] & r[w];
                    zm[s][w] = m[s][w] & ~r[w];
                    if (w < WA) oa += __popcll(m1[w]);
                    else        ob += __popcll(m1[w]);
                }
                const uint32_t zA = ca[s] - oa, zB = cb[s] - ob;
                bool ko, kz;
                if (MODE == MODE_CORE) {
                    const bool live = ca[s] >= 2u && (cr[s] ? act1 : act0);
                    const uint32_t sc = live ? choose2(oa) + choose2(zA) : 0u;
                    if (pack16) {
                        accA += sc << (16u * cr[s]);
                    } else {
                        accA += cr[s] ? 0u : sc;
                        accB += cr[s] ? sc : 0u;
                    }
                    ko = live && oa >= 2u;
                    kz = live && zA >= 2u;
                } else {
                    const bool live = ca[s] + cb[s] >= 2u;
                    if (live) {
                        const uint32_t sa = choose2(oa) + choose2(zA);
                        const uint32_t sb = choose2(ob) + choose2(zB);
                        if (pack16) {
                            accA += sa | (sb << 16);
                        } else {
                            accA += sa;
                            accB += sb;
                        }
                        accP += choose2(oa + ob) + choose2(zA + zB);
                    }
                    ko = live && oa + ob >= 2u;
                    kz = live && zA + zB >= 2u;
                }
                split[s] = ko && kz;
                // the allele-1 child stays if it survives, else the allele-0
                // child; a class with no surviving child becomes empty
#pragma unroll
                for (int w = 0; w < W; ++w) m[s][w] = ko ? m1[w] : zm[s][w];
                za[s] = zA;
                zb[s] = zB;
                ca[s] = ko ? oa : (kz ? zA : 0u);
                cb[s] = ko ? ob : (kz ? zB : 0u);
                anysplit |= __ballot(split[s]);
            }
            uint32_t SA, SB, SP = 0u;
            if (pack16) {
                const uint32_t t = wave_sum(accA);
                SA = t & 0xFFFFu;
                SB = t >> 16;
            } else {
                SA = wave_sum(accA);
                SB = wave_sum(accB);
            }
            if (MODE == MODE_POOLED) SP = wave_sum(accP);

            if (anysplit) {
                compact(split, zm, za, zb);
            } else if (NS > 1 && kend > 64 && (i & 7) == 7) {
                // reclaim the holes left by classes that died, so that the
                // upper slots stop being processed once they are empty
                bool none[NS];
#pragma unroll
                for (int s = 0; s < NS; ++s) none[s] = false;
                compact(none, zm, za, zb);
            }

            // ---- record the step's sums and apply the stop rule -----------
            if (lane == i) { sbA = SA; sbB = SB; sbP = SP; }
            if (MODE == MODE_CORE) {
                if (act0) {
                    steps0 += 1;
                    if (SA <= thr0) act0 = false; else nterm0 = i + 1;
                }
                if (act1) {
                    steps1 += 1;
                    if (SB <= thr1) act1 = false; else nterm1 = i + 1;
                }
            } else {
                steps0 += 1;
                if (SP <= thrP) act0 = false; else nterm0 = i + 1;
            }
        }
        step += i;

        // ---- FP64 trapezoid of this batch: terms lane-parallel, sum in order
        const double g = gl;
        if (MODE == MODE_CORE) {
            if (was0 && nterm0 > 0) {
                const double e = (double)sbA / P0;
                double prev = __shfl_up(e, 1, 64);
                if (lane == 0) prev = ep0;
                const double term = 0.5 * (prev + e) * g;
                for (int q = 0; q < nterm0; ++q) ihh0 += readlane_f64(term, q);
                ep0 = readlane_f64(e, nterm0 - 1);
            }
            if (was1 && nterm1 > 0) {
                const double e = (double)sbB / P1;
                double prev = __shfl_up(e, 1, 64);
                if (lane == 0) prev = ep1;
                const double term = 0.5 * (prev + e) * g;
                for (int q = 0; q < nterm1; ++q) ihh1 += readlane_f64(term, q);
                ep1 = readlane_f64(e, nterm1 - 1);
            }
        } else if (nterm0 > 0) {
            const double eA = (double)sbA / P0;
            const double eB = (double)sbB / P1;
            double pA = __shfl_up(eA, 1, 64);
            double pB = __shfl_up(eB, 1, 64);
            if (lane == 0) { pA = ep0; pB = ep1; }
            const double tA = 0.5 * (pA + eA) * g;
            const double tB = 0.5 * (pB + eB) * g;
            for (int q = 0; q < nterm0; ++q) {
                ihh0 += readlane_f64(tA, q);
                ihh1 += readlane_f64(tB, q);
            }
            ep0 = readlane_f64(eA, nterm0 - 1);
            ep1 = readlane_f64(eB, nterm0 - 1);
        }
        if (status != ST_OK) break;
    }

    if (lane == 0) {
        const size_t o = (size_t)j * 2 + d;
        a.ihh[o * 2 + 0] = ihh0;
        a.ihh[o * 2 + 1] = ihh1;
        a.dstatus[o] = status;
        a.steps[o * 2 + 0] = steps0;
        a.steps[o * 2 + 1] = steps1;
    }
}

template <int MODE, int W>
hipError_t launch_ns(const WalkArgs &a, int ns, int64_t n_blocks, hipStream_t s) {
    dim3 grid((unsigned)n_blocks, 2u, 1u);
    const size_t lds = (size_t)64 * ns * (W + 1) * sizeof(uint64_t);
    switch (ns) {
        case 1: hipLaunchKernelGGL((mask_walk_kernel<MODE, W, 1>), grid, dim3(64), lds, s, a); break;
        case 2: hipLaunchKernelGGL((mask_walk_kernel<MODE, W, 2>), grid, dim3(64), lds, s, a); break;
        case 4: hipLaunchKernelGGL((mask_walk_kernel<MODE, W, 4>), grid, dim3(64), lds, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int MODE>
hipError_t launch_w(const WalkArgs &a, int words, int ns, int64_t n_blocks, hipStream_t s) {
    switch (words) {
        case 1: return launch_ns<MODE, 1>(a, ns, n_blocks, s);
        case 2: return launch_ns<MODE, 2>(a, ns, n_blocks, s);
        case 3: return launch_ns<MODE, 3>(a, ns, n_blocks, s);
        case 4: return launch_ns<MODE, 4>(a, ns, n_blocks, s);
        case 5: return launch_ns<MODE, 5>(a, ns, n_blocks, s);
        case 6: return launch_ns<MODE, 6>(a, ns, n_blocks, s);
        case 7: return launch_ns<MODE, 7>(a, ns, n_blocks, s);
        case 8: return launch_ns<MODE, 8>(a, ns, n_blocks, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool mask_walk_supported(int32_t nA, int32_t nB, int mode) {
    const int words = (nA + 63) / 64 + (mode == MODE_POOLED ? (nB + 63) / 64 : 0);
    const int n = nA + (mode == MODE_POOLED ? nB : 0);
    return words <= 8 && n <= 512;
}

hipError_t launch_mask_walk(const WalkArgs &a, int mode, int64_t n_blocks, hipStream_t s) {
    const int words = a.WA + (mode == MODE_POOLED ? a.WB : 0);
    const int n = a.nA + (mode == MODE_POOLED ? a.nB : 0);
    const int ns = n <= 128 ? 1 : (n <= 256 ? 2 : 4);   // room for n/2 classes
    if (n_blocks <= 0) return hipSuccess;
    if (mode == MODE_CORE) return launch_w<MODE_CORE>(a, words, ns, n_blocks, s);
    return launch_w<MODE_POOLED>(a, words, ns, n_blocks, s);
}

}  // namespace ss

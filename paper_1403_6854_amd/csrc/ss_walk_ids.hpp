// Class-id EHH walk: partition refinement of the haplotypes around one core
// site by one workgroup, as a device function (walk_one) shared by the
// per-locus kernels of ss_walk.hip and, for walks whose classes outgrow a
// register row, by the bitmask walk of ss_walk_mask.hip.
//
// What it computes (Szpiech & Hernandez, arXiv:1403.6854):
//   * Sec. 1.1, Eqs. 1-3: the distinct haplotypes from x0 out to x_i, with x0
//     part of the string, so the classes at x0 are "allele 0" and "allele 1"
//     (the core partition of Eq. 2) and every further marker splits each
//     class by allele.  S = sum over classes of C(n_h, 2) is exact integer
//     arithmetic; EHH = S / C(n, 2) in double.
//   * Sec. 1.2, Eq. 4 and the practical rules below it: the trapezoid
//     1/2 (EHH(x_{i-1}) + EHH(x_i)) g accumulated outward from x0, truncated
//     before the first marker with EHH < cutoff, g scaled by gap_scale / b for
//     gaps b > gap_scale, and the walk aborted at the end of the data or at a
//     gap b > max_gap.
//   * Sec. 1.3, Eq. 7: for XPEHH the partition is over the two populations
//     pooled; each class carries its count in A and in B, and the walk stops
//     where the pooled EHH drops below the cutoff.
//
// MI355X design:
//   * The haplotype matrix is bit-packed marker-major, so one marker row is a
//     handful of 64-bit words.  Slot r of wave w owns the 64 haplotypes of
//     word w + r * (waves per group): its row word is wave-uniform (one scalar
//     load) and lane l's allele is bit l of it.  Class ids live in registers.
//   * Per marker: (1) members with allele 1 add to their class's ones-counter
//     with an LDS atomic (A counts in the low and B counts in the high 16
//     bits, so the pooled walk needs one atomic per member); (2) one pass over
//     the classes turns (size, ones) into the two children, drops children
//     with fewer than two members (they can never contribute again), gives
//     the survivors dense new ids with a wave-aggregated allocation, and sums
//     C(., 2) with wave reductions; (3) members look up their new id.
//     Two workgroup barriers per marker; everything else is per-lane.
//   * Once a core's EHH has fallen below the cutoff its classes are dropped
//     too (except in the trace mode of ss_ehh, which reports both curves to
//     the end of the walk).
//   * Arithmetic that decides where a walk stops stays in the order the
//     definitions give and is compiled without FP contraction, so the FP64
//     results match a plain CPU evaluation bit for bit wherever libm is not
//     involved.
#pragma once

#include "ss_internal.hpp"

namespace ss {

namespace {

constexpr int32_t DEAD = -1;

__device__ __forceinline__ uint32_t choose2(uint32_t x) {
    // x <= 65535, so x * (x - 1) fits in 32 bits
    return (x * (x - 1u)) >> 1;
}

// Sum over the 64 lanes of a wave (DPP reduction in the device library;
// every lane must be active).
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) { return __ockl_wfred_add_u32(v); }

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int i) {
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, i);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), i);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ double readlane_f64(double v, int i) {
    return __builtin_bit_cast(double, readlane64(__builtin_bit_cast(uint64_t, v), i));
}

// Largest S in [0, P] with (double)S / (double)P < cutoff (P >= 1, cutoff >
// 0), found by testing 64 consecutive candidates around cutoff * P, one per
// lane: fl(S / P) is monotone in S, so a stop test is then S <= threshold.
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

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Size word of a class: CORE mode = count | core << 31; POOLED mode =
// countA | countB << 16.  Ones-counter words use the same split.
// One walk: core site j, direction d (0 downstream, 1 upstream), by the whole
// workgroup.
template <int MODE, bool TRACE, int R>
__device__ void walk_one(const WalkArgs &a, int64_t j, int d) {
    extern __shared__ uint32_t smem[];
    const int T = blockDim.x;
    // the thread index comes from a value the compiler cannot share with
    // the caller's (inlined into the bitmask walk as its fallback, addresses
    // built from a shared index were kept from the kernel's start and spilled)
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wpg = T >> 6;
    const int dir = d == 0 ? 1 : -1;
    if (j >= a.M) return;
    if (a.walk_flag && !a.walk_flag[j]) return;

    const int kmax = a.kmax;
    uint32_t *cnt1 = smem;                        // [kmax]   ones per class
    uint32_t *szv0 = cnt1 + kmax;                 // [kmax]   sizes, even steps
    uint32_t *szv1 = szv0 + kmax;                 // [kmax]   sizes, odd steps
    int32_t *map = (int32_t *)(szv1 + kmax);      // [2*kmax] (class, allele) -> child
    uint32_t *sacc = (uint32_t *)(map + 2 * kmax);  // [2][4]   S sums per parity
    int32_t *knext = (int32_t *)(sacc + 8);       // [2]      classes made per parity
    uint32_t *init = (uint32_t *)(knext + 2);     // [2]      class sizes at x0

    for (int i = tid; i < kmax; i += T) cnt1[i] = 0u;
    if (tid < 8) sacc[tid] = 0u;
    if (tid < 2) { knext[tid] = 0; init[tid] = 0u; }

    // Per-slot source row and validity.
    const uint64_t *src[R];
    int64_t stride[R];
    uint32_t inc[R];
    int32_t cls[R];
    bool word[R];   // wave-uniform: the slot's word holds haplotypes
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int wq = wave + r * wpg;
        word[r] = wq < a.WA + (MODE == MODE_POOLED ? a.WB : 0);
        bool valid;
        if (wq < a.WA) {
            src[r] = a.bitsA + wq;
            stride[r] = a.wpsA;
            valid = wq * 64 + lane < a.nA;
            inc[r] = 1u;
        } else if (MODE == MODE_POOLED && wq < a.WA + a.WB) {
            src[r] = a.bitsB + (wq - a.WA);
            stride[r] = a.wpsB;
            valid = (wq - a.WA) * 64 + lane < a.nB;
            inc[r] = 0x10000u;
        } else {
            src[r] = a.bitsA;
            stride[r] = 0;
            valid = false;
            inc[r] = 0u;
        }
        cls[r] = valid ? 0 : DEAD;
        if (!valid) inc[r] = 0u;
    }
    __syncthreads();

    // Classes at x0: id = allele.
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (word[r]) {
            const uint64_t w = src[r][j * stride[r]];
            const int32_t bit = (int32_t)((w >> lane) & 1ull);
            if (cls[r] != DEAD) {
                cls[r] = bit;
                atomicAdd(&init[bit], inc[r]);
            }
        }
    }
    __syncthreads();
    const uint32_t i0 = init[0], i1 = init[1];

    // Per-walk scalar state (identical in every thread).
    // Every wave takes the stop decisions from exact integer thresholds (a core
    // stops at the first marker with S <= thr; XPEHH: the pooled S against
    // thr0); the EHH values and iHH sums are wave 0's, whose thread 0 writes
    // the results.
    bool act0, act1;
    double ihh0 = 0.0, ihh1 = 0.0, ep0, ep1, P0, P1;
    uint32_t thr0 = 0u, thr1 = 0u;
    int32_t steps0 = 0, steps1 = 0;
    if (MODE == MODE_CORE) {
        const uint32_t n0 = i0 & 0xFFFFu, n1 = i1 & 0xFFFFu;
        P0 = (double)choose2(n0);
        P1 = (double)choose2(n1);
        act0 = n0 >= 2u;
        act1 = n1 >= 2u;
        if (act0) thr0 = stop_threshold(choose2(n0), a.cutoff, lane);
        if (act1) thr1 = stop_threshold(choose2(n1), a.cutoff, lane);
        ep0 = 1.0;
        ep1 = 1.0;
        if (tid == 0) {
            szv0[0] = n0;
            szv0[1] = n1 | 0x80000000u;
        }
        if (TRACE && tid == 0) {
            a.trS[(size_t)d * (a.cap + 1) * 2 + 0] = choose2(n0);
            a.trS[(size_t)d * (a.cap + 1) * 2 + 1] = choose2(n1);
            if (a.trSizes) {
                uint32_t *z = a.trSizes + (size_t)d * (a.cap + 1) * a.nA;
                int q = 0;
                if (n0 >= 2u) z[q++] = n0;
                if (n1 >= 2u) z[q++] = n1 | 0x80000000u;
            }
        }
        // classes with fewer than two members can never contribute
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (cls[r] == 0 && n0 < 2u) cls[r] = DEAD;
            if (cls[r] == 1 && n1 < 2u) cls[r] = DEAD;
        }
    } else {
        const uint32_t a0 = i0 & 0xFFFFu, b0 = i0 >> 16, a1 = i1 & 0xFFFFu, b1 = i1 >> 16;
        P0 = (double)choose2((uint32_t)a.nA);   // population A
        P1 = (double)choose2((uint32_t)a.nB);   // population B
        thr0 = stop_threshold(choose2((uint32_t)(a.nA + a.nB)), a.cutoff, lane);
        // x0 is part of the haplotype: each population's curve starts at its
        // whole-sample EHH at x0
        ep0 = (double)(choose2(a0) + choose2(a1)) / P0;
        ep1 = (double)(choose2(b0) + choose2(b1)) / P1;
        act0 = true;
        act1 = false;
        if (tid == 0) {
            szv0[0] = i0;
            szv0[1] = i1;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (cls[r] == 0 && a0 + b0 < 2u) cls[r] = DEAD;
            if (cls[r] == 1 && a1 + b1 < 2u) cls[r] = DEAD;
        }
    }
    __syncthreads();

    int32_t K = 2;
    int32_t status = ST_OK;
    int step = 0;
    while (act0 || act1) {
        // Stage the next 64 markers of the walk: lane i of every wave loads
        // its slots' row words for step (step + 1 + i) and works out that
        // step's segment: end of data, abort gap, or scaled genetic length.
        // The per-marker loop below then reads them with readlane, so no
        // global-memory latency sits on the serial chain of the walk.
        const int64_t kb = j + (int64_t)dir * (int64_t)(step + 1 + lane);
        const bool inr = kb >= 0 && kb < a.M;
        uint64_t rowv[R];
#pragma unroll
        for (int r = 0; r < R; ++r) rowv[r] = (word[r] && inr) ? src[r][kb * stride[r]] : 0ull;
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
                double g = a.physical ? (double)b : a.gpos[lo + 1] - a.gpos[lo];
                if (b > a.gap_scale) g = g * ((double)a.gap_scale / (double)b);
                gl = g;
            }
        }
        const uint64_t abort_mask = __ballot(stl != ST_OK);
        const int nb = abort_mask ? (int)__builtin_ctzll(abort_mask) : 64;
        const int32_t abort_st = abort_mask ? (int32_t)__builtin_amdgcn_readlane(stl, nb) : ST_OK;

        for (int i = 0; i < 64 && (act0 || act1); ++i) {
            if (i == nb) { status = abort_st; goto done; }
            if (TRACE && step >= a.cap) { status = ST_CAP; goto done; }

            const int par = step & 1;
            uint32_t *szc = par ? szv1 : szv0;
            uint32_t *szn = par ? szv0 : szv1;
            uint32_t *sa = sacc + 4 * par;
            int32_t *kn = knext + par;

            // (1) ones per class
            int32_t bit[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                bit[r] = 0;
                if (word[r]) {
                    const uint64_t w = readlane64(rowv[r], i);
                    bit[r] = (int32_t)((w >> lane) & 1ull);
                    if (cls[r] != DEAD && bit[r]) atomicAdd(&cnt1[cls[r]], inc[r]);
                }
            }
            __syncthreads();

            // (2) split every class, keep children with >= 2 members
            for (int c0 = 0; c0 < K; c0 += T) {
                const int c = c0 + tid;
                const bool in = c < K;
                uint32_t one = 0u, sz = 0u;
                if (in) {
                    one = cnt1[c];
                    cnt1[c] = 0u;
                    sz = szc[c];
                }
                bool keepz = false, keepo = false;
                uint32_t wz = 0u, wo = 0u;
                uint32_t s0 = 0u, s1 = 0u, s2 = 0u;
                if (in) {
                    if (MODE == MODE_CORE) {
                        const uint32_t core = sz >> 31;
                        const uint32_t n = sz & 0xFFFFu;
                        const uint32_t o = one, z = n - one;
                        const bool live = TRACE || (core ? act1 : act0);
                        const uint32_t sc = choose2(o) + choose2(z);
                        if (core) s1 = sc; else s0 = sc;
                        keepz = live && z >= 2u;
                        keepo = live && o >= 2u;
                        wz = z | (core << 31);
                        wo = o | (core << 31);
                    } else {
                        const uint32_t nA = sz & 0xFFFFu, nB = sz >> 16;
                        const uint32_t oA = one & 0xFFFFu, oB = one >> 16;
                        const uint32_t zA = nA - oA, zB = nB - oB;
                        s0 = choose2(oA) + choose2(zA);
                        s1 = choose2(oB) + choose2(zB);
                        s2 = choose2(oA + oB) + choose2(zA + zB);
                        keepz = zA + zB >= 2u;
                        keepo = oA + oB >= 2u;
                        wz = zA | (zB << 16);
                        wo = oA | (oB << 16);
                    }
                }
                const uint64_t bz = __ballot(keepz);
                const uint64_t bo = __ballot(keepo);
                const int nz = __popcll(bz), no = __popcll(bo);
                int base = 0;
                if (T == 64) {
                    base = kn[0];
                } else if (lane == 0 && nz + no > 0) {
                    base = atomicAdd(kn, nz + no);
                }
                if (T != 64) base = __shfl(base, 0, 64);
                const int idz = base + (int)lanes_below(bz);
                const int ido = base + nz + (int)lanes_below(bo);
                if (in) {
                    map[2 * c] = keepz ? idz : DEAD;
                    map[2 * c + 1] = keepo ? ido : DEAD;
                }
                if (keepz) szn[idz] = wz;
                if (keepo) szn[ido] = wo;
                if (TRACE && a.trSizes) {
                    uint32_t *z = a.trSizes + ((size_t)d * (a.cap + 1) + (step + 1)) * a.nA;
                    if (keepz) z[idz] = wz;
                    if (keepo) z[ido] = wo;
                }
                s0 = wave_sum(s0);
                s1 = wave_sum(s1);
                if (MODE == MODE_POOLED) s2 = wave_sum(s2);
                if (lane == 0) {
                    if (T == 64) {
                        kn[0] = base + nz + no;
                        sa[0] += s0;
                        sa[1] += s1;
                        if (MODE == MODE_POOLED) sa[2] += s2;
                    } else {
                        if (s0) atomicAdd(&sa[0], s0);
                        if (s1) atomicAdd(&sa[1], s1);
                        if (MODE == MODE_POOLED && s2) atomicAdd(&sa[2], s2);
                    }
                }
                if (T == 64) __syncthreads();   // kn[0] is read again next round
            }
            __syncthreads();

            // (3) new class ids
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (cls[r] != DEAD) cls[r] = map[2 * cls[r] + bit[r]];
            K = kn[0];
            const uint32_t S0 = sa[0], S1 = sa[1], S2 = sa[2];
            if (tid == 0) {
                uint32_t *other = sacc + 4 * (par ^ 1);
                other[0] = other[1] = other[2] = 0u;
                knext[par ^ 1] = 0;
            }
            step += 1;

            if (MODE == MODE_CORE) {
                if (TRACE && tid == 0) {
                    a.trS[((size_t)d * (a.cap + 1) + step) * 2 + 0] = S0;
                    a.trS[((size_t)d * (a.cap + 1) + step) * 2 + 1] = S1;
                }
                if (act0) {
                    steps0 += 1;
                    if (S0 <= thr0) {
                        act0 = false;
                    } else if (wave == 0) {
                        const double e = (double)S0 / P0;
                        ihh0 += 0.5 * (ep0 + e) * readlane_f64(gl, i);
                        ep0 = e;
                    }
                }
                if (act1) {
                    steps1 += 1;
                    if (S1 <= thr1) {
                        act1 = false;
                    } else if (wave == 0) {
                        const double e = (double)S1 / P1;
                        ihh1 += 0.5 * (ep1 + e) * readlane_f64(gl, i);
                        ep1 = e;
                    }
                }
            } else {
                steps0 += 1;
                if (S2 <= thr0) {
                    act0 = false;
                } else if (wave == 0) {
                    const double g = readlane_f64(gl, i);
                    const double eA = (double)S0 / P0;
                    const double eB = (double)S1 / P1;
                    ihh0 += 0.5 * (ep0 + eA) * g;
                    ihh1 += 0.5 * (ep1 + eB) * g;
                    ep0 = eA;
                    ep1 = eB;
                }
            }
        }
    }
done:

    if (tid == 0) {
        const size_t o = (size_t)j * 2 + d;
        if (!TRACE) {
            put_rec(a.rec + o * 2 + 0, ihh0, status, steps0);
            put_rec(a.rec + o * 2 + 1, ihh1, status, steps1);
        } else {
            put_rec(a.rec + d * 2 + 0, ihh0, status, step);
            put_rec(a.rec + d * 2 + 1, ihh1, status, step);
            a.trLen[d] = step;
        }
    }
}

}  // namespace

}  // namespace ss

// EHH walk with the partition held as haplotype bitmasks in registers, one
// wave per walk, for walks over up to 512 haplotypes.
//
// What it computes is the same partition refinement as ss_walk.hip
// (Sec. 1.1, Eqs. 1-3: classes of identical haplotypes from x0 out to x_i;
// Sec. 1.2, Eq. 4 and the rules below it; Sec. 1.3, Eq. 7 for the pooled
// walk of XPEHH); the representation is what differs:
//   * a class is a bitmask over the haplotypes (W 64-bit words in the
//     marker-major packing).  LPC lanes share one class, each holding
//     W / LPC of its words, so a row of the wave holds 64 / LPC classes and
//     rows are processed only while they hold classes.  Splitting a class by
//     the alleles at marker k is an AND with row k and a popcount, summed
//     over the class's lanes with DPP;
//   * for iHS each core allele is walked by its own wave (the two cores never
//     share a class, Eq. 2), so a wave carries only one core's classes; the
//     locus-level rules are recombined afterwards: a direction aborts if a
//     walk of either core aborted, which is exactly when the joint walk would
//     have met the end of the data or the gap while that core was active;
//   * the child with the allele-1 members stays in place if it has >= 2
//     members, else the allele-0 child; when both survive, the second one is
//     appended through LDS (rare once the first markers have separated the
//     founder groups); children with < 2 members are dropped for good;
//   * the stop test EHH = S / C(n,2) < cutoff is evaluated on integers:
//     correctly rounded division is monotone in S, so fl(S/P) < cutoff holds
//     exactly for S <= thr, with thr found once per walk by testing 64
//     candidates around cutoff * P with the same IEEE division;
//   * the FP64 trapezoid terms of 64 markers are formed lane-parallel after
//     the markers have been refined, and added to iHH one by one in marker
//     order, so the sums round exactly as the definition's left-to-right sum;
//   * pairwise phase (iHS walks): sum_h C(n_h, 2) counts the pairs of
//     haplotypes still identical from x0 to x_i.  Once that count S is at
//     most the pair capacity, the classes are expanded into an explicit list
//     of those pairs in LDS, and each pass then covers 64 markers: a pair's 64-bit keys
//     (its haplotypes' alleles at the next 64 markers, read from a
//     haplotype-major copy of the matrix) are XORed, the lowest set bit is
//     the marker where the pair splits, a 64-bin histogram of those markers
//     gives S at each of the 64 markers, and the surviving pairs are compacted
//     in place.  Long walks then cost a few instructions per pair per 64
//     markers instead of a full refinement per marker.
#include "ss_walk_ids.hpp"   // walk_one, choose2, wave_sum, readlane64, readlane_f64, stop_threshold

namespace ss {

namespace {

// Sum of v over the LPC consecutive lanes of a class (LPC = 1, 2, 4 or 8).
template <int LPC>
__device__ __forceinline__ uint32_t group_sum(uint32_t v) {
    if (LPC >= 2) v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    if (LPC >= 4) v += (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    if (LPC >= 8) v += (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x101F);             // lane ^ 4
    return v;
}

// Pairs the pairwise phase keeps in LDS, by mask width.  The capacity is
// where a walk switches from per-marker refinement to 64-marker passes over
// its pair list, and a pass costs in proportion to the pairs: at 4 words a
// pass over up to 1,024 pairs costs more than the per-marker steps it
// replaces while there are that many.  Measured (walk ms,
// copying-model regions of 20,000 sites, 204 x 22,147 for W = 4) over
// capacities 128 / 256 / 384 / 512 / 1,024:
//   W = 2 (100 haplotypes): 0.63 / 0.46 / 0.36 / 0.34 / --
//   W = 4 (204 haplotypes): 0.35 / 0.34 / 0.35 / 0.36 / 0.47
//   W = 8 (400 haplotypes): 1.87 / 1.63 / 1.49 / 1.39 / 1.19
__host__ __device__ constexpr int mask_pair_cap(int W) {
    return W >= 8 ? 1024 : (W == 4 ? 256 : 512);
}

// Inclusive prefix sum over the 64 lanes (once per 64-marker pass), in DPP
// register moves instead of LDS permutes: within each row of 16 lanes by
// shifts of 1, 2, 4 and 8 (lanes shifted in from outside the row read 0), then
// row 0's total broadcast into row 1 and row 2's into row 3, then the total
// of rows 0-1 into rows 2-3.
__device__ __forceinline__ uint32_t wave_prefix(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);   // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);   // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);   // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);   // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return v;
}

// The value of lane - 1 (lane 0 gets `first`): a DPP wave shift instead of an
// LDS permute.
__device__ __forceinline__ double lane_before(double v, double first) {
    const uint64_t x = __builtin_bit_cast(uint64_t, v);
    const uint64_t f = __builtin_bit_cast(uint64_t, first);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)f, (int)(uint32_t)x, 0x138,
                                                              0xF, 0xF, false);   // wave_shr:1
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(f >> 32), (int)(uint32_t)(x >> 32),
                                                              0x138, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Adds the first n of the wave's per-lane terms (lane t: the term of step t
// of a 64-marker batch) to each running iHH sum, one after another in step
// order -- the definition's rounding, identical to adding them one by one.
// The terms are staged in LDS (64 doubles per sum at buf, a region no lane
// reads meanwhile); lanes t >= n stage +0.0, which leaves a non-negative sum
// as it is, so the adds run several at a time from broadcast LDS reads
// instead of two lane reads, a scalar loop step and an add per term.
template <int NS>
__device__ __forceinline__ void add_terms(double (&acc)[NS], const double (&term)[NS], int n,
                                          double *buf) {
    const int lane = threadIdx.x;
#pragma unroll
    for (int s = 0; s < NS; ++s) buf[s * 64 + lane] = lane < n ? term[s] : 0.0;
    __syncthreads();
    // K terms of each sum per iteration, the loop kept rolled: unrolled, its
    // loads in flight took up to 128 VGPRs
    constexpr int K = 8 / NS;
    const double2 *b2 = (const double2 *)buf;
#pragma unroll 1
    for (int b = 0; b < n; b += K) {
        double2 v[NS][K / 2];
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int k = 0; k < K / 2; ++k) v[s][k] = b2[s * 32 + (b >> 1) + k];
#pragma unroll
        for (int k = 0; k < K / 2; ++k)
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                acc[s] += v[s][k].x;
                acc[s] += v[s][k].y;
            }
    }
}

// Waves per SIMD the compiler is held to, the most that fit without spills:
// 4-word iHS walks (129-256 haplotypes) 6 waves in 80 VGPRs (bounded to 7
// they spill 24-44 bytes a lane and run slower: the 204-haplotype walk takes
// 0.265 against 0.270 ms), 8-word iHS walks 4 waves in 128 VGPRs (3
// unbounded); the pooled walks fit 4 or more waves unbounded.
template <int MODE, int W>
constexpr int mask_waves_per_eu() {
    return MODE == MODE_CORE && W == 4 ? 6 : (MODE == MODE_CORE && W == 8 ? 4 : 1);
}

// W: mask words per class (pooled: A's words, then B's); LPC: lanes per
// class; NR: rows of 64 / LPC classes (capacity NR * 64 / LPC classes).
template <int MODE, int W, int LPC, int NR>
__global__ void __launch_bounds__(64, (mask_waves_per_eu<MODE, W>())) mask_walk_kernel(WalkArgs a) {
    constexpr int WPL = W / LPC;    // words per lane
    constexpr int CPR = 64 / LPC;   // classes per row
    // the next batch's rows are loaded during the current one for masks of up
    // to 8 words; wider masks would hold 2 W registers a lane across the
    // whole batch for it, so they load their rows when the batch starts
    constexpr bool kPrefetchRows = W <= 8;
    constexpr int PCAP = MODE == MODE_CORE ? mask_pair_cap(W) : 0;
    extern __shared__ uint64_t lds64[];
    // LDS regions; the pairwise phase stages no rows and compacts no classes,
    // so its buffers share space with those of the per-marker phase.
    constexpr int kStageWords = NR * CPR * (W + 1);
    constexpr int kUnionWords = kStageWords > PCAP / 2 ? kStageWords : PCAP / 2;
    uint64_t *rowbuf = lds64;                  // [64][W] rows of the staged markers
    uint64_t *keys = rowbuf;                   // [64 W] 64-marker keys (pairwise phase)
    uint64_t *stage = rowbuf + 64 * W;         // [NR * CPR][W + 1] class records
    uint32_t *pairs = (uint32_t *)stage;       // [PCAP] a | b << 16, member indices (pairwise phase)
    uint32_t *hist = (uint32_t *)(stage + kUnionWords);   // [64] splits per marker
    uint16_t *memb = (uint16_t *)(hist + 64);  // [64 W] haplotypes of the pair list's members
    // [1 or 2][64] trapezoid terms of a batch, staged once the batch's rows
    // (per-marker phase) or keys (pairwise phase) are no longer read; the
    // pooled walks' second 64 may reach into the class staging area, which is
    // idle between markers
    double *tbuf = (double *)rowbuf;
    static_assert(64 * W + kStageWords >= (MODE == MODE_CORE ? 64 : 128), "room for the terms");

    const int lane = threadIdx.x;
    const int q = lane / LPC;     // class slot within a row
    const int g = lane % LPC;     // word group within the class
    const bool leader = g == 0;
    // one workgroup per (site, direction[, core]), site-major: the walks of a
    // site are neighbours in the grid, so they start together and share the
    // site's rows in cache, and a run of long walks in the middle of a region
    // (a sweep) starts in the middle of the launch, not in its last quarter
    constexpr int kPerSite = MODE == MODE_CORE ? 4 : 2;
    const int d = (int)(blockIdx.x % 2u);
    const int dir = d == 0 ? 1 : -1;
    const int core = MODE == MODE_CORE ? (int)((blockIdx.x / 2u) % 2u) : 0;   // CORE: the allele this wave walks
    const int64_t j = a.site0 + (int64_t)(blockIdx.x / (unsigned)kPerSite);
    if (j >= a.M) return;
    if (a.walk_flag && !a.walk_flag[j]) return;
    const int Wused = MODE == MODE_CORE ? a.WA : a.WA + a.WB;

    auto is_a = [&](int w) -> bool { return MODE == MODE_CORE || w < a.WA; };
    auto rowword = [&](int w, int64_t k) -> uint64_t {
        if (w >= Wused) return 0ull;
        return is_a(w) ? a.bitsA[k * a.wpsA + w] : a.bitsB[k * a.wpsB + (w - a.WA)];
    };
    auto validmask = [&](int w) -> uint64_t {
        if (w >= Wused) return 0ull;
        const int nv = is_a(w) ? a.nA - 64 * w : a.nB - 64 * (w - a.WA);
        return nv >= 64 ? ~0ull : (nv <= 0 ? 0ull : ((1ull << nv) - 1ull));
    };

    // ---- classes at x0 ------------------------------------------------------
    // CORE: one class, the carriers of `core`.  POOLED: allele 0 and allele 1.
    uint64_t m[NR][WPL];
    uint32_t ca[NR], cb[NR];   // class counts in A and B (replicated over the LPC lanes)
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        ca[r] = cb[r] = 0u;
#pragma unroll
        for (int t = 0; t < WPL; ++t) m[r][t] = 0ull;
    }
    uint32_t n0a = 0, n0b = 0, n1a = 0, n1b = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const uint64_t r1 = rowword(w, j) & validmask(w);
        const uint64_t r0 = ~r1 & validmask(w);
        if (is_a(w)) { n0a += __popcll(r0); n1a += __popcll(r1); }
        else         { n0b += __popcll(r0); n1b += __popcll(r1); }
        if (w / WPL == g) {
            const int t = w % WPL;
            if (MODE == MODE_CORE) {
                if (q == 0) m[0][t] = core ? r1 : r0;
            } else {
                if (q == 0) m[0][t] = r0;
                if (q == 1) m[0][t] = r1;
            }
        }
    }
    int kend;
    if (MODE == MODE_CORE) {
        const uint32_t nc = core ? n1a : n0a;
        if (q == 0) ca[0] = nc >= 2u ? nc : 0u;
        kend = 1;
    } else {
        if (q == 0) { ca[0] = n0a; cb[0] = n0b; }
        if (q == 1) { ca[0] = n1a; cb[0] = n1b; }
        if (q < 2 && ca[0] + cb[0] < 2u) ca[0] = cb[0] = 0u;
        kend = 2;
    }

    // ---- staging of 64-marker batches ------------------------------------------
    // Lane i fetches step i of a batch: its row words (per-marker phase only)
    // and its segment's genetic length.  The next batch is fetched while the
    // current one is processed, so the loads' latency overlaps the work.
    auto fetch = [&](int st, bool rows, uint64_t (&rv)[W], double &sv, bool &inr) {
        const int64_t kb = j + (int64_t)dir * (int64_t)(st + 1 + lane);
        inr = kb >= 0 && kb < a.M;
#pragma unroll
        for (int w = 0; w < W; ++w) rv[w] = (rows && inr) ? rowword(w, kb) : 0ull;
        // segment lengths with the gap rules applied come from the scan's
        // segment pass (a.seg is always set for this kernel)
        sv = inr ? a.seg[dir > 0 ? kb : kb + 1] : 0.0;
    };
    uint64_t pf_rows[W];
    double pf_seg;
    bool pf_inr;
    int pf_step = 0;
    fetch(0, true, pf_rows, pf_seg, pf_inr);

    // ---- per-walk constants -------------------------------------------------
    // CORE: one statistic S = sum over the classes of C(n_h, 2), EHH = S / P.
    // POOLED: S_A and S_B (16-bit fields of one value when they fit) and
    // S_pool, which alone decides where the walk stops.
    bool act;
    uint32_t thr;
    double PA, PB = 1.0, epA, epB = 0.0;
    bool pack16 = true;
    if (MODE == MODE_CORE) {
        const uint32_t nc = core ? n1a : n0a;
        PA = (double)choose2(nc);
        act = nc >= 2u;
        thr = act ? stop_threshold(choose2(nc), a.cutoff, lane) : 0u;
        epA = 1.0;
    } else {
        PA = (double)choose2((uint32_t)a.nA);
        PB = (double)choose2((uint32_t)a.nB);
        thr = stop_threshold(choose2((uint32_t)(a.nA + a.nB)), a.cutoff, lane);
        // x0 is part of the haplotype: each population's curve starts at its
        // whole-sample EHH at x0
        epA = (double)(choose2(n0a) + choose2(n1a)) / PA;
        epB = (double)(choose2(n0b) + choose2(n1b)) / PB;
        act = true;
        pack16 = choose2((uint32_t)a.nA) < 65536u && choose2((uint32_t)a.nB) < 65536u;
    }
    double ihhA = 0.0, ihhB = 0.0;
    int32_t steps = 0;
    int32_t status = ST_OK;
    int step = 0;
    // The sums after the last marker refined (S, or S_A | S_B << 16 and S_B
    // when they do not fit): a marker that cuts no live class leaves them as
    // they are.
    uint32_t curS = 0u, curSB = 0u;
    if (MODE == MODE_CORE) {
        curS = act ? choose2(core ? n1a : n0a) : 0u;
    } else {
        const uint32_t sa0 = choose2(n0a) + choose2(n1a), sb0 = choose2(n0b) + choose2(n1b);
        curS = pack16 ? (sa0 | (sb0 << 16)) : sa0;
        curSB = pack16 ? 0u : sb0;
    }

    // Dense re-indexing of the live classes through LDS, with the second
    // child of every split appended after them.
    // Returns false, changing nothing, when the classes do not fit in the
    // wave's NR rows.
    auto compact = [&](const bool (&split)[NR], const uint64_t (&zm)[NR][WPL],
                       const uint32_t (&za)[NR], const uint32_t (&zb)[NR]) -> bool {
        // leader lanes set in a mask below this lane's class: the set lanes
        // below this lane, less its own leader's if this lane is not one
        auto groups_below = [&](uint64_t lmask) -> int {
            const uint32_t b = lanes_below(lmask);
            return (int)(g ? b - (uint32_t)((lmask >> (lane - g)) & 1ull) : b);
        };
        int nlive = 0, nsplit = 0;
        int at[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const uint64_t lm = __ballot(leader && ca[r] + cb[r] >= 2u);
            at[r] = nlive + groups_below(lm);
            nlive += __popcll(lm);
            nsplit += __popcll(__ballot(leader && split[r]));
        }
        if (nlive + nsplit > NR * CPR) return false;
        int nsp = nlive;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (ca[r] + cb[r] >= 2u) {
                uint64_t *e = stage + (size_t)at[r] * (W + 1);
#pragma unroll
                for (int t = 0; t < WPL; ++t) e[g * WPL + t] = m[r][t];
                if (leader) e[W] = (uint64_t)(ca[r] | (cb[r] << 16));
            }
            const uint64_t sm = __ballot(leader && split[r]);
            if (split[r]) {
                uint64_t *e = stage + (size_t)(nsp + groups_below(sm)) * (W + 1);
#pragma unroll
                for (int t = 0; t < WPL; ++t) e[g * WPL + t] = zm[r][t];
                if (leader) e[W] = (uint64_t)(za[r] | (zb[r] << 16));
            }
            nsp += __popcll(sm);
        }
        __syncthreads();
        kend = nsp;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int c = r * CPR + q;
            if (c < kend) {
                const uint64_t *e = stage + (size_t)c * (W + 1);
#pragma unroll
                for (int t = 0; t < WPL; ++t) m[r][t] = e[g * WPL + t];
                const uint32_t x = (uint32_t)e[W];
                ca[r] = x & 0xFFFFu;
                cb[r] = x >> 16;
            } else {
                ca[r] = cb[r] = 0u;
            }
        }
        __syncthreads();
        return true;
    };

    // ---- pairwise phase -------------------------------------------------------
    bool pmode = false;
    bool overflow = false;   // the classes outgrew the wave: the walk is redone elsewhere
    int npairs = 0;
    int nmem = 0;            // members of the pair list (memb), the haplotypes whose keys a pass reads
    uint32_t s_now = 0;   // S after the last marker processed
    if (MODE == MODE_CORE) s_now = choose2(core ? n1a : n0a);
    const bool can_pair = PCAP > 0 && a.hbits != nullptr;

    // Expand the live classes into the list of their member pairs; the class
    // masks are read from the registers of the lanes holding them.
    auto build_pairs = [&]() {
        npairs = 0;
        nmem = 0;
        for (int c = 0; c < kend; ++c) {
            const int rr = c / CPR, qq = c % CPR;
            uint32_t cnt = 0;
#pragma unroll
            for (int r = 0; r < NR; ++r)
                if (r == rr) cnt = __builtin_amdgcn_readlane(ca[r], qq * LPC);
            if (cnt < 2u) continue;   // an empty slot left by a class that died
            int sz = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                uint64_t mw = 0;
#pragma unroll
                for (int r = 0; r < NR; ++r)
                    if (r == rr) mw = readlane64(m[r][w % WPL], qq * LPC + w / WPL);
                if ((mw >> lane) & 1ull) memb[nmem + sz + (int)lanes_below(mw)] = (uint16_t)(64 * w + lane);
                sz += __popcll(mw);
            }
            // the class's members are entries nmem .. nmem + sz - 1 of the
            // member list; its pairs refer to them by entry
            for (int y = 1; y < sz; ++y) {
                const uint32_t my = (uint32_t)(nmem + y);
                const int base = npairs + y * (y - 1) / 2;
                for (int x0 = 0; x0 < y; x0 += 64) {
                    const int x = x0 + lane;
                    if (x < y) pairs[base + x] = (uint32_t)(nmem + x) | (my << 16);
                }
            }
            npairs += sz * (sz - 1) / 2;
            nmem += sz;
            __syncthreads();
        }
    };

    // Alleles of haplotype h at the 64 markers from k0 onwards in the walk's
    // direction, bit i = marker k0 + dir * i: the two words of the
    // haplotype-major row that hold them (zero outside the row) ...
    auto key_words = [&](int h, int64_t k0, uint64_t &lo, uint64_t &hi) {
        const uint64_t *row = a.hbits + (size_t)h * a.mwp;
        const int64_t b = dir > 0 ? k0 + 64 : k0 + 1;   // padded index of the lowest marker
        const int64_t wi = b >> 6;                       // (floor division)
        lo = wi >= 0 && wi < a.mwp ? row[wi] : 0ull;
        hi = wi + 1 >= 0 && wi + 1 < a.mwp ? row[wi + 1] : 0ull;
    };
    // ... and the key cut from them
    auto key_join = [&](int64_t k0, uint64_t lo, uint64_t hi) -> uint64_t {
        const int64_t b = dir > 0 ? k0 + 64 : k0 + 1;
        const int sh = (int)(b & 63);
        const uint64_t x = sh ? ((lo >> sh) | (hi << (64 - sh))) : lo;
        return dir > 0 ? x : __builtin_bitreverse64(x);
    };
    auto key_of = [&](int h, int64_t k0) -> uint64_t {
        uint64_t lo, hi;
        key_words(h, k0, lo, hi);
        return key_join(k0, lo, hi);
    };
    uint64_t pk_lo = 0ull, pk_hi = 0ull;   // member `lane`'s words for the next pass
    int pk_step = -1;                      // the pass they were loaded for

    if (can_pair && act && s_now <= (uint32_t)PCAP) {
        build_pairs();
        pmode = true;
    }

    while (act && !pmode) {
        // Long walks decide how long a whole scan takes: once a walk has gone
        // past a few hundred markers its wave takes issue priority over the
        // short walks sharing its SIMD.
        if (step >= 384) __builtin_amdgcn_s_setprio(3);
        else if (step >= 256) __builtin_amdgcn_s_setprio(2);
        else if (step >= 128) __builtin_amdgcn_s_setprio(1);

        // ---- lane i holds step i of the next 64: its row words go to LDS,
        // its segment (end of data, abort gap, or scaled genetic length)
        // stays in registers for the FP64 pass
        if (pf_step != step || !kPrefetchRows) fetch(step, true, pf_rows, pf_seg, pf_inr);
#pragma unroll
        for (int w = 0; w < W; ++w) rowbuf[lane * W + w] = pf_rows[w];
        const bool inr = pf_inr;
        const double segv = pf_seg;
        fetch(step + 64, kPrefetchRows, pf_rows, pf_seg, pf_inr);   // next batch, if the walk goes on
        pf_step = step + 64;
        int32_t stl = ST_OK;
        double gl = 0.0;
        if (!inr) stl = ST_EDGE;
        else if (segv < 0.0) stl = ST_GAP;
        else gl = segv;
        const uint64_t abort_mask = __ballot(stl != ST_OK);
        const int nb = abort_mask ? (int)__builtin_ctzll(abort_mask) : 64;
        const int32_t abort_st = abort_mask ? (int32_t)__builtin_amdgcn_readlane(stl, nb) : ST_OK;
        __syncthreads();

        // ---- markers that cut no class: with at most a.skip_classes classes
        // alive, lane i tests marker i against every class (a class is cut
        // when some but not all of its members carry allele 1); markers that
        // cut none leave the partition and the sums unchanged and are not
        // refined.  A marker that cuts no class of the batch's first partition
        // cuts none of its refinements either.
        // (The pooled walks of XPEHH end within a few markers of the first
        // splits, so they refine every marker: the test's registers cost
        // them a wave per SIMD and gain nothing.)
        uint64_t cutm = ~0ull;
        if (MODE == MODE_CORE && kend <= a.skip_classes) {
            bool cut = false;
            for (int c = 0; c < kend; ++c) {
                const int rr = c / CPR, qq = c % CPR;
                // a class is cut when it has members with allele 1 and members
                // with allele 0 (an empty slot has neither)
                bool one = false, zero = false;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    uint64_t mw = 0;
#pragma unroll
                    for (int r = 0; r < NR; ++r)
                        if (r == rr) mw = readlane64(m[r][w % WPL], qq * LPC + w / WPL);
                    const uint64_t rw = rowbuf[lane * W + w];
                    one = one || (mw & rw) != 0ull;
                    zero = zero || (mw & ~rw) != 0ull;
                }
                cut = cut || (one && zero);
            }
            cutm = __ballot(cut);
        }

        uint32_t sb = 0, sbB = 0;   // lane i: step i's S (A|B packed, or A) and S_B
        int nterm = 0;              // trapezoid terms of this batch
        int i = 0;
        bool to_pairs = false;
        for (; i < 64 && act; ++i) {
            if (i == nb) { status = abort_st; break; }
            if (!((cutm >> i) & 1ull)) {
                // markers i .. nxt-1 cut no class: the sums stay (above the
                // cutoff and the pair capacity) and each adds its term
                const uint64_t rest = cutm >> i;
                int nxt = rest ? i + (int)__builtin_ctzll(rest) : 64;
                if (nxt > nb) nxt = nb;
                if (lane >= i && lane < nxt) { sb = curS; sbB = curSB; }
                steps += nxt - i;
                nterm = nxt;
                i = nxt - 1;
                continue;
            }
            // the marker's row words, read from LDS where they are used: a
            // copy of the next marker's words held in registers cost more
            // (spills at 4 words, fewer waves at 8) than the LDS latency
            uint64_t rw[WPL];
#pragma unroll
            for (int t = 0; t < WPL; ++t) rw[t] = rowbuf[i * W + g * WPL + t];

            uint32_t acc = 0, accB = 0, accP = 0;
            bool split[NR];
            uint64_t zm[NR][WPL];
            uint32_t za[NR], zb[NR];
            uint64_t anysplit = 0;
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                split[r] = false;
                za[r] = zb[r] = 0u;
                if (r * CPR >= kend) continue;   // uniform
                uint32_t ow = 0;                 // ones in my words, A | B << 16
                uint64_t m1[WPL];
#pragma unroll
                for (int t = 0; t < WPL; ++t) {
                    m1[t] = m[r][t] & rw[t];
                    zm[r][t] = m[r][t] & ~rw[t];
                    const uint32_t pc = (uint32_t)__popcll(m1[t]);
                    ow += is_a(g * WPL + t) ? pc : (pc << 16);
                }
                const uint32_t os = group_sum<LPC>(ow);
                const uint32_t oa = os & 0xFFFFu, ob = os >> 16;
                const uint32_t zA = ca[r] - oa, zB = cb[r] - ob;
                const bool live = ca[r] + cb[r] >= 2u;
                bool ko, kz;
                if (MODE == MODE_CORE) {
                    if (leader && live) acc += choose2(oa) + choose2(zA);
                    ko = live && oa >= 2u;
                    kz = live && zA >= 2u;
                } else {
                    if (leader && live) {
                        const uint32_t sa = choose2(oa) + choose2(zA);
                        const uint32_t sbv = choose2(ob) + choose2(zB);
                        if (pack16) {
                            acc += sa | (sbv << 16);
                        } else {
                            acc += sa;
                            accB += sbv;
                        }
                        accP += choose2(oa + ob) + choose2(zA + zB);
                    }
                    ko = live && oa + ob >= 2u;
                    kz = live && zA + zB >= 2u;
                }
                split[r] = ko && kz;
#pragma unroll
                for (int t = 0; t < WPL; ++t) m[r][t] = ko ? m1[t] : zm[r][t];
                za[r] = zA;
                zb[r] = zB;
                ca[r] = ko ? oa : (kz ? zA : 0u);
                cb[r] = ko ? ob : (kz ? zB : 0u);
                anysplit |= __ballot(leader && split[r]);
            }
            const uint32_t S = wave_sum(acc);
            uint32_t SB = 0u, SP = 0u;
            if (MODE == MODE_POOLED) {
                SP = wave_sum(accP);
                if (!pack16) SB = wave_sum(accB);
            }
            if (anysplit) {
                if (!compact(split, zm, za, zb)) {   // more classes than rows
                    overflow = true;
                    break;
                }
            } else if (NR > 1 && kend > CPR && (i & 7) == 7) {
                // reclaim the holes left by classes that died, so that the
                // upper rows stop being processed once they are empty
                bool none[NR];
#pragma unroll
                for (int r = 0; r < NR; ++r) none[r] = false;
                compact(none, zm, za, zb);
            }

            // ---- record the step's sums and apply the stop rule -----------
            if (lane == i) { sb = S; sbB = SB; }
            curS = S;
            curSB = SB;
            steps += 1;
            const uint32_t Sst = MODE == MODE_CORE ? S : SP;
            if (Sst <= thr) act = false; else nterm = i + 1;
            s_now = S;
            if (can_pair && act && S <= (uint32_t)PCAP) {
                to_pairs = true;   // continue pairwise after this marker
                ++i;
                break;
            }
        }
        step += i;
        if (overflow) break;

        // ---- FP64 trapezoid of this batch: terms lane-parallel, sum in order
        if (nterm > 0) {
            const double g64 = gl;
            if (MODE == MODE_CORE) {
                const double e = (double)sb / PA;
                const double prev = lane_before(e, epA);
                double acc[1] = {ihhA};
                const double term[1] = {0.5 * (prev + e) * g64};
                add_terms<1>(acc, term, nterm, tbuf);
                ihhA = acc[0];
                epA = readlane_f64(e, nterm - 1);
            } else {
                const uint32_t sA = pack16 ? (sb & 0xFFFFu) : sb;
                const uint32_t sB = pack16 ? (sb >> 16) : sbB;
                const double eA = (double)sA / PA;
                const double eB = (double)sB / PB;
                const double pA = lane_before(eA, epA);
                const double pB = lane_before(eB, epB);
                double acc[2] = {ihhA, ihhB};
                const double term[2] = {0.5 * (pA + eA) * g64, 0.5 * (pB + eB) * g64};
                add_terms<2>(acc, term, nterm, tbuf);
                ihhA = acc[0];
                ihhB = acc[1];
                epA = readlane_f64(eA, nterm - 1);
                epB = readlane_f64(eB, nterm - 1);
            }
        }
        if (status != ST_OK) break;
        __syncthreads();   // the next batch overwrites the staged rows
        if (to_pairs) {
            build_pairs();
            pmode = true;
        }
    }

    // ---- pairwise phase: one pass over the pair list per 64 markers
    while (act && !overflow && status == ST_OK) {
        // Long walks decide how long a whole scan takes: once a walk has gone
        // past a few hundred markers its wave takes issue priority over the
        // short walks sharing its SIMD.
        if (step >= 384) __builtin_amdgcn_s_setprio(3);
        else if (step >= 256) __builtin_amdgcn_s_setprio(2);
        else if (step >= 128) __builtin_amdgcn_s_setprio(1);

        // ---- lane i holds step i of the next 64: its row words go to LDS,
        // its segment (end of data, abort gap, or scaled genetic length)
        // stays in registers for the FP64 pass
        if (pf_step != step) fetch(step, false, pf_rows, pf_seg, pf_inr);
        const bool inr = pf_inr;
        const double segv = pf_seg;
        fetch(step + 64, false, pf_rows, pf_seg, pf_inr);   // next batch, if the walk goes on
        pf_step = step + 64;
        int32_t stl = ST_OK;
        double gl = 0.0;
        if (!inr) stl = ST_EDGE;
        else if (segv < 0.0) stl = ST_GAP;
        else gl = segv;
        const uint64_t abort_mask = __ballot(stl != ST_OK);
        const int nb = abort_mask ? (int)__builtin_ctzll(abort_mask) : 64;
        const int32_t abort_st = abort_mask ? (int32_t)__builtin_amdgcn_readlane(stl, nb) : ST_OK;
        __syncthreads();

        uint32_t sb = 0, sbB = 0;   // lane i: step i's S (A|B packed, or A) and S_B
        int nterm = 0;              // trapezoid terms of this batch
        int i = 0;
        {
            // ---- one pass over the pair list covers the next 64 markers ----
            // keys of the pair list's members only; member `lane`'s words were
            // loaded during the previous pass
            const int64_t k0 = j + (int64_t)dir * (int64_t)(step + 1);
            if (lane < nmem) {
                if (pk_step != step) key_words((int)memb[lane], k0, pk_lo, pk_hi);
                keys[lane] = key_join(k0, pk_lo, pk_hi);
            }
            for (int h = lane + 64; h < nmem; h += 64) keys[h] = key_of((int)memb[h], k0);
            if (lane < nmem) key_words((int)memb[lane], k0 + (int64_t)dir * 64, pk_lo, pk_hi);
            pk_step = step + 64;
            hist[lane] = 0u;
            __syncthreads();
            int wpos = 0;
            for (int p0 = 0; p0 < npairs; p0 += 64) {
                const int p = p0 + lane;
                const bool in = p < npairs;
                const uint32_t pr = in ? pairs[p] : 0u;
                const uint64_t x = keys[pr & 0xFFFFu] ^ keys[pr >> 16];
                const int L = x ? (int)__builtin_ctzll(x) : 64;
                if (in && L < 64) atomicAdd(&hist[L], 1u);
                const bool surv = in && L == 64;
                const uint64_t sm = __ballot(surv);
                if (surv) pairs[wpos + (int)lanes_below(sm)] = pr;   // wpos <= p0: in place
                wpos += __popcll(sm);
            }
            __syncthreads();
            const uint32_t si = s_now - wave_prefix(hist[lane]);   // S after step `lane`
            const uint64_t valid = nb >= 64 ? ~0ull : ((1ull << nb) - 1ull);
            const uint64_t stopm = __ballot(si <= thr) & valid;
            if (stopm) {
                i = (int)__builtin_ctzll(stopm) + 1;
                nterm = i - 1;
                act = false;
            } else if (nb < 64) {
                i = nb;
                nterm = nb;
                status = abort_st;
            } else {
                i = 64;
                nterm = 64;
            }
            steps += i;
            sb = si;
            s_now = (uint32_t)__builtin_amdgcn_readlane(si, 63);
            npairs = wpos;
            __syncthreads();
        }
        step += i;

        // ---- FP64 trapezoid of this batch: terms lane-parallel, sum in order
        if (nterm > 0) {
            const double g64 = gl;
            if (MODE == MODE_CORE) {
                const double e = (double)sb / PA;
                const double prev = lane_before(e, epA);
                double acc[1] = {ihhA};
                const double term[1] = {0.5 * (prev + e) * g64};
                add_terms<1>(acc, term, nterm, tbuf);
                ihhA = acc[0];
                epA = readlane_f64(e, nterm - 1);
            } else {
                const uint32_t sA = pack16 ? (sb & 0xFFFFu) : sb;
                const uint32_t sB = pack16 ? (sb >> 16) : sbB;
                const double eA = (double)sA / PA;
                const double eB = (double)sB / PB;
                const double pA = lane_before(eA, epA);
                const double pB = lane_before(eB, epB);
                double acc[2] = {ihhA, ihhB};
                const double term[2] = {0.5 * (pA + eA) * g64, 0.5 * (pB + eB) * g64};
                add_terms<2>(acc, term, nterm, tbuf);
                ihhA = acc[0];
                ihhB = acc[1];
                epA = readlane_f64(eA, nterm - 1);
                epB = readlane_f64(eB, nterm - 1);
            }
        }
        if (status != ST_OK) break;
        __syncthreads();   // the next batch overwrites the staged rows
    }

    if (overflow) {
        // More live classes than the wave holds: this wave walks the site and
        // direction again from x0 with the class-id walk (class ids in
        // registers, counters in this workgroup's LDS), which writes the
        // records of both cores; the other core's wave, if it did not
        // overflow, writes the same values for its own.
        __syncthreads();
        walk_one<MODE, false, W>(a, j, d);
        return;
    }
    if (lane == 0) {
        const size_t o = (size_t)j * 2 + d;
        if (MODE == MODE_CORE) {
            put_rec(a.rec + o * 2 + core, ihhA, status, steps);
        } else {
            put_rec(a.rec + o * 2 + 0, ihhA, status, steps);
            put_rec(a.rec + o * 2 + 1, ihhB, status, 0);
        }
    }
}

template <int MODE, int W, int LPC>
hipError_t launch_nr(const WalkArgs &a, int nr, size_t lds, int64_t n_blocks, hipStream_t s) {
    const int64_t blocks = n_blocks * (MODE == MODE_CORE ? 4 : 2);
    if (blocks >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks);
    // one register row of classes, two for 16-word masks (mask_walk_shape);
    // walks that need more are walked again by the class-id walk
    if (nr == 1) {
        hipLaunchKernelGGL((mask_walk_kernel<MODE, W, LPC, 1>), grid, dim3(64), lds, s, a);
    } else if (nr == 2 && W == 16) {
        hipLaunchKernelGGL((mask_walk_kernel<MODE, W, LPC, 2>), grid, dim3(64), lds, s, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int MODE, int W>
hipError_t launch_lpc(const WalkArgs &a, const MaskShape &sh, int64_t n_blocks, hipStream_t s) {
    switch (sh.lpc) {
        case 1: return launch_nr<MODE, W, 1>(a, sh.rows, sh.lds, n_blocks, s);
        case 2: return launch_nr<MODE, W, (W >= 2 ? 2 : 1)>(a, sh.rows, sh.lds, n_blocks, s);
        case 4: return launch_nr<MODE, W, (W >= 4 ? 4 : 1)>(a, sh.rows, sh.lds, n_blocks, s);
        case 8: return launch_nr<MODE, W, (W >= 8 ? 8 : 1)>(a, sh.rows, sh.lds, n_blocks, s);
        default: return hipErrorInvalidValue;
    }
}

// 16-word masks: two or four lanes a class
template <int MODE>
hipError_t launch_wide(const WalkArgs &a, const MaskShape &sh, int64_t n_blocks, hipStream_t s) {
    switch (sh.lpc) {
        case 2: return launch_nr<MODE, 16, 2>(a, sh.rows, sh.lds, n_blocks, s);
        case 4: return launch_nr<MODE, 16, 4>(a, sh.rows, sh.lds, n_blocks, s);
        default: return hipErrorInvalidValue;
    }
}

int pow2_at_least(int x) {
    int p = 1;
    while (p < x) p *= 2;
    return p;
}

}  // namespace

MaskShape mask_walk_shape(int32_t nA, int32_t nB, int mode, int lpc) {
    MaskShape sh{};
    const int words = (nA + 63) / 64 + (mode == MODE_POOLED ? (nB + 63) / 64 : 0);
    const int n = nA + (mode == MODE_POOLED ? nB : 0);
    if (words > 16 || n > 1024) return sh;
    sh.words = pow2_at_least(words);   // 1, 2, 4, 8 or 16
    // default: one class per lane (64 classes per row) up to 8 words; 16-word
    // masks take two lanes a class (32 classes per row, 8 words a lane)
    if (lpc <= 0) lpc = sh.words == 16 ? 2 : 1;
    if (lpc > sh.words || (lpc & (lpc - 1))) return MaskShape{};
    if (sh.words == 16 && lpc != 2 && lpc != 4) return MaskShape{};
    sh.lpc = lpc;
    const int cpr = 64 / lpc;
    // Walks keep one row of classes in registers (two for 16-word masks, which
    // take two lanes a class); a walk that would need more (more than
    // rows * 64 / lpc multi-member classes at once) is walked again by the
    // class-id walk in the same workgroup, with this LDS.
    sh.rows = sh.words == 16 ? 2 : 1;
    sh.pair_cap = mode == MODE_CORE ? mask_pair_cap(sh.words) : 0;
    const size_t stage_words = (size_t)sh.rows * cpr * (sh.words + 1);
    const size_t union_words = stage_words > (size_t)sh.pair_cap / 2 ? stage_words
                                                                      : (size_t)sh.pair_cap / 2;
    sh.lds = ((size_t)64 * sh.words + union_words) * sizeof(uint64_t) + 64 * sizeof(uint32_t) +
             (size_t)64 * sh.words * sizeof(uint16_t);   // member list of the pair list
    const WalkShape ids = walk_shape(nA, nB, mode);      // the class-id walk's, for overflows
    if (ids.threads != 64 || ids.slots > sh.words) return MaskShape{};
    if (ids.lds > sh.lds) sh.lds = ids.lds;
    sh.ok = true;
    return sh;
}

bool mask_walk_supported(int32_t nA, int32_t nB, int mode) {
    return mask_walk_shape(nA, nB, mode, 0).ok;
}

hipError_t launch_mask_walk(const WalkArgs &a, int mode, int lpc, int64_t n_blocks, hipStream_t s) {
    const MaskShape sh = mask_walk_shape(a.nA, a.nB, mode, lpc);
    if (!sh.ok || !a.seg) return hipErrorInvalidValue;
    if (n_blocks <= 0) return hipSuccess;
    const bool core = mode == MODE_CORE;
    switch (sh.words) {
        case 1: return core ? launch_lpc<MODE_CORE, 1>(a, sh, n_blocks, s)
                            : launch_lpc<MODE_POOLED, 1>(a, sh, n_blocks, s);
        case 2: return core ? launch_lpc<MODE_CORE, 2>(a, sh, n_blocks, s)
                            : launch_lpc<MODE_POOLED, 2>(a, sh, n_blocks, s);
        case 4: return core ? launch_lpc<MODE_CORE, 4>(a, sh, n_blocks, s)
                            : launch_lpc<MODE_POOLED, 4>(a, sh, n_blocks, s);
        case 8: return core ? launch_lpc<MODE_CORE, 8>(a, sh, n_blocks, s)
                            : launch_lpc<MODE_POOLED, 8>(a, sh, n_blocks, s);
        case 16: return core ? launch_wide<MODE_CORE>(a, sh, n_blocks, s)
                             : launch_wide<MODE_POOLED>(a, sh, n_blocks, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ss

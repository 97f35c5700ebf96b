// EHH walks of a batch of regions in one persistent launch: class ids per
// haplotype, a pairwise tail for long walks, and a device work queue.
//
// What it computes is the partition refinement of ss_walk.hip (Sec. 1.1,
// Eqs. 1-3; Sec. 1.2, Eq. 4 and the rules below it; Sec. 1.3, Eq. 7 for the
// pooled XPEHH walk) with the same FP64 arithmetic in the same order.  Work
// items are (region, site, direction); both core alleles of an iHS site share
// one partition (Eq. 2), as in the plain kernel.
//
// Per item one workgroup of T threads:
//   * slot r of wave w holds the 64 haplotypes of word w + r * (T / 64) of the
//     marker rows; lane l's allele is bit l of the row word, its class id a
//     register.  Per marker the members with allele 1 count into their
//     class's LDS counter, then one pass over the classes makes the children,
//     drops those with < 2 members (and the classes of a core whose walk has
//     stopped), gives the survivors dense ids, and sums C(., 2).  iHS walks
//     take two markers per step: each member counts its pair of alleles (one
//     64-bit counter with 21-bit fields for 01, 10 and 11), the class pass
//     makes up to four children and the sums after each of the two markers
//     (the first from the children's sizes by first allele);
//   * once the identical pairs left (the iHS cores' pairs, or the pooled
//     pairs of XPEHH) number at most the pair capacity, the live classes are
//     expanded into the list of those pairs and each pass covers 64 markers:
//     XOR of the pair's 64-marker keys from the haplotype-major copy, lowest
//     set bit = the marker where the pair splits, per-type 64-bin histograms
//     give S at each marker of the pass;
//   * reference passes (iHS walks past their first 64 markers, at most 256
//     classes): a whole 64-marker batch at once when few members differ from
//     their class's lowest member within it.  A member's first difference
//     from the reference, and for members that leave at the same marker the
//     first difference of their keys, give every pair that splits in the
//     batch (Eq. 3 needs only the number of pairs still identical at each
//     marker), and the classes after the batch are the stayers plus the
//     leavers grouped by key.  Long walks through a sweep, a few large
//     classes of near-identical haplotypes, take most of their markers this
//     way;
//   * the grid is persistent: each workgroup takes the next `chunk` items from
//     a global counter until the batch is done, so walks of very different
//     lengths and regions of different sizes balance across the GPU.
#include "ss_internal.hpp"

namespace ss {

namespace {

constexpr int32_t DEAD = -1;
constexpr int kBig = 1 << 30;
// Copies of every class counter (8, or 1 where 8 would not fit in LDS):
// lane l adds into copy l % copies, so that the members of one large class
// spread their LDS atomics over several addresses (banks) instead of
// serializing on one.

__device__ __forceinline__ uint32_t choose2(uint32_t x) { return (x * (x - 1u)) >> 1; }

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) { return __ockl_wfred_add_u32(v); }

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int i) {
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, i);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), i);
    return ((uint64_t)hi << 32) | lo;
}

// A value every lane holds alike, marked wave-uniform for the compiler (so that
// addresses built from it stay in scalar registers and loads through them are
// scalar loads).
__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double readlane_f64(double v, int i) {
    return __builtin_bit_cast(double, readlane64(__builtin_bit_cast(uint64_t, v), i));
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint32_t wave_prefix(uint32_t v, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

__host__ __device__ inline uint64_t low_bits(int n) { return n >= 64 ? ~0ull : ((1ull << n) - 1ull); }

__device__ __forceinline__ uint64_t key_of(const uint64_t *hb, int64_t mwp, int h, int64_t k0,
                                           int dir) {
    const uint64_t *row = hb + (size_t)h * (size_t)mwp;
    const int64_t b = dir > 0 ? k0 + 64 : k0 + 1;   // padded index of the lowest marker
    const int64_t wi = b >> 6;
    const int sh = (int)(b & 63);
    const uint64_t lo = wi < mwp ? row[wi] : 0ull;
    const uint64_t hi = wi + 1 < mwp ? row[wi + 1] : 0ull;
    const uint64_t x = sh ? ((lo >> sh) | (hi << (64 - sh))) : lo;
    return dir > 0 ? x : __builtin_bitreverse64(x);
}

// Largest S in [0, P] with (double)S / (double)P < cutoff (P >= 1, cutoff >
// 0), found by testing 64 consecutive candidates around cutoff * P, one per
// lane: fl(S / P) is monotone in S, so a core's stop test is then the
// integer test S <= threshold.
__device__ __forceinline__ uint32_t stop_threshold(uint32_t P, double cutoff, int lane) {
    const double Pd = (double)P;
    int64_t s = (int64_t)(cutoff * Pd) - 32 + lane;
    if (s < 0) s = 0;
    if (s > (int64_t)P) s = (int64_t)P;
    const uint64_t m = __ballot((double)s / Pd < cutoff);
    const int top = 63 - __builtin_clzll(m);   // m != 0: candidate 0 is always below
    return (uint32_t)__builtin_amdgcn_readlane((uint32_t)s, top);
}

// Exclusive workgroup sum (u64); wtot holds one total per wave.
__device__ __forceinline__ uint64_t block_excl_sum(uint64_t v, uint64_t *wtot, uint64_t &total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t inc = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t a = __shfl_up(inc, off, 64);
        if (lane >= off) inc += a;
    }
    if (lane == 63) wtot[wave] = inc;
    __syncthreads();
    uint64_t off = 0, all = 0;
    const int nw = (int)(blockDim.x >> 6);
    for (int w = 0; w < nw; ++w) {
        const uint64_t s = wtot[w];
        all += s;
        if (w < wave) off += s;
    }
    total = all;
    return off + inc - v;
}

// LDS layout (byte offsets).  The class table lives until the pair list is
// built; keys, the second pair buffer and the histograms then reuse it.
struct BLay {
    uint32_t cnt1, szv0, szv1, map, sacc, knext, init, ovf, wtot, mem, pairs0;
    uint32_t keys, pairs1, hist, pcnt;
    uint32_t dref, dkey, dcnt, doff, ekey, einfo, elead, egid, dhist, dctl;   // reference pass
    uint32_t total;
    int kmax, copies;
};

// Reference pass: a walk that has gone kDevMinStep markers with at most
// kDevClasses classes tries each 64-marker batch in one step; the batch is
// refined marker by marker instead when more than kDevCap members leave
// their class's reference, or when the pairs among the leavers of a class
// (sum of squares of the leaver counts) exceed kDevWork.
constexpr int kDevClasses = 256;
constexpr int kDevCap = 512;
constexpr uint32_t kDevWork = 1u << 16;
constexpr int kDevMinStep = 64;

__host__ __device__ inline uint32_t al16(uint32_t x) { return (x + 15u) & ~15u; }

// kcls > 0 caps the class table (walks that outgrow it are listed for a
// launch with full tables); kcls = 0: room for every class a walk can have.
__host__ __device__ inline BLay batch_layout(int lmax, int kcls, int pcap, int kcap,
                                             int copies, bool dev) {
    BLay l;
    l.kmax = lmax / 2 + 2;
    if (kcls > 0 && kcls < l.kmax) l.kmax = kcls;
    l.copies = copies;
    const uint32_t K = (uint32_t)l.kmax;
    uint32_t o = 0;
    // counters: 32-bit ones per class and copy; steps over two markers use
    // the same space as 64-bit words of 21-bit fields for the allele pairs
    // 01, 10 and 11 (one word a class and copy for iHS, two for XPEHH's two
    // populations), over half or a quarter of the copies
    const uint32_t cw = 4u * K * (uint32_t)copies > 16u * K ? 4u * K * (uint32_t)copies : 16u * K;
    l.cnt1 = o;  o += cw;
    l.szv0 = o;  o += 4u * K;
    l.szv1 = o;  o += 4u * K;
    l.map = o;   o += 8u * K;    // children of each class (16-bit ids: 2 per marker, 4 per two)
    l.sacc = o;  o += 64u;
    l.knext = o; o += 8u;
    l.init = o;  o += 8u;
    l.ovf = o;   o += 8u;
    o = al16(o);
    const uint32_t table_end = o;
    // reuses the class table once the pair list exists
    uint32_t v = 0;
    l.keys = v;   v = al16(v + 8u * (uint32_t)kcap);
    l.pairs1 = v; v = al16(v + 4u * (uint32_t)pcap);
    l.hist = v;   v = al16(v + 4u * 3u * 64u);
    l.pcnt = v;   v = al16(v + 16u);
    o = table_end > v ? table_end : v;
    l.wtot = o;   o = al16(o + 8u * 16u);
    // the member and pair lists of the pairwise tail, and the reference
    // passes' arrays (which end before the tail starts), share what follows
    uint32_t t = o;
    l.mem = t;    t = al16(t + 2u * (uint32_t)kcap);
    l.pairs0 = t; t = al16(t + 4u * (uint32_t)pcap);
    uint32_t r = o;   // (no arrays without iHS walks: the offsets are not used)
    l.dref = r;   r = al16(r + 4u * kDevClasses);
    l.dkey = r;   r = al16(r + 8u * kDevClasses);
    l.dcnt = r;   r = al16(r + 4u * kDevClasses);
    l.doff = r;   r = al16(r + 4u * kDevClasses);
    l.ekey = r;   r = al16(r + 8u * kDevCap);
    l.einfo = r;  r = al16(r + 4u * kDevCap);
    l.elead = r;  r = al16(r + 4u * kDevCap);
    l.egid = r;   r = al16(r + 4u * kDevCap);
    l.dhist = r;  r = al16(r + 4u * 3u * 64u);
    l.dctl = r;   r = al16(r + 16u);
    l.total = dev && r > t ? r : t;
    return l;
}

template <int MODE, int R>
__device__ __forceinline__ void ids_walk(const Region *__restrict__ Gp, int64_t j, int d, char *base,
                         const BLay &Ly, int pcap, int kcap, bool dev, int64_t item, int64_t *redo,
                         int32_t *redo_count) {
    // fields are read through the pointer where they are used (scalar loads),
    // so that a copy of the descriptor does not hold registers for the walk
    const Region &G = *Gp;
    const int T = (int)blockDim.x;
    // (from a value the compiler cannot share with the persistent loop's, so
    // that indices built from it are not kept live across items)
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wpg = T >> 6;
    const int dir = d == 0 ? 1 : -1;
    const int nA = G.nA, nB = MODE == MODE_POOLED ? G.nB : 0;
    const int WA = (nA + 63) >> 6, WB = MODE == MODE_POOLED ? (nB + 63) >> 6 : 0;
    const int kmax = Ly.kmax;
    const int ncp = Ly.copies;   // 1 or 8

    uint32_t *cnt1 = (uint32_t *)(base + Ly.cnt1);
    uint32_t *szv0 = (uint32_t *)(base + Ly.szv0);
    uint32_t *szv1 = (uint32_t *)(base + Ly.szv1);
    int32_t *map = (int32_t *)(base + Ly.map);
    uint32_t *sacc = (uint32_t *)(base + Ly.sacc);
    int32_t *knext = (int32_t *)(base + Ly.knext);
    uint32_t *init = (uint32_t *)(base + Ly.init);
    int32_t *ovf = (int32_t *)(base + Ly.ovf);   // the class table overflowed

    for (int i = tid; i < (ncp > 4 ? kmax * ncp : 4 * kmax); i += T) cnt1[i] = 0u;
    if (tid < 16) sacc[tid] = 0u;
    if (tid < 2) {
        knext[tid] = 0;
        init[tid] = 0u;
    }
    if (tid == 0) *ovf = 0;

    // slot r: 64-haplotype word wq = wave + r * wpg of the pooled word space
    // (A's words, then B's); its row word at site k is computed where needed
    const int Wused = WA + WB;
    auto row_at = [&](int r, int64_t k) -> uint64_t {
        const int wq = wave + r * wpg;
        return wq < WA ? G.bitsA[k * G.wpsA + wq] : G.bitsB[k * G.wpsB + (wq - WA)];
    };
    auto word = [&](int r) -> bool { return wave + r * wpg < Wused; };
    // count increment of slot r's members: 1 in population A, 1 << 16 in B
    // (wave-uniform; iHS has A only)
    auto incu = [&](int r) -> uint32_t {
        return MODE == MODE_CORE ? 1u
                                 : (uint32_t)__builtin_amdgcn_readfirstlane(wave + r * wpg < WA ? 1u : 0x10000u);
    };
    int32_t cls[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int wq = wave + r * wpg;
        const bool valid = wq < WA ? wq * 64 + lane < nA
                                   : (wq < Wused && (wq - WA) * 64 + lane < nB);
        cls[r] = valid ? 0 : DEAD;
    }
    __syncthreads();

    // classes at x0: id = allele
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (word(r)) {
            const uint64_t w = row_at(r, j);
            const int32_t bit = (int32_t)((w >> lane) & 1ull);
            if (cls[r] != DEAD) {
                cls[r] = bit;
                atomicAdd(&init[bit], incu(r));
            }
        }
    }
    __syncthreads();
    const uint32_t i0 = init[0], i1 = init[1];

    bool act0, act1;
    // The EHH values and iHH sums are wave 0's (it writes the results); every
    // wave takes the same stop decisions from exact integer thresholds:
    // a core stops at the first marker with S <= thr (iHS: per core; XPEHH:
    // the pooled S against thr0).
    double ihh0 = 0.0, ihh1 = 0.0, ep0, ep1, P0, P1;
    uint32_t thr0 = 0u, thr1 = 0u;
    int32_t steps0 = 0, steps1 = 0;
    uint32_t sa0, sa1, sa2 = 0;   // S after the last marker (iHS: cores 0, 1; XPEHH: A, B, pooled)
    if (MODE == MODE_CORE) {
        const uint32_t n0 = i0 & 0xFFFFu, n1 = i1 & 0xFFFFu;
        P0 = (double)choose2(n0);
        P1 = (double)choose2(n1);
        act0 = n0 >= 2u;
        act1 = n1 >= 2u;
        if (act0) thr0 = stop_threshold(choose2(n0), G.cutoff, lane);
        if (act1) thr1 = stop_threshold(choose2(n1), G.cutoff, lane);
        ep0 = 1.0;
        ep1 = 1.0;
        sa0 = choose2(n0);
        sa1 = choose2(n1);
        if (tid == 0) {
            szv0[0] = n0;
            szv0[1] = n1 | 0x80000000u;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (cls[r] == 0 && n0 < 2u) cls[r] = DEAD;
            if (cls[r] == 1 && n1 < 2u) cls[r] = DEAD;
        }
    } else {
        const uint32_t a0 = i0 & 0xFFFFu, b0 = i0 >> 16, a1 = i1 & 0xFFFFu, b1 = i1 >> 16;
        P0 = (double)choose2((uint32_t)nA);
        P1 = (double)choose2((uint32_t)nB);
        // x0 is part of the haplotype: each population's curve starts at its
        // whole-sample EHH at x0
        ep0 = (double)(choose2(a0) + choose2(a1)) / P0;
        ep1 = (double)(choose2(b0) + choose2(b1)) / P1;
        act0 = true;
        act1 = false;
        thr0 = stop_threshold(choose2((uint32_t)(nA + nB)), G.cutoff, lane);
        sa0 = choose2(a0) + choose2(a1);
        sa1 = choose2(b0) + choose2(b1);
        sa2 = choose2(a0 + b0) + choose2(a1 + b1);
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

    const bool can_pair = pcap > 0 && G.hbitsA != nullptr &&
                          (MODE == MODE_CORE || G.hbitsB != nullptr);
    int32_t K = 2;
    int32_t status = ST_OK;
    int step = 0;
    bool pmode = false;
    // the two class-size arrays take turns by marker parity; a reference
    // pass (64 markers, an even count) swaps them once more
    int pflip = 0;
    // (iHS walks: the pooled walks of XPEHH end within a few markers of their
    // first splits, and the pass's code would cost their per-marker loop
    // registers)
    const bool can_dev = MODE == MODE_CORE && dev && G.hbitsA != nullptr;

    // End of a 64-marker pass: hist[t][L] counts the class-mate pairs of type
    // t (iHS: core 0, core 1; XPEHH: pooled, A-A, B-B) whose alleles first
    // differ at marker L of the pass, so S after marker L is the S before the
    // pass less the prefix sum; then each walking core's stop test, steps
    // and trapezoid terms (added in marker order).  Markers from nb on are
    // past an abort and are not walked.
    auto settle = [&](const uint32_t *hist, int nb, double gl) {
        const uint64_t valid = low_bits(nb);
        const int lim = nb < 64 ? nb : 64;
        if (MODE == MODE_CORE) {
            // each core stops at its own first sub-cutoff marker of the pass
            const uint32_t si0 = sa0 - wave_prefix(hist[lane], lane);
            const uint32_t si1 = sa1 - wave_prefix(hist[64 + lane], lane);
            if (act0) {
                const uint64_t sm = __ballot(si0 <= thr0) & valid;
                const int nterm = sm ? (int)__builtin_ctzll(sm) : lim;
                steps0 += sm ? nterm + 1 : lim;
                if (nterm > 0) {
                    const double e = (double)si0 / P0;
                    double prev = __shfl_up(e, 1, 64);
                    if (lane == 0) prev = ep0;
                    const double term = 0.5 * (prev + e) * gl;
                    for (int t = 0; t < nterm; ++t) ihh0 += readlane_f64(term, t);
                    ep0 = readlane_f64(e, nterm - 1);
                }
                if (sm) act0 = false;
            }
            if (act1) {
                const uint64_t sm = __ballot(si1 <= thr1) & valid;
                const int nterm = sm ? (int)__builtin_ctzll(sm) : lim;
                steps1 += sm ? nterm + 1 : lim;
                if (nterm > 0) {
                    const double e = (double)si1 / P1;
                    double prev = __shfl_up(e, 1, 64);
                    if (lane == 0) prev = ep1;
                    const double term = 0.5 * (prev + e) * gl;
                    for (int t = 0; t < nterm; ++t) ihh1 += readlane_f64(term, t);
                    ep1 = readlane_f64(e, nterm - 1);
                }
                if (sm) act1 = false;
            }
            sa0 = (uint32_t)__builtin_amdgcn_readlane(si0, 63);
            sa1 = (uint32_t)__builtin_amdgcn_readlane(si1, 63);
        } else {
            const uint32_t siP = sa2 - wave_prefix(hist[lane], lane);
            const uint32_t siA = sa0 - wave_prefix(hist[64 + lane], lane);
            const uint32_t siB = sa1 - wave_prefix(hist[128 + lane], lane);
            const uint64_t sm = __ballot(siP <= thr0) & valid;
            const int nterm = sm ? (int)__builtin_ctzll(sm) : lim;
            steps0 += sm ? nterm + 1 : lim;
            if (nterm > 0) {
                const double eA = (double)siA / P0;
                const double eB = (double)siB / P1;
                double pA = __shfl_up(eA, 1, 64);
                double pBv = __shfl_up(eB, 1, 64);
                if (lane == 0) {
                    pA = ep0;
                    pBv = ep1;
                }
                const double tA = 0.5 * (pA + eA) * gl;
                const double tB = 0.5 * (pBv + eB) * gl;
                for (int t = 0; t < nterm; ++t) {
                    ihh0 += readlane_f64(tA, t);
                    ihh1 += readlane_f64(tB, t);
                }
                ep0 = readlane_f64(eA, nterm - 1);
                ep1 = readlane_f64(eB, nterm - 1);
            }
            if (sm) act0 = false;
            sa2 = (uint32_t)__builtin_amdgcn_readlane(siP, 63);
            sa0 = (uint32_t)__builtin_amdgcn_readlane(siA, 63);
            sa1 = (uint32_t)__builtin_amdgcn_readlane(siB, 63);
        }
    };

    while (act0 || act1) {
        if (can_dev && step >= kDevMinStep && K <= kDevClasses) {
            // ---- reference pass over the next 64 markers ---------------------
            // Each class's lowest member is its reference; a member "leaves" at
            // the first marker where its 64-marker key differs from the
            // reference's.  Two class-mates that leave at different markers
            // (or one that never leaves) first differ where the earlier one
            // leaves; two that leave at the same marker agree there and first
            // differ where their keys do.  So every pair that splits in the
            // pass is counted from the leavers alone, and the classes after
            // the pass are each class's stayers plus its leavers grouped by
            // key.
            const int par = (step & 1) ^ pflip;
            uint32_t *szc = par ? szv1 : szv0;
            uint32_t *szn = par ? szv0 : szv1;
            uint32_t *dref = (uint32_t *)(base + Ly.dref);   // [class] lowest member
            uint64_t *dkey = (uint64_t *)(base + Ly.dkey);   // [class] its key
            uint32_t *dcnt = (uint32_t *)(base + Ly.dcnt);   // [class] leavers, A | B << 16
            uint32_t *doff = (uint32_t *)(base + Ly.doff);   // [class] first entry of its leavers
            uint64_t *ekey = (uint64_t *)(base + Ly.ekey);   // [leaver] key
            uint32_t *einfo = (uint32_t *)(base + Ly.einfo); // [leaver] class | marker << 8 | B << 14 | member << 15
            int32_t *elead = (int32_t *)(base + Ly.elead);   // [leaver] first leaver with its key
            int32_t *egid = (int32_t *)(base + Ly.egid);     // [leaver] group size, then new class
            uint32_t *dhist = (uint32_t *)(base + Ly.dhist); // [3][64] pairs splitting per marker
            uint32_t *dctl = (uint32_t *)(base + Ly.dctl);   // leavers, their pair work, classes, members
            uint64_t *wtot = (uint64_t *)(base + Ly.wtot);
            for (int c = tid; c < K; c += T) {
                dref[c] = 0xFFFFFFFFu;
                dcnt[c] = 0u;
            }
            for (int x = tid; x < 3 * 64; x += T) dhist[x] = 0u;
            if (tid < 4) dctl[tid] = 0u;
            const int64_t k0 = j + (int64_t)dir * (int64_t)(step + 1);
            const int64_t kb = k0 + (int64_t)dir * (int64_t)lane;
            const bool inr = kb >= 0 && kb < G.M;
            const double sv = inr ? G.seg[dir > 0 ? kb : kb + 1] : 0.0;
            const int32_t stl = !inr ? ST_EDGE : (sv < 0.0 ? ST_GAP : ST_OK);
            const double gl = stl == ST_OK ? sv : 0.0;
            const uint64_t abort_mask = __ballot(stl != ST_OK);
            const int nb = abort_mask ? (int)__builtin_ctzll(abort_mask) : 64;
            const int32_t abort_st = abort_mask ? (int32_t)__builtin_amdgcn_readlane(stl, nb) : ST_OK;
            // member index of slot r: (word) * 64 + lane, built from a value
            // the compiler cannot hoist out of the walk's loop (sixteen
            // hoisted indices or row addresses would hold registers for the
            // whole walk)
            uint32_t g0 = (uint32_t)(wave * 64 + lane);
            asm volatile("" : "+v"(g0));
            auto gid = [&](int r) -> uint32_t { return g0 + (uint32_t)(r * wpg * 64); };
            auto hkey = [&](int r) -> uint64_t {
                const int wq = wave + r * wpg;
                return wq < WA ? key_of(G.hbitsA, G.mwp, (int)gid(r), k0, dir)
                               : key_of(G.hbitsB, G.mwp, (int)gid(r) - WA * 64, k0, dir);
            };
            __syncthreads();
            // (1) references.  Members of a stopped core's classes leave the
            // walk now (the next marker would drop them as well).
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (cls[r] != DEAD) {
                    if (MODE == MODE_CORE && !((szc[cls[r]] >> 31) ? act1 : act0)) cls[r] = DEAD;
                    else atomicMin(&dref[cls[r]], gid(r));
                }
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (cls[r] != DEAD && dref[cls[r]] == gid(r)) dkey[cls[r]] = hkey(r);
            __syncthreads();
            // (2) the leavers (bit r of leave: slot r's member leaves), counted
            // per class
            uint32_t leave = 0u, nd = 0u, sq = 0u;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (cls[r] != DEAD && hkey(r) != dkey[cls[r]]) {
                    const uint32_t old = atomicAdd(&dcnt[cls[r]], incu(r));
                    const uint32_t rank = (old & 0xFFFFu) + (old >> 16);
                    leave |= 1u << r;
                    nd += 1u;
                    sq += 2u * rank + 1u;
                }
            }
            nd = wave_sum(nd);
            sq = wave_sum(sq);
            if (lane == 0 && nd) {
                atomicAdd(&dctl[0], nd);
                atomicAdd(&dctl[1], sq);
            }
            __syncthreads();
            const uint32_t D = dctl[0], SQ = dctl[1];
            if (D <= (uint32_t)kDevCap && SQ <= kDevWork) {
                // (3) each class's leavers into one run of entries (dref, no
                // longer needed, becomes each run's fill cursor)
                const int KT = (K + T - 1) / T;
                uint64_t loc = 0;
                for (int qq = 0; qq < KT; ++qq) {
                    const int c = tid * KT + qq;
                    if (c < K) {
                        const uint32_t v = dcnt[c];
                        loc += (v & 0xFFFFu) + (v >> 16);
                    }
                }
                uint64_t tot;
                uint64_t ex = block_excl_sum(loc, wtot, tot);
                for (int qq = 0; qq < KT; ++qq) {
                    const int c = tid * KT + qq;
                    if (c < K) {
                        doff[c] = (uint32_t)ex;
                        dref[c] = (uint32_t)ex;
                        const uint32_t v = dcnt[c];
                        ex += (v & 0xFFFFu) + (v >> 16);
                    }
                }
                __syncthreads();
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if ((leave >> r) & 1u) {
                        const int x = (int)atomicAdd(&dref[cls[r]], 1u);
                        const uint64_t kx = hkey(r);
                        ekey[x] = kx;
                        const uint32_t dx = (uint32_t)__builtin_ctzll(kx ^ dkey[cls[r]]);
                        einfo[x] = (uint32_t)cls[r] | (dx << 8) | ((incu(r) >> 16) << 14) | (gid(r) << 15);
                    }
                }
                __syncthreads();
                // (4) per leaver: its pairs with the class-mates that leave
                // later or never (split where it leaves), its pairs with the
                // earlier entries leaving at the same marker (split where the
                // keys differ), and the first entry with its whole key
                for (int x = tid; x < (int)D; x += T) {
                    const uint32_t inf = einfo[x];
                    const int c = (int)(inf & 0xFFu);
                    const uint32_t dx = (inf >> 8) & 63u;
                    const bool xb = ((inf >> 14) & 1u) != 0u;
                    const uint64_t kx = ekey[x];
                    const int s0 = (int)doff[c];
                    const uint32_t dv = dcnt[c];
                    const int s1 = s0 + (int)((dv & 0xFFFFu) + (dv >> 16));
                    const uint32_t sz = szc[c];
                    uint32_t leA = 0u, leB = 0u, gA = 0u, gB = 0u;
                    int lead = x;
                    for (int y = s0; y < s1; ++y) {
                        const uint32_t iy = einfo[y];
                        const uint32_t dy = (iy >> 8) & 63u;
                        const bool yb = ((iy >> 14) & 1u) != 0u;
                        if (dy <= dx) {
                            if (yb) ++leB;
                            else ++leA;
                        }
                        if (dy == dx) {
                            const uint64_t z = kx ^ ekey[y];
                            if (z == 0ull) {
                                if (yb) ++gB;
                                else ++gA;
                                if (y < lead) lead = y;
                            } else if (y < x) {
                                const int L = (int)__builtin_ctzll(z);
                                if (MODE == MODE_CORE) {
                                    atomicAdd(&dhist[(sz >> 31) * 64u + (uint32_t)L], 1u);
                                } else {
                                    atomicAdd(&dhist[L], 1u);
                                    if (!xb && !yb) atomicAdd(&dhist[64 + L], 1u);
                                    else if (xb && yb) atomicAdd(&dhist[128 + L], 1u);
                                }
                            }
                        }
                    }
                    if (MODE == MODE_CORE) {
                        const uint32_t rest = (sz & 0xFFFFu) - leA;
                        if (rest) atomicAdd(&dhist[(sz >> 31) * 64u + dx], rest);
                    } else {
                        const uint32_t nA = sz & 0xFFFFu, nB = sz >> 16;
                        const uint32_t rest = nA + nB - leA - leB;
                        if (rest) atomicAdd(&dhist[dx], rest);
                        const uint32_t same = xb ? nB - leB : nA - leA;
                        if (same) atomicAdd(&dhist[(xb ? 128u : 64u) + dx], same);
                    }
                    elead[x] = lead;
                    if (lead == x) egid[x] = (int32_t)(gA | (gB << 16));
                }
                __syncthreads();
                settle(dhist, nb, gl);
                if (!(act0 || act1)) goto done;
                if (nb < 64) {
                    status = abort_st;
                    goto done;
                }
                // (5) the classes after the pass: stayers, and groups of
                // leavers with one key, of >= 2 members of a walking core
                for (int c = tid; c < K; c += T) {
                    const uint32_t sz = szc[c], dv = dcnt[c];
                    uint32_t nsz, cnt;
                    bool keep;
                    if (MODE == MODE_CORE) {
                        cnt = (sz & 0xFFFFu) - (dv & 0xFFFFu);
                        keep = ((sz >> 31) ? act1 : act0) && cnt >= 2u;
                        nsz = cnt | (sz & 0x80000000u);
                    } else {
                        const uint32_t ra = (sz & 0xFFFFu) - (dv & 0xFFFFu), rb = (sz >> 16) - (dv >> 16);
                        cnt = ra + rb;
                        keep = cnt >= 2u;
                        nsz = ra | (rb << 16);
                    }
                    int32_t id = DEAD;
                    if (keep) {
                        id = (int32_t)atomicAdd(&dctl[2], 1u);
                        if (id < kmax) szn[id] = nsz;
                        atomicAdd(&dctl[3], cnt);
                    }
                    map[2 * c] = id;
                }
                for (int x = tid; x < (int)D; x += T) {
                    if (elead[x] != x) continue;
                    const uint32_t g = (uint32_t)egid[x];
                    const uint32_t cnt = (g & 0xFFFFu) + (g >> 16);
                    const uint32_t sz = szc[einfo[x] & 0xFFu];
                    const bool keep = (MODE == MODE_CORE ? ((sz >> 31) ? act1 : act0) : true) && cnt >= 2u;
                    int32_t id = DEAD;
                    if (keep) {
                        id = (int32_t)atomicAdd(&dctl[2], 1u);
                        if (id < kmax) szn[id] = MODE == MODE_CORE ? (cnt | (sz & 0x80000000u)) : g;
                        atomicAdd(&dctl[3], cnt);
                    }
                    egid[x] = id;
                }
                __syncthreads();
                const int Kn = (int)dctl[2];
                const uint32_t members = dctl[3];
                if (Kn > kmax) goto overflowed;   // the walk is redone with full tables
                // members: a stayer takes its class's new id, a leaver finds
                // its entry in its class's run and takes its group's
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (cls[r] == DEAD) continue;
                    if ((leave >> r) & 1u) {
                        const int c = cls[r];
                        const int s0 = (int)doff[c];
                        const uint32_t dv = dcnt[c];
                        const int s1 = s0 + (int)((dv & 0xFFFFu) + (dv >> 16));
                        int x = s0;
                        while (x < s1 - 1 && (einfo[x] >> 15) != gid(r)) ++x;
                        cls[r] = egid[elead[x]];
                    } else {
                        cls[r] = map[2 * cls[r]];
                    }
                }
                K = Kn;
                pflip ^= 1;
                step += 64;
                if (tid < 16) sacc[tid] = 0u;
                if (tid < 2) knext[tid] = 0;
                __syncthreads();
                if (can_pair && (act0 || act1)) {
                    const uint32_t left = MODE == MODE_CORE ? (act0 ? sa0 : 0u) + (act1 ? sa1 : 0u) : sa2;
                    if (left <= (uint32_t)pcap && members <= (uint32_t)kcap) {
                        pmode = true;
                        goto pairs;
                    }
                }
                continue;
            }
            __syncthreads();   // a pass not taken: its arrays are free again
        }
        // stage the next 64 markers: lane i holds the row words and the
        // segment of step (step + 1 + i)
        const int64_t kb = j + (int64_t)dir * (int64_t)(step + 1 + lane);
        const bool inr = kb >= 0 && kb < G.M;
        uint64_t rowv[R];
#pragma unroll
        for (int r = 0; r < R; ++r) rowv[r] = (word(r) && inr) ? row_at(r, kb) : 0ull;
        int32_t stl = ST_OK;
        double gl = 0.0;
        if (!inr) {
            stl = ST_EDGE;
        } else {
            const double sv = G.seg[dir > 0 ? kb : kb + 1];
            if (sv < 0.0) stl = ST_GAP;
            else gl = sv;
        }
        const uint64_t abort_mask = __ballot(stl != ST_OK);
        const int nb = abort_mask ? (int)__builtin_ctzll(abort_mask) : 64;
        const int32_t abort_st = abort_mask ? (int32_t)__builtin_amdgcn_readlane(stl, nb) : ST_OK;

        for (int i = 0; i < 64 && (act0 || act1);) {
            if (i == nb) {
                status = abort_st;
                goto done;
            }
            // Walks refine two markers per step while both are walked: one
            // count per member of its alleles at both, one class pass making
            // the up to four children (S after the first marker from the
            // children's pairs by first allele), so half the workgroup
            // barriers and LDS round trips per marker.
            const bool two = i + 1 < nb && i + 1 < 64;
            const int par = (step & 1) ^ pflip;
            uint32_t *szc = par ? szv1 : szv0;
            uint32_t *szn = par ? szv0 : szv1;
            uint32_t *sa = sacc + 8 * par;
            int32_t *kn = knext + par;
            uint64_t *cnt2 = (uint64_t *)cnt1;
            int16_t *cmap = (int16_t *)map;   // children of each class
            const int h2 = ncp > 1 ? ncp >> 1 : 1;   // 64-bit counter copies (iHS)
            const int h4 = ncp > 3 ? ncp >> 2 : 1;   // pairs of them (XPEHH)

            // (1) alleles per class; a member's class id becomes its child's
            // index in the class pass's map: 2 * class + allele, or
            // 4 * class + (first allele) * 2 + second allele
            if (two) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (word(r) && cls[r] != DEAD) {
                        const int32_t b1 = (int32_t)((readlane64(rowv[r], i) >> lane) & 1ull);
                        const int32_t b2 = (int32_t)((readlane64(rowv[r], i + 1) >> lane) & 1ull);
                        const int32_t ab = 2 * b1 + b2;
                        if (MODE == MODE_CORE) {
                            if (ab) atomicAdd(&cnt2[cls[r] * h2 + (lane & (h2 - 1))], 1ull << (21 * (ab - 1)));
                        } else {
                            // two words a copy: population A's, B's
                            if (ab) atomicAdd(&cnt2[2 * (cls[r] * h4 + (lane & (h4 - 1))) + (int)(incu(r) >> 16)],
                                              1ull << (21 * (ab - 1)));
                        }
                        cls[r] = 4 * cls[r] + ab;
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (word(r) && cls[r] != DEAD) {
                        const uint64_t w = readlane64(rowv[r], i);
                        const int32_t bit = (int32_t)((w >> lane) & 1ull);
                        if (bit) atomicAdd(&cnt1[cls[r] * ncp + (lane & (ncp - 1))], incu(r));
                        cls[r] = 2 * cls[r] + bit;
                    }
                }
            }
            __syncthreads();

            // (2) split every class, keep children with >= 2 members
            if (MODE == MODE_CORE && two) {
                for (int c0 = 0; c0 < K; c0 += T) {
                    const int c = c0 + tid;
                    const bool in = c < K;
                    uint64_t f = 0ull;
                    uint32_t sz = 0u;
                    if (in) {
                        for (int q = 0; q < h2; ++q) {
                            f += cnt2[c * h2 + q];
                            cnt2[c * h2 + q] = 0ull;
                        }
                        sz = szc[c];
                    }
                    const uint32_t core = sz >> 31;
                    const uint32_t n = sz & 0xFFFFu;
                    const uint32_t m01 = (uint32_t)(f & 0x1FFFFFull);
                    const uint32_t m10 = (uint32_t)((f >> 21) & 0x1FFFFFull);
                    const uint32_t m11 = (uint32_t)(f >> 42);
                    const uint32_t m00 = n - m01 - m10 - m11;
                    const bool live = in && (core ? act1 : act0);
                    // S after the first marker (children by first allele) and
                    // after the second (the four children)
                    const uint32_t sf = in ? choose2(m00 + m01) + choose2(m10 + m11) : 0u;
                    const uint32_t ss2 = in ? choose2(m00) + choose2(m01) + choose2(m10) + choose2(m11) : 0u;
                    const bool k00 = live && m00 >= 2u, k01 = live && m01 >= 2u;
                    const bool k10 = live && m10 >= 2u, k11 = live && m11 >= 2u;
                    uint32_t s3 = (k00 ? m00 : 0u) + (k01 ? m01 : 0u) + (k10 ? m10 : 0u) + (k11 ? m11 : 0u);
                    const uint64_t b00 = __ballot(k00), b01 = __ballot(k01);
                    const uint64_t b10 = __ballot(k10), b11 = __ballot(k11);
                    const int n00 = __popcll(b00), n01 = __popcll(b01);
                    const int n10 = __popcll(b10), n11 = __popcll(b11);
                    const int nk = n00 + n01 + n10 + n11;
                    int basei = 0;
                    if (wpg == 1) {
                        basei = kn[0];
                    } else {
                        if (lane == 0 && nk > 0) basei = atomicAdd(kn, nk);
                        basei = __shfl(basei, 0, 64);
                    }
                    const int i00 = basei + (int)lanes_below(b00);
                    const int i01 = basei + n00 + (int)lanes_below(b01);
                    const int i10 = basei + n00 + n01 + (int)lanes_below(b10);
                    const int i11 = basei + n00 + n01 + n10 + (int)lanes_below(b11);
                    const bool fits = basei + nk <= kmax;   // wave-uniform
                    if (!fits && lane == 0) *ovf = 1;
                    if (in) {
                        cmap[4 * c + 0] = (int16_t)(k00 ? i00 : DEAD);
                        cmap[4 * c + 1] = (int16_t)(k01 ? i01 : DEAD);
                        cmap[4 * c + 2] = (int16_t)(k10 ? i10 : DEAD);
                        cmap[4 * c + 3] = (int16_t)(k11 ? i11 : DEAD);
                    }
                    if (fits) {
                        const uint32_t cb = core << 31;
                        if (k00) szn[i00] = m00 | cb;
                        if (k01) szn[i01] = m01 | cb;
                        if (k10) szn[i10] = m10 | cb;
                        if (k11) szn[i11] = m11 | cb;
                    }
                    uint32_t f0 = core ? 0u : sf, f1 = core ? sf : 0u;
                    uint32_t t0 = core ? 0u : ss2, t1 = core ? ss2 : 0u;
                    f0 = wave_sum(f0);
                    f1 = wave_sum(f1);
                    t0 = wave_sum(t0);
                    t1 = wave_sum(t1);
                    if (can_pair) s3 = wave_sum(s3);
                    if (lane == 0) {
                        if (wpg == 1) {
                            kn[0] = basei + nk;
                            sa[0] += t0;
                            sa[1] += t1;
                            sa[3] += s3;
                            sa[4] += f0;
                            sa[5] += f1;
                        } else {
                            if (t0) atomicAdd(&sa[0], t0);
                            if (t1) atomicAdd(&sa[1], t1);
                            if (s3) atomicAdd(&sa[3], s3);
                            if (f0) atomicAdd(&sa[4], f0);
                            if (f1) atomicAdd(&sa[5], f1);
                        }
                    }
                    if (wpg == 1) __syncthreads();   // kn[0] is read again next round
                }
            } else if (two) {
                const int h = h4;
                for (int c0 = 0; c0 < K; c0 += T) {
                    const int c = c0 + tid;
                    const bool in = c < K;
                    uint64_t fa = 0ull, fb = 0ull;
                    uint32_t sz = 0u;
                    if (in) {
                        for (int q = 0; q < h; ++q) {
                            fa += cnt2[2 * (c * h + q)];
                            fb += cnt2[2 * (c * h + q) + 1];
                            cnt2[2 * (c * h + q)] = 0ull;
                            cnt2[2 * (c * h + q) + 1] = 0ull;
                        }
                        sz = szc[c];
                    }
                    const uint32_t nA = sz & 0xFFFFu, nB = sz >> 16;
                    const uint32_t a01 = (uint32_t)(fa & 0x1FFFFFull), a10 = (uint32_t)((fa >> 21) & 0x1FFFFFull);
                    const uint32_t a11 = (uint32_t)(fa >> 42), a00 = nA - a01 - a10 - a11;
                    const uint32_t b01 = (uint32_t)(fb & 0x1FFFFFull), b10 = (uint32_t)((fb >> 21) & 0x1FFFFFull);
                    const uint32_t b11 = (uint32_t)(fb >> 42), b00 = nB - b01 - b10 - b11;
                    // S of A, of B and pooled after the first marker and after the second
                    uint32_t fA = 0u, fB = 0u, fP = 0u, tA = 0u, tB = 0u, tP = 0u;
                    if (in) {
                        fA = choose2(a00 + a01) + choose2(a10 + a11);
                        fB = choose2(b00 + b01) + choose2(b10 + b11);
                        fP = choose2(a00 + a01 + b00 + b01) + choose2(a10 + a11 + b10 + b11);
                        tA = choose2(a00) + choose2(a01) + choose2(a10) + choose2(a11);
                        tB = choose2(b00) + choose2(b01) + choose2(b10) + choose2(b11);
                        tP = choose2(a00 + b00) + choose2(a01 + b01) + choose2(a10 + b10) + choose2(a11 + b11);
                    }
                    const bool k00 = in && a00 + b00 >= 2u, k01 = in && a01 + b01 >= 2u;
                    const bool k10 = in && a10 + b10 >= 2u, k11 = in && a11 + b11 >= 2u;
                    uint32_t s3 = (k00 ? a00 + b00 : 0u) + (k01 ? a01 + b01 : 0u) +
                                  (k10 ? a10 + b10 : 0u) + (k11 ? a11 + b11 : 0u);
                    const uint64_t m00 = __ballot(k00), m01 = __ballot(k01);
                    const uint64_t m10 = __ballot(k10), m11 = __ballot(k11);
                    const int n00 = __popcll(m00), n01 = __popcll(m01);
                    const int n10 = __popcll(m10), n11 = __popcll(m11);
                    const int nk = n00 + n01 + n10 + n11;
                    int basei = 0;
                    if (wpg == 1) {
                        basei = kn[0];
                    } else {
                        if (lane == 0 && nk > 0) basei = atomicAdd(kn, nk);
                        basei = __shfl(basei, 0, 64);
                    }
                    const int i00 = basei + (int)lanes_below(m00);
                    const int i01 = basei + n00 + (int)lanes_below(m01);
                    const int i10 = basei + n00 + n01 + (int)lanes_below(m10);
                    const int i11 = basei + n00 + n01 + n10 + (int)lanes_below(m11);
                    const bool fits = basei + nk <= kmax;   // wave-uniform
                    if (!fits && lane == 0) *ovf = 1;
                    if (in) {
                        cmap[4 * c + 0] = (int16_t)(k00 ? i00 : DEAD);
                        cmap[4 * c + 1] = (int16_t)(k01 ? i01 : DEAD);
                        cmap[4 * c + 2] = (int16_t)(k10 ? i10 : DEAD);
                        cmap[4 * c + 3] = (int16_t)(k11 ? i11 : DEAD);
                    }
                    if (fits) {
                        if (k00) szn[i00] = a00 | (b00 << 16);
                        if (k01) szn[i01] = a01 | (b01 << 16);
                        if (k10) szn[i10] = a10 | (b10 << 16);
                        if (k11) szn[i11] = a11 | (b11 << 16);
                    }
                    tA = wave_sum(tA);
                    tB = wave_sum(tB);
                    tP = wave_sum(tP);
                    fA = wave_sum(fA);
                    fB = wave_sum(fB);
                    fP = wave_sum(fP);
                    if (can_pair) s3 = wave_sum(s3);
                    if (lane == 0) {
                        if (wpg == 1) {
                            kn[0] = basei + nk;
                            sa[0] += tA;
                            sa[1] += tB;
                            sa[2] += tP;
                            sa[3] += s3;
                            sa[4] += fA;
                            sa[5] += fB;
                            sa[6] += fP;
                        } else {
                            if (tA) atomicAdd(&sa[0], tA);
                            if (tB) atomicAdd(&sa[1], tB);
                            if (tP) atomicAdd(&sa[2], tP);
                            if (s3) atomicAdd(&sa[3], s3);
                            if (fA) atomicAdd(&sa[4], fA);
                            if (fB) atomicAdd(&sa[5], fB);
                            if (fP) atomicAdd(&sa[6], fP);
                        }
                    }
                    if (wpg == 1) __syncthreads();   // kn[0] is read again next round
                }
            } else {
                for (int c0 = 0; c0 < K; c0 += T) {
                    const int c = c0 + tid;
                    const bool in = c < K;
                    uint32_t one = 0u, sz = 0u;
                    if (in) {
                        for (int q = 0; q < ncp; ++q) {
                            one += cnt1[c * ncp + q];
                            cnt1[c * ncp + q] = 0u;
                        }
                        sz = szc[c];
                    }
                    bool keepz = false, keepo = false;
                    uint32_t wz = 0u, wo = 0u;
                    uint32_t s0 = 0u, s1 = 0u, s2 = 0u, s3 = 0u;   // s3: members kept
                    if (in) {
                        if (MODE == MODE_CORE) {
                            const uint32_t core = sz >> 31;
                            const uint32_t n = sz & 0xFFFFu;
                            const uint32_t o = one, z = n - one;
                            const bool live = core ? act1 : act0;
                            const uint32_t sc = choose2(o) + choose2(z);
                            if (core) s1 = sc;
                            else s0 = sc;
                            keepz = live && z >= 2u;
                            keepo = live && o >= 2u;
                            s3 = (keepz ? z : 0u) + (keepo ? o : 0u);
                            wz = z | (core << 31);
                            wo = o | (core << 31);
                        } else {
                            const uint32_t nAc = sz & 0xFFFFu, nBc = sz >> 16;
                            const uint32_t oA = one & 0xFFFFu, oB = one >> 16;
                            const uint32_t zA = nAc - oA, zB = nBc - oB;
                            s0 = choose2(oA) + choose2(zA);
                            s1 = choose2(oB) + choose2(zB);
                            s2 = choose2(oA + oB) + choose2(zA + zB);
                            keepz = zA + zB >= 2u;
                            keepo = oA + oB >= 2u;
                            s3 = (keepz ? zA + zB : 0u) + (keepo ? oA + oB : 0u);
                            wz = zA | (zB << 16);
                            wo = oA | (oB << 16);
                        }
                    }
                    const uint64_t bz = __ballot(keepz);
                    const uint64_t bo = __ballot(keepo);
                    const int nz = __popcll(bz), no = __popcll(bo);
                    // one wave owns the counters outright; several share them
                    int basei = 0;
                    if (wpg == 1) {
                        basei = kn[0];
                    } else {
                        if (lane == 0 && nz + no > 0) basei = atomicAdd(kn, nz + no);
                        basei = __shfl(basei, 0, 64);
                    }
                    const int idz = basei + (int)lanes_below(bz);
                    const int ido = basei + nz + (int)lanes_below(bo);
                    const bool fits = basei + nz + no <= kmax;   // wave-uniform
                    if (!fits && lane == 0) *ovf = 1;
                    if (in) {
                        cmap[2 * c] = (int16_t)(keepz ? idz : DEAD);
                        cmap[2 * c + 1] = (int16_t)(keepo ? ido : DEAD);
                    }
                    if (fits && keepz) szn[idz] = wz;
                    if (fits && keepo) szn[ido] = wo;
                    s0 = wave_sum(s0);
                    s1 = wave_sum(s1);
                    if (MODE == MODE_POOLED) s2 = wave_sum(s2);
                    if (can_pair) s3 = wave_sum(s3);
                    if (lane == 0) {
                        if (wpg == 1) {
                            kn[0] = basei + nz + no;
                            sa[0] += s0;
                            sa[1] += s1;
                            if (MODE == MODE_POOLED) sa[2] += s2;
                            sa[3] += s3;
                        } else {
                            if (s0) atomicAdd(&sa[0], s0);
                            if (s1) atomicAdd(&sa[1], s1);
                            if (MODE == MODE_POOLED && s2) atomicAdd(&sa[2], s2);
                            if (s3) atomicAdd(&sa[3], s3);
                        }
                    }
                    if (wpg == 1) __syncthreads();   // kn[0] is read again next round
                }
            }
            __syncthreads();
            if (*ovf) goto overflowed;   // the walk is redone with full tables

            // (3) new class ids
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (cls[r] != DEAD) cls[r] = cmap[cls[r]];
            K = kn[0];
            const uint32_t S0 = sa[0], S1 = sa[1], S2 = sa[2], members = sa[3];
            const uint32_t F0 = sa[4], F1 = sa[5], F2 = sa[6];   // two markers: S after the first
            if (tid == 0) {
                uint32_t *other = sacc + 8 * (par ^ 1);
                for (int x = 0; x < 8; ++x) other[x] = 0u;
                knext[par ^ 1] = 0;
            }
            step += two ? 2 : 1;
            if (two) pflip ^= 1;   // the children's sizes are current after an even step

            if (MODE == MODE_CORE && two) {
                // the first marker's stop tests and terms, then the second's
                // for the cores still walking
                if (act0) {
                    steps0 += 1;
                    if (F0 <= thr0) {
                        act0 = false;
                    } else {
                        if (wave == 0) {
                            const double e = (double)F0 / P0;
                            ihh0 += 0.5 * (ep0 + e) * readlane_f64(gl, i);
                            ep0 = e;
                        }
                        steps0 += 1;
                        if (S0 <= thr0) {
                            act0 = false;
                        } else if (wave == 0) {
                            const double e = (double)S0 / P0;
                            ihh0 += 0.5 * (ep0 + e) * readlane_f64(gl, i + 1);
                            ep0 = e;
                        }
                    }
                }
                if (act1) {
                    steps1 += 1;
                    if (F1 <= thr1) {
                        act1 = false;
                    } else {
                        if (wave == 0) {
                            const double e = (double)F1 / P1;
                            ihh1 += 0.5 * (ep1 + e) * readlane_f64(gl, i);
                            ep1 = e;
                        }
                        steps1 += 1;
                        if (S1 <= thr1) {
                            act1 = false;
                        } else if (wave == 0) {
                            const double e = (double)S1 / P1;
                            ihh1 += 0.5 * (ep1 + e) * readlane_f64(gl, i + 1);
                            ep1 = e;
                        }
                    }
                }
                sa0 = S0;
                sa1 = S1;
            } else if (MODE == MODE_CORE) {
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
                sa0 = S0;
                sa1 = S1;
            } else if (two) {
                // pooled: the first marker's stop test and terms, then the
                // second's if the walk goes on
                steps0 += 1;
                if (F2 <= thr0) {
                    act0 = false;
                } else {
                    if (wave == 0) {
                        const double g = readlane_f64(gl, i);
                        const double eA = (double)F0 / P0;
                        const double eB = (double)F1 / P1;
                        ihh0 += 0.5 * (ep0 + eA) * g;
                        ihh1 += 0.5 * (ep1 + eB) * g;
                        ep0 = eA;
                        ep1 = eB;
                    }
                    steps0 += 1;
                    if (S2 <= thr0) {
                        act0 = false;
                    } else if (wave == 0) {
                        const double g = readlane_f64(gl, i + 1);
                        const double eA = (double)S0 / P0;
                        const double eB = (double)S1 / P1;
                        ihh0 += 0.5 * (ep0 + eA) * g;
                        ihh1 += 0.5 * (ep1 + eB) * g;
                        ep0 = eA;
                        ep1 = eB;
                    }
                }
                sa0 = S0;
                sa1 = S1;
                sa2 = S2;
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
                sa0 = S0;
                sa1 = S1;
                sa2 = S2;
            }
            // pairwise tail once few identical pairs are left
            if (can_pair && (act0 || act1)) {
                const uint32_t left = MODE == MODE_CORE ? (act0 ? S0 : 0u) + (act1 ? S1 : 0u) : S2;
                if (left <= (uint32_t)pcap && members <= (uint32_t)kcap) {
                    pmode = true;
                    goto pairs;
                }
            }
            i += two ? 2 : 1;
        }
    }
    goto done;

pairs : {
    // ---- build the list of identical pairs from the live classes ----------------
    // classes of a stopped core are still in the table; they are skipped
    __syncthreads();
    const int par = (step & 1) ^ pflip;
    uint32_t *szc = par ? szv1 : szv0;     // sizes of the current classes
    uint32_t *sbase = par ? szv0 : szv1;   // member offset of each class
    uint64_t *wtot = (uint64_t *)(base + Ly.wtot);
    uint16_t *mem = (uint16_t *)(base + Ly.mem);
    uint32_t *pr0 = (uint32_t *)(base + Ly.pairs0);
    auto csize = [&](int c, uint32_t &tag) -> uint32_t {
        const uint32_t sz = szc[c];
        if (MODE == MODE_CORE) {
            const uint32_t core = sz >> 31;
            tag = core;
            const bool live = core ? act1 : act0;
            return live ? (sz & 0xFFFFu) : 0u;
        }
        tag = 0u;
        return (sz & 0xFFFFu) + (sz >> 16);
    };
    const int KT = (K + T - 1) / T;
    uint64_t loc = 0;
    for (int q = 0; q < KT; ++q) {
        const int c = tid * KT + q;
        if (c < K) {
            uint32_t tg;
            const uint64_t n = csize(c, tg);
            if (n >= 2) loc += n | ((uint64_t)(n * (n - 1) / 2) << 32);
        }
    }
    uint64_t tot;
    uint64_t ex = block_excl_sum(loc, wtot, tot);
    for (int q = 0; q < KT; ++q) {
        const int c = tid * KT + q;
        if (c < K) {
            uint32_t tg;
            const uint64_t n = csize(c, tg);
            const uint32_t mo = (uint32_t)ex, po = (uint32_t)(ex >> 32);
            sbase[c] = mo;
            cnt1[c * ncp] = mo;        // scatter cursor
            map[c] = (int32_t)po;      // pair offset
            if (n >= 2) ex += n | ((uint64_t)(n * (n - 1) / 2) << 32);
        }
    }
    const int L = (int)(uint32_t)tot;
    const int npairs0 = (int)(tot >> 32);
    __syncthreads();
    // members into their class's range of the member list
    int32_t mypos[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        mypos[r] = -1;
        if (cls[r] != DEAD) {
            uint32_t tg;
            if (csize(cls[r], tg) >= 2u) {
                const int wq = wave + r * wpg;
                const int h = wq < WA ? wq * 64 + lane : (0x8000 | ((wq - WA) * 64 + lane));
                const int p = (int)atomicAdd(&cnt1[cls[r] * ncp], 1u);
                mem[p] = (uint16_t)h;
                mypos[r] = p;
            }
        }
    }
    __syncthreads();
    // member at rank p of its class writes its p pairs with the earlier members
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (mypos[r] >= 0) {
            const int c = cls[r];
            uint32_t tg;
            (void)csize(c, tg);
            const int s = (int)sbase[c];
            const int p = mypos[r] - s;
            const uint32_t y = (uint32_t)mypos[r];
            uint32_t out = (uint32_t)map[c] + (uint32_t)(p * (p - 1) / 2);
            const uint32_t ty = MODE == MODE_CORE ? (tg << 15) : (uint32_t)(mem[y] & 0x8000u);
            for (int x = s; x < s + p; ++x) {
                const uint32_t tx = MODE == MODE_CORE ? (tg << 15) : (uint32_t)(mem[x] & 0x8000u);
                pr0[out++] = (uint32_t)x | tx | ((y | ty) << 16);
            }
        }
    }

    // ---- one pass over the pair list per 64 markers ----------------------------
    int npairs = npairs0;
    int pb = 0;
    uint64_t *keys = (uint64_t *)(base + Ly.keys);
    uint32_t *hist = (uint32_t *)(base + Ly.hist);
    uint32_t *pcnt = (uint32_t *)(base + Ly.pcnt);
    uint32_t *pr1 = (uint32_t *)(base + Ly.pairs1);
    while (act0 || act1) {
        uint32_t *pin = pb ? pr1 : pr0;
        uint32_t *pout = pb ? pr0 : pr1;
        __syncthreads();   // pair list complete; the last pass's counts read
        const int64_t k0 = j + (int64_t)dir * (int64_t)(step + 1);
        for (int x = tid; x < L; x += T) {
            const int h = mem[x];
            keys[x] = (h & 0x8000) ? key_of(G.hbitsB, G.mwp, h & 0x7FFF, k0, dir)
                                   : key_of(G.hbitsA, G.mwp, h, k0, dir);
        }
        for (int x = tid; x < 3 * 64; x += T) hist[x] = 0u;
        if (tid == 0) *pcnt = 0u;
        const int64_t kb = k0 + (int64_t)dir * (int64_t)lane;
        const bool inr = kb >= 0 && kb < G.M;
        const double sv = inr ? G.seg[dir > 0 ? kb : kb + 1] : 0.0;
        const int32_t stl = !inr ? ST_EDGE : (sv < 0.0 ? ST_GAP : ST_OK);
        const double gl = stl == ST_OK ? sv : 0.0;
        const uint64_t abort_mask = __ballot(stl != ST_OK);
        const int nb = abort_mask ? (int)__builtin_ctzll(abort_mask) : 64;
        const int32_t abort_st = abort_mask ? (int32_t)__builtin_amdgcn_readlane(stl, nb) : ST_OK;
        __syncthreads();
        for (int p0 = (tid & ~63); p0 < npairs; p0 += T) {
            const int p = p0 + lane;
            const bool in = p < npairs;
            const uint32_t pr = in ? pin[p] : 0u;
            const uint64_t x = keys[pr & 0x7FFFu] ^ keys[(pr >> 16) & 0x7FFFu];
            const int Lx = x ? (int)__builtin_ctzll(x) : 64;
            if (in && Lx < 64) {
                if (MODE == MODE_CORE) {
                    atomicAdd(&hist[((pr >> 15) & 1u) * 64 + Lx], 1u);
                } else {
                    atomicAdd(&hist[Lx], 1u);
                    const uint32_t tb = ((pr >> 15) & 1u) + ((pr >> 31) & 1u);
                    if (tb == 0u) atomicAdd(&hist[64 + Lx], 1u);
                    else if (tb == 2u) atomicAdd(&hist[128 + Lx], 1u);
                }
            }
            const bool surv = in && Lx == 64;
            const uint64_t sm = __ballot(surv);
            uint32_t wo = 0u;
            if (lane == 0 && sm) wo = atomicAdd(pcnt, (uint32_t)__popcll(sm));
            wo = (uint32_t)__shfl((int)wo, 0, 64);
            if (surv) pout[wo + __popcll(sm & low_bits(lane))] = pr;
        }
        __syncthreads();
        settle(hist, nb, gl);
        if ((act0 || act1) && nb < 64) {
            status = abort_st;
            break;
        }
        step += 64;
        npairs = (int)*pcnt;
        pb ^= 1;
    }
}
done:
    (void)pmode;
    if (tid == 0) {
        const size_t o = (size_t)j * 2 + d;
        put_rec(G.rec + o * 2 + 0, ihh0, status, steps0);
        put_rec(G.rec + o * 2 + 1, ihh1, status, MODE == MODE_CORE ? steps1 : 0);
    }
    return;
overflowed:
    if (tid == 0) redo[atomicAdd(redo_count, 1)] = item;
}

// Persistent grid over the batch's items (region, site, direction), taken a
// chunk at a time from the partitioned work queue.  With stride > 1 the items walked are a sample for the autotuner: blocks of
// 256 consecutive items, one block in every `stride`.  With a list, the items
// are those listed (count on the device): the walks a launch with a capped
// class table could not finish.
template <int R>
__global__ void __launch_bounds__(1024) ids_batch_kernel(IdsArgs a) {
    extern __shared__ uint64_t lds_ids[];
    __shared__ int64_t rng[2];   // the chunk being walked
    char *base = (char *)lds_ids;
    const BLay Ly = batch_layout(a.lmax, a.kcls, a.pcap, a.kcap, a.copies, a.dev != 0);
    const int64_t total = a.list ? (int64_t)*a.list_count : a.total;
    // the region of the last item (items of one region are consecutive)
    int g_idx = 0;
    int64_t g_lo = 0, g_hi = -1;
    WorkQueue q;   // thread 0's
    if (threadIdx.x == 0) {
        q.init(a.counter, total, a.chunk);
        int64_t lo, hi;
        q.resolve(lo, hi);
        rng[0] = lo;
        rng[1] = hi;
    }
    __syncthreads();
    for (;;) {
        const int64_t b0 = uniform64(rng[0]), b1 = uniform64(rng[1]);
        if (b0 >= b1) break;
        __syncthreads();   // everyone has read the chunk before it is replaced
        if (threadIdx.x == 0) q.prefetch();
        for (int64_t iv = b0; iv < b1; ++iv) {
            // the item, and with it the region and everything read through
            // it, is the same in every lane
            const int64_t it = uniform64(
                a.list ? a.list[iv]
                       : (a.stride > 1 ? (((iv >> 8) * a.stride) << 8) + (iv & 255) : iv));
            if (it < g_lo || it >= g_hi) {
                int lo = 0, hi = a.nreg - 1;   // last region with item0 <= it
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (a.regs[mid].item0 <= it) lo = mid;
                    else hi = mid - 1;
                }
                g_idx = __builtin_amdgcn_readfirstlane(lo);
                g_lo = uniform64(a.regs[g_idx].item0);
                g_hi = g_idx + 1 < a.nreg ? uniform64(a.regs[g_idx + 1].item0) : INT64_MAX;
            }
            const Region *G = a.regs + g_idx;
            const int64_t loc = it - g_lo;
            const int64_t j = loc >> 1;
            const int d = (int)(loc & 1);
            if (j >= G->M) continue;
            if (G->walk_flag && !G->walk_flag[j]) continue;
            if (G->mode == MODE_CORE)
                ids_walk<MODE_CORE, R>(G, j, d, base, Ly, a.pcap, a.kcap, a.dev != 0, it, a.redo,
                                       a.redo_count);
            else
                ids_walk<MODE_POOLED, R>(G, j, d, base, Ly, a.pcap, a.kcap, false, it, a.redo,
                                         a.redo_count);
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            int64_t lo, hi;
            q.resolve(lo, hi);
            rng[0] = lo;
            rng[1] = hi;
        }
        __syncthreads();   // the next chunk is visible
    }
}

template <int R>
hipError_t launch_r(const IdsArgs &a, const WideCfg &c, hipStream_t s) {
    hipLaunchKernelGGL((ids_batch_kernel<R>), dim3((unsigned)c.blocks), dim3((unsigned)c.threads),
                       c.lds, s, a);
    return hipGetLastError();
}

template <int R>
int occupancy_r(int threads, size_t lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, ids_batch_kernel<R>, threads, lds) !=
        hipSuccess)
        return 0;
    return nb;
}

}  // namespace

int ids_slots(int threads, int wmax) {
    const int waves = threads / 64;
    const int need = (wmax + waves - 1) / waves;
    int r = 1;
    while (r < need) r *= 2;
    return r <= 16 ? r : 0;   // 32 slots would spill registers
}

int ids_threads_for(int wmax, int slots) {
    if (slots < 1 || slots > 16) return 0;
    int t = 64 * ((wmax + slots - 1) / slots);
    if (t > 1024) t = 64 * ((wmax + 15) / 16);   // as many waves as fit, 16 slots each
    return t <= 1024 ? (t > 0 ? t : 64) : 0;
}

size_t ids_lds_bytes(int threads, int lmax, int wmax, int class_cap, int pair_cap, int key_cap,
                     int copies, bool dev) {
    if (threads < 64 || threads > 1024 || threads % 64) return 0;
    if (lmax < 2 || lmax > 32767 || ids_slots(threads, wmax) == 0) return 0;
    if (class_cap < 0 || pair_cap < 0 || key_cap < 0 || key_cap > 32767) return 0;
    if (copies != 1 && copies != 8) return 0;
    return batch_layout(lmax, class_cap, pair_cap, key_cap, copies, dev).total;
}

bool ids_table_capped(int lmax, int class_cap) {
    return class_cap > 0 && class_cap < lmax / 2 + 2;
}

int ids_blocks_per_cu(const WideCfg &c) {
    switch (ids_slots(c.threads, c.wmax)) {
        case 1: return occupancy_r<1>(c.threads, c.lds);
        case 2: return occupancy_r<2>(c.threads, c.lds);
        case 4: return occupancy_r<4>(c.threads, c.lds);
        case 8: return occupancy_r<8>(c.threads, c.lds);
        case 16: return occupancy_r<16>(c.threads, c.lds);
        default: return 0;
    }
}

hipError_t launch_ids_batch(const IdsArgs &a, const WideCfg &c, hipStream_t s) {
    if (a.nreg <= 0 || (!a.list && a.total <= 0)) return hipSuccess;
    if (c.blocks <= 0 || c.chunk <= 0) return hipErrorInvalidValue;
    switch (ids_slots(c.threads, c.wmax)) {
        case 1: return launch_r<1>(a, c, s);
        case 2: return launch_r<2>(a, c, s);
        case 4: return launch_r<4>(a, c, s);
        case 8: return launch_r<8>(a, c, s);
        case 16: return launch_r<16>(a, c, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ss

// EHH walks of a whole batch of regions in one persistent launch, for any
// haplotype count up to 16,384 in the walk (iHS: the core's carriers; XPEHH:
// both populations pooled).
//
// What it computes is the partition refinement of ss_walk.hip (Sec. 1.1,
// Eqs. 1-3; Sec. 1.2, Eq. 4 and the rules below it; Sec. 1.3, Eq. 7 for the
// pooled XPEHH walk), walk by walk, with the same FP64 arithmetic in the same
// order.  The work items of a batch are (region, site, direction, core) for
// iHS regions and (region, site, direction) for XPEHH regions; a grid sized to
// fill the GPU takes them from the partitioned work queue (WorkQueue), so
// walks of very uneven length and regions of different haplotype counts share
// one launch.
//
// One workgroup walks one item:
//   * the walk's haplotypes are a list in LDS in which every class is a
//     contiguous run (class starts marked in a bitmask).  Per marker each
//     thread takes a contiguous chunk of the list, reads its members' alleles
//     from the staged marker row, and one workgroup scan of four packed
//     16-bit counts (allele-0 members of A, of B, members of A, members of
//     classes that have shrunk to one) gives every member its place in the
//     next list: allele-0 children first, then allele-1 children, in the
//     order of the parent classes, with one-member classes left out.  No
//     atomics on class counters, and the work per marker shrinks with the
//     list;
//   * S = sum over the classes of C(n_h, 2) is exact (one 32-bit partial per
//     class head, wave sums, one LDS add per wave);
//   * once S (the number of identical pairs; for XPEHH the pooled count) is
//     at most the pair capacity, the classes are expanded into the list of
//     those pairs and each pass covers 64 markers: the XOR of a pair's 64-bit
//     keys (read from the haplotype-major copy of the matrix), its lowest set
//     bit = the marker where the pair splits, a 64-bin histogram per pair type
//     (pooled, A-A, B-B) gives S at each of the 64 markers;
//   * marker rows are staged in LDS a batch at a time, the next batch's loads
//     in flight while the current batch is refined.
#include "ss_internal.hpp"

namespace ss {

namespace {

constexpr int kBig = 1 << 30;
constexpr int kMaxRB = 16;     // markers staged per batch
constexpr int kPfWords = 4;    // words of the next batch each thread holds in flight

__device__ __forceinline__ uint32_t choose2(uint32_t x) { return (x * (x - 1u)) >> 1; }

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) { return __ockl_wfred_add_u32(v); }

// A value every lane holds alike, marked wave-uniform for the compiler.
__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int i) {
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)v, i);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(v >> 32), i);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ double readlane_f64(double v, int i) {
    return __builtin_bit_cast(double, readlane64(__builtin_bit_cast(uint64_t, v), i));
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

// Packed per-position counts: allele-0 members of A | of B << 16 | members of
// A << 32 | one-member classes << 48.
__device__ __forceinline__ uint64_t pack4(uint64_t zA, uint64_t zB, uint64_t a, uint64_t dd) {
    return (uint64_t)__popcll(zA) | ((uint64_t)__popcll(zB) << 16) |
           ((uint64_t)__popcll(a) << 32) | ((uint64_t)__popcll(dd) << 48);
}

// LDS layout (byte offsets).  The second list buffer and the staged rows are
// needed only before the pairwise phase, the pair lists and keys only during
// it, so they share one area.
struct Lay {
    uint32_t ent0, hm0, hm1, tab, wtot, sacc, ent1, rows, pairs0, pairs1, keys, hist, pcnt, total;
    int hmw;
};

__host__ __device__ inline uint32_t al16(uint32_t x) { return (x + 15u) & ~15u; }

__host__ __device__ inline Lay wide_layout(int T, int lmax, int wmax, int pcap, int kcap) {
    Lay l;
    uint32_t o = 0;
    l.hmw = (lmax + 31) / 32 + 4;   // class-start bits, padded for 96-bit windows
    l.ent0 = o; o = al16(o + 2u * (uint32_t)lmax);
    l.hm0 = o;  o = al16(o + 4u * (uint32_t)l.hmw);
    l.hm1 = o;  o = al16(o + 4u * (uint32_t)l.hmw);
    l.tab = o;  o = al16(o + 40u * (uint32_t)T);   // per thread: wave-exclusive prefix + 4 masks
    l.wtot = o; o = al16(o + 16u * 8u);            // per wave: sum, max, min
    l.sacc = o; o = al16(o + 32u);                 // S sums, two parities
    uint32_t a = o;
    l.ent1 = a; a = al16(a + 2u * (uint32_t)lmax);
    const int rw = kMaxRB * wmax < kPfWords * T ? kMaxRB * wmax : kPfWords * T;
    l.rows = a; a = al16(a + 8u * (uint32_t)rw);
    uint32_t b = o;
    l.pairs0 = b; b = al16(b + 4u * (uint32_t)pcap);
    l.pairs1 = b; b = al16(b + 4u * (uint32_t)pcap);
    l.keys = b;   b = al16(b + 8u * (uint32_t)kcap);
    l.hist = b;   b = al16(b + 4u * 3u * 64u);
    l.pcnt = b;   b = al16(b + 16u);
    l.total = a > b ? a : b;
    return l;
}

// 64 bits of the class-start bitmask from bit e0 on.
__device__ __forceinline__ uint64_t bits_at(const uint32_t *hm, int e0) {
    const int w0 = e0 >> 5, sh = e0 & 31;
    const uint64_t lo = (uint64_t)hm[w0] | ((uint64_t)hm[w0 + 1] << 32);
    const uint64_t hi = hm[w0 + 2];
    return sh ? ((lo >> sh) | (hi << (64 - sh))) : lo;
}

// Alleles of haplotype h at the 64 markers from k0 onwards in the walk's
// direction (bit i = marker k0 + dir * i), from the haplotype-major copy
// ([n][mwp] words, one zero word of padding at each end).
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

// Workgroup scan: exclusive sum of v, exclusive max of hmx over lower
// threads, exclusive min of hmn over higher threads.  pub[tid] receives the
// sum's prefix within the wave before the barrier, so that other threads can
// rebuild any thread's prefix afterwards (adding the totals of lower waves).
// Callers separate two uses of the wave totals by a barrier.
template <int T>
__device__ __forceinline__ void block_scan(uint64_t v, int32_t hmx, int32_t hmn, uint64_t *pub,
                                           uint64_t *wsum, int32_t *wmx, int32_t *wmn,
                                           uint64_t &excl, uint64_t &tot, int32_t &exmax,
                                           int32_t &exmin) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t inc = v;
    int32_t mx = hmx, mn = hmn;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t a = __shfl_up(inc, off, 64);
        const int32_t b = __shfl_up(mx, off, 64);
        const int32_t c = __shfl_down(mn, off, 64);
        if (lane >= off) {
            inc += a;
            mx = mx > b ? mx : b;
        }
        if (lane + off < 64) mn = mn < c ? mn : c;
    }
    const uint64_t wex = inc - v;
    int32_t pmx = __shfl_up(mx, 1, 64);
    int32_t pmn = __shfl_down(mn, 1, 64);
    if (lane == 0) pmx = -1;
    if (lane == 63) pmn = kBig;
    if (pub) pub[threadIdx.x] = wex;
    if (lane == 63) {
        wsum[wave] = inc;
        wmx[wave] = mx;
    }
    if (lane == 0) wmn[wave] = mn;
    __syncthreads();
    uint64_t off = 0, all = 0;
    int32_t cm = -1, cn = kBig;
#pragma unroll
    for (int w = 0; w < T / 64; ++w) {
        const uint64_t s = wsum[w];
        all += s;
        if (w < wave) {
            off += s;
            cm = cm > wmx[w] ? cm : wmx[w];
        }
        if (w > wave) cn = cn < wmn[w] ? cn : wmn[w];
    }
    excl = off + wex;
    tot = all;
    exmax = cm > pmx ? cm : pmx;
    exmin = cn < pmn ? cn : pmn;
}

template <int T>
__device__ void wide_walk_one(const Region &R, int64_t j, int d, int core, char *base,
                              const Lay &Ly, int pcap, int kcap) {
    const int tid = threadIdx.x, lane = tid & 63;
    const int dir = d == 0 ? 1 : -1;
    const bool pooled = R.mode == MODE_POOLED;
    const int nA = R.nA, nB = pooled ? R.nB : 0;
    const int WA = (nA + 63) >> 6, WB = pooled ? (nB + 63) >> 6 : 0;
    const int wtot = WA + WB;

    uint16_t *ent[2] = {(uint16_t *)(base + Ly.ent0), (uint16_t *)(base + Ly.ent1)};
    uint32_t *hm[2] = {(uint32_t *)(base + Ly.hm0), (uint32_t *)(base + Ly.hm1)};
    uint64_t *tpre = (uint64_t *)(base + Ly.tab);
    uint64_t *tzA = tpre + T, *tzB = tpre + 2 * T, *tA = tpre + 3 * T, *tD = tpre + 4 * T;
    uint64_t *wsum = (uint64_t *)(base + Ly.wtot);
    int32_t *wmx = (int32_t *)(wsum + 8);
    int32_t *wmn = wmx + 8;
    uint32_t *sacc = (uint32_t *)(base + Ly.sacc);
    uint64_t *rows = (uint64_t *)(base + Ly.rows);

    auto rowword = [&](int w, int64_t k) -> uint64_t {
        return w < WA ? R.bitsA[k * R.wpsA + w] : R.bitsB[k * R.wpsB + (w - WA)];
    };
    auto validmask = [&](int w) -> uint64_t {
        const int nv = w < WA ? nA - 64 * w : nB - 64 * (w - WA);
        return low_bits(nv);
    };

    // ---- the list at x0 ---------------------------------------------------------
    // iHS: the carriers of the core allele.  XPEHH: allele-0 carriers of A and
    // B, then allele-1 carriers of A and B (pooled index: B's haplotype h is
    // nA + h).  Virtual word v selects one side of one row word.
    const int nv = pooled ? 2 * wtot : WA;
    const int K = (nv + T - 1) / T;
    auto vmask = [&](int v, int &w, int &sel) -> uint64_t {
        w = pooled ? (v < wtot ? v : v - wtot) : v;
        sel = pooled ? (v < wtot ? 0 : 1) : core;
        const uint64_t r = rowword(w, j);
        return (sel ? r : ~r) & validmask(w);
    };
    uint64_t cnt4 = 0;
    for (int q = 0; q < K; ++q) {
        const int v = tid * K + q;
        if (v < nv) {
            int w, sel;
            const uint64_t m = vmask(v, w, sel);
            const uint64_t c = (uint64_t)__popcll(m);
            cnt4 += c << (16 * ((sel ? 2 : 0) + (w < WA ? 0 : 1)));
        }
    }
    // hm words are cleared here: class starts at 0 and, for XPEHH, at the
    // first allele-1 member (set after the scan)
    for (int w = tid; w < Ly.hmw; w += T) {
        hm[0][w] = 0u;
        hm[1][w] = 0u;
    }
    if (tid < 8) sacc[tid] = 0u;
    uint64_t excl, tot;
    int32_t exmax, exmin;
    block_scan<T>(cnt4, -1, kBig, nullptr, wsum, wmx, wmn, excl, tot, exmax, exmin);
    {
        int off = (int)((excl & 0xFFFF) + ((excl >> 16) & 0xFFFF) + ((excl >> 32) & 0xFFFF) +
                        ((excl >> 48) & 0xFFFF));
        for (int q = 0; q < K; ++q) {
            const int v = tid * K + q;
            if (v < nv) {
                int w, sel;
                uint64_t m = vmask(v, w, sel);
                const int hb = w < WA ? 64 * w : nA + 64 * (w - WA);
                while (m) {
                    ent[0][off++] = (uint16_t)(hb + __builtin_ctzll(m));
                    m &= m - 1ull;
                }
            }
        }
    }
    const uint32_t n0a = (uint32_t)(tot & 0xFFFF), n0b = (uint32_t)((tot >> 16) & 0xFFFF);
    const uint32_t n1a = (uint32_t)((tot >> 32) & 0xFFFF), n1b = (uint32_t)((tot >> 48) & 0xFFFF);
    int L;
    bool act;
    double PA, PB = 1.0, PP = 1.0, epA, epB = 0.0;
    uint32_t sP, sA = 0, sB = 0;   // S after the last marker (iHS: sP only)
    if (!pooled) {
        const uint32_t nc = core ? n1a : n0a;
        L = (int)nc;
        act = nc >= 2u;
        PA = (double)choose2(nc);
        epA = 1.0;
        sP = choose2(nc);
    } else {
        L = nA + nB;
        PA = (double)choose2((uint32_t)nA);
        PB = (double)choose2((uint32_t)nB);
        PP = (double)choose2((uint32_t)L);
        // x0 is part of the haplotype: each population's curve starts at its
        // whole-sample EHH at x0
        epA = (double)(choose2(n0a) + choose2(n1a)) / PA;
        epB = (double)(choose2(n0b) + choose2(n1b)) / PB;
        act = true;
        sA = choose2(n0a) + choose2(n1a);
        sB = choose2(n0b) + choose2(n1b);
        sP = choose2(n0a + n0b) + choose2(n1a + n1b);
    }
    __syncthreads();   // the clears of hm are done
    if (tid == 0 && L > 0) {
        hm[0][0] = 1u;
        const int z = (int)(n0a + n0b);
        if (pooled && z > 0 && z < L) hm[0][z >> 5] |= 1u << (z & 31);
    }

    double ihhA = 0.0, ihhB = 0.0;
    int32_t steps = 0;
    int32_t status = ST_OK;
    int step = 0;
    int cur = 0;
    const bool can_pair = R.hbitsA != nullptr && (!pooled || R.hbitsB != nullptr);
    bool pmode = false;
    int npairs = 0;

    // ---- staging of marker rows -------------------------------------------------
    int RB = (kPfWords * T) / (wtot > 0 ? wtot : 1);
    if (RB > kMaxRB) RB = kMaxRB;
    if (RB < 1) RB = 1;
    const int rbw = RB * wtot;
    uint64_t pf[kPfWords];
    auto load_batch = [&](int st) {
#pragma unroll
        for (int q = 0; q < kPfWords; ++q) {
            const int idx = tid + q * T;
            uint64_t x = 0ull;
            if (idx < rbw) {
                const int i = idx / wtot;
                const int w = idx - i * wtot;
                const int64_t k = j + (int64_t)dir * (int64_t)(st + 1 + i);
                if (k >= 0 && k < R.M) x = rowword(w, k);
            }
            pf[q] = x;
        }
    };
    if (act) load_batch(0);

    // ---- phase 1: one marker at a time -----------------------------------------
    while (act) {
        const int ri = step % RB;
        if (ri == 0) {
#pragma unroll
            for (int q = 0; q < kPfWords; ++q) {
                const int idx = tid + q * T;
                if (idx < rbw) rows[idx] = pf[q];
            }
            load_batch(step + RB);   // next batch in flight
        }
        // segment to the next marker: end of data, abort gap or scaled length
        const int64_t k = j + (int64_t)dir * (int64_t)(step + 1);
        if (k < 0 || k >= R.M) {
            status = ST_EDGE;
            break;
        }
        const double g = R.seg[dir > 0 ? k : k + 1];
        if (g < 0.0) {
            status = ST_GAP;
            break;
        }
        __syncthreads();   // staged rows and the previous marker's list are complete

        // (1) alleles of my chunk of the list
        const int E = (L + T - 1) / T;
        const int e0 = tid * E;
        const int ne = L - e0 < E ? (L - e0 > 0 ? L - e0 : 0) : E;
        const uint16_t *ec = ent[cur];
        const uint64_t *rw = rows + ri * wtot;
        uint64_t mzA = 0, mzB = 0, mA = 0, mH = 0, mD = 0;
        for (int q = 0; q < ne; ++q) {
            const int p = ec[e0 + q];
            const bool isA = p < nA;
            const int hp = isA ? p : p - nA;
            const int w = isA ? (hp >> 6) : WA + (hp >> 6);
            const bool one = ((rw[w] >> (hp & 63)) & 1ull) != 0ull;
            const uint64_t b = 1ull << q;
            if (!one) {
                if (isA) mzA |= b;
                else mzB |= b;
            }
            if (isA) mA |= b;
        }
        if (ne > 0) {
            mH = bits_at(hm[cur], e0) & low_bits(ne);
            const int en = e0 + ne;
            const uint64_t nh = en < L ? ((hm[cur][en >> 5] >> (en & 31)) & 1u) : 1ull;
            const uint64_t mNH = (mH >> 1) | (nh << (ne - 1));
            mD = mH & mNH;   // classes of one member: dropped from the next list
        }
        const int32_t lastH = mH ? e0 + 63 - __builtin_clzll(mH) : -1;
        const int32_t firstH = mH ? e0 + __builtin_ctzll(mH) : kBig;
        uint32_t *hn = hm[cur ^ 1];
        for (int w = tid; w < Ly.hmw; w += T) hn[w] = 0u;
        tzA[tid] = mzA;
        tzB[tid] = mzB;
        tA[tid] = mA;
        tD[tid] = mD;
        block_scan<T>(pack4(mzA, mzB, mA, mD), lastH, firstH, tpre, wsum, wmx, wmn, excl, tot,
                      exmax, exmin);

        // (2) places in the next list; class heads add their children's C(., 2)
        const int Lnew = L - (int)(tot >> 48);
        auto Q = [&](int x) -> uint64_t {   // packed counts over list positions < x
            if (x >= L) return tot;
            const int o = x / E;
            const int qq = x - o * E;
            const uint64_t bm = low_bits(qq);
            uint64_t r = tpre[o];
            for (int w = 0; w < (o >> 6); ++w) r += wsum[w];
            return r + pack4(tzA[o] & bm, tzB[o] & bm, tA[o] & bm, tD[o] & bm);
        };
        uint16_t *en = ent[cur ^ 1];
        uint32_t s0 = 0, s1 = 0, s2 = 0;
        uint64_t run = excl;
        int cs = -1, zc = 0, bs = 0;
        uint32_t zs = 0;   // allele-0 members before the class start
        for (int q = 0; q < ne; ++q) {
            const int e = e0 + q;
            const uint64_t b = 1ull << q;
            const uint64_t inc = ((mzA & b) ? 1ull : 0ull) | ((mzB & b) ? (1ull << 16) : 0ull) |
                                 ((mA & b) ? (1ull << 32) : 0ull) | ((mD & b) ? (1ull << 48) : 0ull);
            if (!(mD & b)) {
                const uint64_t upto = b | (b - 1ull);
                const uint64_t hb = mH & upto;
                const int s = hb ? e0 + 63 - __builtin_clzll(hb) : exmax;
                if (s != cs) {
                    const uint64_t ha = mH & ~upto;
                    const int sn = ha ? e0 + __builtin_ctzll(ha) : (exmin < L ? exmin : L);
                    const uint64_t Qs = Q(s);
                    const uint64_t dq = Q(sn) - Qs;
                    const int zA = (int)(dq & 0xFFFF), zB = (int)((dq >> 16) & 0xFFFF);
                    const int nAc = (int)((dq >> 32) & 0xFFFF);
                    const int n = sn - s, nBc = n - nAc;
                    zc = zA + zB;
                    bs = s - (int)(Qs >> 48);
                    zs = (uint32_t)(Qs & 0xFFFF) + (uint32_t)((Qs >> 16) & 0xFFFF);
                    cs = s;
                    if (e == s) {
                        const int oc = n - zc;
                        atomicOr(&hn[bs >> 5], 1u << (bs & 31));
                        if (zc > 0 && oc > 0) {
                            const int h2 = bs + zc;
                            atomicOr(&hn[h2 >> 5], 1u << (h2 & 31));
                        }
                        if (!pooled) {
                            s0 += choose2((uint32_t)zc) + choose2((uint32_t)oc);
                        } else {
                            const uint32_t oA = (uint32_t)(nAc - zA), oB = (uint32_t)(nBc - zB);
                            s0 += choose2((uint32_t)zA) + choose2(oA);
                            s1 += choose2((uint32_t)zB) + choose2(oB);
                            s2 += choose2((uint32_t)zc) + choose2((uint32_t)oc);
                        }
                    }
                }
                const int zb = (int)((uint32_t)(run & 0xFFFF) + (uint32_t)((run >> 16) & 0xFFFF) - zs);
                const bool zero = ((mzA | mzB) & b) != 0ull;
                const int np = zero ? bs + zb : bs + zc + ((e - cs) - zb);
                en[np] = ec[e];
            }
            run += inc;
        }
        const int par = step & 1;
        uint32_t *sa = sacc + 4 * par;
        s0 = wave_sum(s0);
        if (pooled) {
            s1 = wave_sum(s1);
            s2 = wave_sum(s2);
        }
        if (lane == 0) {
            if (s0) atomicAdd(&sa[0], s0);
            if (s1) atomicAdd(&sa[1], s1);
            if (s2) atomicAdd(&sa[2], s2);
        }
        __syncthreads();
        const uint32_t S0 = sa[0], S1 = sa[1], S2 = sa[2];
        if (tid < 4) sacc[4 * (par ^ 1) + tid] = 0u;   // read only after the next barrier
        L = Lnew;
        cur ^= 1;
        step += 1;
        steps += 1;

        // (3) stop rule and trapezoid term, in the definition's order
        uint32_t Sst;
        if (!pooled) {
            const double e = (double)S0 / PA;
            if (e < R.cutoff) {
                act = false;
            } else {
                ihhA += 0.5 * (epA + e) * g;
                epA = e;
            }
            sP = S0;
            Sst = S0;
        } else {
            if ((double)S2 / PP < R.cutoff) {
                act = false;
            } else {
                const double eA = (double)S0 / PA;
                const double eB = (double)S1 / PB;
                ihhA += 0.5 * (epA + eA) * g;
                ihhB += 0.5 * (epB + eB) * g;
                epA = eA;
                epB = eB;
            }
            sA = S0;
            sB = S1;
            sP = S2;
            Sst = S2;
        }
        if (act && can_pair && Sst <= (uint32_t)pcap && L <= kcap) {
            pmode = true;
            break;
        }
    }

    // ---- phase 2: pairs, 64 markers per pass ------------------------------------
    if (pmode) {
        __syncthreads();   // the last marker's list is complete
        if (cur == 1) {
            for (int x = tid; x < L; x += T) ent[0][x] = ent[1][x];
        }
        // pairs (x, y), x < y in one class: member y of a class starting at s
        // has y - s partners before it
        const int E = (L + T - 1) / T;
        const int e0 = tid * E;
        const int ne = L - e0 < E ? (L - e0 > 0 ? L - e0 : 0) : E;
        const uint64_t mH = ne > 0 ? bits_at(hm[cur], e0) & low_bits(ne) : 0ull;
        const int32_t lastH = mH ? e0 + 63 - __builtin_clzll(mH) : -1;
        uint64_t excl, tot;
        int32_t exmax, exmin;
        block_scan<T>(0ull, lastH, kBig, nullptr, wsum, wmx, wmn, excl, tot, exmax, exmin);
        uint64_t npp = 0;
        for (int q = 0; q < ne; ++q) {
            const uint64_t hb = mH & low_bits(q + 1);
            const int s = hb ? e0 + 63 - __builtin_clzll(hb) : exmax;
            npp += (uint64_t)(e0 + q - s);
        }
        const int32_t exm = exmax;
        __syncthreads();   // wave totals are reused
        block_scan<T>(npp, -1, kBig, nullptr, wsum, wmx, wmn, excl, tot, exmax, exmin);
        uint32_t *pr0 = (uint32_t *)(base + Ly.pairs0);
        {
            uint32_t off = (uint32_t)excl;
            for (int q = 0; q < ne; ++q) {
                const int y = e0 + q;
                const uint64_t hb = mH & low_bits(q + 1);
                const int s = hb ? e0 + 63 - __builtin_clzll(hb) : exm;
                const uint32_t ty = (uint32_t)y | (ent[0][y] >= nA ? 0x8000u : 0u);
                for (int x = s; x < y; ++x)
                    pr0[off++] = (uint32_t)x | (ent[0][x] >= nA ? 0x8000u : 0u) | (ty << 16);
            }
        }
        npairs = (int)tot;
    }
    int pb = 0;
    while (pmode && act) {
        uint32_t *pin = (uint32_t *)(base + (pb ? Ly.pairs1 : Ly.pairs0));
        uint32_t *pout = (uint32_t *)(base + (pb ? Ly.pairs0 : Ly.pairs1));
        uint64_t *keys = (uint64_t *)(base + Ly.keys);
        uint32_t *hist = (uint32_t *)(base + Ly.hist);
        uint32_t *pcnt = (uint32_t *)(base + Ly.pcnt);
        __syncthreads();   // pair list written, previous pass's keys and counts read
        const int64_t k0 = j + (int64_t)dir * (int64_t)(step + 1);
        for (int x = tid; x < L; x += T) {
            const int h = ent[0][x];
            keys[x] = h < nA ? key_of(R.hbitsA, R.mwp, h, k0, dir)
                             : key_of(R.hbitsB, R.mwp, h - nA, k0, dir);
        }
        for (int x = tid; x < 3 * 64; x += T) hist[x] = 0u;
        if (tid == 0) *pcnt = 0u;
        // lane i: step i of the pass (the same in every wave)
        const int64_t kb = k0 + (int64_t)dir * (int64_t)lane;
        const bool inr = kb >= 0 && kb < R.M;
        const double sv = inr ? R.seg[dir > 0 ? kb : kb + 1] : 0.0;
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
            const int a = (int)(pr & 0x3FFFu), b = (int)((pr >> 16) & 0x3FFFu);
            const uint64_t x = keys[a] ^ keys[b];
            const int Lx = x ? (int)__builtin_ctzll(x) : 64;
            if (in && Lx < 64) {
                atomicAdd(&hist[Lx], 1u);
                if (pooled) {
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
        // S at each of the 64 markers; every wave evaluates the same values
        const uint32_t siP = sP - wave_prefix(hist[lane], lane);
        uint32_t siA = 0, siB = 0;
        if (pooled) {
            siA = sA - wave_prefix(hist[64 + lane], lane);
            siB = sB - wave_prefix(hist[128 + lane], lane);
        }
        const double Pst = pooled ? PP : PA;
        const uint64_t valid = low_bits(nb);
        const uint64_t stopm = __ballot((double)siP / Pst < R.cutoff) & valid;
        int i, nterm;
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
        step += i;
        if (nterm > 0) {
            if (!pooled) {
                const double e = (double)siP / PA;
                double prev = __shfl_up(e, 1, 64);
                if (lane == 0) prev = epA;
                const double term = 0.5 * (prev + e) * gl;
                for (int t = 0; t < nterm; ++t) ihhA += readlane_f64(term, t);
                epA = readlane_f64(e, nterm - 1);
            } else {
                const double eA = (double)siA / PA;
                const double eB = (double)siB / PB;
                double pA = __shfl_up(eA, 1, 64);
                double pBv = __shfl_up(eB, 1, 64);
                if (lane == 0) {
                    pA = epA;
                    pBv = epB;
                }
                const double tA = 0.5 * (pA + eA) * gl;
                const double tB = 0.5 * (pBv + eB) * gl;
                for (int t = 0; t < nterm; ++t) {
                    ihhA += readlane_f64(tA, t);
                    ihhB += readlane_f64(tB, t);
                }
                epA = readlane_f64(eA, nterm - 1);
                epB = readlane_f64(eB, nterm - 1);
            }
        }
        sP = (uint32_t)__builtin_amdgcn_readlane(siP, 63);
        if (pooled) {
            sA = (uint32_t)__builtin_amdgcn_readlane(siA, 63);
            sB = (uint32_t)__builtin_amdgcn_readlane(siB, 63);
        }
        npairs = (int)*pcnt;
        pb ^= 1;
        if (status != ST_OK) break;
    }

    if (tid == 0) {
        const size_t o = (size_t)j * 2 + d;
        if (!pooled) {
            put_rec(R.rec + o * 2 + core, ihhA, status, steps);
        } else {
            put_rec(R.rec + o * 2 + 0, ihhA, status, steps);
            put_rec(R.rec + o * 2 + 1, ihhB, status, 0);
        }
    }
}

// Persistent grid: every workgroup takes `chunk` consecutive items at a time
// from the partitioned work queue and leaves the loop once it has found every
// part of the queue used up.
template <int T>
__global__ void __launch_bounds__(T) wide_walk_kernel(const Region *__restrict__ regs, int32_t nreg,
                                                      int64_t total, int64_t stride,
                                                      unsigned long long *counter,
                                                      int chunk, int lmax, int wmax, int pcap,
                                                      int kcap) {
    extern __shared__ uint64_t lds_wide[];
    __shared__ int64_t rng[2];   // the chunk being walked
    char *base = (char *)lds_wide;
    const Lay Ly = wide_layout(T, lmax, wmax, pcap, kcap);
    WorkQueue q;   // thread 0's
    if (threadIdx.x == 0) {
        q.init(counter, total, chunk);
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
            // stride > 1: a sample, blocks of 256 items, one in every `stride`
            const int64_t it = stride > 1 ? (((iv >> 8) * stride) << 8) + (iv & 255) : iv;
            int lo = 0, hi = nreg - 1;   // last region with item0 <= it
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (regs[mid].item0 <= it) lo = mid;
                else hi = mid - 1;
            }
            // the same region in every lane: its fields are scalar loads
            const Region R = regs[__builtin_amdgcn_readfirstlane(lo)];
            const int64_t loc = it - R.item0;
            int64_t j;
            int d, core;
            if (R.mode == MODE_CORE) {
                j = loc >> 2;
                d = (int)((loc >> 1) & 1);
                core = (int)(loc & 1);
            } else {
                j = loc >> 1;
                d = (int)(loc & 1);
                core = 0;
            }
            if (j >= R.M) continue;
            if (R.walk_flag && !R.walk_flag[j]) continue;
            wide_walk_one<T>(R, j, d, core, base, Ly, pcap, kcap);
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

// Region descriptors are passed by value (a few per launch) so that the copy
// is an ordinary kernel node when the sequence is captured into a graph.
constexpr int kFillPer = 8;
struct RegionChunk {
    Region r[kFillPer];
};

__global__ void fill_regions_kernel(RegionChunk c, int n, Region *dst) {
    const int i = threadIdx.x;
    if (i < n) dst[i] = c.r[i];
}

__global__ void zero_u64_kernel(unsigned long long *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

template <int T>
hipError_t launch_t(const Region *regs, int32_t nreg, int64_t total, int64_t stride,
                    unsigned long long *counter, const WideCfg &c, hipStream_t s) {
    hipLaunchKernelGGL((wide_walk_kernel<T>), dim3((unsigned)c.blocks), dim3(T), c.lds, s, regs, nreg,
                       total, stride, counter, c.chunk, c.lmax, c.wmax, c.pair_cap, c.key_cap);
    return hipGetLastError();
}

template <int T>
int occupancy_t(size_t lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, wide_walk_kernel<T>, T, lds) != hipSuccess)
        return 0;
    return nb;
}

}  // namespace

size_t wide_lds_bytes(int threads, int lmax, int wmax, int pair_cap, int key_cap) {
    if (threads != 128 && threads != 256 && threads != 512) return 0;
    if (lmax < 1 || lmax > wide_max_list(threads)) return 0;
    if (pair_cap < 0 || key_cap < 0 || key_cap > 16384) return 0;
    return wide_layout(threads, lmax, wmax, pair_cap, key_cap).total;
}

int wide_blocks_per_cu(const WideCfg &c) {
    switch (c.threads) {
        case 128: return occupancy_t<128>(c.lds);
        case 256: return occupancy_t<256>(c.lds);
        case 512: return occupancy_t<512>(c.lds);
        default: return 0;
    }
}

hipError_t launch_fill_regions(const Region *host, int n, Region *dev, hipStream_t s) {
    for (int i = 0; i < n; i += kFillPer) {
        RegionChunk c{};
        const int m = n - i < kFillPer ? n - i : kFillPer;
        for (int q = 0; q < m; ++q) c.r[q] = host[i + q];
        hipLaunchKernelGGL(fill_regions_kernel, dim3(1), dim3(64), 0, s, c, m, dev + i);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t s) {
    hipLaunchKernelGGL(zero_u64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_wide_walk(const Region *regs, int32_t nreg, int64_t total_items,
                            int64_t stride, unsigned long long *counter, const WideCfg &c,
                            hipStream_t s) {
    if (nreg <= 0 || total_items <= 0) return hipSuccess;
    if (c.blocks <= 0 || c.chunk <= 0) return hipErrorInvalidValue;
    switch (c.threads) {
        case 128: return launch_t<128>(regs, nreg, total_items, stride, counter, c, s);
        case 256: return launch_t<256>(regs, nreg, total_items, stride, counter, c, s);
        case 512: return launch_t<512>(regs, nreg, total_items, stride, counter, c, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ss

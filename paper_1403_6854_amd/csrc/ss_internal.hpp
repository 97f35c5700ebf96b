// Internal declarations shared by the library's translation units.
// Not part of the public ABI (that is include/selscan_hip.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace ss {

// Per-site status codes (mirror SS_ST_* of the public header).
enum : int32_t {
    ST_OK = 0, ST_MAF = 1, ST_EDGE = 2, ST_GAP = 3, ST_UNDEF = 4, ST_BIN = 5, ST_CAP = 6
};

enum WalkMode : int { MODE_CORE = 0, MODE_POOLED = 1 };

// Result of one walk -- iHH, abort status and markers walked -- as one 16-byte
// record per (site, direction, slot), the slot being the core allele (iHS) or
// the population (XPEHH), written with one vector store: three separate
// arrays took three partial-line writes per walk.
struct WalkRec {
    double ihh;
    int32_t status;
    int32_t steps;
};
static_assert(sizeof(WalkRec) == 16, "one 16-byte store per walk");

__device__ __forceinline__ void put_rec(WalkRec *r, double ihh, int32_t status, int32_t steps) {
    const uint64_t b = __builtin_bit_cast(uint64_t, ihh);
    *(uint4 *)r = make_uint4((uint32_t)b, (uint32_t)(b >> 32), (uint32_t)status, (uint32_t)steps);
}

// Everything one launch of the EHH walk needs.  The pooled haplotype index
// space places population A in words [0, WA) and population B in words
// [WA, WA + WB), so that every 64-haplotype word belongs to one population.
struct WalkArgs {
    const uint64_t *bitsA;
    int64_t wpsA;
    int32_t nA, WA;
    const uint64_t *bitsB;
    int64_t wpsB;
    int32_t nB, WB;
    int64_t M;
    const int64_t *pos;
    const double *gpos;
    double cutoff;
    int64_t gap_scale;
    int64_t max_gap;
    int32_t physical;           // 1: segment length = physical distance in bp, else genetic
    const uint8_t *walk_flag;   // [M], nonzero = score this site; null = all sites
    const int32_t *sites;       // null: block x walks site site0 + blockIdx.x
    int64_t site0;
    int32_t kmax;               // class-table capacity in LDS
    WalkRec *rec;               // [M][2 dirs][2 slots] walk results (ss_ehh: [2 dirs][2])
    // ss_ehh trace outputs (one site only)
    uint64_t *trS;              // [2][cap+1][2]
    uint32_t *trSizes;          // [2][cap+1][n] or null
    int64_t *trLen;             // [2]
    int64_t cap;
    // haplotype-major copy of population A (pairwise phase of the iHS walk)
    const uint64_t *hbits;      // [nA][mwp], null: no pairwise phase
    int64_t mwp;
    // per-segment genetic lengths with the gap rules applied (segment k-1 -> k
    // at index k; -1 marks an abort gap); null: walks compute them
    const double *seg;
    // bitmask walk: batches with at most this many class slots test all their
    // markers at once and refine only those that cut a class
    int32_t skip_classes;
};


struct WalkShape {
    int threads;      // workgroup size, multiple of 64
    int slots;        // 64-haplotype words handled per wave and step
    size_t lds;       // dynamic LDS bytes
};

WalkShape walk_shape(int32_t nA, int32_t nB, int mode);

// Walk kernel variants: class ids in LDS (any haplotype count) or class
// bitmasks in registers (up to 512 haplotypes).
enum WalkKind : int { WALK_AUTO = 0, WALK_LDS_IDS = 1, WALK_REG_MASKS = 2, WALK_WIDE = 3 };

// Launch shape of the register-bitmask walk: mask words per class (padded to
// 1, 2, 4 or 8), lanes per class, rows of 64/lpc classes, LDS bytes.
struct MaskShape {
    bool ok;
    int words;
    int lpc;
    int rows;
    int pair_cap;   // pairs held in LDS by the pairwise phase (0: none)
    size_t lds;
};
MaskShape mask_walk_shape(int32_t nA, int32_t nB, int mode, int lpc);
bool mask_walk_supported(int32_t nA, int32_t nB, int mode);
hipError_t launch_mask_walk(const WalkArgs &a, int mode, int lpc, int64_t n_blocks, hipStream_t s);
hipError_t launch_walk(const WalkArgs &a, int mode, bool trace, int64_t n_blocks,
                       hipStream_t s);

// ---- batched walks over many regions (ss_walk_wide.hip) ----------------------
// One region of a batch: a haplotype matrix (iHS) or a pair of them (XPEHH),
// its precomputed segment lengths and haplotype-major copies, and where its
// per-(site, direction, core) walk results go.  The batch's work items are
// numbered region by region: an iHS region has 4 items per site (direction,
// core allele), an XPEHH region 2 (direction); region r owns items
// [item0, item0 + items).
struct Region {
    const uint64_t *bitsA;
    const uint64_t *bitsB;
    const uint64_t *hbitsA;     // [nA][mwp], null: no pairwise phase
    const uint64_t *hbitsB;     // [nB][mwp] (XPEHH)
    const double *seg;          // [M]
    const uint8_t *walk_flag;   // [M] or null (every site)
    WalkRec *rec;               // [M][2][2]
    int64_t wpsA, wpsB, M, mwp;
    int64_t item0;
    double cutoff;
    int32_t nA, nB, mode, pad;
};

// Items per site: the class-id batch walk takes both cores of a site in one
// item (2 per site, one per direction); the list walk walks each iHS core
// separately (4 per site).
inline int64_t region_items(int mode, int64_t M, int kernel) {
    return M * (kernel == 1 && mode == MODE_CORE ? 4 : 2);
}

// Launch configuration of the persistent wide walk.
struct WideCfg {
    int kernel;      // 0: class ids with a pairwise tail (ss_walk_batch.hip); 1: lists (ss_walk_wide.hip)
    int threads;     // workgroup size: 64 .. 1024 (kernel 0); 128, 256 or 512 (kernel 1)
    int pair_cap;    // pairs held by the pairwise phase
    int key_cap;     // haplotypes whose 64-marker keys the pairwise phase holds
    int chunk;       // items taken per grab of the work queue
    int blocks;      // workgroups of the persistent grid
    int lmax;        // largest haplotype list of the batch (iHS: n, XPEHH: nA + nB)
    int class_cap;   // kernel 0: class-table capacity (0 = full)
    int copies;      // kernel 0: copies of each class counter (1 or 8)
    int wmax;        // largest row width in words (iHS: W, XPEHH: WA + WB)
    size_t lds;      // dynamic LDS bytes
    int dev;         // kernel 0: room for the iHS walks' reference passes
};

// LDS bytes of the wide walk for a configuration (0 if it cannot run).
size_t wide_lds_bytes(int threads, int lmax, int wmax, int pair_cap, int key_cap);
// Workgroups per CU the wide walk reaches with this configuration.
int wide_blocks_per_cu(const WideCfg &c);
// Largest haplotype list a workgroup of this size can walk.
inline int wide_max_list(int threads) { return 64 * threads < 16384 ? 64 * threads : 16384; }
// Class-id batch walk: slots per thread (0 if the row is too wide), LDS
// bytes (0 if invalid), workgroups per CU, launch.
int ids_slots(int threads, int wmax);
// Smallest workgroup size (64 .. 1024) whose waves hold a row of wmax words
// with at most `slots` words per wave (16 per wave when that would need more
// than 1024 threads); 0 if the row does not fit.
int ids_threads_for(int wmax, int slots);
// dev: the launch holds iHS walks, which take reference passes (their
// arrays share the pairwise tail's space and take more when it is smaller).
size_t ids_lds_bytes(int threads, int lmax, int wmax, int class_cap, int pair_cap, int key_cap,
                     int copies, bool dev);
// True when a class capacity leaves some walks of lmax haplotypes to a
// second launch with full tables.
bool ids_table_capped(int lmax, int class_cap);
int ids_blocks_per_cu(const WideCfg &c);

// Work distribution of the persistent walks.  The items [0, total) are cut
// into kParts equal parts, each with its own counter on its own cache line, so
// that the grabs spread over kParts addresses instead of queueing on one (a
// device-wide atomic on a single address completes only some tens of millions
// of times a second).  A workgroup starts on part blockIdx.x % kParts --
// workgroups are dealt to the XCDs in turn, so one part's neighbouring sites
// stay in one XCD's L2 -- and moves on to the next part when its own is used
// up; it is done once it has found every part empty.  Thread 0 alone holds a
// queue and calls it; the counters are zeroed before the launch.
constexpr int kParts = 8;
constexpr int kCtrStride = 32;                   // u64 words from one counter to the next
constexpr int kQueueWords = kParts * kCtrStride;

struct WorkQueue {
    unsigned long long *ctr;
    int64_t total;
    unsigned long long chunk;
    int part, left;
    unsigned long long pend;   // offset taken in `part`, not yet handed out

    // (inlined: called, the queue would live in scratch memory for its address)
    __device__ __forceinline__ int64_t bound(int x) const { return total * x / kParts; }
    __device__ __forceinline__ void init(unsigned long long *c, int64_t t, int ch) {
        ctr = c;
        total = t;
        chunk = (unsigned long long)ch;
        part = (int)(blockIdx.x % kParts);
        left = kParts;
        pend = atomicAdd(ctr + part * kCtrStride, chunk);
    }
    // The grab issued last as the chunk [lo, hi); lo == hi == total once every
    // part is used up.
    __device__ __forceinline__ void resolve(int64_t &lo, int64_t &hi) {
        for (;;) {
            const int64_t a = bound(part), b = bound(part + 1);
            const int64_t s = a + (int64_t)pend;
            if (s < b) {
                lo = s;
                hi = s + (int64_t)chunk < b ? s + (int64_t)chunk : b;
                return;
            }
            if (--left == 0) {
                lo = hi = total;
                return;
            }
            part = part + 1 == kParts ? 0 : part + 1;
            pend = atomicAdd(ctr + part * kCtrStride, chunk);
        }
    }
    // The next grab in the current part, in flight while a chunk is walked.
    __device__ __forceinline__ void prefetch() { pend = atomicAdd(ctr + part * kCtrStride, chunk); }
};

// Arguments of one launch of the class-id batch walk.
struct IdsArgs {
    const Region *regs;
    int32_t nreg;
    int64_t total;               // items (ignored with a list)
    int64_t stride;              // > 1: sample in blocks of 256 items
    unsigned long long *counter; // kQueueWords work-queue counters, zeroed before the launch
    int chunk;
    int lmax;                    // largest haplotype list of the regions
    int kcls;                    // class-table capacity, 0 = full
    int copies;                  // copies of each class counter (1 or 8)
    int pcap, kcap;              // pair and member capacity of the pairwise tail
    int dev;                     // room for the iHS walks' reference passes
    const int64_t *list;         // null, or the items to walk ...
    const int32_t *list_count;   // ... and their number (on the device)
    int64_t *redo;               // walks that outgrow a capped table go here ...
    int32_t *redo_count;         // ... counted here (zeroed before the launch)
};
hipError_t launch_ids_batch(const IdsArgs &a, const WideCfg &c, hipStream_t s);
hipError_t launch_fill_regions(const Region *host, int n, Region *dev, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long *p, int n, hipStream_t s);
// Persistent walks over total_items items; with stride > 1 item v stands for
// item 256 * stride * (v / 256) + v % 256 (a sample in blocks of 256).
// counter: kQueueWords work-queue counters, zeroed before the launch.
hipError_t launch_wide_walk(const Region *regs, int32_t nreg, int64_t total_items,
                            int64_t stride, unsigned long long *counter, const WideCfg &c,
                            hipStream_t s);

// Site-level kernels.
hipError_t launch_pack(const uint8_t *alleles, int64_t n, int64_t M, int64_t wps,
                       uint64_t *bits, hipStream_t s);
// Haplotype-major transposed matrix: [n][mwp] words, mwp = ceil(M/64) + 2.
inline int64_t hap_major_words(int64_t M) { return (M + 63) / 64 + 2; }
// The per-site passes of a scan before its walk, in one launch: site
// statistics (iHS; skipped when bits is null), segment lengths (always), and
// up to two haplotype-major copies (those with a non-null hbits).
struct SitePass {
    int64_t M;
    // site statistics
    const uint64_t *bits;
    int64_t wps, n;
    double maf_cutoff;
    int32_t nbins;
    double *freq;
    int32_t *bin;
    uint8_t *walk_flag;
    int8_t *status;
    // segments
    const int64_t *pos;
    const double *gpos;
    int64_t gap_scale, max_gap;
    int32_t physical;
    double *seg;
    // haplotype-major copies
    int64_t mwp;
    struct Copy {
        const uint64_t *bits;
        int64_t wps, n;
        uint64_t *hbits;
    } tr[2];
    // workgroups of each part (set by the launcher)
    int64_t b_stats, b_seg, b_tr[2];
};
hipError_t launch_site_pass(SitePass p, hipStream_t s);
hipError_t launch_combine(int mode, int64_t M, const uint8_t *walk_flag,
                          const WalkRec *rec, double *out_a, double *out_b,
                          double *unstd, int8_t *status, int32_t *steps_out,
                          hipStream_t s);
int64_t standardize_scratch_doubles(int64_t M, int32_t nbins);
hipError_t launch_standardize(int64_t M, const double *unstd, int8_t *status,
                              const int32_t *bin, int32_t nbins, double *binstat,
                              double *scratch, double *z, hipStream_t s);
// Genome-wide standardization over many scans' outputs (ss_genome.hip).  The
// regions' 1,024-site tiles are numbered region by region: region r owns
// tiles [tile0, tile0 + genome_tiles(M)).
struct GenomeRegion {
    const double *u;      // [M] unstandardized scores
    const double *freq;   // [M] derived frequency (iHS bins), null: one bin
    int8_t *status;       // [M] in: scan status; out: OK / BIN for scored sites
    double *z;            // [M] standardized scores
    int64_t M;
    int64_t tile0;
    int32_t n, pad;       // haplotypes of an iHS scan
};
int64_t genome_tiles(int64_t n_sites);
size_t genome_scratch_doubles(int64_t total_tiles, int32_t nbins);
hipError_t launch_genome_standardize(const GenomeRegion *host, int32_t nreg, GenomeRegion *dev,
                                     int64_t total_tiles, int32_t nbins, double *binstat,
                                     double *part, hipStream_t s);
hipError_t launch_ehh_finish(int64_t n, int64_t cap, const uint64_t *S, const int64_t *len,
                             const WalkRec *rec, double *ehh,
                             double *ihh, int8_t *status, hipStream_t s);

}  // namespace ss

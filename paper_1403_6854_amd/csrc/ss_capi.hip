// C ABI of the library (declared in include/selscan_hip.h): argument checks,
// workspace layout, the choice of walk kernel, and the launch sequences of
// ss_ehh / ss_ihs / ss_xpehh / ss_scan_batch (with graph capture and the
// autotuner of the persistent walk).  Host code only; every step of the scans
// runs in the HIP kernels of ss_walk*.hip and ss_sites.hip.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "selscan_hip.h"
#include "ss_internal.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

#define SS_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(SS_EDEV, std::string(#call) + ": " + hipGetErrorString(e_));   \
    } while (0)

#define SS_TRY(call)                      \
    do {                                  \
        const int rc_ = (call);           \
        if (rc_ != SS_OK) return rc_;     \
    } while (0)

constexpr int32_t kMaxHaps = 32767;   // class sizes are packed into 15/16-bit fields

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int nbins_of(const ss_params *p) {
    int b = (int)floor(1.0 / p->bin_width + 0.5);
    return b < 1 ? 1 : b;
}

int check_params(const ss_params *p) {
    if (!p) return fail(SS_EARG, "params is null");
    if (!(p->ehh_cutoff > 0.0 && p->ehh_cutoff <= 1.0))
        return fail(SS_EARG, "ehh_cutoff must be in (0, 1]");
    if (!(p->maf_cutoff >= 0.0 && p->maf_cutoff <= 0.5))
        return fail(SS_EARG, "maf_cutoff must be in [0, 0.5]");
    if (p->gap_scale_bp <= 0) return fail(SS_EARG, "gap_scale_bp must be > 0");
    if (p->max_gap_bp < p->gap_scale_bp) return fail(SS_EARG, "max_gap_bp must be >= gap_scale_bp");
    if (!(p->bin_width > 0.0 && p->bin_width <= 1.0))
        return fail(SS_EARG, "bin_width must be in (0, 1]");
    if (nbins_of(p) > 100000) return fail(SS_EARG, "bin_width too small");
    if (p->physical_map != 0 && p->physical_map != 1) return fail(SS_EARG, "physical_map must be 0 or 1");
    return SS_OK;
}

int check_hapmat(const ss_hapmat *h, const char *name) {
    const std::string nm(name);
    if (!h) return fail(SS_EARG, nm + " is null");
    if (!h->bits || !h->pos_bp || !h->gpos_cm) return fail(SS_EARG, nm + ": null device pointer");
    if (h->n_haps < 2 || h->n_haps > kMaxHaps)
        return fail(SS_EARG, nm + ": n_haps must be in [2, 32767]");
    if (h->n_sites < 1 || h->n_sites > ((int64_t)1 << 31) - 1)
        return fail(SS_EARG, nm + ": n_sites must be in [1, 2^31)");
    if (h->words_per_site < (h->n_haps + 63) / 64)
        return fail(SS_EARG, nm + ": words_per_site < ceil(n_haps/64)");
    return SS_OK;
}

int max_lds_per_block() {
    int dev = 0, maxlds = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 0;
    return maxlds;
}

int check_lds(size_t lds) {
    const int maxlds = max_lds_per_block();
    if (lds > (size_t)maxlds)
        return fail(SS_EDEV, "walk needs " + std::to_string(lds) +
                                 " bytes of LDS, device allows " + std::to_string(maxlds));
    return SS_OK;
}

int device_cus() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return n;
}

// Workspace of one scan.
// Counters of one launch group of the persistent walk: the first launch's
// work queue, the second (full-table) launch's, and the count of the walks
// listed for the second launch on a line of its own.
constexpr int kGroupCtrWords = 2 * ss::kQueueWords + ss::kCtrStride;

struct ScanWs {
    uint8_t *walk_flag;   // [M]
    int32_t *bin;         // [M]
    ss::WalkRec *rec;     // [M][2][2] walk results
    double *binstat;      // [nbins][3]
    double *binpart;      // per-tile partial sums of the bin statistics
    uint64_t *hbits;      // [nA (+ nB)][mwp] haplotype-major copies
    double *seg;          // [M] segment lengths with the gap rules applied
    ss::Region *region;   // [1] descriptor for the persistent walk
    unsigned long long *counter;   // [kGroupCtrWords] work queues of the two launches, redo count
    int64_t *wredo;       // [2M] walks the capped class table could not hold
    size_t bytes;
};

ScanWs carve_scan(void *base, int64_t M, int nbins, int64_t n_hapmajor) {
    ScanWs w;
    size_t off = 0;
    auto take = [&](size_t b) {
        char *p = base ? (char *)base + off : nullptr;
        off += align256(b);
        return (void *)p;
    };
    w.walk_flag = (uint8_t *)take((size_t)M);
    w.bin = (int32_t *)take(4 * (size_t)M);
    w.rec = (ss::WalkRec *)take(sizeof(ss::WalkRec) * 4 * (size_t)M);
    w.binstat = (double *)take(24 * (size_t)nbins);
    w.binpart = (double *)take(8 * (size_t)ss::standardize_scratch_doubles(M, nbins));
    w.hbits = (uint64_t *)take(8 * (size_t)n_hapmajor * (size_t)ss::hap_major_words(M));
    w.seg = (double *)take(8 * (size_t)M);
    w.region = (ss::Region *)take(sizeof(ss::Region));
    w.counter = (unsigned long long *)take(kGroupCtrWords * sizeof(unsigned long long));
    w.wredo = (int64_t *)take(8 * 2 * (size_t)M);
    w.bytes = off;
    return w;
}

struct EhhWs {
    ss::WalkRec *rec;  // [2 dirs][2 cores]
    size_t bytes;
};

EhhWs carve_ehh(void *base) {
    EhhWs w;
    w.rec = (ss::WalkRec *)base;
    w.bytes = 256;
    return w;
}

// Walk-kernel timing (events on the caller's stream).
struct Timing {
    std::mutex mu;
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    std::vector<hipEvent_t> pool;
    double ms = 0.0;
    int64_t launches = 0;
};
Timing g_timing;

hipEvent_t take_event() {
    if (!g_timing.pool.empty()) {
        hipEvent_t e = g_timing.pool.back();
        g_timing.pool.pop_back();
        return e;
    }
    // timing only: no system-scope fences (with them, each record held the
    // stream for about 3 us more)
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

int g_walk_kind = ss::WALK_AUTO;
int g_mask_lpc = 0;   // lanes per class of the bitmask walk; 0 = default
int g_mask_skip = 32;       // bitmask walk: most class slots for which markers that cut none are skipped
ss_batch_config g_bcfg = {64, 4096, 1, 0, 0, 1, 0, 1024, 16, 256, 0};
bool g_graph_on = false;
bool g_capturing = false;   // timing events are not recorded into graphs

int check_batch_config(const ss_batch_config &c) {
    if (c.kernel != 0 && c.kernel != 1) return fail(SS_EARG, "kernel must be 0 or 1");
    if (c.kernel == 0 && (c.threads < 64 || c.threads > 1024 || c.threads % 64))
        return fail(SS_EARG, "threads must be a multiple of 64 in [64, 1024] for kernel 0");
    if (c.kernel == 1 && c.threads != 128 && c.threads != 256 && c.threads != 512)
        return fail(SS_EARG, "threads must be 128, 256 or 512 for kernel 1");
    if (c.pair_cap < 0 || c.pair_cap > 16384) return fail(SS_EARG, "pair_cap must be in [0, 16384]");
    if (c.small_pair_cap < 0 || c.small_pair_cap > 16384)
        return fail(SS_EARG, "small_pair_cap must be in [0, 16384]");
    if (c.slots != 4 && c.slots != 8 && c.slots != 16) return fail(SS_EARG, "slots must be 4, 8 or 16");
    if (c.class_cap != 0 && (c.class_cap < 64 || c.class_cap > 16386))
        return fail(SS_EARG, "class_cap must be 0 or in [64, 16386]");
    if (c.counter_copies != 0 && c.counter_copies != 1 && c.counter_copies != 8)
        return fail(SS_EARG, "counter_copies must be 0, 1 or 8");
    if (c.chunk < 1 || c.chunk > 4096) return fail(SS_EARG, "chunk must be in [1, 4096]");
    if (c.blocks_per_cu < 0 || c.blocks_per_cu > 64) return fail(SS_EARG, "blocks_per_cu must be in [0, 64]");
    if (c.order != 0 && c.order != 1) return fail(SS_EARG, "order must be 0 or 1");
    if (c.small_kernel != 0 && c.small_kernel != 1) return fail(SS_EARG, "small_kernel must be 0 or 1");
    return SS_OK;
}

// Launch configuration of the persistent walk for the largest list lmax and
// the widest row wmax of its regions; false if it cannot run.
// dev: the launch holds iHS walks (room for their reference passes).
bool make_wide_cfg(const ss_batch_config &bc, int lmax, int wmax, ss::WideCfg &c, bool dev = true) {
    c.kernel = bc.kernel;
    c.dev = dev ? 1 : 0;
    c.threads = bc.threads;
    c.pair_cap = bc.pair_cap;
    c.chunk = bc.chunk;
    c.lmax = lmax;
    c.wmax = wmax;
    if (bc.kernel == 0) {
        // the configured size is a minimum: wider rows take larger workgroups
        const int need = ss::ids_threads_for(wmax, bc.slots);
        if (need == 0) return false;
        c.threads = std::max(bc.threads, need);
        if (c.threads <= 128) c.pair_cap = bc.small_pair_cap;
        // the member list of the pairwise tail: P pairs in classes of a few
        // members or more come from at most ~P / 4 haplotypes; walks with more
        // members wait in the per-marker phase
        c.key_cap = c.pair_cap > 0 ? std::min(std::max(256, c.pair_cap / 4), 32767) : 0;
        c.class_cap = bc.class_cap;
        // counter copies pay off for the large classes of wide regions; small
        // workgroups keep one copy and their occupancy
        c.copies = bc.counter_copies ? bc.counter_copies : (c.threads >= 256 ? 8 : 1);
        c.lds = ss::ids_lds_bytes(c.threads, lmax, wmax, c.class_cap, c.pair_cap, c.key_cap,
                                  c.copies, dev);
        if (c.lds == 0 || c.lds > (size_t)max_lds_per_block()) {
            c.copies = 1;
            c.lds = ss::ids_lds_bytes(c.threads, lmax, wmax, c.class_cap, c.pair_cap, c.key_cap, 1,
                                      dev);
        }
    } else {
        // a pair list of P pairs holds at most ~P / 4 haplotypes in classes of
        // a few members; walks with more wait in the per-marker phase
        c.key_cap = std::min(std::max(256, bc.pair_cap / 4), ss::wide_max_list(bc.threads));
        c.lds = ss::wide_lds_bytes(c.threads, lmax, wmax, c.pair_cap, c.key_cap);
    }
    if (c.lds == 0 || c.lds > (size_t)max_lds_per_block()) return false;
    const int occ = bc.kernel == 0 ? ss::ids_blocks_per_cu(c) : ss::wide_blocks_per_cu(c);
    if (occ < 1) return false;
    const int per = bc.blocks_per_cu > 0 ? std::min(bc.blocks_per_cu, occ) : occ;
    c.blocks = std::max(1, device_cus() * per);
    return true;
}

// Whether a walk of the scan can reach the pairwise tail of the class-id
// persistent walk, which starts once at most pcap identical pairs are left on
// live cores: a live core with n_c haplotypes holds at least cutoff * C(n_c, 2)
// pairs, and the smallest core a scan walks has at least floor(maf * n) of
// them (XPEHH: the pooled sample).  Scans that cannot get there run without
// pair buffers, and their workgroups take less LDS.
bool tail_possible(int mode, int32_t nA, int32_t nB, double maf, double cutoff, int pcap) {
    if (pcap <= 0) return false;
    int64_t m;
    if (mode == ss::MODE_POOLED) {
        m = (int64_t)nA + nB;
    } else {
        m = (int64_t)std::floor(maf * (double)nA);
        if (m < 2) m = 2;
    }
    return cutoff * 0.5 * (double)m * (double)(m - 1) <= (double)pcap;
}

// Settings the autotuner refined for one launch group of the class-id walk,
// keyed by workgroup size and pair buffers.  Only settings that leave the
// grouping of the regions unchanged are refined per group.
struct GroupTune {
    int32_t set;
    int32_t counter_copies, class_cap, chunk, blocks_per_cu;
    int32_t plain;   // 1: the group's regions are walked by the plain per-locus kernel
};
constexpr int kTuneSizes = 1024 / 64 + 1;
constexpr int kTuneCols = 7;   // a row of ss_get/set_group_tuning
GroupTune g_gtune[kTuneSizes][2];

void clear_group_tuning() {
    for (auto &row : g_gtune)
        for (auto &t : row) t = GroupTune{};
}

// The configuration one launch runs with: the group's workgroup size, no pair
// buffers for scans that cannot reach the pairwise tail, and the group's
// refined settings if the autotuner found any.
ss_batch_config launch_config(const ss_batch_config &bc, int threads, bool pairs) {
    ss_batch_config c = bc;
    c.threads = threads;
    if (bc.kernel != 0) return c;
    if (!pairs) {
        c.pair_cap = 0;
        c.small_pair_cap = 0;
    }
    if (threads > 0 && threads % 64 == 0 && threads / 64 < kTuneSizes) {
        const GroupTune &t = g_gtune[threads / 64][pairs ? 1 : 0];
        if (t.set) {
            c.counter_copies = t.counter_copies;
            c.class_cap = t.class_cap;
            c.chunk = t.chunk;
            c.blocks_per_cu = t.blocks_per_cu;
        }
    }
    return c;
}

// Which kernel walks a scan.
enum Route { RT_MASK, RT_WIDE, RT_IDS };

int list_len(int32_t nA, int32_t nB, int mode) { return nA + (mode == ss::MODE_POOLED ? nB : 0); }
int row_words(int32_t nA, int32_t nB, int mode) {
    return (nA + 63) / 64 + (mode == ss::MODE_POOLED ? (nB + 63) / 64 : 0);
}

// in_batch: the bitmask kernel takes small scans only if the batch
// configuration says so; a single scan uses it whenever it applies.
Route route_for(int32_t nA, int32_t nB, int mode, bool in_batch) {
    if (g_walk_kind == ss::WALK_LDS_IDS) return RT_IDS;
    const bool mask_ok = ss::mask_walk_shape(nA, nB, mode, g_mask_lpc).ok;
    if (g_walk_kind == ss::WALK_REG_MASKS) return mask_ok ? RT_MASK : RT_IDS;
    if (g_walk_kind == ss::WALK_AUTO && mask_ok && (!in_batch || g_bcfg.small_kernel)) return RT_MASK;
    ss::WideCfg c;
    if (make_wide_cfg(g_bcfg, list_len(nA, nB, mode), row_words(nA, nB, mode), c, mode == ss::MODE_CORE))
        return RT_WIDE;
    return RT_IDS;
}

size_t route_lds(Route r, int32_t nA, int32_t nB, int mode) {
    if (r == RT_MASK) return ss::mask_walk_shape(nA, nB, mode, g_mask_lpc).lds;
    if (r == RT_IDS) return ss::walk_shape(nA, nB, mode).lds;
    return 0;   // checked by make_wide_cfg
}

// Events around a walk launch while timing is enabled.
struct TimedRegion {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipStream_t s;
    explicit TimedRegion(hipStream_t st) : s(st) {}
    int begin() {
        std::lock_guard<std::mutex> lk(g_timing.mu);
        if (!g_timing.on || g_capturing) return SS_OK;
        e0 = take_event();
        e1 = take_event();
        if (!e0 || !e1) return fail(SS_EDEV, "hipEventCreate failed");
        SS_HIP(hipEventRecord(e0, s));
        return SS_OK;
    }
    int end() {
        if (!e0) return SS_OK;
        std::lock_guard<std::mutex> lk(g_timing.mu);
        SS_HIP(hipEventRecord(e1, s));
        g_timing.pending.emplace_back(e0, e1);
        return SS_OK;
    }
};

ss::WalkArgs walk_args(const ss_hapmat *a, const ss_hapmat *b, const ss_params *p) {
    ss::WalkArgs w{};
    w.bitsA = a->bits;
    w.wpsA = a->words_per_site;
    w.nA = (int32_t)a->n_haps;
    w.WA = (int32_t)((a->n_haps + 63) / 64);
    if (b) {
        w.bitsB = b->bits;
        w.wpsB = b->words_per_site;
        w.nB = (int32_t)b->n_haps;
        w.WB = (int32_t)((b->n_haps + 63) / 64);
    }
    w.M = a->n_sites;
    w.pos = a->pos_bp;
    w.gpos = a->gpos_cm;
    w.cutoff = p->ehh_cutoff;
    w.gap_scale = p->gap_scale_bp;
    w.max_gap = p->max_gap_bp;
    w.physical = p->physical_map;
    return w;
}

// ---- one scan: preparation, walk and finish -----------------------------------
// A scan request in internal form.
struct Scan {
    int mode;               // MODE_CORE (iHS) or MODE_POOLED (XPEHH)
    const ss_hapmat *a, *b;
    double *out_x, *out_y, *unstd, *stdz, *freq;
    int8_t *status;
    int32_t *steps;
    int nbins;
    double maf;             // MAF filter of the scan (iHS cores)
    Route route;
    ScanWs w;
    ss::WalkArgs args;
};

int64_t hapmajor_rows(int mode, const ss_hapmat *a, const ss_hapmat *b) {
    return a->n_haps + (mode == ss::MODE_POOLED ? b->n_haps : 0);
}

int validate_scan(int mode, const ss_hapmat *a, const ss_hapmat *b, const ss_params *p,
                  const void *x, const void *y, const void *u, const void *z, const void *f,
                  const void *st) {
    if (mode == ss::MODE_CORE) {
        SS_TRY(check_hapmat(a, "hapmat"));
        if (!x || !y || !u || !z || !f || !st) return fail(SS_EARG, "null output pointer");
    } else {
        SS_TRY(check_hapmat(a, "population a"));
        SS_TRY(check_hapmat(b, "population b"));
        if (a->n_sites != b->n_sites) return fail(SS_ESHAPE, "populations have different n_sites");
        if (a->n_haps + b->n_haps > kMaxHaps) return fail(SS_EARG, "n_haps(a) + n_haps(b) > 32767");
        if (!x || !y || !u || !z || !st) return fail(SS_EARG, "null output pointer");
    }
    return check_params(p);
}

size_t scan_bytes(int mode, const ss_hapmat *a, const ss_hapmat *b, const ss_params *p) {
    const int nbins = mode == ss::MODE_CORE ? nbins_of(p) : 1;
    return carve_scan(nullptr, a->n_sites, nbins, hapmajor_rows(mode, a, b)).bytes;
}

void init_scan(Scan &sc, void *base, const ss_params *p) {
    const int nbins = sc.mode == ss::MODE_CORE ? nbins_of(p) : 1;
    sc.w = carve_scan(base, sc.a->n_sites, nbins, hapmajor_rows(sc.mode, sc.a, sc.b));
    sc.args = walk_args(sc.a, sc.mode == ss::MODE_POOLED ? sc.b : nullptr, p);
    ss::WalkArgs &a = sc.args;
    a.walk_flag = sc.mode == ss::MODE_CORE ? sc.w.walk_flag : nullptr;
    a.site0 = 0;
    a.kmax = (int32_t)(list_len(a.nA, a.nB, sc.mode) / 2 + 2);
    a.rec = sc.w.rec;
    a.mwp = ss::hap_major_words(a.M);
    a.hbits = sc.mode == ss::MODE_CORE ? sc.w.hbits : nullptr;
    a.seg = sc.w.seg;
}

ss::Region region_of(const Scan &sc) {
    const ss::WalkArgs &a = sc.args;
    ss::Region r{};
    r.bitsA = a.bitsA;
    r.bitsB = a.bitsB;
    r.hbitsA = sc.w.hbits;
    r.hbitsB = sc.mode == ss::MODE_POOLED ? sc.w.hbits + (size_t)a.nA * (size_t)a.mwp : nullptr;
    r.seg = sc.w.seg;
    r.walk_flag = a.walk_flag;
    r.rec = sc.w.rec;
    r.wpsA = a.wpsA;
    r.wpsB = a.wpsB;
    r.M = a.M;
    r.mwp = a.mwp;
    r.item0 = 0;
    r.cutoff = a.cutoff;
    r.nA = a.nA;
    r.nB = sc.mode == ss::MODE_POOLED ? a.nB : 0;
    r.mode = sc.mode;
    return r;
}

// Per-site passes before the walk.
int prepare_scan(const Scan &sc, const ss_params *p, hipStream_t s) {
    const ss::WalkArgs &a = sc.args;
    ss::SitePass sp{};
    sp.M = a.M;
    if (sc.mode == ss::MODE_CORE) {
        sp.bits = a.bitsA;
        sp.wps = a.wpsA;
        sp.n = a.nA;
        sp.maf_cutoff = p->maf_cutoff;
        sp.nbins = nbins_of(p);
        sp.freq = sc.freq;
        sp.bin = sc.w.bin;
        sp.walk_flag = sc.w.walk_flag;
        sp.status = sc.status;
    }
    sp.pos = a.pos;
    sp.gpos = a.gpos;
    sp.gap_scale = p->gap_scale_bp;
    sp.max_gap = p->max_gap_bp;
    sp.physical = p->physical_map;
    sp.seg = sc.w.seg;
    // haplotype-major copies feed the pairwise phases
    sp.mwp = a.mwp;
    if (sc.route == RT_WIDE || (sc.route == RT_MASK && sc.mode == ss::MODE_CORE))
        sp.tr[0] = {a.bitsA, a.wpsA, a.nA, sc.w.hbits};
    if (sc.route == RT_WIDE && sc.mode == ss::MODE_POOLED)
        sp.tr[1] = {a.bitsB, a.wpsB, a.nB, sc.w.hbits + (size_t)a.nA * (size_t)a.mwp};
    SS_HIP(ss::launch_site_pass(sp, s));
    return SS_OK;
}

// Walk of a scan by the bitmask or class-id kernel (not the persistent one).
int walk_direct(const Scan &sc, hipStream_t s) {
    const ss::WalkArgs &a = sc.args;
    if (sc.route == RT_MASK) {
        ss::WalkArgs m = a;
        m.skip_classes = g_mask_skip;
        SS_HIP(ss::launch_mask_walk(m, sc.mode, g_mask_lpc, a.M, s));
    } else {
        SS_HIP(ss::launch_walk(a, sc.mode, false, a.M, s));
    }
    return SS_OK;
}

int finish_scan(const Scan &sc, hipStream_t s) {
    const int64_t M = sc.args.M;
    SS_HIP(ss::launch_combine(sc.mode, M, sc.mode == ss::MODE_CORE ? sc.w.walk_flag : nullptr,
                              sc.w.rec, sc.out_x, sc.out_y, sc.unstd,
                              sc.status, sc.steps, s));
    if (sc.mode == ss::MODE_CORE)
        SS_HIP(ss::launch_standardize(M, sc.unstd, sc.status, sc.w.bin, sc.nbins, sc.w.binstat,
                                      sc.w.binpart, sc.stdz, s));
    else
        SS_HIP(ss::launch_standardize(M, sc.unstd, sc.status, nullptr, 1, sc.w.binstat, sc.w.binpart,
                                      sc.stdz, s));
    return SS_OK;
}

}  // namespace

namespace {

// One launch group of the class-id batch walk: the persistent launch with the
// configured class table and, when that table is capped, a second launch with
// full tables over the walks the first one listed (it ends at once when the
// list is empty).  ctr: the first launch's work queue, the second launch's,
// then the count of listed walks, zeroed beforehand (kGroupCtrWords words).
int launch_ids_group(const ss::Region *regs, int nreg, int64_t total, int64_t stride,
                     unsigned long long *ctr, int64_t *redo, const ss::WideCfg &c, hipStream_t s) {
    ss::IdsArgs a{};
    a.regs = regs;
    a.nreg = nreg;
    a.total = total;
    a.stride = stride;
    a.counter = ctr;
    a.chunk = c.chunk;
    a.lmax = c.lmax;
    a.kcls = c.class_cap;
    a.copies = c.copies;
    a.pcap = c.pair_cap;
    a.kcap = c.key_cap;
    a.dev = c.dev;
    const bool capped = ss::ids_table_capped(c.lmax, c.class_cap);
    a.redo = capped ? redo : nullptr;
    a.redo_count = capped ? (int32_t *)(ctr + 2 * ss::kQueueWords) : nullptr;
    SS_HIP(ss::launch_ids_batch(a, c, s));
    if (!capped) return SS_OK;
    ss::WideCfg full = c;
    full.class_cap = 0;
    full.lds = ss::ids_lds_bytes(full.threads, full.lmax, full.wmax, 0, full.pair_cap, full.key_cap,
                                 full.copies, full.dev != 0);
    if (full.lds == 0 || full.lds > (size_t)max_lds_per_block()) {
        full.copies = 1;
        full.lds = ss::ids_lds_bytes(full.threads, full.lmax, full.wmax, 0, full.pair_cap,
                                     full.key_cap, 1, full.dev != 0);
    }
    if (full.lds == 0 || full.lds > (size_t)max_lds_per_block())
        return fail(SS_EDEV, "full class table does not fit this device");
    const int occ = ss::ids_blocks_per_cu(full);
    if (occ < 1) return fail(SS_EDEV, "full class table does not fit this device");
    full.blocks = std::max(1, device_cus() * occ);
    ss::IdsArgs b = a;
    b.kcls = 0;
    b.copies = full.copies;
    b.counter = ctr + ss::kQueueWords;
    b.list = redo;
    b.list_count = (const int32_t *)(ctr + 2 * ss::kQueueWords);
    b.redo = nullptr;
    b.redo_count = nullptr;
    b.stride = 1;
    SS_HIP(ss::launch_ids_batch(b, full, s));
    return SS_OK;
}

// Walk of one scan, timed when timing is enabled.
int walk_scan(Scan &sc, hipStream_t s) {
    if (sc.route == RT_WIDE) {
        ss::Region r = region_of(sc);
        const int64_t items = ss::region_items(sc.mode, sc.args.M, g_bcfg.kernel);
        ss::WideCfg c;
        const int lmax = list_len(r.nA, r.nB, sc.mode), wmax = row_words(r.nA, r.nB, sc.mode);
        const bool ihs = sc.mode == ss::MODE_CORE;
        if (!make_wide_cfg(g_bcfg, lmax, wmax, c, ihs))
            return fail(SS_EDEV, "persistent walk does not fit this device");
        if (c.kernel == 0) {   // as the region's launch group in a batch would run
            const bool pairs = tail_possible(sc.mode, r.nA, r.nB, sc.maf, r.cutoff, c.pair_cap);
            const GroupTune &gt = g_gtune[c.threads / 64][pairs ? 1 : 0];
            const ss::WalkShape ws = ss::walk_shape(r.nA, r.nB, sc.mode);
            if (gt.set && gt.plain && ws.threads <= 1024 && ws.lds <= (size_t)max_lds_per_block()) {
                TimedRegion t(s);
                SS_TRY(t.begin());
                SS_HIP(ss::launch_walk(sc.args, sc.mode, false, sc.args.M, s));
                return t.end();
            }
            if (!make_wide_cfg(launch_config(g_bcfg, c.threads, pairs), lmax, wmax, c, ihs))
                return fail(SS_EDEV, "persistent walk does not fit this device");
        }
        SS_HIP(ss::launch_fill_regions(&r, 1, sc.w.region, s));
        SS_HIP(ss::launch_zero_u64(sc.w.counter, kGroupCtrWords, s));
        TimedRegion t(s);
        SS_TRY(t.begin());
        if (c.kernel == 0)
            SS_TRY(launch_ids_group(sc.w.region, 1, items, 1, sc.w.counter, sc.w.wredo, c, s));
        else
            SS_HIP(ss::launch_wide_walk(sc.w.region, 1, items, 1, sc.w.counter, c, s));
        return t.end();
    }
    TimedRegion t(s);
    SS_TRY(t.begin());
    SS_TRY(walk_direct(sc, s));
    return t.end();
}

// ---- batches -------------------------------------------------------------------
// Regions of the persistent walk that share one launch: the class-id kernel
// gives every region the smallest workgroup that holds its rows, so regions
// are grouped by workgroup size; the list kernel takes them all in one group.
struct Group {
    int first = 0, count = 0;   // range of Batch::regions
    int64_t total_items = 0;
    int lmax = 0, wmax = 0, threads = 0;
    bool pairs = true;          // some walk can reach the pairwise tail
    bool ihs = false;           // some region is an iHS scan (reference passes)
};

constexpr int kMaxGroups = 32;

struct Batch;
bool plain_fits(const Batch &B, const Group &g);

// The group is walked by the plain per-locus class-id kernel (the autotuner
// found it faster for this group, and its class tables fit in LDS).
bool group_plain(const ss_batch_config &bc, const Batch &B, const Group &g) {
    if (bc.kernel != 0 || g.threads % 64 || g.threads / 64 >= kTuneSizes) return false;
    const GroupTune &t = g_gtune[g.threads / 64][g.pairs ? 1 : 0];
    return t.set && t.plain && plain_fits(B, g);
}

struct Batch {
    std::vector<Scan> scans;
    std::vector<int> wide;            // scans walked by the persistent kernel
    std::vector<ss::Region> regions;  // their descriptors, group by group (item0 per group)
    std::vector<int> region_scan;     // the scan of each of them
    std::vector<Group> groups;
    ss::Region *d_regions = nullptr;
    unsigned long long *d_counter = nullptr;   // kGroupCtrWords per group
    int64_t *d_redo = nullptr;                 // redo lists, group by group
    int64_t total_items = 0;
    int lmax = 0, wmax = 0;
};

bool plain_fits(const Batch &B, const Group &g) {
    for (int q = g.first; q < g.first + g.count; ++q) {
        const Scan &sc = B.scans[B.region_scan[q]];
        const ss::WalkShape sh = ss::walk_shape(sc.args.nA, sc.args.nB, sc.mode);
        if (sh.threads > 1024 || sh.lds > (size_t)max_lds_per_block()) return false;
    }
    return true;
}

struct BatchLayout {
    std::vector<size_t> offs;
    size_t regions = 0, counter = 0, redo = 0, bytes = 0;
};

int op_mode(int32_t op) { return op == SS_OP_IHS ? ss::MODE_CORE : ss::MODE_POOLED; }

int check_requests(const ss_scan_request *reqs, int32_t n, const ss_params *p) {
    if (!reqs || n < 1) return fail(SS_EARG, "no requests");
    if (n > 65535) return fail(SS_EARG, "more than 65535 requests");
    SS_TRY(check_params(p));
    for (int32_t i = 0; i < n; ++i) {
        const ss_scan_request &r = reqs[i];
        if (r.op != SS_OP_IHS && r.op != SS_OP_XPEHH) return fail(SS_EARG, "request " + std::to_string(i) + ": unknown op");
        const int rc = validate_scan(op_mode(r.op), &r.a, &r.b, p, r.d_ihh_x, r.d_ihh_y, r.d_unstd,
                                     r.d_std, r.d_freq, r.d_status);
        if (rc != SS_OK) return fail(rc, "request " + std::to_string(i) + ": " + g_err);
    }
    return SS_OK;
}

BatchLayout batch_layout(const ss_scan_request *reqs, int32_t n, const ss_params *p) {
    BatchLayout L;
    size_t off = 0;
    for (int32_t i = 0; i < n; ++i) {
        L.offs.push_back(off);
        off += align256(scan_bytes(op_mode(reqs[i].op), &reqs[i].a, &reqs[i].b, p));
    }
    L.regions = off;
    off += align256(sizeof(ss::Region) * (size_t)n);
    L.counter = off;
    off += align256(sizeof(unsigned long long) * kGroupCtrWords * kMaxGroups);
    L.redo = off;   // walks listed for the full-table pass, 2 items per site at most
    size_t sites = 0;
    for (int32_t i = 0; i < n; ++i) sites += (size_t)reqs[i].a.n_sites;
    off += align256(8 * 2 * sites);
    L.bytes = off;
    return L;
}

// Launch groups and item numbering of the persistent walk's regions for a
// configuration (region order within a group: as given, or most haplotypes
// first).
void number_items(Batch &B, const ss_batch_config &bc) {
    struct Key {
        int threads, idx, len;
        bool pairs;
    };
    std::vector<Key> keys;
    for (size_t i = 0; i < B.wide.size(); ++i) {
        const Scan &sc = B.scans[B.wide[i]];
        const int len = list_len(sc.args.nA, sc.args.nB, sc.mode);
        const int wrd = row_words(sc.args.nA, sc.args.nB, sc.mode);
        const int t = bc.kernel == 0 ? std::max(bc.threads, ss::ids_threads_for(wrd, bc.slots))
                                     : bc.threads;
        const bool pairs = bc.kernel != 0 ||
                           tail_possible(sc.mode, sc.args.nA, sc.args.nB, sc.maf, sc.args.cutoff,
                                         t <= 128 ? bc.small_pair_cap : bc.pair_cap);
        keys.push_back({t, (int)i, len, pairs});
    }
    std::stable_sort(keys.begin(), keys.end(), [&](const Key &x, const Key &y) {
        if (x.threads != y.threads) return x.threads > y.threads;
        if (x.pairs != y.pairs) return x.pairs;
        if (bc.order == 1) return x.len > y.len;
        return false;
    });
    B.regions.clear();
    B.region_scan.clear();
    B.groups.clear();
    B.total_items = 0;
    int64_t item = 0;
    for (const Key &k : keys) {
        if (B.groups.empty() || B.groups.back().threads != k.threads ||
            B.groups.back().pairs != k.pairs) {
            Group g;
            g.first = (int)B.regions.size();
            g.threads = k.threads;
            g.pairs = k.pairs;
            B.groups.push_back(g);
            item = 0;
        }
        Group &g = B.groups.back();
        const Scan &sc = B.scans[B.wide[k.idx]];
        ss::Region r = region_of(sc);
        r.item0 = item;
        const int64_t n_items = ss::region_items(sc.mode, sc.args.M, bc.kernel);
        item += n_items;
        g.count += 1;
        g.total_items += n_items;
        g.lmax = std::max(g.lmax, k.len);
        g.wmax = std::max(g.wmax, row_words(sc.args.nA, sc.args.nB, sc.mode));
        g.ihs = g.ihs || sc.mode == ss::MODE_CORE;
        B.total_items += n_items;
        B.regions.push_back(r);
        B.region_scan.push_back(B.wide[k.idx]);
    }
}

int build_batch(const ss_scan_request *reqs, int32_t n, const ss_params *p, void *d_ws,
                size_t ws_bytes, Batch &B) {
    SS_TRY(check_requests(reqs, n, p));
    const BatchLayout L = batch_layout(reqs, n, p);
    if (!d_ws || ws_bytes < L.bytes) return fail(SS_EWS, "workspace smaller than ss_batch_workspace_bytes()");
    B.scans.resize((size_t)n);
    for (int32_t i = 0; i < n; ++i) {
        const ss_scan_request &r = reqs[i];
        Scan &sc = B.scans[(size_t)i];
        sc.mode = op_mode(r.op);
        sc.a = &r.a;
        sc.b = sc.mode == ss::MODE_POOLED ? &r.b : nullptr;
        sc.out_x = r.d_ihh_x;
        sc.out_y = r.d_ihh_y;
        sc.unstd = r.d_unstd;
        sc.stdz = r.d_std;
        sc.freq = r.d_freq;
        sc.status = r.d_status;
        sc.steps = r.d_steps;
        sc.nbins = sc.mode == ss::MODE_CORE ? nbins_of(p) : 1;
        sc.maf = p->maf_cutoff;
        init_scan(sc, (char *)d_ws + L.offs[(size_t)i], p);
        const int32_t nB = sc.mode == ss::MODE_POOLED ? (int32_t)r.b.n_haps : 0;
        sc.route = route_for((int32_t)r.a.n_haps, nB, sc.mode, true);
        if (sc.route != RT_WIDE) {
            const int rc = check_lds(route_lds(sc.route, (int32_t)r.a.n_haps, nB, sc.mode));
            if (rc != SS_OK) return fail(rc, "request " + std::to_string(i) + ": " + g_err);
        } else {
            B.wide.push_back(i);
            B.lmax = std::max(B.lmax, list_len((int32_t)r.a.n_haps, nB, sc.mode));
            B.wmax = std::max(B.wmax, row_words((int32_t)r.a.n_haps, nB, sc.mode));
        }
    }
    B.d_regions = (ss::Region *)((char *)d_ws + L.regions);
    B.d_counter = (unsigned long long *)((char *)d_ws + L.counter);
    B.d_redo = (int64_t *)((char *)d_ws + L.redo);
    number_items(B, g_bcfg);
    if ((int)B.groups.size() > kMaxGroups) return fail(SS_EDEV, "too many launch groups");
    return SS_OK;
}

// The persistent walks over the batch's regions, one launch per group;
// sample_stride > 1 walks only every sample_stride-th item of each group.
// only >= 0: that group alone (the autotuner's per-group timing).
int launch_batch_wide(Batch &B, const ss_batch_config &bc, int64_t sample_stride, hipStream_t s,
                      int only = -1) {
    if (B.wide.empty()) return SS_OK;
    SS_HIP(ss::launch_fill_regions(B.regions.data(), (int)B.regions.size(), B.d_regions, s));
    SS_HIP(ss::launch_zero_u64(B.d_counter, kGroupCtrWords * kMaxGroups, s));
    int64_t redo_off = 0;
    for (size_t gi = 0; gi < B.groups.size(); ++gi) {
        const Group &g = B.groups[gi];
        if (only >= 0 && (int)gi != only) {
            redo_off += g.total_items;
            continue;
        }
        const int64_t stride = sample_stride > 1 ? sample_stride : 1;
        if (group_plain(bc, B, g)) {
            // the plain per-locus kernel, region by region (a sample: the
            // first 1 / stride of each region's sites)
            for (int q = g.first; q < g.first + g.count; ++q) {
                const Scan &sc = B.scans[B.region_scan[q]];
                const int64_t sites = stride > 1 ? (sc.args.M + stride - 1) / stride : sc.args.M;
                SS_HIP(ss::launch_walk(sc.args, sc.mode, false, sites, s));
            }
            redo_off += g.total_items;
            continue;
        }
        ss::WideCfg c;
        if (!make_wide_cfg(launch_config(bc, g.threads, g.pairs), g.lmax, g.wmax, c, g.ihs))
            return fail(SS_EDEV, "persistent walk configuration does not fit this device");
        int64_t total = g.total_items;
        if (stride > 1) {   // blocks of 256 items, one in every `stride`
            const int64_t blocks = (g.total_items + 255) / 256;
            total = 256 * ((blocks + stride - 1) / stride);
        }
        ss::Region *regs = B.d_regions + g.first;
        unsigned long long *ctr = B.d_counter + kGroupCtrWords * gi;
        if (c.kernel == 0)
            SS_TRY(launch_ids_group(regs, g.count, total, stride, ctr, B.d_redo + redo_off, c, s));
        else
            SS_HIP(ss::launch_wide_walk(regs, g.count, total, stride, ctr, c, s));
        redo_off += g.total_items;
    }
    return SS_OK;
}

int enqueue_batch(Batch &B, const ss_params *p, hipStream_t s) {
    for (auto &sc : B.scans) SS_TRY(prepare_scan(sc, p, s));
    TimedRegion t(s);
    SS_TRY(t.begin());
    for (auto &sc : B.scans)
        if (sc.route != RT_WIDE) SS_TRY(walk_direct(sc, s));
    SS_TRY(launch_batch_wide(B, g_bcfg, 1, s));
    SS_TRY(t.end());
    for (auto &sc : B.scans) SS_TRY(finish_scan(sc, s));
    return SS_OK;
}

// Captured graphs of ss_scan_batch, keyed by everything the sequence depends on.
struct GraphCache {
    std::mutex mu;
    std::map<std::string, std::pair<hipGraph_t, hipGraphExec_t>> g;
};
GraphCache g_graphs;

template <typename T>
void put(std::string &k, const T &v) {
    k.append((const char *)&v, sizeof(T));
}

std::string graph_key(const ss_scan_request *reqs, int32_t n, const ss_params *p, void *d_ws,
                      size_t ws_bytes, void *stream) {
    std::string k;
    int dev = 0;
    (void)hipGetDevice(&dev);
    put(k, dev);
    put(k, n);
    // field by field: the structs' padding bytes are not part of the key
    for (int32_t i = 0; i < n; ++i) {
        const ss_scan_request &r = reqs[i];
        put(k, r.op);
        for (const ss_hapmat *h : {&r.a, &r.b}) {
            put(k, h->bits);
            put(k, h->n_haps);
            put(k, h->n_sites);
            put(k, h->words_per_site);
            put(k, h->pos_bp);
            put(k, h->gpos_cm);
        }
        put(k, r.d_ihh_x);
        put(k, r.d_ihh_y);
        put(k, r.d_unstd);
        put(k, r.d_std);
        put(k, r.d_freq);
        put(k, r.d_status);
        put(k, r.d_steps);
    }
    put(k, p->ehh_cutoff);
    put(k, p->maf_cutoff);
    put(k, p->gap_scale_bp);
    put(k, p->max_gap_bp);
    put(k, p->bin_width);
    put(k, p->physical_map);
    put(k, d_ws);
    put(k, ws_bytes);
    put(k, stream);
    put(k, g_bcfg);
    put(k, g_gtune);
    put(k, g_walk_kind);
    put(k, g_mask_lpc);
    put(k, g_mask_skip);
    return k;
}

// ---- static scratch of ss_ihs_static -----------------------------------------
// For callers that cannot allocate device memory: the scan's workspace lives in
// a file-scope device array instead of a caller's buffer.  Each device the
// library runs on holds its own copy until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in for
// the symbol): the device address comes from hipGetSymbolAddress, taken once
// per device with that device current, and is used everywhere instead.
constexpr size_t kStaticScratchBytes = (size_t)32 << 20;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`.
int static_scratch(void **out) {
    int dev = -1;
    SS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SS_EDEV, "device index out of range for the static scratch");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        SS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(SS_EDEV, "hipGetSymbolAddress returned a null address for the static scratch");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SS_OK;
}

}  // namespace

extern "C" {

void ss_default_params(ss_params *p) {
    if (!p) return;
    p->ehh_cutoff = 0.05;
    p->maf_cutoff = 0.05;
    p->gap_scale_bp = 20000;
    p->max_gap_bp = 200000;
    p->bin_width = 0.025;
    p->physical_map = 0;
}

const char *ss_version(void) { return "selscan-hip 0.2 (gfx950)"; }

const char *ss_last_error(void) { return g_err.c_str(); }

int ss_pack(const uint8_t *d_alleles, int64_t n_haps, int64_t n_sites, int64_t words_per_site,
            uint64_t *d_bits, void *stream) {
    g_err.clear();
    if (!d_alleles || !d_bits) return fail(SS_EARG, "null device pointer");
    if (n_haps < 1 || n_sites < 1) return fail(SS_EARG, "n_haps and n_sites must be >= 1");
    if (words_per_site < (n_haps + 63) / 64) return fail(SS_EARG, "words_per_site < ceil(n_haps/64)");
    SS_HIP(ss::launch_pack(d_alleles, n_haps, n_sites, words_per_site, d_bits, (hipStream_t)stream));
    return SS_OK;
}

size_t ss_workspace_bytes(int op, const ss_hapmat *a, const ss_hapmat *b, const ss_params *p,
                          int64_t ehh_cap) {
    (void)ehh_cap;
    if (!a || !p || check_params(p) != SS_OK) return 0;
    switch (op) {
        case SS_OP_EHH: return carve_ehh(nullptr).bytes;
        case SS_OP_IHS: return scan_bytes(ss::MODE_CORE, a, nullptr, p);
        case SS_OP_XPEHH:
            if (!b) return 0;
            return scan_bytes(ss::MODE_POOLED, a, b, p);
        default: return 0;
    }
}

int ss_ehh(const ss_hapmat *h, int64_t core, const ss_params *p, int64_t cap, uint64_t *d_S,
           double *d_ehh, int64_t *d_len, uint32_t *d_class_sizes, double *d_ihh,
           int8_t *d_status, void *d_ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    SS_TRY(check_hapmat(h, "hapmat"));
    SS_TRY(check_params(p));
    if (core < 0 || core >= h->n_sites) return fail(SS_EARG, "core out of range");
    if (cap < 1 || cap > ((int64_t)1 << 30)) return fail(SS_EARG, "cap must be in [1, 2^30]");
    if (!d_S || !d_ehh || !d_len || !d_ihh || !d_status) return fail(SS_EARG, "null output pointer");
    EhhWs w = carve_ehh(d_ws);
    if (!d_ws || ws_bytes < w.bytes) return fail(SS_EWS, "workspace smaller than ss_workspace_bytes()");
    const ss::WalkShape sh = ss::walk_shape((int32_t)h->n_haps, 0, ss::MODE_CORE);
    SS_TRY(check_lds(sh.lds));
    hipStream_t s = (hipStream_t)stream;
    SS_HIP(hipMemsetAsync(d_S, 0, sizeof(uint64_t) * 2 * (size_t)(cap + 1), s));
    if (d_class_sizes)
        SS_HIP(hipMemsetAsync(d_class_sizes, 0,
                              sizeof(uint32_t) * 2 * (size_t)(cap + 1) * (size_t)h->n_haps, s));
    ss::WalkArgs a = walk_args(h, nullptr, p);
    a.site0 = core;
    a.kmax = (int32_t)(h->n_haps / 2 + 2);
    a.rec = w.rec;
    a.trS = d_S;
    a.trSizes = d_class_sizes;
    a.trLen = d_len;
    a.cap = cap;
    SS_HIP(ss::launch_walk(a, ss::MODE_CORE, true, 1, s));
    SS_HIP(ss::launch_ehh_finish(h->n_haps, cap, d_S, d_len, w.rec, d_ehh, d_ihh,
                                 d_status, s));
    return SS_OK;
}

static int run_single(Scan &sc, const ss_params *p, void *d_ws, size_t ws_bytes, hipStream_t s) {
    const size_t need = scan_bytes(sc.mode, sc.a, sc.b, p);
    if (!d_ws || ws_bytes < need) return fail(SS_EWS, "workspace smaller than ss_workspace_bytes()");
    sc.nbins = sc.mode == ss::MODE_CORE ? nbins_of(p) : 1;
    sc.maf = p->maf_cutoff;
    init_scan(sc, d_ws, p);
    const int32_t nB = sc.mode == ss::MODE_POOLED ? (int32_t)sc.b->n_haps : 0;
    sc.route = route_for((int32_t)sc.a->n_haps, nB, sc.mode, false);
    if (sc.route != RT_WIDE) SS_TRY(check_lds(route_lds(sc.route, (int32_t)sc.a->n_haps, nB, sc.mode)));
    SS_TRY(prepare_scan(sc, p, s));
    SS_TRY(walk_scan(sc, s));
    return finish_scan(sc, s);
}

int ss_ihs(const ss_hapmat *h, const ss_params *p, double *d_ihh1, double *d_ihh0,
           double *d_unstd, double *d_std, double *d_freq, int8_t *d_status, int32_t *d_steps,
           void *d_ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    SS_TRY(validate_scan(ss::MODE_CORE, h, nullptr, p, d_ihh1, d_ihh0, d_unstd, d_std, d_freq,
                         d_status));
    Scan sc{};
    sc.mode = ss::MODE_CORE;
    sc.a = h;
    sc.b = nullptr;
    sc.out_x = d_ihh1;
    sc.out_y = d_ihh0;
    sc.unstd = d_unstd;
    sc.stdz = d_std;
    sc.freq = d_freq;
    sc.status = d_status;
    sc.steps = d_steps;
    return run_single(sc, p, d_ws, ws_bytes, (hipStream_t)stream);
}

int ss_xpehh(const ss_hapmat *ha, const ss_hapmat *hb, const ss_params *p, double *d_ihhA,
             double *d_ihhB, double *d_unstd, double *d_std, int8_t *d_status, int32_t *d_steps,
             void *d_ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    SS_TRY(validate_scan(ss::MODE_POOLED, ha, hb, p, d_ihhA, d_ihhB, d_unstd, d_std, nullptr,
                         d_status));
    Scan sc{};
    sc.mode = ss::MODE_POOLED;
    sc.a = ha;
    sc.b = hb;
    sc.out_x = d_ihhA;
    sc.out_y = d_ihhB;
    sc.unstd = d_unstd;
    sc.stdz = d_std;
    sc.freq = nullptr;
    sc.status = d_status;
    sc.steps = d_steps;
    return run_single(sc, p, d_ws, ws_bytes, (hipStream_t)stream);
}

int ss_ihs_static(const ss_hapmat *h, const ss_params *p, double *d_ihh1, double *d_ihh0,
                  double *d_unstd, double *d_std, double *d_freq, int8_t *d_status,
                  int32_t *d_steps, void *stream) {
    g_err.clear();
    SS_TRY(validate_scan(ss::MODE_CORE, h, nullptr, p, d_ihh1, d_ihh0, d_unstd, d_std, d_freq,
                         d_status));
    const size_t need = scan_bytes(ss::MODE_CORE, h, nullptr, p);
    if (need > kStaticScratchBytes)
        return fail(SS_EWS, "scan needs " + std::to_string(need) + " bytes of scratch; the static scratch holds " +
                                std::to_string(kStaticScratchBytes) + " (use ss_ihs with a workspace)");
    void *ws = nullptr;
    SS_TRY(static_scratch(&ws));
    Scan sc{};
    sc.mode = ss::MODE_CORE;
    sc.a = h;
    sc.b = nullptr;
    sc.out_x = d_ihh1;
    sc.out_y = d_ihh0;
    sc.unstd = d_unstd;
    sc.stdz = d_std;
    sc.freq = d_freq;
    sc.status = d_status;
    sc.steps = d_steps;
    return run_single(sc, p, ws, kStaticScratchBytes, (hipStream_t)stream);
}

size_t ss_static_scratch_bytes(void) { return kStaticScratchBytes; }

}  // extern "C"

namespace {

// Workspace of ss_genome_standardize: the region table, the bin statistics
// (unless the caller asks for them in d_binstat) and the per-tile sums.
struct GenomeWs {
    ss::GenomeRegion *table;
    double *binstat;
    double *part;
    int64_t tiles;
    size_t bytes;
};

int check_genome(const ss_std_region *regs, int32_t n, int32_t op, const ss_params *p) {
    if (!regs || n < 1) return fail(SS_EARG, "no regions");
    if (n > (1 << 20)) return fail(SS_EARG, "more than 2^20 regions");
    if (op != SS_OP_IHS && op != SS_OP_XPEHH) return fail(SS_EARG, "op must be SS_OP_IHS or SS_OP_XPEHH");
    SS_TRY(check_params(p));
    for (int32_t i = 0; i < n; ++i) {
        const ss_std_region &r = regs[i];
        const std::string at = "region " + std::to_string(i) + ": ";
        if (r.n_sites < 0 || r.n_sites > ((int64_t)1 << 31) - 1)
            return fail(SS_EARG, at + "n_sites must be in [0, 2^31)");
        if (r.n_sites > 0 && (!r.d_unstd || !r.d_status || !r.d_std))
            return fail(SS_EARG, at + "null device pointer");
        if (op == SS_OP_IHS && r.n_sites > 0) {
            if (!r.d_freq) return fail(SS_EARG, at + "iHS regions need their derived frequencies");
            if (r.n_haps < 2 || r.n_haps > kMaxHaps) return fail(SS_EARG, at + "n_haps must be in [2, 32767]");
        }
    }
    return SS_OK;
}

GenomeWs carve_genome(void *base, const ss_std_region *regs, int32_t n, int nbins, bool own_binstat) {
    GenomeWs w{};
    int64_t tiles = 0;
    for (int32_t i = 0; i < n; ++i) tiles += ss::genome_tiles(regs[i].n_sites);
    w.tiles = tiles;
    size_t off = 0;
    auto take = [&](size_t b) {
        char *q = base ? (char *)base + off : nullptr;
        off += align256(b);
        return (void *)q;
    };
    w.table = (ss::GenomeRegion *)take(sizeof(ss::GenomeRegion) * (size_t)n);
    w.binstat = own_binstat ? (double *)take(24 * (size_t)nbins) : nullptr;
    w.part = (double *)take(8 * std::max<size_t>(1, ss::genome_scratch_doubles(tiles, nbins)));
    w.bytes = off;
    return w;
}

}  // namespace

extern "C" {

size_t ss_genome_workspace_bytes(const ss_std_region *regs, int32_t n_regs, int32_t op,
                                 const ss_params *p) {
    if (check_genome(regs, n_regs, op, p) != SS_OK) return 0;
    const int nbins = op == SS_OP_IHS ? nbins_of(p) : 1;
    return carve_genome(nullptr, regs, n_regs, nbins, true).bytes;
}

int ss_genome_standardize(const ss_std_region *regs, int32_t n_regs, int32_t op, const ss_params *p,
                          double *d_binstat, void *d_ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    SS_TRY(check_genome(regs, n_regs, op, p));
    const int nbins = op == SS_OP_IHS ? nbins_of(p) : 1;
    const GenomeWs need = carve_genome(nullptr, regs, n_regs, nbins, d_binstat == nullptr);
    if (!d_ws || ws_bytes < need.bytes) return fail(SS_EWS, "workspace smaller than ss_genome_workspace_bytes()");
    GenomeWs w = carve_genome(d_ws, regs, n_regs, nbins, d_binstat == nullptr);
    if (d_binstat) w.binstat = d_binstat;
    std::vector<ss::GenomeRegion> host((size_t)n_regs);
    int64_t t0 = 0;
    for (int32_t i = 0; i < n_regs; ++i) {
        const ss_std_region &r = regs[i];
        ss::GenomeRegion &g = host[(size_t)i];
        g.u = r.d_unstd;
        g.freq = op == SS_OP_IHS ? r.d_freq : nullptr;
        g.status = r.d_status;
        g.z = r.d_std;
        g.M = r.n_sites;
        g.tile0 = t0;
        g.n = r.n_haps;
        g.pad = 0;
        t0 += ss::genome_tiles(r.n_sites);
    }
    SS_HIP(ss::launch_genome_standardize(host.data(), n_regs, w.table, w.tiles, nbins, w.binstat, w.part,
                                         (hipStream_t)stream));
    return SS_OK;
}

size_t ss_batch_workspace_bytes(const ss_scan_request *reqs, int32_t n_reqs, const ss_params *p) {
    if (check_requests(reqs, n_reqs, p) != SS_OK) return 0;
    return batch_layout(reqs, n_reqs, p).bytes;
}

int ss_scan_batch(const ss_scan_request *reqs, int32_t n_reqs, const ss_params *p, void *d_ws,
                  size_t ws_bytes, void *stream) {
    g_err.clear();
    Batch B;
    SS_TRY(build_batch(reqs, n_reqs, p, d_ws, ws_bytes, B));
    hipStream_t s = (hipStream_t)stream;
    if (!g_graph_on || !stream) return enqueue_batch(B, p, s);

    const std::string key = graph_key(reqs, n_reqs, p, d_ws, ws_bytes, stream);
    std::lock_guard<std::mutex> lk(g_graphs.mu);
    auto it = g_graphs.g.find(key);
    if (it == g_graphs.g.end()) {
        SS_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        g_capturing = true;
        const int rc = enqueue_batch(B, p, s);
        g_capturing = false;
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(s, &graph);
        if (rc != SS_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (ec != hipSuccess) return fail(SS_EDEV, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
        hipGraphExec_t exec = nullptr;
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return fail(SS_EDEV, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
        }
        it = g_graphs.g.emplace(key, std::make_pair(graph, exec)).first;
    }
    TimedRegion t(s);
    SS_TRY(t.begin());
    SS_HIP(hipGraphLaunch(it->second.second, s));
    return t.end();
}

int ss_get_batch_config(ss_batch_config *c) {
    if (!c) return fail(SS_EARG, "config is null");
    *c = g_bcfg;
    return SS_OK;
}

int ss_set_batch_config(const ss_batch_config *c) {
    if (!c) return fail(SS_EARG, "config is null");
    SS_TRY(check_batch_config(*c));
    g_bcfg = *c;
    clear_group_tuning();
    return SS_OK;
}

int ss_set_group_tuning(const int32_t *rows, int32_t n_rows) {
    if (n_rows < 0 || (n_rows > 0 && !rows)) return fail(SS_EARG, "rows is null");
    for (int32_t i = 0; i < n_rows; ++i) {
        const int32_t *r = rows + kTuneCols * i;
        const bool ok = r[0] >= 64 && r[0] <= 1024 && r[0] % 64 == 0 && (r[1] == 0 || r[1] == 1) &&
                        (r[2] == 0 || r[2] == 1 || r[2] == 8) &&
                        (r[3] == 0 || (r[3] >= 64 && r[3] <= 16386)) && r[4] >= 1 && r[4] <= 4096 &&
                        r[5] >= 0 && r[5] <= 64 && (r[6] == 0 || r[6] == 1);
        if (!ok) return fail(SS_EARG, "group tuning row " + std::to_string(i) + " out of range");
    }
    clear_group_tuning();
    for (int32_t i = 0; i < n_rows; ++i) {
        const int32_t *r = rows + kTuneCols * i;
        g_gtune[r[0] / 64][r[1]] = GroupTune{1, r[2], r[3], r[4], r[5], r[6]};
    }
    return SS_OK;
}

int ss_get_group_tuning(int32_t *rows, int32_t max_rows, int32_t *n_rows) {
    if (!n_rows) return fail(SS_EARG, "n_rows is null");
    if (max_rows < 0 || (max_rows > 0 && !rows)) return fail(SS_EARG, "rows is null");
    int32_t n = 0;
    for (int t = 0; t < kTuneSizes; ++t) {
        for (int pr = 0; pr < 2; ++pr) {
            const GroupTune &g = g_gtune[t][pr];
            if (!g.set) continue;
            if (n < max_rows) {
                int32_t *r = rows + kTuneCols * n;
                r[0] = 64 * t;
                r[1] = pr;
                r[2] = g.counter_copies;
                r[3] = g.class_cap;
                r[4] = g.chunk;
                r[5] = g.blocks_per_cu;
                r[6] = g.plain;
            }
            ++n;
        }
    }
    *n_rows = n;
    return SS_OK;
}

int ss_autotune_batch(const ss_scan_request *reqs, int32_t n_reqs, const ss_params *p, void *d_ws,
                      size_t ws_bytes, void *stream, int64_t sample_items, ss_batch_config *best,
                      double *best_ms) {
    g_err.clear();
    Batch B;
    SS_TRY(build_batch(reqs, n_reqs, p, d_ws, ws_bytes, B));
    hipStream_t s = (hipStream_t)stream;
    for (auto &sc : B.scans) SS_TRY(prepare_scan(sc, p, s));
    clear_group_tuning();
    ss_batch_config cur = g_bcfg;
    if (cur.kernel == 0) cur.threads = 64;
    double cur_ms = 0.0;
    if (!B.wide.empty()) {
        // the sample: blocks of 256 consecutive items (runs of neighbouring
        // sites, as the full walk sees them), one block in every `stride` of
        // each launch group -- the same fraction of the work for every
        // candidate, whether an item is a (site, direction) or, in the list
        // kernel, one core of it
        int64_t pairs = 0;
        for (int i : B.wide) pairs += 2 * B.scans[i].args.M;
        const bool whole = sample_items <= 0 || sample_items >= pairs;
        const int64_t stride = whole ? 1 : pairs / sample_items;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        SS_HIP(hipEventCreate(&e0));
        SS_HIP(hipEventCreate(&e1));
        auto time_cfg = [&](const ss_batch_config &c, double &ms) -> int {
            number_items(B, c);
            for (const Group &g : B.groups) {
                ss::WideCfg wc;
                if ((int)B.groups.size() > kMaxGroups ||
                    !make_wide_cfg(launch_config(c, g.threads, g.pairs), g.lmax, g.wmax, wc, g.ihs)) {
                    ms = 1e30;
                    return SS_OK;
                }
            }
            double bestv = 1e30;
            for (int rep = 0; rep < 2; ++rep) {
                SS_HIP(hipEventRecord(e0, s));
                SS_TRY(launch_batch_wide(B, c, stride, s));
                SS_HIP(hipEventRecord(e1, s));
                SS_HIP(hipEventSynchronize(e1));
                float f = 0.f;
                SS_HIP(hipEventElapsedTime(&f, e0, e1));
                bestv = std::min(bestv, (double)f);
            }
            ms = bestv;
            return SS_OK;
        };
        SS_TRY(time_cfg(cur, cur_ms));   // warm-up and baseline
        SS_TRY(time_cfg(cur, cur_ms));
        // kernel and workgroup size together, then one setting at a time
        // kernel 0 gives each region the smallest workgroup holding its rows
        for (int k : {0, 1}) {
            for (int t : {64, 128, 256, 512}) {
                ss_batch_config c = cur;
                c.kernel = k;
                c.threads = t;
                if (k == 0 && t != 64) continue;
                if (check_batch_config(c) != SS_OK) continue;
                double ms;
                SS_TRY(time_cfg(c, ms));
                if (ms < cur_ms) { cur = c; cur_ms = ms; }
            }
        }
        g_err.clear();
        for (int pass = 0; pass < 2; ++pass) {
            for (int pc : {0, 1024, 2048, 4096, 8192}) {
                ss_batch_config c = cur;
                c.pair_cap = pc;
                double ms;
                SS_TRY(time_cfg(c, ms));
                if (ms < cur_ms) { cur = c; cur_ms = ms; }
            }
            if (cur.kernel == 0) {
                for (int pc : {0, 512, 1024, 2048}) {
                    ss_batch_config c = cur;
                    c.small_pair_cap = pc;
                    double ms;
                    SS_TRY(time_cfg(c, ms));
                    if (ms < cur_ms) { cur = c; cur_ms = ms; }
                }
            }
            for (int bpc : {0, 1, 2, 3, 4}) {
                ss_batch_config c = cur;
                c.blocks_per_cu = bpc;
                double ms;
                SS_TRY(time_cfg(c, ms));
                if (ms < cur_ms) { cur = c; cur_ms = ms; }
            }
            if (cur.kernel == 0) {
                for (int cc : {0, 256, 512, 1024, 2048}) {
                    ss_batch_config c = cur;
                    c.class_cap = cc;
                    double ms;
                    SS_TRY(time_cfg(c, ms));
                    if (ms < cur_ms) { cur = c; cur_ms = ms; }
                }
                for (int cp : {1, 8}) {
                    ss_batch_config c = cur;
                    c.counter_copies = cp;
                    double ms;
                    SS_TRY(time_cfg(c, ms));
                    if (ms < cur_ms) { cur = c; cur_ms = ms; }
                }
                for (int sl : {4, 8, 16}) {
                    ss_batch_config c = cur;
                    c.slots = sl;
                    double ms;
                    SS_TRY(time_cfg(c, ms));
                    if (ms < cur_ms) { cur = c; cur_ms = ms; }
                }
            }
            for (int ch : {1, 2, 4, 8}) {
                ss_batch_config c = cur;
                c.chunk = ch;
                double ms;
                SS_TRY(time_cfg(c, ms));
                if (ms < cur_ms) { cur = c; cur_ms = ms; }
            }
            if (whole && B.wide.size() > 1) {
                for (int o : {0, 1}) {
                    ss_batch_config c = cur;
                    c.order = o;
                    double ms;
                    SS_TRY(time_cfg(c, ms));
                    if (ms < cur_ms) { cur = c; cur_ms = ms; }
                }
            }
        }
        // then each launch group on its own: the settings that leave the
        // grouping unchanged, one at a time, starting from the batch's
        if (cur.kernel == 0 && B.groups.size() > 1) {
            number_items(B, cur);
            for (size_t gi = 0; gi < B.groups.size(); ++gi) {
                const Group &g = B.groups[gi];
                if (g.threads % 64 || g.threads / 64 >= kTuneSizes) continue;
                GroupTune &slot = g_gtune[g.threads / 64][g.pairs ? 1 : 0];
                auto time_group = [&](const GroupTune &t, double &ms) -> int {
                    slot = t;
                    ss::WideCfg wc;
                    if (t.plain ? !plain_fits(B, g)
                                : !make_wide_cfg(launch_config(cur, g.threads, g.pairs), g.lmax,
                                                 g.wmax, wc, g.ihs)) {
                        ms = 1e30;
                        return SS_OK;
                    }
                    double bestv = 1e30;
                    for (int rep = 0; rep < 2; ++rep) {
                        SS_HIP(hipEventRecord(e0, s));
                        SS_TRY(launch_batch_wide(B, cur, stride, s, (int)gi));
                        SS_HIP(hipEventRecord(e1, s));
                        SS_HIP(hipEventSynchronize(e1));
                        float f = 0.f;
                        SS_HIP(hipEventElapsedTime(&f, e0, e1));
                        bestv = std::min(bestv, (double)f);
                    }
                    ms = bestv;
                    return SS_OK;
                };
                GroupTune bt{1, cur.counter_copies, cur.class_cap, cur.chunk, cur.blocks_per_cu};
                double bms;
                SS_TRY(time_group(bt, bms));
                auto try_t = [&](GroupTune t) -> int {
                    double ms;
                    SS_TRY(time_group(t, ms));
                    if (ms < bms) { bt = t; bms = ms; }
                    return SS_OK;
                };
                for (int cp : {1, 8}) { GroupTune t = bt; t.counter_copies = cp; SS_TRY(try_t(t)); }
                for (int cc : {0, 256, 512, 1024, 2048}) { GroupTune t = bt; t.class_cap = cc; SS_TRY(try_t(t)); }
                for (int ch : {1, 2, 4, 8}) { GroupTune t = bt; t.chunk = ch; SS_TRY(try_t(t)); }
                for (int bpc : {0, 2, 3, 4}) { GroupTune t = bt; t.blocks_per_cu = bpc; SS_TRY(try_t(t)); }
                {   // or the plain per-locus kernel for this group's regions
                    GroupTune t = bt;
                    t.plain = 1;
                    SS_TRY(try_t(t));
                }
                slot = bt;
            }
            // kept if the whole batch runs at least as fast with them
            double with_ms;
            SS_TRY(time_cfg(cur, with_ms));
            if (with_ms <= cur_ms) cur_ms = with_ms;
            else clear_group_tuning();
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    g_bcfg = cur;
    if (best) *best = cur;
    if (best_ms) *best_ms = cur_ms;
    return SS_OK;
}

int ss_set_graph(int on) {
    g_graph_on = on != 0;
    return SS_OK;
}

int ss_graph_clear(void) {
    std::lock_guard<std::mutex> lk(g_graphs.mu);
    for (auto &kv : g_graphs.g) {
        (void)hipGraphExecDestroy(kv.second.second);
        (void)hipGraphDestroy(kv.second.first);
    }
    g_graphs.g.clear();
    return SS_OK;
}

int ss_set_walk_kernel(int kind) {
    if (kind < ss::WALK_AUTO || kind > ss::WALK_WIDE) return fail(SS_EARG, "unknown walk kernel");
    g_walk_kind = kind;
    return SS_OK;
}

int ss_set_mask_skip(int max_classes) {
    if (max_classes < 0 || max_classes > 64) return fail(SS_EARG, "max_classes must be in [0, 64]");
    g_mask_skip = max_classes;
    return SS_OK;
}

int ss_set_mask_lanes(int lanes_per_class) {
    if (lanes_per_class != 0 && lanes_per_class != 1 && lanes_per_class != 2 &&
        lanes_per_class != 4 && lanes_per_class != 8)
        return fail(SS_EARG, "lanes_per_class must be 0, 1, 2, 4 or 8");
    g_mask_lpc = lanes_per_class;
    return SS_OK;
}

int ss_timing_enable(int on) {
    std::lock_guard<std::mutex> lk(g_timing.mu);
    g_timing.on = on != 0;
    return SS_OK;
}

int ss_timing_read(double *walk_ms_total, int64_t *walk_launches, int reset) {
    std::lock_guard<std::mutex> lk(g_timing.mu);
    for (auto &pr : g_timing.pending) {
        SS_HIP(hipEventSynchronize(pr.second));
        float ms = 0.f;
        SS_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
        g_timing.ms += ms;
        g_timing.launches += 1;
        g_timing.pool.push_back(pr.first);
        g_timing.pool.push_back(pr.second);
    }
    g_timing.pending.clear();
    if (walk_ms_total) *walk_ms_total = g_timing.ms;
    if (walk_launches) *walk_launches = g_timing.launches;
    if (reset) {
        g_timing.ms = 0.0;
        g_timing.launches = 0;
    }
    return SS_OK;
}

}  // extern "C"

// C ABI of the library (declared in include/selscan_hip.h): argument checks,
// workspace layout, and the launch sequences of ss_ehh / ss_ihs / ss_xpehh.
// Host code only; every step of the scans runs in the HIP kernels of
// ss_walk.hip and ss_sites.hip.
#include <math.h>
#include <stdio.h>

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

int check_lds(size_t lds) {
    int dev = 0, maxlds = 0;
    SS_HIP(hipGetDevice(&dev));
    SS_HIP(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    if (lds > (size_t)maxlds)
        return fail(SS_EDEV, "class table needs " + std::to_string(lds) +
                                 " bytes of LDS, device allows " + std::to_string(maxlds));
    return SS_OK;
}

// Workspace of the scans.
struct ScanWs {
    uint8_t *walk_flag;   // [M]
    int32_t *bin;         // [M]
    double *dihh;         // [M][2][2]
    int32_t *dstatus;     // [M][2][2]
    int32_t *dsteps;      // [M][2][2]
    double *binstat;      // [nbins][3]
    double *binpart;      // per-tile partial sums of the bin statistics
    uint64_t *hbits;      // [n][mwp] haplotype-major copy (iHS only)
    double *seg;          // [M] segment lengths with the gap rules applied
    int32_t *redo;        // [1 + 2M] overflow count, then the walks to redo
    size_t bytes;
};

ScanWs carve_scan(void *base, int64_t M, int nbins, int64_t n_hapmajor = 0) {
    ScanWs w;
    size_t off = 0;
    auto take = [&](size_t b) {
        char *p = base ? (char *)base + off : nullptr;
        off += align256(b);
        return (void *)p;
    };
    w.walk_flag = (uint8_t *)take((size_t)M);
    w.bin = (int32_t *)take(4 * (size_t)M);
    w.dihh = (double *)take(32 * (size_t)M);
    w.dstatus = (int32_t *)take(16 * (size_t)M);
    w.dsteps = (int32_t *)take(16 * (size_t)M);
    w.binstat = (double *)take(24 * (size_t)nbins);
    w.binpart = (double *)take(8 * (size_t)ss::standardize_scratch_doubles(M, nbins));
    w.hbits = n_hapmajor ? (uint64_t *)take(8 * (size_t)n_hapmajor * (size_t)ss::hap_major_words(M))
                         : nullptr;
    w.seg = (double *)take(8 * (size_t)M);
    w.redo = (int32_t *)take(4 * (1 + 2 * (size_t)M));
    w.bytes = off;
    return w;
}

struct EhhWs {
    double *dihh;      // [2][2]
    int32_t *dstatus;  // [2]
    size_t bytes;
};

EhhWs carve_ehh(void *base) {
    EhhWs w;
    w.dihh = (double *)base;
    w.dstatus = base ? (int32_t *)((char *)base + 256) : nullptr;
    w.bytes = 512;
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
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int g_walk_kind = ss::WALK_AUTO;
int g_mask_lpc = 0;   // lanes per class of the bitmask walk; 0 = default

// Automatic choice: the bitmask walk whenever the haplotypes fit (up to 512
// in the walk), the class-id walk otherwise.
bool use_mask_walk(int32_t nA, int32_t nB, int mode) {
    if (g_walk_kind == ss::WALK_LDS_IDS) return false;
    return ss::mask_walk_shape(nA, nB, mode, g_mask_lpc).ok;
}

hipError_t launch_scan_walk(const ss::WalkArgs &a, int mode, int64_t blocks, hipStream_t s) {
    if (use_mask_walk(a.nA, a.nB, mode)) return ss::launch_mask_walk(a, mode, g_mask_lpc, blocks, s);
    return ss::launch_walk(a, mode, false, blocks, s);
}

// LDS needed by the walk chosen for this shape.
size_t scan_walk_lds(int32_t nA, int32_t nB, int mode) {
    if (use_mask_walk(nA, nB, mode)) return ss::mask_walk_shape(nA, nB, mode, g_mask_lpc).lds;
    return ss::walk_shape(nA, nB, mode).lds;
}

// Workgroups of the pass that redoes, with the class-id walk, the walks the
// bitmask kernel could not hold; it exits at once when there are none.
constexpr int kRedoBlocks = 256;

int launch_timed_walk(const ss::WalkArgs &a, int mode, int64_t blocks, hipStream_t s) {
    std::unique_lock<std::mutex> lk(g_timing.mu);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (g_timing.on) {
        e0 = take_event();
        e1 = take_event();
        if (!e0 || !e1) return fail(SS_EDEV, "hipEventCreate failed");
        SS_HIP(hipEventRecord(e0, s));
    }
    SS_HIP(launch_scan_walk(a, mode, blocks, s));
    if (a.redo_count && use_mask_walk(a.nA, a.nB, mode))
        SS_HIP(ss::launch_walk_list(a, mode, kRedoBlocks, s));
    if (g_timing.on) {
        SS_HIP(hipEventRecord(e1, s));
        g_timing.pending.emplace_back(e0, e1);
    }
    return SS_OK;
}

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
    return w;
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
}

const char *ss_version(void) { return "selscan-hip 0.1 (gfx950)"; }

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
        case SS_OP_IHS: return carve_scan(nullptr, a->n_sites, nbins_of(p), a->n_haps).bytes;
        case SS_OP_XPEHH:
            if (!b) return 0;
            return carve_scan(nullptr, a->n_sites, 1).bytes;
        default: return 0;
    }
}

int ss_ehh(const ss_hapmat *h, int64_t core, const ss_params *p, int64_t cap, uint64_t *d_S,
           double *d_ehh, int64_t *d_len, uint32_t *d_class_sizes, double *d_ihh,
           int8_t *d_status, void *d_ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    int rc;
    if ((rc = check_hapmat(h, "hapmat")) != SS_OK) return rc;
    if ((rc = check_params(p)) != SS_OK) return rc;
    if (core < 0 || core >= h->n_sites) return fail(SS_EARG, "core out of range");
    if (cap < 1 || cap > ((int64_t)1 << 30)) return fail(SS_EARG, "cap must be in [1, 2^30]");
    if (!d_S || !d_ehh || !d_len || !d_ihh || !d_status) return fail(SS_EARG, "null output pointer");
    EhhWs w = carve_ehh(d_ws);
    if (!d_ws || ws_bytes < w.bytes) return fail(SS_EWS, "workspace smaller than ss_workspace_bytes()");
    const ss::WalkShape sh = ss::walk_shape((int32_t)h->n_haps, 0, ss::MODE_CORE);
    if ((rc = check_lds(sh.lds)) != SS_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    SS_HIP(hipMemsetAsync(d_S, 0, sizeof(uint64_t) * 2 * (size_t)(cap + 1), s));
    if (d_class_sizes)
        SS_HIP(hipMemsetAsync(d_class_sizes, 0,
                              sizeof(uint32_t) * 2 * (size_t)(cap + 1) * (size_t)h->n_haps, s));
    ss::WalkArgs a = walk_args(h, nullptr, p);
    a.site0 = core;
    a.kmax = (int32_t)(h->n_haps / 2 + 2);
    a.ihh = w.dihh;
    a.dstatus = w.dstatus;
    a.trS = d_S;
    a.trSizes = d_class_sizes;
    a.trLen = d_len;
    a.cap = cap;
    SS_HIP(ss::launch_walk(a, ss::MODE_CORE, true, 1, s));
    SS_HIP(ss::launch_ehh_finish(h->n_haps, cap, d_S, d_len, w.dihh, w.dstatus, d_ehh, d_ihh,
                                 d_status, s));
    return SS_OK;
}

int ss_ihs(const ss_hapmat *h, const ss_params *p, double *d_ihh1, double *d_ihh0,
           double *d_unstd, double *d_std, double *d_freq, int8_t *d_status, int32_t *d_steps,
           void *d_ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    int rc;
    if ((rc = check_hapmat(h, "hapmat")) != SS_OK) return rc;
    if ((rc = check_params(p)) != SS_OK) return rc;
    if (!d_ihh1 || !d_ihh0 || !d_unstd || !d_std || !d_freq || !d_status)
        return fail(SS_EARG, "null output pointer");
    const int nbins = nbins_of(p);
    ScanWs w = carve_scan(d_ws, h->n_sites, nbins, h->n_haps);
    if (!d_ws || ws_bytes < w.bytes) return fail(SS_EWS, "workspace smaller than ss_workspace_bytes()");
    if ((rc = check_lds(scan_walk_lds((int32_t)h->n_haps, 0, ss::MODE_CORE))) != SS_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int64_t M = h->n_sites;
    SS_HIP(ss::launch_site_stats(h->bits, h->words_per_site, h->n_haps, M, p->maf_cutoff, nbins,
                                 d_freq, w.bin, w.walk_flag, d_status, s));
    ss::WalkArgs a = walk_args(h, nullptr, p);
    a.walk_flag = w.walk_flag;
    a.site0 = 0;
    a.kmax = (int32_t)(h->n_haps / 2 + 2);
    a.ihh = w.dihh;
    a.dstatus = w.dstatus;
    a.steps = w.dsteps;
    a.mwp = ss::hap_major_words(M);
    a.hbits = w.hbits;
    a.seg = w.seg;
    a.redo_count = w.redo;
    a.redo_list = w.redo + 1;
    SS_HIP(ss::launch_transpose(h->bits, h->words_per_site, h->n_haps, M, a.mwp, w.hbits, s));
    SS_HIP(ss::launch_segments(M, h->pos_bp, h->gpos_cm, p->gap_scale_bp, p->max_gap_bp, w.seg,
                               w.redo, s));
    if ((rc = launch_timed_walk(a, ss::MODE_CORE, M, s)) != SS_OK) return rc;
    SS_HIP(ss::launch_combine(ss::MODE_CORE, M, w.walk_flag, w.dihh, w.dstatus, w.dsteps, d_ihh1,
                              d_ihh0, d_unstd, d_status, d_steps, s));
    SS_HIP(ss::launch_standardize(M, d_unstd, d_status, w.bin, nbins, w.binstat, w.binpart, d_std,
                                  s));
    return SS_OK;
}

int ss_xpehh(const ss_hapmat *ha, const ss_hapmat *hb, const ss_params *p, double *d_ihhA,
             double *d_ihhB, double *d_unstd, double *d_std, int8_t *d_status, int32_t *d_steps,
             void *d_ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    int rc;
    if ((rc = check_hapmat(ha, "population a")) != SS_OK) return rc;
    if ((rc = check_hapmat(hb, "population b")) != SS_OK) return rc;
    if ((rc = check_params(p)) != SS_OK) return rc;
    if (ha->n_sites != hb->n_sites) return fail(SS_ESHAPE, "populations have different n_sites");
    if (ha->n_haps + hb->n_haps > kMaxHaps) return fail(SS_EARG, "n_haps(a) + n_haps(b) > 32767");
    if (!d_ihhA || !d_ihhB || !d_unstd || !d_std || !d_status)
        return fail(SS_EARG, "null output pointer");
    ScanWs w = carve_scan(d_ws, ha->n_sites, 1);
    if (!d_ws || ws_bytes < w.bytes) return fail(SS_EWS, "workspace smaller than ss_workspace_bytes()");
    if ((rc = check_lds(scan_walk_lds((int32_t)ha->n_haps, (int32_t)hb->n_haps, ss::MODE_POOLED))) !=
        SS_OK)
        return rc;
    hipStream_t s = (hipStream_t)stream;
    const int64_t M = ha->n_sites;
    ss::WalkArgs a = walk_args(ha, hb, p);
    a.walk_flag = nullptr;
    a.site0 = 0;
    a.kmax = (int32_t)((ha->n_haps + hb->n_haps) / 2 + 2);
    a.ihh = w.dihh;
    a.dstatus = w.dstatus;
    a.steps = w.dsteps;
    a.seg = w.seg;
    a.redo_count = w.redo;
    a.redo_list = w.redo + 1;
    SS_HIP(ss::launch_segments(M, ha->pos_bp, ha->gpos_cm, p->gap_scale_bp, p->max_gap_bp, w.seg,
                               w.redo, s));
    if ((rc = launch_timed_walk(a, ss::MODE_POOLED, M, s)) != SS_OK) return rc;
    SS_HIP(ss::launch_combine(ss::MODE_POOLED, M, nullptr, w.dihh, w.dstatus, w.dsteps, d_ihhA,
                              d_ihhB, d_unstd, d_status, d_steps, s));
    SS_HIP(ss::launch_standardize(M, d_unstd, d_status, nullptr, 1, w.binstat, w.binpart, d_std, s));
    return SS_OK;
}

int ss_set_walk_kernel(int kind) {
    if (kind < ss::WALK_AUTO || kind > ss::WALK_REG_MASKS) return fail(SS_EARG, "unknown walk kernel");
    g_walk_kind = kind;
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

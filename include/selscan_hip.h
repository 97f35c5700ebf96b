/*
 * selscan_hip.h -- C ABI of the MI355X (gfx950) library for EHH-based
 * selection scans: EHH, iHS and XPEHH as defined by Szpiech & Hernandez,
 * "selscan: an efficient multi-threaded program to perform EHH-based scans
 * for positive selection" (arXiv:1403.6854).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Plain C: no HIP or framework types.  `stream` is a hipStream_t passed as
 *    an opaque pointer (NULL = the default stream).  Calls enqueue work on
 *    `stream` and return without synchronizing; outputs are valid once the
 *    stream has been synchronized.
 *  - Pointers prefixed `d_` and every pointer inside `ss_hapmat` are DEVICE
 *    pointers on the current HIP device.  Descriptors (`ss_hapmat`,
 *    `ss_params`) are HOST structs, read during the call only.
 *  - The caller owns every buffer.  The library never allocates device
 *    memory: scratch space is the caller's workspace, sized by
 *    ss_workspace_bytes() and passed as (d_ws, ws_bytes), 256-byte aligned.
 *    One workspace must not be used by two calls that overlap in time.
 *  - Allele encoding (Sec. 1.1): bit 1 = derived allele, bit 0 = ancestral.
 *    Haplotype matrices are bit-packed MARKER-major: site s occupies
 *    words_per_site uint64 words at bits + s*words_per_site; haplotype h is
 *    bit (h % 64) of word (h / 64).  Padding bits above n_haps must be 0.
 *  - "Downstream" is increasing site index, "upstream" decreasing.
 *  - Return codes: SS_OK, or a negative SS_E* code with a message available
 *    from ss_last_error() (per calling thread).  Argument errors are detected
 *    before anything is enqueued.  Content checks that need the data (sorted
 *    positions, zero padding, identical sites in both XPEHH populations) are
 *    the caller's responsibility (the Python binding does them on the host).
 */
#ifndef SELSCAN_HIP_H
#define SELSCAN_HIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define SS_OK 0
#define SS_EARG (-1)    /* invalid argument (null pointer, size or parameter) */
#define SS_ESHAPE (-2)  /* XPEHH populations with different site counts       */
#define SS_EWS (-3)     /* workspace missing or smaller than required          */
#define SS_EDEV (-4)    /* HIP runtime error or device limit exceeded          */

/* Per-site status codes (int8 outputs). Any status other than SS_ST_OK leaves
 * NaN in the scores it affects. */
#define SS_ST_OK 0
#define SS_ST_MAF 1        /* iHS: core site with MAF below the cutoff (Sec. 1.2)       */
#define SS_ST_EDGE 2       /* end of the data reached before the cutoff (Sec. 1.2)      */
#define SS_ST_GAP 3        /* a gap longer than max_gap_bp was crossed (Sec. 1.2)       */
#define SS_ST_UNDEFINED 4  /* a core has < 2 haplotypes, or an iHH is 0                 */
#define SS_ST_BIN 5        /* scores valid but the standardization bin has < 2 loci or
                              zero spread: the standardized score is NaN               */
#define SS_ST_CAPACITY 6   /* ss_ehh: a walk needed more than `cap` markers             */

/* Operation selector for ss_workspace_bytes(). */
#define SS_OP_EHH 0
#define SS_OP_IHS 1
#define SS_OP_XPEHH 2

/* The flexible parameters of Sec. 1.2 (and Sec. 1.3 for XPEHH).  Defaults in
 * brackets are the paper's values; bin_width is the iHS frequency-bin width. */
typedef struct ss_params {
    double ehh_cutoff;     /* EHH truncation value, in (0, 1]               [0.05]   */
    double maf_cutoff;     /* iHS core-site MAF cutoff, in [0, 0.5]         [0.05]   */
    int64_t gap_scale_bp;  /* gaps b > this scale g by gap_scale_bp / b, > 0 [20000] */
    int64_t max_gap_bp;    /* gaps b > this abort the locus, >= gap_scale  [200000] */
    double bin_width;      /* derived-allele-frequency bin width, (0, 1]   [0.025]  */
    int32_t physical_map;  /* 0: integrate EHH over the genetic map, g = difference of
                              gpos_cm [default]; 1: over the physical map, g = difference
                              of pos_bp in base pairs (the rehh convention the paper
                              compares against in Sec. 2.1); the gap rules apply to
                              both in the same way                              [0]      */
} ss_params;

/* A bit-packed haplotype matrix with its physical and genetic map
 * (non-owning descriptor; all pointers are device pointers). */
typedef struct ss_hapmat {
    const uint64_t *bits;     /* [n_sites][words_per_site], see above                  */
    int64_t n_haps;           /* haplotypes, 2 .. 32767                                  */
    int64_t n_sites;          /* sites, >= 1                                             */
    int64_t words_per_site;   /* row stride in words, >= ceil(n_haps / 64)               */
    const int64_t *pos_bp;    /* [n_sites] physical positions, non-decreasing           */
    const double *gpos_cm;    /* [n_sites] genetic positions (cM), non-decreasing       */
} ss_hapmat;

/* Fills *p with the paper's default parameters. */
void ss_default_params(ss_params *p);

/* Version string of the library build. */
const char *ss_version(void);

/* Message of the last failing call made by this thread ("" if none). */
const char *ss_last_error(void);

/*
 * ss_pack -- bit-pack 0/1 alleles into the marker-major layout (Sec. 1.1's
 * 0 = ancestral, 1 = derived).
 *   d_alleles  [n_sites][n_haps] uint8, 0 or 1 (any nonzero byte counts as 1)
 *   d_bits     [n_sites][words_per_site] uint64 output; padding bits written 0
 * Errors: SS_EARG for null pointers, n_haps < 1, n_sites < 1 or
 * words_per_site < ceil(n_haps/64).
 */
int ss_pack(const uint8_t *d_alleles, int64_t n_haps, int64_t n_sites,
            int64_t words_per_site, uint64_t *d_bits, void *stream);

/*
 * ss_workspace_bytes -- device workspace needed by one call of `op` on these
 * shapes (b is used for SS_OP_XPEHH only; ehh_cap for SS_OP_EHH only).
 * Returns 0 for invalid arguments.
 */
size_t ss_workspace_bytes(int op, const ss_hapmat *a, const ss_hapmat *b,
                          const ss_params *p, int64_t ehh_cap);

/*
 * ss_ehh -- EHH at one core site (Sec. 1.1, Eq. 1 and Eq. 3), both
 * directions, with the truncation and gap rules of Sec. 1.2 (the MAF cutoff
 * does not apply).  Walks continue while either core's EHH_c is at or above
 * the cutoff; every class of both cores is tracked to the end of the walk.
 *   core            site index of x0, 0 <= core < n_sites
 *   cap             most markers recorded per direction (>= 1)
 *   d_S             [2 dirs][cap+1][2] uint64: S_c(x_i) = sum over the classes
 *                   of core c of C(n_h, 2), i = 0..len (i = 0 is x0)
 *   d_ehh           [2][cap+1][3] double: EHH_0, EHH_1 (Eq. 3) and the whole-
 *                   sample EHH (Eq. 1) at x_i; NaN past len or where C(n_c,2)=0
 *   d_len           [2] int64: markers walked downstream (0) and upstream (1)
 *   d_class_sizes   NULL, or [2][cap+1][n_haps] uint32: the sizes of the
 *                   classes with >= 2 members at x_i, in no particular order,
 *                   core allele in bit 31, zero-filled
 *   d_ihh           [2] double: iHH_0, iHH_1 (Eq. 4), NaN unless status OK
 *   d_status        [1] int8: OK, EDGE, GAP, UNDEFINED or CAPACITY
 * Errors: SS_EARG, SS_EWS, SS_EDEV.
 */
int ss_ehh(const ss_hapmat *h, int64_t core, const ss_params *p, int64_t cap,
           uint64_t *d_S, double *d_ehh, int64_t *d_len, uint32_t *d_class_sizes,
           double *d_ihh, int8_t *d_status, void *d_ws, size_t ws_bytes, void *stream);

/*
 * ss_ihs -- iHS scan over every site of h (Sec. 1.2, Eqs. 3-6).
 * For each core site with MAF >= maf_cutoff: iHH_1 and iHH_0 by trapezoidal
 * quadrature of EHH_c over the genetic map, truncated before the first marker
 * with EHH_c < ehh_cutoff, with gap scaling and the edge / gap aborts; the
 * unstandardized score ln(iHH_1/iHH_0); and the score standardized within
 * derived-allele-frequency bins (bin = min(floor(B n1/n), B-1),
 * B = round(1/bin_width); mean and N-1 standard deviation of the OK loci).
 *   d_ihh1, d_ihh0, d_unstd, d_std   [n_sites] double outputs
 *   d_freq                           [n_sites] double: derived frequency n1/n
 *   d_status                         [n_sites] int8 (SS_ST_*)
 *   d_steps     NULL or [n_sites][2 dirs][2 cores] int32: markers each core
 *               walked (incl. the one where it stopped); 0 for unscored sites
 * Errors: SS_EARG, SS_EWS, SS_EDEV.
 */
int ss_ihs(const ss_hapmat *h, const ss_params *p, double *d_ihh1, double *d_ihh0,
           double *d_unstd, double *d_std, double *d_freq, int8_t *d_status,
           int32_t *d_steps, void *d_ws, size_t ws_bytes, void *stream);

/*
 * ss_xpehh -- XPEHH scan of population a against b over every site
 * (Sec. 1.3, Eqs. 7-9).  Both populations share the sites (same n_sites and
 * the same pos_bp / gpos_cm contents).  Per site: iHH_A and iHH_B integrate
 * each population's whole-sample EHH (Eq. 1, the core site being part of the
 * haplotype, so each curve starts at [C(n0,2)+C(n1,2)]/C(n,2)), both truncated
 * before the first marker where the EHH of the pooled sample drops below the
 * cutoff; the unstandardized score ln(iHH_A/iHH_B); and the score standardized
 * over all OK sites.  There is no MAF filter.
 *   d_ihhA, d_ihhB, d_unstd, d_std   [n_sites] double outputs
 *   d_status                         [n_sites] int8
 *   d_steps     NULL or [n_sites][2 dirs] int32: pooled markers walked
 * Errors: SS_EARG, SS_ESHAPE, SS_EWS, SS_EDEV.
 */
int ss_xpehh(const ss_hapmat *a, const ss_hapmat *b, const ss_params *p,
             double *d_ihhA, double *d_ihhB, double *d_unstd, double *d_std,
             int8_t *d_status, int32_t *d_steps, void *d_ws, size_t ws_bytes,
             void *stream);

/*
 * ss_ihs_static -- ss_ihs for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same scan, the same kernels and the same results, with its
 * scratch in a static device array of ss_static_scratch_bytes() bytes (32 MiB)
 * that each GPU the library runs on holds until the process ends, instead of a
 * caller's workspace.  The caller passes the inputs and outputs as for ss_ihs.
 * It calls no allocating routine.  Every call on one GPU shares that GPU's
 * array, and each call clears what it needs cleared: calls that overlap in
 * time on one GPU (two streams, two threads) race and must be serialized by
 * the caller.
 * Errors: as ss_ihs; SS_EWS when the scan needs more scratch than the array
 * holds (ss_workspace_bytes(SS_OP_IHS, ...) > ss_static_scratch_bytes()).
 */
int ss_ihs_static(const ss_hapmat *h, const ss_params *p, double *d_ihh1, double *d_ihh0,
                  double *d_unstd, double *d_std, double *d_freq, int8_t *d_status,
                  int32_t *d_steps, void *stream);

/* Size of the static scratch array of ss_ihs_static, in bytes. */
size_t ss_static_scratch_bytes(void);

/*
 * Genome-wide standardization.  The paper standardizes iHS within
 * derived-allele-frequency bins over the entire genome (Sec. 1.2, Eq. 6) and
 * XPEHH over all loci (Sec. 1.3, Eq. 9).  ss_ihs, ss_xpehh and ss_scan_batch
 * standardize each scan on its own; ss_genome_standardize re-standardizes the
 * outputs of many scans -- the chromosomes of a genome, the regions of a
 * batch -- together, as one sequence of loci (regions in the order given,
 * sites in order within each): per bin, N and the mean of every scored score,
 * then the N-1 standard deviation, then z = (u - mean) / sd, as the per-scan
 * standardization does for one scan.
 */
typedef struct ss_std_region {
    const double *d_unstd;   /* [n_sites] a scan's unstandardized scores (d_unstd output)   */
    const double *d_freq;    /* [n_sites] iHS: the scan's derived frequencies (d_freq
                                output), which give each site's bin; ignored for XPEHH   */
    int8_t *d_status;        /* [n_sites] in/out: the scan's statuses.  Sites with OK or
                                BIN are scored and come out OK, or BIN when their
                                genome-wide bin has fewer than 2 loci or zero spread;
                                other statuses are left unchanged                        */
    double *d_std;           /* [n_sites] out: genome-wide standardized scores (NaN where
                                the status is not OK)                                    */
    int64_t n_sites;         /* >= 0                                                     */
    int32_t n_haps;          /* iHS: haplotypes of the scan (2 .. 32767); ignored for XPEHH */
    int32_t reserved;
} ss_std_region;

/* Workspace of ss_genome_standardize (0 for invalid arguments). */
size_t ss_genome_workspace_bytes(const ss_std_region *regs, int32_t n_regs, int32_t op,
                                 const ss_params *p);

/*
 * ss_genome_standardize -- standardize the regions' scores together.
 *   op          SS_OP_IHS (bins of width p->bin_width) or SS_OP_XPEHH (one bin)
 *   d_binstat   NULL, or [nbins][3] double out: N, mean and SD of each bin
 * The regions' buffers must not overlap one another.  Results are the same
 * from run to run (sums in a fixed order).
 * Errors: SS_EARG, SS_EWS, SS_EDEV.
 */
int ss_genome_standardize(const ss_std_region *regs, int32_t n_regs, int32_t op,
                          const ss_params *p, double *d_binstat, void *d_ws, size_t ws_bytes,
                          void *stream);

/*
 * ss_set_walk_kernel -- choose the EHH-walk kernel used by ss_ihs / ss_xpehh
 * (process-wide; results are identical, only speed differs):
 *   0 = automatic (bitmask kernel when it applies, else the persistent
 *       walk of ss_scan_batch, else class ids),
 *   1 = class ids in LDS (any haplotype count): the plain kernel, one
 *       workgroup per (site, direction), launched over every site,
 *   2 = class bitmasks in registers (up to 1,024 haplotypes in the walk,
 *       pooled for XPEHH; larger inputs use class ids),
 *   3 = the persistent walk of ss_scan_batch with its current configuration
 *       (ss_set_batch_config); inputs it cannot take use class ids.
 * Errors: SS_EARG for any other value.
 */
int ss_set_walk_kernel(int kind);

/*
 * Batched scans.  One call scans many regions -- iHS regions and XPEHH
 * region pairs of any sizes -- and runs the EHH walks of all of them in one
 * persistent launch: a grid sized to the GPU takes work items (region, site,
 * direction[, core]) from device counters (the items cut into 8 parts, one
 * counter each), so walks of very uneven length and regions of different
 * haplotype counts share the launch.  Every result
 * is the one ss_ihs / ss_xpehh gives for that region alone (Sec. 1.2 and
 * Sec. 1.3; standardization is per region).
 */
typedef struct ss_scan_request {
    int32_t op;          /* SS_OP_IHS or SS_OP_XPEHH                                */
    ss_hapmat a;         /* the haplotypes (iHS), population A (XPEHH)              */
    ss_hapmat b;         /* population B (XPEHH only; same sites as a)              */
    double *d_ihh_x;     /* [n_sites] iHS: iHH_1; XPEHH: iHH_A                      */
    double *d_ihh_y;     /* [n_sites] iHS: iHH_0; XPEHH: iHH_B                      */
    double *d_unstd;     /* [n_sites]                                               */
    double *d_std;       /* [n_sites]                                               */
    double *d_freq;      /* [n_sites] iHS derived frequency; ignored for XPEHH      */
    int8_t *d_status;    /* [n_sites]                                               */
    int32_t *d_steps;    /* NULL, or the layout of ss_ihs / ss_xpehh                */
} ss_scan_request;

/* Workspace of ss_scan_batch for these requests (0 for invalid arguments). */
size_t ss_batch_workspace_bytes(const ss_scan_request *reqs, int32_t n_reqs,
                                const ss_params *p);

/*
 * ss_scan_batch -- every request's scan, as one sequence on `stream`.
 * The requests' output buffers must not overlap.  With graphs enabled
 * (ss_set_graph) and a non-NULL stream, the sequence is captured into a HIP
 * graph the first time a call with identical arguments is made, and replayed
 * afterwards.
 * Errors: SS_EARG, SS_ESHAPE, SS_EWS, SS_EDEV (with the failing request's
 * index in ss_last_error()).
 */
int ss_scan_batch(const ss_scan_request *reqs, int32_t n_reqs, const ss_params *p,
                  void *d_ws, size_t ws_bytes, void *stream);

/* Launch configuration of the persistent walk (process-wide). */
typedef struct ss_batch_config {
    int32_t threads;        /* workgroup size.  Kernel 0: a multiple of 64 in [64, 1024],
                               a minimum -- each region takes the smallest size that
                               holds its rows (`slots` 64-haplotype words per wave), and
                               regions of one size share one launch; kernel 1: 128, 256
                               or 512                                                   */
    int32_t pair_cap;       /* pairs, and haplotypes, the pairwise phase holds: 0..16384
                               (kernel 0: launches of 256 threads or more)              */
    int32_t chunk;          /* work items taken per grab of the counter, >= 1            */
    int32_t blocks_per_cu;  /* persistent workgroups per CU; 0 = as many as fit          */
    int32_t order;          /* 0: regions in the order given; 1: most haplotypes first   */
    int32_t small_kernel;   /* 1: regions of <= 1,024 haplotypes in the walk use the
                               bitmask kernel; 0: the persistent launch takes them too  */
    int32_t kernel;         /* 0: class ids per haplotype with a pairwise tail, one item
                               per (site, direction) [default]; 1: per-core walks over
                               sorted member lists, one item per (site, direction, core) */
    int32_t small_pair_cap; /* kernel 0: pair capacity of the launches of 64 or 128
                               threads (regions of up to 2048 haplotypes in the walk),
                               whose occupancy the pair buffers would halve; 0..16384    */
    int32_t slots;          /* kernel 0: 64-haplotype words per wave (4, 8 or 16
                               [default]): fewer words per wave spread a walk over more
                               waves; rows wider than 16 waves of them take 16 per wave */
    int32_t class_cap;      /* kernel 0: classes the LDS table holds (0 = as many as a
                               walk can have, n/2 + 2; else 64..16386, default 256):
                               walks that outgrow it are redone by a second launch with
                               full tables                                             */
    int32_t counter_copies; /* kernel 0: copies of each class counter, over which the
                               members of one class spread their LDS atomics (1 or 8;
                               0 = 8 for workgroups of 256 threads or more, else 1)    */
} ss_batch_config;

int ss_get_batch_config(ss_batch_config *c);
/* Errors: SS_EARG for a field out of range.  Also drops the per-group
 * settings the autotuner found (ss_get_group_tuning). */
int ss_set_batch_config(const ss_batch_config *c);

/*
 * ss_get_group_tuning -- the settings ss_autotune_batch refined for single
 * launch groups of kernel 0 (a group: the regions of one workgroup size, with
 * or without pair buffers).  They replace the process-wide counter_copies,
 * class_cap, chunk and blocks_per_cu for launches of that group, or (plain =
 * 1) walk the group's regions with the plain per-locus class-id kernel
 * instead, in batches and in single scans taken by the persistent walk.
 * rows: host int32 array of 7 * max_rows, filled with {threads, pair buffers
 * (0/1), counter_copies, class_cap, chunk, blocks_per_cu, plain (0/1)} per
 * group; *n_rows: the number of groups with refined settings (may exceed
 * max_rows; the rest are not written).  Host only.
 * Errors: SS_EARG for a null n_rows, or null rows with max_rows > 0.
 */
int ss_get_group_tuning(int32_t *rows, int32_t max_rows, int32_t *n_rows);

/*
 * ss_set_group_tuning -- replace the per-group settings by n_rows rows of
 * the layout ss_get_group_tuning fills (host int32, 7 * n_rows; n_rows = 0
 * drops them all).  The plain kernel is used for a group only where every
 * region's class table fits in LDS.  Host only.  Errors: SS_EARG for a null
 * rows with n_rows > 0 or a field out of range (nothing is changed then).
 */
int ss_set_group_tuning(const int32_t *rows, int32_t n_rows);

/*
 * ss_autotune_batch -- time candidate configurations of the persistent walk on
 * these requests (the walks of about sample_items work items per launch group,
 * spread evenly over its sites, or all if sample_items <= 0), keep the fastest
 * as the process-wide configuration and return it with its time.  With several
 * launch groups it then refines counter_copies, class_cap, chunk and
 * blocks_per_cu for each group on its own (kept if the whole batch is then at
 * least as fast; see ss_get_group_tuning).  Blocks until the timings are done; the outputs of
 * the requests are left undefined (run ss_scan_batch afterwards).
 * Errors: as ss_scan_batch.
 */
int ss_autotune_batch(const ss_scan_request *reqs, int32_t n_reqs, const ss_params *p,
                      void *d_ws, size_t ws_bytes, void *stream, int64_t sample_items,
                      ss_batch_config *best, double *best_ms);

/* Graph capture of ss_scan_batch on (1) or off (0, default); ss_graph_clear
 * destroys the cached graphs (call before freeing buffers they use). */
int ss_set_graph(int on);
int ss_graph_clear(void);

/*
 * ss_set_mask_skip -- tuning of the bitmask walk (process-wide): a batch of
 * 64 markers that starts with at most max_classes live classes (0 .. 64;
 * default 32) first tests every marker against every class at once, and
 * refines only the markers that cut a class (the others change no class and
 * no sum); 0 refines every marker.  Results are identical for every setting.
 * Errors: SS_EARG outside [0, 64].
 */
int ss_set_mask_skip(int max_classes);

/*
 * ss_set_mask_lanes -- tuning of the bitmask walk kernel (process-wide):
 * how many lanes of a wave hold one class (1, 2, 4 or 8; each lane holds
 * words_per_class / lanes of its mask), or 0 for the default (1 lane up to
 * 8 words a class, 2 lanes for the 16-word masks of 513-1,024 haplotypes,
 * which take 2 or 4).  More lanes per class cut the per-marker work when few
 * classes are alive; fewer lanes fit more classes in one row; inputs a
 * setting does not fit use class ids.  Results are identical for every
 * setting.
 * Errors: SS_EARG for any other value.
 */
int ss_set_mask_lanes(int lanes_per_class);

/*
 * Kernel timing for measurement: while enabled, ss_ihs / ss_xpehh record HIP
 * events on their stream around the EHH walk kernel; ss_timing_read() waits
 * for the recorded events and returns the summed walk-kernel time (ms) and
 * the number of launches since the last reset.
 */
int ss_timing_enable(int on);
int ss_timing_read(double *walk_ms_total, int64_t *walk_launches, int reset);

#ifdef __cplusplus
}
#endif

#endif /* SELSCAN_HIP_H */

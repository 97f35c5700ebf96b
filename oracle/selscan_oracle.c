/*
 * selscan_oracle.c -- plain, slow FP64 CPU oracle for EHH, iHS and XPEHH.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the yardstick the GPU library is
 * checked against; it shares no code, header, table or helper with the GPU
 * path and must never be linked into, imported by or called from the
 * product.  Only the tests, the smoke check and the benchmark's CPU-baseline
 * leg use it.
 *
 * Everything here is the paper's definitions written out one marker at a
 * time (Szpiech & Hernandez, "selscan", arXiv:1403.6854):
 *   - haplotypes are strings of 0/1 alleles, 0 ancestral and 1 derived, and
 *     the core site x0 is part of the string (Sec. 1.1, the example with
 *     C = {0,1} and C(x1) = {11,10,00,01});
 *   - whole-sample EHH is sum_h C(n_h,2)/C(n,2) over the distinct haplotypes
 *     from x0 out to x_i (Sec. 1.1, Eq. 1); core EHH_c restricts the sum to
 *     the haplotypes that carry allele c at x0 and divides by C(n_c,2)
 *     (Sec. 1.1, Eqs. 2-3);
 *   - iHH is the trapezoid sum of 1/2 (EHH(x_{i-1}) + EHH(x_i)) g(x_{i-1},x_i)
 *     over the downstream markers plus the same sum over the upstream markers
 *     (Sec. 1.2, Eq. 4; Sec. 1.3, Eq. 7);
 *   - unstandardized iHS = ln(iHH_1/iHH_0) (Sec. 1.2, Eq. 5) and XPEHH =
 *     ln(iHH_A/iHH_B) (Sec. 1.3, Eq. 8);
 *   - the practical rules of Sec. 1.2: sums truncated once EHH drops below
 *     the cutoff, gaps b > 20 kb scale g by 20/b, reaching the end of the
 *     data or crossing a gap b > 200 kb aborts the locus, core sites with
 *     MAF < cutoff are not scored; for XPEHH the truncation point is where
 *     the EHH of the two populations pooled drops below the cutoff (Sec. 1.3);
 *   - standardization within derived-allele-frequency bins for iHS (Eq. 6)
 *     and genome-wide for XPEHH (Eq. 9).
 *
 * Readings taken where the paper is silent (each one is listed with its
 * reason in the design notes of this repository):
 *   R1  the term ending at the first marker with EHH < cutoff is not added;
 *   R2  the cutoff test is (double)S/(double)P < cutoff, IEEE division;
 *   R3  g is scaled iff the gap is strictly larger than gap_scale_bp, by the
 *       factor (double)gap_scale_bp/(double)gap;
 *   R4  the abort test covers every segment the walk crosses while any
 *       tracked statistic is still at or above the cutoff, including the
 *       segment to the marker where it stops; strict ">" max_gap_bp;
 *   R5  for iHS the locus aborts if the end is reached in either direction
 *       while either core is still at or above the cutoff;
 *   R7  XPEHH starts each population's curve at its whole-sample EHH at x0,
 *       [C(n0,2)+C(n1,2)]/C(n,2), because x0 is part of the haplotype;
 *   R9  MAF = min(n0,n1)/n in double; a site is filtered iff MAF < cutoff;
 *   R10 frequency bin = min(floor(B*n1/n), B-1), B = round(1/bin_width),
 *       in integer arithmetic on the derived count n1;
 *   R11 standard deviation uses N-1; bins with N < 2 or SD = 0 give NaN;
 *   R14 a core with fewer than 2 haplotypes, or an iHH equal to 0, leaves
 *       the score undefined;
 *   R15 iHH = (downstream sum) + (upstream sum), each accumulated from x0
 *       outward; the per-direction locus status is the downstream abort if
 *       any, else the upstream one;
 *   R16 with the physical-map option the segment length g is the physical
 *       distance b in base pairs, and the gap rules apply to it unchanged
 *       (a scaled segment then counts gap_scale_bp base pairs).
 *
 * Build:  gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double ehh_cutoff;     /* EHH truncation value; paper default 0.05       */
    double maf_cutoff;     /* core-site MAF cutoff; paper default 0.05       */
    int64_t gap_scale_bp;  /* gaps above this scale g; paper default 20 kb   */
    int64_t max_gap_bp;    /* gaps above this abort; paper default 200 kb    */
    double bin_width;      /* iHS frequency-bin width; 0.025 here            */
    int32_t physical_map;  /* 1: integrate over physical distance in bp      */
} or_params;

enum { OR_OK = 0, OR_MAF = 1, OR_EDGE = 2, OR_GAP = 3, OR_UNDEF = 4,
       OR_BIN = 5, OR_CAP = 6 };

static int64_t choose2(int64_t x) { return x * (x - 1) / 2; }

/* ---------------------------------------------------------------------- */
/* Partition of the haplotypes into distinct strings on [x0, x_k].          */
/* ---------------------------------------------------------------------- */
typedef struct {
    int64_t n;        /* haplotypes in the walk                             */
    int64_t nA;       /* the first nA belong to population A, the rest to B */
    int *lab;         /* class label of every haplotype                     */
    int *nxt;         /* labels after the next marker                       */
    int *child;       /* (old label, allele) -> new label, 2 per old label  */
    int64_t *cntA;    /* class sizes in population A                        */
    int64_t *cntB;    /* class sizes in population B                        */
    int *core;        /* allele at x0 shared by the members of each class   */
    int *newcore;     /* scratch for core[] while splitting                 */
    int nlab;         /* number of classes                                  */
} partition;

static int part_init(partition *pt, int64_t n, int64_t nA) {
    pt->n = n; pt->nA = nA; pt->nlab = 0;
    pt->lab = (int *)malloc(sizeof(int) * (size_t)n);
    pt->nxt = (int *)malloc(sizeof(int) * (size_t)n);
    pt->child = (int *)malloc(sizeof(int) * (size_t)(2 * n + 2));
    pt->cntA = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    pt->cntB = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    pt->core = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    pt->newcore = (int *)malloc(sizeof(int) * (size_t)(2 * n + 2));
    return pt->lab && pt->nxt && pt->child && pt->cntA && pt->cntB && pt->core &&
           pt->newcore;
}

static void part_free(partition *pt) {
    free(pt->lab); free(pt->nxt); free(pt->child);
    free(pt->cntA); free(pt->cntB); free(pt->core); free(pt->newcore);
}

static void part_count(partition *pt) {
    for (int c = 0; c < pt->nlab; ++c) { pt->cntA[c] = 0; pt->cntB[c] = 0; }
    for (int64_t h = 0; h < pt->n; ++h) {
        if (h < pt->nA) pt->cntA[pt->lab[h]] += 1;
        else            pt->cntB[pt->lab[h]] += 1;
    }
}

/* Classes at x0: one per allele (label = allele). */
static void part_start(partition *pt, const uint8_t *row) {
    for (int64_t h = 0; h < pt->n; ++h) pt->lab[h] = row[h] ? 1 : 0;
    pt->nlab = 2;
    pt->core[0] = 0; pt->core[1] = 1;
    part_count(pt);
}

/* Split every class by the allele each member carries at the next marker. */
static void part_refine(partition *pt, const uint8_t *row) {
    for (int i = 0; i < 2 * pt->nlab; ++i) pt->child[i] = -1;
    int made = 0;
    int *newcore = pt->newcore;
    for (int64_t h = 0; h < pt->n; ++h) {
        int key = 2 * pt->lab[h] + (row[h] ? 1 : 0);
        if (pt->child[key] < 0) {
            newcore[made] = pt->core[pt->lab[h]];
            pt->child[key] = made++;
        }
        pt->nxt[h] = pt->child[key];
    }
    int *t = pt->lab; pt->lab = pt->nxt; pt->nxt = t;
    pt->nlab = made;
    for (int c = 0; c < made; ++c) pt->core[c] = newcore[c];
    part_count(pt);
}

/* Row k of the pooled walk: A's alleles then B's. */
static void pooled_row(const uint8_t *HA, int64_t nA, const uint8_t *HB, int64_t nB,
                       int64_t k, uint8_t *row) {
    memcpy(row, HA + k * nA, (size_t)nA);
    if (nB > 0) memcpy(row + nA, HB + k * nB, (size_t)nB);
}

/* Physical gap and (scaled) length of the segment crossed when the walk
 * moves from marker k-dir to marker k, on the genetic map or, with the
 * physical-map option, in base pairs (the map rehh integrates over, which the
 * paper's Sec. 2.1 compares against); the gap rules are the same for both.
 * Returns 0 to go on, or OR_GAP. */
static int segment(const int64_t *pos, const double *gpos, int64_t k, int dir,
                   const or_params *p, double *g_out) {
    int64_t lo = dir > 0 ? k - 1 : k;
    int64_t hi = lo + 1;
    int64_t b = pos[hi] - pos[lo];
    if (b > p->max_gap_bp) return OR_GAP;
    double g = p->physical_map ? (double)b : gpos[hi] - gpos[lo];
    if (b > p->gap_scale_bp) g = g * ((double)p->gap_scale_bp / (double)b);
    *g_out = g;
    return 0;
}

/* ---------------------------------------------------------------------- */
/* One direction of the core-EHH walk used by iHS and EHH.                  */
/* trace (may be NULL): per step, S_0 and S_1 and the class sizes.          */
/* ---------------------------------------------------------------------- */
typedef struct {
    int64_t cap;        /* maximum steps recorded                          */
    uint64_t *S;        /* [cap+1][2]                                      */
    uint32_t *sizes;    /* [cap+1][n] or NULL                              */
    int64_t len;        /* steps taken                                     */
    int capped;
} core_trace;

static int core_walk(const uint8_t *H, int64_t n, int64_t M, const int64_t *pos,
                     const double *gpos, int64_t j, int dir, const or_params *p,
                     partition *pt, double ihh[2], int64_t steps[2], core_trace *tr) {
    int64_t nc[2] = {0, 0};
    for (int64_t h = 0; h < n; ++h) nc[H[j * n + h] ? 1 : 0] += 1;
    double P[2] = {(double)choose2(nc[0]), (double)choose2(nc[1])};
    int active[2] = {nc[0] >= 2, nc[1] >= 2};
    double eprev[2] = {1.0, 1.0};
    ihh[0] = ihh[1] = 0.0;
    steps[0] = steps[1] = 0;
    pt->nA = n;
    part_start(pt, H + j * n);
    if (tr) {
        tr->len = 0; tr->capped = 0;
        for (int c = 0; c < 2; ++c) {
            uint64_t s = 0;
            for (int l = 0; l < pt->nlab; ++l)
                if (pt->core[l] == c) s += (uint64_t)choose2(pt->cntA[l]);
            tr->S[c] = s;
        }
        if (tr->sizes) {
            int q = 0;
            memset(tr->sizes, 0, sizeof(uint32_t) * (size_t)n);
            for (int l = 0; l < pt->nlab; ++l)
                if (pt->cntA[l] >= 2)
                    tr->sizes[q++] = (uint32_t)pt->cntA[l] | ((uint32_t)pt->core[l] << 31);
        }
    }
    int64_t k = j;
    while (active[0] || active[1]) {
        k += dir;
        if (k < 0 || k >= M) return OR_EDGE;
        double g;
        if (segment(pos, gpos, k, dir, p, &g)) return OR_GAP;
        if (tr && tr->len >= tr->cap) { tr->capped = 1; return OR_CAP; }
        part_refine(pt, H + k * n);
        uint64_t S[2] = {0, 0};
        for (int l = 0; l < pt->nlab; ++l)
            S[pt->core[l]] += (uint64_t)choose2(pt->cntA[l]);
        if (tr) {
            tr->len += 1;
            tr->S[2 * tr->len + 0] = S[0];
            tr->S[2 * tr->len + 1] = S[1];
            if (tr->sizes) {
                uint32_t *z = tr->sizes + tr->len * n;
                int q = 0;
                memset(z, 0, sizeof(uint32_t) * (size_t)n);
                for (int l = 0; l < pt->nlab; ++l)
                    if (pt->cntA[l] >= 2)
                        z[q++] = (uint32_t)pt->cntA[l] | ((uint32_t)pt->core[l] << 31);
            }
        }
        for (int c = 0; c < 2; ++c) {
            if (!active[c]) continue;
            steps[c] += 1;
            double e = (double)S[c] / P[c];
            if (e < p->ehh_cutoff) {
                active[c] = 0;
            } else {
                ihh[c] += 0.5 * (eprev[c] + e) * g;
                eprev[c] = e;
            }
        }
    }
    return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* One direction of the pooled walk used by XPEHH.                          */
/* ---------------------------------------------------------------------- */
typedef struct {
    int64_t cap;
    uint64_t *S;        /* [cap+1][3]: S_A, S_B, S_pool                     */
    int64_t len;
    int capped;
} pool_trace;

static int pooled_walk(const uint8_t *HA, int64_t nA, const uint8_t *HB, int64_t nB,
                       int64_t M, const int64_t *pos, const double *gpos, int64_t j,
                       int dir, const or_params *p, partition *pt, uint8_t *row,
                       double ihh[2], int64_t *steps, pool_trace *tr) {
    int64_t n = nA + nB;
    double PA = (double)choose2(nA), PB = (double)choose2(nB), PP = (double)choose2(n);
    pooled_row(HA, nA, HB, nB, j, row);
    pt->nA = nA;
    part_start(pt, row);
    uint64_t SA = 0, SB = 0, SP = 0;
    for (int l = 0; l < pt->nlab; ++l) {
        SA += (uint64_t)choose2(pt->cntA[l]);
        SB += (uint64_t)choose2(pt->cntB[l]);
        SP += (uint64_t)choose2(pt->cntA[l] + pt->cntB[l]);
    }
    double eprevA = (double)SA / PA, eprevB = (double)SB / PB;
    ihh[0] = ihh[1] = 0.0;
    *steps = 0;
    if (tr) {
        tr->len = 0; tr->capped = 0;
        tr->S[0] = SA; tr->S[1] = SB; tr->S[2] = SP;
    }
    int64_t k = j;
    for (;;) {
        k += dir;
        if (k < 0 || k >= M) return OR_EDGE;
        double g;
        if (segment(pos, gpos, k, dir, p, &g)) return OR_GAP;
        if (tr && tr->len >= tr->cap) { tr->capped = 1; return OR_CAP; }
        pooled_row(HA, nA, HB, nB, k, row);
        part_refine(pt, row);
        SA = SB = SP = 0;
        for (int l = 0; l < pt->nlab; ++l) {
            SA += (uint64_t)choose2(pt->cntA[l]);
            SB += (uint64_t)choose2(pt->cntB[l]);
            SP += (uint64_t)choose2(pt->cntA[l] + pt->cntB[l]);
        }
        if (tr) {
            tr->len += 1;
            tr->S[3 * tr->len + 0] = SA;
            tr->S[3 * tr->len + 1] = SB;
            tr->S[3 * tr->len + 2] = SP;
        }
        *steps += 1;
        if ((double)SP / PP < p->ehh_cutoff) return OR_OK;
        double eA = (double)SA / PA, eB = (double)SB / PB;
        ihh[0] += 0.5 * (eprevA + eA) * g;
        ihh[1] += 0.5 * (eprevB + eB) * g;
        eprevA = eA; eprevB = eB;
    }
}

/* ---------------------------------------------------------------------- */
/* Standardization (Eq. 6 / Eq. 9): z = (u - mean_bin) / sd_bin over the    */
/* loci with status OK, visited in ascending site order.                    */
/* ---------------------------------------------------------------------- */
int or_standardize(const double *u, int8_t *status, const int32_t *bin, int64_t M,
                   int nbins, double *z, double *bin_mean, double *bin_sd,
                   int64_t *bin_n) {
    for (int64_t j = 0; j < M; ++j) z[j] = NAN;
    for (int b = 0; b < nbins; ++b) {
        int64_t N = 0;
        double sum = 0.0;
        for (int64_t j = 0; j < M; ++j)
            if (status[j] == OR_OK && bin[j] == b) { sum += u[j]; N += 1; }
        double mean = N > 0 ? sum / (double)N : NAN;
        double ss = 0.0;
        for (int64_t j = 0; j < M; ++j)
            if (status[j] == OR_OK && bin[j] == b) { double d = u[j] - mean; ss += d * d; }
        double sd = N > 1 ? sqrt(ss / (double)(N - 1)) : NAN;
        if (bin_mean) bin_mean[b] = mean;
        if (bin_sd) bin_sd[b] = sd;
        if (bin_n) bin_n[b] = N;
        /* a locus belongs to exactly one bin, so relabelling this bin's loci
           cannot change any other bin's statistics */
        for (int64_t j = 0; j < M; ++j) {
            if (status[j] != OR_OK || bin[j] != b) continue;
            if (N >= 2 && sd > 0.0) z[j] = (u[j] - mean) / sd;
            else status[j] = OR_BIN;
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* iHS over all sites (loci == NULL) or over a list of sites.               */
/* steps (may be NULL): [M][2 directions][2 cores] markers walked per core,  */
/* including the marker where the core stopped (direction 0 = downstream).  */
/* ---------------------------------------------------------------------- */
int or_ihs(const uint8_t *H, int64_t n, int64_t M, const int64_t *pos, const double *gpos,
           const or_params *p, const int64_t *loci, int64_t n_loci,
           double *ihh1, double *ihh0, double *unstd, double *stdz, double *freq,
           int8_t *status, int32_t *bin, int64_t *steps, int nthreads) {
    if (n < 2 || M < 1) return -1;
    int64_t L = loci ? n_loci : M;
    int B = (int)floor(1.0 / p->bin_width + 0.5);
    if (B < 1) B = 1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int failed = 0;
#pragma omp parallel
    {
        partition pt;
        if (!part_init(&pt, n, n)) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 8)
        for (int64_t t = 0; t < L; ++t) {
            if (failed) continue;
            int64_t j = loci ? loci[t] : t;
            int64_t n1 = 0;
            for (int64_t h = 0; h < n; ++h) n1 += H[j * n + h] ? 1 : 0;
            int64_t n0 = n - n1;
            freq[j] = (double)n1 / (double)n;
            int64_t bb = ((int64_t)B * n1) / n;
            bin[j] = (int32_t)(bb > B - 1 ? B - 1 : bb);
            ihh1[j] = ihh0[j] = unstd[j] = stdz[j] = NAN;
            if (steps) for (int q = 0; q < 4; ++q) steps[4 * j + q] = 0;
            double maf = (double)(n0 < n1 ? n0 : n1) / (double)n;
            if (maf < p->maf_cutoff) { status[j] = OR_MAF; continue; }
            if (n0 < 2 || n1 < 2) { status[j] = OR_UNDEF; continue; }
            double dn[2], up[2];
            int64_t sd[2], su[2];
            int s_dn = core_walk(H, n, M, pos, gpos, j, +1, p, &pt, dn, sd, NULL);
            int s_up = core_walk(H, n, M, pos, gpos, j, -1, p, &pt, up, su, NULL);
            if (steps) {
                steps[4 * j + 0] = sd[0]; steps[4 * j + 1] = sd[1];
                steps[4 * j + 2] = su[0]; steps[4 * j + 3] = su[1];
            }
            int st = s_dn != OR_OK ? s_dn : s_up;
            if (st != OR_OK) { status[j] = (int8_t)st; continue; }
            double i0 = dn[0] + up[0];
            double i1 = dn[1] + up[1];
            if (!(i0 > 0.0) || !(i1 > 0.0)) { status[j] = OR_UNDEF; continue; }
            ihh0[j] = i0; ihh1[j] = i1;
            unstd[j] = log(i1 / i0);
            status[j] = OR_OK;
        }
        part_free(&pt);
    }
    if (failed) return -2;
    if (!loci) or_standardize(unstd, status, bin, M, B, stdz, NULL, NULL, NULL);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* XPEHH over all sites (loci == NULL) or a list of sites.                  */
/* steps (may be NULL): [M][2 directions] pooled markers walked.            */
/* ---------------------------------------------------------------------- */
int or_xpehh(const uint8_t *HA, int64_t nA, const uint8_t *HB, int64_t nB, int64_t M,
             const int64_t *pos, const double *gpos, const or_params *p,
             const int64_t *loci, int64_t n_loci, double *ihhA, double *ihhB,
             double *unstd, double *stdz, int8_t *status, int64_t *steps, int nthreads) {
    if (nA < 2 || nB < 2 || M < 1) return -1;
    int64_t L = loci ? n_loci : M;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int failed = 0;
#pragma omp parallel
    {
        partition pt;
        uint8_t *row = (uint8_t *)malloc((size_t)(nA + nB));
        if (!part_init(&pt, nA + nB, nA) || !row) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 8)
        for (int64_t t = 0; t < L; ++t) {
            if (failed) continue;
            int64_t j = loci ? loci[t] : t;
            ihhA[j] = ihhB[j] = unstd[j] = stdz[j] = NAN;
            double dn[2], up[2];
            int64_t sd, su;
            int s_dn = pooled_walk(HA, nA, HB, nB, M, pos, gpos, j, +1, p, &pt, row, dn, &sd, NULL);
            int s_up = pooled_walk(HA, nA, HB, nB, M, pos, gpos, j, -1, p, &pt, row, up, &su, NULL);
            if (steps) { steps[2 * j + 0] = sd; steps[2 * j + 1] = su; }
            int st = s_dn != OR_OK ? s_dn : s_up;
            if (st != OR_OK) { status[j] = (int8_t)st; continue; }
            double a = dn[0] + up[0];
            double b = dn[1] + up[1];
            if (!(a > 0.0) || !(b > 0.0)) { status[j] = OR_UNDEF; continue; }
            ihhA[j] = a; ihhB[j] = b;
            unstd[j] = log(a / b);
            status[j] = OR_OK;
        }
        part_free(&pt);
        free(row);
    }
    if (failed) return -2;
    if (!loci) {
        int32_t *bin = (int32_t *)calloc((size_t)M, sizeof(int32_t));
        double bm, bs;
        int64_t bn;
        or_standardize(unstd, status, bin, M, 1, stdz, &bm, &bs, &bn);
        free(bin);
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* EHH at one core site, both directions, with per-marker traces.           */
/* S: [2 dirs][cap+1][2]; ehh: [2 dirs][cap+1][3] = EHH_0, EHH_1, EHH_all;   */
/* len: [2]; sizes: [2 dirs][cap+1][n] or NULL; ihh: [2] = iHH_0, iHH_1.     */
/* The MAF cutoff does not apply (EHH is defined at every site).            */
/* ---------------------------------------------------------------------- */
int or_ehh(const uint8_t *H, int64_t n, int64_t M, const int64_t *pos, const double *gpos,
           const or_params *p, int64_t core, int64_t cap, uint64_t *S, double *ehh,
           int64_t *len, uint32_t *sizes, double *ihh, int8_t *status) {
    if (n < 2 || core < 0 || core >= M || cap < 1) return -1;
    partition pt;
    if (!part_init(&pt, n, n)) return -2;
    int64_t nc[2] = {0, 0};
    for (int64_t h = 0; h < n; ++h) nc[H[core * n + h] ? 1 : 0] += 1;
    double P0 = (double)choose2(nc[0]), P1 = (double)choose2(nc[1]);
    double Pall = (double)choose2(n);
    int st[2];
    double hh[2][2];
    for (int d = 0; d < 2; ++d) {
        core_trace tr;
        tr.cap = cap;
        tr.S = S + (size_t)d * (size_t)(cap + 1) * 2;
        tr.sizes = sizes ? sizes + (size_t)d * (size_t)(cap + 1) * (size_t)n : NULL;
        memset(tr.S, 0, sizeof(uint64_t) * (size_t)(cap + 1) * 2);
        if (tr.sizes) memset(tr.sizes, 0, sizeof(uint32_t) * (size_t)(cap + 1) * (size_t)n);
        int64_t stp[2];
        st[d] = core_walk(H, n, M, pos, gpos, core, d == 0 ? +1 : -1, p, &pt, hh[d], stp, &tr);
        len[d] = tr.len;
        double *e = ehh + (size_t)d * (size_t)(cap + 1) * 3;
        for (int64_t i = 0; i <= cap; ++i) {
            if (i <= tr.len) {
                e[3 * i + 0] = (double)tr.S[2 * i + 0] / P0;
                e[3 * i + 1] = (double)tr.S[2 * i + 1] / P1;
                e[3 * i + 2] = (double)(tr.S[2 * i + 0] + tr.S[2 * i + 1]) / Pall;
            } else {
                e[3 * i + 0] = e[3 * i + 1] = e[3 * i + 2] = NAN;
            }
        }
    }
    part_free(&pt);
    int s = st[0] != OR_OK ? st[0] : st[1];
    if (s == OR_OK && (nc[0] < 2 || nc[1] < 2)) s = OR_UNDEF;
    ihh[0] = ihh[1] = NAN;
    if (s == OR_OK) {
        double i0 = hh[0][0] + hh[1][0];
        double i1 = hh[0][1] + hh[1][1];
        if (!(i0 > 0.0) || !(i1 > 0.0)) s = OR_UNDEF;
        else { ihh[0] = i0; ihh[1] = i1; }
    }
    *status = (int8_t)s;
    return 0;
}

/* XPEHH trace at one site: S: [2 dirs][cap+1][3] = S_A, S_B, S_pool. */
int or_xpehh_trace(const uint8_t *HA, int64_t nA, const uint8_t *HB, int64_t nB, int64_t M,
                   const int64_t *pos, const double *gpos, const or_params *p, int64_t site,
                   int64_t cap, uint64_t *S, int64_t *len, double *ihh, int8_t *status) {
    if (nA < 2 || nB < 2 || site < 0 || site >= M || cap < 1) return -1;
    partition pt;
    uint8_t *row = (uint8_t *)malloc((size_t)(nA + nB));
    if (!part_init(&pt, nA + nB, nA) || !row) return -2;
    int st[2];
    double hh[2][2];
    for (int d = 0; d < 2; ++d) {
        pool_trace tr;
        tr.cap = cap;
        tr.S = S + (size_t)d * (size_t)(cap + 1) * 3;
        memset(tr.S, 0, sizeof(uint64_t) * (size_t)(cap + 1) * 3);
        int64_t stp;
        st[d] = pooled_walk(HA, nA, HB, nB, M, pos, gpos, site, d == 0 ? +1 : -1, p, &pt,
                            row, hh[d], &stp, &tr);
        len[d] = tr.len;
    }
    part_free(&pt);
    free(row);
    int s = st[0] != OR_OK ? st[0] : st[1];
    ihh[0] = ihh[1] = NAN;
    if (s == OR_OK) {
        double i0 = hh[0][0] + hh[1][0];
        double i1 = hh[0][1] + hh[1][1];
        if (!(i0 > 0.0) || !(i1 > 0.0)) s = OR_UNDEF;
        else { ihh[0] = i0; ihh[1] = i1; }
    }
    *status = (int8_t)s;
    return 0;
}

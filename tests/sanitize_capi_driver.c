/*
 * Calls the C ABI's argument checks -- every call below fails them or sizes a
 * workspace, before any device work -- for a host build of the library with
 * AddressSanitizer and UndefinedBehaviorSanitizer.  No GPU is needed.  Test
 * infrastructure only (tests/test_sanitizers.py).
 */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "selscan_hip.h"
#include "selscan_micro.h"

#define EXPECT(cond)                                                          \
    do {                                                                      \
        if (!(cond)) {                                                        \
            fprintf(stderr, "failed at line %d: %s\n", __LINE__, #cond);      \
            return 1;                                                         \
        }                                                                     \
    } while (0)

int main(void) {
    void *x = (void *)0x1000;   /* never dereferenced: the checks fail first */
    ss_params p;
    ss_default_params(&p);
    ss_hapmat h = {(const uint64_t *)x, 204, 22147, 4, (const int64_t *)x, (const double *)x};
    size_t ws = ss_workspace_bytes(SS_OP_IHS, &h, NULL, &p, 0);
    EXPECT(ws > 0);
    EXPECT(ss_workspace_bytes(SS_OP_XPEHH, &h, NULL, &p, 0) == 0);
    /* workspace sizes over many shapes */
    for (int64_t n = 2; n <= 32767; n = n * 3 + 1)
        for (int64_t m = 1; m <= 1 << 22; m = m * 7 + 3) {
            ss_hapmat a = h;
            a.n_haps = n;
            a.n_sites = m;
            a.words_per_site = (n + 63) / 64;
            EXPECT(ss_workspace_bytes(SS_OP_IHS, &a, NULL, &p, 0) > 0);
            EXPECT(ss_workspace_bytes(SS_OP_XPEHH, &a, &a, &p, 0) > 0);
        }
    double *d = (double *)x;
    int8_t *st = (int8_t *)x;
    /* invalid arguments of the scans */
    EXPECT(ss_ihs(NULL, &p, d, d, d, d, d, st, NULL, x, ws, NULL) == SS_EARG);
    EXPECT(ss_ihs(&h, NULL, d, d, d, d, d, st, NULL, x, ws, NULL) == SS_EARG);
    EXPECT(ss_ihs(&h, &p, NULL, d, d, d, d, st, NULL, x, ws, NULL) == SS_EARG);
    EXPECT(ss_ihs(&h, &p, d, d, d, d, d, st, NULL, x, ws - 1, NULL) == SS_EWS);
    EXPECT(strlen(ss_last_error()) > 0);
    ss_params bad = p;
    bad.ehh_cutoff = 0.0;
    EXPECT(ss_ihs(&h, &bad, d, d, d, d, d, st, NULL, x, ws, NULL) == SS_EARG);
    bad = p;
    bad.physical_map = 3;
    EXPECT(ss_ihs(&h, &bad, d, d, d, d, d, st, NULL, x, ws, NULL) == SS_EARG);
    bad = p;
    bad.bin_width = 1e-9;
    EXPECT(ss_ihs(&h, &bad, d, d, d, d, d, st, NULL, x, ws, NULL) == SS_EARG);
    ss_hapmat b = h;
    b.n_sites = 10;
    EXPECT(ss_xpehh(&h, &b, &p, d, d, d, d, st, NULL, x, 1 << 30, NULL) == SS_ESHAPE);
    EXPECT(ss_ehh(&h, -1, &p, 16, (uint64_t *)x, d, (int64_t *)x, NULL, d, st, x, 512, NULL) == SS_EARG);
    EXPECT(ss_ehh(&h, 0, &p, 0, (uint64_t *)x, d, (int64_t *)x, NULL, d, st, x, 512, NULL) == SS_EARG);
    EXPECT(ss_pack(NULL, 10, 10, 1, (uint64_t *)x, NULL) == SS_EARG);
    /* the static-scratch entry point refuses a scan larger than its array */
    ss_hapmat big = h;
    big.n_haps = 1000;
    big.n_sites = 300000;
    big.words_per_site = 16;
    EXPECT(ss_ihs_static(&big, &p, d, d, d, d, d, st, NULL, NULL) == SS_EWS);
    /* batches */
    ss_scan_request rq[300];
    memset(rq, 0, sizeof(rq));
    for (int i = 0; i < 300; ++i) {
        rq[i].op = i % 3 ? SS_OP_IHS : SS_OP_XPEHH;
        rq[i].a = h;
        rq[i].a.n_haps = 2 + (i * 37) % 3000;
        rq[i].a.words_per_site = (rq[i].a.n_haps + 63) / 64;
        rq[i].a.n_sites = 1 + (i * 101) % 50000;
        rq[i].b = rq[i].a;
        rq[i].d_ihh_x = rq[i].d_ihh_y = rq[i].d_unstd = rq[i].d_std = rq[i].d_freq = d;
        rq[i].d_status = st;
    }
    size_t bws = ss_batch_workspace_bytes(rq, 300, &p);
    EXPECT(bws > 0);
    EXPECT(ss_scan_batch(rq, 300, &p, x, bws - 1, NULL) == SS_EWS);
    rq[150].op = 7;
    EXPECT(ss_batch_workspace_bytes(rq, 300, &p) == 0);
    EXPECT(ss_scan_batch(rq, 0, &p, x, bws, NULL) == SS_EARG);
    ss_batch_config c;
    EXPECT(ss_get_batch_config(&c) == SS_OK);
    ss_batch_config cb = c;
    cb.threads = 100;
    EXPECT(ss_set_batch_config(&cb) == SS_EARG);
    int32_t rows[7 * 4];
    int32_t nrows = -1;
    EXPECT(ss_get_group_tuning(rows, 4, &nrows) == SS_OK && nrows == 0);
    int32_t badrow[7] = {64, 1, 3, 1024, 1, 0, 0};
    EXPECT(ss_set_group_tuning(badrow, 1) == SS_EARG);
    /* genome-wide standardization */
    ss_std_region g[3];
    for (int i = 0; i < 3; ++i) {
        g[i].d_unstd = d;
        g[i].d_freq = d;
        g[i].d_status = st;
        g[i].d_std = d;
        g[i].n_sites = 1000 * (i + 1);
        g[i].n_haps = 204;
        g[i].reserved = 0;
    }
    size_t gws = ss_genome_workspace_bytes(g, 3, SS_OP_IHS, &p);
    EXPECT(gws > 0);
    EXPECT(ss_genome_standardize(g, 3, SS_OP_IHS, &p, NULL, x, gws - 1, NULL) == SS_EWS);
    g[1].d_freq = NULL;
    EXPECT(ss_genome_standardize(g, 3, SS_OP_IHS, &p, NULL, x, gws, NULL) == SS_EARG);
    EXPECT(ss_genome_workspace_bytes(g, 3, SS_OP_XPEHH, &p) > 0);
    /* tuning setters */
    EXPECT(ss_set_walk_kernel(9) == SS_EARG);
    EXPECT(ss_set_mask_lanes(3) == SS_EARG);
    EXPECT(ss_set_mask_skip(65) == SS_EARG);
    /* measurement kernels */
    double ms = 0.0, ops = 0.0;
    EXPECT(ss_micro_copy(NULL, x, 4096, 1, NULL, &ms) == SS_EARG);
    EXPECT(ss_micro_valu(NULL, 4, 1, NULL, &ms, &ops) == SS_EARG);
    printf("sanitized host checks passed\n");
    return 0;
}

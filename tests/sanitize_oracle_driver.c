/*
 * Runs the CPU oracle's entry points on small random inputs (all sizes and
 * core sites, the edge cases of a tiny region), for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer: any out-of-bounds access,
 * leak, overflow or undefined shift is reported by the sanitizers and fails
 * the process.  Test infrastructure only (tests/test_sanitizers.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double ehh_cutoff, maf_cutoff;
    int64_t gap_scale_bp, max_gap_bp;
    double bin_width;
    int32_t physical_map;
} params_t;

int or_ihs(const uint8_t *H, int64_t n, int64_t M, const int64_t *pos, const double *gpos,
           const params_t *p, const int64_t *loci, int64_t n_loci, double *ihh1, double *ihh0,
           double *unstd, double *stdz, double *freq, int8_t *status, int32_t *bin, int64_t *steps,
           int nthreads);
int or_xpehh(const uint8_t *HA, int64_t nA, const uint8_t *HB, int64_t nB, int64_t M,
             const int64_t *pos, const double *gpos, const params_t *p, const int64_t *loci,
             int64_t n_loci, double *ihhA, double *ihhB, double *unstd, double *stdz,
             int8_t *status, int64_t *steps, int nthreads);
int or_ehh(const uint8_t *H, int64_t n, int64_t M, const int64_t *pos, const double *gpos,
           const params_t *p, int64_t core, int64_t cap, uint64_t *S, double *ehh, int64_t *len,
           uint32_t *sizes, double *ihh, int8_t *status);
int or_xpehh_trace(const uint8_t *HA, int64_t nA, const uint8_t *HB, int64_t nB, int64_t M,
                   const int64_t *pos, const double *gpos, const params_t *p, int64_t site,
                   int64_t cap, uint64_t *S, int64_t *len, double *ihh, int8_t *status);

static uint64_t state = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64(void) {   /* xorshift64* */
    state ^= state >> 12; state ^= state << 25; state ^= state >> 27;
    return state * 2685821657736338717ull;
}

static void fill(uint8_t *H, int64_t M, int64_t n, int founders) {
    /* a few founder haplotypes copied with switches, so that walks run for a while */
    uint8_t *f = malloc((size_t)(founders * M));
    for (int64_t i = 0; i < founders * M; ++i) f[i] = (uint8_t)(next_u64() & 1);
    for (int64_t h = 0; h < n; ++h) {
        int cur = (int)(next_u64() % (uint64_t)founders);
        for (int64_t k = 0; k < M; ++k) {
            if (next_u64() % 50 == 0) cur = (int)(next_u64() % (uint64_t)founders);
            H[k * n + h] = f[cur * M + k];
        }
    }
    free(f);
}

int main(void) {
    int runs = 0;
    for (int trial = 0; trial < 40; ++trial) {
        const int64_t n = 2 + (int64_t)(next_u64() % 60), nB = 2 + (int64_t)(next_u64() % 40);
        const int64_t M = 1 + (int64_t)(next_u64() % 120);
        uint8_t *H = malloc((size_t)(n * M)), *HB = malloc((size_t)(nB * M));
        int64_t *pos = malloc(sizeof(int64_t) * (size_t)M);
        double *gpos = malloc(sizeof(double) * (size_t)M);
        fill(H, M, n, 1 + trial % 5);
        fill(HB, M, nB, 1 + trial % 4);
        int64_t x = 0;
        for (int64_t k = 0; k < M; ++k) {
            x += (int64_t)(next_u64() % (trial % 3 == 0 ? 300000 : 30000));   /* some abort gaps */
            pos[k] = x;
            gpos[k] = (double)x * 1e-6;
        }
        params_t p = {trial % 4 == 0 ? 0.001 : 0.05, trial % 2 ? 0.0 : 0.05, 20000, 200000,
                      trial % 5 == 0 ? 0.3 : 0.025, trial % 3 == 1};
        double *a = malloc(sizeof(double) * (size_t)M * 5);
        int8_t *st = malloc((size_t)M);
        int32_t *bin = malloc(sizeof(int32_t) * (size_t)M);
        int64_t *steps = malloc(sizeof(int64_t) * (size_t)M * 4);
        if (or_ihs(H, n, M, pos, gpos, &p, NULL, 0, a, a + M, a + 2 * M, a + 3 * M, a + 4 * M, st, bin,
                   steps, 2) != 0) return 2;
        if (or_xpehh(H, n, HB, nB, M, pos, gpos, &p, NULL, 0, a, a + M, a + 2 * M, a + 3 * M, st,
                     steps, 2) != 0) return 3;
        const int64_t cap = 1 + (int64_t)(next_u64() % 64);
        uint64_t *S = malloc(sizeof(uint64_t) * 2 * (size_t)(cap + 1) * 3);
        double *e = malloc(sizeof(double) * 2 * (size_t)(cap + 1) * 3);
        uint32_t *sz = malloc(sizeof(uint32_t) * 2 * (size_t)(cap + 1) * (size_t)n);
        int64_t len[2];
        double ihh[2];
        int8_t s1;
        for (int64_t core = 0; core < M; core += 1 + M / 7) {
            if (or_ehh(H, n, M, pos, gpos, &p, core, cap, S, e, len, sz, ihh, &s1) != 0) return 4;
            if (or_xpehh_trace(H, n, HB, nB, M, pos, gpos, &p, core, cap, S, len, ihh, &s1) != 0) return 5;
            runs += 2;
        }
        free(H); free(HB); free(pos); free(gpos); free(a); free(st); free(bin); free(steps);
        free(S); free(e); free(sz);
        runs += 2;
    }
    printf("sanitized oracle runs: %d\n", runs);
    return 0;
}

// Copying-model haplotypes generated on the GPU for the served request stream
// (input generation only; none of the scan's arithmetic is here).
//
// Every random draw is a hash of (key, row, column): splitmix64's finalizer
// (Steele, Lea & Flood, OOPSLA 2014) applied to key ^ (row << 32 | column).
// A uniform is 24 bits of the hash times 2^-24, exact in float32.  The numpy
// generator in hapgen/__init__.py evaluates the same hashes, integer steps and
// float32 operations (no fused multiply-add), so both give the same matrices.
//
//   * positions: spacings max(1, floor(-ln(1 - u) bp)) for 53-bit uniforms u,
//     the first site at 1 (a Poisson process of about one site per bp);
//   * site frequency p ~ Beta(1/2, 1/2), the arcsine law: (x, y) uniform in
//     the unit disk by rejection, p = x^2 / (x^2 + y^2); a founder carries the
//     derived allele when u (x^2 + y^2) < x^2, i.e. u < p without a division;
//   * population B's founders keep A's entry with probability share, else
//     draw afresh from their own site frequencies;
//   * haplotype h starts on founder floor(F b / 2^32) for 32 hash bits b; at
//     each site s >= 1 one hash w gives the switch (top 24 bits < switch_p),
//     the founder switched to (f + 1 + floor((F - 1) (w & 0xffff) / 2^16)) mod F
//     and the flip (bits 16..39 < flip_p) of the copied allele.
// The founder path is a scan along the sites: per block of 64 sites the sum of
// the switch offsets modulo F, an exclusive scan of those sums per haplotype
// (by the caller), then every block replayed from its starting founder.
#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace {

constexpr int kBlk = 64;
constexpr int kMaxTries = 64;   // rejection draws; all 64 rejected (p ~ 1e-43): p = 1/2

__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t draw(uint64_t key, uint32_t row, uint32_t col) {
    return mix64(key ^ (((uint64_t)row << 32) | col));
}

__device__ __forceinline__ float top24(uint64_t w) {
    return (float)(uint32_t)(w >> 40) * (1.0f / 16777216.0f);
}

__device__ __forceinline__ float mid24(uint64_t w) {
    return (float)(uint32_t)((w >> 16) & 0xFFFFFFu) * (1.0f / 16777216.0f);
}

// gaps[s] between consecutive sites: 1 at s = 0, else max(1, floor(-ln(1 - u) bp))
// for a 53-bit uniform u (exponential spacings of mean about bp)
__global__ void gaps_kernel(uint64_t kg, int64_t M, double bp, int64_t *gaps) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= M) return;
    int64_t g = 1;
    if (s > 0) {
        const double u = (double)(draw(kg, 0, (uint32_t)s) >> 11) * 0x1p-53;
        const double e = floor(-log1p(-u) * bp);
        g = e > 1.0 ? (int64_t)e : 1;
    }
    gaps[s] = g;
}

// founders[f][s] for one site per thread
__global__ void founders_kernel(uint64_t kp, uint64_t ka, uint64_t kk, int F, int64_t M,
                                const uint8_t *base, float share, uint8_t *out) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= M) return;
    float xx = 0.5f, r = 1.0f;
    for (int t = 0; t < kMaxTries; ++t) {
        const float x = 2.0f * top24(draw(kp, 2 * t, (uint32_t)s)) - 1.0f;
        const float y = 2.0f * top24(draw(kp, 2 * t + 1, (uint32_t)s)) - 1.0f;
        const float x2 = x * x, y2 = y * y;
        const float rr = x2 + y2;
        if (rr <= 1.0f && rr > 0.0f) { xx = x2; r = rr; break; }
    }
    for (int f = 0; f < F; ++f) {
        uint8_t a = top24(draw(ka, f, (uint32_t)s)) * r < xx ? 1 : 0;
        if (base && top24(draw(kk, f, (uint32_t)s)) < share) a = base[(int64_t)f * M + s];
        out[(int64_t)f * M + s] = a;
    }
}

__device__ __forceinline__ int switch_offset(uint64_t w, int F) {
    return 1 + (int)(((uint32_t)(F - 1) * (uint32_t)(w & 0xFFFFu)) >> 16);
}

// sums[h][b]: switch offsets of haplotype h over the sites of block b, mod F
__global__ void block_offsets_kernel(uint64_t ks, int F, int64_t M, int n, float sw, int32_t *sums) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t b = blockIdx.y;
    if (h >= n) return;
    int acc = 0;
    const int64_t s0 = b * kBlk, s1 = s0 + kBlk < M ? s0 + kBlk : M;
    for (int64_t s = s0 < 1 ? 1 : s0; s < s1; ++s) {
        const uint64_t w = draw(ks, (uint32_t)h, (uint32_t)s);
        if (top24(w) < sw) acc += switch_offset(w, F);
    }
    sums[(int64_t)h * gridDim.y + b] = acc % F;
}

// out[s][h] for the sites of block b, from the block's starting founder
__global__ void copy_kernel(uint64_t ks, uint64_t k0, int F, int64_t M, int n, float sw, float fp,
                            const uint8_t *founders, const int64_t *excl, uint8_t *out) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t b = blockIdx.y;
    if (h >= n) return;
    const uint32_t b32 = (uint32_t)(draw(k0, (uint32_t)h, 0) >> 32);
    const int64_t f0 = (int64_t)(((uint64_t)b32 * (uint64_t)F) >> 32);
    int f = (int)((f0 + excl[(int64_t)h * gridDim.y + b]) % F);
    const int64_t s0 = b * kBlk, s1 = s0 + kBlk < M ? s0 + kBlk : M;
    for (int64_t s = s0; s < s1; ++s) {
        const uint64_t w = draw(ks, (uint32_t)h, (uint32_t)s);
        if (s >= 1 && top24(w) < sw) f = (f + switch_offset(w, F)) % F;
        uint8_t a = founders[(int64_t)f * M + s];
        if (mid24(w) < fp) a ^= 1;
        out[s * n + h] = a;
    }
}

uint64_t key_of(uint64_t seed, int tag) { return mix64(seed * 16 + (uint64_t)tag); }

bool fits(int F, int64_t M, int n) {
    return F >= 1 && F <= 65536 && M >= 1 && M < (int64_t)1 << 31 && n >= 0 && n < (1 << 30) &&
           (M + kBlk - 1) / kBlk <= 65535;
}

}  // namespace

extern "C" {

// Spacings (int64 [M], device) of the sites of a region; their running sum
// gives positions 1, 1 + gaps[1], ...  Same returns as hg_founders.
int hg_gaps(uint64_t seed, int64_t M, double bp_per_site, int64_t *gaps, void *stream) {
    if (!fits(1, M, 0) || !gaps || !(bp_per_site > 0.0)) return -1;
    hipLaunchKernelGGL(gaps_kernel, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       key_of(seed, 15), M, bp_per_site, gaps);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

// Founder alleles, uint8 [F][M] row-major, into out (device, F*M bytes).
// tag: the population's stream tag (0 for A, 8 for B); base (device, [F][M])
// and share: with base non-null each entry is base's with probability share.
// Returns 0, -1 for bad sizes or null out, -4 when the launch fails.
int hg_founders(uint64_t seed, int tag, int F, int64_t M, const uint8_t *base, float share,
                uint8_t *out, void *stream) {
    if (!fits(F, M, 0) || !out) return -1;
    const unsigned blocks = (unsigned)((M + 255) / 256);
    hipLaunchKernelGGL(founders_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                       key_of(seed, tag + 0), key_of(seed, tag + 1), key_of(seed, tag + 2), F, M,
                       base, share, out);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

// Pass 1 of the copy: int32 sums [n][ceil(M/64)] (device) of the switch
// offsets per block of 64 sites, modulo F.  Same returns as hg_founders.
int hg_block_offsets(uint64_t seed, int tag, int F, int64_t M, int n, float switch_p, int32_t *sums,
                     void *stream) {
    if (!fits(F, M, n) || !sums) return -1;
    if (n == 0) return 0;
    const int64_t nb = (M + kBlk - 1) / kBlk;
    hipLaunchKernelGGL(block_offsets_kernel, dim3((unsigned)((n + 63) / 64), (unsigned)nb), dim3(64), 0,
                       (hipStream_t)stream, key_of(seed, tag + 3), F, M, n, switch_p, sums);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

// Pass 2: alleles uint8 [M][n] (device) from the founders and excl, the
// exclusive prefix sums (int64 [n][ceil(M/64)], device) of pass 1's sums
// along each haplotype's row.  Same returns as hg_founders.
int hg_copy(uint64_t seed, int tag, const uint8_t *founders, int F, int64_t M, int n, float switch_p,
            float flip_p, const int64_t *excl, uint8_t *out, void *stream) {
    if (!fits(F, M, n) || !founders || !excl || !out) return -1;
    if (n == 0) return 0;
    const int64_t nb = (M + kBlk - 1) / kBlk;
    hipLaunchKernelGGL(copy_kernel, dim3((unsigned)((n + 63) / 64), (unsigned)nb), dim3(64), 0,
                       (hipStream_t)stream, key_of(seed, tag + 3), key_of(seed, tag + 5), F, M, n,
                       switch_p, flip_p, founders, excl, out);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // extern "C"

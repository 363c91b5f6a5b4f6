// ga.hip -- one GA generation over a population of genomes (Sec. II-C, Table I):
// elites by rank, two k-tournaments per child, uniform crossover, per-gene
// Gaussian mutation, every random decision drawn from Philox-4x64-10 at the
// counter (generation, child, purpose, block) with key (seed, 0).
#include <cmath>

#include "internal.h"

namespace sr {

namespace {

// Philox-4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11): per round,
// words 0 and 2 are multiplied by the two round multipliers; the high halves
// are xored with the other words and the key, the low halves move over; the
// key is bumped by the two Weyl constants between rounds.
struct U64x4 {
    uint64_t w[4];
};

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0,
                                               uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        const uint64_t y0 = hi1 ^ c1 ^ k0, y2 = hi0 ^ c3 ^ k1;
        c0 = y0;
        c1 = lo1;
        c2 = y2;
        c3 = lo0;
    }
    U64x4 r;
    r.w[0] = c0;
    r.w[1] = c1;
    r.w[2] = c2;
    r.w[3] = c3;
    return r;
}

enum { PUR_TOUR_A = 0, PUR_TOUR_B = 1, PUR_CX = 2, PUR_CX_MASK = 3, PUR_MUT = 4, PUR_GAUSS = 5 };

struct GAArgs {
    const float *fit;
    const float *gin;
    float *gout;
    int P, L, E, k;
    uint64_t p_cross_thr, p_mut_thr;
    float sigma;
    uint64_t seed, gen;
    int32_t *dec;
};

// a is better than b: larger fitness (NaN counts as -inf), ties to the lower index
__device__ __forceinline__ bool better(const float *fit, int a, int b) {
    float fa = fit[a], fb = fit[b];
    if (fa != fa) fa = -INFINITY;
    if (fb != fb) fb = -INFINITY;
    if (fa != fb) return fa > fb;
    return a < b;
}

// Block i ranks individual i against the whole population and, if it is among
// the E best, copies its genome unchanged to slot rank(i).
__global__ __launch_bounds__(256) void k_ga_elite(GAArgs A) {
    __shared__ int part[4];
    const int i = blockIdx.x;
    int cnt = 0;
    for (int j = threadIdx.x; j < A.P; j += 256) cnt += better(A.fit, j, i) ? 1 : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cnt;
    __syncthreads();
    const int rank = part[0] + part[1] + part[2] + part[3];
    if (rank >= A.E) return;
    const float *src = A.gin + (size_t)i * A.L;
    float *dst = A.gout + (size_t)rank * A.L;
    for (int q = threadIdx.x; q < A.L; q += 256) dst[q] = src[q];
    if (threadIdx.x == 0 && A.dec) {
        A.dec[3 * rank] = i;
        A.dec[3 * rank + 1] = i;
        A.dec[3 * rank + 2] = 0;
    }
}

__device__ int tournament(const GAArgs &A, int child, int purpose) {
    int win = -1;
    U64x4 r;
    for (int t = 0; t < A.k; ++t) {
        if ((t & 3) == 0) r = philox4x64_10(A.gen, (uint64_t)child, (uint64_t)purpose, (uint64_t)(t >> 2), A.seed, 0);
        const uint64_t hi = r.w[t & 3] >> 32;
        const int idx = (int)((hi * (uint64_t)A.P) >> 32);
        if (win < 0 || better(A.fit, idx, win)) win = idx;
    }
    return win;
}

// Block per child slot c >= E; each thread makes four consecutive genes.
__global__ __launch_bounds__(256) void k_ga_child(GAArgs A) {
    __shared__ int sh[3];
    const int c = A.E + blockIdx.x;
    if (threadIdx.x == 0) {
        const int a = tournament(A, c, PUR_TOUR_A);
        const int b = tournament(A, c, PUR_TOUR_B);
        const U64x4 r = philox4x64_10(A.gen, (uint64_t)c, PUR_CX, 0, A.seed, 0);
        sh[0] = a;
        sh[1] = b;
        sh[2] = r.w[0] < A.p_cross_thr;
        if (A.dec) {
            A.dec[3 * c] = a;
            A.dec[3 * c + 1] = b;
            A.dec[3 * c + 2] = sh[2] ? 2 : 1;
        }
    }
    __syncthreads();
    const int pa = sh[0], pb = sh[1];
    const bool cx = sh[2] != 0;
    const float *ga = A.gin + (size_t)pa * A.L, *gb = A.gin + (size_t)pb * A.L;
    float *out = A.gout + (size_t)c * A.L;
    for (int g0 = 4 * threadIdx.x; g0 < A.L; g0 += 4 * 256) {
        // one draw block gives the four mutation words of genes g0..g0+3
        const U64x4 mut = philox4x64_10(A.gen, (uint64_t)c, PUR_MUT, (uint64_t)(g0 >> 2), A.seed, 0);
        uint64_t cxw = 0;
        if (cx) {
            const U64x4 m = philox4x64_10(A.gen, (uint64_t)c, PUR_CX_MASK, (uint64_t)(g0 >> 8), A.seed, 0);
            cxw = m.w[(g0 & 255) >> 6];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int g = g0 + q;
            if (g >= A.L) break;
            const bool fromB = cx && ((cxw >> (g & 63)) & 1ULL);
            float val = fromB ? gb[g] : ga[g];
            if (mut.w[q] < A.p_mut_thr) {
                // Box-Muller from two 53-bit uniforms, u1 in (0, 1], u2 in [0, 1)
                const U64x4 z = philox4x64_10(A.gen, (uint64_t)c, PUR_GAUSS, (uint64_t)(g >> 1), A.seed, 0);
                const int w0 = 2 * (g & 1);
                const double u1 = ((double)(z.w[w0] >> 11) + 1.0) * 0x1.0p-53;
                const double u2 = (double)(z.w[w0 + 1] >> 11) * 0x1.0p-53;
                const double nz = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
                val = (float)((double)val + (double)A.sigma * nz);
            }
            out[g] = val;
        }
    }
}

}  // namespace

hipError_t launch_ga(const float *fit, const float *gin, float *gout, int P, int L, int E, int k, uint64_t pc,
                     uint64_t pm, float sigma, uint64_t seed, uint64_t gen, int32_t *dec, hipStream_t st) {
    GAArgs A;
    A.fit = fit;
    A.gin = gin;
    A.gout = gout;
    A.P = P;
    A.L = L;
    A.E = E;
    A.k = k;
    A.p_cross_thr = pc;
    A.p_mut_thr = pm;
    A.sigma = sigma;
    A.seed = seed;
    A.gen = gen;
    A.dec = dec;
    hipLaunchKernelGGL(k_ga_elite, dim3(P), dim3(256), 0, st, A);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || E >= P) return e;
    hipLaunchKernelGGL(k_ga_child, dim3(P - E), dim3(256), 0, st, A);
    return hipGetLastError();
}

}  // namespace sr

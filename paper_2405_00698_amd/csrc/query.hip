// query.hip -- genome MLP over every robot's voxel grid (Sec. II-B Eq. (1), Sec. II-C).
//
// For voxel (i,j,k) of an n^3 grid the query point is v = ((i+1/2)/n, (j+1/2)/n, (k+1/2)/n);
// gamma(v) = [cos(2 pi B v), sin(2 pi B v)] (32 + 32 entries), h1 = tanh(W1 gamma + b1),
// h2 = tanh(W2 h1 + b2), o = W3 h2 + b3; the class is argmax o[0..4] (lowest id on ties) and
// the weight is sigmoid(o[5]).
#include "internal.h"

namespace sr {

namespace {

constexpr int QB = 256;  // voxels (threads) per workgroup
constexpr int OFF_W1 = 0, OFF_B1 = 4096, OFF_W2 = 4160, OFF_B2 = 8256, OFF_W3 = 8320, OFF_B3 = 8704;

// FP32 form: one voxel per thread, the robot's weights staged in LDS and read
// as broadcasts (every lane reads the same weight).
__global__ __launch_bounds__(QB) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_query_fp32(const RobotInfo *robots, const float *genomes, const float *B,
                                                   uint8_t *cls, float *w) {
    __shared__ float Ws[SR_GENOME_LEN];
    __shared__ float Bs[3 * SR_PE_M];
    const int r = blockIdx.y;
    const RobotInfo ri = robots[r];
    const int nv = ri.n * ri.n * ri.n;
    if ((int)(blockIdx.x * QB) >= nv) return;
    const float *g = genomes + (size_t)r * SR_GENOME_LEN;
    for (int q = threadIdx.x; q < SR_GENOME_LEN; q += QB) Ws[q] = g[q];
    for (int q = threadIdx.x; q < 3 * SR_PE_M; q += QB) Bs[q] = B[q];
    __syncthreads();
    const int vid = blockIdx.x * QB + threadIdx.x;
    if (vid >= nv) return;
    const int n = ri.n;
    const float inv = 1.0f / (float)n;
    const float vx = ((vid % n) + 0.5f) * inv, vy = (((vid / n) % n) + 0.5f) * inv, vz = ((vid / (n * n)) + 0.5f) * inv;
    float gam[2 * SR_PE_M];
#pragma unroll
    for (int q = 0; q < SR_PE_M; ++q) {
        // 2 pi (B v) taken as pi * (2 B v) so the angle scaling is exact
        const float t = 2.0f * fmaf(Bs[3 * q + 2], vz, fmaf(Bs[3 * q + 1], vy, Bs[3 * q] * vx));
        float s, c;
        sincospif(t, &s, &c);
        gam[q] = c;
        gam[SR_PE_M + q] = s;
    }
    float h1[64];
#pragma unroll
    for (int i = 0; i < 64; ++i) {
        float a = Ws[OFF_B1 + i];
#pragma unroll
        for (int j = 0; j < 64; ++j) a = fmaf(Ws[OFF_W1 + 64 * i + j], gam[j], a);
        h1[i] = tanhf(a);
    }
    float h2[64];
#pragma unroll
    for (int i = 0; i < 64; ++i) {
        float a = Ws[OFF_B2 + i];
#pragma unroll
        for (int j = 0; j < 64; ++j) a = fmaf(Ws[OFF_W2 + 64 * i + j], h1[j], a);
        h2[i] = tanhf(a);
    }
    float o[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        float a = Ws[OFF_B3 + i];
#pragma unroll
        for (int j = 0; j < 64; ++j) a = fmaf(Ws[OFF_W3 + 64 * i + j], h2[j], a);
        o[i] = a;
    }
    int best = 0;
#pragma unroll
    for (int q = 1; q < 5; ++q)
        if (o[q] > o[best]) best = q;
    cls[ri.vox_base + vid] = (uint8_t)best;
    w[ri.vox_base + vid] = 1.0f / (1.0f + expf(-o[5]));
}

// ---------------------------------------------------------------- BF16 MFMA form
// Activations are kept transposed (features x voxels), so each layer is
// D = W H^T with the weights as the MFMA A operand and the activations as B.
// gfx950's v_mfma_f32_16x16x32_bf16: lane l of A holds row l%16 and eight
// values of k, lane l of B column l%16 and the same eight k, lane l of D
// column l%16 and rows 4(l/16)..+3.  A contraction may number its k in any
// order that A and B share; here k = 8 kq + j (kq = l/16, j = 0..7) of K-block
// b is feature 32 b + 16 (j/4) + 4 kq + j%4.  Then the D fragments of output
// blocks 2b and 2b + 1, side by side, are exactly the B fragment of K-block b
// of the next layer, so activations never leave registers, and a lane's A
// fragment is two 8-byte runs of one weight row.  One wave handles 16 voxels.
// Weights are staged in LDS as BF16 (round to nearest even) in rows padded to
// 72 entries, so the 8-byte reads of half a wave fall on distinct banks.
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int WROW = 72;  // padded LDS row of a BF16 weight matrix

__device__ __forceinline__ unsigned short f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ s16x4 pack4(float a, float b, float c, float d) {
    s16x4 r;
    r[0] = (short)f2bf(a);
    r[1] = (short)f2bf(b);
    r[2] = (short)f2bf(c);
    r[3] = (short)f2bf(d);
    return r;
}

__device__ __forceinline__ bf16x8 cat8(s16x4 lo, s16x4 hi) {
    return __builtin_bit_cast(bf16x8, __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7));
}

// A fragment of rows 16 mb + col, K-block b, for the lane of k-quarter kq
__device__ __forceinline__ bf16x8 wfrag(const unsigned short *W, int row, int b, int kq) {
    const unsigned short *p = W + WROW * row + 32 * b + 4 * kq;
    const uint2 lo = *reinterpret_cast<const uint2 *>(p);
    const uint2 hi = *reinterpret_cast<const uint2 *>(p + 16);
    return __builtin_bit_cast(bf16x8, make_uint4(lo.x, lo.y, hi.x, hi.y));
}

__global__ __launch_bounds__(256) void k_query_bf16(const RobotInfo *robots, const float *genomes, const float *B,
                                                    uint8_t *cls, float *w) {
    __shared__ __align__(16) unsigned short W1s[64 * WROW], W2s[64 * WROW], W3s[16 * WROW];
    __shared__ float bias[64 + 64 + 6];
    __shared__ float Bs[3 * SR_PE_M];
    const int r = blockIdx.x;
    const RobotInfo ri = robots[r];
    const int n = ri.n, nv = n * n * n;
    const float *g = genomes + (size_t)r * SR_GENOME_LEN;
    for (int q = threadIdx.x; q < 64 * 64; q += 256) {
        const int o = WROW * (q >> 6) + (q & 63);
        W1s[o] = f2bf(g[OFF_W1 + q]);
        W2s[o] = f2bf(g[OFF_W2 + q]);
    }
    for (int q = threadIdx.x; q < 16 * 64; q += 256)
        W3s[WROW * (q >> 6) + (q & 63)] = q < 6 * 64 ? f2bf(g[OFF_W3 + q]) : 0;
    for (int q = threadIdx.x; q < 64; q += 256) {
        bias[q] = g[OFF_B1 + q];
        bias[64 + q] = g[OFF_B2 + q];
    }
    if (threadIdx.x < 6) bias[128 + threadIdx.x] = g[OFF_B3 + threadIdx.x];
    for (int q = threadIdx.x; q < 3 * SR_PE_M; q += 256) Bs[q] = B[q];
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int col = lane & 15, kq = lane >> 4;  // voxel column and k quarter of this lane
    const float inv = 1.0f / (float)n;
    for (int v0 = wave * 16; v0 < nv; v0 += 64) {
        const int vid = v0 + col;
        const int vc = vid < nv ? vid : nv - 1;
        const float vx = ((vc % n) + 0.5f) * inv, vy = (((vc / n) % n) + 0.5f) * inv, vz = ((vc / (n * n)) + 0.5f) * inv;
        // gamma(v) in 16-feature blocks X[m] (features 16 m + 4 kq + i of voxel `col`):
        // blocks 0, 1 are cos(2 pi b_q . v) and blocks 2, 3 sin of the same q
        s16x4 X[4];
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            float cs[4], sn[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int q = 16 * m + 4 * kq + i;
                const float t = 2.0f * fmaf(Bs[3 * q + 2], vz, fmaf(Bs[3 * q + 1], vy, Bs[3 * q] * vx));
                sincospif(t, &sn[i], &cs[i]);
            }
            X[m] = pack4(cs[0], cs[1], cs[2], cs[3]);
            X[m + 2] = pack4(sn[0], sn[1], sn[2], sn[3]);
        }
        // two tanh layers
        s16x4 H[4];
#pragma unroll
        for (int layer = 0; layer < 2; ++layer) {
            const unsigned short *W = layer == 0 ? W1s : W2s;
            const float *bb = bias + 64 * layer;
            const s16x4 *in = layer == 0 ? X : H;
            const bf16x8 b0 = cat8(in[0], in[1]), b1 = cat8(in[2], in[3]);
            s16x4 Hn[4];
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) {
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wfrag(W, 16 * mb + col, 0, kq), b0, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wfrag(W, 16 * mb + col, 1, kq), b1, acc, 0, 0, 0);
                const int f0 = 16 * mb + 4 * kq;
                Hn[mb] = pack4(tanhf(acc[0] + bb[f0]), tanhf(acc[1] + bb[f0 + 1]), tanhf(acc[2] + bb[f0 + 2]),
                               tanhf(acc[3] + bb[f0 + 3]));
            }
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) H[mb] = Hn[mb];
        }
        // output layer: rows 0..5 of a 16-row block
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wfrag(W3s, col, 0, kq), cat8(H[0], H[1]), acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wfrag(W3s, col, 1, kq), cat8(H[2], H[3]), acc, 0, 0, 0);
        // lane col (kq = 0) holds o0..o3, lane col + 16 (kq = 1) holds o4, o5
        const float o4 = __shfl(acc[0], col + 16, 64);
        const float o5 = __shfl(acc[1], col + 16, 64);
        if (kq == 0 && vid < nv) {
            float o[5] = {acc[0] + bias[128], acc[1] + bias[129], acc[2] + bias[130], acc[3] + bias[131],
                          o4 + bias[132]};
            int best = 0;
#pragma unroll
            for (int q = 1; q < 5; ++q)
                if (o[q] > o[best]) best = q;
            cls[ri.vox_base + vid] = (uint8_t)best;
            w[ri.vox_base + vid] = 1.0f / (1.0f + expf(-(o5 + bias[133])));
        }
    }
}

}  // namespace

hipError_t launch_query(const RobotInfo *robots, int R, int max_side, const float *genomes, const float *B, int precision,
                        uint8_t *cls, float *w, hipStream_t st) {
    if (precision == SR_QUERY_BF16) {
        hipLaunchKernelGGL(k_query_bf16, dim3(R), dim3(256), 0, st, robots, genomes, B, cls, w);
        return hipGetLastError();
    }
    const int maxv = max_side * max_side * max_side;
    dim3 grid((maxv + QB - 1) / QB, R);
    hipLaunchKernelGGL(k_query_fp32, grid, dim3(QB), 0, st, robots, genomes, B, cls, w);
    return hipGetLastError();
}

}  // namespace sr

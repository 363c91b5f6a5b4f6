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
// Activations are kept transposed (features x voxels) so that each layer is
// D = W * H^T with the weights as the MFMA A operand and the activations as B:
// with v_mfma_f32_16x16x16 (A: lane l holds row l%16, k = 4(l/16)..+3; B: lane l
// holds column l%16, the same k; D: lane l holds column l%16, rows 4(l/16)..+3)
// the D fragment of output block m is exactly the B fragment of input block m of
// the next layer, so activations never leave registers.  One wave handles 16
// voxels; weights are staged in LDS as BF16 (round to nearest even).
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d) {
    bf16x4 r;
    r[0] = (short)f2bf(a);
    r[1] = (short)f2bf(b);
    r[2] = (short)f2bf(c);
    r[3] = (short)f2bf(d);
    return r;
}

__global__ __launch_bounds__(256) void k_query_bf16(const RobotInfo *robots, const float *genomes, const float *B,
                                                    uint8_t *cls, float *w) {
    __shared__ unsigned short W1s[64 * 64], W2s[64 * 64], W3s[16 * 64];
    __shared__ float bias[64 + 64 + 6];
    __shared__ float Bs[3 * SR_PE_M];
    const int r = blockIdx.x;
    const RobotInfo ri = robots[r];
    const int n = ri.n, nv = n * n * n;
    const float *g = genomes + (size_t)r * SR_GENOME_LEN;
    for (int q = threadIdx.x; q < 64 * 64; q += 256) {
        W1s[q] = f2bf(g[OFF_W1 + q]);
        W2s[q] = f2bf(g[OFF_W2 + q]);
    }
    for (int q = threadIdx.x; q < 16 * 64; q += 256) W3s[q] = q < 6 * 64 ? f2bf(g[OFF_W3 + q]) : 0;
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
        // B fragments of gamma(v): feature 16 kb + 4 kq + i of voxel `col`
        bf16x4 X[4];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            float f[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int j = 16 * kb + 4 * kq + i;
                const int q = j & 31;
                const float t = 2.0f * fmaf(Bs[3 * q + 2], vz, fmaf(Bs[3 * q + 1], vy, Bs[3 * q] * vx));
                float sn, cs;
                sincospif(t, &sn, &cs);
                f[i] = j < 32 ? cs : sn;
            }
            X[kb] = pack4(f[0], f[1], f[2], f[3]);
        }
        // two tanh layers
        bf16x4 H[4];
#pragma unroll
        for (int layer = 0; layer < 2; ++layer) {
            const unsigned short *W = layer == 0 ? W1s : W2s;
            const float *bb = bias + 64 * layer;
            bf16x4 Hn[4];
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) {
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < 4; ++kb) {
                    const unsigned short *wr = W + 64 * (16 * mb + col) + 16 * kb + 4 * kq;
                    bf16x4 a;
                    a[0] = (short)wr[0];
                    a[1] = (short)wr[1];
                    a[2] = (short)wr[2];
                    a[3] = (short)wr[3];
                    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, layer == 0 ? X[kb] : H[kb], acc, 0, 0, 0);
                }
                const int f0 = 16 * mb + 4 * kq;
                Hn[mb] = pack4(tanhf(acc[0] + bb[f0]), tanhf(acc[1] + bb[f0 + 1]), tanhf(acc[2] + bb[f0 + 2]),
                               tanhf(acc[3] + bb[f0 + 3]));
            }
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) H[mb] = Hn[mb];
        }
        // output layer: rows 0..5 of a 16-row block
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            const unsigned short *wr = W3s + 64 * col + 16 * kb + 4 * kq;
            bf16x4 a;
            a[0] = (short)wr[0];
            a[1] = (short)wr[1];
            a[2] = (short)wr[2];
            a[3] = (short)wr[3];
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, H[kb], acc, 0, 0, 0);
        }
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

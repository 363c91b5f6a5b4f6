// mesh.hip -- voxels -> robot: largest component, nodes, springs, incidence, initial state.
//
// One workgroup of 1024 threads builds one robot entirely in LDS (Sec. II-A:
// masses on voxel corners; springs on the 12 edges, 12 face diagonals and 4
// body diagonals of every kept voxel).  All integer decisions use integer
// arithmetic or integer LDS atomics, so the result is independent of thread
// timing.
#include "internal.h"

// No contraction of a*b + c into FMAs in this file: the spring parameters are
// sums of separately rounded per-voxel products, which the step kernels that
// rebuild them from voxels repeat operation by operation.
#pragma clang fp contract(off)

namespace sr {

namespace {

constexpr int BT = 1024;          // threads per robot
constexpr int MAXV = SR_MAX_SIDE * SR_MAX_SIDE * SR_MAX_SIDE;
constexpr int MAXS = (SR_MAX_SIDE + 1) * (SR_MAX_SIDE + 1) * (SR_MAX_SIDE + 1);

struct BuildArgs {
    const RobotInfo *robots;
    RobotInfo *robots_out;
    const uint8_t *cls;
    const float *w;
    uint8_t *kept;
    Planes pl;
    int32_t *sid;
    float4 *x0, *x, *v;
    int32_t *slot_node, *node_slot;
    NodeRow *rows;
    Entry *entries;
    uint8_t *bad_class, *diverged;
    float k_class[5], ac_cos[5], ac_sin[5];
    float a_class[5], phi_class[5];  // for weight-scaled actuation
    int weight_act;
    float dash2m;  // 2 m zeta_spring^2: a voxel spring's dashpot is sqrt(dash2m k_c w)
    float voxel_len;
};

// A kept voxel's contributions to each of its springs (parallel-sum rule):
// x = k_c w, y = k_c w amp cos(ph), z = k_c w amp sin(ph), w = its dashpot.
// Separately rounded operations (contraction is off in this file), so that a
// spring's sums can be rebuilt bit for bit from these per-voxel values.
__device__ float4 voxel_terms(const BuildArgs &A, int kc, float wv) {
    const float kw = A.k_class[kc] * wv;
    float cz, sz;
    if (A.weight_act) {
        // amplitude w a_c and phase w phi_c (Table II maxima times the weight)
        const float amp = wv * A.a_class[kc], ph = wv * A.phi_class[kc];
        cz = amp * cosf(ph);
        sz = amp * sinf(ph);
    } else {
        cz = A.ac_cos[kc];
        sz = A.ac_sin[kc];
    }
    return make_float4(kw, kw * cz, kw * sz, sqrtf(A.dash2m * kw));
}

// exclusive prefix sum over the block in thread order; returns the block total in *total
__device__ int block_exscan(int val, int *tmp, int *total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int inc = val;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) tmp[wv] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int q = 0; q < BT / 64; ++q) {
            int t = tmp[q];
            tmp[q] = run;
            run += t;
        }
        tmp[BT / 64] = run;
    }
    __syncthreads();
    int res = tmp[wv] + inc - val;
    *total = tmp[BT / 64];
    __syncthreads();
    return res;
}

__global__ __launch_bounds__(BT) void k_build_mesh(BuildArgs A) {
    __shared__ int lab[MAXV];
    __shared__ uint8_t cl[MAXV];
    __shared__ int cnt[MAXV];
    __shared__ int nid[MAXS];        // node id per slot, -1 absent
    __shared__ uint16_t emask[MAXS]; // bit d: forward spring (slot, d) exists
    __shared__ int sbase[MAXS];      // canonical id of the slot's first forward spring
    __shared__ int tmp[BT / 64 + 1];
    __shared__ int flag[3];
    __shared__ unsigned bestkey;
    __shared__ int zmin_c;

    const int r = blockIdx.x, tid = threadIdx.x;
    const RobotInfo ri = A.robots[r];
    const int n = ri.n, N = ri.N, nv = n * n * n, SL = ri.slots;
    const uint8_t *cin = A.cls + ri.vox_base;

    // 1. classes; out-of-range classes are reported and treated as empty
    for (int q = tid; q < nv; q += BT) {
        int c = cin[q];
        if (c > 4) { A.bad_class[r] = 1; c = 0; }
        cl[q] = (uint8_t)c;
        lab[q] = c ? q : 0x7fffffff;
        cnt[q] = 0;
    }
    if (tid < 3) flag[tid] = 0;
    if (tid == 0) { bestkey = 0u; zmin_c = 0x7fffffff; }
    __syncthreads();

    // 2. face-connected components by min-label propagation with pointer
    // jumping; the fixed point is the smallest voxel id of each component
    for (int it = 0;; ++it) {
        if (tid == 0) flag[(it + 1) % 3] = 0;
        for (int q = tid; q < nv; q += BT) {
            if (!cl[q]) continue;
            int i = q % n, j = (q / n) % n, k = q / (n * n);
            int m = lab[q];
            if (i > 0 && cl[q - 1]) m = min(m, lab[q - 1]);
            if (i < n - 1 && cl[q + 1]) m = min(m, lab[q + 1]);
            if (j > 0 && cl[q - n]) m = min(m, lab[q - n]);
            if (j < n - 1 && cl[q + n]) m = min(m, lab[q + n]);
            if (k > 0 && cl[q - n * n]) m = min(m, lab[q - n * n]);
            if (k < n - 1 && cl[q + n * n]) m = min(m, lab[q + n * n]);
            m = min(m, lab[m]);
            if (m < lab[q]) {
                lab[q] = m;
                flag[it % 3] = 1;
            }
        }
        __syncthreads();
        if (flag[it % 3] == 0) break;
    }

    // 3. component sizes; the largest wins, ties to the smallest root id
    for (int q = tid; q < nv; q += BT)
        if (cl[q]) atomicAdd(&cnt[lab[q]], 1);
    __syncthreads();
    for (int q = tid; q < nv; q += BT)
        if (cl[q] && lab[q] == q) atomicMax(&bestkey, ((unsigned)cnt[q] << 16) | (unsigned)(0xffff - q));
    __syncthreads();
    const int best = bestkey ? 0xffff - (int)(bestkey & 0xffff) : -1;
    for (int q = tid; q < nv; q += BT) {
        uint8_t c = (cl[q] && lab[q] == best) ? cl[q] : 0;
        A.kept[ri.vox_base + q] = c;
        lab[q] = c; // lab now holds the kept class
    }
    __syncthreads();

    // 4. nodes: lattice points touching a kept voxel; lowest z layer
    for (int s = tid; s < SL; s += BT) {
        int a = s % N, b = (s / N) % N, c = s / (N * N);
        int pres = 0;
        for (int dz = -1; dz <= 0; ++dz)
            for (int dy = -1; dy <= 0; ++dy)
                for (int dx = -1; dx <= 0; ++dx) {
                    int i = a + dx, j = b + dy, k = c + dz;
                    if (i >= 0 && i < n && j >= 0 && j < n && k >= 0 && k < n && lab[i + n * (j + n * k)])
                        pres = 1;
                }
        nid[s] = pres;
        if (pres) atomicMin(&zmin_c, c);
    }
    __syncthreads();

    // 5. canonical node ids (ascending slot) by an ordered block scan
    const int CH = (SL + BT - 1) / BT;
    const int s0 = tid * CH, s1 = min(s0 + CH, SL);
    int total;
    {
        int c = 0;
        for (int s = s0; s < s1; ++s) c += nid[s];
        int off = block_exscan(c, tmp, &total);
        for (int s = s0; s < s1; ++s) nid[s] = nid[s] ? off++ : -1;
    }
    const int M = total;
    __syncthreads();

    // 6. springs from each lower slot along the 13 forward directions; the
    // kept voxels holding both ends add up in parallel (fixed order)
    const float L0e = A.voxel_len, L0f = A.voxel_len * sqrtf(2.0f), L0b = A.voxel_len * sqrtf(3.0f);
    const int pbase = NDIR * ri.slot_base;
    for (int s = tid; s < SL; s += BT) {
        int a = s % N, b = (s / N) % N, c = s / (N * N);
        unsigned mask = 0;
        for (int d = 0; d < NDIR; ++d) {
            const int dx = dir_dx(d), dy = dir_dy(d), dz = dir_dz(d);
            float ks = 0.f, zr = 0.f, zi = 0.f, cd = 0.f;
            int hits = 0;
            const int a2 = a + dx, b2 = b + dy, c2 = c + dz;
            if (nid[s] >= 0 && a2 >= 0 && a2 < N && b2 >= 0 && b2 < N && c2 < N) {
                // voxel index range per axis: both coordinates must lie in [v, v+1]
                const int vx0 = min(a, a2) - (dx == 0), vx1 = min(a, a2);
                const int vy0 = min(b, b2) - (dy == 0), vy1 = min(b, b2);
                const int vz0 = c - 1 + dz, vz1 = c;  // dz is 0 or 1
                for (int vz = vz0; vz <= vz1; ++vz)
                    for (int vy = vy0; vy <= vy1; ++vy)
                        for (int vx = vx0; vx <= vx1; ++vx) {
                            if (vx < 0 || vx >= n || vy < 0 || vy >= n || vz < 0 || vz >= n) continue;
                            const int kc = lab[vx + n * (vy + n * vz)];
                            if (!kc) continue;
                            const float4 t = voxel_terms(A, kc, A.w[ri.vox_base + vx + n * (vy + n * vz)]);
                            ks += t.x;
                            zr += t.y;
                            zi += t.z;
                            cd += t.w;
                            ++hits;
                        }
            }
            const int len2 = dir_len2(d);
            const float L0 = len2 == 1 ? L0e : len2 == 2 ? L0f : L0b;
            const int pi = pbase + d * SL + s;
            if (hits) mask |= 1u << d;
            A.pl.k[pi] = hits ? ks : 0.f;
            A.pl.kL0[pi] = hits ? ks * L0 : 0.f;
            A.pl.kal[pi] = hits ? zr * L0 : 0.f;
            A.pl.kbe[pi] = hits ? zi * L0 : 0.f;
            A.pl.kd[pi] = hits ? cd : 0.f;
        }
        emask[s] = (uint16_t)mask;
        // the voxel whose lowest corner is this slot, for kernels that rebuild
        // spring parameters from voxels (zero where there is no kept voxel)
        float4 vt = make_float4(0.f, 0.f, 0.f, 0.f);
        if (a < n && b < n && c < n) {
            const int kc = lab[a + n * (b + n * c)];
            if (kc) vt = voxel_terms(A, kc, A.w[ri.vox_base + a + n * (b + n * c)]);
        }
        A.pl.vkp[ri.slot_base + s] = vt;
    }
    __syncthreads();

    // 7. canonical spring ids: lower node ascending, then direction
    {
        int c = 0;
        for (int s = s0; s < s1; ++s) c += __popc((unsigned)emask[s]);
        int off = block_exscan(c, tmp, &total);
        for (int s = s0; s < s1; ++s) {
            sbase[s] = off;
            off += __popc((unsigned)emask[s]);
        }
    }
    const int S = total;
    __syncthreads();
    for (int s = tid; s < SL; s += BT) {
        int id = sbase[s];
        for (int d = 0; d < NDIR; ++d) {
            int v = -1;
            if ((emask[s] >> d) & 1) v = id++;
            A.sid[pbase + d * SL + s] = v;
        }
    }

    // 8. incidence rows for the per-step kernel: forward entries in direction
    // order, then backward entries in direction order
    {
        int c = 0;
        for (int s = s0; s < s1; ++s) {
            if (nid[s] < 0) continue;
            int a = s % N, b = (s / N) % N, cc = s / (N * N);
            c += __popc((unsigned)emask[s]);
            for (int d = 0; d < NDIR; ++d) {
                int a2 = a - dir_dx(d), b2 = b - dir_dy(d), c2 = cc - dir_dz(d);
                if (a2 >= 0 && a2 < N && b2 >= 0 && b2 < N && c2 >= 0 && ((emask[a2 + N * (b2 + N * c2)] >> d) & 1))
                    ++c;
            }
        }
        int off = block_exscan(c, tmp, &total) + 2 * NDIR * ri.slot_base;
        for (int s = s0; s < s1; ++s) {
            if (nid[s] < 0) continue;
            int a = s % N, b = (s / N) % N, cc = s / (N * N);
            NodeRow row;
            row.gslot = ri.slot_base + s;
            row.start = off;
            for (int d = 0; d < NDIR; ++d)
                if ((emask[s] >> d) & 1) {
                    Entry e;
                    e.nbr = ri.slot_base + s + dir_off(d, N);
                    e.plane = pbase + d * SL + s;
                    A.entries[off++] = e;
                }
            row.mid = off;
            for (int d = 0; d < NDIR; ++d) {
                int a2 = a - dir_dx(d), b2 = b - dir_dy(d), c2 = cc - dir_dz(d);
                if (a2 >= 0 && a2 < N && b2 >= 0 && b2 < N && c2 >= 0) {
                    int lo = a2 + N * (b2 + N * c2);
                    if ((emask[lo] >> d) & 1) {
                        Entry e;
                        e.nbr = ri.slot_base + lo;
                        e.plane = pbase + d * SL + lo;
                        A.entries[off++] = e;
                    }
                }
            }
            row.end = off;
            A.rows[ri.slot_base + nid[s]] = row;
        }
    }

    // 9. initial state: lattice positions with the lowest node on z = 0.  An
    // absent lattice point sits far outside the robot (2e4 m plus its lattice
    // offset, beyond the 1e4 m ghost slots): the step kernels evaluate every
    // stencil spring, and an absent one (zero parameters) then never meets a
    // zero length.
    const int zc = M > 0 ? zmin_c : 0;
    for (int s = tid; s < SL; s += BT) {
        int a = s % N, b = (s / N) % N, c = s / (N * N);
        const bool here = nid[s] >= 0;
        const float far = here ? 0.f : 2e4f;
        float4 p = make_float4(far + A.voxel_len * a, far + A.voxel_len * b, far + A.voxel_len * (c - zc),
                               here ? 1.f : 0.f);
        const int g = ri.slot_base + s;
        A.x0[g] = p;
        A.x[g] = p;
        A.v[g] = make_float4(0.f, 0.f, 0.f, 0.f);
        A.slot_node[g] = nid[s];
        if (nid[s] >= 0) A.node_slot[ri.slot_base + nid[s]] = s;
    }
    if (tid == 0) {
        RobotInfo o = ri;
        o.M = M;
        o.S = S;
        A.robots_out[r] = o;
        A.diverged[r] = 0;
    }
}

}  // namespace

hipError_t launch_build_mesh(const RobotInfo *robots, int R, int max_side, const sr_sim_params &p,
                             const uint8_t *cls, const float *w, uint8_t *kept, Planes pl, int32_t *sid,
                             float4 *x0, float4 *x, float4 *v, int32_t *slot_node, int32_t *node_slot,
                             NodeRow *rows, Entry *entries, uint8_t *bad_class, uint8_t *diverged,
                             hipStream_t st) {
    (void)max_side;
    BuildArgs A;
    A.robots = robots;
    A.robots_out = const_cast<RobotInfo *>(robots);
    A.cls = cls;
    A.w = w;
    A.kept = kept;
    A.pl = pl;
    A.sid = sid;
    A.x0 = x0;
    A.x = x;
    A.v = v;
    A.slot_node = slot_node;
    A.node_slot = node_slot;
    A.rows = rows;
    A.entries = entries;
    A.bad_class = bad_class;
    A.diverged = diverged;
    for (int c = 0; c < 5; ++c) {
        A.k_class[c] = p.k_class[c];
        A.ac_cos[c] = (float)((double)p.a_class[c] * cos((double)p.phi_class[c]));
        A.ac_sin[c] = (float)((double)p.a_class[c] * sin((double)p.phi_class[c]));
        A.a_class[c] = p.a_class[c];
        A.phi_class[c] = p.phi_class[c];
    }
    A.weight_act = (p.flags & SR_WEIGHT_ACTUATION) != 0;
    A.dash2m = (float)(2.0 * (double)p.mass * (double)p.zeta_spring * (double)p.zeta_spring);
    A.voxel_len = p.voxel_len;
    hipLaunchKernelGGL(k_build_mesh, dim3(R), dim3(BT), 0, st, A);
    return hipGetLastError();
}

}  // namespace sr

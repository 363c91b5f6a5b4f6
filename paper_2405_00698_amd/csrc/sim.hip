// sim.hip -- time stepping (per-step and persistent forms), fitness, state I/O.
#include "spring.h"

namespace sr {

SimConst make_sim_const(const sr_sim_params &p) {
    SimConst c;
    c.dt = (float)p.dt;
    c.dt_m = (float)(p.dt / (double)p.mass);
    c.damping = p.damping;
    c.mg = (float)((double)p.mass * (double)p.gravity);
    c.kc = p.k_ground;
    c.mu_kc_dt_m = (float)((double)p.mu * (double)p.k_ground * p.dt / (double)p.mass);
    c.lim = (float)(1e3 * (double)p.voxel_len);
    // the same float products the mesh build uses for k * L0
    c.L0e = p.voxel_len * sqrtf(1.0f);
    c.L0f = p.voxel_len * sqrtf(2.0f);
    c.L0b = p.voxel_len * sqrtf(3.0f);
    c.mus_kc_dt_m = (float)((double)p.mu_static * (double)p.k_ground * p.dt / (double)p.mass);
    c.cg = (float)(2.0 * (double)p.zeta_ground * sqrt((double)p.k_ground * (double)p.mass));
    c.mu_dt_m = (float)((double)p.mu * p.dt / (double)p.mass);
    c.mus_dt_m = (float)((double)p.mu_static * p.dt / (double)p.mass);
    c.gravity = !(p.flags & SR_NO_GRAVITY);
    c.ground = !(p.flags & SR_NO_GROUND);
    c.actuation = !(p.flags & SR_NO_ACTUATION);
    c.gdamp = p.zeta_ground != 0.f;
    c.dash = p.zeta_spring != 0.f;
    return c;
}

namespace {

// ---------------------------------------------------------------- time table
// (sin, cos)(w t_n) for the steps of one call, t_n = n dt from the integer n.
// Without actuation the table is zero, so k L(t) = kL0.
__global__ void k_sincos(float2 *sc, const int64_t *d_step, int n, double omega_dt, int on) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!on) {
        sc[i] = make_float2(0.f, 0.f);
        return;
    }
    const double arg = omega_dt * (double)(*d_step + i);
    double s, c;
    sincos(arg, &s, &c);
    sc[i] = make_float2((float)s, (float)c);
}

__global__ void k_sincos_at(float2 *sc, int64_t step0, int n, double omega_dt, int on) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!on) {
        sc[i] = make_float2(0.f, 0.f);
        return;
    }
    const double arg = omega_dt * (double)(step0 + i);
    double s, c;
    sincos(arg, &s, &c);
    sc[i] = make_float2((float)s, (float)c);
}

__global__ void k_advance(int64_t *d_step, int n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *d_step += n;
}

// ---------------------------------------------------------------- per-step form
// One thread per node; positions and velocities in HBM, one launch per step.
// The node gathers over its incidence row (forward springs, then backward
// springs), recomputing every spring force it touches.  DASH adds the spring
// dashpots (neighbour velocities read from HBM too).
template <bool PHASE, bool DASH>
__global__ __launch_bounds__(256) void k_plain(const RobotInfo *robots, int total_slots, const int32_t *slot_robot,
                                               const NodeRow *rows, const Entry *entries, Planes pl,
                                               const float4 *__restrict__ x, const float4 *__restrict__ v,
                                               float4 *__restrict__ xn, float4 *__restrict__ vn,
                                               const float2 *sc_tab, int t, const uint8_t *diverged, SimConst c) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const float2 sc = sc_tab[t];
    if (g >= total_slots) return;
    const int r = slot_robot[g];
    const RobotInfo ri = robots[r];
    if (g - ri.slot_base >= ri.M || diverged[r]) return;
    const NodeRow row = rows[g];
    const float4 X = x[row.gslot];
    const float4 V = v[row.gslot];
    float3 Ff = make_float3(0.f, 0.f, 0.f), Fb = make_float3(0.f, 0.f, 0.f);
    for (int e = row.start; e < row.mid; ++e) {
        const Entry E = entries[e];
        const float4 Y = x[E.nbr];
        const float dx = Y.x - X.x, dy = Y.y - X.y, dz = Y.z - X.z;
        float cf;
        if constexpr (DASH) {
            const float4 VY = v[E.nbr];
            cf = spring_coef_d<PHASE>(pl.k[E.plane], pl.kL0[E.plane], pl.kal[E.plane], PHASE ? pl.kbe[E.plane] : 0.f,
                                      sc.x, sc.y, len2(dx, dy, dz), pl.kd[E.plane],
                                      rate(VY.x - V.x, VY.y - V.y, VY.z - V.z, dx, dy, dz));
        } else {
            cf = spring_coef<PHASE>(pl.k[E.plane], pl.kL0[E.plane], pl.kal[E.plane], PHASE ? pl.kbe[E.plane] : 0.f,
                                    sc.x, sc.y, len2(dx, dy, dz));
        }
        Ff.x = fmaf(cf, dx, Ff.x);
        Ff.y = fmaf(cf, dy, Ff.y);
        Ff.z = fmaf(cf, dz, Ff.z);
    }
    for (int e = row.mid; e < row.end; ++e) {
        const Entry E = entries[e];
        const float4 Y = x[E.nbr];
        const float dx = Y.x - X.x, dy = Y.y - X.y, dz = Y.z - X.z;
        float cf;
        if constexpr (DASH) {
            const float4 VY = v[E.nbr];
            cf = spring_coef_d<PHASE>(pl.k[E.plane], pl.kL0[E.plane], pl.kal[E.plane], PHASE ? pl.kbe[E.plane] : 0.f,
                                      sc.x, sc.y, len2(dx, dy, dz), pl.kd[E.plane],
                                      rate(VY.x - V.x, VY.y - V.y, VY.z - V.z, dx, dy, dz));
        } else {
            cf = spring_coef<PHASE>(pl.k[E.plane], pl.kL0[E.plane], pl.kal[E.plane], PHASE ? pl.kbe[E.plane] : 0.f,
                                    sc.x, sc.y, len2(dx, dy, dz));
        }
        Fb.x = fmaf(cf, dx, Fb.x);
        Fb.y = fmaf(cf, dy, Fb.y);
        Fb.z = fmaf(cf, dz, Fb.z);
    }
    float3 xs = make_float3(X.x, X.y, X.z);
    float3 vs = make_float3(V.x, V.y, V.z);
    integrate_node(c, xs, vs, Ff, Fb);
    xn[row.gslot] = make_float4(xs.x, xs.y, xs.z, 1.f);
    vn[row.gslot] = make_float4(vs.x, vs.y, vs.z, 0.f);
}

__global__ __launch_bounds__(256) void k_check_div(const RobotInfo *robots, const float4 *x, const float4 *v,
                                                   uint8_t *diverged, float lim_per_side) {
    __shared__ int bad;
    const RobotInfo ri = robots[blockIdx.x];
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    const float lim = lim_per_side * ri.n;
    for (int s = threadIdx.x; s < ri.slots; s += blockDim.x) {
        const float4 X = x[ri.slot_base + s], V = v[ri.slot_base + s];
        if (X.w != 0.f && node_bad(make_float3(X.x, X.y, X.z), make_float3(V.x, V.y, V.z), lim)) bad = 1;
    }
    __syncthreads();
    if (threadIdx.x == 0 && bad) diverged[blockIdx.x] = 1;
}

// ---------------------------------------------------------------- persistent form
// One workgroup holds one robot for a whole block of steps.  Positions sit in
// LDS as float4 on the dense (n+1)^3 lattice (double-buffered, with ghost
// padding so every stencil neighbour address is in range); velocities and
// spring parameters sit in VGPRs.  Each thread owns NPT lattice slots.
//
// Force assembly per step (all in a fixed order, no atomics):
//  - variant 1/2 (exchange): a slot computes the spring coefficient of each of
//    its 13 forward springs once, adds its share to its own forward sum and
//    writes the coefficient to LDS at its own index; after a barrier the upper
//    endpoint reads the coefficient of each of its 13 backward springs at the
//    lower slot's index and adds coef * (x_lower - x_self).  The coefficient
//    rows have PAD zero entries in front, which stand for the missing lower
//    neighbours of the first slots and are never written.  Variant 2 does this
//    in two direction chunks to halve the LDS buffer.
//  - variant 0 (recompute): the upper endpoint recomputes the coefficient
//    itself from the lower slot's parameters (held in its own VGPRs).
// All variants produce identical bits: each coefficient is computed from the
// same operands with the same operations.
//
// DASH (spring dashpots, Table II model): velocities are mirrored into one LDS
// buffer so a spring can read both endpoint velocities.  It is written in the
// node update, after the barrier that ends every read of the step (the
// recompute variant gets that extra barrier), and read after the end-of-step
// barrier.
struct PArgs {
    const RobotInfo *robots;
    const int32_t *list;
    int count;
    Planes pl;
    float4 *x, *v;
    const float2 *sc;
    int n_steps;
    uint8_t *diverged;
    SimConst c;
    // recording form: per step the positions x_n and the pre-friction velocity v'_n
    // of every slot, at rec_x[n_steps * slot_base + t * slots + s]; rec_u (when
    // not null) the velocity v_n at the start of the step
    float4 *rec_x, *rec_v, *rec_u;
};

// Spring parameters rebuilt from voxels (VOX): every spring touching a lattice
// point lies in one of the 8 voxels sharing that corner, so a slot can rebuild
// its forward springs' (k, k L0 a cos phi, k L0 a sin phi, dashpot) each step
// from those 8 voxels' parallel-sum terms, summed in the mesh build's voxel
// order with the same explicitly rounded operations, i.e. bit for bit the
// planes.  VOX 1 does so for the 10 face and body diagonals, VOX 2 for all 13
// directions; the registers this frees hold more slots without spilling.
// Voxel i of a slot (i = 0..7) is the one with offset (ox, oy, oz) =
// (i & 1, i >> 1 & 1, i >> 2) - 1 from the slot; the voxels of direction d are
// those whose unit cell holds both ends, in the build's (z, y, x) order.
__host__ __device__ constexpr bool from_vox(int VOX, int d) { return VOX >= 2 || (VOX == 1 && dir_len2(d) >= 2); }

// never fused into an FMA, as in the mesh build
__device__ __forceinline__ float add_nf(float a, float b) {
#pragma clang fp contract(off)
    return a + b;
}
__device__ __forceinline__ float mul_nf(float a, float b) {
#pragma clang fp contract(off)
    return a * b;
}

// Coefficient rows.  Uniform rows (one per direction of a chunk, CL entries
// each): slot s stores chunk-local direction j at j CL + PAD + s, and the
// backward read of slot s at s - off(d) stays inside the row's PAD leading
// zeros, which no chunk ever writes.  Tight rows (one chunk only): row d is
// preceded by just off(d) zeros, 13 SL + sum of off(d) entries in all, which
// lets the one-chunk exchange of the 12^3 lattice (13^3 points) fit in LDS
// beside one position buffer.  (With several chunks the rows of the later
// chunks would start elsewhere, and their leading zeros would land on the
// coefficients the first chunk wrote.)
template <int N>
__host__ __device__ constexpr int tight_row(int d) {
    int r = 0;
    for (int e = 0; e < d; ++e) r += N * N * N + dir_off(e, N);
    return r;
}
// + s: where slot s stores its forward coefficient of direction d
template <int N, bool TCR>
__host__ __device__ constexpr int coef_w(int d, int d0) {
    return TCR ? tight_row<N>(d) + dir_off(d, N) : (d - d0) * Geo<N>::CL + Geo<N>::PAD;
}
// + s: where slot s reads the coefficient of its backward spring of direction d
template <int N, bool TCR>
__host__ __device__ constexpr int coef_r(int d, int d0) {
    return TCR ? tight_row<N>(d) : (d - d0) * Geo<N>::CL + Geo<N>::PAD - dir_off(d, N);
}
template <int N, int NDC, bool TCR>
__host__ __device__ constexpr int coef_len() {
    return TCR ? tight_row<N>(NDIR) : NDC * Geo<N>::CL;
}

template <int N, int BS, int VAR, bool DASH = false, int VOX = 0, bool SBX = false, bool TCR = false>
constexpr size_t lds_bytes() {
    using G = Geo<N>;
    constexpr int NDC = VAR == 0 ? 0 : (NDIR + VAR - 1) / VAR;
    return ((SBX ? 1 : 2) + (DASH ? 1 : 0)) * sizeof(float4) * G::XL +
           sizeof(float) * (NDC > 0 ? coef_len<N, NDC, TCR>() : 0) + (VOX ? sizeof(float4) * G::CL : 0);
}

// Direction geometry as plain arithmetic, for loops over a run-time (wave-
// uniform) direction: the forward directions are the 3x3x3 neighbourhood
// cells after the centre in (dz, dy, dx) order, cell f = d + 14.  Written with
// selects on the components only, so no lookup table is built.
__host__ __device__ constexpr int rdx(int d) { return (d + 14) % 3 - 1; }
__host__ __device__ constexpr int rdy(int d) { return (d + 14) / 3 % 3 - 1; }
__host__ __device__ constexpr int rdz(int d) { return (d + 14) / 9 - 1; }
__host__ __device__ constexpr int rdir_off(int d, int N) { return rdx(d) + N * (rdy(d) + N * rdz(d)); }
__host__ __device__ constexpr int rvox_cnt(int d) {
    return (rdx(d) == 0 ? 2 : 1) * (rdy(d) == 0 ? 2 : 1) * (rdz(d) == 0 ? 2 : 1);
}
__host__ __device__ constexpr int rvox_idx(int d, int i) {
    const int dx = rdx(d), dy = rdy(d), dz = rdz(d);
    const int nx = dx == 0 ? 2 : 1, ny = dy == 0 ? 2 : 1;
    const int ix = i % nx, iy = (i / nx) % ny, iz = i / (nx * ny);
    const int ox = dx == 0 ? ix - 1 : (dx == 1 ? 0 : -1);
    const int oy = dy == 0 ? iy - 1 : (dy == 1 ? 0 : -1);
    const int oz = dz == 0 ? iz - 1 : 0;
    return (ox + 1) + 2 * (oy + 1) + 4 * (oz + 1);
}
constexpr bool rdir_matches() {
    for (int d = 0; d < NDIR; ++d) {
        if (rdx(d) != dir_dx(d) || rdy(d) != dir_dy(d) || rdz(d) != dir_dz(d) || rvox_cnt(d) != vox_cnt(d))
            return false;
        for (int i = 0; i < vox_cnt(d); ++i)
            if (rvox_idx(d, i) != vox_idx(d, i)) return false;
    }
    return true;
}
static_assert(rdir_matches(), "run-time direction geometry must equal the stencil table");

template <int V>
struct IC {
    static constexpr int value = V;
};

// Balanced slot plan (CLS kernels).  The lattice slots are cut into runs of 64
// in slot order, one wave each.  A run that lies wholly in the top plane
// (c = N - 1) has no forward spring that steps up in z (directions 4..12: their
// upper ends would lie above the lattice), and one wholly in the bottom plane
// (c = 0) no backward spring of those directions (their lower ends would lie
// below it), so such runs skip those directions: they are light in the forward
// phase of a step (top) or in the backward-and-update phase (bottom).  A
// skipped coefficient is that of a spring that does not exist: its entry keeps
// the zero written when the robot was loaded, which is what the few stencil
// reads that wrap around the lattice's edge (from slots near the top plane's
// start) find there.  The
// runs are dealt to the (slot index k, wave w) places of a workgroup, wave w
// running on SIMD w mod 4, so that the SIMDs carry equal work in each phase:
// every light run goes where the larger of the two phase maxima is smallest
// (exhaustively over the few light runs), after the runs are spread as evenly
// as the places allow.  Estimated work per run, in VALU instructions: forward
// 14 per direction, backward 6 per direction plus 25 for the node update.
enum { RUN_FULL = 0, RUN_TOP = 1, RUN_BOTTOM = 2 };

template <int N>
__host__ __device__ constexpr int run_class(int u) {
    constexpr int SL = N * N * N, P = N * N;
    const int first = 64 * u, last = (64 * u + 63 < SL ? 64 * u + 63 : SL - 1);
    return last < P ? RUN_BOTTOM : (first >= SL - P ? RUN_TOP : RUN_FULL);
}

template <int N, int BS>
struct SlotPlan {
    static constexpr int SL = N * N * N, W = BS / 64, NPT = (SL + BS - 1) / BS, U = (SL + 63) / 64;
    int unit[NPT][W];  // run held by place (k, w); -1: none
};

template <int N, int BS>
constexpr SlotPlan<N, BS> make_slot_plan() {
    using P = SlotPlan<N, BS>;
    constexpr int U = P::U, W = P::W, NPT = P::NPT;
    constexpr int FF = 13 * 14, FB = 13 * 6 + 25, TF = 4 * 14, BB = 4 * 6 + 25;
    SlotPlan<N, BS> plan{};
    int cap[4] = {0, 0, 0, 0}, cnt[4] = {0, 0, 0, 0};
    for (int w = 0; w < W; ++w) cap[w % 4] += NPT;
    for (int i = 0; i < U; ++i) {  // runs per SIMD, as even as the places allow
        int best = -1;
        for (int s = 0; s < 4; ++s)
            if (cnt[s] < cap[s] && (best < 0 || cnt[s] < cnt[best])) best = s;
        ++cnt[best];
    }
    int light[U > 0 ? U : 1] = {}, nl = 0;
    for (int u = 0; u < U; ++u)
        if (run_class<N>(u) != RUN_FULL) light[nl++] = u;
    int combos = 1;
    for (int i = 0; i < nl; ++i) combos *= 4;
    int best_code = 0, best_cost = 1 << 30;
    for (int code = 0; code < combos; ++code) {
        int nlt[4] = {0, 0, 0, 0}, f[4] = {0, 0, 0, 0}, b[4] = {0, 0, 0, 0};
        bool ok = true;
        for (int i = 0, c = code; i < nl; ++i, c /= 4) {
            const int s = c % 4;
            if (++nlt[s] > cnt[s]) ok = false;
            const bool top = run_class<N>(light[i]) == RUN_TOP;
            f[s] += top ? TF : FF;
            b[s] += top ? FB : BB;
        }
        if (!ok) continue;
        int mf = 0, mb = 0;
        for (int s = 0; s < 4; ++s) {
            f[s] += (cnt[s] - nlt[s]) * FF;
            b[s] += (cnt[s] - nlt[s]) * FB;
            mf = f[s] > mf ? f[s] : mf;
            mb = b[s] > mb ? b[s] : mb;
        }
        if (mf + mb < best_cost) {
            best_cost = mf + mb;
            best_code = code;
        }
    }
    // runs of each SIMD: its light runs, then full runs in slot order
    int simd_of[U > 0 ? U : 1] = {};
    int used[4] = {0, 0, 0, 0};
    for (int i = 0, c = best_code; i < nl; ++i, c /= 4) {
        simd_of[light[i]] = c % 4;
        ++used[c % 4];
    }
    for (int u = 0; u < U; ++u) {
        if (run_class<N>(u) != RUN_FULL) continue;
        int s = 0;
        while (used[s] >= cnt[s]) ++s;
        simd_of[u] = s;
        ++used[s];
    }
    for (int k = 0; k < NPT; ++k)
        for (int w = 0; w < W; ++w) plan.unit[k][w] = -1;
    for (int u = 0; u < U; ++u) {
        const int s = simd_of[u];
        bool placed = false;
        for (int k = 0; k < NPT && !placed; ++k)
            for (int w = s; w < W && !placed; w += 4)
                if (plan.unit[k][w] < 0) {
                    plan.unit[k][w] = u;
                    placed = true;
                }
    }
    return plan;
}

// every run placed exactly once
template <int N, int BS>
constexpr bool slot_plan_ok() {
    constexpr auto p = make_slot_plan<N, BS>();
    int seen[SlotPlan<N, BS>::U] = {};
    for (int k = 0; k < SlotPlan<N, BS>::NPT; ++k)
        for (int w = 0; w < SlotPlan<N, BS>::W; ++w)
            if (p.unit[k][w] >= 0) ++seen[p.unit[k][w]];
    for (int u = 0; u < SlotPlan<N, BS>::U; ++u)
        if (seen[u] != 1) return false;
    return true;
}

template <bool WIDEV>
struct VoxT {
    typedef float2 T;
};
template <>
struct VoxT<true> {
    typedef float4 T;
};
__device__ __forceinline__ float4 vox4(float2 v) { return make_float4(v.x, v.y, 0.f, 0.f); }
__device__ __forceinline__ float4 vox4(float4 v) { return v; }
__device__ __forceinline__ void vox_store(float2 &d, float4 v) { d = make_float2(v.x, v.y); }
__device__ __forceinline__ void vox_store(float4 &d, float4 v) { d = v; }

// Template parameters of the persistent step kernel:
//   N      lattice points per side (grid side + 1), so stencil offsets are immediates
//   BS     threads per workgroup; each thread owns ceil(N^3 / BS) lattice slots
//   VAR    0 recompute, 1 exchange coefficients through LDS, 2 in two direction chunks
//   FENCE  a scheduling barrier after each slot bounds the reads in flight
//   PHASE  the actuation has per-spring phases (k L0 a sin(phi) plane)
//   REC    recording form for the adjoint (writes x_n and v'_n every step)
//   WIDE   16-byte position reads (12-byte otherwise)
//   DASH   spring dashpots: velocities mirrored in LDS
//   VOX    1 / 2: diagonal / all springs' parameters rebuilt from voxel terms
//   SBX    one position buffer (one more barrier per step)
//   LAG, LAGB, BSWP, FSWP  how the neighbour reads are pipelined (below)
//   ROLL   0: direction loops fully unrolled; U > 0: left rolled and unrolled
//          by U, with no per-direction arrays: each iteration reads, computes
//          and stores one direction (offsets are wave-uniform)
//   CLS    the balanced slot plan: runs of 64 slots, top- and bottom-plane runs
//          skip the directions that leave the lattice
//   TCR    tight coefficient rows (one-chunk exchange, above)
//   PK     robots per workgroup: PK robots of BS / PK threads each, every one
//          with its own LDS, stepping together (small grids)
//
// LAG (exchange variants, 16-byte reads): the neighbour reads of a slot are
// issued back to back with at most LAG + 1 outstanding; the read LAG places
// earlier is waited for by keeping its .w alive, the last LAG ones where their
// direction's arithmetic needs them anyway.  LAG 0 waits for each read before
// issuing the next.  LAGB, when not negative, sets the backward-spring reads'
// lag apart from the forward ones'.  BSWP software-pipelines the backward
// springs instead: direction d's arithmetic follows the issue of direction
// d + LAGB's reads, so only a window of reads is held in registers; FSWP does
// the same for the forward springs with window LAG (and stores each
// coefficient as soon as it is computed).
template <int N, int BS, int VAR, bool FENCE, bool PHASE, bool REC = false, bool WIDE = true, bool DASH = false,
          int VOX = 0, bool SBX = false, int LAG = 0, int LAGB = -1, bool BSWP = false, bool FSWP = false,
          int ROLL = 0, bool CLS = false, bool TCR = false, int PK = 1>
__global__ __launch_bounds__(BS) void k_persist(PArgs A) {
    constexpr int BR = BS / PK;  // threads per robot
    static_assert(BS % PK == 0 && BR % 64 == 0, "whole waves per robot");
    static_assert(PK == 1 || (!CLS && !REC && ROLL == 0), "packed robots use the plain slot mapping");
    static_assert(!TCR || (VAR == 1 && ROLL == 0), "tight coefficient rows hold one chunk of unrolled directions");
    static_assert(!CLS || VAR == 1 || ROLL > 0,
                  "the balanced slot plan skips directions in the one-chunk or the rolled exchange");
    static_assert(!CLS || VAR == 0 || (NDIR + VAR - 1) / VAR >= 4, "the first chunk holds the in-plane directions");
    static_assert(ROLL == 0 || (VAR >= 1 && VOX == 2 && !DASH && !REC && WIDE && LAG == 0 && !FSWP && !BSWP),
                  "the rolled direction loop is a form of the exchange with every parameter from voxels");
    static_assert(!FSWP || (WIDE && VAR == 1 && LAG > 0),
                  "the software-pipelined forward springs are a form of the one-chunk exchange");
    constexpr int LB = LAGB < 0 ? LAG : LAGB;
    static_assert(VOX == 0 || VAR != 0, "voxel-rebuilt parameters need an exchange variant");
    static_assert((LAG == 0 && LB == 0) || VAR == 1,
                  "pipelined reads need the one-chunk exchange (constant direction indices)");
    using G = Geo<N>;
    constexpr int SL = G::SL, PAD = G::PAD, XL = G::XL, CL = G::CL;
    constexpr int NPT = (SL + BR - 1) / BR;
    constexpr int NCH = VAR == 0 ? 1 : VAR;
    constexpr int NDC = VAR == 0 ? 0 : (NDIR + VAR - 1) / VAR;
    constexpr int NQ = VAR == 0 ? NDIR : 1;  // backward parameter copies (recompute variant)
    constexpr int NB = PHASE ? NDIR : 1;
    // three distinct LDS objects, so the compiler knows coefficient stores
    // never alias position loads and can keep many loads in flight
    constexpr int CLEN = NDC > 0 ? coef_len<N, NDC, TCR>() : 1;
    typedef typename VoxT<PHASE || DASH>::T VT;
    __shared__ float4 xb0s[PK * XL];
    __shared__ float4 xb1s[SBX ? 1 : PK * XL];
    __shared__ float coefs[PK * CLEN];
    __shared__ float4 vbs[DASH ? PK * XL : 1];
    __shared__ VT vvs[VOX ? PK * CL : 1];
    __shared__ int bads[PK];
    const int tid = threadIdx.x;
    // this thread's robot j of the workgroup and its index lt among that robot's threads
    const int j = PK == 1 ? 0 : tid / BR, lt = PK == 1 ? tid : tid % BR;
    float4 *const xb0 = xb0s + j * XL;
    float4 *const xb1 = SBX ? xb1s : xb1s + j * XL;
    float *const coef = coefs + j * CLEN;
    float4 *const vb = DASH ? vbs + j * XL : vbs;
    VT *const vv = VOX ? vvs + j * CL : vvs;
    int &bad = bads[j];
    const SimConst c = A.c;
    // the lattice slot of each of this thread's NPT places: slot lt + k BR,
    // or (CLS) lane tid mod 64 of the run the balanced plan gives the wave;
    // top / bot: the wave's run lies in the top / bottom plane
    int sk[NPT];
    bool lk0[NPT], topk[NPT], botk[NPT];
    {
        const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            if constexpr (CLS) {
                static_assert(slot_plan_ok<N, BS>(), "every run placed once");
                constexpr SlotPlan<N, BS> plan = make_slot_plan<N, BS>();
                const int u = plan.unit[k][w];
                sk[k] = 64 * u + (tid & 63);
                lk0[k] = u >= 0 && sk[k] < SL;
                // wave-uniform (scalar) so that branches and loop bounds on them stay scalar
                topk[k] = __builtin_amdgcn_readfirstlane(u >= 0 && run_class<N>(u) == RUN_TOP ? 1 : 0) != 0;
                botk[k] = __builtin_amdgcn_readfirstlane(u >= 0 && run_class<N>(u) == RUN_BOTTOM ? 1 : 0) != 0;
            } else {
                sk[k] = lt + k * BR;
                lk0[k] = sk[k] < SL;
                topk[k] = false;
                botk[k] = false;
            }
        }
    }

    for (int q0 = blockIdx.x * PK; q0 < A.count; q0 += gridDim.x * PK) {
        // a packed workgroup steps all its robots together: one without a
        // robot (or with a diverged one) has no live slot but keeps the barriers
        const int q = q0 + j;
        const int r = q < A.count ? A.list[q] : 0;
        const bool act = q < A.count && !A.diverged[r];
        if (PK == 1 && !act) continue;
        bool lk[NPT];
#pragma unroll
        for (int k = 0; k < NPT; ++k) lk[k] = lk0[k] && act;
        const int base = act ? A.robots[r].slot_base : 0;
        const int pbase = NDIR * base;
        const float lim = c.lim * (N - 1);

        if (VAR != 0)
            for (int i = lt; i < CLEN; i += BR) coef[i] = 0.f;
        const float4 ghost = make_float4(1e4f, 1e4f, 1e4f, 0.f);
        for (int i = lt; i < PAD; i += BR) {
            xb0[i] = ghost;
            xb0[PAD + SL + i] = ghost;
            if constexpr (!SBX) {
                xb1[i] = ghost;
                xb1[PAD + SL + i] = ghost;
            }
            if constexpr (VOX > 0) vox_store(vv[i], make_float4(0.f, 0.f, 0.f, 0.f));
            if constexpr (DASH) {
                vb[i] = make_float4(0.f, 0.f, 0.f, 0.f);
                vb[PAD + SL + i] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
        if (lt == 0) bad = 0;

        float3 xr[NPT], vr[NPT];
        bool pres[NPT];
        float pk[NPT][NDIR], pa[NPT][NDIR], pb[NPT][NB];
        float qk[NPT][NQ], qa[NPT][NQ], qb[NPT][NQ];
        float pd[NPT][DASH ? NDIR : 1], qd[NPT][DASH ? NQ : 1];
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int s = sk[k];
            const bool live = lk[k];
            const int sc_ = live ? s : 0;
            const float4 X = A.x[base + sc_];
            const float4 V = A.v[base + sc_];
            if (live) {
                xb0[PAD + s] = X;
                if constexpr (!SBX) xb1[PAD + s] = X;
                if constexpr (DASH) vb[PAD + s] = V;
                if constexpr (VOX > 0) vox_store(vv[PAD + s], A.pl.vkp[base + s]);
            }
            xr[k] = make_float3(X.x, X.y, X.z);
            vr[k] = make_float3(V.x, V.y, V.z);
            pres[k] = live && X.w != 0.f;
#pragma unroll
            for (int d = 0; d < NDIR; ++d) {
                if (from_vox(VOX, d)) continue;
                const int pi = pbase + d * SL + sc_;
                pk[k][d] = live ? A.pl.k[pi] : 0.f;
                pa[k][d] = live ? A.pl.kal[pi] : 0.f;
                if (PHASE) pb[k][d] = live ? A.pl.kbe[pi] : 0.f;
                if constexpr (DASH) pd[k][d] = live ? A.pl.kd[pi] : 0.f;
            }
            if (VAR == 0) {
#pragma unroll
                for (int d = 0; d < NQ; ++d) {
                    const int lo = s - dir_off(d, N);
                    const bool ok = live && lo >= 0;
                    const int pi = pbase + d * SL + (ok ? lo : 0);
                    qk[k][d] = ok ? A.pl.k[pi] : 0.f;
                    qa[k][d] = ok ? A.pl.kal[pi] : 0.f;
                    qb[k][d] = (ok && PHASE) ? A.pl.kbe[pi] : 0.f;
                    if constexpr (DASH) qd[k][d] = ok ? A.pl.kd[pi] : 0.f;
                }
            }
        }
        // a wave whose 64 slots are all absent lattice points has no spring to
        // evaluate: its forward coefficients stay the zeros written above, and
        // absent points are never integrated, so it skips both phases
        bool wk[NPT];
#pragma unroll
        for (int k = 0; k < NPT; ++k) wk[k] = lk[k] && __ballot(pres[k] ? 1 : 0) != 0ull;
        __syncthreads();

        float2 sc_next = A.sc[0];
        for (int t = 0; t < A.n_steps; ++t) {
            const float2 sct = sc_next;
            if (t + 1 < A.n_steps) sc_next = A.sc[t + 1];
            const float4 *const xc = (SBX || !(t & 1)) ? xb0 : xb1;
            float4 *const xn = (SBX || (t & 1)) ? xb0 : xb1;
            float3 Ff[NPT], Fb[NPT];
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                Ff[k] = make_float3(0.f, 0.f, 0.f);
                Fb[k] = make_float3(0.f, 0.f, 0.f);
            }
            if (VAR == 0) {
#pragma unroll
                for (int k = 0; k < NPT; ++k) {
                    const int s = sk[k];
                    if (wk[k]) {
#pragma unroll
                        for (int d = 0; d < NDIR; ++d) {
                            const float3 Y = ldx<WIDE>(xc + s + (PAD + dir_off(d, N)));
                            const float dx = Y.x - xr[k].x, dy = Y.y - xr[k].y, dz = Y.z - xr[k].z;
                            float cf;
                            if constexpr (DASH) {
                                const float3 VY = ldx<WIDE>(vb + s + (PAD + dir_off(d, N)));
                                cf = spring_coef_d<PHASE>(pk[k][d], pk[k][d] * L0d(c, d), pa[k][d],
                                                          PHASE ? pb[k][d] : 0.f, sct.x, sct.y, len2(dx, dy, dz),
                                                          pd[k][d],
                                                          rate(VY.x - vr[k].x, VY.y - vr[k].y, VY.z - vr[k].z, dx, dy, dz));
                            } else {
                                cf = spring_coef<PHASE>(pk[k][d], pk[k][d] * L0d(c, d), pa[k][d],
                                                        PHASE ? pb[k][d] : 0.f, sct.x, sct.y, len2(dx, dy, dz));
                            }
                            Ff[k].x = fmaf(cf, dx, Ff[k].x);
                            Ff[k].y = fmaf(cf, dy, Ff[k].y);
                            Ff[k].z = fmaf(cf, dz, Ff[k].z);
                        }
#pragma unroll
                        for (int d = 0; d < NQ; ++d) {
                            const float3 Y = ldx<WIDE>(xc + s + (PAD - dir_off(d, N)));
                            const float ex = Y.x - xr[k].x, ey = Y.y - xr[k].y, ez = Y.z - xr[k].z;
                            float cf;
                            if constexpr (DASH) {
                                const float3 VY = ldx<WIDE>(vb + s + (PAD - dir_off(d, N)));
                                cf = spring_coef_d<PHASE>(qk[k][d], qk[k][d] * L0d(c, d), qa[k][d], qb[k][d], sct.x,
                                                          sct.y, len2(ex, ey, ez), qd[k][d],
                                                          rate(VY.x - vr[k].x, VY.y - vr[k].y, VY.z - vr[k].z, ex, ey, ez));
                            } else {
                                cf = spring_coef<PHASE>(qk[k][d], qk[k][d] * L0d(c, d), qa[k][d], qb[k][d], sct.x,
                                                        sct.y, len2(ex, ey, ez));
                            }
                            Fb[k].x = fmaf(cf, ex, Fb[k].x);
                            Fb[k].y = fmaf(cf, ey, Fb[k].y);
                            Fb[k].z = fmaf(cf, ez, Fb[k].z);
                        }
                    }
                }
            } else if constexpr (ROLL > 0) {
                // Rolled form: one direction per iteration and nothing indexed by
                // it but LDS addresses, so no per-direction arrays go to scratch.
                // The operations and their order are those of the unrolled form.
                // The chunk loop unrolls, so each direction loop has a constant
                // trip count (a runtime one would stay rolled: its body holds
                // inline asm, which the unroller will not give a remainder loop).
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    const int d0 = ch * NDC;
                    const int d1 = (ch + 1) * NDC < NDIR ? (ch + 1) * NDC : NDIR;
                    if constexpr (SR_POISON_LDS) {
                        // only the entries this phase writes: a top-plane run's skipped
                        // directions keep the zeros of the robot's start (below)
#pragma unroll
                        for (int k = 0; k < NPT; ++k)
                            if (wk[k]) {
                                const int dw = (CLS && topk[k]) ? (d1 < 4 ? d1 : 4) : d1;
                                for (int d = d0; d < dw; ++d) coef[(d - d0) * CL + PAD + sk[k]] = __builtin_nanf("");
                            }
                    }
#pragma unroll
                    for (int k = 0; k < NPT; ++k) {
                        const int s = sk[k];
                        if (wk[k]) {
                            const float4 *xs = xc + s;
                            float *cs = coef + s;
                            int vo = PAD + s;
                            __asm__ volatile("" : "+v"(vo));
                            auto fwd = [&](int d) {
                                const float4 q = xs[PAD + rdir_off(d, N)];
                                keep_w(q.w);
                                const float dx = q.x - xr[k].x, dy = q.y - xr[k].y, dz = q.z - xr[k].z;
                                float4 sm = vox4(vv[vo + vox_off(rvox_idx(d, 0), N)]);
                                const int cnt = rvox_cnt(d);
                                for (int i = 1; i < cnt; ++i) {
                                    const float4 u = vox4(vv[vo + vox_off(rvox_idx(d, i), N)]);
                                    sm.x = add_nf(sm.x, u.x);
                                    sm.y = add_nf(sm.y, u.y);
                                    if (PHASE) sm.z = add_nf(sm.z, u.z);
                                }
                                const int l2 = rdx(d) * rdx(d) + rdy(d) * rdy(d) + rdz(d) * rdz(d);
                                const float L0 = l2 == 1 ? c.L0e : l2 == 2 ? c.L0f : c.L0b;
                                const float kk = sm.x;
                                const float cf = spring_coef<PHASE>(kk, kk * L0, mul_nf(sm.y, L0),
                                                                    PHASE ? mul_nf(sm.z, L0) : 0.f, sct.x, sct.y,
                                                                    len2(dx, dy, dz));
                                cs[(d - d0) * CL + PAD] = cf;
                                Ff[k].x = fmaf(cf, dx, Ff[k].x);
                                Ff[k].y = fmaf(cf, dy, Ff[k].y);
                                Ff[k].z = fmaf(cf, dz, Ff[k].z);
                            };
                            // a top-plane run has only the four in-plane directions, all in
                            // the first chunk (constant trip count, so the loop unrolls)
                            if (CLS && topk[k]) {
                                if (ch == 0) {
#pragma unroll ROLL
                                    for (int d = 0; d < 4; ++d) fwd(d);
                                }
                            } else {
#pragma unroll ROLL
                                for (int d = d0; d < d1; ++d) fwd(d);
                            }
                        }
                        if (FENCE) __builtin_amdgcn_sched_barrier(0);
                    }
                    __syncthreads();
#pragma unroll
                    for (int k = 0; k < NPT; ++k) {
                        const int s = sk[k];
                        if (wk[k]) {
                            const float4 *xs = xc + s;
                            const float *cs = coef + s;
                            auto bwd = [&](int d) {
                                const float4 q = xs[PAD - rdir_off(d, N)];
                                const float cf = cs[(d - d0) * CL + (PAD - rdir_off(d, N))];
                                keep_w(q.w);
                                const float ex = q.x - xr[k].x, ey = q.y - xr[k].y, ez = q.z - xr[k].z;
                                Fb[k].x = fmaf(cf, ex, Fb[k].x);
                                Fb[k].y = fmaf(cf, ey, Fb[k].y);
                                Fb[k].z = fmaf(cf, ez, Fb[k].z);
                            };
                            // a bottom-plane run has only the four in-plane directions
                            if (CLS && botk[k]) {
                                if (ch == 0) {
#pragma unroll ROLL
                                    for (int d = 0; d < 4; ++d) bwd(d);
                                }
                            } else {
#pragma unroll ROLL
                                for (int d = d0; d < d1; ++d) bwd(d);
                            }
                        }
                        if (FENCE) __builtin_amdgcn_sched_barrier(0);
                    }
                    if (ch + 1 < NCH) __syncthreads();
                }
            } else {
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    const int d0 = ch * NDC;
                    const int d1 = (ch + 1) * NDC < NDIR ? (ch + 1) * NDC : NDIR;
                    if constexpr (SR_POISON_LDS) {
                        // only the entries this phase writes: a top-plane run's skipped
                        // directions keep the zeros of the robot's start (below)
#pragma unroll
                        for (int k = 0; k < NPT; ++k)
                            if (wk[k]) {
                                const int dw = (CLS && topk[k]) ? (d1 < 4 ? d1 : 4) : d1;
                                for (int d = d0; d < dw; ++d) coef[coef_w<N, TCR>(d, d0) + sk[k]] = __builtin_nanf("");
                            }
                    }
#pragma unroll
                    for (int k = 0; k < NPT; ++k) {
                        const int s = sk[k];
                        if (wk[k]) {
                            // every neighbour read of this slot is issued before any use;
                            // addresses are one base plus non-negative immediates
                            const float4 *xs = xc + s;
                            float *cs = coef + s;
                            // forward springs of directions d0 .. DE - 1: a run in the top
                            // plane has only the four that stay in the plane
                            auto forward = [&](auto DEC) {
                                constexpr int DE = decltype(DEC)::value;
                                const int de = DE < d1 ? DE : d1;
                                if constexpr (FSWP) {
                                    float4 Q[NDIR], QV[DASH ? NDIR : 1];
                                    float4 Vx[VOX > 0 ? 8 : 1];
                                    if constexpr (VOX > 0) {
                                        // re-read every step (see below)
                                        int vo = PAD + s;
                                        __asm__ volatile("" : "+v"(vo));
    #pragma unroll
                                        for (int i = 0; i < 8; ++i) Vx[i] = vox4(vv[vo + vox_off(i, N)]);
                                    }
    #pragma unroll
                                    for (int d = 0; d < NDIR; ++d)
                                        if (d >= d0 && d < de && d < d0 + LAG) {
                                            Q[d] = xs[PAD + dir_off(d, N)];
                                            if constexpr (DASH) QV[DASH ? d : 0] = vb[s + PAD + dir_off(d, N)];
                                        }
    #pragma unroll
                                    for (int d = 0; d < NDIR; ++d) {
                                        if (d < d0 || d >= de) continue;
                                        const int e = d + LAG < de ? d + LAG : d0;
                                        if (d + LAG < de) {
                                            Q[e] = xs[PAD + dir_off(e, N)];
                                            if constexpr (DASH) QV[DASH ? e : 0] = vb[s + PAD + dir_off(e, N)];
                                        }
                                        keep_w(Q[d].w);
                                        if constexpr (DASH) keep_w(QV[DASH ? d : 0].w);
                                        const float dx = Q[d].x - xr[k].x, dy = Q[d].y - xr[k].y, dz = Q[d].z - xr[k].z;
                                        float kk, al, be, cd;
                                        if (from_vox(VOX, d)) {
                                            float4 sm = Vx[VOX > 0 ? vox_idx(d, 0) : 0];
    #pragma unroll
                                            for (int i = 1; i < vox_cnt(d); ++i) {
                                                const float4 u = Vx[VOX > 0 ? vox_idx(d, i) : 0];
                                                sm.x = add_nf(sm.x, u.x);
                                                sm.y = add_nf(sm.y, u.y);
                                                if (PHASE) sm.z = add_nf(sm.z, u.z);
                                                if (DASH) sm.w = add_nf(sm.w, u.w);
                                            }
                                            kk = sm.x;
                                            al = mul_nf(sm.y, L0d(c, d));
                                            be = PHASE ? mul_nf(sm.z, L0d(c, d)) : 0.f;
                                            cd = sm.w;
                                        } else {
                                            kk = pk[k][d];
                                            al = pa[k][d];
                                            be = PHASE ? pb[k][d] : 0.f;
                                            cd = DASH ? pd[k][DASH ? d : 0] : 0.f;
                                        }
                                        float cf;
                                        if constexpr (DASH) {
                                            const float4 W = QV[DASH ? d : 0];
                                            cf = spring_coef_d<PHASE>(kk, kk * L0d(c, d), al, be, sct.x, sct.y, len2(dx, dy, dz),
                                                                      cd,
                                                                      rate(W.x - vr[k].x, W.y - vr[k].y, W.z - vr[k].z, dx, dy, dz));
                                        } else {
                                            cf = spring_coef<PHASE>(kk, kk * L0d(c, d), al, be, sct.x, sct.y, len2(dx, dy, dz));
                                        }
                                        cs[coef_w<N, TCR>(d, d0)] = cf;
                                        Ff[k].x = fmaf(cf, dx, Ff[k].x);
                                        Ff[k].y = fmaf(cf, dy, Ff[k].y);
                                        Ff[k].z = fmaf(cf, dz, Ff[k].z);
                                    }
                                } else {
                                float3 Y[NDIR], VY[DASH ? NDIR : 1];
                                float Wk[NDIR], Wv[DASH ? NDIR : 1];
                                if constexpr (WIDE && LAG > 0) {
    #pragma unroll
                                    for (int d = d0; d < de; ++d) {
                                        const float4 q = xs[PAD + dir_off(d, N)];
                                        Y[d] = make_float3(q.x, q.y, q.z);
                                        Wk[d] = q.w;
                                        if constexpr (DASH) {
                                            const float4 u = vb[s + PAD + dir_off(d, N)];
                                            VY[DASH ? d : 0] = make_float3(u.x, u.y, u.z);
                                            Wv[DASH ? d : 0] = u.w;
                                        }
                                        if (d - LAG >= d0) {
                                            keep_w(Wk[d - LAG >= 0 ? d - LAG : 0]);
                                            if constexpr (DASH) keep_w(Wv[DASH && d - LAG >= 0 ? d - LAG : 0]);
                                        }
                                    }
                                } else {
    #pragma unroll
                                    for (int d = d0; d < de; ++d) Y[d] = ldx<WIDE>(xs + (PAD + dir_off(d, N)));
                                }
                                if constexpr (DASH && !(WIDE && LAG > 0)) {
    #pragma unroll
                                    for (int d = d0; d < de; ++d) VY[DASH ? d : 0] = ldx<WIDE>(vb + s + (PAD + dir_off(d, N)));
                                }
                                float4 Vx[VOX > 0 ? 8 : 1];
                                if constexpr (VOX > 0) {
                                    // the voxel terms never change, but they must be re-read every
                                    // step: hoisting them out of the time loop would hold them in
                                    // registers, which is what this variant avoids
                                    int vo = PAD + s;
                                    __asm__ volatile("" : "+v"(vo));
    #pragma unroll
                                    for (int i = 0; i < 8; ++i) Vx[i] = vox4(vv[vo + vox_off(i, N)]);
                                }
                                float cfv[NDIR];
    #pragma unroll
                                for (int d = d0; d < de; ++d) {
                                    if constexpr (WIDE && LAG > 0) {
                                        if (d + LAG >= de) {
                                            keep_w(Wk[d]);
                                            if constexpr (DASH) keep_w(Wv[DASH ? d : 0]);
                                        }
                                    }
                                    const float dx = Y[d].x - xr[k].x, dy = Y[d].y - xr[k].y, dz = Y[d].z - xr[k].z;
                                    float kk, al, be, cd;
                                    if (from_vox(VOX, d)) {
                                        // the build's sums, term by term in its order
                                        float4 sm = Vx[VOX > 0 ? vox_idx(d, 0) : 0];
    #pragma unroll
                                        for (int i = 1; i < vox_cnt(d); ++i) {
                                            const float4 u = Vx[VOX > 0 ? vox_idx(d, i) : 0];
                                            sm.x = add_nf(sm.x, u.x);
                                            sm.y = add_nf(sm.y, u.y);
                                            if (PHASE) sm.z = add_nf(sm.z, u.z);
                                            if (DASH) sm.w = add_nf(sm.w, u.w);
                                        }
                                        kk = sm.x;
                                        al = mul_nf(sm.y, L0d(c, d));
                                        be = PHASE ? mul_nf(sm.z, L0d(c, d)) : 0.f;
                                        cd = sm.w;
                                    } else {
                                        kk = pk[k][d];
                                        al = pa[k][d];
                                        be = PHASE ? pb[k][d] : 0.f;
                                        cd = DASH ? pd[k][DASH ? d : 0] : 0.f;
                                    }
                                    float cf;
                                    if constexpr (DASH) {
                                        const float3 W = VY[DASH ? d : 0];
                                        cf = spring_coef_d<PHASE>(kk, kk * L0d(c, d), al, be, sct.x, sct.y, len2(dx, dy, dz),
                                                                  cd,
                                                                  rate(W.x - vr[k].x, W.y - vr[k].y, W.z - vr[k].z, dx, dy, dz));
                                    } else {
                                        cf = spring_coef<PHASE>(kk, kk * L0d(c, d), al, be, sct.x, sct.y, len2(dx, dy, dz));
                                    }
                                    cfv[d] = cf;
                                    Ff[k].x = fmaf(cf, dx, Ff[k].x);
                                    Ff[k].y = fmaf(cf, dy, Ff[k].y);
                                    Ff[k].z = fmaf(cf, dz, Ff[k].z);
                                }
    #pragma unroll
                                for (int d = d0; d < de; ++d) cs[coef_w<N, TCR>(d, d0)] = cfv[d];
                                }
                            };
                            if (CLS && topk[k])
                                forward(IC<4>{});
                            else
                                forward(IC<NDIR>{});
                        }
                        if (FENCE) __builtin_amdgcn_sched_barrier(0);
                    }
                    __syncthreads();
#pragma unroll
                    for (int k = 0; k < NPT; ++k) {
                        const int s = sk[k];
                        if (wk[k]) {
                            const float4 *xs = xc + s;
                            const float *cs = coef + s;
                            // backward springs of directions d0 .. DE - 1: a run in the bottom
                            // plane has only the four that stay in the plane
                            auto backward = [&](auto DEC) {
                                constexpr int DE = decltype(DEC)::value;
                                const int de = DE < d1 ? DE : d1;
                                float3 Y[NDIR];
                                float cfv[NDIR], Wk[NDIR];
                                if constexpr (WIDE && BSWP) {
                                    float4 Q[NDIR];
    #pragma unroll
                                    for (int d = 0; d < NDIR; ++d) {
                                        if (d < d0 || d >= de || d >= d0 + LB) continue;
                                        Q[d] = xs[PAD - dir_off(d, N)];
                                        cfv[d] = cs[coef_r<N, TCR>(d, d0)];
                                    }
    #pragma unroll
                                    for (int d = 0; d < NDIR; ++d) {
                                        if (d < d0 || d >= de) continue;
                                        const int e = d + LB < de ? d + LB : d0;
                                        if (d + LB < de) {
                                            Q[e] = xs[PAD - dir_off(e, N)];
                                            cfv[e] = cs[coef_r<N, TCR>(e, d0)];
                                        }
                                        keep_w(Q[d].w);
                                        const float ex = Q[d].x - xr[k].x, ey = Q[d].y - xr[k].y, ez = Q[d].z - xr[k].z;
                                        Fb[k].x = fmaf(cfv[d], ex, Fb[k].x);
                                        Fb[k].y = fmaf(cfv[d], ey, Fb[k].y);
                                        Fb[k].z = fmaf(cfv[d], ez, Fb[k].z);
                                    }
                                } else {
    #pragma unroll
                                for (int d = d0; d < de; ++d) {
                                    if constexpr (WIDE && LB > 0) {
                                        const float4 q = xs[PAD - dir_off(d, N)];
                                        Y[d] = make_float3(q.x, q.y, q.z);
                                        Wk[d] = q.w;
                                        if (d - LB >= d0) keep_w(Wk[d - LB >= 0 ? d - LB : 0]);
                                    } else {
                                        Y[d] = ldx<WIDE>(xs + (PAD - dir_off(d, N)));
                                    }
                                    cfv[d] = cs[coef_r<N, TCR>(d, d0)];
                                }
    #pragma unroll
                                for (int d = d0; d < de; ++d) {
                                    if constexpr (WIDE && LB > 0) {
                                        if (d + LB >= de) keep_w(Wk[d]);
                                    }
                                    const float ex = Y[d].x - xr[k].x, ey = Y[d].y - xr[k].y, ez = Y[d].z - xr[k].z;
                                    Fb[k].x = fmaf(cfv[d], ex, Fb[k].x);
                                    Fb[k].y = fmaf(cfv[d], ey, Fb[k].y);
                                    Fb[k].z = fmaf(cfv[d], ez, Fb[k].z);
                                }
                                }
                            };
                            if (CLS && botk[k])
                                backward(IC<4>{});
                            else
                                backward(IC<NDIR>{});
                        }
                        if (FENCE) __builtin_amdgcn_sched_barrier(0);
                    }
                    if (ch + 1 < NCH) __syncthreads();
                }
            }
            // every velocity read (dashpots, recompute variant) or position read
            // (single position buffer) of the step is done before the update
            if constexpr ((DASH && VAR == 0) || SBX) __syncthreads();
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                const int s = sk[k];
                if (pres[k]) {
                    float3 vp;
                    if (REC) A.rec_x[(size_t)A.n_steps * base + (size_t)t * SL + s] = make_float4(xr[k].x, xr[k].y, xr[k].z, 1.f);
                    if (REC && A.rec_u)
                        A.rec_u[(size_t)A.n_steps * base + (size_t)t * SL + s] = make_float4(vr[k].x, vr[k].y, vr[k].z, 0.f);
                    integrate_node(c, xr[k], vr[k], Ff[k], Fb[k], REC ? &vp : nullptr);
                    if (REC) A.rec_v[(size_t)A.n_steps * base + (size_t)t * SL + s] = make_float4(vp.x, vp.y, vp.z, 0.f);
                    xn[PAD + s] = make_float4(xr[k].x, xr[k].y, xr[k].z, 1.f);
                    if constexpr (DASH) vb[PAD + s] = make_float4(vr[k].x, vr[k].y, vr[k].z, 0.f);
                }
            }
            __syncthreads();
        }

        bool mybad = false;
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int s = sk[k];
            if (pres[k]) {
                A.x[base + s] = make_float4(xr[k].x, xr[k].y, xr[k].z, 1.f);
                A.v[base + s] = make_float4(vr[k].x, vr[k].y, vr[k].z, 0.f);
                mybad |= node_bad(xr[k], vr[k], lim);
            }
        }
        if (mybad) bad = 1;
        __syncthreads();
        if (lt == 0 && bad && act) A.diverged[r] = 1;
        __syncthreads();
    }
}

// ---------------------------------------------------------------- fitness
__global__ __launch_bounds__(256) void k_fitness(const RobotInfo *robots, const float4 *x, const float4 *x0,
                                                 const uint8_t *diverged, float *fit) {
    __shared__ float part[4];
    const RobotInfo ri = robots[blockIdx.x];
    float s = 0.f;
    for (int q = threadIdx.x; q < ri.slots; q += 256) {
        const float4 X0 = x0[ri.slot_base + q];
        if (X0.w != 0.f) s += x[ri.slot_base + q].x - X0.x;
    }
    // fixed-order wave tree, then waves in order
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float tot = (part[0] + part[1]) + (part[2] + part[3]);
        // a robot with no kept voxel has no body to move: worst fitness
        float f = ri.M > 0 ? tot / (float)ri.M : -INFINITY;
        if (diverged[blockIdx.x] || !(fabsf(f) <= 3.0e38f)) f = -INFINITY;
        fit[blockIdx.x] = f;
    }
}

// ---------------------------------------------------------------- state / spring I/O
__global__ void k_gather_state(const RobotInfo *robots, int total_slots, const int32_t *slot_robot,
                               const int32_t *slot_node, const int64_t *mass_off, float4 *x, float4 *v, float *xo,
                               float *vo, int scatter) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total_slots) return;
    const int id = slot_node[g];
    if (id < 0) return;
    const int64_t o = 3 * (mass_off[slot_robot[g]] + id);
    if (!scatter) {
        const float4 X = x[g], V = v[g];
        if (xo) { xo[o] = X.x; xo[o + 1] = X.y; xo[o + 2] = X.z; }
        if (vo) { vo[o] = V.x; vo[o + 1] = V.y; vo[o + 2] = V.z; }
    } else {
        if (xo) x[g] = make_float4(xo[o], xo[o + 1], xo[o + 2], 1.f);
        if (vo) v[g] = make_float4(vo[o], vo[o + 1], vo[o + 2], 0.f);
    }
}

__global__ void k_springs_io(const RobotInfo *robots, int total_slots, const int32_t *slot_robot,
                             const int32_t *slot_node, const int32_t *sid, const int64_t *spring_off, Planes pl,
                             float voxel_len, int32_t *ij, float *L0o, float *ko, float *ao, float *phio,
                             const float *kin, const float *ain, const float *phin, int write) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total_slots) return;
    const int r = slot_robot[g];
    const RobotInfo ri = robots[r];
    const int s = g - ri.slot_base;
    for (int d = 0; d < NDIR; ++d) {
        const int pi = NDIR * ri.slot_base + d * ri.slots + s;
        const int id = sid[pi];
        if (id < 0) continue;
        const int64_t o = spring_off[r] + id;
        const float L0 = voxel_len * sqrtf((float)dir_len2(d));
        if (!write) {
            if (ij) {
                ij[2 * o] = slot_node[g];
                ij[2 * o + 1] = slot_node[g + dir_off(d, ri.N)];
            }
            if (L0o) L0o[o] = L0;
            const float k = pl.k[pi], kL0 = pl.kL0[pi], kal = pl.kal[pi], kbe = pl.kbe[pi];
            float a = 0.f, ph = 0.f;
            if (kL0 != 0.f) {
                if (kbe == 0.f) a = kal / kL0;
                else {
                    a = sqrtf(kal * kal + kbe * kbe) / kL0;
                    ph = atan2f(kbe, kal);
                }
            }
            if (ko) ko[o] = k;
            if (ao) ao[o] = a;
            if (phio) phio[o] = ph;
        } else {
            // read the current values for fields that are not given
            float k = pl.k[pi], kL0 = pl.kL0[pi], kal = pl.kal[pi], kbe = pl.kbe[pi];
            float a = 0.f, ph = 0.f;
            if (kL0 != 0.f) {
                if (kbe == 0.f) a = kal / kL0;
                else {
                    a = sqrtf(kal * kal + kbe * kbe) / kL0;
                    ph = atan2f(kbe, kal);
                }
            }
            if (kin) k = kin[o];
            if (ain) a = ain[o];
            if (phin) ph = phin[o];
            pl.k[pi] = k;
            pl.kL0[pi] = k * L0;
            if (ph == 0.f) {
                pl.kal[pi] = k * L0 * a;
                pl.kbe[pi] = 0.f;
            } else {
                pl.kal[pi] = k * L0 * a * cosf(ph);
                pl.kbe[pi] = k * L0 * a * sinf(ph);
            }
        }
    }
}

// ---------------------------------------------------------------- persistent dispatch table
typedef void (*PersistFn)(PArgs);
struct PersistEntry {
    int n, block, variant;
    PersistFn fn, fn_phase;
    size_t lds;
    int pack = 1;  // robots per workgroup
};

// Variant codes (the sum documented at pop_set_persist_variant): exchange
// variant (0, 1, 2); + 4 scheduling fences bound the LDS loads in flight; + 8
// 12-byte instead of 16-byte position loads; + 16 spring-dashpot kernels;
// + 32 * VOX spring parameters of the face and body diagonals (VOX 1) or of
// every direction (VOX 2) rebuilt from voxels each step; + 128 one position
// buffer (one more barrier per step, less LDS); + 256 * LAG pipelined 16-byte
// neighbour reads; + 4096 * (LB + 1) a separate backward lag; + 131072 / + 262144
// software-pipelined backward / forward springs; + 2097152 rolled direction
// loops with every parameter from voxels, + 4194304 * (U - 1) unrolled by U;
// + 524288 the balanced slot plan (top- and bottom-plane runs skip the
// directions that leave the lattice, runs dealt evenly over the SIMDs);
// + 1048576 tight coefficient rows; + 16777216 * (PK - 1) PK robots per
// workgroup.
// Every entry's LDS arrays must fit one CU's 160 KiB (checked at compile time
// here, and for the code objects as built by a CPU test, since the compiler may
// add LDS of its own).
template <size_t B>
constexpr size_t lds_ok() {
    static_assert(B <= 160 * 1024, "persistent kernel configuration exceeds the 160 KiB of LDS per CU");
    return B;
}
#define SR_PE(NN, BS, VAR, F, W)                                                                        \
    {                                                                                                   \
        NN, BS, VAR + 4 * F + 8 * (1 - W), k_persist<NN + 1, BS, VAR, F, false, false, W>,              \
            k_persist<NN + 1, BS, VAR, F, true, false, W>, lds_ok<lds_bytes<NN + 1, BS, VAR>()>()                 \
    }
#define SR_PLF(NN, BS, F, LF, LB, BSW)                                                                     \
    {                                                                                                        \
        NN, BS, 1 + 4 * F + 256 * LF + 4096 * (LB + 1) + 131072 * BSW + 262144,                              \
            k_persist<NN + 1, BS, 1, F, false, false, true, false, 0, false, LF, LB, BSW, true>,             \
            k_persist<NN + 1, BS, 1, F, true, false, true, false, 0, false, LF, LB, BSW, true>,              \
            lds_ok<lds_bytes<NN + 1, BS, 1>()>()                                                                       \
    }
// + 524288: the balanced slot plan with top- and bottom-plane runs skipping
// the directions that leave the lattice (CLS)
#define SR_PLSC(NN, BS, F, LF, LB)                                                                         \
    {                                                                                                        \
        NN, BS, 1 + 4 * F + 256 * LF + 4096 * (LB + 1) + 131072 + 524288,                                    \
            k_persist<NN + 1, BS, 1, F, false, false, true, false, 0, false, LF, LB, true, false, 0, true>,  \
            k_persist<NN + 1, BS, 1, F, true, false, true, false, 0, false, LF, LB, true, false, 0, true>,   \
            lds_ok<lds_bytes<NN + 1, BS, 1>()>()                                                                       \
    }
// several small robots per workgroup (the default pipelined form)
#define SR_PLFP(NN, BR, PK)                                                                                  \
    {                                                                                                        \
        NN, BR * PK, 1 + 256 * 3 + 4096 * 4 + 131072 + 262144 + 16777216 * (PK - 1),                         \
            k_persist<NN + 1, BR * PK, 1, false, false, false, true, false, 0, false, 3, 3, true, true, 0, false, false, PK>, \
            k_persist<NN + 1, BR * PK, 1, false, true, false, true, false, 0, false, 3, 3, true, true, 0, false, false, PK>,  \
            lds_ok<PK * lds_bytes<NN + 1, BR * PK, 1>()>(), PK                                                \
    }
// + 1048576: tight coefficient rows (with the balanced slot plan, software-
// pipelined backward springs, optionally pipelined forward ones and one
// position buffer)
#define SR_PLT(NN, BS, F, LF, LB, SBX, FSW)                                                                 \
    {                                                                                                        \
        NN, BS, 1 + 4 * F + 128 * SBX + 256 * LF + 4096 * (LB + 1) + 131072 + 262144 * FSW + 524288 + 1048576, \
            k_persist<NN + 1, BS, 1, F, false, false, true, false, 0, SBX, LF, LB, true, FSW, 0, true, true>,  \
            k_persist<NN + 1, BS, 1, F, true, false, true, false, 0, SBX, LF, LB, true, FSW, 0, true, true>,   \
            lds_ok<lds_bytes<NN + 1, BS, 1, false, 0, SBX, true>()>()                                                  \
    }
#define SR_PRUC(NN, BS, VAR, SBX, F, U)                                                                      \
    {                                                                                                        \
        NN, BS, VAR + 4 * F + 64 + 128 * SBX + 2097152 + 4194304 * (U - 1) + 524288,                         \
            k_persist<NN + 1, BS, VAR, F, false, false, true, false, 2, SBX, 0, -1, false, false, U, true>,  \
            k_persist<NN + 1, BS, VAR, F, true, false, true, false, 2, SBX, 0, -1, false, false, U, true>,   \
            lds_ok<lds_bytes<NN + 1, BS, VAR, false, 2, SBX>()>()                                                      \
    }
#define SR_PVL(NN, BS, VAR, VOX, SBX, F, LG)                                                              \
    {                                                                                                        \
        NN, BS, VAR + 4 * F + 32 * VOX + 128 * SBX + 256 * LG,                                               \
            k_persist<NN + 1, BS, VAR, F, false, false, true, false, VOX, SBX, LG>,                          \
            k_persist<NN + 1, BS, VAR, F, true, false, true, false, VOX, SBX, LG>,                           \
            lds_ok<lds_bytes<NN + 1, BS, VAR, false, VOX, SBX>()>()                                                    \
    }
// dashpot kernels with the balanced slot plan and tight coefficient rows
#define SR_PDT(NN, BS, LF, LB, SBX)                                                                         \
    {                                                                                                        \
        NN, BS, 1 + 16 + 128 * SBX + 256 * LF + 4096 * (LB + 1) + 131072 + 262144 + 524288 + 1048576,         \
            k_persist<NN + 1, BS, 1, false, true, false, true, true, 0, SBX, LF, LB, true, true, 0, true, true>, \
            k_persist<NN + 1, BS, 1, false, true, false, true, true, 0, SBX, LF, LB, true, true, 0, true, true>, \
            lds_ok<lds_bytes<NN + 1, BS, 1, true, 0, SBX, true>()>()                                                   \
    }
// two-chunk dashpot exchange with one position buffer (12^3)
#define SR_PDC(NN, BS)                                                                                       \
    {                                                                                                        \
        NN, BS, 2 + 16 + 128, k_persist<NN + 1, BS, 2, false, true, false, true, true, 0, true>,              \
            k_persist<NN + 1, BS, 2, false, true, false, true, true, 0, true>,                                   \
            lds_ok<lds_bytes<NN + 1, BS, 2, true, 0, true>()>()                                                  \
    }
// dashpot kernels carry the phase plane always (with a zero plane the results
// are the same bits as without it); SR_PDF / SR_PDVF software-pipeline their
// position and velocity reads
#define SR_PD(NN, BS, VAR)                                                                              \
    {                                                                                                   \
        NN, BS, VAR + 16, k_persist<NN + 1, BS, VAR, false, true, false, true, true>,                   \
            k_persist<NN + 1, BS, VAR, false, true, false, true, true>, lds_ok<lds_bytes<NN + 1, BS, VAR, true>()>() \
    }
#define SR_PDF(NN, BS, LF, LB)                                                                              \
    {                                                                                                        \
        NN, BS, 1 + 16 + 256 * LF + 4096 * (LB + 1) + 131072 + 262144,                                       \
            k_persist<NN + 1, BS, 1, false, true, false, true, true, 0, false, LF, LB, true, true>,          \
            k_persist<NN + 1, BS, 1, false, true, false, true, true, 0, false, LF, LB, true, true>,          \
            lds_ok<lds_bytes<NN + 1, BS, 1, true>()>()                                                                 \
    }
#define SR_PDVF(NN, BS, VOX, SBX, LF, LB)                                                                   \
    {                                                                                                        \
        NN, BS, 1 + 16 + 32 * VOX + 128 * SBX + 256 * LF + 4096 * (LB + 1) + 131072 + 262144,                \
            k_persist<NN + 1, BS, 1, false, true, false, true, true, VOX, SBX, LF, LB, true, true>,          \
            k_persist<NN + 1, BS, 1, false, true, false, true, true, VOX, SBX, LF, LB, true, true>,          \
            lds_ok<lds_bytes<NN + 1, BS, 1, true, VOX, SBX>()>()                                                       \
    }

// The first entry of each side is its default configuration, the first one
// without voxel terms the default when the spring parameters were set directly.
// The table keeps, per side, the configurations a measured workload chose
// (4096 robots of 10^3; the sides of the uneven population; the Table II model
// at 5^3 and 8^3) and the plain one-chunk exchange as a cross-check of the
// pipelined forms; the configurations measured slower are not compiled.
const PersistEntry kPersist[] = {
    // defaults
    SR_PE(1, 64, 1, 0, 1),      SR_PE(2, 64, 1, 0, 1),      SR_PE(3, 64, 1, 0, 1),
    SR_PLF(4, 128, 0, 3, 3, 1), SR_PLF(5, 256, 0, 3, 3, 1), SR_PLF(6, 384, 0, 3, 3, 1), SR_PLF(7, 512, 0, 3, 3, 1),
    SR_PLF(8, 768, 0, 3, 3, 1), SR_PLF(9, 1024, 0, 3, 3, 1), SR_PLT(10, 768, 0, 2, 2, 0, 1),
    SR_PLT(11, 1024, 0, 2, 2, 0, 1), SR_PLT(12, 768, 0, 3, 2, 1, 1),
    // the next best measured
    SR_PLT(10, 768, 0, 3, 3, 0, 1), SR_PLSC(10, 512, 0, 12, 3),
    SR_PLT(11, 896, 0, 2, 2, 0, 1), SR_PRUC(11, 896, 1, 1, 1, 3), SR_PVL(11, 256, 1, 2, 1, 1, 4),
    SR_PLT(12, 768, 0, 2, 2, 1, 1), SR_PRUC(12, 768, 2, 1, 1, 3),
    SR_PLT(8, 768, 0, 3, 3, 0, 1),  // slot plan at 8^3: 3 % faster with one robot per CU, slower with two
    // several small robots per workgroup (measured slower in the uneven population)
    SR_PLFP(4, 128, 4), SR_PLFP(5, 256, 2), SR_PLFP(6, 384, 2),
    // plain one-chunk exchange (cross-check of the pipelined forms) and the recompute variant
    SR_PE(4, 128, 1, 0, 1),     SR_PE(5, 256, 1, 0, 1),     SR_PE(6, 384, 1, 0, 1),     SR_PE(7, 512, 1, 0, 1),
    SR_PE(8, 768, 1, 0, 1),     SR_PE(9, 1024, 1, 0, 1),    SR_PE(10, 512, 1, 0, 1),    SR_PE(10, 704, 0, 0, 1),
    // spring dashpots (Table II model)
    SR_PD(1, 64, 1),            SR_PD(2, 64, 1),            SR_PD(3, 64, 1),
    SR_PDF(4, 128, 3, 3),       SR_PDF(5, 256, 3, 3),       SR_PDF(6, 384, 3, 3),       SR_PDF(7, 512, 3, 3),
    SR_PDF(8, 768, 3, 3),       SR_PDF(9, 1024, 3, 3),      SR_PDT(10, 768, 2, 2, 1),   SR_PDT(11, 1024, 1, 1, 1),
    SR_PDC(12, 768),            SR_PDVF(10, 704, 2, 1, 3, 3),
    SR_PD(8, 768, 1),
};

#define SR_REC(NN, BS, VAR) \
    { NN, BS, VAR, k_persist<NN + 1, BS, VAR, false, false, true>, k_persist<NN + 1, BS, VAR, false, true, true>, 0 }
#define SR_RECL(NN, BS, LF, LB, SW)                                                                      \
    {                                                                                                    \
        NN, BS, 1, k_persist<NN + 1, BS, 1, false, false, true, true, false, 0, false, LF, LB, SW, SW>, \
            k_persist<NN + 1, BS, 1, false, true, true, true, false, 0, false, LF, LB, SW, SW>, 0        \
    }

// recording forms of the tight-row kernels (balanced slot plan, software-
// pipelined springs, optionally one position buffer)
#define SR_RECT(NN, BS, LF, LB, SBX)                                                                             \
    {                                                                                                          \
        NN, BS, 1, k_persist<NN + 1, BS, 1, false, false, true, true, false, 0, SBX, LF, LB, true, true, 0, true, true>, \
            k_persist<NN + 1, BS, 1, false, true, true, true, false, 0, SBX, LF, LB, true, true, 0, true, true>, 0      \
    }

// recording forms (used to recompute checkpointed segments for the adjoint)
const PersistEntry kRec[] = {
    SR_REC(1, 64, 1),            SR_REC(2, 64, 1),            SR_REC(3, 64, 1),            SR_RECL(4, 128, 4, 4, false),
    SR_RECL(5, 256, 4, 4, false), SR_RECL(6, 384, 4, 4, false), SR_RECL(7, 512, 4, 4, false), SR_RECL(8, 768, 3, 3, true),
    SR_RECL(9, 1024, 3, 3, true), SR_RECT(10, 768, 2, 2, 0),    SR_RECT(11, 1024, 2, 2, 0),  SR_RECT(12, 768, 3, 2, 1),
};

// recording forms of the spring-dashpot kernels (they carry the phase plane)
#define SR_RECD(NN, BS, VAR)                                                                               \
    {                                                                                                       \
        NN, BS, VAR + 16, k_persist<NN + 1, BS, VAR, false, true, true, true, true>,                        \
            k_persist<NN + 1, BS, VAR, false, true, true, true, true>, 0                                    \
    }
// recording forms of the pipelined, tight-row and two-chunk dashpot kernels
#define SR_RECDF(NN, BS, LF, LB)                                                                             \
    {                                                                                                       \
        NN, BS, 1 + 16, k_persist<NN + 1, BS, 1, false, true, true, true, true, 0, false, LF, LB, true, true>, \
            k_persist<NN + 1, BS, 1, false, true, true, true, true, 0, false, LF, LB, true, true>, 0          \
    }
#define SR_RECDT(NN, BS, LF, LB, SBX)                                                                        \
    {                                                                                                       \
        NN, BS, 1 + 16,                                                                                     \
            k_persist<NN + 1, BS, 1, false, true, true, true, true, 0, SBX, LF, LB, true, true, 0, true, true>, \
            k_persist<NN + 1, BS, 1, false, true, true, true, true, 0, SBX, LF, LB, true, true, 0, true, true>, 0 \
    }
#define SR_RECDC(NN, BS)                                                                                     \
    {                                                                                                       \
        NN, BS, 2 + 16, k_persist<NN + 1, BS, 2, false, true, true, true, true, 0, true>,                     \
            k_persist<NN + 1, BS, 2, false, true, true, true, true, 0, true>, 0                               \
    }
const PersistEntry kRecD[] = {
    SR_RECD(1, 64, 1),         SR_RECD(2, 64, 1),          SR_RECD(3, 64, 1),         SR_RECDF(4, 128, 3, 3),
    SR_RECDF(5, 256, 3, 3),    SR_RECDF(6, 384, 3, 3),     SR_RECDF(7, 512, 3, 3),    SR_RECDF(8, 768, 3, 3),
    SR_RECDF(9, 1024, 3, 3),   SR_RECDT(10, 768, 2, 2, 1), SR_RECDT(11, 1024, 1, 1, 1), SR_RECDC(12, 768),
};

const PersistEntry *find_persist(const PersistCfg &cfg) {
    for (const auto &e : kPersist)
        if (e.n == cfg.n && e.block == cfg.block && e.variant == cfg.variant) return &e;
    return nullptr;
}

}  // namespace

bool persist_supported(const PersistCfg &cfg, bool phase) {
    (void)phase;
    return find_persist(cfg) != nullptr;
}

size_t persist_lds_bytes(const PersistCfg &cfg) {
    const PersistEntry *e = find_persist(cfg);
    return e ? e->lds : 0;
}

int persist_list(int n, int32_t *blocks, int32_t *variants, int cap) {
    int cnt = 0;
    for (const auto &e : kPersist)
        if (e.n == n) {
            if (cnt < cap) {
                if (blocks) blocks[cnt] = e.block;
                if (variants) variants[cnt] = e.variant;
            }
            ++cnt;
        }
    return cnt;
}

int persist_default_block(int n, bool dash, bool vox, int *variant) {
    for (const auto &e : kPersist)
        if (e.n == n && ((e.variant & 16) != 0) == dash && (vox || !(e.variant & 96))) {
            *variant = e.variant;
            return e.block;
        }
    return 0;
}

hipError_t launch_persistent(const PersistCfg &cfg, bool phase, const RobotInfo *robots, const int32_t *list, int count,
                             int grid, Planes pl, float4 *x, float4 *v, const float2 *sc, int n_steps,
                             uint8_t *diverged, SimConst c, hipStream_t st) {
    const PersistEntry *e = find_persist(cfg);
    if (!e) return hipErrorInvalidConfiguration;
    PArgs A;
    A.robots = robots;
    A.list = list;
    A.count = count;
    A.pl = pl;
    A.x = x;
    A.v = v;
    A.sc = sc;
    A.n_steps = n_steps;
    A.diverged = diverged;
    A.c = c;
    A.rec_x = nullptr;
    A.rec_v = nullptr;
    A.rec_u = nullptr;
    PersistFn fn = phase ? e->fn_phase : e->fn;
    hipLaunchKernelGGL(fn, dim3((grid + e->pack - 1) / e->pack), dim3(e->block), 0, st, A);
    return hipGetLastError();
}

hipError_t launch_record(int n, bool phase, const RobotInfo *robots, const int32_t *list, int count, Planes pl,
                         float4 *x, float4 *v, const float2 *sc, int n_steps, uint8_t *diverged, SimConst c,
                         float4 *rec_x, float4 *rec_v, float4 *rec_u, hipStream_t st) {
    // the spring-dashpot model records with the dashpot kernels (the same bits
    // as its production kernels)
    const PersistEntry *e = nullptr;
    if (c.dash) {
        for (const auto &q : kRecD)
            if (q.n == n) e = &q;
    } else {
        for (const auto &q : kRec)
            if (q.n == n) e = &q;
    }
    if (!e) return hipErrorInvalidConfiguration;
    PArgs A;
    A.robots = robots;
    A.list = list;
    A.count = count;
    A.pl = pl;
    A.x = x;
    A.v = v;
    A.sc = sc;
    A.n_steps = n_steps;
    A.diverged = diverged;
    A.c = c;
    A.rec_x = rec_x;
    A.rec_v = rec_v;
    A.rec_u = rec_u;
    hipLaunchKernelGGL(phase ? e->fn_phase : e->fn, dim3(count), dim3(e->block), 0, st, A);
    return hipGetLastError();
}

hipError_t launch_sincos(float2 *sc, const int64_t *d_step, int n, double omega_dt, int on, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sincos, dim3((n + 255) / 256), dim3(256), 0, st, sc, d_step, n, omega_dt, on);
    return hipGetLastError();
}

hipError_t launch_sincos_at(float2 *sc, int64_t step0, int n, double omega_dt, int on, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sincos_at, dim3((n + 255) / 256), dim3(256), 0, st, sc, step0, n, omega_dt, on);
    return hipGetLastError();
}

hipError_t launch_advance(int64_t *d_step, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, d_step, n);
    return hipGetLastError();
}

hipError_t launch_plain_step(const RobotInfo *robots, int R, int total_slots, const NodeRow *rows, const Entry *entries,
                             Planes pl, const float4 *x, const float4 *v, float4 *xn, float4 *vn, const float2 *sc,
                             int t, bool phase, const uint8_t *diverged, const int32_t *slot_robot, SimConst c,
                             hipStream_t st) {
    (void)R;
    auto fn = c.dash ? (phase ? k_plain<true, true> : k_plain<false, true>)
                     : (phase ? k_plain<true, false> : k_plain<false, false>);
    hipLaunchKernelGGL(fn, dim3((total_slots + 255) / 256), dim3(256), 0, st, robots, total_slots, slot_robot, rows,
                       entries, pl, x, v, xn, vn, sc, t, diverged, c);
    return hipGetLastError();
}

hipError_t launch_check_div(const RobotInfo *robots, int R, const float4 *x, const float4 *v, uint8_t *diverged,
                            float lim, hipStream_t st) {
    hipLaunchKernelGGL(k_check_div, dim3(R), dim3(256), 0, st, robots, x, v, diverged, lim);
    return hipGetLastError();
}

hipError_t launch_fitness(const RobotInfo *robots, int R, const float4 *x, const float4 *x0, const uint8_t *diverged,
                          float *fit, hipStream_t st) {
    hipLaunchKernelGGL(k_fitness, dim3(R), dim3(256), 0, st, robots, x, x0, diverged, fit);
    return hipGetLastError();
}

hipError_t launch_gather_state(const RobotInfo *robots, int R, int total_slots, const int32_t *slot_robot,
                               const int32_t *slot_node, const int64_t *mass_off, const float4 *x, const float4 *v,
                               float *xo, float *vo, int scatter, hipStream_t st) {
    (void)R;
    hipLaunchKernelGGL(k_gather_state, dim3((total_slots + 255) / 256), dim3(256), 0, st, robots, total_slots,
                       slot_robot, slot_node, mass_off, const_cast<float4 *>(x), const_cast<float4 *>(v), xo, vo,
                       scatter);
    return hipGetLastError();
}

hipError_t launch_springs_io(const RobotInfo *robots, int R, int total_slots, const int32_t *slot_robot,
                             const int32_t *slot_node, const int32_t *sid, const int64_t *spring_off, Planes pl,
                             float voxel_len, int32_t *ij, float *L0, float *k, float *a, float *phi,
                             const float *k_in, const float *a_in, const float *phi_in, int write, hipStream_t st) {
    (void)R;
    hipLaunchKernelGGL(k_springs_io, dim3((total_slots + 255) / 256), dim3(256), 0, st, robots, total_slots,
                       slot_robot, slot_node, sid, spring_off, pl, voxel_len, ij, L0, k, a, phi, k_in, a_in, phi_in,
                       write);
    return hipGetLastError();
}

}  // namespace sr

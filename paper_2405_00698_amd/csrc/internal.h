// internal.h -- declarations shared by the library's own translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/softrobot.h"

namespace sr {

// Lattice stencil.  Every spring of a voxel robot joins two lattice points of
// one voxel, so it points along one of 13 directions up to sign: 3 edges,
// 6 face diagonals, 4 body diagonals.  They are listed in lexicographic
// (dz, dy, dx) order, which is the order of the neighbour's lattice index, so a
// node's forward springs come out in canonical (lower id, higher id) order.
constexpr int NDIR = 13;
__host__ __device__ constexpr int dir_dx(int d) {
    return d == 0 ? 1 : d == 1 ? -1 : d == 2 ? 0 : d == 3 ? 1 : d == 4 ? -1 : d == 5 ? 0 : d == 6 ? 1
         : d == 7 ? -1 : d == 8 ? 0 : d == 9 ? 1 : d == 10 ? -1 : d == 11 ? 0 : 1;
}
__host__ __device__ constexpr int dir_dy(int d) {
    return d == 0 ? 0 : d == 1 ? 1 : d == 2 ? 1 : d == 3 ? 1 : d <= 6 ? -1 : d <= 9 ? 0 : 1;
}
__host__ __device__ constexpr int dir_dz(int d) { return d <= 3 ? 0 : 1; }
// squared lattice length: 1 edge, 2 face diagonal, 3 body diagonal
__host__ __device__ constexpr int dir_len2(int d) {
    return dir_dx(d) * dir_dx(d) + dir_dy(d) * dir_dy(d) + dir_dz(d) * dir_dz(d);
}
// linear offset of direction d on a lattice of side N (index a + N (b + N c))
__host__ __device__ constexpr int dir_off(int d, int N) { return dir_dx(d) + N * (dir_dy(d) + N * dir_dz(d)); }

// The voxels of a spring: voxel i (0..7) around a lattice point is the one
// with offset (ox, oy, oz) = (i & 1, i >> 1 & 1, i >> 2) - 1, and the forward
// spring of direction d from that point lies in vox_cnt(d) of them (4 for an
// edge, 2 for a face diagonal, 1 for a body diagonal), listed by vox_idx in the
// mesh build's (z, y, x) order.
__host__ __device__ constexpr int vox_cnt(int d) {
    return (dir_dx(d) == 0 ? 2 : 1) * (dir_dy(d) == 0 ? 2 : 1) * (dir_dz(d) == 0 ? 2 : 1);
}
__host__ __device__ constexpr int vox_idx(int d, int i) {
    const int nx = dir_dx(d) == 0 ? 2 : 1, ny = dir_dy(d) == 0 ? 2 : 1;
    const int ix = i % nx, iy = (i / nx) % ny, iz = i / (nx * ny);
    const int ox = dir_dx(d) == 0 ? ix - 1 : (dir_dx(d) == 1 ? 0 : -1);
    const int oy = dir_dy(d) == 0 ? iy - 1 : (dir_dy(d) == 1 ? 0 : -1);
    const int oz = dir_dz(d) == 0 ? iz - 1 : 0;
    return (ox + 1) + 2 * (oy + 1) + 4 * (oz + 1);
}
__host__ __device__ constexpr int vox_off(int i, int N) { return ((i & 1) - 1) + N * (((i >> 1) & 1) - 1) + N * N * ((i >> 2) - 1); }

// Per-robot metadata, device resident.
struct RobotInfo {
    int32_t n;          // voxels per side
    int32_t N;          // lattice points per side, n + 1
    int32_t slots;      // N^3
    int32_t slot_base;  // offset of the robot's lattice slots in slot-indexed arrays
    int32_t vox_base;   // offset of its voxels in voxel arrays
    int32_t M;          // nodes (written by the build)
    int32_t S;          // springs (written by the build)
    int32_t pad;
};

// Spring parameters live in four stencil planes, each [13][slots] per robot
// (plane index 13 * slot_base + d * slots + lower_slot):
//   k     stiffness (0 where no spring)
//   kL0   k * L0
//   kal   k * L0 * a cos(phi)   (coefficient of sin(w t) in k L(t))
//   kbe   k * L0 * a sin(phi)   (coefficient of cos(w t))
// so that k L(t) = kL0 + kal sin(w t) + kbe cos(w t); and
//   kd    dashpot coefficient c beside the spring (Table II model; 0 otherwise).
struct Planes {
    float *k, *kL0, *kal, *kbe, *kd;
    // per slot: the parallel-sum terms (k_c w, k_c w a cos, k_c w a sin, dashpot)
    // of the voxel whose lowest corner is the slot; the planes above are the
    // explicitly rounded sums of these over each spring's voxels
    float4 *vkp;
};

// Node incidence for the per-step kernel: for node i of a robot (slot-space
// index slot_base + i), its global slot and the ranges of its forward
// (lower endpoint) and backward (upper endpoint) entries.
struct NodeRow {
    int32_t gslot, start, mid, end;
};
struct Entry {
    int32_t nbr;   // global slot of the other endpoint
    int32_t plane; // global plane index of the spring
};

struct SimConst {
    float dt, dt_m, damping, mg, kc, mu_kc_dt_m, lim;
    float L0e, L0f, L0b;  // rest lengths of edge, face-diagonal, body-diagonal springs
    // Table II contact terms: static friction threshold factor (mu_static k_ground
    // dt / m), ground damper c_g and the friction factors per unit normal force
    // (mu dt / m, mu_static dt / m) used when the damper is on
    float mus_kc_dt_m, cg, mu_dt_m, mus_dt_m;
    int32_t gravity, ground, actuation, gdamp, dash;
};

SimConst make_sim_const(const sr_sim_params &p);

// ---- kernels (launchers); each returns hipError_t of the launch ----
hipError_t launch_build_mesh(const RobotInfo *robots, int R, int max_side, const sr_sim_params &p,
                             const uint8_t *cls, const float *w, uint8_t *kept, Planes pl,
                             int32_t *sid, float4 *x0, float4 *x, float4 *v, int32_t *slot_node,
                             int32_t *node_slot, NodeRow *rows, Entry *entries, uint8_t *bad_class,
                             uint8_t *diverged, hipStream_t st);

hipError_t launch_query(const RobotInfo *robots, int R, int max_side, const float *genomes, const float *B,
                        int precision, uint8_t *cls, float *w, hipStream_t st);

hipError_t launch_ga(const float *fit, const float *gin, float *gout, int P, int L, int E, int k, uint64_t pc,
                     uint64_t pm, float sigma, uint64_t seed, uint64_t gen, int32_t *dec, hipStream_t st);

hipError_t launch_micro(int which, int iters, int grid, float *out, hipStream_t st, double *units);
hipError_t launch_micro_hbm(const float4 *src, float4 *dst, size_t n, int grid, int passes, hipStream_t st,
                            double *units);

hipError_t launch_sincos(float2 *sc, const int64_t *d_step, int n, double omega_dt, int on, hipStream_t st);
hipError_t launch_sincos_at(float2 *sc, int64_t step0, int n, double omega_dt, int on, hipStream_t st);

// recording forward for the adjoint: x_n and the pre-friction velocity v'_n of
// every step, and (rec_u not null: dashpots or a damped ground) v_n as well
hipError_t launch_record(int n, bool phase, const RobotInfo *robots, const int32_t *list, int count, Planes pl,
                         float4 *x, float4 *v, const float2 *sc, int n_steps, uint8_t *diverged, SimConst c,
                         float4 *rec_x, float4 *rec_v, float4 *rec_u, hipStream_t st);
// reverse step over one recorded segment; for a side whose adjoint is split
// (adjoint_is_split), rec_l (a buffer like rec_x) takes lambda_F of every step
// and launch_adj_grad then forms the segment's parameter-gradient sums
bool adjoint_is_split(int n, bool vel);
hipError_t launch_adj_grad(int n, bool phase, const RobotInfo *robots, const int32_t *list, int count, Planes pl,
                           const float4 *x0, const float4 *rec_x, const float4 *rec_u, float4 *rec_l, int n_steps,
                           const float2 *sc, float *gk, float *gs, float *gc, float *gd, SimConst c, hipStream_t st);
hipError_t launch_adjoint(int n, bool phase, const RobotInfo *robots, const int32_t *list, int count, Planes pl,
                          const float4 *x0, const float4 *rec_x, const float4 *rec_v, const float4 *rec_u,
                          float4 *rec_l, int n_steps, const float2 *sc, float4 *lx, float4 *lv, float *gk, float *gs,
                          float *gc, float *gd, SimConst c, hipStream_t st);
hipError_t launch_adj_init(const RobotInfo *robots, int total_slots, const int32_t *slot_robot, const float4 *x0,
                           const float *dJ, float4 *lx, float4 *lv, float *gk, float *gs, float *gc, float *gd,
                           hipStream_t st);
hipError_t launch_adj_springs(const RobotInfo *robots, int total_slots, const int32_t *slot_robot, const int32_t *sid,
                              const int64_t *spring_off, Planes pl, float voxel_len, const float *gk, const float *gs,
                              const float *gc, float *g_k, float *g_a, float *g_phi, hipStream_t st);
hipError_t launch_adj_genome(const RobotInfo *robots, int R, int total_vox, const int32_t *vox_robot,
                             const uint8_t *kept, const float *w, Planes pl, const float *gk, const float *gs,
                             const float *gc, const float *gd, const sr_sim_params &p, const float *genomes,
                             const float *B, float *dJdw, float *g_gen, hipStream_t st);
hipError_t launch_advance(int64_t *d_step, int n, hipStream_t st);

hipError_t launch_plain_step(const RobotInfo *robots, int R, int total_slots, const NodeRow *rows,
                             const Entry *entries, Planes pl, const float4 *x, const float4 *v,
                             float4 *xn, float4 *vn, const float2 *sc, int t, bool phase,
                             const uint8_t *diverged, const int32_t *slot_robot, SimConst c, hipStream_t st);

hipError_t launch_check_div(const RobotInfo *robots, int R, const float4 *x, const float4 *v,
                            uint8_t *diverged, float lim, hipStream_t st);

// persistent LDS-resident kernel for robots of side n; `list` holds the robot
// ids to step (all of side n).  variant: 0 recompute, 1 exchange, 2 exchange
// in two direction chunks (+4 fences, +8 12-byte loads, +16 spring dashpots,
// +32/+64 parameters rebuilt from voxels, +128 one position buffer).
struct PersistCfg {
    int n, block, variant;
};
bool persist_supported(const PersistCfg &cfg, bool phase);
int persist_default_block(int n, bool dash, bool vox, int *variant);
int persist_list(int n, int32_t *blocks, int32_t *variants, int cap);
size_t persist_lds_bytes(const PersistCfg &cfg);
hipError_t launch_persistent(const PersistCfg &cfg, bool phase, const RobotInfo *robots, const int32_t *list,
                             int count, int grid, Planes pl, float4 *x, float4 *v, const float2 *sc,
                             int n_steps, uint8_t *diverged, SimConst c, hipStream_t st);

hipError_t launch_fitness(const RobotInfo *robots, int R, const float4 *x, const float4 *x0,
                          const uint8_t *diverged, float *fit, hipStream_t st);

hipError_t launch_gather_state(const RobotInfo *robots, int R, int total_slots, const int32_t *slot_robot,
                               const int32_t *slot_node, const int64_t *mass_off, const float4 *x,
                               const float4 *v, float *xo, float *vo, int scatter, hipStream_t st);

hipError_t launch_springs_io(const RobotInfo *robots, int R, int total_slots, const int32_t *slot_robot,
                             const int32_t *slot_node, const int32_t *sid, const int64_t *spring_off,
                             Planes pl, float voxel_len, int32_t *ij, float *L0, float *k, float *a,
                             float *phi, const float *k_in, const float *a_in, const float *phi_in,
                             int write, hipStream_t st);

}  // namespace sr

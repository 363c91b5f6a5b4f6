// spring.h -- the per-spring force coefficient and the per-node update, shared
// by the per-step kernel and the persistent kernel so that both produce the
// same bits for the same state.
#pragma once

#include "internal.h"

// Debug build (SR_POISON_LDS = 1): at the start of each exchange phase every
// thread fills its own slots' exchange entries in LDS with NaN before it
// writes them, so an entry read without having been written in that phase (a
// missing barrier, a skipped direction that is read after all) shows up as a
// NaN in the results.  Product builds compile it out.
#ifndef SR_POISON_LDS
#define SR_POISON_LDS 0
#endif

namespace sr {

// Dense lattice of a robot with side n (N = n + 1 points per side) as held in
// LDS: SL slots, PAD ghost slots before and after (the largest stencil offset
// is N^2 + N + 1), XL = SL + 2 PAD; CL is one coefficient row (PAD zero
// entries in front of SL slot entries).
template <int N>
struct Geo {
    static constexpr int SL = N * N * N;
    static constexpr int PAD = N * N + N + 1;
    static constexpr int XL = SL + 2 * PAD;
    static constexpr int CL = SL + PAD;
};

// Hooke spring with actuated rest length L(t) = L0 (1 + a sin(w t + phi)):
// the force on the lower endpoint is k (r - L) d / r = (k - k L / r) d, with
// d = x_upper - x_lower.  k L = kL0 + kal S + kbe C with (S, C) = (sin, cos)(w t).
// Returns the scalar coefficient of d.  An absent spring (all parameters zero)
// contributes an exact zero as long as r^2 > 0: every stencil neighbour of a
// lattice point is another point, an absent lattice point (held far outside
// the robot, each at its own place) or a ghost slot (farther still), so only
// a spring collapsed to zero length meets r^2 = 0, and its non-finite force
// flags the robot as diverged.
template <bool PHASE>
__device__ __forceinline__ float spring_coef(float k, float kL0, float kal, float kbe, float S, float C,
                                             float r2) {
    float kL = fmaf(kal, S, kL0);
    if (PHASE) kL = fmaf(kbe, C, kL);
    const float ir = __builtin_amdgcn_rsqf(r2);
    return fmaf(-kL, ir, k);
}

// The same with a dashpot of coefficient kd beside the spring: the force on
// the lower endpoint gains kd ((v_upper - v_lower).d / r) d / r, i.e. the
// coefficient of d gains kd vr / r^2 with vr = (v_upper - v_lower).d.  Swapping
// the endpoints negates both differences, so either end gets the same bits.
template <bool PHASE>
__device__ __forceinline__ float spring_coef_d(float k, float kL0, float kal, float kbe, float S, float C, float r2,
                                               float kd, float vr) {
    float kL = fmaf(kal, S, kL0);
    if (PHASE) kL = fmaf(kbe, C, kL);
    const float ir = __builtin_amdgcn_rsqf(r2);
    return fmaf(kd * vr, ir * ir, fmaf(-kL, ir, k));
}

__device__ __forceinline__ float rate(float dvx, float dvy, float dvz, float dx, float dy, float dz) {
    return fmaf(dvz, dz, fmaf(dvy, dy, dvx * dx));
}

// rest length of direction d: voxel edge times 1, sqrt 2 or sqrt 3
__device__ __forceinline__ float L0d(const SimConst &c, int d) {
    return dir_len2(d) == 1 ? c.L0e : dir_len2(d) == 2 ? c.L0f : c.L0b;
}

// xyz of a float4 slot.  A full 16-byte LDS read: on gfx950 ds_read_b128
// streams at about twice the rate of ds_read_b96 (measured 113 vs 54 TB/s).
// The empty asm keeps .w alive so the load is not narrowed back to 12 bytes.
__device__ __forceinline__ float3 ld3(const float4 *p) {
    const float4 v = *p;
    __asm__("" ::"v"(v.w));
    return make_float3(v.x, v.y, v.z);
}

// Keeps a loaded .w alive without using it: the empty asm makes the compiler
// wait for that one load (and keeps the load 16 bytes wide), nothing else.
__device__ __forceinline__ void keep_w(float w) { __asm__("" ::"v"(w)); }

// xyz of a float4 slot as one 12-byte read (fewer registers in flight).
typedef float f3v __attribute__((ext_vector_type(3)));
__device__ __forceinline__ float3 ld3n(const float4 *p) {
    const f3v v = *reinterpret_cast<const f3v *>(__builtin_assume_aligned(p, 16));
    return make_float3(v.x, v.y, v.z);
}

template <bool WIDE>
__device__ __forceinline__ float3 ldx(const float4 *p) {
    return WIDE ? ld3(p) : ld3n(p);
}

__device__ __forceinline__ float len2(float dx, float dy, float dz) { return fmaf(dz, dz, fmaf(dy, dy, dx * dx)); }

// One node's update from its total spring force (forward-direction sum Ff and
// backward-direction sum Fb, added in that order): gravity, ground normal
// (with the Table II contact damper, clamped at zero, when c.gdamp), semi-
// implicit Euler, velocity-level Coulomb friction (sticking within the larger
// of the static and kinetic thresholds), damping.
__device__ __forceinline__ void integrate_node(const SimConst &c, float3 &x, float3 &v, float3 Ff, float3 Fb,
                                               float3 *vprime = nullptr) {
    float Fx = Ff.x + Fb.x, Fy = Ff.y + Fb.y, Fz = Ff.z + Fb.z;
    const bool below = c.ground && x.z < 0.f;
    if (c.gravity) Fz -= c.mg;
    float Nf = 0.f;
    if (below) {
        if (c.gdamp) {
            Nf = fmaxf(fmaf(-c.cg, v.z, c.kc * -x.z), 0.f);
            Fz += Nf;
        } else {
            Fz = fmaf(c.kc, -x.z, Fz);
        }
    }
    float vx = fmaf(c.dt_m, Fx, v.x), vy = fmaf(c.dt_m, Fy, v.y), vz = fmaf(c.dt_m, Fz, v.z);
    if (vprime) *vprime = make_float3(vx, vy, vz);
    if (below) {
        const float dv = c.gdamp ? c.mu_dt_m * Nf : c.mu_kc_dt_m * (-x.z);
        const float dvs = c.gdamp ? c.mus_dt_m * Nf : c.mus_kc_dt_m * (-x.z);
        const float u = sqrtf(fmaf(vy, vy, vx * vx));
        if (u <= fmaxf(dv, dvs)) {
            vx = 0.f;
            vy = 0.f;
        } else {
            const float s = 1.f - dv / u;
            vx *= s;
            vy *= s;
        }
    }
    v.x = c.damping * vx;
    v.y = c.damping * vy;
    v.z = c.damping * vz;
    x.x = fmaf(c.dt, v.x, x.x);
    x.y = fmaf(c.dt, v.y, x.y);
    x.z = fmaf(c.dt, v.z, x.z);
}

__device__ __forceinline__ bool node_bad(float3 x, float3 v, float lim) {
    // NaN fails every comparison, so test the good range and negate
    const bool ok = fabsf(x.x) <= lim && fabsf(x.y) <= lim && fabsf(x.z) <= lim && fabsf(v.x) <= 3.0e38f &&
                    fabsf(v.y) <= 3.0e38f && fabsf(v.z) <= 3.0e38f;
    return !ok;
}

}  // namespace sr

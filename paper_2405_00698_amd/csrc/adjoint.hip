// adjoint.hip -- reverse-mode gradient of J = sum_r g_r fitness_r through the
// time steps, the spring parameters, the parallel-sum rule and the genome MLP.
//
// Forward step n (all nodes, positions x_n): F = springs(x_n, t_n) + gravity +
// ground(z_n); v' = v_n + dt F / m; v'' = friction(v', z_n); v_{n+1} = damping v'';
// x_{n+1} = x_n + dt v_{n+1}.  Its reverse, for adjoints (lx, lv) of (x_{n+1}, v_{n+1}):
//   lvt = damping (lv + dt lx);  lv' = friction Jacobian^T lvt (and a z term);
//   lF = dt/m lv';  lv_n = lv';  lx_n = lx + ground/friction z terms + sum over
//   springs of K_s (lF_hi - lF_lo) (to the lower end, minus to the upper end),
// with K_s = k [(1 - L/r)(I - d^ d^T) + d^ d^T] the spring Hessian.  Per spring
// dJ/dk += -(r - L) d^.(lF_hi - lF_lo) and dJ/dL = k d^.(lF_hi - lF_lo), split by
// L = L0 + L0 a (sin(w t) cos phi + cos(w t) sin phi) into sums GS, GC of
// dJ/dL times sin(w t_n) and cos(w t_n).  Contact and friction branches are those
// the forward run took (the recorded states decide them).
#include <cmath>

#include "spring.h"

namespace sr {

namespace {

struct AArgs {
    const RobotInfo *robots;
    const int32_t *list;
    int count;
    Planes pl;
    const float4 *x0;
    const float4 *rec_x, *rec_v;  // [n_steps * slot_base + t * slots + s]
    const float4 *rec_u;          // v_n (dashpots, damped ground), same layout
    float4 *rec_l;                // lambda_F of every step (split form), same layout
    int n_steps;
    const float2 *sc;
    float4 *lx, *lv;    // per slot
    float *gk, *gs, *gc;  // per stencil entry
    float *gd;            // dJ/dc per stencil entry (dashpots)
    SimConst c;
};

// The parameter-gradient terms of one spring at one step (d = x_hi - x_lo,
// u = lambda_F,hi - lambda_F,lo, r2 = |d|^2, ir = 1/r, kL = k L(t), du = d.u):
//   dJ/dk  += -(r - L(t)) du / r,   dJ/d(k L0 a cos phi) += k du / r S,
//   dJ/d(k L0 a sin phi) += k du / r C.
// One helper for the fused reverse step and the split gradient pass, so both
// take the same operations and give the same bits.
__device__ __forceinline__ void spring_grad_sums(float r2, float ir, float kL, float du, float k, float ik, float2 sct,
                                                 float &gk, float &gs, float &gc) {
    const float dhu = du * ir;
    gk = fmaf(-(r2 * ir - kL * ik), dhu, gk);
    const float gL = k * dhu;
    gs = fmaf(gL, sct.x, gs);
    gc = fmaf(gL, sct.y, gc);
}

// XCH: each spring's K_s (lF_hi - lF_lo) is computed once by its lower end and
// handed to the upper end through LDS (three rows per direction, PAD zero
// entries in front); otherwise the upper end recomputes it.  Both give the
// same bits.  The exchange keeps one position/adjoint buffer and adds a
// barrier per step.
// ALAG (exchange form): the position and adjoint reads of direction d + ALAG
// are issued before direction d's arithmetic, which waits for its own two reads
// only (ALAG 0: each read is waited for before the next is issued).
// ONEBUF (recompute form): one position/adjoint buffer instead of two, with a
// barrier at the start of each step, so that 12^3 robots fit in LDS.
// DASH (recompute form, one buffer; Table II model): the forces also depend on
// the velocities v_n of the step.  A spring's dashpot c (v_j - v_i).d^ adds,
// with d = x_j - x_i, u = lambda_F,j - lambda_F,i, w = (v_j - v_i).d and
// du = d.u,
//   lambda_x,i += c/r^2 [du (v_j - v_i) + w u - 2 w du d / r^2]  (minus at j),
//   lambda_v,i += c du d / r^2                                     (minus at j),
//   dJ/dc      += -w du / r^2,
// and the ground force N = k_g(-z) - c_g v_z (where it is not clamped at zero)
// feeds lambda_z and lambda_vz, with the friction threshold following N.
// FNC: a scheduling barrier after each direction's spring work, so the
// compiler does not hoist every neighbour read of the slot (which spilled the
// non-exchange form at 9^3: 1265 VGPRs without, 51 with)
// XCC (exchange form): the directions are taken in XCC chunks, each with its
// own forward half, barrier and receiving half, so that only one chunk's rows
// need LDS (at 9^3-12^3 all 13 directions' rows would not fit beside the
// state).  Each node then adds its forward springs' terms and subtracts its
// backward springs' chunk by chunk, so the sums round differently from one
// chunk (the oracle bounds both).
// NOG (split form): the reverse step keeps no parameter-gradient sums; it
// writes each step's lambda_F to rec_l instead, and k_adj_grad forms the sums
// from the recorded positions and those lambda_F afterwards.  The 13 springs'
// three sums per slot no longer take registers beside the adjoint recursion.
template <int N, int BS, bool PHASE, bool XCH, int ALAG = 0, bool ONEBUF = false, bool DASH = false, bool FNC = false,
          bool NOG = false, int XCC = 1>
__global__ __launch_bounds__(BS) void k_adjoint(AArgs A) {
    static_assert(XCC == 1 || XCH, "direction chunks are a form of the exchange");
    static_assert(ALAG == 0 || XCH, "pipelined reads are for the exchange form");
    static_assert(!DASH || XCH || ONEBUF, "the dashpot adjoint keeps one buffer");
    static_assert(!DASH || ALAG == 0, "the dashpot exchange reads its neighbours in order");
    using G = Geo<N>;
    constexpr int SL = G::SL, PAD = G::PAD, XL = G::XL, CL = G::CL;
    constexpr int NPT = (SL + BS - 1) / BS;
    constexpr int NBUF = (XCH || ONEBUF) ? 1 : 2;
    constexpr int NQ = XCH ? 1 : NDIR;
    constexpr int NCH = XCH ? XCC : 1;                 // direction chunks
    constexpr int NDC = (NDIR + NCH - 1) / NCH;        // directions per chunk
    constexpr int NR = DASH ? 4 : 3;                   // exchange rows per direction
    __shared__ float4 xs[NBUF][XL];
    __shared__ float4 lf[NBUF][XL];
    __shared__ float4 vs[DASH ? NBUF : 1][DASH ? XL : 1];
    __shared__ float ku[XCH ? NR * NDC * CL : 1];
    const int tid = threadIdx.x;
    const SimConst c = A.c;
    const bool ground = c.ground != 0;
    const float fz = c.mu_kc_dt_m;  // d(dv)/d(-z) = mu kc dt / m

    for (int q = blockIdx.x; q < A.count; q += gridDim.x) {
        const int r = A.list[q];
        const int base = A.robots[r].slot_base;
        const int pbase = NDIR * base;
        const size_t rbase = (size_t)A.n_steps * base;
        const float4 ghost = make_float4(1e4f, 1e4f, 1e4f, 0.f), zero = make_float4(0.f, 0.f, 0.f, 0.f);
        if (XCH)
            for (int i = tid; i < NR * NDC * CL; i += BS) ku[i] = 0.f;
        for (int i = tid; i < PAD; i += BS) {
#pragma unroll
            for (int b = 0; b < NBUF; ++b) {
                xs[b][i] = ghost;
                xs[b][PAD + SL + i] = ghost;
                lf[b][i] = zero;
                lf[b][PAD + SL + i] = zero;
                if constexpr (DASH) {
                    vs[b][i] = zero;
                    vs[b][PAD + SL + i] = zero;
                }
            }
        }

        bool pres[NPT];
        float3 X0[NPT], lx[NPT], lv[NPT];
        float pk[NPT][NDIR], pa[NPT][NDIR], pb[NPT][NDIR], pik[NPT][NDIR];
        float qk[NPT][NQ], qa[NPT][NQ], qb[NPT][NQ];
        constexpr int NG = NOG ? 1 : NDIR;
        float gk[NPT][NG], gs[NPT][NG], gc[NPT][NG];
        float pd[NPT][DASH ? NDIR : 1], qd[NPT][DASH ? NQ : 1], gd[NPT][DASH && !NOG ? NDIR : 1];
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int s = tid + k * BS;
            const bool live = s < SL;
            const int sc_ = live ? s : 0;
            const float4 P0 = A.x0[base + sc_];
            pres[k] = live && P0.w != 0.f;
            X0[k] = make_float3(P0.x, P0.y, P0.z);
            const float4 LX = A.lx[base + sc_], LV = A.lv[base + sc_];
            lx[k] = make_float3(LX.x, LX.y, LX.z);
            lv[k] = make_float3(LV.x, LV.y, LV.z);
#pragma unroll
            for (int d = 0; d < NDIR; ++d) {
                const int pi = pbase + d * SL + sc_;
                const float kk = live ? A.pl.k[pi] : 0.f;
                pk[k][d] = kk;
                pa[k][d] = live ? A.pl.kal[pi] : 0.f;
                pb[k][d] = (live && PHASE) ? A.pl.kbe[pi] : 0.f;
                pik[k][d] = kk != 0.f ? 1.0f / kk : 0.f;
                if constexpr (!NOG) {
                    gk[k][d] = live ? A.gk[pi] : 0.f;
                    gs[k][d] = live ? A.gs[pi] : 0.f;
                    gc[k][d] = live ? A.gc[pi] : 0.f;
                }
                if constexpr (DASH) {
                    pd[k][d] = live ? A.pl.kd[pi] : 0.f;
                    if constexpr (!NOG) gd[k][DASH && !NOG ? d : 0] = live ? A.gd[pi] : 0.f;
                }
            }
            if (!XCH) {
#pragma unroll
                for (int d = 0; d < NQ; ++d) {
                    const int lo = s - dir_off(d, N);
                    const bool ok = live && lo >= 0;
                    const int qi = pbase + d * SL + (ok ? lo : 0);
                    qk[k][d] = ok ? A.pl.k[qi] : 0.f;
                    qa[k][d] = ok ? A.pl.kal[qi] : 0.f;
                    qb[k][d] = (ok && PHASE) ? A.pl.kbe[qi] : 0.f;
                    if constexpr (DASH) qd[k][d] = ok ? A.pl.kd[qi] : 0.f;
                }
            }
        }
        __syncthreads();

        // the recorded state of each step is read one step ahead, so the global
        // loads are in flight during the previous step's spring part
        float4 XRn[NPT], VPn[NPT], VNn[DASH ? NPT : 1];
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int s = tid + k * BS;
            if (pres[k] && A.n_steps > 0) {
                XRn[k] = A.rec_x[rbase + (size_t)(A.n_steps - 1) * SL + s];
                VPn[k] = A.rec_v[rbase + (size_t)(A.n_steps - 1) * SL + s];
                if constexpr (DASH) VNn[k] = A.rec_u[rbase + (size_t)(A.n_steps - 1) * SL + s];
            } else {
                XRn[k] = make_float4(0.f, 0.f, 0.f, 0.f);
                VPn[k] = XRn[k];
                if constexpr (DASH) VNn[k] = XRn[k];
            }
        }
        float2 sc_next = A.n_steps > 0 ? A.sc[A.n_steps - 1] : make_float2(0.f, 0.f);
        for (int t = A.n_steps - 1; t >= 0; --t) {
            const int b = NBUF == 1 ? 0 : (t & 1);
            if (NBUF == 1) __syncthreads();  // the previous step's readers are done with the buffers
            const float2 sct = sc_next;
            if (t > 0) sc_next = A.sc[t - 1];
            float4 XRc[NPT], VPc[NPT], VNc[DASH ? NPT : 1];
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                const int s = tid + k * BS;
                XRc[k] = XRn[k];
                VPc[k] = VPn[k];
                if constexpr (DASH) VNc[k] = VNn[k];
                if (pres[k] && t > 0) {
                    XRn[k] = A.rec_x[rbase + (size_t)(t - 1) * SL + s];
                    VPn[k] = A.rec_v[rbase + (size_t)(t - 1) * SL + s];
                    if constexpr (DASH) VNn[k] = A.rec_u[rbase + (size_t)(t - 1) * SL + s];
                }
            }
            float3 Xr[NPT], LF[NPT], Vr[DASH ? NPT : 1];
            // node-local part of the reverse step
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                const int s = tid + k * BS;
                if (s >= SL) continue;
                float3 X = X0[k], lF = make_float3(0.f, 0.f, 0.f);
                if (pres[k]) {
                    const float4 XR = XRc[k];
                    const float4 VP = VPc[k];
                    X = make_float3(XR.x, XR.y, XR.z);
                    float ux = c.damping * fmaf(c.dt, lx[k].x, lv[k].x);
                    float uy = c.damping * fmaf(c.dt, lx[k].y, lv[k].y);
                    const float uz = c.damping * fmaf(c.dt, lx[k].z, lv[k].z);
                    const bool below = ground && X.z < 0.f;
                    if (DASH && c.gdamp) {
                        // the damped ground: N = max(k_g (-z) - c_g v_z, 0), the
                        // friction threshold follows N; the forward's operations
                        const float4 VN = VNc[DASH ? k : 0];
                        const float Nf = below ? fmaxf(fmaf(-c.cg, VN.z, c.kc * -X.z), 0.f) : 0.f;
                        float lN = 0.f;
                        if (Nf > 0.f) {
                            const float dv = c.mu_dt_m * Nf;
                            const float u = sqrtf(fmaf(VP.y, VP.y, VP.x * VP.x));
                            if (u <= fmaxf(dv, c.mus_dt_m * Nf)) {
                                ux = 0.f;
                                uy = 0.f;
                            } else {
                                const float hx = VP.x / u, hy = VP.y / u;
                                const float dot = fmaf(hy, uy, hx * ux);
                                lN = -c.mu_dt_m * dot;
                                const float cc = dv / u;
                                const float nx = ux - cc * (ux - hx * dot);
                                const float ny = uy - cc * (uy - hy * dot);
                                ux = nx;
                                uy = ny;
                            }
                        }
                        lF = make_float3(c.dt_m * ux, c.dt_m * uy, c.dt_m * uz);
                        float lvz = uz;
                        if (Nf > 0.f) {
                            lN += lF.z;
                            lx[k].z = fmaf(-c.kc, lN, lx[k].z);
                            lvz = fmaf(-c.cg, lN, lvz);
                        }
                        lv[k] = make_float3(ux, uy, lvz);
                    } else {
                        if (below) {
                            const float dv = c.mu_kc_dt_m * (-X.z);
                            const float u = sqrtf(fmaf(VP.y, VP.y, VP.x * VP.x));
                            if (u <= fmaxf(dv, c.mus_kc_dt_m * (-X.z))) {
                                ux = 0.f;
                                uy = 0.f;
                            } else {
                                const float hx = VP.x / u, hy = VP.y / u;
                                const float dot = fmaf(hy, uy, hx * ux);
                                lx[k].z = fmaf(fz, dot, lx[k].z);
                                const float cc = dv / u;
                                const float nx = ux - cc * (ux - hx * dot);
                                const float ny = uy - cc * (uy - hy * dot);
                                ux = nx;
                                uy = ny;
                            }
                        }
                        lv[k] = make_float3(ux, uy, uz);
                        lF = make_float3(c.dt_m * ux, c.dt_m * uy, c.dt_m * uz);
                        if (below) lx[k].z = fmaf(-c.kc, lF.z, lx[k].z);
                    }
                }
                Xr[k] = X;
                LF[k] = lF;
                if (NOG && pres[k]) A.rec_l[rbase + (size_t)t * SL + s] = make_float4(lF.x, lF.y, lF.z, 0.f);
                xs[b][PAD + s] = make_float4(X.x, X.y, X.z, 0.f);
                lf[b][PAD + s] = make_float4(lF.x, lF.y, lF.z, 0.f);
                if constexpr (DASH) {
                    const float4 VN = pres[k] ? VNc[DASH ? k : 0] : zero;
                    Vr[DASH ? k : 0] = make_float3(VN.x, VN.y, VN.z);
                    vs[DASH ? b : 0][PAD + s] = make_float4(VN.x, VN.y, VN.z, 0.f);
                }
            }
            __syncthreads();
            // spring part: every node takes K_s (lF_hi - lF_lo) from each spring it touches
            float3 accs[NPT], accv[DASH ? NPT : 1];
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                accs[k] = make_float3(0.f, 0.f, 0.f);
                if constexpr (DASH) accv[DASH ? k : 0] = make_float3(0.f, 0.f, 0.f);
            }
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
            const int d0 = ch * NDC, d1 = d0 + NDC < NDIR ? d0 + NDC : NDIR;
            if (ch > 0) __syncthreads();  // the previous chunk's receivers are done with the rows
#if SR_POISON_LDS
            // debug build: each thread's own exchange entries of the chunk hold NaN
            // until it writes them
            if (XCH)
                for (int k = 0; k < NPT; ++k) {
                    const int s = tid + k * BS;
                    if (s < SL && pres[k])  // absent slots never write theirs (they stay zero)
                        for (int q = 0; q < NR; ++q)
                            for (int j = 0; j < d1 - d0; ++j) ku[(q * NDC + j) * CL + PAD + s] = __builtin_nanf("");
                }
#endif
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                const int s = tid + k * BS;
                if (s >= SL || !pres[k]) continue;
                const float4 *xsb = xs[b] + s;
                const float4 *lfb = lf[b] + s;
                const float4 *vsb = vs[DASH ? b : 0] + s;
                float3 acc = accs[k], av = make_float3(0.f, 0.f, 0.f);
                if constexpr (DASH) av = accv[DASH ? k : 0];
                float4 QY[NDIR], QL[NDIR];
                if constexpr (ALAG > 0) {
#pragma unroll
                    for (int d = 0; d < NDIR; ++d) {
                        if (d < d0 || d >= d1 || d >= d0 + ALAG) continue;
                        QY[d] = xsb[PAD + dir_off(d, N)];
                        QL[d] = lfb[PAD + dir_off(d, N)];
                    }
                }
#pragma unroll
                for (int d = 0; d < NDIR; ++d) {
                    if (d < d0 || d >= d1) continue;
                    // forward spring: self is the lower end
                    float3 Y, LJ;
                    if constexpr (ALAG > 0) {
                        constexpr int dummy = 0;
                        const int e = d + ALAG < d1 ? d + ALAG : dummy;
                        if (d + ALAG < d1) {
                            QY[e] = xsb[PAD + dir_off(e, N)];
                            QL[e] = lfb[PAD + dir_off(e, N)];
                        }
                        keep_w(QY[d].w);
                        keep_w(QL[d].w);
                        Y = make_float3(QY[d].x, QY[d].y, QY[d].z);
                        LJ = make_float3(QL[d].x, QL[d].y, QL[d].z);
                    } else {
                        Y = ld3(xsb + (PAD + dir_off(d, N)));
                        LJ = ld3(lfb + (PAD + dir_off(d, N)));
                    }
                    const float dx = Y.x - Xr[k].x, dy = Y.y - Xr[k].y, dz = Y.z - Xr[k].z;
                    const float ux = LJ.x - LF[k].x, uy = LJ.y - LF[k].y, uz = LJ.z - LF[k].z;
                    const float r2 = len2(dx, dy, dz);
                    const float ir = __builtin_amdgcn_rsqf(r2);
                    float kL = fmaf(pa[k][d], sct.x, pk[k][d] * L0d(c, d));
                    if (PHASE) kL = fmaf(pb[k][d], sct.y, kL);
                    const float c1 = fmaf(-kL, ir, pk[k][d]);
                    const float du = fmaf(dz, uz, fmaf(dy, uy, dx * ux));
                    const float c2 = (kL * ir) * ir * ir * du;
                    float kx = fmaf(c1, ux, c2 * dx), ky = fmaf(c1, uy, c2 * dy), kz = fmaf(c1, uz, c2 * dz);
                    if constexpr (DASH) {
                        // dashpot beside the spring (self is the lower end i)
                        const float3 VJ = ld3(vsb + (PAD + dir_off(d, N)));
                        const float3 VI = Vr[DASH ? k : 0];
                        const float wx = VJ.x - VI.x, wy = VJ.y - VI.y, wz = VJ.z - VI.z;
                        const float cd = pd[k][DASH ? d : 0];
                        const float ir2 = ir * ir;
                        const float wv = fmaf(dz, wz, fmaf(dy, wy, dx * wx));
                        const float ce = cd * ir2, q2 = -2.f * wv * du * ir2;
                        kx = fmaf(ce, fmaf(du, wx, fmaf(wv, ux, q2 * dx)), kx);
                        ky = fmaf(ce, fmaf(du, wy, fmaf(wv, uy, q2 * dy)), ky);
                        kz = fmaf(ce, fmaf(du, wz, fmaf(wv, uz, q2 * dz)), kz);
                        const float cv = ce * du;
                        av.x = fmaf(cv, dx, av.x);
                        av.y = fmaf(cv, dy, av.y);
                        av.z = fmaf(cv, dz, av.z);
                        // the upper end forms its velocity-adjoint term c du d / r^2
                        // from this scalar and its own difference vector
                        if (XCH) ku[(3 * NDC + d - d0) * CL + PAD + s] = cv;
                        if constexpr (!NOG) gd[k][DASH && !NOG ? d : 0] = fmaf(-wv * du, ir2, gd[k][DASH && !NOG ? d : 0]);
                    }
                    acc.x += kx;
                    acc.y += ky;
                    acc.z += kz;
                    if (XCH) {
                        ku[(0 * NDC + d - d0) * CL + PAD + s] = kx;
                        ku[(1 * NDC + d - d0) * CL + PAD + s] = ky;
                        ku[(2 * NDC + d - d0) * CL + PAD + s] = kz;
                    }
                    if constexpr (!NOG)
                        spring_grad_sums(r2, ir, kL, du, pk[k][d], pik[k][d], sct, gk[k][NOG ? 0 : d], gs[k][NOG ? 0 : d],
                                         gc[k][NOG ? 0 : d]);
                    if (FNC) __builtin_amdgcn_sched_barrier(0);
                }
                if (!XCH) {
#pragma unroll
                    for (int d = 0; d < NQ; ++d) {
                        // backward spring: self is the upper end
                        const float3 Y = ld3(xsb + (PAD - dir_off(d, N)));
                        const float3 LI = ld3(lfb + (PAD - dir_off(d, N)));
                        const float dx = Xr[k].x - Y.x, dy = Xr[k].y - Y.y, dz = Xr[k].z - Y.z;
                        const float ux = LF[k].x - LI.x, uy = LF[k].y - LI.y, uz = LF[k].z - LI.z;
                        const float r2 = len2(dx, dy, dz);
                        const float ir = __builtin_amdgcn_rsqf(r2);
                        float kL = fmaf(qa[k][d], sct.x, qk[k][d] * L0d(c, d));
                        if (PHASE) kL = fmaf(qb[k][d], sct.y, kL);
                        const float c1 = fmaf(-kL, ir, qk[k][d]);
                        const float du = fmaf(dz, uz, fmaf(dy, uy, dx * ux));
                        const float c2 = (kL * ir) * ir * ir * du;
                        float kx = fmaf(c1, ux, c2 * dx), ky = fmaf(c1, uy, c2 * dy), kz = fmaf(c1, uz, c2 * dz);
                        if constexpr (DASH) {
                            // dashpot beside the spring (self is the upper end j)
                            const float3 VI = ld3(vsb + (PAD - dir_off(d, N)));
                            const float3 VJ = Vr[DASH ? k : 0];
                            const float wx = VJ.x - VI.x, wy = VJ.y - VI.y, wz = VJ.z - VI.z;
                            const float cd = qd[k][DASH ? d : 0];
                            const float ir2 = ir * ir;
                            const float wv = fmaf(dz, wz, fmaf(dy, wy, dx * wx));
                            const float ce = cd * ir2, q2 = -2.f * wv * du * ir2;
                            kx = fmaf(ce, fmaf(du, wx, fmaf(wv, ux, q2 * dx)), kx);
                            ky = fmaf(ce, fmaf(du, wy, fmaf(wv, uy, q2 * dy)), ky);
                            kz = fmaf(ce, fmaf(du, wz, fmaf(wv, uz, q2 * dz)), kz);
                            const float cv = ce * du;
                            av.x = fmaf(-cv, dx, av.x);
                            av.y = fmaf(-cv, dy, av.y);
                            av.z = fmaf(-cv, dz, av.z);
                        }
                        acc.x -= kx;
                        acc.y -= ky;
                        acc.z -= kz;
                        if (FNC) __builtin_amdgcn_sched_barrier(0);
                    }
                }
                accs[k] = acc;
                if constexpr (DASH) accv[DASH ? k : 0] = av;
            }
            if (XCH) {
                __syncthreads();
#pragma unroll
                for (int k = 0; k < NPT; ++k) {
                    const int s = tid + k * BS;
                    if (s >= SL || !pres[k]) continue;
                    float3 acc = accs[k];
#pragma unroll
                    for (int d = 0; d < NDIR; ++d) {
                        if (d < d0 || d >= d1) continue;
                        const int lo = PAD + s - dir_off(d, N);
                        acc.x -= ku[(0 * NDC + d - d0) * CL + lo];
                        acc.y -= ku[(1 * NDC + d - d0) * CL + lo];
                        acc.z -= ku[(2 * NDC + d - d0) * CL + lo];
                    }
                    accs[k] = acc;
                    if constexpr (DASH) {
                        // the recompute form's operations at the upper end: d = x_hi - x_lo
                        float3 av = accv[DASH ? k : 0];
#pragma unroll
                        for (int d = 0; d < NDIR; ++d) {
                            if (d < d0 || d >= d1) continue;
                            const int lo = PAD + s - dir_off(d, N);
                            const float3 Y = ld3(xs[b] + lo);
                            const float cv = ku[(3 * NDC + d - d0) * CL + lo];
                            av.x = fmaf(-cv, Xr[k].x - Y.x, av.x);
                            av.y = fmaf(-cv, Xr[k].y - Y.y, av.y);
                            av.z = fmaf(-cv, Xr[k].z - Y.z, av.z);
                        }
                        accv[DASH ? k : 0] = av;
                    }
                }
            }
            }  // direction chunks
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                const int s = tid + k * BS;
                if (s >= SL || !pres[k]) continue;
                const float3 acc = accs[k];
                lx[k].x += acc.x;
                lx[k].y += acc.y;
                lx[k].z += acc.z;
                if constexpr (DASH) {
                    const float3 av = accv[DASH ? k : 0];
                    lv[k].x += av.x;
                    lv[k].y += av.y;
                    lv[k].z += av.z;
                }
            }
        }
        // the adjoint state and the gradient sums carry over to the previous segment
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int s = tid + k * BS;
            if (s >= SL) continue;
            A.lx[base + s] = make_float4(lx[k].x, lx[k].y, lx[k].z, 0.f);
            A.lv[base + s] = make_float4(lv[k].x, lv[k].y, lv[k].z, 0.f);
#pragma unroll
            for (int d = 0; d < NDIR; ++d) {
                const int pi = pbase + d * SL + s;
                if constexpr (!NOG) {
                    A.gk[pi] = gk[k][NOG ? 0 : d];
                    A.gs[pi] = gs[k][NOG ? 0 : d];
                    A.gc[pi] = gc[k][NOG ? 0 : d];
                }
                if constexpr (DASH && !NOG) A.gd[pi] = gd[k][DASH && !NOG ? d : 0];
            }
        }
        __syncthreads();
    }
}

// Split form, second pass: the parameter-gradient sums of the forward springs
// of directions D0 .. D1 - 1 over one segment, from the recorded positions x_t
// (rec_x; an absent slot sits at its build position) and the reverse step's
// lambda_F (rec_l; zero on absent slots), step by step from the segment's end
// to its start as in the fused form, through the same helper: the same bits.
// One LDS buffer of positions and one of lambda_F, two barriers per step.
template <int N, int BS, bool PHASE, int D0, int D1, bool DASH>
__device__ __forceinline__ void adj_grad_robot(const AArgs &A, int q, float4 *xs, float4 *lf, float4 *vs) {
    using G = Geo<N>;
    constexpr int SL = G::SL, PAD = G::PAD;
    constexpr int NPT = (SL + BS - 1) / BS;
    constexpr int ND = D1 - D0;
    const int tid = threadIdx.x;
    const SimConst c = A.c;
    {
        const int r = A.list[q];
        const int base = A.robots[r].slot_base;
        const int pbase = NDIR * base;
        const size_t rbase = (size_t)A.n_steps * base;
        const float4 ghost = make_float4(1e4f, 1e4f, 1e4f, 0.f), zero = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int i = tid; i < PAD; i += BS) {
            xs[i] = ghost;
            xs[PAD + SL + i] = ghost;
            lf[i] = zero;
            lf[PAD + SL + i] = zero;
            if constexpr (DASH) {
                vs[i] = zero;
                vs[PAD + SL + i] = zero;
            }
        }
        bool pres[NPT];
        float3 X0[NPT];
        float pk[NPT][ND], pa[NPT][ND], pb[NPT][ND], pik[NPT][ND], gk[NPT][ND], gs[NPT][ND], gc[NPT][ND];
        float gd[NPT][DASH ? ND : 1];
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int s = tid + k * BS;
            const bool live = s < SL;
            const int sc_ = live ? s : 0;
            const float4 P0 = A.x0[base + sc_];
            pres[k] = live && P0.w != 0.f;
            X0[k] = make_float3(P0.x, P0.y, P0.z);
#pragma unroll
            for (int j = 0; j < ND; ++j) {
                const int pi = pbase + (D0 + j) * SL + sc_;
                const float kk = live ? A.pl.k[pi] : 0.f;
                pk[k][j] = kk;
                pa[k][j] = live ? A.pl.kal[pi] : 0.f;
                pb[k][j] = (live && PHASE) ? A.pl.kbe[pi] : 0.f;
                pik[k][j] = kk != 0.f ? 1.0f / kk : 0.f;
                gk[k][j] = live ? A.gk[pi] : 0.f;
                gs[k][j] = live ? A.gs[pi] : 0.f;
                gc[k][j] = live ? A.gc[pi] : 0.f;
                if constexpr (DASH) gd[k][DASH ? j : 0] = live ? A.gd[pi] : 0.f;
            }
        }
        // each step's recorded values are loaded one step ahead, so the global
        // loads are in flight during the previous step's spring work
        float4 XRn[NPT], LLn[NPT], VNn[DASH ? NPT : 1];
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int s = tid + k * BS;
            XRn[k] = zero;
            LLn[k] = zero;
            if constexpr (DASH) VNn[DASH ? k : 0] = zero;
            if (pres[k] && A.n_steps > 0) {
                XRn[k] = A.rec_x[rbase + (size_t)(A.n_steps - 1) * SL + s];
                LLn[k] = A.rec_l[rbase + (size_t)(A.n_steps - 1) * SL + s];
                if constexpr (DASH) VNn[DASH ? k : 0] = A.rec_u[rbase + (size_t)(A.n_steps - 1) * SL + s];
            }
        }
        for (int t = A.n_steps - 1; t >= 0; --t) {
            __syncthreads();  // the previous step's readers are done with the buffers
            const float2 sct = A.sc[t];
            float3 Xr[NPT], LF[NPT], Vr[DASH ? NPT : 1];
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                const int s = tid + k * BS;
                if (s >= SL) continue;
                float3 X = X0[k];
                float4 L = zero, V = zero;
                if (pres[k]) {
                    const float4 XR = XRn[k];
                    X = make_float3(XR.x, XR.y, XR.z);
                    L = LLn[k];
                    if constexpr (DASH) V = VNn[DASH ? k : 0];
                    if (t > 0) {
                        XRn[k] = A.rec_x[rbase + (size_t)(t - 1) * SL + s];
                        LLn[k] = A.rec_l[rbase + (size_t)(t - 1) * SL + s];
                        if constexpr (DASH) VNn[DASH ? k : 0] = A.rec_u[rbase + (size_t)(t - 1) * SL + s];
                    }
                }
                Xr[k] = X;
                LF[k] = make_float3(L.x, L.y, L.z);
                xs[PAD + s] = make_float4(X.x, X.y, X.z, 0.f);
                lf[PAD + s] = make_float4(L.x, L.y, L.z, 0.f);
                if constexpr (DASH) {
                    Vr[DASH ? k : 0] = make_float3(V.x, V.y, V.z);
                    vs[PAD + s] = make_float4(V.x, V.y, V.z, 0.f);
                }
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                const int s = tid + k * BS;
                if (s >= SL || !pres[k]) continue;
#pragma unroll
                for (int j = 0; j < ND; ++j) {
                    const int d = D0 + j;
                    const float3 Y = ld3(xs + s + (PAD + dir_off(d, N)));
                    const float3 LJ = ld3(lf + s + (PAD + dir_off(d, N)));
                    const float dx = Y.x - Xr[k].x, dy = Y.y - Xr[k].y, dz = Y.z - Xr[k].z;
                    const float ux = LJ.x - LF[k].x, uy = LJ.y - LF[k].y, uz = LJ.z - LF[k].z;
                    const float r2 = len2(dx, dy, dz);
                    const float ir = __builtin_amdgcn_rsqf(r2);
                    float kL = fmaf(pa[k][j], sct.x, pk[k][j] * L0d(c, d));
                    if (PHASE) kL = fmaf(pb[k][j], sct.y, kL);
                    const float du = fmaf(dz, uz, fmaf(dy, uy, dx * ux));
                    spring_grad_sums(r2, ir, kL, du, pk[k][j], pik[k][j], sct, gk[k][j], gs[k][j], gc[k][j]);
                    if constexpr (DASH) {
                        // dJ/dc of the dashpot beside the spring, as in the fused reverse step
                        const float3 VJ = ld3(vs + s + (PAD + dir_off(d, N)));
                        const float3 VI = Vr[DASH ? k : 0];
                        const float wx = VJ.x - VI.x, wy = VJ.y - VI.y, wz = VJ.z - VI.z;
                        const float ir2 = ir * ir;
                        const float wv = fmaf(dz, wz, fmaf(dy, wy, dx * wx));
                        gd[k][DASH ? j : 0] = fmaf(-wv * du, ir2, gd[k][DASH ? j : 0]);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int s = tid + k * BS;
            if (s >= SL) continue;
#pragma unroll
            for (int j = 0; j < ND; ++j) {
                const int pi = pbase + (D0 + j) * SL + s;
                A.gk[pi] = gk[k][j];
                A.gs[pi] = gs[k][j];
                A.gc[pi] = gc[k][j];
                if constexpr (DASH) A.gd[pi] = gd[k][DASH ? j : 0];
            }
        }
        __syncthreads();
    }
}

// The gradient pass over directions D0 .. D1 - 1, or (D2 > D1) over D0 .. D1 - 1
// in the workgroups with blockIdx.y 0 and D1 .. D2 - 1 in those with 1: the two
// halves of a robot run side by side (they write disjoint sums).
// DASH: also dJ/dc of the spring dashpots, from the recorded velocities v_n.
template <int N, int BS, bool PHASE, int D0, int D1, int D2 = D1, bool DASH = false>
__global__ __launch_bounds__(BS) void k_adj_grad(AArgs A) {
    __shared__ float4 xs[Geo<N>::XL];
    __shared__ float4 lf[Geo<N>::XL];
    __shared__ float4 vs[DASH ? Geo<N>::XL : 1];
    for (int q = blockIdx.x; q < A.count; q += gridDim.x) {
        if constexpr (D2 == D1) {
            adj_grad_robot<N, BS, PHASE, D0, D1, DASH>(A, q, xs, lf, vs);
        } else {
            if (blockIdx.y == 0)
                adj_grad_robot<N, BS, PHASE, D0, D1, DASH>(A, q, xs, lf, vs);
            else
                adj_grad_robot<N, BS, PHASE, D1, D2, DASH>(A, q, xs, lf, vs);
        }
    }
}

// Terminal adjoint of J = sum_r g_r (1/M_r) sum_i (x_i,x - x0_i,x): lx = g_r / M_r e_x on
// present nodes, lv = 0, gradient sums zero.
__global__ void k_adj_init(const RobotInfo *robots, int total_slots, const int32_t *slot_robot, const float4 *x0,
                           const float *dJ, float4 *lx, float4 *lv, float *gk, float *gs, float *gc, float *gd) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total_slots) return;
    const int r = slot_robot[g];
    const RobotInfo ri = robots[r];
    const bool pres = x0[g].w != 0.f;
    const float val = (pres && ri.M > 0) ? dJ[r] / (float)ri.M : 0.f;
    lx[g] = make_float4(val, 0.f, 0.f, 0.f);
    lv[g] = make_float4(0.f, 0.f, 0.f, 0.f);
    const int s = g - ri.slot_base;
    for (int d = 0; d < NDIR; ++d) {
        const int pi = NDIR * ri.slot_base + d * ri.slots + s;
        gk[pi] = 0.f;
        gs[pi] = 0.f;
        gc[pi] = 0.f;
        if (gd) gd[pi] = 0.f;
    }
}

// Per spring: dJ/dk, dJ/da, dJ/dphi in canonical order, from the stencil sums.
__global__ void k_adj_springs(const RobotInfo *robots, int total_slots, const int32_t *slot_robot, const int32_t *sid,
                              const int64_t *spring_off, Planes pl, float voxel_len, const float *gk, const float *gs,
                              const float *gc, float *g_k, float *g_a, float *g_phi) {
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
        const float kL0 = pl.kL0[pi], kal = pl.kal[pi], kbe = pl.kbe[pi];
        float a = 0.f, cph = 1.f, sph = 0.f;
        if (kL0 != 0.f) {
            if (kbe == 0.f) a = kal / kL0;
            else {
                a = sqrtf(kal * kal + kbe * kbe) / kL0;
                const float ph = atan2f(kbe, kal);
                cph = cosf(ph);
                sph = sinf(ph);
            }
        }
        if (g_k) g_k[o] = gk[pi];
        if (g_a) g_a[o] = L0 * (gs[pi] * cph + gc[pi] * sph);
        if (g_phi) g_phi[o] = L0 * a * (gc[pi] * cph - gs[pi] * sph);
    }
}

// dJ/dw per voxel through the parallel-sum rule.  Write Z = k a e^{i phi} for a
// spring, so k L(t) = k L0 + L0 (Re Z sin wt + Im Z cos wt): then dJ/dRe Z =
// L0 gs / k, dJ/dIm Z = L0 gc / k and, at fixed Z, dJ/dk = gk - (kal gs + kbe gc) / k^2
// (gk is dJ/dk at fixed a, phi; gs, gc the sums of dJ/dL k sin wt, k cos wt).
// Voxel v adds k_c w to k and k_c w amp e^{i ph} to Z of each of its 28 springs,
// with (amp, ph) = (a_c, phi_c), or (w a_c, w phi_c) under weight-scaled
// actuation, whose w-derivative is k_c a_c (2 w + i w^2 phi_c) e^{i w phi_c};
// and zeta sqrt(2 m k_c w) to the spring's dashpot c, whose w-derivative is
// zeta sqrt(2 m k_c w) / (2 w).
struct DwArgs {
    const RobotInfo *robots;
    int total_vox;
    const int32_t *vox_robot;
    const uint8_t *kept;
    const float *w;
    Planes pl;
    const float *gk, *gs, *gc, *gd;
    float k_class[5], a_class[5], phi_class[5];
    int weight_act;
    float voxel_len;
    float dash_c;  // d c / d w of this voxel's dashpot, up to sqrt(k_c / w): zeta sqrt(2 m) / 2
    float *dJdw;
};

__global__ void k_adj_dw(DwArgs A) {
    const int gv = blockIdx.x * blockDim.x + threadIdx.x;
    if (gv >= A.total_vox) return;
    const int r = A.vox_robot[gv];
    const RobotInfo ri = A.robots[r];
    const int v = gv - ri.vox_base;
    const int c = A.kept[gv];
    if (c == 0) {
        A.dJdw[gv] = 0.f;
        return;
    }
    const int n = ri.n, N = ri.N;
    const int i = v % n, j = (v / n) % n, kk = v / (n * n);
    const float kc = A.k_class[c], ac = A.a_class[c], pc = A.phi_class[c], wv = A.w[gv];
    const float dcdw = (A.gd && wv > 0.f) ? A.dash_c * sqrtf(kc / wv) : 0.f;
    float dzr, dzi;  // d(k_c w amp e^{i ph})/dw
    if (A.weight_act) {
        const float cs = cosf(wv * pc), sn = sinf(wv * pc);
        dzr = kc * ac * (2.f * wv * cs - wv * wv * pc * sn);
        dzi = kc * ac * (2.f * wv * sn + wv * wv * pc * cs);
    } else {
        dzr = kc * ac * cosf(pc);
        dzi = kc * ac * sinf(pc);
    }
    float sum = 0.f;
    for (int c1 = 0; c1 < 8; ++c1) {
        const int a1 = i + (c1 & 1), b1 = j + ((c1 >> 1) & 1), z1 = kk + (c1 >> 2);
        const int l1 = a1 + N * (b1 + N * z1);
        for (int c2 = 0; c2 < 8; ++c2) {
            const int a2 = i + (c2 & 1), b2 = j + ((c2 >> 1) & 1), z2 = kk + (c2 >> 2);
            const int l2 = a2 + N * (b2 + N * z2);
            if (l2 <= l1) continue;
            // forward direction from corner 1 to corner 2
            const int dx = a2 - a1, dy = b2 - b1, dz = z2 - z1;
            int d = -1;
            for (int q = 0; q < NDIR; ++q)
                if (dir_dx(q) == dx && dir_dy(q) == dy && dir_dz(q) == dz) d = q;
            const int pi = NDIR * ri.slot_base + d * ri.slots + l1;
            const float ks = A.pl.k[pi];
            const float L0 = A.voxel_len * sqrtf((float)dir_len2(d));
            const float gs = A.gs[pi], gc = A.gc[pi];
            float t = kc * A.gk[pi];
            if (ks != 0.f) {
                const float ik = 1.f / ks;
                t -= kc * (A.pl.kal[pi] * gs + A.pl.kbe[pi] * gc) * ik * ik;
                t += L0 * ik * (dzr * gs + dzi * gc);
            }
            if (A.gd) t = fmaf(dcdw, A.gd[pi], t);
            sum += t;
        }
    }
    A.dJdw[gv] = sum;
}

// Genome gradient: for each voxel with dJ/dw != 0, recompute the FP32 forward
// (encoding, two tanh layers, sigmoid head), g5 = dJ/dw w (1 - w), then back
// through W3 row 5, W2 and W1.  One workgroup per robot; weight gradients are
// accumulated in registers over tiles of 64 voxels staged in LDS.
constexpr int OFF_W1 = 0, OFF_B1 = 4096, OFF_W2 = 4160, OFF_B2 = 8256, OFF_W3 = 8320, OFF_B3 = 8704;

__global__ __launch_bounds__(256) void k_mlp_backward(const RobotInfo *robots, const float *genomes, const float *B,
                                                      const float *dJdw, float *g_gen) {
    __shared__ float W1[64 * 64], W2[64 * 64], w3[64], b1[64], b2[64];
    __shared__ float Bs[96];
    __shared__ float gam[64][65], h1[64][65], h2[64][65], d2[64][65], d1[64][65];
    __shared__ float gv5[64];
    __shared__ float b3s;
    const int r = blockIdx.x;
    const RobotInfo ri = robots[r];
    const int n = ri.n, nv = n * n * n;
    const float *g = genomes + (size_t)r * SR_GENOME_LEN;
    float *out = g_gen + (size_t)r * SR_GENOME_LEN;
    const int tid = threadIdx.x;
    for (int q = tid; q < 4096; q += 256) {
        W1[q] = g[OFF_W1 + q];
        W2[q] = g[OFF_W2 + q];
    }
    if (tid < 64) {
        w3[tid] = g[OFF_W3 + 5 * 64 + tid];
        b1[tid] = g[OFF_B1 + tid];
        b2[tid] = g[OFF_B2 + tid];
    }
    if (tid < 96) Bs[tid] = B[tid];
    if (tid == 0) b3s = g[OFF_B3 + 5];
    __syncthreads();
    // accumulators: thread owns W1/W2 gradient entries e = tid + 256 m, m < 16
    float aW1[16], aW2[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        aW1[m] = 0.f;
        aW2[m] = 0.f;
    }
    float aB1 = 0.f, aB2 = 0.f, aW3 = 0.f, aB3 = 0.f;
    const float inv = 1.0f / (float)n;
    for (int v0 = 0; v0 < nv; v0 += 64) {
        // forward for voxel v0 + lane of wave 0..3: each thread does a quarter of one voxel's work
        const int vl = tid & 63, part = tid >> 6;
        const int vid = v0 + vl;
        const bool act = vid < nv && dJdw[ri.vox_base + vid] != 0.f;
        {
            const float vx = (((vid % n)) + 0.5f) * inv, vy = (((vid / n) % n) + 0.5f) * inv, vz = ((vid / (n * n)) + 0.5f) * inv;
            for (int q = part * 8; q < part * 8 + 8; ++q) {
                const float t = 2.0f * fmaf(Bs[3 * q + 2], vz, fmaf(Bs[3 * q + 1], vy, Bs[3 * q] * vx));
                float sn, cs;
                sincospif(t, &sn, &cs);
                gam[vl][q] = act ? cs : 0.f;
                gam[vl][32 + q] = act ? sn : 0.f;
            }
        }
        __syncthreads();
        for (int o = part * 16; o < part * 16 + 16; ++o) {
            float a = b1[o];
#pragma unroll 8
            for (int jj = 0; jj < 64; ++jj) a = fmaf(W1[o * 64 + jj], gam[vl][jj], a);
            h1[vl][o] = act ? tanhf(a) : 0.f;
        }
        __syncthreads();
        for (int o = part * 16; o < part * 16 + 16; ++o) {
            float a = b2[o];
#pragma unroll 8
            for (int jj = 0; jj < 64; ++jj) a = fmaf(W2[o * 64 + jj], h1[vl][jj], a);
            h2[vl][o] = act ? tanhf(a) : 0.f;
        }
        __syncthreads();
        if (part == 0) {
            float o5 = b3s;
            for (int jj = 0; jj < 64; ++jj) o5 = fmaf(w3[jj], h2[vl][jj], o5);
            const float w = 1.0f / (1.0f + expf(-o5));
            gv5[vl] = act ? dJdw[ri.vox_base + vid] * w * (1.0f - w) : 0.f;
        }
        __syncthreads();
        // W3 row 5 and b3[5] gradients (threads 0..63 own one entry each of W3 row 5)
        if (tid < 64) {
            float sacc = 0.f;
            for (int vv = 0; vv < 64; ++vv) sacc = fmaf(gv5[vv], h2[vv][tid], sacc);
            aW3 += sacc;
        }
        if (tid == 64) {
            float sacc = 0.f;
            for (int vv = 0; vv < 64; ++vv) sacc += gv5[vv];
            aB3 += sacc;
        }
        __syncthreads();
        // d2 = g5 w3 (1 - h2^2)
        for (int o = part * 16; o < part * 16 + 16; ++o) {
            const float hh = h2[vl][o];
            d2[vl][o] = gv5[vl] * w3[o] * (1.0f - hh * hh);
        }
        __syncthreads();
        // d1 = (W2^T d2) (1 - h1^2)
        for (int o = part * 16; o < part * 16 + 16; ++o) {
            float a = 0.f;
#pragma unroll 8
            for (int ii = 0; ii < 64; ++ii) a = fmaf(W2[ii * 64 + o], d2[vl][ii], a);
            const float hh = h1[vl][o];
            d1[vl][o] = a * (1.0f - hh * hh);
        }
        __syncthreads();
        // outer products over the tile's voxels; entry e = tid + 256 m is row
        // (tid >> 6) + 4 m, column tid & 63 of W1 / W2
        {
            const int ij = tid & 63, oi0 = tid >> 6;
#pragma unroll 2
            for (int vv = 0; vv < 64; ++vv) {
                const float gj = gam[vv][ij], hj = h1[vv][ij];
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    aW1[m] = fmaf(d1[vv][oi0 + 4 * m], gj, aW1[m]);
                    aW2[m] = fmaf(d2[vv][oi0 + 4 * m], hj, aW2[m]);
                }
            }
        }
        if (tid < 64) {
            float s1 = 0.f, s2 = 0.f;
            for (int vv = 0; vv < 64; ++vv) {
                s1 += d1[vv][tid];
                s2 += d2[vv][tid];
            }
            aB1 += s1;
            aB2 += s2;
        }
        __syncthreads();
    }
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int e = tid + 256 * m;
        out[OFF_W1 + e] = aW1[m];
        out[OFF_W2 + e] = aW2[m];
    }
    if (tid < 64) {
        out[OFF_B1 + tid] = aB1;
        out[OFF_B2 + tid] = aB2;
        for (int row = 0; row < 6; ++row) out[OFF_W3 + row * 64 + tid] = row == 5 ? aW3 : 0.f;
    }
    if (tid < 5) out[OFF_B3 + tid] = 0.f;  // class logits carry no gradient
    if (tid == 64) out[OFF_B3 + 5] = aB3;
}

typedef void (*AdjFn)(AArgs);
struct AdjEntry {
    int n, block;
    AdjFn fn, fn_phase;
    // split form: fn is the reverse step without gradient sums, and the
    // gradient pass g0 runs gblock threads per workgroup on a grid of robots
    // x gy (gy 2: directions 0..6 and 7..12 in workgroups side by side)
    int gblock = 0;
    AdjFn g0 = nullptr, g0_phase = nullptr;
    int gy = 1;
};
#define SR_AE(NN, BS, X) \
    { NN, BS, k_adjoint<NN + 1, BS, false, X>, k_adjoint<NN + 1, BS, true, X> }
#define SR_AEL(NN, BS, LG) \
    { NN, BS, k_adjoint<NN + 1, BS, false, true, LG>, k_adjoint<NN + 1, BS, true, true, LG> }
// split exchange form with a one-launch gradient pass
#define SR_AESL(NN, BS, LG, GBS)                                                                                \
    {                                                                                                          \
        NN, BS, k_adjoint<NN + 1, BS, false, true, LG, false, false, false, true>,                              \
            k_adjoint<NN + 1, BS, true, true, LG, false, false, false, true>, GBS,                              \
            k_adj_grad<NN + 1, GBS, false, 0, 13>, k_adj_grad<NN + 1, GBS, true, 0, 13>                          \
    }
// split exchange form in XC direction chunks (one chunk's rows in LDS at a
// time), the gradient pass over all directions in one workgroup per robot
// (SR_AESC1) or in two side by side (SR_AESC)
#define SR_AESC1(NN, BS, LG, XC, GBS)                                                                           \
    {                                                                                                          \
        NN, BS, k_adjoint<NN + 1, BS, false, true, LG, false, false, false, true, XC>,                          \
            k_adjoint<NN + 1, BS, true, true, LG, false, false, false, true, XC>, GBS,                          \
            k_adj_grad<NN + 1, GBS, false, 0, 13>, k_adj_grad<NN + 1, GBS, true, 0, 13>                          \
    }
#define SR_AESC(NN, BS, LG, XC, GBS)                                                                            \
    {                                                                                                          \
        NN, BS, k_adjoint<NN + 1, BS, false, true, LG, false, false, false, true, XC>,                          \
            k_adjoint<NN + 1, BS, true, true, LG, false, false, false, true, XC>, GBS,                          \
            k_adj_grad<NN + 1, GBS, false, 0, 7, 13>, k_adj_grad<NN + 1, GBS, true, 0, 7, 13>, 2                 \
    }
const AdjEntry kAdj[] = {SR_AE(1, 64, true),    SR_AE(2, 64, true),    SR_AE(3, 64, true),   SR_AEL(4, 128, 2),
                         SR_AEL(5, 256, 2),     SR_AEL(6, 384, 2),     SR_AEL(7, 512, 2),    SR_AESL(8, 768, 2, 768),
                         SR_AESC1(9, 1024, 2, 2, 1024), SR_AESC(10, 768, 2, 3, 704), SR_AESC(11, 1024, 0, 4, 1024),
                         SR_AESC(12, 768, 0, 7, 768)};
// spring dashpots or the damped ground (Table II model): the one-buffer
// recompute form with the velocity terms
#define SR_AED(NN, BS) \
    { NN, BS, k_adjoint<NN + 1, BS, false, false, 0, true, true>, k_adjoint<NN + 1, BS, true, false, 0, true, true> }
// the exchange form with the velocity terms: four rows per direction (K_s u and
// the scalar of the upper end's velocity-adjoint term), XC direction chunks
#define SR_AEDX(NN, BS, XC)                                                                                    \
    {                                                                                                          \
        NN, BS, k_adjoint<NN + 1, BS, false, true, 0, false, true, false, false, XC>,                           \
            k_adjoint<NN + 1, BS, true, true, 0, false, true, false, false, XC>                                 \
    }
// split form of the above: the reverse recursion alone, then the gradient
// pass with the dashpot terms in two direction halves side by side
#define SR_AEDS(NN, BS, XC, GBS)                                                                               \
    {                                                                                                          \
        NN, BS, k_adjoint<NN + 1, BS, false, true, 0, false, true, false, true, XC>,                            \
            k_adjoint<NN + 1, BS, true, true, 0, false, true, false, true, XC>, GBS,                            \
            k_adj_grad<NN + 1, GBS, false, 0, 7, 13, true>, k_adj_grad<NN + 1, GBS, true, 0, 7, 13, true>, 2     \
    }
const AdjEntry kAdjD[] = {SR_AED(1, 64),        SR_AED(2, 64),        SR_AED(3, 64),        SR_AEDX(4, 128, 1),
                          SR_AEDX(5, 256, 1),   SR_AEDX(6, 384, 1),   SR_AEDX(7, 512, 1),   SR_AEDS(8, 768, 2, 768),
                          SR_AEDS(9, 1024, 3, 1024), SR_AEDS(10, 768, 5, 768), SR_AEDS(11, 1024, 7, 1024),
                          SR_AEDS(12, 768, 13, 768)};

}  // namespace

bool adjoint_is_split(int n, bool vel) {
    for (const auto &q : (vel ? kAdjD : kAdj))
        if (q.n == n) return q.g0 != nullptr;
    return false;
}

hipError_t launch_adjoint(int n, bool phase, const RobotInfo *robots, const int32_t *list, int count, Planes pl,
                          const float4 *x0, const float4 *rec_x, const float4 *rec_v, const float4 *rec_u,
                          float4 *rec_l, int n_steps, const float2 *sc, float4 *lx, float4 *lv, float *gk, float *gs,
                          float *gc, float *gd, SimConst c, hipStream_t st) {
    const bool vel = c.dash || c.gdamp;  // forces that depend on the velocities
    if (vel && (!rec_u || !gd)) return hipErrorInvalidValue;
    const AdjEntry *e = nullptr;
    for (const auto &q : (vel ? kAdjD : kAdj))
        if (q.n == n) e = &q;
    if (!e) return hipErrorInvalidConfiguration;
    AArgs A;
    A.robots = robots;
    A.list = list;
    A.count = count;
    A.pl = pl;
    A.x0 = x0;
    A.rec_x = rec_x;
    A.rec_v = rec_v;
    A.rec_u = rec_u;
    A.rec_l = rec_l;
    A.n_steps = n_steps;
    A.sc = sc;
    A.lx = lx;
    A.lv = lv;
    A.gk = gk;
    A.gs = gs;
    A.gc = gc;
    A.gd = gd;
    A.c = c;
    if (e->g0 && !rec_l) return hipErrorInvalidValue;
    hipLaunchKernelGGL(phase ? e->fn_phase : e->fn, dim3(count), dim3(e->block), 0, st, A);
    return hipGetLastError();
}

hipError_t launch_adj_grad(int n, bool phase, const RobotInfo *robots, const int32_t *list, int count, Planes pl,
                           const float4 *x0, const float4 *rec_x, const float4 *rec_u, float4 *rec_l, int n_steps,
                           const float2 *sc, float *gk, float *gs, float *gc, float *gd, SimConst c, hipStream_t st) {
    const bool vel = c.dash || c.gdamp;
    if (vel && (!rec_u || !gd)) return hipErrorInvalidValue;
    const AdjEntry *e = nullptr;
    for (const auto &q : (vel ? kAdjD : kAdj))
        if (q.n == n) e = &q;
    if (!e || !e->g0 || !rec_l) return hipErrorInvalidValue;
    AArgs A = {};
    A.robots = robots;
    A.list = list;
    A.count = count;
    A.pl = pl;
    A.x0 = x0;
    A.rec_x = rec_x;
    A.rec_u = rec_u;
    A.rec_l = rec_l;
    A.n_steps = n_steps;
    A.sc = sc;
    A.gk = gk;
    A.gs = gs;
    A.gc = gc;
    A.gd = gd;
    A.c = c;
    hipLaunchKernelGGL(phase ? e->g0_phase : e->g0, dim3(count, e->gy), dim3(e->gblock), 0, st, A);
    return hipGetLastError();
}

hipError_t launch_adj_init(const RobotInfo *robots, int total_slots, const int32_t *slot_robot, const float4 *x0,
                           const float *dJ, float4 *lx, float4 *lv, float *gk, float *gs, float *gc, float *gd,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_adj_init, dim3((total_slots + 255) / 256), dim3(256), 0, st, robots, total_slots, slot_robot,
                       x0, dJ, lx, lv, gk, gs, gc, gd);
    return hipGetLastError();
}

hipError_t launch_adj_springs(const RobotInfo *robots, int total_slots, const int32_t *slot_robot, const int32_t *sid,
                              const int64_t *spring_off, Planes pl, float voxel_len, const float *gk, const float *gs,
                              const float *gc, float *g_k, float *g_a, float *g_phi, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_springs, dim3((total_slots + 255) / 256), dim3(256), 0, st, robots, total_slots,
                       slot_robot, sid, spring_off, pl, voxel_len, gk, gs, gc, g_k, g_a, g_phi);
    return hipGetLastError();
}

hipError_t launch_adj_genome(const RobotInfo *robots, int R, int total_vox, const int32_t *vox_robot,
                             const uint8_t *kept, const float *w, Planes pl, const float *gk, const float *gs,
                             const float *gc, const float *gd, const sr_sim_params &p, const float *genomes,
                             const float *B, float *dJdw, float *g_gen, hipStream_t st) {
    DwArgs A;
    A.robots = robots;
    A.total_vox = total_vox;
    A.vox_robot = vox_robot;
    A.kept = kept;
    A.w = w;
    A.pl = pl;
    A.gk = gk;
    A.gs = gs;
    A.gc = gc;
    A.gd = p.zeta_spring != 0.f ? gd : nullptr;
    A.dash_c = (float)(0.5 * (double)p.zeta_spring * sqrt(2.0 * (double)p.mass));
    for (int c = 0; c < 5; ++c) {
        A.k_class[c] = p.k_class[c];
        A.a_class[c] = p.a_class[c];
        A.phi_class[c] = p.phi_class[c];
    }
    A.weight_act = (p.flags & SR_WEIGHT_ACTUATION) != 0;
    A.voxel_len = p.voxel_len;
    A.dJdw = dJdw;
    hipLaunchKernelGGL(k_adj_dw, dim3((total_vox + 255) / 256), dim3(256), 0, st, A);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_backward, dim3(R), dim3(256), 0, st, robots, genomes, B, dJdw, g_gen);
    return hipGetLastError();
}

}  // namespace sr

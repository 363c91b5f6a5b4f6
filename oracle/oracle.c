/*
 * oracle.c -- plain, slow FP64 CPU oracle for the soft-robot co-design hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant generator with the HIP library; both sides only
 * consume the same seeded inputs.
 *
 * What it follows (arXiv 2405.00698, "CUDA-Accelerated Soft Robot Neural
 * Evolution with Large Language Model Supervision"):
 *   - Sec. II-B, Eq. (1): Gaussian positional encoding
 *       gamma(v) = [cos(2 pi B v), sin(2 pi B v)]^T, B entries ~ N(0, sigma^2).
 *   - Sec. II-A: 3D voxel robot, materials {empty, expanding muscle,
 *     contracting muscle, soft tissue, hard bone}.
 *   - Sec. II-C: one MLP genome per robot; a softmax branch picks the material
 *     category, a sigmoid branch gives a weight that multiplies the material
 *     parameter; crossover, mutation and elite selection over the population.
 *   - Table I (GA rates) and Table II (physics, material, plane parameters).
 * The paper gives no integrator, force law, contact model, MLP shape or GA
 * operator details; the readings used here are listed in the design notes
 * (voxel edge = rest length, parallel-sum rule for shared springs,
 * symplectic Euler with Jacobi forces, penalty ground, velocity-level Coulomb
 * friction, per-step velocity damping, COM-x fitness, Philox-4x64-10 RNG).
 *
 * Everything is the definition written out: forces are summed over the
 * canonical spring list, the adjoint stores every state and reverses each
 * forward operation, the GA enumerates its random draws one by one.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define OR_PI 3.14159265358979323846

/* simulation switches (test modes) */
#define OR_NO_GRAVITY 1
#define OR_NO_GROUND 2
#define OR_NO_ACTUATION 4
/* Table II material model: the sigmoid weight also scales each muscle voxel's
 * actuation amplitude and phase (Sec. II-C; Table II maximum amplitude and phase) */
#define OR_WEIGHT_ACTUATION 8

/* genome layout: W1[64][64] b1[64] W2[64][64] b2[64] W3[6][64] b3[6] */
#define OR_PE_M 32
#define OR_HID 64
#define OR_NOUT 6
#define OR_OFF_W1 0
#define OR_OFF_B1 (OR_OFF_W1 + OR_HID * 2 * OR_PE_M)
#define OR_OFF_W2 (OR_OFF_B1 + OR_HID)
#define OR_OFF_B2 (OR_OFF_W2 + OR_HID * OR_HID)
#define OR_OFF_W3 (OR_OFF_B2 + OR_HID)
#define OR_OFF_B3 (OR_OFF_W3 + OR_NOUT * OR_HID)
#define OR_GENOME_LEN (OR_OFF_B3 + OR_NOUT)

typedef struct {
    double dt;          /* time step [s] */
    double gravity;     /* |g| [m/s^2], acts along -z */
    double damping;     /* velocity factor per step */
    double mass;        /* mass of every node [kg] */
    double voxel_len;   /* voxel edge = rest length of an edge spring [m] */
    double k_ground;    /* ground penalty stiffness [N/m] */
    double mu;          /* Coulomb friction coefficient */
    double act_freq;    /* muscle actuation frequency [Hz] */
    double k_class[5];  /* stiffness per material class [N/m] */
    double a_class[5];  /* actuation amplitude per class (relative to L0) */
    double phi_class[5];/* actuation phase per class [rad] */
    int32_t flags;
    /* Table II extensions; zero gives the base model */
    double mu_static;   /* static friction coefficient (acts only above mu) */
    double zeta_spring; /* damping ratio of the dashpot beside every spring */
    double zeta_ground; /* damping ratio of the ground contact */
} or_params;

int or_genome_len(void) { return OR_GENOME_LEN; }

/* ------------------------------------------------------------------------ */
/* Build step: encoding, MLP, heads                                          */
/* ------------------------------------------------------------------------ */

/* Eq. (1): first the m cosines, then the m sines of 2 pi B v. */
void or_encode(const double *B, const double *v, double *g)
{
    for (int q = 0; q < OR_PE_M; ++q) {
        double t = 2.0 * OR_PI * (B[3 * q + 0] * v[0] + B[3 * q + 1] * v[1] + B[3 * q + 2] * v[2]);
        g[q] = cos(t);
        g[OR_PE_M + q] = sin(t);
    }
}

/* MLP of Sec. II-C: two tanh layers of 64 and a 6-output linear layer. */
void or_mlp(const double *gen, const double *g, double *h1, double *h2, double *o)
{
    const double *W1 = gen + OR_OFF_W1, *b1 = gen + OR_OFF_B1;
    const double *W2 = gen + OR_OFF_W2, *b2 = gen + OR_OFF_B2;
    const double *W3 = gen + OR_OFF_W3, *b3 = gen + OR_OFF_B3;
    for (int i = 0; i < OR_HID; ++i) {
        double s = b1[i];
        for (int j = 0; j < 2 * OR_PE_M; ++j) s += W1[i * 2 * OR_PE_M + j] * g[j];
        h1[i] = tanh(s);
    }
    for (int i = 0; i < OR_HID; ++i) {
        double s = b2[i];
        for (int j = 0; j < OR_HID; ++j) s += W2[i * OR_HID + j] * h1[j];
        h2[i] = tanh(s);
    }
    for (int i = 0; i < OR_NOUT; ++i) {
        double s = b3[i];
        for (int j = 0; j < OR_HID; ++j) s += W3[i * OR_HID + j] * h2[j];
        o[i] = s;
    }
}

/* Query point of voxel (i,j,k) on an n^3 grid: its centre in (0,1)^3. */
static void voxel_centre(int n, int vid, double *v)
{
    int i = vid % n, j = (vid / n) % n, k = vid / (n * n);
    v[0] = (i + 0.5) / n;
    v[1] = (j + 0.5) / n;
    v[2] = (k + 0.5) / n;
}

/* logits[n^3][6] of one robot's genome over its grid. */
int or_query(const double *genome, const double *B, int n, double *logits)
{
    if (n < 1) return -1;
    double v[3], g[2 * OR_PE_M], h1[OR_HID], h2[OR_HID];
    for (int vid = 0; vid < n * n * n; ++vid) {
        voxel_centre(n, vid, v);
        or_encode(B, v, g);
        or_mlp(genome, g, h1, h2, logits + 6 * vid);
    }
    return 0;
}

/* Heads: the softmax branch's category is the argmax of logits 0..4 (softmax
 * is monotone); ties go to the lowest class id.  The sigmoid branch gives
 * w = 1 / (1 + exp(-o5)). */
void or_heads(const double *logits, int nvox, uint8_t *cls, double *w)
{
    for (int v = 0; v < nvox; ++v) {
        const double *o = logits + 6 * v;
        int best = 0;
        for (int q = 1; q < 5; ++q)
            if (o[q] > o[best]) best = q;
        cls[v] = (uint8_t)best;
        w[v] = 1.0 / (1.0 + exp(-o[5]));
    }
}

/* ------------------------------------------------------------------------ */
/* Morphology: largest face-connected component                              */
/* ------------------------------------------------------------------------ */

/* kept[v] = cls[v] if voxel v is in the largest 6-connected component of the
 * occupied (cls != 0) voxels, else 0.  Ties between equally large components
 * go to the one holding the smallest linear voxel id.  Returns its size. */
int or_lcc(const uint8_t *cls, int n, uint8_t *kept)
{
    int nv = n * n * n;
    int *comp = (int *)malloc(sizeof(int) * nv);
    int *stack = (int *)malloc(sizeof(int) * nv);
    for (int v = 0; v < nv; ++v) comp[v] = -1;
    int best_root = -1, best_size = 0;
    for (int v = 0; v < nv; ++v) {
        if (cls[v] == 0 || comp[v] >= 0) continue;
        /* depth-first flood fill from v, which is the component's smallest id */
        int size = 0, top = 0;
        stack[top++] = v;
        comp[v] = v;
        while (top > 0) {
            int u = stack[--top];
            ++size;
            int i = u % n, j = (u / n) % n, k = u / (n * n);
            int nb[6], c = 0;
            if (i > 0) nb[c++] = u - 1;
            if (i < n - 1) nb[c++] = u + 1;
            if (j > 0) nb[c++] = u - n;
            if (j < n - 1) nb[c++] = u + n;
            if (k > 0) nb[c++] = u - n * n;
            if (k < n - 1) nb[c++] = u + n * n;
            for (int q = 0; q < c; ++q) {
                int w = nb[q];
                if (cls[w] != 0 && comp[w] < 0) {
                    comp[w] = v;
                    stack[top++] = w;
                }
            }
        }
        if (size > best_size) { best_size = size; best_root = v; }
    }
    for (int v = 0; v < nv; ++v) kept[v] = (best_root >= 0 && comp[v] == best_root) ? cls[v] : 0;
    free(comp);
    free(stack);
    return best_size;
}

/* ------------------------------------------------------------------------ */
/* Robot: nodes, springs, state                                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    or_params p;
    int n, N;          /* voxels per side, lattice points per side (n + 1) */
    int M, S;          /* nodes, springs */
    uint8_t *kept;     /* [n^3] class of kept voxels, 0 elsewhere */
    double *w;         /* [n^3] sigmoid weight per voxel */
    int32_t *node_lat; /* [M] lattice index a + N (b + N c) */
    int32_t *lat_node; /* [N^3] node id or -1 */
    int32_t *ij;       /* [S][2] node ids, ij[2s] < ij[2s+1] */
    double *L0, *k, *a, *phi; /* [S] rest length, stiffness, amplitude, phase */
    double *cd;        /* [S] dashpot coefficient [N s/m] */
    int32_t *sv_ptr;   /* [S+1] range of voxels holding each spring */
    int32_t *sv;       /* voxel ids */
    double *x, *v, *x0;/* [M][3] */
    int64_t step;
    int diverged;
} or_robot;

typedef struct { int32_t lo, hi, vox; } pair_t;

static int cmp_pair(const void *A, const void *B)
{
    const pair_t *a = (const pair_t *)A, *b = (const pair_t *)B;
    if (a->lo != b->lo) return a->lo < b->lo ? -1 : 1;
    if (a->hi != b->hi) return a->hi < b->hi ? -1 : 1;
    return (a->vox > b->vox) - (a->vox < b->vox);
}

/* Actuation amplitude and phase of one voxel of class c and weight w.  Base
 * model: the class values.  Table II model: the weight scales both, up to the
 * class maxima. */
static void voxel_actuation(const or_params *p, int c, double w, double *amp, double *ph)
{
    if (p->flags & OR_WEIGHT_ACTUATION) {
        *amp = w * p->a_class[c];
        *ph = w * p->phi_class[c];
    } else {
        *amp = p->a_class[c];
        *ph = p->phi_class[c];
    }
}

/* Spring parameters by the parallel-sum rule: a spring shared by several
 * kept voxels is the parallel combination of their springs, so
 *   k_s = sum_v k_c(v) w(v),   k_s a_s e^{i phi_s} = sum_v k_c(v) w(v) a_v e^{i phi_v},
 * and the dashpots beside them add too: c_s = sum_v zeta sqrt(2 m k_c(v) w(v))
 * (damping ratio zeta of each voxel spring between two nodes of mass m).
 * When every term is in phase the amplitude is kept signed with phi = 0. */
static void spring_params_from_voxels(or_robot *R, int s)
{
    double ks = 0.0, zr = 0.0, zi = 0.0, cs = 0.0;
    for (int q = R->sv_ptr[s]; q < R->sv_ptr[s + 1]; ++q) {
        int v = R->sv[q];
        int c = R->kept[v];
        double kw = R->p.k_class[c] * R->w[v];
        double amp, ph;
        voxel_actuation(&R->p, c, R->w[v], &amp, &ph);
        ks += kw;
        zr += kw * amp * cos(ph);
        zi += kw * amp * sin(ph);
        cs += R->p.zeta_spring * sqrt(2.0 * R->p.mass * kw);
    }
    R->k[s] = ks;
    R->cd[s] = cs;
    if (ks == 0.0) { R->a[s] = 0.0; R->phi[s] = 0.0; }
    else if (zi == 0.0) { R->a[s] = zr / ks; R->phi[s] = 0.0; }
    else { R->a[s] = sqrt(zr * zr + zi * zi) / ks; R->phi[s] = atan2(zi, zr); }
}

static void robot_reset_state(or_robot *R)
{
    double zmin = 1e300;
    for (int i = 0; i < R->M; ++i) {
        int l = R->node_lat[i];
        int c = l / (R->N * R->N);
        double z = R->p.voxel_len * c;
        if (z < zmin) zmin = z;
    }
    for (int i = 0; i < R->M; ++i) {
        int l = R->node_lat[i];
        int a = l % R->N, b = (l / R->N) % R->N, c = l / (R->N * R->N);
        R->x0[3 * i + 0] = R->p.voxel_len * a;
        R->x0[3 * i + 1] = R->p.voxel_len * b;
        R->x0[3 * i + 2] = R->p.voxel_len * c - zmin;
        for (int d = 0; d < 3; ++d) { R->x[3 * i + d] = R->x0[3 * i + d]; R->v[3 * i + d] = 0.0; }
    }
    R->step = 0;
    R->diverged = 0;
}

void or_robot_destroy(or_robot *R)
{
    if (!R) return;
    free(R->kept); free(R->w); free(R->node_lat); free(R->lat_node); free(R->ij);
    free(R->L0); free(R->k); free(R->a); free(R->phi); free(R->cd); free(R->sv_ptr); free(R->sv);
    free(R->x); free(R->v); free(R->x0);
    free(R);
}

/* Build a robot from per-voxel classes and weights (Sec. II-A, II-C):
 * keep the largest component, put a node on every corner of a kept voxel
 * (ids ascending in lattice index), a spring on each of the 28 corner pairs
 * of each kept voxel (12 edges, 12 face diagonals, 4 body diagonals),
 * deduplicated and ordered by (min id, max id).  Returns NULL when no voxel
 * is occupied. */
or_robot *or_robot_create(const or_params *p, int n, const uint8_t *cls, const double *w)
{
    if (n < 1) return NULL;
    int nv = n * n * n, N = n + 1, NL = N * N * N;
    or_robot *R = (or_robot *)calloc(1, sizeof(or_robot));
    R->p = *p;
    R->n = n;
    R->N = N;
    R->kept = (uint8_t *)malloc(nv);
    R->w = (double *)malloc(sizeof(double) * nv);
    memcpy(R->w, w, sizeof(double) * nv);
    int kept_count = or_lcc(cls, n, R->kept);
    if (kept_count == 0) { or_robot_destroy(R); return NULL; }

    /* nodes */
    R->lat_node = (int32_t *)malloc(sizeof(int32_t) * NL);
    for (int l = 0; l < NL; ++l) R->lat_node[l] = -1;
    for (int vid = 0; vid < nv; ++vid) {
        if (!R->kept[vid]) continue;
        int i = vid % n, j = (vid / n) % n, kk = vid / (n * n);
        for (int c = 0; c < 8; ++c) {
            int l = (i + (c & 1)) + N * ((j + ((c >> 1) & 1)) + N * (kk + ((c >> 2) & 1)));
            R->lat_node[l] = 0;
        }
    }
    R->M = 0;
    for (int l = 0; l < NL; ++l)
        if (R->lat_node[l] >= 0) R->lat_node[l] = R->M++;
    R->node_lat = (int32_t *)malloc(sizeof(int32_t) * R->M);
    for (int l = 0; l < NL; ++l)
        if (R->lat_node[l] >= 0) R->node_lat[R->lat_node[l]] = l;

    /* all corner pairs of all kept voxels */
    pair_t *pr = (pair_t *)malloc(sizeof(pair_t) * 28 * kept_count);
    int np = 0;
    for (int vid = 0; vid < nv; ++vid) {
        if (!R->kept[vid]) continue;
        int i = vid % n, j = (vid / n) % n, kk = vid / (n * n);
        int corner[8];
        for (int c = 0; c < 8; ++c)
            corner[c] = (i + (c & 1)) + N * ((j + ((c >> 1) & 1)) + N * (kk + ((c >> 2) & 1)));
        for (int c1 = 0; c1 < 8; ++c1)
            for (int c2 = c1 + 1; c2 < 8; ++c2) {
                int l1 = corner[c1], l2 = corner[c2];
                pr[np].lo = l1 < l2 ? l1 : l2;
                pr[np].hi = l1 < l2 ? l2 : l1;
                pr[np].vox = vid;
                ++np;
            }
    }
    qsort(pr, np, sizeof(pair_t), cmp_pair);
    int S = 0;
    for (int q = 0; q < np; ++q)
        if (q == 0 || pr[q].lo != pr[q - 1].lo || pr[q].hi != pr[q - 1].hi) ++S;
    R->S = S;
    R->ij = (int32_t *)malloc(sizeof(int32_t) * 2 * S);
    R->L0 = (double *)malloc(sizeof(double) * S);
    R->k = (double *)malloc(sizeof(double) * S);
    R->a = (double *)malloc(sizeof(double) * S);
    R->phi = (double *)malloc(sizeof(double) * S);
    R->cd = (double *)malloc(sizeof(double) * S);
    R->sv_ptr = (int32_t *)malloc(sizeof(int32_t) * (S + 1));
    R->sv = (int32_t *)malloc(sizeof(int32_t) * np);
    int s = -1;
    for (int q = 0; q < np; ++q) {
        if (q == 0 || pr[q].lo != pr[q - 1].lo || pr[q].hi != pr[q - 1].hi) {
            ++s;
            R->sv_ptr[s] = q;
            R->ij[2 * s] = R->lat_node[pr[q].lo];
            R->ij[2 * s + 1] = R->lat_node[pr[q].hi];
            int d0 = pr[q].hi % N - pr[q].lo % N;
            int d1 = (pr[q].hi / N) % N - (pr[q].lo / N) % N;
            int d2 = pr[q].hi / (N * N) - pr[q].lo / (N * N);
            R->L0[s] = p->voxel_len * sqrt((double)(d0 * d0 + d1 * d1 + d2 * d2));
        }
        R->sv[q] = pr[q].vox;
    }
    R->sv_ptr[S] = np;
    free(pr);
    for (s = 0; s < S; ++s) spring_params_from_voxels(R, s);

    R->x = (double *)malloc(sizeof(double) * 3 * R->M);
    R->v = (double *)malloc(sizeof(double) * 3 * R->M);
    R->x0 = (double *)malloc(sizeof(double) * 3 * R->M);
    robot_reset_state(R);
    return R;
}

void or_robot_counts(const or_robot *R, int32_t *M, int32_t *S)
{
    *M = R->M;
    *S = R->S;
}

void or_robot_voxels(const or_robot *R, uint8_t *kept)
{
    memcpy(kept, R->kept, R->n * R->n * R->n);
}

void or_robot_nodes(const or_robot *R, int32_t *node_lat) { memcpy(node_lat, R->node_lat, sizeof(int32_t) * R->M); }

void or_robot_springs(const or_robot *R, int32_t *ij, double *L0, double *k, double *a, double *phi)
{
    if (ij) memcpy(ij, R->ij, sizeof(int32_t) * 2 * R->S);
    if (L0) memcpy(L0, R->L0, sizeof(double) * R->S);
    if (k) memcpy(k, R->k, sizeof(double) * R->S);
    if (a) memcpy(a, R->a, sizeof(double) * R->S);
    if (phi) memcpy(phi, R->phi, sizeof(double) * R->S);
}

void or_robot_set_springs(or_robot *R, const double *k, const double *a, const double *phi)
{
    if (k) memcpy(R->k, k, sizeof(double) * R->S);
    if (a) memcpy(R->a, a, sizeof(double) * R->S);
    if (phi) memcpy(R->phi, phi, sizeof(double) * R->S);
}

void or_robot_get_state(const or_robot *R, double *x, double *v, int64_t *step, int32_t *diverged)
{
    if (x) memcpy(x, R->x, sizeof(double) * 3 * R->M);
    if (v) memcpy(v, R->v, sizeof(double) * 3 * R->M);
    if (step) *step = R->step;
    if (diverged) *diverged = R->diverged;
}

void or_robot_set_state(or_robot *R, const double *x, const double *v, int64_t step)
{
    if (x) memcpy(R->x, x, sizeof(double) * 3 * R->M);
    if (v) memcpy(R->v, v, sizeof(double) * 3 * R->M);
    R->step = step;
}

void or_robot_get_x0(const or_robot *R, double *x0) { memcpy(x0, R->x0, sizeof(double) * 3 * R->M); }

/* ------------------------------------------------------------------------ */
/* Time step                                                                 */
/* ------------------------------------------------------------------------ */

/* Actuated rest length of spring s at time t = step * dt:
 * L = L0 (1 + a sin(2 pi f t + phi)); muscles follow a sinusoid. */
static double rest_length(const or_robot *R, int s, int64_t step)
{
    if (R->p.flags & OR_NO_ACTUATION) return R->L0[s];
    double t = (double)step * R->p.dt;
    return R->L0[s] * (1.0 + R->a[s] * sin(2.0 * OR_PI * R->p.act_freq * t + R->phi[s]));
}

/* Ground normal force on a node at height z with vertical velocity vz:
 * zero above the plane; below it the penalty k_ground (-z) plus, in the
 * Table II model, a contact damper -c_g vz with c_g = 2 zeta_g sqrt(k_ground m),
 * never pulling the node down (the total is clamped at zero). */
static double ground_normal(const or_robot *R, double z, double vz)
{
    if ((R->p.flags & OR_NO_GROUND) || !(z < 0.0)) return 0.0;
    double N = R->p.k_ground * (-z);
    if (R->p.zeta_ground != 0.0) {
        N -= 2.0 * R->p.zeta_ground * sqrt(R->p.k_ground * R->p.mass) * vz;
        if (N < 0.0) N = 0.0;
    }
    return N;
}

/* Total force on every node at state (x, v), time step `step`:
 * Hooke springs f_s = k_s (r - L_s) along the spring, a dashpot
 * c_s (v_j - v_i).d^ beside each spring, gravity -m g e_z, and the ground
 * normal. */
static void forces(const or_robot *R, const double *x, const double *v, int64_t step, double *F)
{
    memset(F, 0, sizeof(double) * 3 * R->M);
    for (int s = 0; s < R->S; ++s) {
        int i = R->ij[2 * s], j = R->ij[2 * s + 1];
        double d[3] = {x[3 * j] - x[3 * i], x[3 * j + 1] - x[3 * i + 1], x[3 * j + 2] - x[3 * i + 2]};
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (r < 1e-9) continue; /* a collapsed spring has no direction */
        double f = R->k[s] * (r - rest_length(R, s, step));
        if (R->cd[s] != 0.0) {
            double rate = 0.0; /* (v_j - v_i) . d / r */
            for (int q = 0; q < 3; ++q) rate += (v[3 * j + q] - v[3 * i + q]) * d[q] / r;
            f += R->cd[s] * rate;
        }
        for (int q = 0; q < 3; ++q) {
            F[3 * i + q] += f * d[q] / r;
            F[3 * j + q] -= f * d[q] / r;
        }
    }
    for (int i = 0; i < R->M; ++i) {
        if (!(R->p.flags & OR_NO_GRAVITY)) F[3 * i + 2] -= R->p.mass * R->p.gravity;
        F[3 * i + 2] += ground_normal(R, x[3 * i + 2], v[3 * i + 2]);
    }
}

/* Velocity-level Coulomb friction for a node pressed on the ground with
 * normal force N: the tangential velocity u sticks (becomes zero) when
 * |u| <= max(mu_s, mu_k) N dt / m, and otherwise loses mu_k N dt / m of its
 * length without reversing.  mu_s only matters when it exceeds mu_k. */
static void friction(const or_robot *R, double N, double *vp)
{
    if (!(N > 0.0)) return;
    double dvk = R->p.mu * N * R->p.dt / R->p.mass;
    double dvs = R->p.mu_static * N * R->p.dt / R->p.mass;
    double u = sqrt(vp[0] * vp[0] + vp[1] * vp[1]);
    if (u <= dvk || u <= dvs) { vp[0] = 0.0; vp[1] = 0.0; }
    else { vp[0] *= (1.0 - dvk / u); vp[1] *= (1.0 - dvk / u); }
}

static int robot_state_bad(const or_robot *R)
{
    double lim = 1e3 * R->n * R->p.voxel_len;
    for (int q = 0; q < 3 * R->M; ++q)
        if (!isfinite(R->x[q]) || !isfinite(R->v[q]) || fabs(R->x[q]) > lim) return 1;
    return 0;
}

/* One explicit step n -> n+1 (semi-implicit Euler, all forces from x_n):
 *   v' = v + dt F(x_n, t_n) / m;  friction on v' where z_n < 0;
 *   v_{n+1} = damping * v';  x_{n+1} = x_n + dt v_{n+1}. */
static void step_once(or_robot *R, double *F)
{
    forces(R, R->x, R->v, R->step, F);
    for (int i = 0; i < R->M; ++i) {
        double vp[3];
        double N = ground_normal(R, R->x[3 * i + 2], R->v[3 * i + 2]);
        for (int q = 0; q < 3; ++q) vp[q] = R->v[3 * i + q] + R->p.dt * F[3 * i + q] / R->p.mass;
        friction(R, N, vp);
        for (int q = 0; q < 3; ++q) {
            R->v[3 * i + q] = R->p.damping * vp[q];
            R->x[3 * i + q] += R->p.dt * R->v[3 * i + q];
        }
    }
    R->step += 1;
}

/* Advance n_steps.  A robot whose state is non-finite or absurdly far away at
 * the end of a call is flagged as diverged and is not stepped again. */
int or_robot_step(or_robot *R, int n_steps)
{
    if (R->diverged) return 0;
    double *F = (double *)malloc(sizeof(double) * 3 * R->M);
    for (int t = 0; t < n_steps; ++t) step_once(R, F);
    free(F);
    if (robot_state_bad(R)) R->diverged = 1;
    return 0;
}

/* Many robots at once, one robot per host thread (used for CPU timing). */
int or_pop_step(or_robot **robots, int n_robots, int n_steps)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < n_robots; ++r) or_robot_step(robots[r], n_steps);
    return 0;
}

int or_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

/* Fitness: displacement of the centre of mass along +x since the build
 * (equal node masses, so the COM is the node mean).  -inf when diverged. */
double or_robot_fitness(const or_robot *R)
{
    if (R->diverged || robot_state_bad(R)) return -INFINITY;
    double s = 0.0;
    for (int i = 0; i < R->M; ++i) s += R->x[3 * i] - R->x0[3 * i];
    return s / R->M;
}

/* Diagnostics for the invariant pins. */
void or_robot_momentum(const or_robot *R, double *P, double *Lang)
{
    double m = R->p.mass;
    for (int q = 0; q < 3; ++q) { P[q] = 0.0; Lang[q] = 0.0; }
    for (int i = 0; i < R->M; ++i) {
        const double *x = R->x + 3 * i, *v = R->v + 3 * i;
        for (int q = 0; q < 3; ++q) P[q] += m * v[q];
        Lang[0] += m * (x[1] * v[2] - x[2] * v[1]);
        Lang[1] += m * (x[2] * v[0] - x[0] * v[2]);
        Lang[2] += m * (x[0] * v[1] - x[1] * v[0]);
    }
}

/* Kinetic + spring (at the un-actuated rest length) + gravity + ground energy. */
double or_robot_energy(const or_robot *R)
{
    double E = 0.0, m = R->p.mass;
    for (int i = 0; i < R->M; ++i) {
        const double *x = R->x + 3 * i, *v = R->v + 3 * i;
        E += 0.5 * m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        if (!(R->p.flags & OR_NO_GRAVITY)) E += m * R->p.gravity * x[2];
        if (!(R->p.flags & OR_NO_GROUND) && x[2] < 0.0) E += 0.5 * R->p.k_ground * x[2] * x[2];
    }
    for (int s = 0; s < R->S; ++s) {
        int i = R->ij[2 * s], j = R->ij[2 * s + 1];
        double d0 = R->x[3 * j] - R->x[3 * i], d1 = R->x[3 * j + 1] - R->x[3 * i + 1], d2 = R->x[3 * j + 2] - R->x[3 * i + 2];
        double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        E += 0.5 * R->k[s] * (r - R->L0[s]) * (r - R->L0[s]);
    }
    return E;
}

/* ------------------------------------------------------------------------ */
/* Adjoint                                                                   */
/* ------------------------------------------------------------------------ */

/* Gradient of J = g * fitness after n_steps from the robot's current state
 * with respect to every spring's parameters, by reverse accumulation through
 * each forward operation (every state stored).  Contact and friction branches
 * are the ones the forward run took, and so is the clamp of the damped ground
 * force at zero.  The robot itself is not modified.
 * Two parametrisations of the actuated rest length
 *   L = L0 (1 + a sin(w t + phi)) = L0 + L0 (Zr sin wt + Zi cos wt) / k,
 * Z = k a e^{i phi}, are reported: (gk, ga, gphi) = dJ/d(k, a, phi) and
 * (gkz, gzr, gzi) = dJ/d(k, Zr, Zi) (k at fixed Z); gcd = dJ/dc per spring
 * dashpot coefficient (k, a, phi at fixed c); any output may be NULL.
 * With the dashpots (Table II model) a spring's force is
 *   f = k (r - L) + c (v_j - v_i).d^
 * and the ground's normal force N = k_ground (-z) - c_g v_z (clamped at zero),
 * so the forces also depend on the velocities of the step: the reverse step
 * adds dF/dv^T lambda_F to the velocity adjoint. */
static double backward_impl(const or_robot *R, int n_steps, double g, double *gk, double *ga, double *gphi,
                            double *gkz, double *gzr, double *gzi, double *gcd)
{
    int M = R->M, S = R->S;
    const or_params *p = &R->p;
    double cg = 2.0 * p->zeta_ground * sqrt(p->k_ground * p->mass); /* ground damper, as in ground_normal */
    double m = p->mass, dt = p->dt;
    int ground = !(p->flags & OR_NO_GROUND);
    int act = !(p->flags & OR_NO_ACTUATION);
    double *xs = (double *)malloc(sizeof(double) * 3 * M * (size_t)(n_steps + 1));
    double *vs = (double *)malloc(sizeof(double) * 3 * M * (size_t)(n_steps + 1));
    double *F = (double *)malloc(sizeof(double) * 3 * M);
    or_robot tmp = *R; /* shallow copy with private state arrays */
    tmp.x = (double *)malloc(sizeof(double) * 3 * M);
    tmp.v = (double *)malloc(sizeof(double) * 3 * M);
    memcpy(tmp.x, R->x, sizeof(double) * 3 * M);
    memcpy(tmp.v, R->v, sizeof(double) * 3 * M);
    memcpy(xs, tmp.x, sizeof(double) * 3 * M);
    memcpy(vs, tmp.v, sizeof(double) * 3 * M);
    for (int t = 0; t < n_steps; ++t) {
        step_once(&tmp, F);
        memcpy(xs + (size_t)3 * M * (t + 1), tmp.x, sizeof(double) * 3 * M);
        memcpy(vs + (size_t)3 * M * (t + 1), tmp.v, sizeof(double) * 3 * M);
    }
    double J = 0.0;
    for (int i = 0; i < M; ++i) J += tmp.x[3 * i] - R->x0[3 * i];
    J = g * J / M;

    double *lx = (double *)calloc(3 * M, sizeof(double));
    double *lv = (double *)calloc(3 * M, sizeof(double));
    double *lF = (double *)malloc(sizeof(double) * 3 * M);
    double *acc = (double *)calloc(7 * (size_t)S, sizeof(double)); /* gk ga gphi gkz gzr gzi gcd */
    /* terminal condition: dJ/dx_N = g/M e_x, dJ/dv_N = 0 */
    for (int i = 0; i < M; ++i) lx[3 * i] = g / M;

    for (int t = n_steps - 1; t >= 0; --t) {
        const double *x = xs + (size_t)3 * M * t, *v = vs + (size_t)3 * M * t;
        int64_t step = R->step + t;
        forces(R, x, v, step, F);
        for (int i = 0; i < M; ++i) {
            double lvt[3], vp[3];
            /* x_{n+1} = x_n + dt v_{n+1}: v_{n+1} collects dt * lambda_x */
            for (int q = 0; q < 3; ++q) lvt[q] = lv[3 * i + q] + dt * lx[3 * i + q];
            /* v_{n+1} = damping * v'' */
            for (int q = 0; q < 3; ++q) lvt[q] *= p->damping;
            /* friction v'' = P(v', N) with the normal force N of the step */
            for (int q = 0; q < 3; ++q) vp[q] = v[3 * i + q] + dt * F[3 * i + q] / m;
            double z = x[3 * i + 2];
            double N = ground ? ground_normal(R, z, v[3 * i + 2]) : 0.0;
            double lN = 0.0; /* dJ/dN */
            if (N > 0.0) {
                double dv = p->mu * N * dt / m;
                double dvs = p->mu_static * N * dt / m;
                double u = sqrt(vp[0] * vp[0] + vp[1] * vp[1]);
                if (u <= dv || u <= dvs) {
                    lvt[0] = 0.0;
                    lvt[1] = 0.0;
                } else {
                    double uh[2] = {vp[0] / u, vp[1] / u};
                    double dot = uh[0] * lvt[0] + uh[1] * lvt[1];
                    /* dP/d(dv) = -uh and d(dv)/dN = mu dt / m */
                    lN += -(p->mu * dt / m) * dot;
                    double c = dv / u;
                    double l0 = lvt[0] - c * (lvt[0] - uh[0] * dot);
                    double l1 = lvt[1] - c * (lvt[1] - uh[1] * dot);
                    lvt[0] = l0;
                    lvt[1] = l1;
                }
            }
            /* v' = v_n + dt F / m */
            for (int q = 0; q < 3; ++q) {
                lv[3 * i + q] = lvt[q];
                lF[3 * i + q] = dt / m * lvt[q];
            }
            /* the normal force enters F_z; where it is not clamped,
             * dN/dz = -k_ground and dN/dv_z = -c_g */
            if (N > 0.0) {
                lN += lF[3 * i + 2];
                lx[3 * i + 2] += -p->k_ground * lN;
                lv[3 * i + 2] += -cg * lN;
            }
        }
        /* springs */
        double wt = 2.0 * OR_PI * p->act_freq * (double)step * dt;
        double Sw = act ? sin(wt) : 0.0, Cw = act ? cos(wt) : 0.0;
        for (int s = 0; s < S; ++s) {
            int i = R->ij[2 * s], j = R->ij[2 * s + 1];
            double d[3] = {x[3 * j] - x[3 * i], x[3 * j + 1] - x[3 * i + 1], x[3 * j + 2] - x[3 * i + 2]};
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            if (r < 1e-9) continue;
            double dh[3] = {d[0] / r, d[1] / r, d[2] / r};
            double sn = act ? sin(wt + R->phi[s]) : 0.0;
            double cs = act ? cos(wt + R->phi[s]) : 0.0;
            double L = act ? R->L0[s] * (1.0 + R->a[s] * sn) : R->L0[s];
            double u[3], du = 0.0;
            for (int q = 0; q < 3; ++q) { u[q] = lF[3 * j + q] - lF[3 * i + q]; du += dh[q] * u[q]; }
            /* K u with K = k [(1 - L/r)(I - dh dh^T) + dh dh^T] */
            for (int q = 0; q < 3; ++q) {
                double Ku = R->k[s] * ((1.0 - L / r) * (u[q] - dh[q] * du) + dh[q] * du);
                lx[3 * i + q] += Ku;
                lx[3 * j + q] -= Ku;
            }
            /* dashpot c (v_j - v_i).d^ along d^: its force on i is c w d^ with the
             * rate w = (v_j - v_i).d^, so with D = (c / r) [(dv - w d^) du + w (u - du d^)]
             * node i takes D and node j -D in lambda_x, and c du d^ and -c du d^ in
             * lambda_v; dJ/dc = -w du */
            double wr = 0.0, dvv[3];
            for (int q = 0; q < 3; ++q) {
                dvv[q] = v[3 * j + q] - v[3 * i + q];
                wr += dvv[q] * dh[q];
            }
            if (R->cd[s] != 0.0) {
                for (int q = 0; q < 3; ++q) {
                    double D = R->cd[s] / r * ((dvv[q] - wr * dh[q]) * du + wr * (u[q] - du * dh[q]));
                    lx[3 * i + q] += D;
                    lx[3 * j + q] -= D;
                    lv[3 * i + q] += R->cd[s] * du * dh[q];
                    lv[3 * j + q] -= R->cd[s] * du * dh[q];
                }
            }
            double *A = acc + 7 * (size_t)s;
            A[0] += -(r - L) * du;
            A[3] += -(r - R->L0[s]) * du;
            A[6] += -wr * du;
            if (act) {
                double gL = R->k[s] * du;
                A[1] += gL * R->L0[s] * sn;
                A[2] += gL * R->L0[s] * R->a[s] * cs;
                A[4] += R->L0[s] * Sw * du;
                A[5] += R->L0[s] * Cw * du;
            }
        }
    }
    double *out[7] = {gk, ga, gphi, gkz, gzr, gzi, gcd};
    for (int q = 0; q < 7; ++q)
        if (out[q])
            for (int s = 0; s < S; ++s) out[q][s] = acc[7 * (size_t)s + q];
    free(acc);
    free(xs); free(vs); free(F); free(tmp.x); free(tmp.v); free(lx); free(lv); free(lF);
    return J;
}

double or_robot_backward(const or_robot *R, int n_steps, double g, double *gk, double *ga, double *gphi)
{
    return backward_impl(R, n_steps, g, gk, ga, gphi, NULL, NULL, NULL, NULL);
}

double or_robot_backward_z(const or_robot *R, int n_steps, double g, double *gkz, double *gzr, double *gzi,
                           double *gcd)
{
    return backward_impl(R, n_steps, g, NULL, NULL, NULL, gkz, gzr, gzi, gcd);
}

/* dJ/dc per spring dashpot coefficient (with the (k, a, phi) gradients), for
 * the finite-difference pin of the dashpot terms. */
double or_robot_backward_c(const or_robot *R, int n_steps, double g, double *gcd)
{
    return backward_impl(R, n_steps, g, NULL, NULL, NULL, NULL, NULL, NULL, gcd);
}

/* The dashpot coefficients of every spring (in and out), for the same pin. */
void or_robot_dashpots(or_robot *R, double *cd_out, const double *cd_in)
{
    if (cd_out) memcpy(cd_out, R->cd, sizeof(double) * R->S);
    if (cd_in) memcpy(R->cd, cd_in, sizeof(double) * R->S);
}

/* dJ/dw for every voxel from the per-spring gradients dJ/d(k, Zr, Zi, c)
 * through the sum rule: voxel v adds k_c w to k_s, k_c w amp_v e^{i ph_v} to Z_s
 * and zeta sqrt(2 m k_c w) to the dashpot c_s of each of its springs, so
 *   dJ/dw_v = sum_{s of v} k_c dJ/dk_s + dRe(.)/dw dJ/dZr_s + dIm(.)/dw dJ/dZi_s
 *             + zeta sqrt(2 m k_c w) / (2 w) dJ/dc_s
 * with, for the base model (amp, ph fixed per class),
 *   d(k_c w a_c e^{i phi_c})/dw = k_c a_c e^{i phi_c},
 * and for the Table II model (amp = w a_c, ph = w phi_c),
 *   d(k_c a_c w^2 e^{i w phi_c})/dw = k_c a_c (2 w + i w^2 phi_c) e^{i w phi_c}.
 * gcd may be NULL when the spring dashpots are off. */
int or_robot_dJdw(const or_robot *R, const double *gkz, const double *gzr, const double *gzi, const double *gcd,
                  double *dJdw)
{
    if (R->p.zeta_spring != 0.0 && !gcd) return -1;
    int nv = R->n * R->n * R->n;
    for (int v = 0; v < nv; ++v) dJdw[v] = 0.0;
    for (int s = 0; s < R->S; ++s) {
        for (int q = R->sv_ptr[s]; q < R->sv_ptr[s + 1]; ++q) {
            int v = R->sv[q];
            int c = R->kept[v];
            double kc = R->p.k_class[c], ac = R->p.a_class[c], pc = R->p.phi_class[c], w = R->w[v];
            double dzr, dzi;
            if (R->p.flags & OR_WEIGHT_ACTUATION) {
                dzr = kc * ac * (2.0 * w * cos(w * pc) - w * w * pc * sin(w * pc));
                dzi = kc * ac * (2.0 * w * sin(w * pc) + w * w * pc * cos(w * pc));
            } else {
                dzr = kc * ac * cos(pc);
                dzi = kc * ac * sin(pc);
            }
            dJdw[v] += kc * gkz[s] + dzr * gzr[s] + dzi * gzi[s];
            if (R->p.zeta_spring != 0.0 && w > 0.0)
                dJdw[v] += R->p.zeta_spring * sqrt(2.0 * R->p.mass * kc * w) / (2.0 * w) * gcd[s];
        }
    }
    return 0;
}

/* Genome gradient from dJ/dw per voxel: w = sigmoid(o5), then back through
 * the MLP.  Categories (argmax), the kept component and the topology carry
 * no gradient. */
int or_mlp_backward(const double *genome, const double *B, int n, const double *dJdw, double *g_gen)
{
    for (int q = 0; q < OR_GENOME_LEN; ++q) g_gen[q] = 0.0;
    const double *W2 = genome + OR_OFF_W2, *W3 = genome + OR_OFF_W3;
    double v[3], g[2 * OR_PE_M], h1[OR_HID], h2[OR_HID], o[OR_NOUT], d1[OR_HID], d2[OR_HID];
    for (int vid = 0; vid < n * n * n; ++vid) {
        if (dJdw[vid] == 0.0) continue;
        voxel_centre(n, vid, v);
        or_encode(B, v, g);
        or_mlp(genome, g, h1, h2, o);
        double w = 1.0 / (1.0 + exp(-o[5]));
        double g5 = dJdw[vid] * w * (1.0 - w);
        for (int j = 0; j < OR_HID; ++j) g_gen[OR_OFF_W3 + 5 * OR_HID + j] += g5 * h2[j];
        g_gen[OR_OFF_B3 + 5] += g5;
        for (int j = 0; j < OR_HID; ++j) d2[j] = g5 * W3[5 * OR_HID + j] * (1.0 - h2[j] * h2[j]);
        for (int i = 0; i < OR_HID; ++i) {
            for (int j = 0; j < OR_HID; ++j) g_gen[OR_OFF_W2 + i * OR_HID + j] += d2[i] * h1[j];
            g_gen[OR_OFF_B2 + i] += d2[i];
        }
        for (int j = 0; j < OR_HID; ++j) {
            double s = 0.0;
            for (int i = 0; i < OR_HID; ++i) s += W2[i * OR_HID + j] * d2[i];
            d1[j] = s * (1.0 - h1[j] * h1[j]);
        }
        for (int i = 0; i < OR_HID; ++i) {
            for (int j = 0; j < 2 * OR_PE_M; ++j) g_gen[OR_OFF_W1 + i * 2 * OR_PE_M + j] += d1[i] * g[j];
            g_gen[OR_OFF_B1 + i] += d1[i];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Counter-based RNG: Philox-4x64-10                                         */
/* ------------------------------------------------------------------------ */

/* Philox-4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11): each round multiplies words 0 and 2
 * by the two round multipliers, swaps the halves and xors in the key, which
 * is bumped by the two Weyl constants between rounds. */
void or_philox4x64_10(const uint64_t *ctr, const uint64_t *key, uint64_t *out)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        unsigned __int128 p0 = (unsigned __int128)M0 * x0;
        unsigned __int128 p1 = (unsigned __int128)M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------ */
/* GA generation                                                             */
/* ------------------------------------------------------------------------ */

/* a is better than b: larger fitness, NaN counted as -inf, ties to the lower index */
static int better(const double *fit, int a, int b)
{
    double fa = isnan(fit[a]) ? -INFINITY : fit[a];
    double fb = isnan(fit[b]) ? -INFINITY : fit[b];
    if (fa != fb) return fa > fb;
    return a < b;
}

static uint64_t draw(uint64_t seed, uint64_t gen, uint64_t child, uint64_t purpose, uint64_t block, int word)
{
    uint64_t ctr[4] = {gen, child, purpose, block}, key[2] = {seed, 0}, out[4];
    or_philox4x64_10(ctr, key, out);
    return out[word];
}

static int tournament(const double *fit, int P, int k, uint64_t seed, uint64_t gen, uint64_t child, uint64_t purpose)
{
    int win = -1;
    for (int t = 0; t < k; ++t) {
        uint64_t r = draw(seed, gen, child, purpose, (uint64_t)(t / 4), t % 4);
        int idx = (int)(((r >> 32) * (uint64_t)P) >> 32);
        if (win < 0 || better(fit, idx, win)) win = idx;
    }
    return win;
}

/* One generation (Sec. II-C, Table I): the best floor(elite_frac * P)
 * individuals are copied unchanged in rank order; every other slot gets a
 * child of two tournament winners (k draws with replacement each), uniform
 * crossover with probability p_cross, then per-gene Gaussian mutation with
 * probability p_mut.  Probabilities arrive as 64-bit thresholds
 * floor(p * 2^64); a draw r passes when r < threshold.  decisions[3c..3c+2] =
 * (parent A, parent B, kind) with kind 0 elite, 1 copy of A, 2 crossover. */
int or_ga_generation(const double *fit, const double *gin, double *gout, int P, int L,
                     double elite_frac, int k, uint64_t p_cross_thr, uint64_t p_mut_thr, double sigma,
                     uint64_t seed, uint64_t gen, int32_t *decisions)
{
    if (P < 1 || L < 1 || k < 1) return -1;
    int E = (int)floor(elite_frac * (double)P);
    if (E > P) E = P;
    if (E < 0) E = 0;
    /* rank by selection sort on the better() order */
    int *order = (int *)malloc(sizeof(int) * P);
    char *used = (char *)calloc(P, 1);
    for (int r = 0; r < P; ++r) {
        int best = -1;
        for (int i = 0; i < P; ++i)
            if (!used[i] && (best < 0 || better(fit, i, best))) best = i;
        used[best] = 1;
        order[r] = best;
    }
    for (int c = 0; c < E; ++c) {
        memcpy(gout + (size_t)c * L, gin + (size_t)order[c] * L, sizeof(double) * L);
        if (decisions) { decisions[3 * c] = order[c]; decisions[3 * c + 1] = order[c]; decisions[3 * c + 2] = 0; }
    }
    for (int c = E; c < P; ++c) {
        int A = tournament(fit, P, k, seed, gen, c, 0);
        int B = tournament(fit, P, k, seed, gen, c, 1);
        int cx = draw(seed, gen, c, 2, 0, 0) < p_cross_thr;
        if (decisions) { decisions[3 * c] = A; decisions[3 * c + 1] = B; decisions[3 * c + 2] = cx ? 2 : 1; }
        for (int q = 0; q < L; ++q) {
            int src = A;
            if (cx) {
                uint64_t bits = draw(seed, gen, c, 3, (uint64_t)(q / 256), (q % 256) / 64);
                if ((bits >> (q % 64)) & 1) src = B;
            }
            double val = gin[(size_t)src * L + q];
            if (draw(seed, gen, c, 4, (uint64_t)(q / 4), q % 4) < p_mut_thr) {
                uint64_t w0 = draw(seed, gen, c, 5, (uint64_t)(q / 2), 2 * (q % 2));
                uint64_t w1 = draw(seed, gen, c, 5, (uint64_t)(q / 2), 2 * (q % 2) + 1);
                double u1 = ((double)(w0 >> 11) + 1.0) * 0x1.0p-53; /* (0, 1] */
                double u2 = (double)(w1 >> 11) * 0x1.0p-53;         /* [0, 1) */
                double z = sqrt(-2.0 * log(u1)) * cos(2.0 * OR_PI * u2); /* Box-Muller */
                val += sigma * z;
            }
            gout[(size_t)c * L + q] = val;
        }
    }
    free(order);
    free(used);
    return 0;
}

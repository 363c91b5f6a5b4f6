// runtime.hip -- population handle, memory plan and the C ABI of softrobot.h.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

using namespace sr;

namespace {
thread_local std::string g_err;

int set_err(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}
}  // namespace

// Step time table of pop_step_noalloc: (sin, cos)(w t_n) for up to
// SR_NOALLOC_MAX_STEPS steps (512 KiB), one copy per device for the life of
// the process.  Host code never passes this name to a kernel: it uses the
// device address that hipGetSymbolAddress returns on each device.
static __device__ __align__(256) float2 scratch[SR_NOALLOC_MAX_STEPS];

namespace {
constexpr int kMaxDevices = 64;
constexpr int NSET = 3;  // segment buffer sets of the adjoint pipeline
std::mutex g_scratch_mu;
float2 *g_scratch[kMaxDevices] = {};

// Resolves (once per device, with that device current) and returns the
// device address of `scratch` on `dev`.
int noalloc_table(int dev, float2 **out) {
    if (dev < 0 || dev >= kMaxDevices) return set_err(SR_EUNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
        void *p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess) return set_err(SR_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch[dev] = static_cast<float2 *>(p);
    }
    *out = g_scratch[dev];
    return SR_OK;
}
}  // namespace

struct SideGroup {
    int n, offset, count;
    PersistCfg cfg;
};

struct GraphKey {
    int n_steps, mode, cur, spl;
    bool operator<(const GraphKey &o) const {
        if (n_steps != o.n_steps) return n_steps < o.n_steps;
        if (mode != o.mode) return mode < o.mode;
        if (cur != o.cur) return cur < o.cur;
        return spl < o.spl;
    }
};

struct sr_pop {
    sr_sim_params p;
    SimConst c;
    hipStream_t st = nullptr;
    int device = 0;  // the device that was current at pop_create
    int R = 0, max_side = 0;
    std::vector<RobotInfo> h_robots;
    RobotInfo *d_robots = nullptr;
    int total_slots = 0, total_vox = 0;
    uint8_t *kept = nullptr;
    float *w = nullptr;
    Planes pl{};
    int32_t *sid = nullptr;
    float4 *x0 = nullptr, *xbuf[2] = {nullptr, nullptr}, *vbuf[2] = {nullptr, nullptr};
    int cur = 0;
    int32_t *slot_node = nullptr, *node_slot = nullptr, *slot_robot = nullptr;
    NodeRow *rows = nullptr;
    Entry *entries = nullptr;
    uint8_t *bad_class = nullptr, *diverged = nullptr;
    int64_t *d_step = nullptr;
    int64_t h_step = 0, h_step_stage = 0;
    float2 *sc = nullptr;
    int sc_cap = 0;
    int32_t *d_lists = nullptr;
    std::vector<SideGroup> groups;
    // persistent-step schedule: size groups in launch order, each on a lane
    // (0: the population's stream, k > 0: side[k - 1])
    std::vector<int> order, lane;
    int64_t *d_mass_off = nullptr, *d_spring_off = nullptr;
    std::vector<int64_t> h_mass_off, h_spring_off;
    bool counts_valid = false;
    bool built = false;
    bool phase = false;
    bool dash = false;  // spring dashpots: only the +16 persistent kernels
    bool vox_ok = false;  // the per-voxel terms match the spring planes (no pop_set_spring_params since the build)
    int mode = SR_STEP_AUTO, spl = 0;
    int sticky = 0;
    // genome query scratch
    uint8_t *q_cls = nullptr;
    float *q_w = nullptr;
    int32_t *vox_robot = nullptr;
    // adjoint: checkpoints of (x, v) at steps 0, K, 2K, ... since the build
    int ck_every = 0, ck_cap = 0;
    bool rec_valid = false;
    float4 *ck_x = nullptr, *ck_v = nullptr;
    // adjoint scratch (grown on demand)
    // (two sets of segment buffers: segment s - 1 is recomputed on adj_st while
    // segment s is reversed on the population's stream)
    int rec_cap = 0;
    // three sets: while segment s is reversed, segment s - 1 is recomputed and
    // (split form) the gradient passes of segment s + 1 still read theirs
    float4 *rec_x[NSET] = {}, *rec_v[NSET] = {};
    float4 *rec_u[NSET] = {};  // v_n per step (dashpots or a damped ground)
    float4 *rec_l[NSET] = {};  // lambda_F per step (split adjoint of the largest sides)
    float4 *tmp_x[NSET] = {}, *tmp_v[NSET] = {};
    float4 *lx = nullptr, *lv = nullptr;
    float *gk = nullptr, *gs = nullptr, *gc = nullptr, *gd = nullptr, *dJdw = nullptr;
    float2 *sc_seg[NSET] = {};
    hipStream_t adj_st = nullptr, adj_gst = nullptr;  // recomputation; gradient passes (split form)
    // start, recorded[NSET], reversed[NSET], gradient sums formed[NSET]
    hipEvent_t adj_ev[1 + 3 * NSET] = {};
    // captured step graphs: one per (n_steps, mode, current buffer, steps per launch)
    bool use_graphs = true;
    hipStream_t cap = nullptr;
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> ev;
    std::map<GraphKey, hipGraphExec_t> graphs;
};

namespace {

int fail_hip(sr_pop *pop, hipError_t e, const char *what) {
    if (pop) pop->sticky = SR_EHIP;
    return set_err(SR_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIPC(pop, x)                                         \
    do {                                                     \
        hipError_t e_ = (x);                                 \
        if (e_ != hipSuccess) return fail_hip(pop, e_, #x);  \
    } while (0)

#define CHECK_POP(pop)                                                                    \
    do {                                                                                  \
        if (!(pop)) return set_err(SR_EINVAL, "null population handle");                  \
        if ((pop)->sticky) return set_err((pop)->sticky, "population is in an error state"); \
    } while (0)

template <class T>
hipError_t dalloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc(reinterpret_cast<void **>(p), sizeof(T) * count);
}

void clear_graphs(sr_pop *pop) {
    for (auto &kv : pop->graphs) (void)hipGraphExecDestroy(kv.second);
    pop->graphs.clear();
}

void pop_free(sr_pop *pop) {
    clear_graphs(pop);
    for (auto s : pop->side) (void)hipStreamDestroy(s);
    for (auto e : pop->ev) (void)hipEventDestroy(e);
    if (pop->cap) (void)hipStreamDestroy(pop->cap);
    void *ptrs[] = {pop->d_robots, pop->kept, pop->w, pop->pl.k, pop->pl.kL0, pop->pl.kal, pop->pl.kbe, pop->pl.kd, pop->pl.vkp,
                    pop->sid, pop->x0, pop->xbuf[0], pop->xbuf[1], pop->vbuf[0], pop->vbuf[1],
                    pop->slot_node, pop->node_slot, pop->slot_robot, pop->rows, pop->entries,
                    pop->bad_class, pop->diverged, pop->d_step, pop->sc, pop->d_lists, pop->d_mass_off,
                    pop->d_spring_off, pop->q_cls, pop->q_w, pop->vox_robot, pop->ck_x, pop->ck_v,
                    pop->lx, pop->lv, pop->gk, pop->gs, pop->gc, pop->gd, pop->dJdw};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (int b = 0; b < NSET; ++b) {
        void *seg[] = {pop->rec_x[b], pop->rec_v[b], pop->rec_u[b], pop->rec_l[b], pop->tmp_x[b], pop->tmp_v[b],
                       pop->sc_seg[b]};
        for (void *p : seg)
            if (p) (void)hipFree(p);
    }
    for (auto e : pop->adj_ev)
        if (e) (void)hipEventDestroy(e);
    if (pop->adj_st) (void)hipStreamDestroy(pop->adj_st);
    if (pop->adj_gst) (void)hipStreamDestroy(pop->adj_gst);
}

int ensure_counts(sr_pop *pop) {
    if (pop->counts_valid) return SR_OK;
    HIPC(pop, hipMemcpyAsync(pop->h_robots.data(), pop->d_robots, sizeof(RobotInfo) * pop->R, hipMemcpyDeviceToHost,
                             pop->st));
    HIPC(pop, hipStreamSynchronize(pop->st));
    pop->h_mass_off.assign(pop->R + 1, 0);
    pop->h_spring_off.assign(pop->R + 1, 0);
    for (int r = 0; r < pop->R; ++r) {
        pop->h_mass_off[r + 1] = pop->h_mass_off[r] + pop->h_robots[r].M;
        pop->h_spring_off[r + 1] = pop->h_spring_off[r] + pop->h_robots[r].S;
    }
    HIPC(pop, hipMemcpyAsync(pop->d_mass_off, pop->h_mass_off.data(), sizeof(int64_t) * (pop->R + 1),
                             hipMemcpyHostToDevice, pop->st));
    HIPC(pop, hipMemcpyAsync(pop->d_spring_off, pop->h_spring_off.data(), sizeof(int64_t) * (pop->R + 1),
                             hipMemcpyHostToDevice, pop->st));
    HIPC(pop, hipStreamSynchronize(pop->st));
    pop->counts_valid = true;
    return SR_OK;
}

int ensure_sc(sr_pop *pop, int n) {
    if (n <= pop->sc_cap) return SR_OK;
    HIPC(pop, hipStreamSynchronize(pop->st));
    if (pop->sc) HIPC(pop, hipFree(pop->sc));
    pop->sc = nullptr;
    clear_graphs(pop);  // graphs hold the old table address
    int cap = n < 1024 ? 1024 : n;
    HIPC(pop, dalloc(&pop->sc, (size_t)cap));
    pop->sc_cap = cap;
    return SR_OK;
}

// Runs after any build: resets step, buffers and cached counts.
int finish_build(sr_pop *pop) {
    pop->cur = 0;
    HIPC(pop, hipMemcpyAsync(pop->xbuf[1], pop->xbuf[0], sizeof(float4) * pop->total_slots, hipMemcpyDeviceToDevice,
                             pop->st));
    HIPC(pop, hipMemcpyAsync(pop->vbuf[1], pop->vbuf[0], sizeof(float4) * pop->total_slots, hipMemcpyDeviceToDevice,
                             pop->st));
    pop->h_step = 0;
    pop->h_step_stage = 0;
    HIPC(pop, hipMemcpyAsync(pop->d_step, &pop->h_step_stage, sizeof(int64_t), hipMemcpyHostToDevice, pop->st));
    pop->rec_valid = pop->ck_every > 0;
    std::vector<uint8_t> bad(pop->R);
    HIPC(pop, hipMemcpyAsync(bad.data(), pop->bad_class, pop->R, hipMemcpyDeviceToHost, pop->st));
    HIPC(pop, hipStreamSynchronize(pop->st));
    pop->counts_valid = false;
    for (int r = 0; r < pop->R; ++r)
        if (bad[r]) {
            pop->built = false;
            HIPC(pop, hipMemsetAsync(pop->bad_class, 0, pop->R, pop->st));
            return set_err(SR_EINVAL, "robot %d has a voxel class outside 0..4", r);
        }
    pop->built = true;
    pop->vox_ok = true;
    return SR_OK;
}

}  // namespace

extern "C" {

const char *sr_last_error(void) { return g_err.c_str(); }

int sr_version(void) { return 1; }

int sr_microbench(int32_t which, int32_t iters, double *seconds, double *units) {
    if (which < 0 || which > 5 || iters < 1 || !seconds || !units) return set_err(SR_EINVAL, "bad microbenchmark request");
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int grid = (cus > 0 ? cus : 256) * 8;
    const size_t hbm_n = (size_t)32 << 20;  // 32 Mi float4 = 512 MiB per buffer
    float *out = nullptr;
    float4 *src = nullptr, *dst = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipMalloc(&out, sizeof(float) * grid * 256);
    if (e == hipSuccess && which == 5) e = hipMalloc(&src, sizeof(float4) * hbm_n);
    if (e == hipSuccess && which == 5) e = hipMalloc(&dst, sizeof(float4) * hbm_n);
    if (e == hipSuccess && which == 5) e = hipMemset(src, 0, sizeof(float4) * hbm_n);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    double u = 0.0;
    auto run = [&]() {
        return which == 5 ? launch_micro_hbm(src, dst, hbm_n, grid * 4, iters, st, &u)
                          : launch_micro(which, iters, grid, out, st, &u);
    };
    if (e == hipSuccess) e = run();  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    if (e == hipSuccess) e = run();
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    if (out) (void)hipFree(out);
    if (src) (void)hipFree(src);
    if (dst) (void)hipFree(dst);
    if (e != hipSuccess) return set_err(SR_EHIP, "microbenchmark: %s", hipGetErrorString(e));
    *seconds = ms * 1e-3;
    *units = u;
    return SR_OK;
}

int sr_persist_configs(int32_t n, int32_t *blocks, int32_t *variants, int32_t cap) {
    if (n < 1 || n > SR_MAX_SIDE) return set_err(SR_EINVAL, "side %d outside 1..%d", n, SR_MAX_SIDE);
    return persist_list(n, blocks, variants, cap < 0 ? 0 : cap);
}

int sr_default_params(sr_sim_params *out) {
    if (!out) return set_err(SR_EINVAL, "null output");
    memset(out, 0, sizeof *out);
    out->dt = 1e-4;
    out->gravity = 9.81f;
    out->damping = 0.999f;
    out->mass = 0.1f;
    out->voxel_len = 0.1f;
    out->k_ground = 1e5f;
    out->mu = 0.5f;
    out->act_freq = 4.0f;
    const float kc[5] = {0.f, 1e4f, 1e4f, 3e3f, 3e4f};
    const float ac[5] = {0.f, 0.2f, -0.2f, 0.f, 0.f};
    for (int c = 0; c < 5; ++c) {
        out->k_class[c] = kc[c];
        out->a_class[c] = ac[c];
        out->phi_class[c] = 0.f;
    }
    out->flags = 0;
    return SR_OK;
}

int sr_table2_params(sr_sim_params *out) {
    if (!out) return set_err(SR_EINVAL, "null output");
    sr_default_params(out);
    out->dt = 1e-5;
    out->damping = 1.0f;
    out->mu = 1.0f;
    out->mu_static = 0.6f;
    out->zeta_spring = 0.1f;
    out->zeta_ground = 0.1f;
    const float kc[5] = {0.f, 2e3f, 2e3f, 1e3f, 1e4f};
    const float ac[5] = {0.f, 0.25f, -0.25f, 0.f, 0.f};
    const float pc[5] = {0.f, (float)M_PI, (float)M_PI, 0.f, 0.f};
    for (int c = 0; c < 5; ++c) {
        out->k_class[c] = kc[c];
        out->a_class[c] = ac[c];
        out->phi_class[c] = pc[c];
    }
    out->flags = SR_WEIGHT_ACTUATION;
    return SR_OK;
}

int pop_create(const sr_sim_params *params, int32_t n_robots, const int32_t *grid_side, void *stream, sr_pop **out) {
    if (!params || !grid_side || !out) return set_err(SR_EINVAL, "null argument");
    *out = nullptr;
    if (n_robots < 1) return set_err(SR_EINVAL, "n_robots must be >= 1 (got %d)", n_robots);
    if (!(params->dt > 0) || !(params->mass > 0) || !(params->voxel_len > 0))
        return set_err(SR_EINVAL, "dt, mass and voxel_len must be positive");
    if (!(params->mu_static >= 0) || !(params->zeta_spring >= 0) || !(params->zeta_ground >= 0))
        return set_err(SR_EINVAL, "mu_static, zeta_spring and zeta_ground must be >= 0");
    for (int r = 0; r < n_robots; ++r)
        if (grid_side[r] < 1 || grid_side[r] > SR_MAX_SIDE)
            return set_err(SR_EINVAL, "grid_side[%d] = %d outside 1..%d", r, grid_side[r], SR_MAX_SIDE);
    int dev = 0;
    hipError_t de = hipGetDevice(&dev);
    if (de != hipSuccess) return set_err(SR_EHIP, "hipGetDevice: %s", hipGetErrorString(de));
    float2 *table = nullptr;
    int trc = noalloc_table(dev, &table);  // resolve the no-allocation step table on this device
    if (trc) return trc;
    sr_pop *pop = new sr_pop();
    pop->device = dev;
    pop->p = *params;
    pop->c = make_sim_const(*params);
    pop->st = reinterpret_cast<hipStream_t>(stream);
    pop->R = n_robots;
    pop->h_robots.resize(n_robots);
    int64_t slots = 0, vox = 0;
    std::map<int, std::vector<int>> by_side;
    for (int r = 0; r < n_robots; ++r) {
        RobotInfo &ri = pop->h_robots[r];
        ri.n = grid_side[r];
        ri.N = ri.n + 1;
        ri.slots = ri.N * ri.N * ri.N;
        ri.slot_base = (int32_t)slots;
        ri.vox_base = (int32_t)vox;
        ri.M = 0;
        ri.S = 0;
        ri.pad = 0;
        slots += ri.slots;
        vox += (int64_t)ri.n * ri.n * ri.n;
        by_side[ri.n].push_back(r);
        if (ri.n > pop->max_side) pop->max_side = ri.n;
    }
    if (slots * 2 * NDIR >= INT32_MAX) {
        delete pop;
        return set_err(SR_EINVAL, "population too large for 32-bit slot indexing");
    }
    for (int c = 0; c < 5; ++c)
        if (params->phi_class[c] != 0.f) pop->phase = true;
    pop->dash = params->zeta_spring != 0.f;
    pop->total_slots = (int)slots;
    pop->total_vox = (int)vox;
    const size_t S = slots, P = slots * NDIR;
    hipError_t e = hipSuccess;
#define ALLOC(ptr, cnt) \
    if (e == hipSuccess) e = dalloc(&(ptr), (cnt))
    ALLOC(pop->d_robots, (size_t)n_robots);
    ALLOC(pop->kept, (size_t)vox);
    ALLOC(pop->w, (size_t)vox);
    ALLOC(pop->pl.k, P);
    ALLOC(pop->pl.kL0, P);
    ALLOC(pop->pl.kal, P);
    ALLOC(pop->pl.kbe, P);
    ALLOC(pop->pl.kd, P);
    ALLOC(pop->pl.vkp, S);
    ALLOC(pop->sid, P);
    ALLOC(pop->x0, S);
    ALLOC(pop->xbuf[0], S);
    ALLOC(pop->xbuf[1], S);
    ALLOC(pop->vbuf[0], S);
    ALLOC(pop->vbuf[1], S);
    ALLOC(pop->slot_node, S);
    ALLOC(pop->node_slot, S);
    ALLOC(pop->slot_robot, S);
    ALLOC(pop->rows, S);
    ALLOC(pop->entries, 2 * P);
    ALLOC(pop->bad_class, (size_t)n_robots);
    ALLOC(pop->diverged, (size_t)n_robots);
    ALLOC(pop->d_step, 1);
    ALLOC(pop->d_lists, (size_t)n_robots);
    ALLOC(pop->d_mass_off, (size_t)n_robots + 1);
    ALLOC(pop->d_spring_off, (size_t)n_robots + 1);
    ALLOC(pop->q_cls, (size_t)vox);
    ALLOC(pop->q_w, (size_t)vox);
    ALLOC(pop->vox_robot, (size_t)vox);
#undef ALLOC
    if (e != hipSuccess) {
        pop_free(pop);
        delete pop;
        return set_err(e == hipErrorOutOfMemory ? SR_ENOMEM : SR_EHIP, "allocation failed: %s", hipGetErrorString(e));
    }
    std::vector<int32_t> slot_robot(S);
    for (int r = 0; r < n_robots; ++r)
        for (int s = 0; s < pop->h_robots[r].slots; ++s) slot_robot[pop->h_robots[r].slot_base + s] = r;
    std::vector<int32_t> vox_robot((size_t)vox);
    for (int r = 0; r < n_robots; ++r)
        for (int q = 0; q < pop->h_robots[r].n * pop->h_robots[r].n * pop->h_robots[r].n; ++q)
            vox_robot[pop->h_robots[r].vox_base + q] = r;
    std::vector<int32_t> lists;
    for (auto &kv : by_side) {
        SideGroup g;
        g.n = kv.first;
        g.offset = (int)lists.size();
        g.count = (int)kv.second.size();
        g.cfg.n = kv.first;
        g.cfg.block = persist_default_block(kv.first, pop->dash, true, &g.cfg.variant);
        lists.insert(lists.end(), kv.second.begin(), kv.second.end());
        pop->groups.push_back(g);
    }
    // default schedule: largest side first, each group on a lane of its own
    {
        const int G = (int)pop->groups.size();
        pop->lane.assign(G, 0);
        for (int q = 0; q < G; ++q) {
            pop->order.push_back(G - 1 - q);
            pop->lane[G - 1 - q] = q;
        }
    }
    int rc = SR_OK;
    // private streams (default priority) for capturing step graphs: one per
    // extra size group, so the groups become parallel branches of one graph
    e = hipStreamCreateWithFlags(&pop->cap, hipStreamNonBlocking);
    for (size_t g = 0; g + 1 < pop->groups.size() && e == hipSuccess; ++g) {
        hipStream_t s2;
        e = hipStreamCreateWithFlags(&s2, hipStreamNonBlocking);
        if (e == hipSuccess) pop->side.push_back(s2);
    }
    for (size_t g = 0; g < 2 * pop->groups.size() && e == hipSuccess; ++g) {
        hipEvent_t ev;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) pop->ev.push_back(ev);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(pop->d_robots, pop->h_robots.data(), sizeof(RobotInfo) * n_robots, hipMemcpyHostToDevice,
                           pop->st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(pop->slot_robot, slot_robot.data(), sizeof(int32_t) * S, hipMemcpyHostToDevice, pop->st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(pop->vox_robot, vox_robot.data(), sizeof(int32_t) * vox, hipMemcpyHostToDevice, pop->st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(pop->d_lists, lists.data(), sizeof(int32_t) * n_robots, hipMemcpyHostToDevice, pop->st);
    if (e == hipSuccess) e = hipMemsetAsync(pop->bad_class, 0, n_robots, pop->st);
    if (e == hipSuccess) e = hipMemsetAsync(pop->diverged, 0, n_robots, pop->st);
    if (e == hipSuccess) e = hipStreamSynchronize(pop->st);
    if (e != hipSuccess) rc = set_err(SR_EHIP, "create: %s", hipGetErrorString(e));
    if (rc != SR_OK) {
        pop_free(pop);
        delete pop;
        return rc;
    }
    *out = pop;
    return SR_OK;
}

int pop_destroy(sr_pop *pop) {
    if (!pop) return SR_OK;
    (void)hipStreamSynchronize(pop->st);
    pop_free(pop);
    delete pop;
    return SR_OK;
}

int pop_build_from_voxels(sr_pop *pop, const uint8_t *cls, const float *w) {
    CHECK_POP(pop);
    if (!cls || !w) return set_err(SR_EINVAL, "null voxel array");
    if (cls != pop->q_cls)
        HIPC(pop, hipMemcpyAsync(pop->q_cls, cls, pop->total_vox, hipMemcpyDeviceToDevice, pop->st));
    HIPC(pop, hipMemcpyAsync(pop->w, w, sizeof(float) * pop->total_vox, hipMemcpyDeviceToDevice, pop->st));
    HIPC(pop, launch_build_mesh(pop->d_robots, pop->R, SR_MAX_SIDE, pop->p, cls, pop->w, pop->kept, pop->pl, pop->sid,
                                pop->x0, pop->xbuf[0], pop->vbuf[0], pop->slot_node, pop->node_slot, pop->rows,
                                pop->entries, pop->bad_class, pop->diverged, pop->st));
    return finish_build(pop);
}

int pop_build_from_genomes(sr_pop *pop, const float *genomes, const float *B, int32_t precision) {
    CHECK_POP(pop);
    if (!genomes || !B) return set_err(SR_EINVAL, "null genome or B");
    if (precision != SR_QUERY_FP32 && precision != SR_QUERY_BF16)
        return set_err(SR_EINVAL, "unknown query precision %d", precision);
    HIPC(pop, launch_query(pop->d_robots, pop->R, pop->max_side, genomes, B, precision, pop->q_cls, pop->q_w, pop->st));
    return pop_build_from_voxels(pop, pop->q_cls, pop->q_w);
}

int pop_set_step_config(sr_pop *pop, int32_t mode, int32_t block, int32_t steps_per_launch) {
    CHECK_POP(pop);
    if (mode < SR_STEP_AUTO || mode > SR_STEP_PLAIN) return set_err(SR_EINVAL, "unknown step mode %d", mode);
    pop->mode = mode;
    pop->spl = steps_per_launch > 0 ? steps_per_launch : 0;
    clear_graphs(pop);
    if (block > 0) {
        for (auto &g : pop->groups) {
            bool found = false;
            for (int var : {1, 5, 2, 6, 0, 4}) {
                PersistCfg c{g.n, block, var + (pop->dash ? 16 : 0)};
                if (persist_supported(c, pop->phase)) {
                    g.cfg = c;
                    found = true;
                    break;
                }
            }
            if (!found) return set_err(SR_EUNSUPPORTED, "no persistent kernel for n=%d block=%d", g.n, block);
        }
    }
    return SR_OK;
}

int pop_set_schedule(sr_pop *pop, int32_t n, const int32_t *sides, const int32_t *lanes) {
    CHECK_POP(pop);
    const int G = (int)pop->groups.size();
    if (n != G) return set_err(SR_EINVAL, "schedule of %d sides for a population of %d", n, G);
    if (!sides || !lanes) return set_err(SR_EINVAL, "null schedule");
    std::vector<int> order, lane(G, -1);
    for (int q = 0; q < n; ++q) {
        int g = -1;
        for (int h = 0; h < G; ++h)
            if (pop->groups[h].n == sides[q]) g = h;
        if (g < 0) return set_err(SR_EINVAL, "no robot of side %d", sides[q]);
        if (lane[g] >= 0) return set_err(SR_EINVAL, "side %d listed twice", sides[q]);
        if (lanes[q] < 0 || lanes[q] >= G) return set_err(SR_EINVAL, "lane %d outside 0..%d", lanes[q], G - 1);
        lane[g] = lanes[q];
        order.push_back(g);
    }
    pop->order = order;
    pop->lane = lane;
    clear_graphs(pop);
    return SR_OK;
}

int pop_get_schedule(sr_pop *pop, int32_t *sides, int32_t *lanes) {
    CHECK_POP(pop);
    if (!sides || !lanes) return set_err(SR_EINVAL, "null output");
    for (size_t q = 0; q < pop->order.size(); ++q) {
        sides[q] = pop->groups[pop->order[q]].n;
        lanes[q] = pop->lane[pop->order[q]];
    }
    return SR_OK;
}

int pop_set_persist_variant(sr_pop *pop, int32_t n, int32_t block, int32_t variant) {
    CHECK_POP(pop);
    for (auto &g : pop->groups)
        if (g.n == n) {
            PersistCfg c{n, block, variant};
            if (!persist_supported(c, pop->phase))
                return set_err(SR_EUNSUPPORTED, "no persistent kernel for n=%d block=%d variant=%d", n, block, variant);
            if ((variant & 96) && !pop->vox_ok)
                return set_err(SR_EUNSUPPORTED, "variant %d rebuilds spring parameters from voxels, but they were "
                               "set with pop_set_spring_params", variant);
            if (((variant & 16) != 0) != pop->dash)
                return set_err(SR_EUNSUPPORTED, "variant %d %s spring dashpots; this population has %s", variant,
                               (variant & 16) ? "has" : "lacks", pop->dash ? "them" : "none");
            g.cfg = c;
            clear_graphs(pop);
            return SR_OK;
        }
    return set_err(SR_EINVAL, "no robot of side %d", n);
}

int pop_get_persist_variant(sr_pop *pop, int32_t n, int32_t *block, int32_t *variant) {
    CHECK_POP(pop);
    for (const auto &g : pop->groups)
        if (g.n == n) {
            if (block) *block = g.cfg.block;
            if (variant) *variant = g.cfg.variant;
            return SR_OK;
        }
    return set_err(SR_EINVAL, "no robot of side %d", n);
}

namespace {
// Enqueues n_steps on stream st without checkpoints: the time table, then the
// step kernels (persistent: one launch per size group and block of steps, the
// groups on their own streams so they run side by side; plain: one launch per
// step), then the step counter.  Used eagerly and under graph capture.
int enqueue_steps(sr_pop *pop, int n_steps, float2 *sc, hipStream_t st) {
    const double omega_dt = 2.0 * M_PI * (double)pop->p.act_freq * pop->p.dt;
    HIPC(pop, launch_sincos(sc, pop->d_step, n_steps, omega_dt, pop->c.actuation, st));
    const int spl = pop->spl > 0 ? pop->spl : n_steps;
    if (pop->mode == SR_STEP_PLAIN) {
        for (int t = 0; t < n_steps; ++t) {
            const int a = pop->cur, b = 1 - pop->cur;
            HIPC(pop, launch_plain_step(pop->d_robots, pop->R, pop->total_slots, pop->rows, pop->entries, pop->pl,
                                        pop->xbuf[a], pop->vbuf[a], pop->xbuf[b], pop->vbuf[b], sc, t,
                                        pop->phase, pop->diverged, pop->slot_robot, pop->c, st));
            pop->cur = b;
        }
        HIPC(pop, launch_check_div(pop->d_robots, pop->R, pop->xbuf[pop->cur], pop->vbuf[pop->cur], pop->diverged,
                                   pop->c.lim, st));
    } else {
        // the size groups in the schedule's order, each on its lane's stream;
        // the lanes fork from and join back into st
        const int G = (int)pop->groups.size();
        bool used[SR_MAX_SIDE] = {};  // at most one group per side
        for (int g = 0; g < G; ++g) used[pop->lane[g]] = true;
        if (G > 1) {
            HIPC(pop, hipEventRecord(pop->ev[0], st));
            for (int l = 1; l < G; ++l)
                if (used[l]) HIPC(pop, hipStreamWaitEvent(pop->side[l - 1], pop->ev[0], 0));
        }
        for (int t0 = 0; t0 < n_steps; t0 += spl) {
            const int cnt = (n_steps - t0) < spl ? (n_steps - t0) : spl;
            for (int q = 0; q < G; ++q) {
                const int g = pop->order[q];
                const SideGroup &gr = pop->groups[g];
                hipStream_t sq = pop->lane[g] == 0 ? st : pop->side[pop->lane[g] - 1];
                HIPC(pop, launch_persistent(gr.cfg, pop->phase, pop->d_robots, pop->d_lists + gr.offset, gr.count,
                                            gr.count, pop->pl, pop->xbuf[pop->cur], pop->vbuf[pop->cur],
                                            sc + t0, cnt, pop->diverged, pop->c, sq));
            }
        }
        for (int l = 1; l < G; ++l)
            if (used[l]) {
                HIPC(pop, hipEventRecord(pop->ev[l], pop->side[l - 1]));
                HIPC(pop, hipStreamWaitEvent(st, pop->ev[l], 0));
            }
    }
    HIPC(pop, launch_advance(pop->d_step, n_steps, st));
    return SR_OK;
}
}  // namespace

int pop_set_graphs(sr_pop *pop, int32_t enable) {
    CHECK_POP(pop);
    pop->use_graphs = enable != 0;
    if (!pop->use_graphs) clear_graphs(pop);
    return SR_OK;
}

namespace {
// Steps with checkpoints: the time table in sc (n_steps entries), then blocks
// of steps that end at every checkpoint, each checkpoint copied into the
// buffers pop_record allocated.
int recorded_steps(sr_pop *pop, int n_steps, float2 *sc) {
    const double omega_dt = 2.0 * M_PI * (double)pop->p.act_freq * pop->p.dt;
    HIPC(pop, launch_sincos(sc, pop->d_step, n_steps, omega_dt, pop->c.actuation, pop->st));
    const int K = pop->rec_valid ? pop->ck_every : 0;
    for (int t = 0; t < n_steps;) {
        const int64_t g = pop->h_step + t;  // step index at the start of this block
        int len = n_steps - t;
        if (pop->spl > 0 && len > pop->spl) len = pop->spl;
        if (K > 0 && pop->rec_valid) {
            if (g % K == 0) {
                const int64_t cidx = g / K;
                if (cidx < pop->ck_cap) {
                    const size_t off = (size_t)cidx * pop->total_slots;
                    HIPC(pop, hipMemcpyAsync(pop->ck_x + off, pop->xbuf[pop->cur], sizeof(float4) * pop->total_slots,
                                             hipMemcpyDeviceToDevice, pop->st));
                    HIPC(pop, hipMemcpyAsync(pop->ck_v + off, pop->vbuf[pop->cur], sizeof(float4) * pop->total_slots,
                                             hipMemcpyDeviceToDevice, pop->st));
                } else {
                    pop->rec_valid = false;  // past the recorded horizon
                }
            }
            const int to_ck = (int)(K - g % K);
            if (len > to_ck) len = to_ck;
        }
        if (pop->mode == SR_STEP_PLAIN) {
            for (int q = 0; q < len; ++q) {
                const int a = pop->cur, b = 1 - pop->cur;
                HIPC(pop, launch_plain_step(pop->d_robots, pop->R, pop->total_slots, pop->rows, pop->entries, pop->pl,
                                            pop->xbuf[a], pop->vbuf[a], pop->xbuf[b], pop->vbuf[b], sc, t + q,
                                            pop->phase, pop->diverged, pop->slot_robot, pop->c, pop->st));
                pop->cur = b;
            }
        } else {
            for (const auto &gr : pop->groups) {
                HIPC(pop, launch_persistent(gr.cfg, pop->phase, pop->d_robots, pop->d_lists + gr.offset, gr.count,
                                            gr.count, pop->pl, pop->xbuf[pop->cur], pop->vbuf[pop->cur], sc + t,
                                            len, pop->diverged, pop->c, pop->st));
            }
        }
        t += len;
    }
    if (pop->mode == SR_STEP_PLAIN)
        HIPC(pop, launch_check_div(pop->d_robots, pop->R, pop->xbuf[pop->cur], pop->vbuf[pop->cur], pop->diverged,
                                   pop->c.lim, pop->st));
    HIPC(pop, launch_advance(pop->d_step, n_steps, pop->st));
    pop->h_step += n_steps;
    return SR_OK;
}
}  // namespace

int pop_step(sr_pop *pop, int32_t n_steps) {
    CHECK_POP(pop);
    if (!pop->built) return set_err(SR_ESTATE, "pop_step before a build");
    if (n_steps < 0) return set_err(SR_EINVAL, "n_steps < 0");
    if (n_steps == 0) return SR_OK;
    int rc = ensure_sc(pop, n_steps);
    if (rc) return rc;
    const bool recording = pop->rec_valid && pop->ck_every > 0;
    if (recording) return recorded_steps(pop, n_steps, pop->sc);
    if (!pop->use_graphs) {
        rc = enqueue_steps(pop, n_steps, pop->sc, pop->st);
        if (rc) return rc;
    } else {
        const GraphKey key{n_steps, pop->mode == SR_STEP_PLAIN ? 1 : 0, pop->cur, pop->spl};
        auto it = pop->graphs.find(key);
        const int cur0 = pop->cur;
        if (it == pop->graphs.end()) {
            HIPC(pop, hipStreamBeginCapture(pop->cap, hipStreamCaptureModeThreadLocal));
            rc = enqueue_steps(pop, n_steps, pop->sc, pop->cap);
            hipGraph_t graph = nullptr;
            hipError_t e2 = hipStreamEndCapture(pop->cap, &graph);
            if (rc) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc;
            }
            HIPC(pop, e2);
            hipGraphExec_t exec = nullptr;
            hipError_t e3 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            HIPC(pop, e3);
            it = pop->graphs.emplace(key, exec).first;
        }
        // the graph carries the buffer flips of the per-step form
        pop->cur = cur0 ^ ((pop->mode == SR_STEP_PLAIN) ? (n_steps & 1) : 0);
        HIPC(pop, hipGraphLaunch(it->second, pop->st));
    }
    pop->h_step += n_steps;
    return SR_OK;
}

int pop_step_noalloc(sr_pop *pop, int32_t n_steps) {
    CHECK_POP(pop);
    if (!pop->built) return set_err(SR_ESTATE, "pop_step_noalloc before a build");
    if (n_steps < 0) return set_err(SR_EINVAL, "n_steps < 0");
    if (n_steps > SR_NOALLOC_MAX_STEPS)
        return set_err(SR_EINVAL, "pop_step_noalloc: n_steps %d exceeds its step table of %d steps", n_steps,
                       SR_NOALLOC_MAX_STEPS);
    if (n_steps == 0) return SR_OK;
    float2 *sc = nullptr;
    int rc = noalloc_table(pop->device, &sc);
    if (rc) return rc;
    // direct launches only: capturing and instantiating a graph may allocate
    if (pop->rec_valid && pop->ck_every > 0) return recorded_steps(pop, n_steps, sc);
    rc = enqueue_steps(pop, n_steps, sc, pop->st);
    if (rc) return rc;
    pop->h_step += n_steps;
    return SR_OK;
}

int pop_fitness(sr_pop *pop, float *fitness) {
    CHECK_POP(pop);
    if (!pop->built) return set_err(SR_ESTATE, "pop_fitness before a build");
    if (!fitness) return set_err(SR_EINVAL, "null fitness");
    HIPC(pop, launch_fitness(pop->d_robots, pop->R, pop->xbuf[pop->cur], pop->x0, pop->diverged, fitness, pop->st));
    return SR_OK;
}

int pop_get_counts(sr_pop *pop, int32_t *n_masses, int32_t *n_springs, int64_t *mass_offset, int64_t *spring_offset) {
    CHECK_POP(pop);
    if (!pop->built) return set_err(SR_ESTATE, "pop_get_counts before a build");
    int rc = ensure_counts(pop);
    if (rc) return rc;
    for (int r = 0; r < pop->R; ++r) {
        if (n_masses) n_masses[r] = pop->h_robots[r].M;
        if (n_springs) n_springs[r] = pop->h_robots[r].S;
    }
    if (mass_offset) memcpy(mass_offset, pop->h_mass_off.data(), sizeof(int64_t) * (pop->R + 1));
    if (spring_offset) memcpy(spring_offset, pop->h_spring_off.data(), sizeof(int64_t) * (pop->R + 1));
    return SR_OK;
}

int pop_get_voxels(sr_pop *pop, uint8_t *kept, float *w) {
    CHECK_POP(pop);
    if (!pop->built) return set_err(SR_ESTATE, "pop_get_voxels before a build");
    if (kept) HIPC(pop, hipMemcpyAsync(kept, pop->kept, pop->total_vox, hipMemcpyDeviceToDevice, pop->st));
    if (w) HIPC(pop, hipMemcpyAsync(w, pop->w, sizeof(float) * pop->total_vox, hipMemcpyDeviceToDevice, pop->st));
    return SR_OK;
}

int pop_get_query(sr_pop *pop, uint8_t *cls, float *w) {
    CHECK_POP(pop);
    if (!pop->built) return set_err(SR_ESTATE, "pop_get_query before a build");
    if (cls) HIPC(pop, hipMemcpyAsync(cls, pop->q_cls, pop->total_vox, hipMemcpyDeviceToDevice, pop->st));
    if (w) HIPC(pop, hipMemcpyAsync(w, pop->w, sizeof(float) * pop->total_vox, hipMemcpyDeviceToDevice, pop->st));
    return SR_OK;
}

int pop_get_springs(sr_pop *pop, int32_t *ij, float *L0, float *k, float *a, float *phi) {
    CHECK_POP(pop);
    if (!pop->built) return set_err(SR_ESTATE, "pop_get_springs before a build");
    int rc = ensure_counts(pop);
    if (rc) return rc;
    HIPC(pop, launch_springs_io(pop->d_robots, pop->R, pop->total_slots, pop->slot_robot, pop->slot_node, pop->sid,
                                pop->d_spring_off, pop->pl, pop->p.voxel_len, ij, L0, k, a, phi, nullptr, nullptr,
                                nullptr, 0, pop->st));
    return SR_OK;
}

int pop_set_spring_params(sr_pop *pop, const float *k, const float *a, const float *phi) {
    CHECK_POP(pop);
    if (!pop->built) return set_err(SR_ESTATE, "pop_set_spring_params before a build");
    int rc = ensure_counts(pop);
    if (rc) return rc;
    if (phi && !pop->phase) {
        // the captured step graphs hold the kernels without the phase plane
        pop->phase = true;
        clear_graphs(pop);
    }
    if (pop->h_step > 0) pop->rec_valid = false;  // the recorded run used other parameters
    // kernels that rebuild the parameters from voxels would not see the new values
    pop->vox_ok = false;
    for (auto &g : pop->groups)
        if (g.cfg.variant & 96) {
            g.cfg.block = persist_default_block(g.n, pop->dash, false, &g.cfg.variant);
            clear_graphs(pop);
        }
    HIPC(pop, launch_springs_io(pop->d_robots, pop->R, pop->total_slots, pop->slot_robot, pop->slot_node, pop->sid,
                                pop->d_spring_off, pop->pl, pop->p.voxel_len, nullptr, nullptr, nullptr, nullptr,
                                nullptr, k, a, phi, 1, pop->st));
    return SR_OK;
}

int pop_get_state(sr_pop *pop, float *x, float *v, int64_t *step) {
    CHECK_POP(pop);
    if (!pop->built) return set_err(SR_ESTATE, "pop_get_state before a build");
    int rc = ensure_counts(pop);
    if (rc) return rc;
    HIPC(pop, launch_gather_state(pop->d_robots, pop->R, pop->total_slots, pop->slot_robot, pop->slot_node,
                                  pop->d_mass_off, pop->xbuf[pop->cur], pop->vbuf[pop->cur], x, v, 0, pop->st));
    if (step) *step = pop->h_step;
    return SR_OK;
}

int pop_set_state(sr_pop *pop, const float *x, const float *v, int64_t step) {
    CHECK_POP(pop);
    if (!pop->built) return set_err(SR_ESTATE, "pop_set_state before a build");
    if (step < 0) return set_err(SR_EINVAL, "step < 0");
    int rc = ensure_counts(pop);
    if (rc) return rc;
    HIPC(pop, launch_gather_state(pop->d_robots, pop->R, pop->total_slots, pop->slot_robot, pop->slot_node,
                                  pop->d_mass_off, pop->xbuf[pop->cur], pop->vbuf[pop->cur], const_cast<float *>(x),
                                  const_cast<float *>(v), 1, pop->st));
    HIPC(pop, hipStreamSynchronize(pop->st));
    pop->h_step = step;
    pop->h_step_stage = step;
    pop->rec_valid = false;
    HIPC(pop, hipMemcpyAsync(pop->d_step, &pop->h_step_stage, sizeof(int64_t), hipMemcpyHostToDevice, pop->st));
    HIPC(pop, hipMemsetAsync(pop->diverged, 0, pop->R, pop->st));
    HIPC(pop, hipStreamSynchronize(pop->st));
    return SR_OK;
}

int pop_get_status(sr_pop *pop, uint8_t *diverged) {
    CHECK_POP(pop);
    if (!diverged) return set_err(SR_EINVAL, "null output");
    HIPC(pop, hipMemcpyAsync(diverged, pop->diverged, pop->R, hipMemcpyDeviceToDevice, pop->st));
    return SR_OK;
}

int pop_reset(sr_pop *pop) {
    CHECK_POP(pop);
    if (!pop->built) return set_err(SR_ESTATE, "pop_reset before a build");
    HIPC(pop, hipMemcpyAsync(pop->xbuf[0], pop->x0, sizeof(float4) * pop->total_slots, hipMemcpyDeviceToDevice, pop->st));
    HIPC(pop, hipMemsetAsync(pop->vbuf[0], 0, sizeof(float4) * pop->total_slots, pop->st));
    HIPC(pop, hipMemsetAsync(pop->diverged, 0, pop->R, pop->st));
    pop->cur = 0;
    HIPC(pop, hipMemcpyAsync(pop->xbuf[1], pop->xbuf[0], sizeof(float4) * pop->total_slots, hipMemcpyDeviceToDevice,
                             pop->st));
    HIPC(pop, hipMemcpyAsync(pop->vbuf[1], pop->vbuf[0], sizeof(float4) * pop->total_slots, hipMemcpyDeviceToDevice,
                             pop->st));
    pop->h_step = 0;
    pop->h_step_stage = 0;
    HIPC(pop, hipMemcpyAsync(pop->d_step, &pop->h_step_stage, sizeof(int64_t), hipMemcpyHostToDevice, pop->st));
    HIPC(pop, hipStreamSynchronize(pop->st));
    pop->rec_valid = pop->ck_every > 0;
    return SR_OK;
}

int pop_record(sr_pop *pop, int32_t checkpoint_every, int32_t max_steps) {
    CHECK_POP(pop);
    if (checkpoint_every < 0 || max_steps < 0) return set_err(SR_EINVAL, "negative checkpoint interval or horizon");
    if (pop->ck_x) HIPC(pop, hipStreamSynchronize(pop->st));
    if (pop->ck_x) HIPC(pop, hipFree(pop->ck_x));
    if (pop->ck_v) HIPC(pop, hipFree(pop->ck_v));
    pop->ck_x = pop->ck_v = nullptr;
    pop->ck_every = 0;
    pop->ck_cap = 0;
    pop->rec_valid = false;
    if (checkpoint_every == 0) return SR_OK;
    const int cap = max_steps / checkpoint_every + 1;
    hipError_t e = dalloc(&pop->ck_x, (size_t)cap * pop->total_slots);
    if (e == hipSuccess) e = dalloc(&pop->ck_v, (size_t)cap * pop->total_slots);
    if (e != hipSuccess) return set_err(SR_ENOMEM, "checkpoint storage: %s", hipGetErrorString(e));
    pop->ck_every = checkpoint_every;
    pop->ck_cap = cap;
    pop->rec_valid = pop->built && pop->h_step == 0;
    return SR_OK;
}

namespace {
int ensure_adj_scratch(sr_pop *pop, int K) {
    if (K <= pop->rec_cap) return SR_OK;
    HIPC(pop, hipStreamSynchronize(pop->st));
    void *old[] = {pop->lx, pop->lv, pop->gk, pop->gs, pop->gc, pop->gd, pop->dJdw};
    for (void *p : old)
        if (p) HIPC(pop, hipFree(p));
    for (int b = 0; b < NSET; ++b) {
        void *seg[] = {pop->rec_x[b], pop->rec_v[b], pop->rec_u[b], pop->rec_l[b], pop->tmp_x[b], pop->tmp_v[b],
                       pop->sc_seg[b]};
        for (void *p : seg)
            if (p) HIPC(pop, hipFree(p));
        pop->rec_u[b] = pop->rec_l[b] = nullptr;
    }
    pop->gd = nullptr;
    const size_t S = pop->total_slots;
    const bool vel = pop->c.dash || pop->c.gdamp;  // the reverse step needs v_n
    bool split = false;  // some side's reverse step hands lambda_F to a gradient pass
    for (const auto &g : pop->groups) split = split || adjoint_is_split(g.n, vel);
    hipError_t e = hipSuccess;
    for (int b = 0; b < NSET; ++b) {
        if (e == hipSuccess) e = dalloc(&pop->rec_x[b], S * K);
        if (e == hipSuccess) e = dalloc(&pop->rec_v[b], S * K);
        if (e == hipSuccess && vel) e = dalloc(&pop->rec_u[b], S * K);
        if (e == hipSuccess && split) e = dalloc(&pop->rec_l[b], S * K);
        if (e == hipSuccess) e = dalloc(&pop->tmp_x[b], S);
        if (e == hipSuccess) e = dalloc(&pop->tmp_v[b], S);
        if (e == hipSuccess) e = dalloc(&pop->sc_seg[b], (size_t)K);
    }
    if (e == hipSuccess) e = dalloc(&pop->lx, S);
    if (e == hipSuccess) e = dalloc(&pop->lv, S);
    if (e == hipSuccess) e = dalloc(&pop->gk, S * NDIR);
    if (e == hipSuccess) e = dalloc(&pop->gs, S * NDIR);
    if (e == hipSuccess) e = dalloc(&pop->gc, S * NDIR);
    if (e == hipSuccess && vel) e = dalloc(&pop->gd, S * NDIR);
    if (e == hipSuccess) e = dalloc(&pop->dJdw, (size_t)pop->total_vox);
    if (e == hipSuccess && !pop->adj_st) e = hipStreamCreateWithFlags(&pop->adj_st, hipStreamNonBlocking);
    if (e == hipSuccess && !pop->adj_gst) e = hipStreamCreateWithFlags(&pop->adj_gst, hipStreamNonBlocking);
    for (auto &ev : pop->adj_ev)
        if (e == hipSuccess && !ev) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        pop->rec_cap = 0;
        return set_err(SR_ENOMEM, "adjoint scratch: %s", hipGetErrorString(e));
    }
    pop->rec_cap = K;
    return SR_OK;
}
}  // namespace

int pop_backward(sr_pop *pop, const float *dJ_dfitness, float *g_k, float *g_a, float *g_phi, const float *genomes,
                 const float *B, float *g_genome) {
    CHECK_POP(pop);
    if (!dJ_dfitness) return set_err(SR_EINVAL, "null dJ/dfitness");
    if (!pop->built) return set_err(SR_ESTATE, "pop_backward before a build");
    if (!pop->rec_valid || pop->ck_every <= 0)
        return set_err(SR_ESTATE, "no recorded run: call pop_record right after the build, then pop_step");
    if (g_genome && (!genomes || !B)) return set_err(SR_EINVAL, "genome gradient needs the genomes and B");
    const int K = pop->ck_every;
    int rc = ensure_adj_scratch(pop, K);
    if (rc) return rc;
    rc = ensure_counts(pop);
    if (rc) return rc;
    const double omega_dt = 2.0 * M_PI * (double)pop->p.act_freq * pop->p.dt;
    HIPC(pop, launch_adj_init(pop->d_robots, pop->total_slots, pop->slot_robot, pop->x0, dJ_dfitness, pop->lx, pop->lv,
                              pop->gk, pop->gs, pop->gc, pop->gd, pop->st));
    const int64_t T = pop->h_step;
    const int nseg = (int)((T + K - 1) / K);
    // Segments are reversed last to first on the population's stream.  The
    // recomputation (checkpoint -> recorded states) of the segment before runs
    // meanwhile on adj_st into the other buffer set, so a population too small
    // to fill the GPU overlaps the two; for the sides whose adjoint is split,
    // the gradient passes of a segment run on adj_gst while the next segment is
    // reversed (they read only that segment's buffers and the gradient sums,
    // which the reversal does not touch).  Events order every buffer reuse.
    const bool vel = pop->c.dash || pop->c.gdamp;
    bool split = false;
    for (const auto &g : pop->groups) split = split || adjoint_is_split(g.n, vel);
    hipEvent_t ev_start = pop->adj_ev[0], *ev_rec = pop->adj_ev + 1, *ev_rev = pop->adj_ev + 1 + NSET,
               *ev_grd = pop->adj_ev + 1 + 2 * NSET;
    hipEvent_t *ev_free = split ? ev_grd : ev_rev;  // buffer set b's last readers are done
    HIPC(pop, hipEventRecord(ev_start, pop->st));
    HIPC(pop, hipStreamWaitEvent(pop->adj_st, ev_start, 0));
    auto recompute = [&](int seg) -> int {
        const int b = seg % NSET;
        const int64_t s0 = (int64_t)seg * K;
        const int len = (int)((T - s0) < K ? (T - s0) : K);
        const size_t off = (size_t)seg * pop->total_slots;
        // buffer set b was last read by the reversal (and gradient passes) of segment seg + NSET
        if (seg + NSET < nseg) HIPC(pop, hipStreamWaitEvent(pop->adj_st, ev_free[b], 0));
        HIPC(pop, hipMemcpyAsync(pop->tmp_x[b], pop->ck_x + off, sizeof(float4) * pop->total_slots,
                                 hipMemcpyDeviceToDevice, pop->adj_st));
        HIPC(pop, hipMemcpyAsync(pop->tmp_v[b], pop->ck_v + off, sizeof(float4) * pop->total_slots,
                                 hipMemcpyDeviceToDevice, pop->adj_st));
        HIPC(pop, launch_sincos_at(pop->sc_seg[b], s0, len, omega_dt, pop->c.actuation, pop->adj_st));
        for (const auto &gr : pop->groups)
            HIPC(pop, launch_record(gr.n, pop->phase, pop->d_robots, pop->d_lists + gr.offset, gr.count, pop->pl,
                                    pop->tmp_x[b], pop->tmp_v[b], pop->sc_seg[b], len, pop->diverged, pop->c,
                                    pop->rec_x[b], pop->rec_v[b], pop->rec_u[b], pop->adj_st));
        HIPC(pop, hipEventRecord(ev_rec[b], pop->adj_st));
        return SR_OK;
    };
    if (nseg > 0 && (rc = recompute(nseg - 1))) return rc;
    for (int seg = nseg - 1; seg >= 0; --seg) {
        const int b = seg % NSET;
        const int64_t s0 = (int64_t)seg * K;
        const int len = (int)((T - s0) < K ? (T - s0) : K);
        if (seg > 0 && (rc = recompute(seg - 1))) return rc;
        HIPC(pop, hipStreamWaitEvent(pop->st, ev_rec[b], 0));
        for (const auto &gr : pop->groups)
            HIPC(pop, launch_adjoint(gr.n, pop->phase, pop->d_robots, pop->d_lists + gr.offset, gr.count, pop->pl,
                                     pop->x0, pop->rec_x[b], pop->rec_v[b], pop->rec_u[b], pop->rec_l[b], len,
                                     pop->sc_seg[b],
                                     pop->lx, pop->lv, pop->gk, pop->gs, pop->gc, pop->gd, pop->c, pop->st));
        HIPC(pop, hipEventRecord(ev_rev[b], pop->st));
        if (split) {
            HIPC(pop, hipStreamWaitEvent(pop->adj_gst, ev_rev[b], 0));
            for (const auto &gr : pop->groups)
                if (adjoint_is_split(gr.n, vel))
                    HIPC(pop, launch_adj_grad(gr.n, pop->phase, pop->d_robots, pop->d_lists + gr.offset, gr.count,
                                              pop->pl, pop->x0, pop->rec_x[b], pop->rec_u[b], pop->rec_l[b], len,
                                              pop->sc_seg[b], pop->gk, pop->gs, pop->gc, pop->gd, pop->c,
                                              pop->adj_gst));
            HIPC(pop, hipEventRecord(ev_grd[b], pop->adj_gst));
        }
    }
    if (split && nseg > 0) HIPC(pop, hipStreamWaitEvent(pop->st, ev_grd[0], 0));  // segment 0's sums
    HIPC(pop, launch_adj_springs(pop->d_robots, pop->total_slots, pop->slot_robot, pop->sid, pop->d_spring_off, pop->pl,
                                 pop->p.voxel_len, pop->gk, pop->gs, pop->gc, g_k, g_a, g_phi, pop->st));
    if (g_genome)
        HIPC(pop, launch_adj_genome(pop->d_robots, pop->R, pop->total_vox, pop->vox_robot, pop->kept, pop->w, pop->pl,
                                    pop->gk, pop->gs, pop->gc, pop->gd, pop->p, genomes, B, pop->dJdw, g_genome,
                                    pop->st));
    return SR_OK;
}

int ga_generation(const float *fitness, const float *genomes_in, float *genomes_out, int32_t P, int32_t L,
                  const sr_ga_params *params, uint64_t seed, uint64_t generation, int32_t *decisions, void *stream) {
    if (!fitness || !genomes_in || !genomes_out || !params) return set_err(SR_EINVAL, "null argument");
    if (P < 1 || L < 1) return set_err(SR_EINVAL, "P and L must be >= 1 (got %d, %d)", P, L);
    if (params->tournament_k < 1 || params->tournament_k > 64)
        return set_err(SR_EINVAL, "tournament_k %d outside 1..64", params->tournament_k);
    if (!(params->elite_frac >= 0.0 && params->elite_frac <= 1.0))
        return set_err(SR_EINVAL, "elite_frac outside [0, 1]");
    const char *a0 = reinterpret_cast<const char *>(genomes_in), *b0 = reinterpret_cast<const char *>(genomes_out);
    const size_t bytes = sizeof(float) * (size_t)P * (size_t)L;
    if (a0 < b0 + bytes && b0 < a0 + bytes) return set_err(SR_EINVAL, "genomes_out overlaps genomes_in");
    int E = (int)floor(params->elite_frac * (double)P);
    if (E > P) E = P;
    hipError_t e = launch_ga(fitness, genomes_in, genomes_out, P, L, E, params->tournament_k, params->p_cross_thr,
                             params->p_mut_thr, params->mut_sigma, seed, generation, decisions,
                             reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) return set_err(SR_EHIP, "ga_generation: %s", hipGetErrorString(e));
    return SR_OK;
}

}  // extern "C"

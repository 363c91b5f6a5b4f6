/*
 * softrobot.h -- C ABI of the MI355X (gfx950) soft-robot co-design hot path.
 *
 * Method: arXiv 2405.00698, "CUDA-Accelerated Soft Robot Neural Evolution with
 * Large Language Model Supervision".  A population of voxel robots (Sec. II-A)
 * is built from per-robot MLP genomes queried over each robot's voxel grid
 * through the Gaussian positional encoding of Eq. (1) (Sec. II-B), simulated
 * as spring-mass systems, scored, and evolved by a GA with elites, crossover
 * and mutation (Sec. II-C; rates in Table I; physics in Table II).
 *
 * Conventions shared by every call:
 *  - Return value: SR_OK (0) or a negative SR_E* code; sr_last_error() gives a
 *    thread-local message for the last failing call.  SR_EHIP is sticky on a
 *    population: once a device error is seen the handle only accepts
 *    pop_destroy.
 *  - Pointers marked "dev" are device memory (e.g. torch tensor data_ptr()s),
 *    pointers marked "host" are host memory.  The caller owns all of them; the
 *    library never frees or keeps them past the call.
 *  - Every device call is asynchronous on the stream given to pop_create (or
 *    to the free function); calls that return host data synchronise it.
 *  - Voxel arrays are concatenated over robots in robot order; robot r holds
 *    n_r^3 entries with linear id i + n_r (j + n_r k) (x fastest, z up).
 *  - Node (mass) ids of a robot are its lattice points (a, b, c) in [0, n]^3
 *    that touch a kept voxel, numbered in ascending a + (n+1)(b + (n+1) c).
 *    Springs are numbered by (lower node id, higher node id).  Per-robot node
 *    and spring arrays are concatenated in robot order (offsets from
 *    pop_get_counts).
 *  - A handle is not thread-safe.
 */
#ifndef SOFTROBOT_H
#define SOFTROBOT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SR_OK 0
#define SR_EINVAL (-1)       /* bad argument, size or shape */
#define SR_ENOMEM (-2)       /* device or host allocation failed */
#define SR_EHIP (-3)         /* HIP runtime error (sticky on the handle) */
#define SR_ESTATE (-4)       /* call out of order, e.g. step before build */
#define SR_EUNSUPPORTED (-5) /* valid request this build cannot serve */

/* sr_sim_params.flags: test modes */
#define SR_NO_GRAVITY 1u
#define SR_NO_GROUND 2u
#define SR_NO_ACTUATION 4u
/* Table II material model: a muscle voxel's actuation amplitude and phase are
 * its class values (the maxima) times its sigmoid weight (Sec. II-C). */
#define SR_WEIGHT_ACTUATION 8u

#define SR_GENOME_LEN 8710 /* W1[64][64] b1[64] W2[64][64] b2[64] W3[6][64] b3[6] */
#define SR_PE_M 32         /* rows of the encoding matrix B (Eq. (1)), d = 3 */
#define SR_MAX_SIDE 12     /* largest grid side n */
#define SR_NOALLOC_MAX_STEPS 65536 /* largest n_steps of pop_step_noalloc */

/* Build precision of the genome query. */
#define SR_QUERY_FP32 0 /* FP32 FMA throughout */
#define SR_QUERY_BF16 1 /* BF16 inputs, FP32 accumulate on MFMA */

/* Step kernels. */
#define SR_STEP_AUTO 0       /* persistent, tuned configuration */
#define SR_STEP_PERSISTENT 1 /* LDS-resident, many steps per launch */
#define SR_STEP_PLAIN 2      /* one launch per step, state in HBM */

/* Physics.  Table II gives gravity 9.81 m/s^2, 0.1 kg per node, rest length
 * 0.1 m and ground stiffness 1e5 N/m; sr_default_params fills those, the
 * workload's dt = 1e-4 s, damping 0.999 per step, friction mu = 0.5, class
 * stiffness {0, 1e4, 1e4, 3e3, 3e4} N/m for {empty, expanding muscle,
 * contracting muscle, soft tissue, bone} and the muscle law
 * L0 (1 +- 0.2 sin(2 pi 4 Hz t)). */
typedef struct {
    double dt;          /* time step [s] */
    float gravity;      /* |g| [m/s^2], along -z */
    float damping;      /* velocity factor applied every step */
    float mass;         /* mass of every node [kg] */
    float voxel_len;    /* voxel edge = edge-spring rest length [m] */
    float k_ground;     /* penalty stiffness of the plane z = 0 [N/m] */
    float mu;           /* Coulomb friction coefficient */
    float act_freq;     /* actuation frequency [Hz] */
    float k_class[5];   /* stiffness per material class [N/m] */
    float a_class[5];   /* actuation amplitude per class, relative to L0 */
    float phi_class[5]; /* actuation phase per class [rad] */
    uint32_t flags;     /* SR_NO_* test modes, SR_WEIGHT_ACTUATION */
    /* Table II contact and damping terms; zero leaves them out.
     * mu_static: a node pressed on the ground sticks when its tangential speed
     *   is within max(mu_static, mu) N dt / m (N the normal force); otherwise
     *   kinetic friction mu acts.  Only matters when above mu.
     * zeta_spring: damping ratio of a dashpot beside each voxel spring,
     *   c = zeta sqrt(2 m k_c w); a shared spring sums its voxels' dashpots.
     * zeta_ground: damping ratio of the ground contact, c_g = 2 zeta sqrt(k_ground m);
     *   the normal force k_ground (-z) - c_g v_z is clamped at zero. */
    float mu_static;
    float zeta_spring;
    float zeta_ground;
    float reserved;
} sr_sim_params;

/* GA rates (Table I: mutation rate 0.1, crossover rate 0.4, elite 0.3;
 * tournament size 4 and mutation N(0, 0.02^2) from the workload).
 * Probabilities are 64-bit thresholds floor(p * 2^64): a draw r passes when
 * r < threshold. */
typedef struct {
    double elite_frac;    /* elites = floor(elite_frac * P) */
    int32_t tournament_k; /* draws per tournament, with replacement, 1..64 */
    int32_t reserved;
    uint64_t p_cross_thr; /* uniform-crossover probability threshold */
    uint64_t p_mut_thr;   /* per-gene mutation probability threshold */
    float mut_sigma;      /* standard deviation of a mutation step */
    float reserved2;
} sr_ga_params;

typedef struct sr_pop sr_pop; /* opaque, library-owned */

const char *sr_last_error(void);
int sr_version(void);

/* Fills *out with the defaults above. */
int sr_default_params(sr_sim_params *out);

/* Fills *out with Table II as printed: class stiffness {0, 2e3, 2e3, 1e3, 1e4} N/m,
 * dt = 1e-5 s, muscle amplitude up to 0.25 and phase up to pi scaled by the
 * voxel weight (SR_WEIGHT_ACTUATION; expanding +0.25, contracting -0.25),
 * spring and ground damping ratio 0.1, static friction 0.6 and kinetic 1.0,
 * no per-step velocity damping; 4 Hz muscles as in the defaults. */
int sr_table2_params(sr_sim_params *out);

/* Creates a population of n_robots robots; grid_side (host [n_robots]) gives
 * each robot's side n, 1..SR_MAX_SIDE.  stream: hipStream_t for every call on
 * the handle (NULL = default stream). */
int pop_create(const sr_sim_params *params, int32_t n_robots, const int32_t *grid_side,
               void *stream, sr_pop **out);
int pop_destroy(sr_pop *pop);

/* Builds every robot from voxel classes and weights (Sec. II-A, II-C).
 * cls (dev, uint8, concatenated n_r^3): material class 0..4 (0 = empty);
 * w (dev, float): sigmoid weight per voxel.  Keeps the largest face-connected
 * component (ties: the one with the smallest voxel id), puts a node on every
 * corner of a kept voxel and a spring on each of the 28 corner pairs of a kept
 * voxel, deduplicated.  A spring shared by several voxels is their parallel
 * combination: k = sum k_c w, k a e^{i phi} = sum k_c w a_c e^{i phi_c}.
 * Resets the state to step 0 (lattice positions, lowest node on the ground,
 * zero velocity).  SR_EINVAL when a class is out of range. */
int pop_build_from_voxels(sr_pop *pop, const uint8_t *cls, const float *w);

/* Queries every robot's genome MLP over its grid, then builds as above.
 * genomes (dev, [n_robots][SR_GENOME_LEN] float); B (dev, [SR_PE_M][3] float).
 * Query point of voxel (i,j,k): ((i+1/2)/n, (j+1/2)/n, (k+1/2)/n);
 * gamma(v) = [cos(2 pi B v), sin(2 pi B v)] (Eq. (1)); h1 = tanh(W1 gamma + b1);
 * h2 = tanh(W2 h1 + b2); o = W3 h2 + b3; class = argmax o[0..4] (lowest id on
 * ties; the softmax branch), w = sigmoid(o[5]) (the sigmoid branch).
 * precision: SR_QUERY_FP32 or SR_QUERY_BF16. */
int pop_build_from_genomes(sr_pop *pop, const float *genomes, const float *B, int32_t precision);

/* Chooses the step kernel; block / steps_per_launch <= 0 keep the tuned or
 * default values.  SR_EUNSUPPORTED for a configuration the kernels lack. */
int pop_set_step_config(sr_pop *pop, int32_t mode, int32_t block, int32_t steps_per_launch);

/* Roofline microbenchmark on the current device (synchronous): which = 0, 1,
 * 2 LDS reads of 16, 12, 4 bytes per lane; 3 FP32 FMA; 4 v_rsq_f32; 5 HBM
 * streaming copy of 512 MiB (iters passes; allocates its two buffers).
 * Returns the time of one launch (*seconds) and its work (*units: bytes for
 * the LDS reads and the copy (read plus written), lane operations for the
 * VALU cases). */
int sr_microbench(int32_t which, int32_t iters, double *seconds, double *units);

/* Lists the persistent kernel configurations compiled for side n: writes up
 * to cap (block, variant) pairs (host arrays, may be NULL when cap is 0) and
 * returns how many exist (>= 0), or SR_EINVAL. */
int sr_persist_configs(int32_t n, int32_t *blocks, int32_t *variants, int32_t cap);

/* Steps without checkpoints run as captured HIP graphs (one per step count,
 * step form and state buffer), with one parallel branch per grid side;
 * enable = 0 launches the kernels directly instead.  On by default. */
int pop_set_graphs(sr_pop *pop, int32_t enable);

/* Picks the persistent kernel for robots of side n: block threads per
 * workgroup and variant, a sum of
 *   0 recompute every spring force at both ends, 1 exchange spring
 *     coefficients through LDS, 2 exchange in two direction chunks;
 *   +4 bounds the LDS loads in flight to save registers;
 *   +8 reads positions with 12-byte instead of 16-byte LDS loads;
 *   +16 marks the kernels with spring dashpots, which also share velocities
 *     through LDS: a population with zeta_spring != 0 accepts only those, any
 *     other population only the rest;
 *   +32 / +64 rebuild the diagonal / all springs' parameters each step from
 *     per-voxel terms (not after pop_set_spring_params); +128 keeps one
 *     position buffer;
 *   +256 * L keeps up to L + 1 neighbour reads in flight (L < 16);
 *   +4096 * (B + 1) sets the backward springs' reads apart (B in flight);
 *   +131072 / +262144 software-pipeline the backward / forward springs;
 *   +524288 cuts the slots into runs of 64, one wave each, so that runs in
 *     the top / bottom lattice plane skip the directions leaving the lattice;
 *   +1048576 pads each coefficient row only by its own stencil offset (less
 *     LDS, for the one-chunk exchange at the largest sides);
 *   +2097152 + 4194304 * (U - 1) leaves the direction loops rolled (unrolled
 *     by U), with every parameter rebuilt from voxels;
 *   +16777216 * (P - 1) steps P robots in one workgroup (block / P threads
 *     each), for small grids.
 * sr_persist_configs lists the compiled combinations.  All variants of one
 * kind give bit-identical results.  SR_EUNSUPPORTED for a combination the
 * library lacks or that does not match the population's physics. */
int pop_set_persist_variant(sr_pop *pop, int32_t n, int32_t block, int32_t variant);
/* Launch schedule of the persistent step kernels (batching of uneven
 * populations, the paper's one-robot-per-block launch generalised to several
 * grid sides, Sec. II-C): the population's robots of one side form a group,
 * launched as one kernel per block of steps.  sides (host, n entries) lists
 * every side present, once, in launch order; lanes (host, n entries) puts
 * each on a stream: 0 is the population's stream, k in 1..n-1 a private one.
 * Groups on one lane run one after another; lanes run side by side (forked
 * from and joined back into the population's stream, also inside captured
 * step graphs).  Results do not depend on the schedule.  Default: largest
 * side first, every group on its own lane.  SR_EINVAL unless n is the number
 * of distinct sides and the lists are valid.  Clears the captured graphs. */
int pop_set_schedule(sr_pop *pop, int32_t n, const int32_t *sides, const int32_t *lanes);
/* The schedule in use (host outputs, one entry per distinct side). */
int pop_get_schedule(sr_pop *pop, int32_t *sides, int32_t *lanes);
/* The persistent kernel configuration in use for side n (host outputs). */
int pop_get_persist_variant(sr_pop *pop, int32_t n, int32_t *block, int32_t *variant);

/* Time stepping of the spring-mass robots (Sec. II-C: every robot's springs
 * and masses advanced in parallel; physics per Table II: rest length, mass per
 * node, stiffness per material, muscle actuation, gravity, ground elasticity
 * and friction).
 * Advances every robot n_steps >= 0 steps.  Step n -> n+1 (t_n = n dt):
 * spring forces k (r - L(t_n)) along each spring with L = L0 (1 + a sin(2 pi f
 * t_n + phi)) plus, with zeta_spring, the dashpot c (v_j - v_i).d^; gravity
 * -m g e_z; ground normal N = k_ground max(0, -z) (minus the contact damper
 * c_g v_z with zeta_ground, clamped at zero); v' = v + dt F / m; where N > 0
 * the horizontal part of v' sticks at zero within max(mu_static, mu) N dt / m
 * and otherwise loses mu N dt / m without reversing; v <- damping v';
 * x <- x + dt v.  All forces use the state of step n.  A robot whose state is non-finite or beyond
 * 1e3 n voxel lengths at the end of a launch is flagged diverged and frozen. */
int pop_step(sr_pop *pop, int32_t n_steps);

/* pop_step for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * steps, kernels and results (bit for bit) as pop_step, and like it
 * asynchronous on the population's stream, but it calls no hipMalloc, hipFree
 * or allocating runtime routine and captures no graph: the per-step time
 * table lives in a static device array of SR_NOALLOC_MAX_STEPS entries
 * (512 KiB per device, held until the process ends), and the kernels are
 * launched directly.  n_steps above SR_NOALLOC_MAX_STEPS: SR_EINVAL.  Every
 * call on one device shares that table: calls that overlap on one device
 * (two populations stepped concurrently on different streams) race, so
 * order them on one stream or with events.  Checkpoints go to the buffers
 * pop_record allocated, as in pop_step. */
int pop_step_noalloc(sr_pop *pop, int32_t n_steps);

/* Puts every robot back at its build state (step 0, lattice positions, zero
 * velocity, no divergence flag), keeping the spring parameters; restarts a
 * recording that pop_record turned on. */
int pop_reset(sr_pop *pop);

/* Turns on checkpointing for the adjoint: the state is saved every
 * checkpoint_every steps of the run that starts at the build (call right
 * after the build, before pop_step), up to max_steps steps; 0 turns it off.
 * Another build restarts the recording; pop_set_state, and new spring
 * parameters after the first step, end it. */
int pop_record(sr_pop *pop, int32_t checkpoint_every, int32_t max_steps);

/* Reverse-mode gradient of J = sum_r dJ_dfitness[r] * fitness_r for the steps
 * recorded since the build (dev [n_robots] float), by segments: each
 * checkpointed segment is recomputed storing its states, then reversed
 * step by step (contact and friction branches as taken).  Outputs (dev,
 * canonical spring order, NULL to skip): dJ/dk, dJ/da, dJ/dphi per spring.
 * g_genome (dev [n_robots][SR_GENOME_LEN] or NULL): dJ/dgenome through the
 * sigmoid weight head, the parallel-sum rule and the MLP in FP32 (the class
 * head, the component step and the topology carry no gradient; with
 * SR_WEIGHT_ACTUATION also through the weight-scaled amplitude and phase);
 * needs the genomes and B (dev) of the build.  With the Table II dashpots
 * (zeta_spring, zeta_ground) the forces also depend on the velocities: the
 * recording keeps v_n of every step as well, dJ/dk is taken at fixed dashpot
 * coefficients, and the genome gradient also flows through c = zeta
 * sqrt(2 m k_c w).  SR_ESTATE without a recorded run.  Gradients of a
 * diverged robot are undefined. */
int pop_backward(sr_pop *pop, const float *dJ_dfitness, float *g_k, float *g_a, float *g_phi,
                 const float *genomes, const float *B, float *g_genome);

/* fitness (dev, [n_robots] float): mean over nodes of x_x(now) - x_x(build),
 * i.e. the centre-of-mass displacement along +x; -inf for a diverged robot
 * and for a robot with no occupied voxel (it has no body). */
int pop_fitness(sr_pop *pop, float *fitness);

/* Introspection (host outputs; synchronise the stream).  Any pointer may be
 * NULL.  n_masses / n_springs: host [n_robots]; mass_offset / spring_offset:
 * host [n_robots + 1] prefix sums. */
int pop_get_counts(sr_pop *pop, int32_t *n_masses, int32_t *n_springs, int64_t *mass_offset,
                   int64_t *spring_offset);
/* kept (dev uint8, concatenated n_r^3): class of kept voxels, 0 elsewhere;
 * w (dev float): the sigmoid weight per voxel (from the build input). */
int pop_get_voxels(sr_pop *pop, uint8_t *kept, float *w);
/* The build's per-voxel input before the component step (dev, concatenated
 * n_r^3): cls the material class, w the sigmoid weight.  After
 * pop_build_from_genomes these are the genome query's heads. */
int pop_get_query(sr_pop *pop, uint8_t *cls, float *w);
/* Springs in canonical order (dev, concatenated over robots): ij [S][2] int32
 * node ids within the robot, L0 rest length, k stiffness, a amplitude, phi
 * phase (a signed and phi = 0 when every term of the parallel sum is in phase). */
int pop_get_springs(sr_pop *pop, int32_t *ij, float *L0, float *k, float *a, float *phi);
/* Overwrites spring parameters (dev, canonical order; NULL keeps a field). */
int pop_set_spring_params(sr_pop *pop, const float *k, const float *a, const float *phi);
/* State in canonical node order (dev, [total masses][3] float) and the step
 * index (host).  set_state keeps the build positions as the fitness origin. */
int pop_get_state(sr_pop *pop, float *x, float *v, int64_t *step);
int pop_set_state(sr_pop *pop, const float *x, const float *v, int64_t step);
/* diverged (dev, [n_robots] uint8). */
int pop_get_status(sr_pop *pop, uint8_t *diverged);

/* One GA generation (Sec. II-C; rates of Table I).  Individuals are ranked
 * by fitness (larger first, NaN as -inf, ties to the lower index); the
 * floor(elite_frac * P) best are copied unchanged into slots 0.. in rank
 * order.  Every other slot c gets a child: two tournaments of tournament_k
 * draws with replacement (index = (hi32(r) * P) >> 32; best wins, ties to
 * the lower index); with probability p_cross uniform crossover (gene g from
 * the second parent when bit g mod 64 of word (g mod 256) / 64 of the
 * crossover draw block g / 256 is set), otherwise a copy of the first
 * parent; then each gene mutates with probability p_mut by
 * mut_sigma * N(0, 1) (Box-Muller on two 53-bit uniforms).  Every random
 * word is Philox-4x64-10 (Salmon et al., SC'11) with key (seed, 0) and
 * counter (generation, c, purpose, block), purpose 0/1 the two tournaments,
 * 2 the crossover flag, 3 the crossover mask, 4 the mutation flags (word g mod
 * 4 of block g / 4), 5 the Gaussian pairs (words 2 (g mod 2), +1 of block
 * g / 2).  fitness (dev [P] float), genomes_in / genomes_out (dev [P][L]
 * float, must not overlap), decisions (dev [P][3] int32 or NULL): (parent A,
 * parent B, kind) with kind 0 elite, 1 copy, 2 crossover.  Asynchronous on
 * stream (hipStream_t, NULL = default). */
int ga_generation(const float *fitness, const float *genomes_in, float *genomes_out, int32_t P, int32_t L,
                  const sr_ga_params *params, uint64_t seed, uint64_t generation, int32_t *decisions,
                  void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SOFTROBOT_H */

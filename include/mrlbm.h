/*
 * mrlbm.h -- C ABI of the MI355X multiresolution-adapted lattice Boltzmann library.
 *
 * One handle holds one adaptive MR-LBM run (or a batch of independent runs) on the GPU:
 * a DdQq scheme with lattice velocity lambda, relaxation rates s and built-in
 * equilibria (Sec. 2.1 and Sec. 5 of Bellotti, Gouarin, Graille, Massot, "Multiresolution-
 * based mesh adaptation and error control for lattice Boltzmann methods with applications
 * to hyperbolic conservation laws"), nested dyadic lattices J_min..J (Sec. 3), the centered
 * prediction of half-width gamma (Sec. 3.1), the threshold eps (Sec. 3.4) and the
 * regularity guess mu_bar of the enlargement rule (Sec. 4.2).
 *
 * Conventions shared by every entry point
 *  - Every call returns a status code (MRLBM_OK = 0 or a negative MRLBM_E*); nothing
 *    throws or aborts across the ABI.
 *  - Parameters are validated on the host before any device allocation or launch.
 *  - Host buffers are owned by the caller; create copies what it needs, queries write
 *    into caller-provided arrays of stated capacity. If a capacity is too small the call
 *    returns MRLBM_ECAPACITY and sets the required size in *n_out.
 *  - Device memory is owned by the handle (allocated in create, freed in destroy).
 *  - Work is ordered on the handle's HIP stream (the one passed at create, or a private
 *    non-blocking stream when NULL is passed). step/adapt only enqueue; queries and
 *    stats synchronize the stream.
 *  - A handle is not thread-safe. MRLBM_ENUMERIC (a NaN met in a detail or a collision) is
 *    sticky: afterwards every call but destroy and last_error returns it.
 *  - Conserved moments are ordered by physics: advection/Burgers (u); shallow water
 *    (h, hu); Euler (rho, rho u, E). Populations are internal.
 */
#ifndef MRLBM_H
#define MRLBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MRLBM_ABI_VERSION 1

enum mrlbm_status {
    MRLBM_OK = 0,
    MRLBM_EINVAL = -1,    /* invalid argument or parameter set                  */
    MRLBM_ENOMEM = -2,    /* device allocation failed                           */
    MRLBM_EDEVICE = -3,   /* HIP runtime error (no device, launch failure, ...) */
    MRLBM_ENUMERIC = -4,  /* NaN met in a detail or collision; sticky           */
    MRLBM_ECAPACITY = -5, /* output capacity too small, or J beyond the limit   */
    MRLBM_ESTATE = -6     /* call not valid in the handle's state               */
};

/* Schemes (Sec. 5.1.1 D1Q2, Sec. 5.2.1 D1Q3 and D1Q5, Sec. 5.3 vectorial D1Q2^k). D1Q5 has
 * the velocities 0, +-lambda, +-2 lambda: its stream reaches two cells (sigma = 2). */
enum mrlbm_scheme { MRLBM_D1Q2 = 0, MRLBM_D1Q3 = 1, MRLBM_D1Q2x2 = 2, MRLBM_D1Q2x3 = 3, MRLBM_D1Q5 = 4 };
/* Physics (equilibria). Valid pairs: D1Q2+{ADVECTION,BURGERS}, D1Q3+{BURGERS,SHALLOW_WATER},
 * D1Q2x2+SHALLOW_WATER, D1Q2x3+EULER, D1Q5+SHALLOW_WATER. */
enum mrlbm_physics { MRLBM_ADVECTION = 0, MRLBM_BURGERS = 1, MRLBM_SHALLOW_WATER = 2, MRLBM_EULER = 3 };
/* Boundary reading: wrap, or map an out-of-range index to the nearest cell of its level. */
enum mrlbm_bc { MRLBM_PERIODIC = 0, MRLBM_CLAMP = 1 };
/* Storage precision: FP64, or FP32 state with details and thresholds evaluated in FP64. */
enum mrlbm_precision { MRLBM_FP64 = 0, MRLBM_FP32_STORAGE = 1 };
/* Where moments are reported: on the complete leaves (spatial order) or reconstructed
 * on every cell of the finest lattice (Sec. 3.3, reconstruction operator). */
enum mrlbm_where { MRLBM_LEAVES = 0, MRLBM_FINEST = 1 };

/* Largest finest level. Up to MRLBM_ONCHIP_MAX_J a run's tree arrays live in its workgroup's
 * LDS; above it (a handle with such a run) every run of the handle keeps its tree arrays and
 * values in device memory. That mode is much slower and has no launch classes, tuner,
 * refinement predictor or reconstructed collision (ESTATE / EINVAL). */
#define MRLBM_MAX_J 24
#define MRLBM_ONCHIP_MAX_J 16

/* Collision of the adaptive step (mrlbm_params.flags). Default (0): the leaves collision
 * (Sec. 4.5, eq. LeavesCollision), every complete leaf collides on its own value.
 * MRLBM_FLAG_RECONSTRUCTED_COLLISION: the reconstructed collision (Sec. 4.3.1,
 * eq. reconstructedCollision): the leaf values of the new tree are projected up, every
 * complete leaf (l, k) reconstructs its 2^(J-l) finest cells, and its non-conserved moments
 * relax towards the mean over them of the equilibria of the reconstructed conserved moments
 * (summed in cell order, scaled by 2^-(J-l)); its conserved moments stay. It costs
 * O(2^(J-l) (J-l)) per leaf and is the collision the paper's error estimate covers. Not
 * available together with the refinement predictor (mrlbm_set_predictor returns
 * MRLBM_EINVAL). */
#define MRLBM_FLAG_RECONSTRUCTED_COLLISION 1u

typedef struct {
    int32_t abi_version; /* must be MRLBM_ABI_VERSION                                    */
    int32_t scheme;      /* enum mrlbm_scheme                                              */
    int32_t physics;     /* enum mrlbm_physics                                             */
    int32_t bc;          /* enum mrlbm_bc                                                  */
    int32_t precision;   /* enum mrlbm_precision                                           */
    int32_t n_s;         /* number of rates in s: 1 (broadcast) or q - q_cons              */
    double lambda;       /* lattice velocity > 0; dt = dx_J / lambda (Sec. 2.1)            */
    double s[8];         /* relaxation rates of the non-conserved moments, in (0, 2]       */
    double phys[4];      /* [0] advection velocity V (D1Q5: beta of the fifth-moment
                            equilibrium beta lambda^2 M2eq), [1] gravity g > 0,
                            [2] gamma_gas > 1, [3] alpha > 0 of the D1Q3 Burgers
                            third-moment equilibrium alpha lambda^2 u (D1Q5: of the
                            fourth-moment equilibrium alpha lambda^2 hu)                  */
    double x_min, x_max; /* domain [a, b], a < b (Sec. 2)                                  */
    int32_t j_min;       /* coarsest level, 0 <= j_min <= j_max (periodic: see below)      */
    int32_t j_max;       /* finest level J <= MRLBM_MAX_J                                   */
    int32_t gamma;       /* prediction half-width 1..3 (Sec. 3.1)                          */
    int32_t mu_bar;      /* regularity guess of enlargement rule (b), 0..30 (Sec. 4.2)      */
    double eps;          /* threshold eps >= 0, finite; eps_j = 2^(j-J) eps (Sec. 3.4)       */
    uint32_t flags;      /* 0 or MRLBM_FLAG_RECONSTRUCTED_COLLISION                         */
    int32_t reserved;
} mrlbm_params;

typedef struct {
    int64_t steps;        /* time steps taken                                            */
    int64_t leaves;       /* #S(Lambda) of the current tree                               */
    int64_t leaf_updates; /* sum over steps of #S(Lambda^{n+1}): leaf-cell updates        */
    int32_t numeric_error;/* 1 once a NaN was met                                         */
    int32_t q;            /* populations per cell                                         */
    int32_t q_cons;       /* conserved moments per cell                                   */
    int32_t j_max;
    int64_t tree_cells;   /* #R(Lambda): cells of the complete tree (leaves + split cells) */
    int64_t misses;       /* refinement predictor: declined pairs the judge found wrong     */
    int64_t redos;        /* refinement predictor: steps redone after a miss                */
} mrlbm_stats_t;

typedef struct mrlbm_s* mrlbm_t;
typedef struct mrlbm_batch_s* mrlbm_batch_t;

/* Validate p on the host; returns MRLBM_OK or MRLBM_EINVAL/MRLBM_ECAPACITY without
 * touching the device. Useful to test a parameter set before create. */
int mrlbm_validate(const mrlbm_params* p);

/* Create one run. m_cons0: host array [q_cons][2^j_max] of finest-level conserved cell
 * averages at t = 0 (Sec. 2: averages on the finest lattice); populations start at
 * equilibrium and Lambda^0 is the full tree (Sec. 4.4, start of the error analysis).
 * hip_stream: a hipStream_t cast to void*, or NULL for a private stream.
 * On success *out holds the handle; on failure *out is NULL. */
int mrlbm_create(const mrlbm_params* p, const double* m_cons0, void* hip_stream, mrlbm_t* out);

/* Mesh adaptation only: Lambda <- G(H_eps(T_eps(Lambda))) with the data transfer of
 * Sec. 4.1.1 (projection for coarsened cells, prediction for added cells). */
int mrlbm_adapt(mrlbm_t h);

/* nsteps >= 0 full time steps: adaptation, leaves collision (Sec. 4.5, eq.
 * LeavesCollision) and the compact reconstructed stream (Sec. 4.3.2, eq.
 * AdaptiveStreamPhase). Enqueued on the handle's stream. */
int mrlbm_step(mrlbm_t h, int32_t nsteps);

/* Conserved moments, written as out[c * n + i] for moment c and position i.
 * where = MRLBM_LEAVES: i runs over the complete leaves in spatial order, n = #S.
 * where = MRLBM_FINEST: i runs over the 2^J finest cells (reconstruction), n = 2^J.
 * cap is the capacity of out in doubles (>= q_cons * n); *n_out receives n. */
int mrlbm_moments(mrlbm_t h, int32_t where, double* out, int64_t cap, int64_t* n_out);

/* Populations on the complete leaves in spatial order, out[h * n + i]; same capacity
 * rules (cap >= q * n). FP32 storage is widened to double. */
int mrlbm_populations(mrlbm_t h, double* out, int64_t cap, int64_t* n_out);

/* Complete leaves (Sec. 3.3) in spatial order: level[i], index[i]; cap entries each. */
int mrlbm_leaves(mrlbm_t h, int32_t* level, int64_t* index, int64_t cap, int64_t* n_leaves);

int mrlbm_stats(mrlbm_t h, mrlbm_stats_t* st);

/* Wall time of nsteps steps measured with HIP events on the handle's stream around the
 * launches (milliseconds). Synchronizes. */
int mrlbm_step_timed(mrlbm_t h, int32_t nsteps, double* elapsed_ms);

void mrlbm_destroy(mrlbm_t h);

/* Last error message of the handle (or of the last failed create when h is NULL). The
 * string is owned by the library and valid until the next call on the handle. */
const char* mrlbm_last_error(mrlbm_t h);

/* ---------------------------------------------------------------- batched engine
 * n independent runs advanced by one launch per call (or by launches of at most
 * mrlbm_batch_set_launch_steps steps): one workgroup per run, every step of the run inside
 * the workgroup (intra-workgroup barriers only). All runs of one batch
 * share scheme, precision and gamma; J, eps, physics and the other parameters may differ.
 * m_cons0[i] points to run i's [q_cons][2^j_max(i)] host array. The launch for a given
 * nsteps is captured once in a HIP graph and replayed. */
int mrlbm_batch_create(const mrlbm_params* p, int32_t n, const double* const* m_cons0,
                       void* hip_stream, mrlbm_batch_t* out);
int mrlbm_batch_step(mrlbm_batch_t b, int32_t nsteps);
int mrlbm_batch_step_timed(mrlbm_batch_t b, int32_t nsteps, double* elapsed_ms);
int mrlbm_batch_moments(mrlbm_batch_t b, int32_t inst, int32_t where, double* out, int64_t cap,
                        int64_t* n_out);
int mrlbm_batch_leaves(mrlbm_batch_t b, int32_t inst, int32_t* level, int64_t* index, int64_t cap,
                       int64_t* n_leaves);
int mrlbm_batch_stats(mrlbm_batch_t b, int32_t inst, mrlbm_stats_t* st);
/* Sum of leaf_updates over all runs of the batch. Synchronizes. */
int mrlbm_batch_total_updates(mrlbm_batch_t b, int64_t* total);
/* Launch shape used by the batch: threads per workgroup (64..512, multiple of 64), 0 =
 * let the built-in tuner choose. Takes effect at the next step call. MRLBM_ESTATE while
 * launch classes are set (mrlbm_batch_set_classes: each class has its own shape). */
int mrlbm_batch_set_block(mrlbm_batch_t b, int32_t threads);
int mrlbm_batch_get_block(mrlbm_batch_t b, int32_t* threads);
/* On-chip capacity: a run keeps the values of its tree in the workgroup's LDS while the tree
 * has at most this many cells of R(Lambda), and in its HBM arrays otherwise (same results).
 * cells = -1: the largest capacity the device's LDS allows (default); 0: always HBM.
 * get_capacity returns the capacity of the single launch (the classes' own capacities come
 * from mrlbm_batch_get_classes). MRLBM_ESTATE while launch classes are set. */
int mrlbm_batch_set_capacity(mrlbm_batch_t b, int32_t cells);
/* Built-in tuner: times trial_steps steps of the batch for every candidate launch shape
 * (threads per workgroup 128/256/384/512 x LDS capacity for 1, 2, 3, 4 or 8 runs per compute
 * unit, at most 32 waves per compute unit), then for every candidate schedule (see
 * mrlbm_batch_set_schedule: identity, the device's CU count, 8, heaviest first); when the
 * runs' j_max span three levels or more, also three two-class launches (see
 * mrlbm_batch_set_classes: the runs up to j_max - 2 or j_max - 1 in 128-thread workgroups
 * sized for eight per compute unit, the others in 256-thread workgroups for four, or in
 * 512-thread workgroups for two). It restores the runs' state after each trial and keeps the
 * fastest (leaf-cell updates/s); the runs end in the state they had before the call.
 * Allocates a temporary snapshot of the handle's device memory. The chosen block size and
 * capacity are returned when the pointers are non-NULL, both 0 when launch classes won
 * (mrlbm_batch_get_classes has them). MRLBM_ESTATE for a handle with a run beyond
 * MRLBM_ONCHIP_MAX_J (nothing on chip to tune). */
int mrlbm_batch_tune(mrlbm_batch_t b, int32_t trial_steps, int32_t* threads, int32_t* cells);
/* Workgroup-to-run schedule of the batched launch (results do not depend on it). stride 0:
 * workgroup i advances run i. stride s > 0: runs ranked heaviest first by a-priori cost
 * (larger j_max, then smaller eps, which keeps more cells, then more leaves at the call);
 * the workgroups i with (i / s) even take the heaviest runs in order and workgroup i + s the
 * lightest ones, so that workgroups sharing a compute unit pair a heavy run with a light one
 * (the launch lasts as long as its slowest run). stride >= the number of runs: heaviest
 * first (for batches larger than the device holds at once, the light runs fill the slots
 * the heavy ones free). get_schedule returns the stride in use. */
int mrlbm_batch_set_schedule(mrlbm_batch_t b, int32_t stride);
int mrlbm_batch_get_schedule(mrlbm_batch_t b, int32_t* stride);
/* Longest launch: a step call of more steps is issued as consecutive launches of at most
 * `steps` steps each on the handle's stream (same results). 0 (default): one launch per
 * call. */
int mrlbm_batch_set_launch_steps(mrlbm_batch_t b, int32_t steps);
/* Checkpoint of every run of the batch (stored values, trees, leaf lists and statistics),
 * kept in device memory that the handle allocates at the first call (one more copy of the
 * batch's device pool) and frees with it; a later call overwrites it. restore puts every
 * run back to the checkpoint (MRLBM_EINVAL when none was taken); the launch shape, the
 * schedule and the predictor settings are not part of it. Both synchronise the handle's
 * stream. */
int mrlbm_batch_checkpoint(mrlbm_batch_t b);
int mrlbm_batch_restore(mrlbm_batch_t b);
int mrlbm_batch_get_capacity(mrlbm_batch_t b, int32_t* cells);
/* Launch classes. A launch gives every workgroup the LDS its largest run needs, so in a batch
 * of uneven J the small runs hold more LDS than they use and fewer of them share a compute unit.
 * With n classes (1..4) the runs are split by j_max: class c holds the runs with
 * j_upper[c-1] < j_max <= j_upper[c] (j_upper increasing, the last one >= the largest j_max);
 * each class is advanced by a grid of its own with threads[c] per workgroup (64..512, a multiple
 * of 64) and the on-chip capacity that lets runs_per_cu[c] (1..16) of its workgroups share a
 * compute unit's LDS. The class grids are forked from the handle's stream onto a second stream
 * of the same priority and joined back (in one captured graph), so they run side by side; within
 * a class the runs go heaviest first (mrlbm_batch_set_schedule then reorders within each class).
 * Results do not depend on the classes. n = 0 restores the single launch; mrlbm_batch_tune
 * replaces the classes with its own choice; not available with the refinement predictor
 * (MRLBM_EINVAL either way) or for a handle with a run beyond MRLBM_ONCHIP_MAX_J (MRLBM_ESTATE).
 * get_classes returns the number of classes in *n and, for cap_n >= *n,
 * the runs and the on-chip capacity of each class. */
int mrlbm_batch_set_classes(mrlbm_batch_t b, int32_t n, const int32_t* j_upper, const int32_t* threads,
                            const int32_t* runs_per_cu);
int mrlbm_batch_get_classes(mrlbm_batch_t b, int32_t cap_n, int32_t* n, int32_t* counts, int32_t* cells);
void mrlbm_batch_destroy(mrlbm_batch_t b);
const char* mrlbm_batch_last_error(mrlbm_batch_t b);

/* ---------------------------------------------------------------- refinement predictor
 * Not part of the paper's method: a small network (32 inputs, two hidden layers of 64 ReLU
 * units, one logit; bfloat16 parameters, float32 sums) stands in for enlargement rule (b)
 * (Sec. 4.2, eq. HartenLossOfRegularity) on the pairs that rule would refine with
 * D < gate * 2^(mu_bar+1) eps_l; rule (a) is unchanged. The paper's heuristic judges every
 * step: a declined pair whose detail after the step still reaches the rule-(b) threshold is a
 * miss (eq. DetailRatio); the step is then redone from t^n with the missed pairs refined, so
 * the enlarged mesh never falls below what the judge demands. Runs with FP64 storage and
 * gamma = 1. Parameter vector order: W1[64][32], b1[64], W2[64][64], b2[64], w3[64], b3.
 * Features of a pair (split cell p of level l): d / (|d| + eps_{l+1}) of the details of the
 * split cells p-2..p+2 for every population ([delta][population]; 0 where not split), then
 * (l+1)/J, zero-padded to 32. */
#define MRLBM_MLP_INPUTS 32
#define MRLBM_MLP_PARAMS 6337
enum mrlbm_predictor_mode { MRLBM_PRED_OFF = 0, MRLBM_PRED_LEARNED = 1, MRLBM_PRED_RECORD = 2 };

/* Attach the predictor to every run of a handle. bf16_params: MRLBM_MLP_PARAMS bfloat16
 * values (host, copied; required for MRLBM_PRED_LEARNED). MRLBM_PRED_RECORD: plain rule (b),
 * and every rule-(b) pair of every step becomes a training sample (features at t^n, label 1
 * when the pair's detail after the step still reaches the rule-(b) threshold, i.e. when
 * declining it would have been a miss), up to
 * sample_capacity samples (the buffer restarts empty at each call). MRLBM_PRED_OFF restores
 * the plain method. FP64 storage and gamma = 1 only (MRLBM_EINVAL); MRLBM_ESTATE for a handle
 * with a run beyond MRLBM_ONCHIP_MAX_J. */
int mrlbm_set_predictor(mrlbm_t h, const uint16_t* bf16_params, int32_t mode, double gate, int64_t sample_capacity);
int mrlbm_batch_set_predictor(mrlbm_batch_t b, const uint16_t* bf16_params, int32_t mode, double gate,
                              int64_t sample_capacity);
/* Recorded samples: X[n][MRLBM_MLP_INPUTS] and y[n] (host arrays of cap rows). */
int mrlbm_samples(mrlbm_t h, float* X, float* y, int64_t cap, int64_t* n);
int mrlbm_batch_samples(mrlbm_batch_t b, float* X, float* y, int64_t cap, int64_t* n);

/* Training of the network on the GPU (weighted binary cross-entropy on the logit, Adam on
 * float32 master parameters; forward and backward products on the matrix cores with
 * bfloat16 operands). theta0: initial float32 parameters (host). */
typedef struct mrlbm_mlp_s* mrlbm_mlp_t;
int mrlbm_mlp_create(const float* theta0, mrlbm_mlp_t* out);
/* Mean loss and its gradient (float32, MRLBM_MLP_PARAMS) on n host samples. */
int mrlbm_mlp_loss_grad(mrlbm_mlp_t m, const float* X, const float* y, int64_t n, float pos_weight, float* loss,
                        float* grad);
/* epochs over n host samples in minibatches of `batch` (a multiple of 64), reshuffled from
 * seed every epoch; *last_loss = mean minibatch loss of the last epoch. */
int mrlbm_mlp_train(mrlbm_mlp_t m, const float* X, const float* y, int64_t n, int32_t epochs, int32_t batch, float lr,
                    float pos_weight, uint64_t seed, float* last_loss);
/* Current parameters: float32 master copy and/or the bfloat16 copy the steps use. */
int mrlbm_mlp_params(mrlbm_mlp_t m, float* theta, uint16_t* bf16);
/* Logits of n host feature rows with the bfloat16 parameters, as the steps compute them. */
int mrlbm_mlp_logits(mrlbm_mlp_t m, const float* X, int64_t n, float* logits);
void mrlbm_mlp_destroy(mrlbm_mlp_t m);
const char* mrlbm_mlp_last_error(mrlbm_mlp_t m);

/* ---------------------------------------------------------------- two dimensions
 * The multi-dimensional extension the paper outlines in its conclusion (dimension d = 2): a
 * quadtree of dyadic squares J_min..J on [0, 1]^2, projection as the mean over the four children,
 * the tensor product of the centered prediction (Sec. 3.1) with four details per parent, level
 * thresholds eps_l = 2^{d (l - J)} eps (Sec. 3.4 as the conclusion modifies it), enlargement rule
 * (a) on sigma-boxes and rule (b) at 2^{mu_bar + d} eps_l (Sec. 4.2), grading on gamma-boxes
 * (Sec. 3.3), the leaves collision (Sec. 4.5) and the compact stream (Sec. 4.3.2), for each leaf
 * and velocity the difference of the strips of reconstructed values entering and leaving it.
 * The scheme is D2Q4 for u_t + phi_x(u)_x + phi_y(u)_y = 0 (velocities lambda (+-1, 0),
 * (0, +-1); moments u, m1 = lambda (f0 - f1), m2 = lambda (f2 - f3), m3 = lambda^2 (f0 + f1 - f2 - f3);
 * equilibria phi_x(u), phi_y(u), 0 with phi = (Vx u, Vy u) for advection, (u^2/2, u^2/2) for
 * Burgers): the paper leaves multi-D schemes to a companion work. Levels are held densely in
 * device memory and stepped by level-wide kernels; J <= 12. Conventions of the 1D handle apply
 * (status codes, host validation, caller-owned host buffers, calls ordered on the stream). */
typedef struct {
    int32_t abi_version; /* MRLBM_ABI_VERSION                                   */
    int32_t physics;     /* MRLBM_ADVECTION or MRLBM_BURGERS                     */
    int32_t bc;          /* MRLBM_PERIODIC or MRLBM_CLAMP, in both directions    */
    int32_t gamma;       /* prediction half-width 1..3                           */
    double lambda;       /* lattice velocity > 0                                 */
    double s[3];         /* relaxation rates of m1, m2, m3, in (0, 2]            */
    double V[2];         /* advection velocity (advection only)                  */
    int32_t j_min, j_max;/* 0 <= j_min <= j_max <= 12 (periodic: 2^j_min >= 2 gamma + 1) */
    int32_t mu_bar;      /* regularity guess of rule (b), 0..30                  */
    int32_t reserved;
    double eps;          /* threshold eps >= 0                                   */
} mrlbm2d_params;
typedef struct mrlbm2d_s* mrlbm2d_t;
int mrlbm2d_validate(const mrlbm2d_params* p);
/* u0: host array [2^J][2^J] (index i * 2^J + j, i along x) of finest cell averages at t = 0;
 * populations at equilibrium on the full tree. */
int mrlbm2d_create(const mrlbm2d_params* p, const double* u0, void* hip_stream, mrlbm2d_t* out);
/* nsteps time steps (adaptation, leaves collision, compact stream), enqueued on the handle's
 * stream; the leaf counts stay on the device and are read back once, at the end of the call
 * (which synchronizes the stream). MRLBM_ENUMERIC when a value became NaN. */
int mrlbm2d_step(mrlbm2d_t h, int32_t nsteps);
/* mrlbm2d_step with the time between HIP events recorded on the handle's stream before the
 * first and after the last step, in *ms. */
int mrlbm2d_step_timed(mrlbm2d_t h, int32_t nsteps, float* ms);
/* u reconstructed on every finest cell, out[i * 2^J + j] (cap >= 4^J). */
int mrlbm2d_moments(mrlbm2d_t h, double* out, int64_t cap);
/* split flags of level j_min <= level < j_max, out[i * 2^level + j] (cap >= 4^level). */
int mrlbm2d_split(mrlbm2d_t h, int32_t level, uint8_t* out, int64_t cap);
/* time steps taken, complete leaves of the current tree, sum over steps of the leaves. */
int mrlbm2d_stats(mrlbm2d_t h, int64_t* steps, int64_t* leaves, int64_t* leaf_updates);
void mrlbm2d_destroy(mrlbm2d_t h);
const char* mrlbm2d_last_error(mrlbm2d_t h);

/* ---------------------------------------------------------------- allocation-free run
 * For callers that cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc. One run is set up from p and the finest-level
 * conserved averages d_m_cons0 (a DEVICE array [q_cons][2^j_max], read only), advanced by
 * nsteps >= 0 full steps, and its conserved moments reconstructed on the finest level are
 * written to d_m_out (a DEVICE array [q_cons][2^j_max], owned by the caller): the same bits as
 * mrlbm_create + mrlbm_step(nsteps) + mrlbm_moments(MRLBM_FINEST) on the same data.
 *
 * Nothing is allocated. The run's state (values, tree, leaf list, interface pairs, descriptor)
 * lives in a file-scope device array of MRLBM_NOALLOC_SCRATCH_BYTES bytes that every GPU the
 * library runs on holds until the process ends; its address on a device is looked up once,
 * at the first call with that device current. Every call on one GPU shares that array and
 * overwrites it (it is cleared by a fill kernel at the start of each call): calls that overlap
 * on one GPU (different streams or host threads) race, and the caller must order them.
 *
 * Enqueued on hip_stream (NULL: the null stream); returns without synchronizing. Errors:
 * MRLBM_EINVAL for an invalid parameter set (mrlbm_validate), nsteps < 0 or a NULL pointer;
 * MRLBM_ECAPACITY when the run's state exceeds the scratch array (for FP64 that is J <= 14 with
 * six populations, J <= 15 with two); MRLBM_EDEVICE on a HIP error. The device input is not
 * checked for NaN: a NaN met in a step propagates into d_m_out. No message is kept
 * (mrlbm_last_error is not updated). */
#define MRLBM_NOALLOC_SCRATCH_BYTES (5u << 20)
int mrlbm_run_noalloc(const mrlbm_params* p, const double* d_m_cons0, int32_t nsteps, double* d_m_out,
                      void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* MRLBM_H */

/*
 * bmotor.h -- C ABI of libbmotor: Monte Carlo integration of Brownian-motor
 * Langevin equations on one AMD Instinct MI355X (gfx950).
 *
 * The method (Spiechowicz, Kostur & Machura, "GPU accelerated Monte Carlo
 * simulation of Brownian motors dynamics with CUDA"):
 *   - eq. (24):  x' = -V'(x) + eta(t) + Gamma(t) + xi(t)   (overdamped), and the
 *     inertial form  x'' + gamma x' = -V'(x) + a cos(omega t) + F + noise;
 *   - Algorithm 1: weak order 2.0 predictor-corrector step, three drift
 *     evaluations per step;
 *   - Algorithm 2 / eq. (25): simplified three-point Gaussian increment;
 *   - Algorithm 3 / eqs. (3)-(8), (26)-(27): white Poissonian increment, by
 *     default with the kicks on the fixed step grid (the integer countdown of the
 *     algorithm); BM_NOISE_JUMP_GRID puts them at their exact times;
 *   - Algorithm 4 / eqs. (13)-(17), (29)-(30): dichotomous increment;
 *   - Sec. 5 (Instruction optimization): x kept modulo L, periods counted apart;
 *   - eq. (31): <v> = < (x(t_f) - x(t_i)) / (t_f - t_i) > over the ensemble.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.   The caller owns all device memory.  Pointers named d_* are device
 *           pointers (e.g. torch tensors' data_ptr()), h_* are host pointers.
 *           The library never allocates device memory for user data; a handle
 *           owns only host-side metadata.  A workspace must outlive every handle
 *           created on it and every call enqueued with it.
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *           Device work is enqueued asynchronously on it; results are valid once
 *           the stream has been synchronised.  Host structs are read during the
 *           call only.
 * Errors.   Every int-returning call returns BM_OK (0) or a negative BM_ERR_*.
 *           Arguments are validated before anything is enqueued; on error
 *           nothing is enqueued and no state changes.  bm_last_error() gives a
 *           message for the calling thread's last failure.  Non-finite path
 *           velocities are counted in bm_stats, not reported as errors.
 * Threads.  A handle is not thread-safe; distinct handles are independent.
 * Randomness. Counter-based Philox4x32-10 (Salmon et al., SC'11), key = seed,
 *           counter = (block, path, point, stream tag).  Results depend only on
 *           (model, run, path index, step index): never on launch shape, chunking
 *           or which other paths run alongside.
 */
#ifndef BMOTOR_H
#define BMOTOR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BM_ABI_VERSION 2u

/* return codes */
#define BM_OK               0
#define BM_ERR_INVALID_ARG (-1)  /* NULL pointer, bad size field, out-of-range parameter */
#define BM_ERR_UNSUPPORTED (-2)  /* valid but outside what the kernels implement           */
#define BM_ERR_WORKSPACE   (-3)  /* workspace too small or misaligned (256 B)              */
#define BM_ERR_DEVICE      (-4)  /* no usable gfx950 device, or a HIP call failed          */
#define BM_ERR_STATE       (-5)  /* call not valid in the handle's current state           */

/* bm_model.dyn */
#define BM_OVERDAMPED 0u   /* eq. (24)                                                     */
#define BM_INERTIAL   1u   /* x'' + gamma x' = -V'(x) + a cos(omega t) + F + noise         */

/* bm_model.pot: the periodic potential V(x) and its period L */
#define BM_POT_SIN     0u  /* V = sin(2 pi x), L = 1                                       */
#define BM_POT_RATCHET 1u  /* V = -sin(2 pi x) - sin(4 pi x)/4, L = 1                      */
#define BM_POT_TENT    2u  /* eq. (2): V = 1 + x on [-1,0), 1 - x on [0,1], L = 2          */
#define BM_POT_FREE    3u  /* V = 0 (L = 1 for the folding)                                */

/* bm_model.noise: bit mask */
#define BM_NOISE_GAUSS   1u  /* xi: Gaussian white noise, Algorithm 2                       */
#define BM_NOISE_POISSON 2u  /* eta: white Poissonian noise, Algorithm 3                    */
#define BM_NOISE_DICH    4u  /* Gamma: dichotomous noise, Algorithm 4                       */
/* xi integrated with normal increments N(0, G^2 dt) instead of eq. (25)'s three-point
 * law: the non-simplified scheme, for comparison (Sec. 4).  The standard normal of
 * step n is the Box-Muller transform of words (2j, 2j+1), j = (n mod 4)/2, of the
 * Philox block (n/4, path, point, tag 0): cos for even n, sin for odd n.  Excludes
 * BM_NOISE_GAUSS; ensembles only (bm_scan rejects it with BM_ERR_UNSUPPORTED). */
#define BM_NOISE_NORMAL  8u
/* With BM_NOISE_POISSON: the jump-adapted grid of Sec. 4 (kicks at their exact
 * times t_i; waiting times E/lambda are not rounded to the step).  A step that holds
 * kicks is cut at each t_i; each piece is integrated by Algorithm 1 with its own
 * length and a Gaussian increment of matching variance (the step's own draw scaled
 * by sqrt(piece/dt) for the first piece; for the piece after kick k a draw from tag
 * 5 indexed by k), and the kick is added at the end of its piece.  Requires
 * BM_NOISE_POISSON and shot_rate*dt <= 16; ensembles only (bm_scan rejects it). */
#define BM_NOISE_JUMP_GRID 16u

/* bm_run.prec: arithmetic of the path state (statistics are always FP64) */
#define BM_F64 0u
#define BM_F32 1u

typedef struct bm_model {
    uint32_t size;         /* = sizeof(bm_model)                                          */
    uint32_t dyn;          /* BM_OVERDAMPED | BM_INERTIAL                                 */
    uint32_t pot;          /* BM_POT_*                                                    */
    uint32_t noise;        /* BM_NOISE_* mask                                             */
    double gamma;          /* friction (inertial only), > 0                               */
    double drive_amp;      /* a in a cos(omega t); needs steps_per_period > 0 if != 0     */
    double drive_omega;    /* omega > 0 when steps_per_period > 0                         */
    double force;          /* constant tilt F                                             */
    double D;              /* Gaussian intensity D_G >= 0: G = sqrt(2D) (overdamped),
                              sqrt(2 gamma D) (inertial)                                   */
    double shot_rate;      /* lambda > 0, eq. (4)                                         */
    double shot_mean;      /* zeta >= 0, eq. (5); bias a = lambda zeta, eq. (6)            */
    double dich_Fa;        /* eq. (13): level -Fa (Fa >= 0)                                */
    double dich_Fb;        /* eq. (13): level +Fb (Fb >= 0)                                */
    double dich_mua;       /* eq. (14): rate of leaving -Fa, > 0                           */
    double dich_mub;       /* eq. (14): rate of leaving +Fb, > 0                           */
} bm_model;

typedef struct bm_run {
    uint32_t size;             /* = sizeof(bm_run)                                         */
    uint32_t prec;             /* BM_F64 | BM_F32                                          */
    uint32_t steps_per_period; /* spp > 0: dt = (2 pi / omega) / spp and the drive phase is
                                  the integer step index mod spp; 0: no periodic drive      */
    uint32_t point_id;         /* parameter-point index in the random-stream counter        */
    double dt;                 /* time step if spp == 0 (> 0); must be 0 if spp > 0         */
    uint64_t n_steps;          /* horizon t_f = n_steps dt (used by bm_scan)                */
    uint64_t window_start;     /* eq. (31): t_i = window_start dt                           */
    uint64_t n_paths;          /* 1 .. 2^32 - 1                                             */
    uint64_t seed;             /* Philox key                                                */
    double x0_lo, x0_hi;       /* x(0) ~ U[x0_lo, x0_hi)                                    */
    double v0_lo, v0_hi;       /* v(0) ~ U[v0_lo, v0_hi) (inertial)                         */
    double step_tol;           /* step-size control on chi (see below); 0: fixed step dt    */
    uint32_t max_halvings;     /* with step_tol > 0: smallest step dt / 2^max_halvings, 1..8 */
    uint32_t pad;              /* 0                                                         */
} bm_run;

/* Step-size control.  The paper notes after Algorithm 1 that chi = (predictor) -
 * (corrector) estimates the local error and may steer the step size; it gives no
 * controller.  This library's: steps are dt / 2^l, 0 <= l <= max_halvings, starting
 * at the smallest; one controller serves each group of 64 consecutive paths
 * (64 g .. 64 g + 63, those below n_paths) -- one wavefront of the kernel.  After
 * each step, if some path of the group has max(|chi_x|, |chi_v|) > step_tol (or a
 * NaN) the next step is halved; if all have it below step_tol / 16 it is doubled,
 * where the doubled step starts on its own grid (so no step crosses a multiple of
 * dt); otherwise it is kept.  Every step is accepted.  Step k of a path (counting
 * steps of every size) takes the k-th Algorithm 2 draw of its tag-0 stream scaled
 * by G sqrt(3 h).  The drive at t = (n + u / 2^L) dt is a cos(2 pi ((n mod spp)
 * 2^L + u) / (spp 2^L)) + F, L = max_halvings.  The Poisson and dichotomous
 * processes keep their dt grid: a flip at step n sets the level of the whole step,
 * a kick drawn at step n is added after its last sub-step.  A path's result depends
 * on the paths of its group (not on the launch shape or chunking).  n_steps and
 * window_start still count steps of dt.  Ensembles only (bm_scan rejects it); not
 * with BM_NOISE_NORMAL or BM_NOISE_JUMP_GRID (BM_ERR_UNSUPPORTED); one path per
 * lane. */

typedef struct bm_stats {
    uint64_t n;            /* paths with a finite velocity                                */
    uint64_t n_nonfinite;  /* paths whose velocity is NaN or infinite                     */
    double mean;           /* <v>, eq. (31)                                               */
    double var;            /* unbiased sample variance of the per-path velocities          */
    double se;             /* standard error sqrt(var / n)                                 */
    double t_window;       /* t_f - t_i used                                               */
} bm_stats;

typedef struct bm_tune {
    uint32_t size;            /* = sizeof(bm_tune)                                         */
    uint32_t paths_per_lane;  /* 1 or 2 (2: FP32 paths only)                               */
    uint32_t block;           /* work-group size: 64, 128, 256, 512                         */
    uint32_t groups_per_cu;   /* persistent scan: work-groups per CU (0: as many as fit)   */
} bm_tune;

typedef struct bm_ensemble bm_ensemble;

/* Library version of this header (BM_ABI_VERSION). */
uint32_t bm_abi_version(void);

/* Message of the calling thread's last failed call ("" if none).  The pointer
 * stays valid until that thread's next call into the library. */
const char *bm_last_error(void);

/* Bytes of device workspace an ensemble of (model, run) needs (multiple of 256). */
int bm_ensemble_workspace_size(const bm_model *model, const bm_run *run, size_t *bytes);

/* Create an ensemble of run->n_paths independent realisations on the workspace
 * d_ws (256-byte aligned, >= bm_ensemble_workspace_size bytes) and enqueue the
 * initial conditions on `stream`: x(0), v(0) uniform, Poisson countdown
 * s = floor(E / (lambda dt)) with E ~ Exp(1), dichotomous state drawn from its
 * stationary law Pr{+Fb} = mu_a / (mu_a + mu_b) and entered at step 0.
 * The drive table (a cos(2 pi k / spp) + F in FP64) is uploaded from host memory
 * and create returns once that copy is complete (it synchronises `stream`).
 * The handle is written to *out.  BM_ERR_DEVICE if no gfx950 device is usable. */
int bm_ensemble_create(const bm_model *model, const bm_run *run, void *d_ws, size_t ws_bytes,
                       void *stream, bm_ensemble **out);

/* Checkpoint / resume.  The caller-owned workspace holds the whole state of an
 * ensemble (positions, velocities, window snapshot, jump countdowns and counts,
 * per-path velocities); the handle holds only host metadata and the step count
 * bm_ensemble_steps reports.  A checkpoint is therefore a byte copy of the
 * workspace (device or host) taken after the stream has completed, plus that
 * step count.  bm_ensemble_attach opens a handle on such a workspace (d_ws,
 * 256-byte aligned, >= bm_ensemble_workspace_size bytes) without touching the
 * path state: integrating from there gives bit for bit what an uninterrupted run
 * gives (the random streams are counter-based).  model and run must equal those
 * the workspace was created with -- the library cannot check this.  Uploads the
 * drive table like bm_ensemble_create (and synchronises `stream`). */
int bm_ensemble_attach(const bm_model *model, const bm_run *run, void *d_ws, size_t ws_bytes,
                       uint64_t steps_done, void *stream, bm_ensemble **out);

/* Release the handle (host metadata only; the workspace stays the caller's). */
int bm_ensemble_destroy(bm_ensemble *e);

/* Choose the launch shape (NULL: the default for this model, see bm_tune_set_default).
 * Results never depend on it.  BM_ERR_UNSUPPORTED if the jump queues of the shape
 * exceed 64 KiB of LDS per work-group. */
int bm_ensemble_set_tune(bm_ensemble *e, const bm_tune *tune);

/* Advance every path by n_steps steps of Algorithm 1 (with Algorithms 2-4 for
 * the enabled noises), enqueued on the ensemble's stream.  Resumable: any
 * split of a horizon into calls gives bit-identical states.  The position at
 * step window_start is recorded for eq. (31). */
int bm_integrate(bm_ensemble *e, uint64_t n_steps);

/* Steps integrated so far (host-side counter; no synchronisation). */
int bm_ensemble_steps(const bm_ensemble *e, uint64_t *n_done);

/* Enqueue the FP64 ensemble reduction of eq. (31) over the current state:
 * per path v_p = ((w - w_i) L + (x - x_i)) / ((n - n_i) dt), then count, mean,
 * unbiased variance and standard error with compensated (double-double) sums in
 * a fixed order (independent of the launch shape).  Writes one bm_stats to the
 * device pointer d_out.  BM_ERR_STATE unless steps done > window_start. */
int bm_reduce(bm_ensemble *e, bm_stats *d_out);

/* The whole state of one path, lossless: what Algorithm 5 of the paper loads into
 * registers before a kernel call and saves after it (position kept modulo L as in
 * "Instruction optimization", the noise countdowns of Algorithms 3 and 4, the
 * eq. (31) window snapshot).  Values are widened to FP64 / int64 on export, so a
 * record read from an ensemble and written back reproduces its state bit for bit. */
typedef struct bm_path {
    int64_t periods;         /* w: periods folded away; unwrapped position = periods L + x */
    double x;                /* folded position (within a couple of periods of [0, L))  */
    double v;                /* velocity (inertial; 0 for overdamped paths)             */
    int64_t periods_window;  /* w and x at the window start t_i of eq. (31); 0 in      */
    double x_window;         /* records read before the window start                    */
    double kick_frac;        /* jump-adapted grid: fraction of its step at which the
                                next kick falls (0 otherwise)                          */
    int64_t noise[5];        /* Poisson countdown, Poisson kicks so far, dichotomous
                                countdown, dichotomous flips so far, dichotomous state
                                (0: -Fa, 1: +Fb); 0 for absent noises                  */
    int64_t step_level;      /* step control: the next step is dt / 2^step_level       */
    int64_t steps_taken;     /* step control: steps taken (all sizes); 0 otherwise     */
} bm_path;

/* Enqueue a copy of paths [first, first + count) to device arrays (any may be
 * NULL): d_x unwrapped position w L + x (FP64), d_v velocity (FP64),
 * d_noise 5 x int64 per path (the layout of bm_path.noise), d_vp (FP64) the
 * eq. (31) per-path velocity once steps done > window_start (else it is left
 * untouched), d_state one bm_path record per path (8-byte aligned). */
int bm_read_paths(bm_ensemble *e, uint64_t first, uint64_t count,
                  double *d_x, double *d_v, int64_t *d_noise, double *d_vp, bm_path *d_state);

/* Inverse of bm_read_paths: enqueue a copy of the records d_state [count] (device,
 * 8-byte aligned) into paths [first, first + count), interpreted as their state
 * after the steps the ensemble has done (bm_ensemble_steps).  Stored in the path
 * precision (FP32 rounds; a record read from an FP32 ensemble round-trips
 * exactly).  The window snapshot is taken from the record when steps done >
 * window_start, set to the written position when steps done == window_start, and
 * left to the integration otherwise.  Only the noise fields of the model's noises
 * are used.  Values outside their ranges are clamped on the device (periods to
 * int32, countdowns to [0, 2^31 - 1], counts to [0, 2^32 - 1], state to 0/1,
 * kick_frac outside [0, 1) or NaN to 0, step_level to [0, max_halvings], steps_taken
 * to [0, 2^32 - 1]): a bad record gives a wrong path, never a fault.  Under step
 * control the records of a group of 64 paths must share step_level and steps_taken
 * (as exported); the kernel takes the group's values from its first path.  To resume exported states in a fresh workspace, open it with
 * bm_ensemble_attach (steps_done = the exporter's) and write every path; writing
 * at step 0 after bm_ensemble_create sets arbitrary initial conditions. */
int bm_write_paths(bm_ensemble *e, uint64_t first, uint64_t count, const bm_path *d_state);

/* eq. (19): add a histogram of the current folded positions y = x mod L of all
 * paths to d_counts (n_bins uint64 counters, device; the caller zeroes them):
 * bin floor(y n_bins / L) of n_bins equal bins of [0, L), computed in FP64.
 * Calling it at several times between bm_integrate calls accumulates the time
 * average of the stationary density p(y).  Non-finite positions are skipped. */
int bm_density(bm_ensemble *e, uint32_t n_bins, uint64_t *d_counts);

/* ------------------------------------------------------------------------- */
/* Batched parameter scan (Sec. 5, Execution configuration optimizations: the  */
/* stochastic dynamics solved for many parameter values in one kernel call).   */
/* ------------------------------------------------------------------------- */
typedef struct bm_scan_plan bm_scan_plan;

/* Bytes of device workspace for a scan over the n_points (models[i], runs[i])
 * pairs (multiple of 256; enough for any launch shape).  Every point must pass
 * the checks of bm_ensemble_workspace_size, have n_steps > window_start, and share
 * dyn, pot, noise and prec with the others (else BM_ERR_UNSUPPORTED). */
int bm_scan_workspace_size(const bm_model *models, const bm_run *runs, size_t n_points, size_t *bytes);

/* Plan a scan: upload the per-point constants and FP64-built forcing tables to
 * d_ws, order the work items -- chunks of 64 paths (128 with two paths per lane)
 * of every point -- longest horizon first, and capture into a hipGraph
 * [reset the work counter; one persistent work-stealing launch in which every
 * wave claims items with an atomic add and integrates them with the ensemble
 * path's code; one per-point reduction].  Point i's result goes to d_results[i]
 * (n_points bm_stats, device) and is bit-identical to bm_integrate(runs[i].n_steps)
 * + bm_reduce on an ensemble of that point.  tune: NULL = bm_tune_get_default.
 * Returns once the upload is complete (it synchronises `stream`). */
int bm_scan_plan_create(const bm_model *models, const bm_run *runs, size_t n_points, const bm_tune *tune,
                        void *d_ws, size_t ws_bytes, bm_stats *d_results, void *stream, bm_scan_plan **out);

/* Enqueue one replay of the plan's graph on its stream (results overwritten). */
int bm_scan_plan_launch(bm_scan_plan *plan);

/* Release the plan (graph and host metadata; the workspace stays the caller's). */
int bm_scan_plan_destroy(bm_scan_plan *plan);

/* One-shot scan: plan, launch, wait for the launch, release (synchronises `stream`). */
int bm_scan(const bm_model *models, const bm_run *runs, size_t n_points, const bm_tune *tune,
            void *d_ws, size_t ws_bytes, bm_stats *d_results, void *stream);

/* Autotuner: times every launch shape (paths per lane 1/2 for FP32, block 64..512,
 * occupancy-limited groups per CU) on copies of the points whose horizons are all
 * scaled by the factor that makes the longest max_steps (each at least 32 steps, none
 * lengthened; window = second half), on `stream` (one warm-up launch, then the
 * better of two timed launches per shape), and stores the fastest in *best (and as
 * the default for this (dyn, pot, noise, prec)).  *best_ms, if not NULL, receives
 * its time.  Synchronises `stream`.  The workspace must fit the scan. */
int bm_scan_autotune(const bm_model *models, const bm_run *runs, size_t n_points, uint64_t max_steps,
                     void *d_ws, size_t ws_bytes, bm_stats *d_results, void *stream,
                     bm_tune *best, float *best_ms);

/* Default launch shape per (dyn, pot, noise, prec) for this process (used when
 * a call gets no bm_tune); the built-in default is 1 path per lane, block 256,
 * groups_per_cu 0, except FP32 inertial models without Poisson or dichotomous
 * noise: 2 paths per lane, block 128. */
int bm_tune_set_default(uint32_t dyn, uint32_t pot, uint32_t noise, uint32_t prec, const bm_tune *tune);
int bm_tune_get_default(uint32_t dyn, uint32_t pot, uint32_t noise, uint32_t prec, bm_tune *out);

/* The shape installed for this key by bm_tune_set_default, bm_scan_autotune or
 * bm_tune_load: BM_OK and *out, or BM_ERR_STATE (with the built-in default in *out)
 * when none is installed. */
int bm_tune_lookup(uint32_t dyn, uint32_t pot, uint32_t noise, uint32_t prec, bm_tune *out);

/* Persistent tuning cache (the "ideal number of particles" of the paper's
 * performance section depends on the device: a tuned shape is kept per device).
 * bm_tune_save writes every installed shape, with the architecture name and CU
 * count of the device it was installed on, to the JSON file `path` (a temporary
 * file renamed over it):
 *   {"format": "libbmotor-tune", "version": 1, "entries": [
 *     {"arch": "gfx950", "cus": 256, "dyn": 1, "pot": 0, "noise": 1, "prec": 1,
 *      "paths_per_lane": 2, "block": 128, "groups_per_cu": 0}, ...]}
 * bm_tune_load installs the entries of such a file whose arch and CU count match
 * the current device (others are skipped; each entry is checked like
 * bm_tune_set_default) and writes their number to *n_loaded (may be NULL).
 * BM_ERR_INVALID_ARG for an unreadable or malformed file (nothing installed),
 * BM_ERR_DEVICE without a gfx950 device. */
int bm_tune_save(const char *path);
int bm_tune_load(const char *path, uint32_t *n_loaded);

/* ------------------------------------------------------------------------- */
/* Learned surrogate of <v>(a, omega, F, D, gamma): an ensemble of MLPs         */
/* 5 -> 256 -> 256 -> 256 -> 1 with tanh-GELU (Hendrycks & Gimpel), BF16       */
/* weights and FP32 accumulation (the 256 x 256 layers on MFMA), trained with  */
/* Adam (Kingma & Ba) on <v> values produced by bm_scan.  Plain Monte Carlo    */
/* stays the fallback: bm_surrogate_query routes the queries whose ensemble    */
/* spread exceeds a threshold.                                                  */
/*                                                                             */
/* Inputs x are rows (a, omega, F, D, gamma) of FP32, normalised inside onto   */
/* [-1, 1] over a in [0, 8], omega in [1, 10], F in [-0.5, 0.5],               */
/* log10 D in [-4, -1], gamma in [0.5, 2].                                      */
/* Parameters: d_params [n_members][BM_MLP_PARAMS] FP32, per member            */
/* W1[256][5] b1[256] W2[256][256] b2[256] W3[256][256] b3[256] W4[256] b4     */
/* (row-major [out][in]).  BF16 weight copies: d_wbf [n_members][BM_MLP_BF16]  */
/* = W1 | W2 | W3 | W4 (round to nearest even), refreshed by bm_mlp_cast and   */
/* bm_mlp_adam_step.                                                            */
/* ------------------------------------------------------------------------- */
#define BM_MLP_INPUTS 5
#define BM_MLP_HIDDEN 256
#define BM_MLP_PARAMS 133377
#define BM_MLP_BF16 132608
#define BM_MLP_MAX_MEMBERS 16

/* Device workspace bytes for a forward / query (training = 0) or a backward
 * (training = 1) over `batch` rows.  Training batches: multiple of 64, <= 65536. */
int bm_mlp_workspace_size(uint32_t n_members, uint64_t batch, uint32_t training, size_t *bytes);

/* Initial parameters: every weight and bias of a layer with fan-in f drawn from
 * U(-1/sqrt(f), 1/sqrt(f)) with Philox (key = seed, tag 4).  Enqueued on stream. */
int bm_mlp_init(uint32_t n_members, uint64_t seed, float *d_params, void *stream);

/* BF16 copies of the weights of d_params into d_wbf. */
int bm_mlp_cast(uint32_t n_members, const float *d_params, uint16_t *d_wbf, void *stream);

/* Predictions d_y [n_members][batch] (FP32) for the rows d_x [batch][5]. */
int bm_mlp_forward(uint32_t n_members, const float *d_params, const uint16_t *d_wbf, const float *d_x,
                   uint64_t batch, float *d_y, void *d_ws, size_t ws_bytes, void *stream);

/* Gradient of each member's mean squared error over its minibatch:
 * member m uses rows d_idx[m * batch + r] of d_x / d_t (d_idx NULL: rows 0..batch-1).
 * Writes d_grad [n_members][BM_MLP_PARAMS] (FP32, layout of d_params) and, if not
 * NULL, d_loss [n_members]. */
int bm_mlp_backward(uint32_t n_members, const float *d_params, const uint16_t *d_wbf, const float *d_x,
                    const float *d_t, const uint32_t *d_idx, uint64_t batch, float *d_grad, float *d_loss,
                    void *d_ws, size_t ws_bytes, void *stream);

/* One Adam step (Kingma & Ba; step counts from 1; bias-corrected moments d_m,
 * d_v, FP32) on d_params, followed by the BF16 copies in d_wbf. */
int bm_mlp_adam_step(uint32_t n_members, float *d_params, const float *d_grad, float *d_m, float *d_v,
                     uint16_t *d_wbf, uint32_t step, float lr, float beta1, float beta2, float eps, void *stream);

/* Ensemble query: d_mean / d_std [batch] = mean and population standard
 * deviation of the members' predictions; the rows with std > threshold (or a
 * non-finite std) are written to d_fallback_idx in increasing order (capacity
 * batch) and their number to *d_fallback_count (device). */
int bm_surrogate_query(uint32_t n_members, const float *d_params, const uint16_t *d_wbf, const float *d_x,
                       uint64_t batch, float threshold, float *d_mean, float *d_std, uint32_t *d_fallback_idx,
                       uint32_t *d_fallback_count, void *d_ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): bm_surrogate_query with the
 * same arguments, results and kernels, but no workspace.  The members' predictions
 * and the routing counts go to a scratch array of BM_QUERY_SCRATCH_BYTES built into
 * the library, one per GPU, held from the first call on that GPU until the process
 * ends; the call itself allocates nothing.  A query needs
 * bm_mlp_workspace_size(n_members, batch, 0) bytes of it (5 members x 10^6 rows fit);
 * larger queries get BM_ERR_WORKSPACE and must use bm_surrogate_query.  Every call
 * on one GPU uses that GPU's one array: calls that overlap on one GPU (on different
 * streams, or from different threads without ordering) race and give undefined
 * results; calls ordered on one stream are safe. */
#define BM_QUERY_SCRATCH_BYTES 33554432u
int bm_surrogate_query_noalloc(uint32_t n_members, const float *d_params, const uint16_t *d_wbf,
                               const float *d_x, uint64_t batch, float threshold, float *d_mean, float *d_std,
                               uint32_t *d_fallback_idx, uint32_t *d_fallback_count, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* BMOTOR_H */

/*
 * nbody.h -- C ABI of the MI355X (gfx950) library for the direct-summation,
 * sixth-order Hermite, block-time-step N-body method of Capuzzo-Dolcetta,
 * Spera & Punzo (arXiv:1207.2367).
 *
 * The library keeps the whole Hermite state on one GPU and runs every step
 * of a block time step there: active-set selection, prediction of all
 * sources, evaluation of acceleration, jerk, snap and potential of the
 * active particles against all sources, the split-source reduction, the
 * corrector, the higher-derivative interpolation and the new block step.
 *
 * General rules
 *   - Pointers named d_* are DEVICE pointers on the current HIP device;
 *     everything else is host memory.  The caller owns every buffer,
 *     including the workspace; the library never allocates device memory.
 *   - Vectors are row-major [n][3] FP64 (x, y, z of one particle adjacent),
 *     the layout of a contiguous torch tensor of shape [n, 3].
 *   - Work is enqueued on cfg->stream (a hipStream_t; NULL = the default
 *     stream).  Calls marked "asynchronous" return before the GPU work is
 *     done; their outputs are valid after a stream synchronization.
 *   - Units: G = 1.
 *   - A context is not thread-safe: use one context per host thread.
 *   - Return codes: NBODY_OK (0) or one of the negative codes below; the
 *     text of the last error of a context is nbody_last_error(ctx).
 */
#ifndef NBODY_H
#define NBODY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NBODY_OK 0
#define NBODY_EINVAL (-1)     /* invalid argument, size or workspace       */
#define NBODY_EDEVICE (-2)    /* a HIP runtime call failed                 */
#define NBODY_ENONFINITE (-3) /* NaN or Inf in the state or the inputs     */
#define NBODY_EDTMIN (-4)     /* a particle needs a step below dt_min      */
#define NBODY_ESTATE (-5)     /* call not valid in the context's state     */

/* Precision of the evaluation (the state, predictor, corrector, step
   criterion and energy are FP64 in every mode):
   MIXED (default): r_j - r_i, r^2, 1/r (FP32 rsqrt seed + one FP64 Newton
     step), the acceleration, jerk and potential terms and their sums in
     FP64; the snap terms in FP32 with compensated (double-single)
     accumulation.  Acceleration, jerk and potential are within 1e-6
     (relative, per particle) of an FP64 evaluation; the snap within about
     1e-6 times the condition number of its sum.  Energy conservation over
     many block steps matches the FP64 mode's (|dE/E| within 2x, measured
     on Plummer spheres of 2^15 and 2^16 bodies) for eta <= 0.8; at eta = 1
     the criterion no longer resolves close encounters in either mode and
     the two runs differ by up to ~3x.  The step criterion's
     fifth-derivative estimate amplifies the acceleration's absolute error
     by ~720/h^5, which with FP32 acceleration terms can drive steps down
     to dt_min.
   FP32PAIR: every pair term in FP32 (from the FP64 difference r_j - r_i)
     with compensated accumulation -- fastest; safe only where steps stay
     near their natural length.
   FP64: every operation in FP64 (comparison path; 1/r from the FP32
     rsqrt seed refined to FP64 accuracy by one third-order step).       */
#define NBODY_PREC_MIXED 0
#define NBODY_PREC_FP64 1
#define NBODY_PREC_FP32PAIR 2

typedef struct nbody_config {
    double eta;      /* accuracy parameter of the step criterion, > 0     */
    double eta_init; /* first step: eta_init A(1)/A(2) (p = 4), see init   */
    double dt_min;   /* smallest block step, a power of two               */
    double dt_max;   /* largest block step, a power of two >= dt_min      */
    int32_t precision;  /* NBODY_PREC_MIXED, _FP64 or _FP32PAIR           */
    int32_t n_clusters; /* 0 or 1: one system; > 1: independent clusters  */
    /* host array [n_clusters + 1], ascending, 0 ... n: particles
       [off[c], off[c+1]) form cluster c; pairs across clusters do not
       interact and each cluster has its own block times.  NULL when
       n_clusters <= 1.  Copied by nbody_init.                            */
    const int64_t *cluster_offsets;
    void *stream;       /* hipStream_t                                    */
    int32_t validate;   /* nonzero: nbody_force checks its index list     */
    /* nonzero: nbody_init only copies the inputs (acceleration and higher
       derivatives zero, t = 0, dt = dt_max); the caller then provides the
       Hermite state with nbody_set_state.                                */
    int32_t skip_startup;
} nbody_config;

typedef struct nbody_ctx nbody_ctx;

typedef struct nbody_step_stats {
    int64_t block_steps;  /* global block steps taken                      */
    int64_t active_total; /* sum of N_act over steps (all clusters)       */
    double interactions;  /* sum over steps and clusters of N_c * N_act,c */
    /* hist[b]: number of (step, cluster) blocks with 2^b <= N_act < 2^(b+1) */
    int64_t hist[40];
} nbody_step_stats;

/* Fill *cfg with the defaults: eta 0.45, eta_init 0.1, dt_min 2^-25,
   dt_max 1/16, mixed precision, one system, default stream.            */
void nbody_default_config(nbody_config *cfg);

/* Device bytes that nbody_init needs for n particles under cfg
   (state, source records, split-source partials, active lists and
   scratch).  Returns 0 if n <= 0 or cfg is invalid.                    */
size_t nbody_workspace_bytes(int64_t n, const nbody_config *cfg);

/* Create a context for n particles with masses d_mass[n], positions
   d_pos[n][3] and velocities d_vel[n][3] (copied; the caller keeps them)
   and softening eps >= 0 (the softened potential of paper Sect. 2,
   Eq. softpot).  d_workspace must hold nbody_workspace_bytes(n, cfg)
   bytes, 256-byte aligned, and stay alive until nbody_free.
   Initialization (the paper does not describe it), in FP64 whatever the
   precision: acceleration and jerk of every particle, then a second
   evaluation with those as the sources' values for the snap and the
   crackle (the third derivative, by the same pairwise differentiation);
   t_i = 0; first step = the paper's generalized criterion (Eqs. indtstp,
   As) at the order these derivatives allow, p = 4: eta_init A(1)/A(2),
   A(2) = sqrt(|da||a(3)| + |d2a|^2), rounded down to a power of two and
   clamped to [dt_min, dt_max].  Synchronizes.
   Errors: EINVAL (n <= 0, eps < 0 or not finite, eta or eta_init <= 0,
   dt bounds not powers of two or dt_min > dt_max, bad cluster offsets,
   NULL pointer, workspace too small or misaligned), EDEVICE,
   ENONFINITE (NaN/Inf in the inputs), EDTMIN.                           */
int nbody_init(nbody_ctx **out, int64_t n, const double *d_mass,
               const double *d_pos, const double *d_vel, double eps,
               const nbody_config *cfg, void *d_workspace, size_t ws_bytes);

/* Release the host-side context (the workspace stays with the caller);
   waits for the work queued on the context's stream first.             */
void nbody_free(nbody_ctx *ctx);

/* Evaluation step alone (paper Sect. 3, item 2, with softening): for the
   n_act particles d_idx[0..n_act) (strictly ascending, in [0, n)) the
   acceleration, jerk and snap d_acc/d_jrk/d_snp[n_act][3] and the
   potential d_pot[n_act] (negative, -sum m_j / sqrt(r^2 + eps^2)) from
   all sources j != i of the particle's cluster, using the current state
   of every particle as the source values (positions, velocities and
   accelerations as stored; at a synchronized time this is the predicted
   state).  Any output pointer may be NULL (d_pot) -- acc, jrk and snp are
   required.  n_act = 0 does nothing and returns NBODY_OK.  Asynchronous.
   Does not change the state.
   Errors: EINVAL (n_act < 0 or > n, NULL pointer; with cfg->validate the
   index list is checked on the device, the call synchronizes, and an
   out-of-range or non-ascending list gives EINVAL; without it an index
   outside [0, n) is skipped -- its outputs are not written -- and
   reported as EINVAL by the next call that synchronizes), EDEVICE.     */
int nbody_force(nbody_ctx *ctx, int64_t n_act, const int32_t *d_idx,
                double *d_acc, double *d_jrk, double *d_snp, double *d_pot);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the
   evaluation of nbody_force without a context or workspace.  Sources are
   the caller's arrays d_mass[n], d_pos/d_vel/d_acc[n][3] (row-major FP64,
   one system, softening eps >= 0, evaluation precision as in
   nbody_config); outputs, index list and NULL rules as for nbody_force
   (d_idx strictly ascending in [0, n), not checked).  The source records
   and split-source partials live in a fixed 64 MiB device array inside the
   library, one per GPU, kept until the process ends; the call allocates
   nothing.  Limit: n * R + 80 * n_act plus about 1 KiB within 64 MiB,
   R = 68 (mixed), 56 (FP32 pair), 80 (FP64) bytes -- e.g. up to
   n = n_act = 2^18 in every precision.  Asynchronous on the stream
   (a hipStream_t, NULL = default).  Calls that overlap on one GPU share
   that array and race: order them on one stream.
   Errors: EINVAL (sizes beyond the limit, n_act > n, NULL pointer, bad
   eps or precision), EDEVICE.                                            */
int nbody_force_noalloc(int64_t n, const double *d_mass, const double *d_pos,
                        const double *d_vel, const double *d_acc, double eps,
                        int32_t precision, int64_t n_act, const int32_t *d_idx,
                        double *d_acc_out, double *d_jrk_out, double *d_snp_out,
                        double *d_pot_out, void *stream);

/* Prediction step alone (paper Sect. 3, item 1): Taylor series of every
   particle's position, velocity and acceleration from its own time t_i
   to time t (h = t - t_i), written to d_pos/d_vel/d_acc[n][3] in FP64.
   The state is not changed.  Asynchronous.  Errors: EINVAL, EDEVICE.   */
int nbody_predict(nbody_ctx *ctx, double t, double *d_pos, double *d_vel,
                  double *d_acc);

/* Active-set selection alone (paper Sect. 5.4, Table 1, section 1): for
   each cluster not yet at t_target, the block time min_i (t_i + dt_i) and
   the particles due then, written as ascending indices to d_idx (room for
   n entries), cluster after cluster.  *n_act gets the total count and
   *t_next the earliest block time (+inf if every cluster has reached
   t_target).  Synchronizes.  Errors: EINVAL, EDEVICE.                  */
int nbody_schedule(nbody_ctx *ctx, double t_target, int32_t *d_idx,
                   int64_t *n_act, double *t_next);

/* Corrector alone (paper Sect. 3, item 3) followed by the interpolation
   of crackle, pop and the fifth derivative at the end of the step and
   the new block step (generalized Aarseth criterion, Eqs. indtstp/As with
   p = 6, power-of-two rules): for the listed particles (ascending, the
   whole active block of their cluster) with new acceleration, jerk and
   snap d_acc/d_jrk/d_snp[n_act][3] evaluated at their block time
   t_i + dt_i.  t_target caps the new steps.  Synchronizes.
   Errors: EINVAL (also an index outside [0, n), which is skipped; with
   cfg->validate the list is checked for range and order before any
   change), EDEVICE, EDTMIN, ENONFINITE.                                 */
int nbody_correct(nbody_ctx *ctx, int64_t n_act, const int32_t *d_idx,
                  double t_target, const double *d_acc, const double *d_jrk,
                  const double *d_snp);

/* One block time step of every cluster not yet at t_target (schedule,
   predict, evaluate, reduce, correct, new steps; paper Sect. 3 and Table
   1).  *n_act gets the number of particles advanced and *t_block the
   earliest block time of the step.  Waits for the scheduler's totals
   (the host sizes the evaluation from them); the evaluation and the
   correction are then queued on the stream, so later calls on the same
   stream see the completed step.
   Errors: EINVAL (t_target not a multiple of dt_min or < 0), EDEVICE,
   EDTMIN, ENONFINITE.                                                   */
int nbody_block_step(nbody_ctx *ctx, double t_target, int64_t *n_act,
                     double *t_block);

/* Advance every particle of every cluster to t_target (a multiple of
   dt_min, not behind any particle).  Steps that would pass t_target are
   halved.  stats may be NULL.  Synchronizes.
   Errors: EINVAL, EDEVICE, EDTMIN, ENONFINITE.                          */
int nbody_step(nbody_ctx *ctx, double t_target, nbody_step_stats *stats);

/* Copy the Hermite state out (checkpoint) or in (resume / test set-up):
   positions, velocities, acceleration, jerk, snap, crackle [n][3], own
   times t[n] and steps dt[n].  Any pointer may be NULL (skipped).
   set_state requires each t_i to be a multiple of dt_i and dt_i a power
   of two in [dt_min, dt_max] (not checked on the device).  Asynchronous.
   Errors: EINVAL, EDEVICE.                                              */
int nbody_get_state(nbody_ctx *ctx, double *d_pos, double *d_vel,
                    double *d_acc, double *d_jrk, double *d_snp,
                    double *d_crk, double *d_t, double *d_dt);
int nbody_set_state(nbody_ctx *ctx, const double *d_pos, const double *d_vel,
                    const double *d_acc, const double *d_jrk,
                    const double *d_snp, const double *d_crk,
                    const double *d_t, const double *d_dt);

/* Energy and angular momentum in FP64 (paper Sect. 5.1): kinetic energy,
   softened potential energy -sum_{i<j} m_i m_j / sqrt(r^2 + eps^2) (pairs
   within a cluster), and L = sum m r x v, summed over all clusters, from
   the stored state.  Requires every particle of a cluster to be at one
   time (clusters may differ).  Synchronizes.
   Errors: ESTATE (particles of a cluster at different times; nothing is
   computed), EDEVICE.                                                   */
int nbody_energy(nbody_ctx *ctx, double *ekin, double *epot, double L[3]);

/* Measure launch shapes of the force kernel for active-set sizes
   1, 2, 4, ... up to the largest cluster -- with one system, that many
   particles spread over it; with clusters, up to that many particles of
   every cluster, as in a batched block step -- (sizes whose single launch
   would exceed ~2^35 pairs keep the launch rule), and keep the fastest for
   each size range in the context (the autotuner).  Without it a fixed rule picks the
   shape.  max_ms bounds the time spent per size.  Uses the stored state
   as sources; does not change it.  Synchronizes.  Errors: EDEVICE.      */
int nbody_autotune(nbody_ctx *ctx, double max_ms);

/* Force kernel launch shape: lanes per active particle (1..64, a power of
   two), waves per workgroup (1, 2 or 4), split-source factor (>= 1) and
   active particles per group of lanes_per_i lanes (1 or 2, 2 only with
   lanes_per_i <= 4: each source read from LDS then serves two pairs; 0
   means 1).  nbody_set_launch pins a shape for every later force
   evaluation (0 in lanes_per_i, waves or split restores automatic choice;
   EINVAL for a shape outside these ranges); nbody_get_launch reports the
   shape that automatic choice takes for n_act active particles.       */
typedef struct nbody_launch {
    int32_t lanes_per_i;
    int32_t waves;
    int32_t split;
    int32_t i_per_lane;
} nbody_launch;
int nbody_set_launch(nbody_ctx *ctx, const nbody_launch *shape);
int nbody_get_launch(nbody_ctx *ctx, int64_t n_act, nbody_launch *shape);

/* The autotuner's table, so that a measured table can be stored by the
   caller and reused (the same shapes, hence the same bits, in every run):
   entry b is the shape for active sets 2^b <= N_act < 2^(b+1), all-zero
   where no shape was measured (the launch rule applies).
   nbody_get_tuning copies up to max entries and returns the number of
   entries (0 before nbody_autotune), or EINVAL.  nbody_set_tuning replaces
   the table with count (<= 40) entries; each must be all-zero or a valid
   shape (as for nbody_set_launch), else EINVAL and the table is kept.  */
int nbody_get_tuning(nbody_ctx *ctx, nbody_launch *table, int32_t max);
int nbody_set_tuning(nbody_ctx *ctx, const nbody_launch *table, int32_t count);

/* Device-resident block steps (the small-block regime of paper Sect. 3,
   last part, where selecting the active set and reducing the split
   partials cost as much as the evaluation).  For a context with one
   system, no pinned launch shape and profiling off, nbody_step runs its
   block steps inside one cooperative launch (64 workgroups, three grid
   barriers per block step: schedule, prediction, evaluation with split
   sources, fixed-order reduction and corrector) for as long as every
   block has at most max_active active particles; a larger block goes
   through the host-sized path and the loop resumes after it.  Results
   equal the host-sized path's to the rounding of the split sums (a
   different launch shape).  max_active < 0 (the default): automatic, i.e.
   on for systems of up to 4096 bodies with blocks of up to ~2^21 pairs
   (at least 4 particles), off for larger systems, where the host-sized
   path is faster; 0: off; > 0: on with that limit (capped by the
   split-partials capacity).  If the runtime refuses the cooperative
   launch, the context keeps to the host-sized path.  A grid barrier that
   waits for more than about two seconds ends the launch with
   NBODY_EDEVICE instead of hanging.  Returns NBODY_EINVAL for a NULL ctx. */
int nbody_set_step_loop(nbody_ctx *ctx, int64_t max_active);

/* How nbody_step finds the next block of a single system on the host-sized
   path (the block-step scheme of paper Sect. 2 and the active-set selection
   of Table 1, section 1).  mode 0 (the default): from per-level counts --
   the number of particles on each step dt_max 2^-k, kept up to date by the
   corrector -- whenever the state allows it (every step a power of two in
   [dt_min, dt_max], every particle at a multiple of its step and short of
   its next one, which the integrator keeps; checked once per nbody_step
   call): the next block time is the earliest next multiple of an occupied
   level's step, its particles those of the levels whose step divides it, so
   no sweep over all particles is needed; the active list is then filled in
   chunk order of completion (the results do not depend on it).  mode 1: a
   sweep of every particle's next time per block step (always used for
   several clusters, by the device-resident loops and by nbody_schedule and
   nbody_block_step).  Both give the same blocks.  Returns NBODY_EINVAL for
   a NULL ctx or another mode. */
int nbody_set_schedule(nbody_ctx *ctx, int mode);

/* GPU time per phase of the block step, measured with HIP events on the
   context's stream while profiling is on (phases follow the paper's
   Table 1: 0 active-set selection, 1 prediction, 2 evaluation (force
   kernel), 3 split-source reduction (of nbody_force; a block step fuses
   it into 4), 4 correction and new steps, 5 energy; a block step times
   the compaction of its active list with the prediction, which shares its
   launch).  While profiling is on, nbody_step does not use the
   device-resident loop (its phases share one launch).
   nbody_profile(ctx, enable, out): enable = 1 starts (and clears), 0 stops;
   with out != NULL the totals so far are written (synchronizes).  The
   force-kernel launches are also logged one by one: nbody_profile_force_log
   copies up to max entries of (active particles, pairs, milliseconds) and
   returns the number of entries logged.                                 */
#define NBODY_NPHASE 6
typedef struct nbody_profile_times {
    double ms[NBODY_NPHASE];
    int64_t launches[NBODY_NPHASE];
    double pairs; /* interactions evaluated by the force kernel */
} nbody_profile_times;
int nbody_profile(nbody_ctx *ctx, int enable, nbody_profile_times *out);
int64_t nbody_profile_force_log(nbody_ctx *ctx, int64_t max, int64_t *n_act,
                                double *pairs, double *ms);

/* Static text of a return code, and the last error message of a context. */
const char *nbody_strerror(int code);
const char *nbody_last_error(const nbody_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* NBODY_H */

/*
 * nbody.h -- C ABI of the MI355X direct N-body force library.
 *
 * The library evaluates, by direct summation on the GPU, the Plummer-softened
 * gravitational acceleration, its time derivative (jerk) and the potential of
 * a set of i-particles due to a set of j-particles (Eq. 1 of the paper, with
 * the softening of Section 3.3 and the jerk and potential of Section 3), and
 * drives a fourth-order Hermite predictor-corrector with block time steps
 * (Section 3 and 3.1) whose prediction, correction and block selection also
 * run on the GPU.
 *
 * Conventions (apply to every function):
 *  - Every function returns an int status: NBODY_OK (0) or a negative
 *    NBODY_ERR_* code.  nbody_last_error(ctx) gives a human-readable detail
 *    for the last failing call on that context.  The library never aborts
 *    and never prints.
 *  - Array arguments are DEVICE pointers unless stated otherwise: contiguous
 *    float64 structure-of-arrays rows (one pointer per component), 8-byte
 *    aligned, owned by the caller.  The library never frees or keeps them
 *    after a call returns.
 *  - Work is enqueued asynchronously on the given HIP stream (NULL = the
 *    default stream); outputs are ready when the stream reaches that point.
 *    Argument errors are reported synchronously, before anything is
 *    launched; a device fault surfaces at a later call or at nbody_sync.
 *  - Scratch memory (packed particle copies, split partial sums, block
 *    lists) belongs to the context, grows on demand and is kept until
 *    nbody_destroy; nbody_reserve pre-sizes it outside timed regions.
 *  - A context is not thread-safe: use one per host thread.  Two calls on
 *    one context that overlap in time on different streams race on the
 *    context's scratch memory.
 *  - Particle counts are int64 arguments but must not exceed 2^31 - 1
 *    (kernels index with int32).
 *  - G and eps are float64; eps must be finite and >= 0.  eps == 0 selects
 *    the unsoftened form, in which a pair at zero separation contributes
 *    nothing (the zero-softening check of Section 3.3).
 *  - Outputs are overwritten, never accumulated into.
 */
#ifndef NBODY_H
#define NBODY_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NBODY_ABI_VERSION 1

enum {
    NBODY_OK = 0,
    NBODY_ERR_ARG = -1,          /* invalid argument (NULL, size, eps, alignment) */
    NBODY_ERR_NOMEM = -2,        /* device or host allocation failed */
    NBODY_ERR_DEVICE = -3,       /* HIP runtime error (launch, copy, fault) */
    NBODY_ERR_UNSUPPORTED = -4,  /* valid request the library does not serve */
    NBODY_ERR_STATE = -5         /* object used out of order */
};

/* Arithmetic of the pairwise loop.
 *  NBODY_PREC_FP32: positions and velocities rounded to float32 (the 7
 *    input floats per particle of Section 3.1), float32 pair arithmetic,
 *    float32 accumulation over all j.
 *  NBODY_PREC_DS_COMP: positions as double-single (hi = fl32(x),
 *    lo = fl32(x - hi)); the relative coordinate is formed as
 *    (x_j,hi - x_i,hi) + (x_j,lo - x_i,lo); float32 pair arithmetic; float32
 *    partial sums per j-tile folded into a two-sum (hi, lo) accumulator. */
typedef enum { NBODY_PREC_FP32 = 0, NBODY_PREC_DS_COMP = 1 } nbody_prec;

typedef struct nbody_ctx nbody_ctx;

/* Particle source: device float64 rows of length n.  m may be NULL where a
 * function says masses are unused (the i side of nbody_force). */
typedef struct {
    const double *x, *y, *z, *vx, *vy, *vz, *m;
} nbody_src;

/* Force output: device float64 rows of length n_i. */
typedef struct {
    double *ax, *ay, *az, *jx, *jy, *jz, *pot;
} nbody_out;

/* Launch shape of the pairwise kernel (also the autotuner's search space).
 *  tile_j: j-particles per tile (staged in LDS when jsrc = 0; the interval
 *          between compensated folds when jsrc = 1): 64, 128, 256, and 16
 *          or 32 with ipt 1 and wg 64 or 128 (short sweeps for small j
 *          sets); jsrc = 1: 128.
 *  ipt:    i-particles held in registers per lane, one of 1, 2, 4.
 *  wg:     work-group size in lanes: 128 or 256 (jsrc = 1: 64 or 256;
 *          16- and 32-record tiles: 64 or 128).
 *  split:  number of j-ranges the j set is cut into (>= 1; 0 = choose
 *          from the shape and the sizes: enough work-groups to fill the
 *          device, and for long evaluations at least 32768 work-groups,
 *          each range keeping at least 64 tiles); partial sums are reduced
 *          in float64 in fixed order (Section 3.2).
 *  jsrc:   0 = j records staged tile by tile in LDS (Section 3.1, Fig. 1);
 *          1 = j records read by wave-uniform loads through the scalar data
 *          cache (no LDS, no barrier).
 *  unroll: unroll depth of the j loop (0 = the default 4).
 *  waves:  waves per SIMD requested from the compiler, a register cap
 *          (0 = none).
 * Only the shapes compiled into the library exist; nbody_set_tile rejects
 * others and nbody_autotune visits all of them. */
typedef struct {
    int tile_j, ipt, wg, split, jsrc, unroll, waves;
} nbody_tile;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device` (the caller's current device is
 * restored).  tune_cache_path: JSON file the autotuner reads and writes, or
 * NULL for $NBODY_TUNE_CACHE (unset: no persistent cache).  On failure *ctx
 * is set to NULL and the code is returned (details cannot be queried).
 * Environment read here:
 *  NBODY_TRACE=<path>  append one JSON line per Hermite step of this
 *    context's integrators to <path>: {"mode": "block" | "shared", "step",
 *    "t_ticks", "t", "n_act", "shape": "small" | "large" (block steps: the
 *    launch shape the device plan chose; shared steps: "direct"), "groups"
 *    (i-groups of the block step), "ranges" (j-ranges)}.  Block steps are
 *    recorded on the device and written at each chunk's plan readback (no
 *    extra synchronisation per step).  A path that cannot be opened turns
 *    tracing off.
 *  NBODY_FORCE_TILE=tile_j,ipt,wg[,split[,jsrc[,unroll[,waves]]]]  pin the
 *    launch shape of the pairwise kernel (nbody_tile fields; omitted ones
 *    0), as nbody_set_tile does, for each precision that has the shape
 *    compiled; NBODY_ERR_ARG from nbody_create when no precision has it.
 *  NBODY_DEBUG_FAIL_ALLOC=<k>  the k-th device allocation of the context
 *    fails with NBODY_ERR_NOMEM (failure-path testing).
 *  NBODY_DEBUG_SELF_CHECK=1  see nbody_force. */
int nbody_create(nbody_ctx **ctx, int device, const char *tune_cache_path);

/* Release the context and all of its device memory.  NULL is accepted. */
int nbody_destroy(nbody_ctx *ctx);

/* Pre-size scratch for up to max_i i-particles against max_j j-particles. */
int nbody_reserve(nbody_ctx *ctx, int64_t max_i, int64_t max_j);

/* Wait for all work on `stream`; reports deferred device errors. */
int nbody_sync(nbody_ctx *ctx, hipStream_t stream);

/* Text of the last error on this context ("" if none).  Owned by ctx. */
const char *nbody_last_error(const nbody_ctx *ctx);

/* NBODY_ABI_VERSION of the loaded library. */
int nbody_abi_version(void);

/* Kernel timing.  While enabled, every launch of the pairwise kernel made
 * through this context is bracketed by two HIP events recorded on the
 * launch stream.  nbody_kernel_time waits for the recorded events, returns
 * the summed kernel time in milliseconds and the number of launches (HOST
 * outputs) and starts a new tally.  The events stay owned by the context. */
int nbody_kernel_timing(nbody_ctx *ctx, int enable);
int nbody_kernel_time(nbody_ctx *ctx, double *total_ms, int64_t *launches);

/* Force the launch shape used for `prec` (a shape that exists, see
 * nbody_tile; split may be 0), or clear the override when t is NULL. */
int nbody_set_tile(nbody_ctx *ctx, nbody_prec prec, const nbody_tile *t);

/* The launch shape the next nbody_force call would use for this shape. */
int nbody_get_tile(nbody_ctx *ctx, nbody_prec prec, int64_t n_i, int64_t n_j, nbody_tile *t);

/* Autotuner (the number of threads per bundle is the tuning knob the paper
 * leaves to the user, Section 5): time every launch shape tile_j x ipt x wg
 * (split chosen from the shape) on the given inputs, `reps` timed
 * evaluations each after one warm-up, keep the fastest for this precision
 * and shape bucket (floor log2 of n_i and n_j), and write the cache file if
 * the context has one.  `out` receives the last evaluation.  *best and
 * *best_ms (HOST, may be NULL) report the choice and its time per
 * evaluation in milliseconds.  Synchronises `stream`. */
int nbody_autotune(nbody_ctx *ctx, hipStream_t stream, nbody_prec prec, double G, double eps,
                   int64_t n_i, nbody_src I, int64_t n_j, nbody_src J, nbody_out out, int reps,
                   nbody_tile *best, double *best_ms);

/* ---- force (Eq. 1, Section 3) -------------------------------------------- */

/* Acceleration, jerk and potential of n_i i-particles due to n_j
 * j-particles (Eq. 1 with Plummer softening, Section 3.3; jerk and
 * potential, Section 3):
 *   a_i    =  G sum_j m_j r / s^(3/2)
 *   jerk_i =  G sum_j m_j (u / s^(3/2) - 3 (r.u) r / s^(5/2))
 *   pot_i  = -G sum_j m_j / s^(1/2)
 * with r = x_j - x_i, u = v_j - v_i, s = |r|^2 + eps^2.
 * i_self: device int32[n_i] giving, for each i, the j index of that same
 * particle (excluded from the sums) or -1; NULL excludes nothing.  The
 * kernel sweeps every j (Section 3.1 counts all N^2 pairs); in the one or
 * two j-tiles that hold j = i_self[i] the pair is given zero mass, so it
 * contributes nothing to a, jerk or pot and the large self potential
 * m_i/eps never enters a float32 partial sum.  An i_self value outside
 * [0, n_j) excludes nothing.  With the environment variable
 * NBODY_DEBUG_SELF_CHECK=1 set when the context is created, the call also
 * checks that each i row equals the j row i_self names (the same particle)
 * and that every i_self < n_j, synchronising the stream, and returns
 * NBODY_ERR_ARG when one does not.
 * I.m is unused.  Returns NBODY_ERR_ARG for NULL rows, n_i < 0, n_j < 0,
 * counts above 2^31 - 1, non-finite G or eps, eps < 0. */
int nbody_force(nbody_ctx *ctx, hipStream_t stream, nbody_prec prec, double G, double eps,
                int64_t n_i, nbody_src I, const int32_t *i_self,
                int64_t n_j, nbody_src J, nbody_out out);

/* nbody_force without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, outputs and errors as nbody_force.
 * Its packed particle records and split partial sums live in one 64 MiB
 * array of device memory per GPU that the library holds from its first
 * context on that device until the process ends; the call allocates and
 * frees nothing (no hipMalloc, hipFree, events or library allocations).
 * Limit: the packed records, 48 bytes per particle (DS) or 32 (FP32), for
 * the j set plus the i set (the i set only when it is not the j set itself)
 * must fit in 64 MiB, else NBODY_ERR_ARG with the sizes in
 * nbody_last_error.  When the split partial sums (56 bytes per i and
 * j-range) of the launch shape nbody_force would use do not fit in the
 * rest, fewer j-ranges are used; the results then differ from
 * nbody_force's in rounding only.  Every call on one GPU uses that GPU's
 * array, across all contexts: two calls that overlap in time on one GPU
 * (different streams, threads or contexts) race and give wrong results.
 * Nothing in the array needs to start at zero.  NBODY_DEBUG_SELF_CHECK and
 * kernel timing do not apply to this call. */
int nbody_force_noalloc(nbody_ctx *ctx, hipStream_t stream, nbody_prec prec, double G, double eps,
                        int64_t n_i, nbody_src I, const int32_t *i_self,
                        int64_t n_j, nbody_src J, nbody_out out);

/* Force-only evaluation: acceleration and potential as in nbody_force,
 * without the jerk.  Section 4 runs the library under a treecode, which
 * integrates with the acceleration alone, with the jerk and nearest-neighbour
 * work switched off (38 instead of 60 conventional flops per interaction,
 * Table 3).  The velocity rows of I and J are not read and may be NULL;
 * out.jx, out.jy, out.jz are not written and may be NULL.  Otherwise as
 * nbody_force (arguments, self handling, errors). */
int nbody_force_acc(nbody_ctx *ctx, hipStream_t stream, nbody_prec prec, double G, double eps,
                    int64_t n_i, nbody_src I, const int32_t *i_self,
                    int64_t n_j, nbody_src J, nbody_out out);

/* nbody_force plus the nearest neighbour of every i (Section 3.3: the GRAPE
 * hardware reports it alongside force, jerk and potential, and the GPU finds
 * it with one distance comparison per pair in the force loop).
 * nn: device int32[n_i], required: the j index with the smallest unsoftened
 * squared distance |x_j - x_i|^2 among j != i_self[i]; the lowest such j
 * when several are equally close; -1 if there is no candidate.
 * nn_r2: device double[n_i] or NULL: that squared distance as the kernel
 * computed it (float32, from the relative coordinate of the chosen
 * precision), +inf where nn is -1.  Distances are compared in float32, so
 * two j whose distances differ by less than float32 rounding may be taken
 * in either order.  Errors as nbody_force, plus NBODY_ERR_ARG for
 * nn == NULL with n_i > 0. */
int nbody_force_nn(nbody_ctx *ctx, hipStream_t stream, nbody_prec prec, double G, double eps,
                   int64_t n_i, nbody_src I, const int32_t *i_self,
                   int64_t n_j, nbody_src J, nbody_out out, int32_t *nn, double *nn_r2);

/* Shared-step kick-drift-kick leapfrog of n particles on the force-only
 * evaluation (the acceleration-only integration of Section 4):
 *   v += a dt/2;  x += v dt;  a = a(x);  v += a dt/2   (nsteps times),
 * every particle acting on every other, self excluded.
 * x, v, acc: device double[3][n] (rows x, y, z), updated in place; acc must
 * hold a(x) on entry when have_acc != 0, else it is computed first; on
 * return it holds a(x) at the end, so runs chain without a re-evaluation.
 * m: device double[n].  pot: device double[n] or NULL: the potential at the
 * end.  Enqueued on `stream` without host synchronisation.  Returns
 * NBODY_ERR_ARG for NULL x, v, m or acc with n > 0, misaligned rows,
 * nsteps < 0, non-finite dt, and as nbody_force for G and eps. */
int nbody_leapfrog(nbody_ctx *ctx, hipStream_t stream, nbody_prec prec, double G, double eps,
                   double dt, int nsteps, int64_t n, double *x, double *v, const double *m,
                   double *acc, double *pot, int have_acc);

/* ---- adjoint of the force ------------------------------------------------- */

/* Vector-Jacobian product of nbody_force (the derivative of the sums of
 * Eq. 1 with Plummer softening, jerk and potential): for output cotangents
 * ga (acceleration), gj (jerk), gp (potential) of the i-particles it returns
 *   gxi, gvi = dL/dx_i, dL/dv_i   and   gxj, gvj, gmj = dL/dx_j, dL/dv_j, dL/dm_j
 * of L = sum_i ga_i.a_i + gj_i.jerk_i + gp_i pot_i.  Per pair, with the
 * notation of nbody_force and C = s^-5/2:
 *   g_r = G m_j [s^-3/2 ga - P r - 3C (gj.r) u - 3C (r.u) gj],
 *   P   = 3C (ga.r + gj.u - 5 (r.u)(gj.r)/s) - gp s^-3/2,
 *   g_u = G m_j [s^-3/2 gj - 3C (gj.r) r],
 * x_j gets +g_r, x_i gets -g_r (v likewise), and
 *   dL/dm_j += G [s^-3/2 (ga.r + gj.u) - 3C (r.u)(gj.r) - gp s^-1/2].
 * Self pairs (i_self) and, with eps = 0, pairs at zero separation are
 * excluded as in nbody_force.
 * Layout: ga, gj, gxi, gvi are single device pointers to float64 [3][n_i]
 * (x row, y row, z row); gxj, gvj are [3][n_j]; gp is [n_i], gmj [n_j].
 * gj and gp may be NULL (zero cotangents); any output may be NULL (not
 * computed).  The i side and the j side are two passes (lane = i, then
 * lane = j); both gather, no atomics, so results are run-to-run identical.
 * Errors as nbody_force, plus NBODY_ERR_ARG for ga == NULL with n_i > 0. */
int nbody_force_vjp(nbody_ctx *ctx, hipStream_t stream, nbody_prec prec, double G, double eps,
                    int64_t n_i, nbody_src I, const int32_t *i_self, int64_t n_j, nbody_src J,
                    const double *ga, const double *gj, const double *gp,
                    double *gxi, double *gvi, double *gxj, double *gvj, double *gmj);

/* The same adjoint for one self-gravitating set (every particle is both an
 * i and a j, self excluded): returns the total gx = dL/dx, gv = dL/dv,
 * gm = dL/dm of each particle in ONE fused pass in which a lane evaluates
 * each pair once and applies both its own (i) and its partner's (j) half.
 * Layout as nbody_force_vjp with n_i = n_j = n ([3][n] rows; gp, gm [n]). */
int nbody_force_vjp_self(nbody_ctx *ctx, hipStream_t stream, nbody_prec prec, double G, double eps,
                         int64_t n, nbody_src P, const double *ga, const double *gj, const double *gp,
                         double *gx, double *gv, double *gm);

/* ---- differentiable shared-step integration ---------------------------------- */

/* Fourth-order Hermite integration of one self-gravitating set with one
 * shared step dt for nsteps steps (Section 3, Makino & Aarseth 1992 scheme;
 * every particle active every step, self excluded):
 *   x_p = x + v dt + a dt^2/2 + j dt^3/6,  v_p = v + a dt + j dt^2/2,
 *   (a1, j1) = force at (x_p, v_p),
 *   a2 = (-6 (a - a1) - dt (4 j + 2 j1)) / dt^2,  a3 = (12 (a - a1) + 6 dt (j + j1)) / dt^3,
 *   x = x_p + a2 dt^4/24 + a3 dt^5/120,  v = v_p + a2 dt^3/6 + a3 dt^4/24,  a = a1, j = j1,
 * starting from (x0, v0) = P0 with a, j evaluated there.  x_out, v_out:
 * device float64 [3][n].  ckpt: device buffer of nbody_shared_ckpt_bytes
 * bytes (or NULL) that receives (x, v, a, j) before every ckpt_every-th
 * step, for nbody_shared_adjoint.  n is at most 715827882 ((2^31-1)/3: the
 * [3][n] rows are indexed as one int32 range); NBODY_ERR_ARG beyond, and
 * nbody_shared_ckpt_bytes returns -1. */
int64_t nbody_shared_ckpt_bytes(int64_t n, int nsteps, int ckpt_every);
int nbody_shared_run(nbody_ctx *ctx, hipStream_t stream, nbody_prec prec, double G, double eps,
                     double dt, int nsteps, int64_t n, nbody_src P0, double *x_out, double *v_out,
                     double *ckpt, int ckpt_every);

/* Gradient of L = <gx_end, x(T)> + <gv_end, v(T)> of the run above with
 * respect to x0, v0 and the masses.  Each checkpoint segment is recomputed
 * forward (deterministically, so the predicted states match the first run
 * bit for bit) and then differentiated step by step backwards:
 * corrector adjoint (float64), the fused force adjoint of
 * nbody_force_vjp_self with the acceleration and jerk cotangents, then the
 * predictor adjoint (float64); finally the adjoint of the initial force
 * evaluation.  gv_end may be NULL (zero).  gx0, gv0: [3][n]; gm: [n].
 * Arguments must match the nbody_shared_run call that filled ckpt. */
int nbody_shared_adjoint(nbody_ctx *ctx, hipStream_t stream, nbody_prec prec, double G, double eps,
                         double dt, int nsteps, int64_t n, nbody_src P0, const double *ckpt,
                         int ckpt_every, const double *gx_end, const double *gv_end,
                         double *gx0, double *gv0, double *gm);

/* ---- many independent clusters ------------------------------------------------- */

/* Acceleration, jerk and potential (as nbody_force) of n_clusters
 * independent clusters in ONE persistent launch.  Cluster c holds the
 * particles [offsets[c], offsets[c+1]) of the concatenated rows P (device
 * rows of length n_total); every particle of a cluster is both an i and a j
 * (self excluded), there are no cross-cluster forces, and cluster c uses
 * softening eps[c].  offsets (int64 [n_clusters+1]) and eps (float64
 * [n_clusters]) are DEVICE arrays; ranges are clamped to [0, n_total], and
 * particles outside every cluster get zero output.  A one-work-group plan
 * kernel orders the clusters by size (largest first) and cuts them into
 * (cluster, i-block) work items; the persistent kernel's work-groups take
 * items from a device counter until none is left, each running the same
 * tile loop as nbody_force.  With the same launch shape forced
 * (nbody_set_tile, split 1) a cluster's rows equal nbody_force on that
 * cluster bit for bit.  Kernels only (no host synchronisation); scratch
 * grows on the first call, so capture into a graph after one call. */
int nbody_force_batched(nbody_ctx *ctx, hipStream_t stream, nbody_prec prec, double G,
                        int32_t n_clusters, const int64_t *offsets, const double *eps,
                        int64_t n_total, nbody_src P, nbody_out out);

/* nsteps shared Hermite steps of length dt for every cluster at once (the
 * scheme of nbody_shared_run, forces from the batched kernel).  x, v, a, j:
 * device float64 [3][n_total] state, updated in place; a and j must hold the
 * forces at the starting state (e.g. from nbody_force_batched).  m: [n_total].
 * use_graph = 1 captures the whole nsteps-step sequence (plan, then per step
 * predict, pack, batched force, correct) into one hipGraph on a
 * context-owned stream the first time a given argument set is seen and
 * replays it afterwards, ordered after and before `stream` by events. */
int nbody_batch_hermite(nbody_ctx *ctx, hipStream_t stream, nbody_prec prec, double G,
                        int32_t n_clusters, const int64_t *offsets, const double *eps,
                        int64_t n_total, double dt, int nsteps, double *x, double *v, double *a,
                        double *j, const double *m, int use_graph);

/* Autotuner of the batched launch: times every launch shape on the given
 * clusters and keeps the fastest for this precision and (n_total,
 * n_clusters) bucket.  As nbody_autotune. */
int nbody_autotune_batched(nbody_ctx *ctx, hipStream_t stream, nbody_prec prec, double G,
                           int32_t n_clusters, const int64_t *offsets, const double *eps,
                           int64_t n_total, nbody_src P, nbody_out out, int reps,
                           nbody_tile *best, double *best_ms);

/* ---- active-block selection (Section 3.1) ---------------------------------- */

/* Block time steps: with integer times t[k] and steps dt[k] (device int64,
 * ticks of 2^-20 time units), t_next = min_k (t[k] + dt[k]) and the active
 * block is { k : t[k] + dt[k] == t_next } in ascending k.  Writes
 * idx[0 .. n_act-1] (device int32[n]); *n_act and *t_next are HOST
 * pointers and the call synchronises `stream`.  Pure integer work: the
 * result is bit-exact.  n == 0 gives n_act = 0. */
int nbody_select_active(nbody_ctx *ctx, hipStream_t stream, int64_t n, const int64_t *t,
                        const int64_t *dt, int32_t *idx, int64_t *n_act, int64_t *t_next);

/* ---- Hermite block-step driver (Section 3, 3.1) ----------------------------- */

typedef struct nbody_hermite nbody_hermite;

/* Options.  eta: Aarseth accuracy parameter; eta_start: first step
 * eta_start |a| / |jerk|; dt levels 2^dt_min_log2 .. 2^dt_max_log2 time
 * units (each in [-20, 0]); shared_dt_log2 != 0 gives every particle the
 * fixed step 2^shared_dt_log2 (all particles active every step). */
typedef struct {
    double G, eps, eta, eta_start;
    int dt_min_log2, dt_max_log2;
    int shared_dt_log2;
    nbody_prec prec;
} nbody_hermite_opts;

typedef struct {
    int64_t steps;        /* block steps taken */
    int64_t sum_active;   /* sum over steps of the block size */
    int64_t t_ticks;      /* current block time (ticks) */
} nbody_hermite_stats;

/* Allocate device state for n particles (all arrays library-owned). */
int nbody_hermite_create(nbody_ctx *ctx, nbody_hermite **h, int64_t n,
                         const nbody_hermite_opts *opts);
int nbody_hermite_destroy(nbody_hermite *h);

/* Load positions, velocities, masses (device rows of length n, copied) at
 * time 0; evaluate a and jerk of every particle and choose first steps. */
int nbody_hermite_set_state(nbody_hermite *h, hipStream_t stream, nbody_src P);

/* Copy the current state out (device rows of length n; any may be NULL):
 * x, v (as P's layout), a, jerk, t and dt in ticks (int64 rows). */
int nbody_hermite_get_state(nbody_hermite *h, hipStream_t stream, nbody_src P_out_as_mutable,
                            double *ax, double *ay, double *az, double *jx, double *jy,
                            double *jz, int64_t *t, int64_t *dt);

/* One block step: select, predict all, evaluate the block, correct, new
 * steps.  *n_active and *t_ticks (HOST, may be NULL) receive the block size
 * and the new block time.  With block steps this synchronises `stream` (the
 * block is chosen on the device and read back); with shared steps the block
 * is every particle and nothing waits. */
int nbody_hermite_step(nbody_hermite *h, hipStream_t stream, int64_t *n_active, int64_t *t_ticks);

/* Block steps until the next block time would exceed t_end_ticks.  With
 * block steps the block size, the launch shape and geometry of the pairwise
 * kernel (j-parallel for blocks under 256 particles, LDS tiles above;
 * i-groups, j-ranges) and the end-time gate are decided on the device, by
 * the last work-group of the selection pass; steps are enqueued in growing
 * chunks (1, 2, 4, ... up to 256; 64 with NBODY_TRACE or graph replay) and the host reads the plan's statistics
 * once per chunk (so the call returns with `stream` synchronised).  With
 * the environment variable NBODY_BLOCK_GRAPH=1 set when the integrator is
 * created, chunks of 64 steps are replayed from one captured hipGraph
 * (captured on a context-owned stream on first use) instead of being
 * launched step by step; the results are bit-identical.  A step whose block time lies beyond t_end_ticks
 * leaves the state untouched.  With shared steps the block is always every
 * particle and nothing is read back; a shared step of fewer than 4096
 * particles is one launch (each work-group gets its particles' forces and
 * corrects them), unless the environment variable NBODY_FUSED_CORRECT=0 was
 * set when the integrator was created (then a pairwise launch and a
 * corrector launch, with bit-identical results). */
int nbody_hermite_advance(nbody_hermite *h, hipStream_t stream, int64_t t_end_ticks,
                          nbody_hermite_stats *stats);

/* Total kinetic and potential energy (Eq. 2) at the current state, with
 * every particle predicted to the latest block time (HOST outputs;
 * synchronises `stream`). */
int nbody_hermite_energy(nbody_hermite *h, hipStream_t stream, double *ekin, double *epot);

/* Save / restore the complete integrator state to / from a host buffer of
 * nbody_hermite_state_bytes(h) bytes (checkpoint and resume; a restored
 * run continues bit-identically). */
int64_t nbody_hermite_state_bytes(const nbody_hermite *h);
int nbody_hermite_save(nbody_hermite *h, hipStream_t stream, void *host_buf);
int nbody_hermite_load(nbody_hermite *h, hipStream_t stream, const void *host_buf);

/* The power-of-two step rule applied by the corrector (Section 3.1 block
 * steps), evaluated on the host: largest 2^k <= crit (time units), clamped
 * to [2^lmin, 2^lmax]; a criterion that is zero, negative or not finite
 * gives 2^lmin; dt_old <= 0 is a first step; a smaller level is taken at
 * once, a larger one only as one doubling when t_new is a multiple of
 * 2 dt_old.  Ticks in and out; -1 for an invalid level range.  No device
 * work. */
int64_t nbody_block_level(double crit, int64_t dt_old, int64_t t_new, int lmin, int lmax);

#ifdef __cplusplus
}
#endif

#endif /* NBODY_H */

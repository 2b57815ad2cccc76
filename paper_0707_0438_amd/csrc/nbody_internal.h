// Internal declarations shared by the kernel and host translation units of
// libnbody.  Not installed; the public interface is include/nbody.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch_shape.h"

namespace nb {

// One tick of integer time is 2^-20 N-body time units; block steps are
// powers of two between 2^-20 and 2^0, so every block time is an exact
// integer number of ticks.
constexpr double kTick = 1.0 / 1048576.0;
constexpr int kTickLog2 = -20;

// Packed particle records (float4 units).
//  FP32 : {x, y, z, m}, {vx, vy, vz, 0}
//  DS   : {x_hi, y_hi, z_hi, m}, {vx, vy, vz, 0}, {x_lo, y_lo, z_lo, 0}
constexpr int kRecFP32 = 2;
constexpr int kRecDS = 3;
inline int rec_words(int prec) { return prec == 0 ? kRecFP32 : kRecDS; }


// One block step as the plan recorded it (NBODY_TRACE): written by the
// device into a ring of kTraceCap records, read by the host at each chunk's
// plan readback (a chunk holds at most kTraceCap steps).
struct TraceRec {
    int64_t step, t_next, n_act;
    int shape, nb, S, pad_;
};
constexpr int kTraceCap = 64;

// Block-step state the device keeps between launches (one per driver).
struct DevPlan {
    int64_t n_act;              // block size after the end-time gate (0: nothing to do)
    int64_t t_next;
    int64_t steps, sum_active;  // running statistics
    int64_t t_last;             // latest block time taken
    int64_t t_limit;            // end time of the current advance (ticks)
    int nb, S, jchunk, frozen;  // launch geometry; frozen = the gate stopped a step
    int shape, pad_;            // launch shape of the block: 0 small, 1 large (see below)
    TraceRec* ring;             // per-step records (NULL: not traced)
};

// Launch shapes of the plan-driven pairwise kernel (block steps).  Small
// blocks are latency-bound and take short j-ranges in small work-groups;
// blocks of at least kBlkBigMin particles take the shape of the large
// direct evaluations.  Each step launches both kernels and the one whose
// shape the plan did not pick returns at once.
#ifndef NB_BLK_SMALL_TJ
#define NB_BLK_SMALL_TJ 64
#endif
#ifndef NB_BLK_SMALL_WG
#define NB_BLK_SMALL_WG 128
#endif
#ifndef NB_BLK_BIG_MIN
#define NB_BLK_BIG_MIN 256
#endif
constexpr int kBlkSmallTile = NB_BLK_SMALL_TJ, kBlkSmallWG = NB_BLK_SMALL_WG;
constexpr int kBlkBigTile = 256, kBlkBigWG = 256;
constexpr int kBlkBigMin = NB_BLK_BIG_MIN;   // 0: the large shape is never used
constexpr int kBlkGrid = 2048;               // work-groups of each plan-driven launch
// Block-step launches after the front end.  2 (default): one pairwise
// launch for either shape (blk_step_kernel, 256-lane work-groups; blocks
// under kBlkBigMin particles j-parallel, in groups of kJparIG i-particles
// against j-ranges swept 256 x kJparJPL records at a time; larger ones in
// LDS tiles), then split reduce + corrector.  0: the pairwise launches by
// shape (force_kernel_plan, two launches, kBlkGrid work-groups each), then
// split reduce + corrector.  The split partials' size: blk_part_rows.
#ifndef NB_BLK_STEP_FUSED
#define NB_BLK_STEP_FUSED 2
#endif
constexpr int kBlkStepWG = 256;
// i-particles per lane of the tile shape in the block-step launch, per
// precision (DS, FP32)
#ifndef NB_BLK_BIG_IPT_DS
#define NB_BLK_BIG_IPT_DS 1
#endif
#ifndef NB_BLK_BIG_IPT_FP32
#define NB_BLK_BIG_IPT_FP32 1
#endif
__host__ __device__ constexpr int blk_big_ipt(int prec) { return prec == 1 ? NB_BLK_BIG_IPT_DS : NB_BLK_BIG_IPT_FP32; }
#ifndef NB_JPAR_IG
#define NB_JPAR_IG 2
#endif
constexpr int kJparIG = NB_JPAR_IG;   // i-particles per group of the j-parallel shape
#ifndef NB_JPAR_JPL
#define NB_JPAR_JPL 2
#endif
constexpr int kJparJPL = NB_JPAR_JPL;
#ifndef NB_JPAR_ITEMS
#define NB_JPAR_ITEMS 2048
#endif
#ifndef NB_JPAR_MAXS
#define NB_JPAR_MAXS 64
#endif
#ifndef NB_BLK_STEP_GRID
#define NB_BLK_STEP_GRID 6144
#endif
constexpr int kJparItems = NB_JPAR_ITEMS;   // (group, range) items a small block aims for
constexpr int kJparMaxS = NB_JPAR_MAXS;     // j-ranges of a small block at most
constexpr int kBlkStepGrid = NB_BLK_STEP_GRID;   // work-groups of the block-step pairwise launch
#ifndef NB_BLK_RC_GRID
#define NB_BLK_RC_GRID 1024
#endif
constexpr int kBlkRcGrid = NB_BLK_RC_GRID;       // work-groups of the block steps' reduce + corrector launch
// shared steps of at most this many particles take one j-range (no split
// reduce): 6-8% faster than two or more ranges at N = 1024 ... 4000
#ifndef NB_SHARED_ONE_RANGE_MAX
#define NB_SHARED_ONE_RANGE_MAX 4096
#endif
constexpr int kSharedOneRangeMax = NB_SHARED_ONE_RANGE_MAX;
// shared steps of at most this many particles run as one launch
// (launch_shared_step): N = 1024 DS 10.3 -> 8.4 us per step, N = 4000 (with
// four j records per lane per sweep) DS 34.5 -> 30.2 us
#ifndef NB_SHARED_ONE_LAUNCH_MAX
#define NB_SHARED_ONE_LAUNCH_MAX 4096
#endif
constexpr int kSharedOneLaunchMax = NB_SHARED_ONE_LAUNCH_MAX;
// i-particles per work-group of the one-launch shared step
#ifndef NB_SHARED_IG
#define NB_SHARED_IG 2
#endif
constexpr int kSharedIG = NB_SHARED_IG;
// the one-launch shared step sweeps 2 j records per lane per sweep up to
// this many particles (bit-identical to the two-launch form) and 4 above:
// N = 2048 and 3000 6-9% faster, N = 1024 the same
#ifndef NB_SHARED_JPL2_MAX
#define NB_SHARED_JPL2_MAX 1536
#endif
constexpr int kSharedJpl2Max = NB_SHARED_JPL2_MAX;
// shared steps of fewer particles use the j-parallel launch as well
#ifndef NB_SHARED_JPAR_MAX
#define NB_SHARED_JPAR_MAX 4096
#endif
constexpr int kSharedJparMax = NB_SHARED_JPAR_MAX;
// Geometry of a j-parallel pairwise launch of `total` i-particles against
// n j-particles: nb groups of kJparIG, S j-ranges of jc records (a whole
// number of kBlkStepWG x kJparJPL sweeps each): enough (group, range) items
// to spread over the device (about kJparItems), at most kJparMaxS ranges.
__host__ __device__ inline void jpar_plan(int64_t total, int n, int* nb_out, int* S_out, int* jc_out) {
    const int sweep = kBlkStepWG * kJparJPL;
    const int nb = (int)((total + kJparIG - 1) / kJparIG);
    int64_t smax = ((int64_t)n + sweep - 1) / sweep;
    smax = smax < kJparMaxS ? smax : kJparMaxS;
    int64_t sw = ((int64_t)kJparItems + nb - 1) / nb;
    sw = sw < smax ? sw : smax;
    sw = sw > 1 ? sw : 1;
    const int jc = (int)((((int64_t)n + sw - 1) / sw + sweep - 1) / sweep * sweep);
    *nb_out = nb;
    *jc_out = jc;
    *S_out = (int)(((int64_t)n + jc - 1) / jc);
}

// Four-launch form (NB_BLK_STEP_FUSED 0): small blocks split j down to this
// many tiles per range (latency-bound: short j-ranges on many work-groups
// finish sooner); blocks of at most kBlkTinyMax particles (one i-block) go
// down to one tile per range.
constexpr int kBlkMinTiles = 2;
#ifndef NB_BLK_TINY_MAX
#define NB_BLK_TINY_MAX 128
#endif
constexpr int kBlkTinyMax = NB_BLK_TINY_MAX;

// (i-group, j-range) items the split of a large block aims at: 6144 (24 per
// CU) was the fastest of 1280 ... 8192 for block steps at N = 65536
#ifndef NB_BLK_BIG_ITEMS
#define NB_BLK_BIG_ITEMS 6144
#endif
constexpr int kBlkBigItems = NB_BLK_BIG_ITEMS;

// Launch geometry of a block step of `total` particles among n: nb i-groups,
// S j-ranges of jc records; returns the launch shape (1: LDS tiles, 0: the
// small-block shape).  The device plan and the host's sizing of the split
// partials (blk_part_rows) both use it.
__host__ __device__ inline int blk_plan_geometry(int64_t total, int n, int big_ok, int prec, int* nb, int* S,
                                                 int* jc) {
    const int big = big_ok && kBlkBigMin > 0 && total >= kBlkBigMin;
#if NB_BLK_STEP_FUSED
    if (big) {
        // about kBlkBigItems (i-group, j-range) items (split_plan's rule with
        // that target)
        const int per = kBlkStepWG * blk_big_ipt(prec);
        const int64_t nbl = (total + per - 1) / per;
        int64_t sr = nbl >= kBlkBigItems / 2 ? 1 : ((int64_t)kBlkBigItems + nbl - 1) / nbl;
        const int64_t smax = n / kBlkBigTile;
        sr = sr > smax ? smax : sr;
        split_plan(total, n, per, kBlkBigTile, sr < 1 ? 1 : (int)sr, nb, S, jc, 1);
    } else {
        jpar_plan(total, n, nb, S, jc);
    }
#else
    (void)prec;
    if (big)
        split_plan(total, n, kBlkBigWG, kBlkBigTile, 0, nb, S, jc, 1);
    else
        split_plan(total, n, kBlkSmallWG, kBlkSmallTile, 0, nb, S, jc, total <= kBlkTinyMax ? 1 : kBlkMinTiles);
#endif
    return big;
}

// Rows of split partials a block step of any size among n particles may
// write (S x n_act; each row holds 7 (hi, lo) float2).  Bound: the split
// targets at most about T = max(kBlkBigItems, 2048) (i-group, range) items,
// so S x nb <= T + nb and S x n_act <= (T + nb) x per-group i count, which
// is at most (T + 1) x per_blk + n for the tile shapes and
// (kJparItems + 1) x kJparIG + n for the j-parallel one.  (The host checks
// the plans of every block size against it.)
inline int64_t blk_part_rows(int64_t n, int prec) {
#if NB_BLK_STEP_FUSED
    const int64_t per_blk = (int64_t)kBlkStepWG * blk_big_ipt(prec);
#else
    (void)prec;
    const int64_t per_blk = kBlkSmallWG > kBlkBigWG ? kBlkSmallWG : kBlkBigWG;
#endif
    const int64_t items = (kBlkBigItems > 2048 ? kBlkBigItems : 2048) + 1;
    const int64_t tiles = items * per_blk, jpar = (int64_t)(kJparItems + 1) * kJparIG;
    return (tiles > jpar ? tiles : jpar) + n;
}

// waves per SIMD asked of the compiler for blk_step_kernel (a register cap:
// the large-block tile loop keeps the occupancy of its direct-launch form)
#ifndef NB_BLK_STEP_WAVES
#define NB_BLK_STEP_WAVES 5
#endif
constexpr int kBlkStepWaves = NB_BLK_STEP_WAVES;
// 1: the block-step front end runs as one launch (launch_blk_front_fused)
#ifndef NB_BLK_FRONT_FUSED
#define NB_BLK_FRONT_FUSED 1
#endif

struct ForceArgs;   // force_block.h

struct ReduceArgs {
    int ni, S;
    const float2* part;
    double G;
    double* out[7];
    const DevPlan* plan;    // plan-driven launch: ni and S come from here
};

// Launch the pairwise kernel for one configuration; returns hipError_t.
// jsrc 0: j tiles staged in LDS; 1: j records through wave-uniform scalar loads.
// unr: unroll depth of the j loop (0 = 4); wpe: requested waves per SIMD (0 = none).
// kind 0: acceleration, jerk, potential; 1: acceleration and potential only;
// 2: kind 0 plus the nearest neighbour (ForceArgs.nn / nn_r2 / nnpart).
hipError_t launch_force(int prec, int ipt, int tile_j, int wg, int jsrc, int unr, int wpe, bool eps0, int n_iblocks,
                        int S, const ForceArgs& a, hipStream_t st, int kind = 0);
bool force_variant_exists(int prec, int ipt, int tile_j, int wg, int jsrc, int unr, int wpe, bool eps0,
                          int kind = 0);
int force_variant_count();
bool force_variant_at(int k, int* prec, int* ipt, int* tj, int* wg, int* jsrc, int* unr, int* wpe, bool* eps0,
                      int* kind);
// Rows of ReduceArgs.out that are NULL are skipped.
hipError_t launch_reduce(const ReduceArgs& a, hipStream_t st);
hipError_t launch_nn_reduce(int ni, int S, const float2* nnpart, int32_t* nn, double* nn_r2, hipStream_t st);
// Leapfrog: v += a h, x += v dt, then pack x (and m) into j records; and v += a h.
hipError_t launch_lf_kick_drift_pack(int prec, int n, double* x, double* v, const double* acc, const double* m,
                                     double h, double dt, float4* out, hipStream_t st);
hipError_t launch_lf_kick(int n, double* v, const double* acc, double h, hipStream_t st);
// Plan-driven launches (block sizes known only on the device).
// Plan-driven pairwise launches of one block step (both shapes; eps0: the
// small shape only).
hipError_t launch_force_plan(int prec, bool eps0, const ForceArgs& a,
                             hipStream_t st);

// ---- batched clusters ----
struct BatchArgs {
    const int2* items;       // (cluster, i-block)
    const int* n_items;      // device scalar
    int* counter;            // device work counter (zeroed before the launch)
    const int* cbeg;         // clamped cluster ranges
    const int* cend;
    const double* eps;       // per-cluster softening
};
struct PlanArgs {
    int n_clusters;
    const int64_t* offsets;  // device [n_clusters + 1]
    int n_total;
    int per;                 // i-particles per work item (WG * IPT)
    int64_t cap;             // item table capacity
    int *cbeg, *cend, *order, *start, *n_items;
    int2* items;
};
hipError_t launch_batch_plan(const PlanArgs& p, hipStream_t st);
hipError_t launch_force_batched(int prec, int ipt, int tile_j, int wg, int grid, const ForceArgs& a,
                                const BatchArgs& b, hipStream_t st);
hipError_t launch_fill_i32(int* p, int n, int v, hipStream_t st);

// Pack float64 rows into records; with t != NULL every particle is first
// predicted to the block time *tnext (device) by the Hermite predictor.
struct PackArgs {
    int n, prec;
    const double *x, *y, *z, *vx, *vy, *vz, *m;
    const double *ax, *ay, *az, *jx, *jy, *jz;   // predictor inputs (or NULL)
    const int64_t* t;                              // ticks (or NULL: no prediction)
    const int64_t* tnext;                          // device scalar (NULL: use tn)
    int64_t tn;                                    // block time when tnext is NULL
    float4* out;
};
hipError_t launch_pack(const PackArgs& a, hipStream_t st);
// Debug: *bad = number of i rows whose self index names a j record that is
// not bit-identical in position and velocity (or lies beyond nj).
hipError_t launch_self_check(int ni, int nj, int prec, const float4* ip, const int32_t* iself, const float4* jp,
                             int* bad, hipStream_t st);

// Active-block selection: out2[0] = n_act, out2[1] = t_next.  scratch: device
// int64 words, at least select_scratch_words(n).
int select_scratch_words(int n);
hipError_t launch_select(int n, const int64_t* t, const int64_t* dt, int32_t* idx, int64_t* out2,
                         int64_t* scratch, hipStream_t st);

struct CorrectArgs {
    int n_act;
    const int32_t* idx;               // block list (NULL: particles 0 .. n_act-1)
    const int64_t* tnext;             // device scalar (NULL: use tn)
    int64_t tn;                       // block time when tnext is NULL
    double *x, *y, *z, *vx, *vy, *vz;
    double *ax, *ay, *az, *jx, *jy, *jz;
    int64_t *t, *dt;
    const double* f[6];               // new a (3) and jerk (3) of the block, [n_act]
    double eta;
    int lmin, lmax, shared;           // shared != 0: keep dt
    int64_t* tnow;                    // receives the block time (written by one thread; may be NULL)
    // Shared steps: after its correction each particle is predicted to
    // tick tn_next and its record written to pack_next in precision
    // pack_prec (pack_one, so the same bits as a pack pass).  NULL: not done.
    const double* m;
    float4* pack_next;
    int64_t tn_next;
    int pack_prec;
    // Block steps: each corrected particle's new t + dt lowers the minimum of
    // its chunk of gch particles in gmin_next (NULL: not kept).
    int64_t* gmin_next;
    int gch;
};
hipError_t launch_correct(const CorrectArgs& a, hipStream_t st);

// Block-step front end: selection, prediction/packing of all j to the block
// time, and the device plan (see hermite.hip).  pa.t and pa.n give the
// ticks and count.  The particles fall into chunks of blk_chunk_size(n);
// gmin and gmin_next hold one int64 per chunk (blk_scratch_words(n) / 2):
// this step's chunk minima of t + dt (computed first when need_min) and the
// next step's, which the corrector completes (CorrectArgs.gmin_next).
// scratch holds blk_scratch_words(n) / 2 int64 words.  big_ok: the plan may
// pick the large launch shape.
int blk_chunk_size(int n);
int blk_scratch_words(int n);
hipError_t launch_blk_front(const PackArgs& pa, const int64_t* dt, int32_t* idx, int64_t* sel2, DevPlan* plan,
                            int64_t* scratch, int64_t* gmin, int64_t* gmin_next, bool need_min, bool big_ok,
                            hipStream_t st);
// The same front end as one launch (count, pack, ordered compaction and plan):
// pub holds one word per chunk (zeroed once when allocated) in which each
// step publishes its chunk counts tagged with the step's tag; *tagp (zeroed
// with pub) holds the last tag used and is advanced by the launch itself.
hipError_t launch_blk_front_fused(const PackArgs& pa, const int64_t* dt, int32_t* idx, int64_t* sel2, DevPlan* plan,
                                  uint64_t* pub, uint32_t* tagp, int64_t* gmin, int64_t* gmin_next, bool need_min,
                                  bool big_ok, hipStream_t st);
// The pairwise launch of a block step (NB_BLK_STEP_FUSED): the sums of the
// plan's block (a.plan) for either shape, as the plan's split partials
// (a.part) or, with one range, the final acceleration and jerk (a.out).
hipError_t launch_blk_step(int prec, bool eps0, const ForceArgs& a, hipStream_t st);
// A shared step of a.ni <= kSharedOneRangeMax particles in one launch: the
// j-parallel sums with one range, then the corrector of each group's
// particles in the same work-group (ca.pack_next must differ from a.jpack).
hipError_t launch_shared_step(int prec, bool eps0, const ForceArgs& a, const CorrectArgs& ca, hipStream_t st);
// Block steps: split reduce (when the plan has S > 1) fused with the corrector.
// With r.plan NULL the block is particles 0 .. r.ni-1 and the split is r.S.
hipError_t launch_blk_reduce_correct(const ReduceArgs& r, const CorrectArgs& ca, int grid, hipStream_t st);

// First steps after the initial force evaluation.
struct InitDtArgs {
    int n;
    const double *ax, *ay, *az, *jx, *jy, *jz;
    int64_t *t, *dt;
    double eta_s;
    int lmin, lmax, shared_log2;
};
hipError_t launch_init_dt(const InitDtArgs& a, hipStream_t st);

// Deterministic float64 sums: out[0] = sum 0.5 m v^2, out[1] = sum 0.5 m pot.
hipError_t launch_energy(int n, const double* vx, const double* vy, const double* vz,
                         const double* m, const double* pot, double* out2, hipStream_t st);

// ---- adjoint (vjp.hip) ----
struct VjpPackArgs {
    int n, prec;
    const double *x, *y, *z, *vx, *vy, *vz, *m;   // m may be NULL (0)
    const double *ga, *gj, *gp;                    // [3][n], [3][n], [n]; NULL = 0
    int key_mode;                                  // 0: key = index, 1: key = iself[k] (or -1)
    const int32_t* iself;
    float4* out;                                   // 5 float4 per particle
};
hipError_t launch_vjp_pack(const VjpPackArgs& a, hipStream_t st);

struct VjpArgs {
    const float4* lrec;   // lane particles
    int nl;
    const float4* trec;   // tile particles
    int nt;
    int jchunk;           // tile particles per split (multiple of the tile)
    float eps2;
    double G;
    int own;              // lane cotangents enter (final combination reads ga, gj)
    const double *ga, *gj;   // lane float64 cotangents [3][nl] (own only; NULL = 0)
    double *gx, *gv, *gm;    // outputs [3][nl], [3][nl], [nl] (NULL: skip)
    float2* part;            // split partials [S][9][nl] or NULL
};
hipError_t launch_vjp(int prec, bool own, bool partner, int S, const VjpArgs& a, hipStream_t st);
int vjp_tile();
int vjp_wg();
int vjp_acc();

// ---- shared-step integration and its adjoint (shared.hip); [3][n] rows ----
hipError_t launch_shared_predict(int n, double D, const double* x, const double* v, const double* a,
                                 const double* j, double* xp, double* vp, hipStream_t st);
hipError_t launch_shared_correct(int n, double D, const double* xp, const double* vp, double* x, double* v,
                                 double* a, double* j, const double* a1, const double* j1, hipStream_t st);
hipError_t launch_adj_correct(int n, double D, const double* X, const double* V, double* Aa, double* Jj,
                              double* ga, double* gj, hipStream_t st);
hipError_t launch_adj_predict(int n, double D, double* X, double* V, double* Aa, double* Jj, const double* tx,
                              const double* tv, hipStream_t st);
hipError_t launch_axpy(int n, double* y, const double* x, hipStream_t st);
hipError_t launch_sum2(int n, double* out, const double* a, const double* b, hipStream_t st);
hipError_t launch_fill_f64(int n, double* y, double v, hipStream_t st);

// p[0 .. n-1] = v (a kernel, so that graph capture records no memset node)
hipError_t launch_fill_i64(int64_t* p, int n, int64_t v, hipStream_t st);

// Predict every particle to *tnext in float64 (energy diagnostics).
hipError_t launch_predict_all(int n, const double* const* state /*x y z vx vy vz ax ay az jx jy jz*/,
                              const int64_t* t, const int64_t* tnext, double* const* outxv,
                              hipStream_t st);

// Hermite predictor (float64), Horner form of
//   x_p = x + v D + a D^2/2 + j D^3/6,  v_p = v + a D + j D^2/2.
__device__ __forceinline__ void predict1(double x, double v, double ac, double jk, double D,
                                         double& xp, double& vp) {
    xp = x + D * (v + D * (0.5 * ac + D * (jk * (1.0 / 6.0))));
    vp = v + D * (ac + D * (0.5 * jk));
}

// A packed record is written with a non-temporal store: the next launch
// reads it, from any XCD, so it gains nothing from this XCD's L2.  (Block
// steps at N = 65536 took 1-2% less time per step than with plain stores.)
__device__ __forceinline__ void st_rec(float4* p, float4 v) {
    typedef float v4f __attribute__((ext_vector_type(4)));
    const v4f w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<v4f*>(p));
}

// The float64 inputs of particle k's j record, loaded ahead of the pack
// (acceleration and jerk only when it predicts).
struct PackIn {
    double x[3], v[3], ac[3], jk[3];
    float m;
};
__device__ __forceinline__ void pack_load(const PackArgs& a, int k, bool predict, PackIn& s) {
    s.x[0] = a.x[k];
    s.x[1] = a.y[k];
    s.x[2] = a.z[k];
    s.v[0] = a.vx ? a.vx[k] : 0.0;
    s.v[1] = a.vy ? a.vy[k] : 0.0;
    s.v[2] = a.vz ? a.vz[k] : 0.0;
    if (predict) {
        s.ac[0] = a.ax[k];
        s.ac[1] = a.ay[k];
        s.ac[2] = a.az[k];
        s.jk[0] = a.jx[k];
        s.jk[1] = a.jy[k];
        s.jk[2] = a.jz[k];
    }
    s.m = a.m ? (float)a.m[k] : 0.f;
}

// Predict particle k over the interval D (when `predict`) and write its j
// record: float32 position (DS: hi = fl32(x), lo = fl32(x - hi)), mass,
// velocity.
template <int PREC>
__device__ __forceinline__ void pack_write(const PackArgs& a, int k, const PackIn& s, bool predict, double D) {
    double px = s.x[0], py = s.x[1], pz = s.x[2];
    double qx = s.v[0], qy = s.v[1], qz = s.v[2];
    if (predict) {
        predict1(px, qx, s.ac[0], s.jk[0], D, px, qx);
        predict1(py, qy, s.ac[1], s.jk[1], D, py, qy);
        predict1(pz, qz, s.ac[2], s.jk[2], D, pz, qz);
    }
    const float m = s.m;
    if (PREC == 0) {
        st_rec(&a.out[2 * (size_t)k], make_float4((float)px, (float)py, (float)pz, m));
        st_rec(&a.out[2 * (size_t)k + 1], make_float4((float)qx, (float)qy, (float)qz, 0.f));
    } else {
        const float hx = (float)px, hy = (float)py, hz = (float)pz;
        const float lx = (float)(px - (double)hx), ly = (float)(py - (double)hy),
                    lz = (float)(pz - (double)hz);
        st_rec(&a.out[3 * (size_t)k], make_float4(hx, hy, hz, m));
        st_rec(&a.out[3 * (size_t)k + 1], make_float4((float)qx, (float)qy, (float)qz, 0.f));
        st_rec(&a.out[3 * (size_t)k + 2], make_float4(lx, ly, lz, 0.f));
    }
}

template <int PREC>
__device__ __forceinline__ void pack_one_dt(const PackArgs& a, int k, bool predict, double D) {
    PackIn s;
    pack_load(a, k, predict, s);
    pack_write<PREC>(a, k, s, predict, D);
}

// The same with the interval from the particle's tick a.t[k] to tick tn
// (no prediction when a.t is NULL).
template <int PREC>
__device__ __forceinline__ void pack_one(const PackArgs& a, int k, int64_t tn) {
    pack_one_dt<PREC>(a, k, a.t != nullptr, a.t ? (double)(tn - a.t[k]) * kTick : 0.0);
}

// j index of the particle that i-slot `ii` is (or -1): see ForceArgs::self_mode.
__device__ __forceinline__ int self_index(int mode, const int32_t* iidx, const int32_t* iself, int ii) {
    if (mode == 1) return iidx[ii];
    if (mode == 2) return ii;
    return iself ? iself[ii] : -1;
}

// Step-level rule shared by the corrector kernel and the host API.
__host__ __device__ inline int64_t block_level(double crit, int64_t dt_old, int64_t t_new, int lmin,
                                               int lmax) {
    const int64_t dmin = (int64_t)1 << (lmin + 20);
    const int64_t dmax = (int64_t)1 << (lmax + 20);
    int64_t q = dmin;
    // crit must be a positive finite number; otherwise the smallest level.
    if (crit > 0.0 && isfinite(crit)) {
        // largest power of two (in ticks) not above crit, within [dmin, dmax]
        const double c_ticks = crit * 1048576.0;
        while (q < dmax && (double)(q << 1) <= c_ticks) q <<= 1;
    }
    if (dt_old <= 0) return q;
    if (q < dt_old) return q;
    if (q > dt_old && (dt_old << 1) <= dmax && (t_new % (dt_old << 1)) == 0) return dt_old << 1;
    return dt_old;
}

__device__ __forceinline__ double norm3(double a, double b, double c) { return sqrt(a * a + b * b + c * c); }

// Corrector for the active block (Makino & Aarseth 1992 Hermite scheme):
// with D = dt_i, the predicted state recomputed exactly as in the pack,
//   a2 = (-6 (a0 - a1) - D (4 j0 + 2 j1)) / D^2
//   a3 = (12 (a0 - a1) + 6 D (j0 + j1)) / D^3
//   x1 = x_p + a2 D^4/24 + a3 D^5/120,  v1 = v_p + a2 D^3/6 + a3 D^4/24,
// then the Aarseth criterion with a2 carried to the new time, and the
// power-of-two level rule.
// The corrector's float64 inputs of particle i (its state and ticks),
// loaded ahead of the arithmetic.
struct CorrIn {
    double x[3], v[3], ac[3], jk[3];
    int64_t t, dt;
};
__device__ __forceinline__ void corr_load(const CorrectArgs& a, int i, CorrIn& s) {
    s.x[0] = a.x[i];
    s.x[1] = a.y[i];
    s.x[2] = a.z[i];
    s.v[0] = a.vx[i];
    s.v[1] = a.vy[i];
    s.v[2] = a.vz[i];
    s.ac[0] = a.ax[i];
    s.ac[1] = a.ay[i];
    s.ac[2] = a.az[i];
    s.jk[0] = a.jx[i];
    s.jk[1] = a.jy[i];
    s.jk[2] = a.jz[i];
    s.t = a.t[i];
    s.dt = a.dt[i];
}

// Correct block entry c (particle i) from its loaded inputs s and its new
// acceleration and jerk; tn is the block time.
__device__ __forceinline__ void correct_apply(const CorrectArgs& a, int c, int i, const CorrIn& s, int64_t tn,
                                              const double* a1in, const double* j1in) {
    if (c == 0 && a.tnow) *a.tnow = tn;
    const double D = (double)s.dt * kTick;
    double* X[3] = {a.x, a.y, a.z};
    double* V[3] = {a.vx, a.vy, a.vz};
    double* A[3] = {a.ax, a.ay, a.az};
    double* J[3] = {a.jx, a.jy, a.jz};
    const double Dp = (double)(tn - s.t) * kTick;   // equals D for an active particle
    double a1[3], j1[3], a2[3], a3[3];
    const double iD = 1.0 / D, iD2 = iD * iD, iD3 = iD2 * iD;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double xp, vp;
        predict1(s.x[k], s.v[k], s.ac[k], s.jk[k], Dp, xp, vp);
        a1[k] = a1in[k];
        j1[k] = j1in[k];
        const double a0 = s.ac[k], j0 = s.jk[k];
        const double da = a0 - a1[k];
        a2[k] = (-6.0 * da - D * (4.0 * j0 + 2.0 * j1[k])) * iD2;
        a3[k] = (12.0 * da + 6.0 * D * (j0 + j1[k])) * iD3;
        const double D2 = D * D, D3 = D2 * D, D4 = D3 * D;
        X[k][i] = xp + D4 * (a2[k] * (1.0 / 24.0) + D * a3[k] * (1.0 / 120.0));
        V[k][i] = vp + D3 * (a2[k] * (1.0 / 6.0) + D * a3[k] * (1.0 / 24.0));
        A[k][i] = a1[k];
        J[k][i] = j1[k];
    }
    a.t[i] = tn;
    if (a.pack_next) {
        // the next shared step's record of this particle, from the state just
        // written (read back through memory, as a pack pass reads it)
        PackArgs p{};
        p.x = a.x; p.y = a.y; p.z = a.z;
        p.vx = a.vx; p.vy = a.vy; p.vz = a.vz;
        p.m = a.m;
        p.ax = a.ax; p.ay = a.ay; p.az = a.az;
        p.jx = a.jx; p.jy = a.jy; p.jz = a.jz;
        p.t = a.t;
        p.out = a.pack_next;
        if (a.pack_prec == 1)
            pack_one<1>(p, i, a.tn_next);
        else
            pack_one<0>(p, i, a.tn_next);
    }
    if (!a.shared) {
        const double b0 = a2[0] + a3[0] * D, b1 = a2[1] + a3[1] * D, b2 = a2[2] + a3[2] * D;
        const double na = norm3(a1[0], a1[1], a1[2]), nj = norm3(j1[0], j1[1], j1[2]);
        const double n2 = norm3(b0, b1, b2), n3 = norm3(a3[0], a3[1], a3[2]);
        const double crit = sqrt(a.eta * (na * n2 + nj * nj) / (nj * n3 + n2 * n2));
        const int64_t dtn = block_level(crit, s.dt, tn, a.lmin, a.lmax);
        a.dt[i] = dtn;
        // the next block time of this particle joins its chunk's minimum
        // (ticks are non-negative, so the unsigned minimum is the minimum)
        if (a.gmin_next)
            atomicMin((unsigned long long*)&a.gmin_next[i / a.gch], (unsigned long long)(tn + dtn));
    }
}

__device__ __forceinline__ void correct_core(const CorrectArgs& a, int c, const double* a1in,
                                             const double* j1in) {
    const int i = a.idx ? a.idx[c] : c;
    const int64_t tn = a.tnext ? *a.tnext : a.tn;
    CorrIn s;
    corr_load(a, i, s);
    correct_apply(a, c, i, s, tn, a1in, j1in);
}


__device__ __forceinline__ void correct_one(const CorrectArgs& a, int c) {
    double a1[3], j1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        a1[k] = a.f[k][c];
        j1[k] = a.f[3 + k][c];
    }
    correct_core(a, c, a1, j1);
}

}  // namespace nb

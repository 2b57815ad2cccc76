// Pairwise acceleration / jerk / potential kernel for gfx950 (CDNA4).
//
// What is computed (Eq. 1 with Plummer softening, Section 3.3; jerk and
// potential, Section 3): for each i of an i-list and every j of a j-set,
//   r = x_j - x_i, u = v_j - v_i, s = r.r + eps^2, q = s^-1/2,
//   a += m q^3 r,  jerk += m q^3 (u - 3 (r.u) q^2 r),  phi -= m q.
//
// Scheme (the tile scheme of Section 3.1 and Fig. 1, re-laid for CDNA4):
//  * each lane keeps IPT i-particles in registers for the whole j sweep;
//  * the work-group stages j records tile by tile in LDS (double buffered,
//    one barrier per tile); every lane then reads each record with a
//    wave-uniform (broadcast) LDS load;
//  * float32 VALU arithmetic with one hardware v_rsq_f32 per pair, no
//    branch in the loop (the ragged tail is padded with massless records
//    far away); all N^2 pairs are visited (Section 3.1).  The self pair is
//    excluded by index: a tile that holds the own j index of some lane of
//    the wave (one or two tiles of a self-gravitating sweep) runs a copy of
//    the loop in which that pair's mass is zeroed, so the large self
//    potential m_i/eps never enters a float32 partial sum (the paper
//    subtracts it after the loop; in float32 that leaves the rounding of
//    every later addition of the tile at the scale of m_i/eps);
//  * DS_COMP: positions are double-single and the relative coordinate is
//    (x_j,hi - x_i,hi) + (x_j,lo - x_i,lo); per-tile float32 partial sums
//    are folded into a two-sum (hi, lo) accumulator;
//  * small i-lists: the j set is cut into S ranges handled by different
//    work-groups that write (hi, lo) partials, reduced afterwards in
//    float64 in fixed order (the j-split of Section 3.2, with the combine
//    moved from the host to the device).
//
// Kinds of evaluation (compile-time, so the default kernel carries no extra
// work): KIND 0 acceleration + jerk + potential; KIND 1 acceleration +
// potential only (the force-only evaluation of Section 4, which a
// treecode or leapfrog needs); KIND 2 adds to KIND 0 the nearest neighbour
// of each i (Section 3.3): one unsoftened r^2 per pair, kept when smaller
// than the best so far and j is not i itself, so the lowest j wins a tie.
#include <type_traits>

#include "force_block.h"

namespace nb {

// WPE > 0 asks the compiler for at least WPE waves per SIMD (a register cap).
// UNR encodes the loop form: d (< 100) unroll d; 100 + d the
// software-pipelined LDS loop; 200 + d the low-register form (LOW above);
// 300 + d both.
constexpr int unr_depth(int u) { return u % 100; }
constexpr bool unr_pipe(int u) { return (u / 100) % 2 == 1; }
constexpr bool unr_low(int u) { return u >= 200; }

template <int PREC, int IPT, int TJ, int WG, bool EPS0, int UNR, int WPE>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(WPE > 0 ? WPE : 1)))
void force_kernel(ForceArgs a) {
    constexpr bool LOW = unr_low(UNR);
    __shared__ float4 sh[LOW ? 1 : 2][TJ * Rec<PREC>::R];
    __shared__ float losh[LOW && PREC == 1 ? 7 * IPT * WG : 1];
    const int jb = blockIdx.y * a.jchunk;
    const int je = min(a.nj, jb + a.jchunk);
    force_block<PREC, IPT, TJ, WG, EPS0, false, unr_depth(UNR), unr_pipe(UNR), 0, LOW>(
        a, sh, blockIdx.x * (WG * IPT), a.ni, jb, je, a.eps2, blockIdx.y, losh);
}

// The force-only (KIND 1) and nearest-neighbour (KIND 2) evaluations.
template <int PREC, int KIND, int IPT, int TJ, int WG, bool EPS0, int UNR>
__global__ __launch_bounds__(WG) void force_kernel_kind(ForceArgs a) {
    __shared__ float4 sh[2][TJ * Rec<PREC>::R];
    const int jb = blockIdx.y * a.jchunk;
    const int je = min(a.nj, jb + a.jchunk);
    force_block<PREC, IPT, TJ, WG, EPS0, false, unr_depth(UNR), unr_pipe(UNR), KIND>(
        a, sh, blockIdx.x * (WG * IPT), a.ni, jb, je, a.eps2, blockIdx.y);
}

// Plan-driven launch for block steps: the block size and the split come
// from the device plan; a fixed grid strides over the nb x S (i-block,
// j-range) pairs.  Each pair runs exactly the code of force_kernel.  SHAPE
// >= 0: only when the plan picked that shape.
template <int PREC, int IPT, int TJ, int WG, bool EPS0, int UNR = 4, int SHAPE = -1>
__global__ __launch_bounds__(WG) void force_kernel_plan(ForceArgs a) {
    __shared__ float4 sh[2][TJ * Rec<PREC>::R];
    const DevPlan* pl = a.plan;
    const int n = (int)pl->n_act;
    if (n <= 0 || (SHAPE >= 0 && pl->shape != SHAPE)) return;
    const int nb = pl->nb, S = pl->S;
    ForceArgs b = a;
    b.ni = n;
    b.jchunk = pl->jchunk;
    b.partial = S > 1 ? 1 : 0;
    for (int v = blockIdx.x; v < nb * S; v += gridDim.x) {
        const int ib = v % nb, s = v / nb;
        const int jb = s * b.jchunk;
        const int je = min(b.nj, jb + b.jchunk);
        force_block<PREC, IPT, TJ, WG, EPS0, false, unr_depth(UNR), unr_pipe(UNR)>(
            b, sh, ib * (WG * IPT), n, jb, je, b.eps2, s);
    }
}

// Same work with the j records read through the scalar data cache instead of
// LDS (every lane of a wave needs the same j record, so one wave-uniform load
// serves the wave).  TJ only sets the compensated-fold interval.
template <int PREC, int IPT, int TJ, int WG, bool EPS0, int UNR, int WPE>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(WPE > 0 ? WPE : 1)))
void force_kernel_js(ForceArgs a) {
    const int jb = blockIdx.y * a.jchunk;
    const int je = min(a.nj, jb + a.jchunk);
    force_block<PREC, IPT, TJ, WG, EPS0, true, UNR>(a, nullptr, blockIdx.x * (WG * IPT), a.ni, jb, je, a.eps2,
                                                     blockIdx.y);
}

// Many independent clusters in one persistent launch.  Work items
// (cluster, i-block) come from the plan, largest clusters first; each
// work-group takes the next item from a device counter until none is left.
// Within a cluster every particle is both an i and a j (self excluded);
// there are no cross-cluster terms.
template <int PREC, int IPT, int TJ, int WG>
__global__ __launch_bounds__(WG) void force_batched_kernel(ForceArgs a, BatchArgs b) {
    __shared__ float4 sh[2][TJ * Rec<PREC>::R];
    __shared__ int item_sh;
    const int n_items = *b.n_items;
    for (;;) {
        if (threadIdx.x == 0) item_sh = atomicAdd(b.counter, 1);
        __syncthreads();
        const int item = item_sh;
        __syncthreads();
        if (item >= n_items) break;
        const int2 it = b.items[item];
        const int beg = b.cbeg[it.x], end = b.cend[it.x];
        const double e = b.eps[it.x];
        force_block<PREC, IPT, TJ, WG, false>(a, sh, beg + it.y * (WG * IPT), end, beg, end,
                                              (float)(e * e), 0);
    }
}

// Float64 reduction of split partials in a fixed order, then the factor G
// (the self pair never entered a partial).  Few ranges: one thread per
// (quantity, i) sums s = 0 .. S-1 in order.  Many ranges: one wave per
// (quantity, i); lane l sums s = l, l + 64, ... in order, then a fixed
// butterfly over the 64 lane sums.  Either way the result depends only on S.
__device__ __forceinline__ double reduce_finish(const ReduceArgs& a, int q, double s) {
    return q < 6 ? a.G * s : -a.G * s;
}

__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs a) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 7 * (int64_t)a.ni) return;
    const int q = (int)(t / a.ni);
    const int i = (int)(t - (int64_t)q * a.ni);
    if (!a.out[q]) return;   // a row the evaluation does not produce
    double s = 0.0;
    for (int sp = 0; sp < a.S; ++sp) {
        const float2 p = a.part[((size_t)sp * 7 + q) * a.ni + i];
        s += (double)p.x;
        s += (double)p.y;
    }
    a.out[q][i] = reduce_finish(a, q, s);
}

__global__ __launch_bounds__(256) void reduce_wave_kernel(ReduceArgs a) {
    const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (w >= 7 * (int64_t)a.ni) return;   // whole waves leave together
    const int q = (int)(w / a.ni);
    const int i = (int)(w - (int64_t)q * a.ni);
    if (!a.out[q]) return;   // the whole wave shares q
    double s = 0.0;
    for (int sp = lane; sp < a.S; sp += 64) {
        const float2 p = a.part[((size_t)sp * 7 + q) * a.ni + i];
        s += (double)p.x;
        s += (double)p.y;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) a.out[q][i] = reduce_finish(a, q, s);
}

// Nearest neighbour over the j-ranges: the smallest r^2, the lower range
// (hence the lower j) on ties.
__global__ __launch_bounds__(256) void nn_reduce_kernel(int ni, int S, const float2* __restrict__ nnpart,
                                                        int32_t* __restrict__ nn, double* __restrict__ nn_r2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ni) return;
    float best = __builtin_inff();
    int bj = -1;
    for (int sp = 0; sp < S; ++sp) {
        const float2 p = nnpart[(size_t)sp * ni + i];
        const int j = __float_as_int(p.y);
        if (j >= 0 && (bj < 0 || p.x < best)) {
            best = p.x;
            bj = j;
        }
    }
    nn[i] = bj;
    if (nn_r2) nn_r2[i] = bj >= 0 ? (double)best : (double)__builtin_inff();
}

hipError_t launch_nn_reduce(int ni, int S, const float2* nnpart, int32_t* nn, double* nn_r2, hipStream_t st) {
    if (ni <= 0) return hipSuccess;
    hipLaunchKernelGGL(nn_reduce_kernel, dim3((ni + 255) / 256), dim3(256), 0, st, ni, S, nnpart, nn, nn_r2);
    return hipGetLastError();
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t st) {
    if (a.ni <= 0) return hipSuccess;
    const int64_t n = 7 * (int64_t)a.ni;
    if (a.S >= 32) {
        hipLaunchKernelGGL(reduce_wave_kernel, dim3((unsigned)((n * 64 + 255) / 256)), dim3(256), 0, st, a);
    } else {
        hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
    }
    return hipGetLastError();
}

// Plan: one work-group orders the clusters by size (largest first), splits
// each into i-blocks of `per` particles and writes the (cluster, block) items
// and their count.  Cluster ranges are clamped to [0, n_total] so that
// inconsistent offsets can never send a kernel out of bounds; items beyond
// the table capacity are dropped.
__global__ __launch_bounds__(1024) void batch_plan_kernel(PlanArgs p) {
    const int tid = threadIdx.x;
    const int C = p.n_clusters;
    for (int c = tid; c < C; c += 1024) {
        int64_t lo = p.offsets[c], hi = p.offsets[c + 1];
        lo = lo < 0 ? 0 : (lo > p.n_total ? p.n_total : lo);
        hi = hi < lo ? lo : (hi > p.n_total ? p.n_total : hi);
        p.cbeg[c] = (int)lo;
        p.cend[c] = (int)hi;
    }
    __syncthreads();
    // rank by size, descending; ties by index (a permutation)
    for (int c = tid; c < C; c += 1024) {
        const int sz = p.cend[c] - p.cbeg[c];
        int r = 0;
        if (C <= 16384) {
            for (int d = 0; d < C; ++d) {
                const int sd = p.cend[d] - p.cbeg[d];
                r += (sd > sz || (sd == sz && d < c)) ? 1 : 0;
            }
        } else {
            r = c;
        }
        p.order[r] = c;
    }
    __syncthreads();
    if (tid == 0) {
        int64_t acc = 0;
        for (int r = 0; r < C; ++r) {
            const int c = p.order[r];
            p.start[r] = (int)acc;
            acc += (p.cend[c] - p.cbeg[c] + p.per - 1) / p.per;
        }
        *p.n_items = (int)(acc < p.cap ? acc : p.cap);
    }
    __syncthreads();
    for (int r = tid; r < C; r += 1024) {
        const int c = p.order[r];
        const int nb = (p.cend[c] - p.cbeg[c] + p.per - 1) / p.per;
        for (int k = 0; k < nb; ++k) {
            const int64_t slot = (int64_t)p.start[r] + k;
            if (slot < p.cap) p.items[slot] = make_int2(c, k);
        }
    }
}

hipError_t launch_batch_plan(const PlanArgs& p, hipStream_t st) {
    hipLaunchKernelGGL(batch_plan_kernel, dim3(1), dim3(1024), 0, st, p);
    return hipGetLastError();
}

// ---- variant table -----------------------------------------------------------

template <int PREC, int IPT, int TJ, int WG, bool EPS0, int UNR, int WPE>
static hipError_t launch_one(int nb, int S, const ForceArgs& a, hipStream_t st) {
    hipLaunchKernelGGL((force_kernel<PREC, IPT, TJ, WG, EPS0, UNR, WPE>), dim3(nb, S), dim3(WG), 0, st, a);
    return hipGetLastError();
}

template <int PREC, int IPT, int TJ, int WG, bool EPS0, int UNR, int WPE>
static hipError_t launch_one_js(int nb, int S, const ForceArgs& a, hipStream_t st) {
    hipLaunchKernelGGL((force_kernel_js<PREC, IPT, TJ, WG, EPS0, UNR, WPE>), dim3(nb, S), dim3(WG), 0, st, a);
    return hipGetLastError();
}

template <int PREC, int KIND, int IPT, int TJ, int WG, bool EPS0, int UNR>
static hipError_t launch_kind(int nb, int S, const ForceArgs& a, hipStream_t st) {
    hipLaunchKernelGGL((force_kernel_kind<PREC, KIND, IPT, TJ, WG, EPS0, UNR>), dim3(nb, S), dim3(WG), 0, st, a);
    return hipGetLastError();
}

template <int PREC, int IPT, int TJ, int WG, bool EPS0>
static hipError_t launch_batched_one(int grid, const ForceArgs& a, const BatchArgs& b, hipStream_t st) {
    if (EPS0) return hipErrorInvalidValue;
    hipLaunchKernelGGL((force_batched_kernel<PREC, IPT, TJ, WG>), dim3(grid), dim3(WG), 0, st, a, b);
    return hipGetLastError();
}

typedef hipError_t (*LaunchFn)(int, int, const ForceArgs&, hipStream_t);
typedef hipError_t (*BatchedFn)(int, const ForceArgs&, const BatchArgs&, hipStream_t);

struct Variant {
    int prec, ipt, tj, wg, jsrc, unr, wpe;
    bool eps0;
    int kind;
    LaunchFn fn;
    BatchedFn bfn;
};

#define NB_V(P, I, T, W, E) \
    {P, I, T, W, 0, 4, 0, E, 0, &launch_one<P, I, T, W, E, 4, 0>, &launch_batched_one<P, I, T, W, E>}
#define NB_X(P, I, T, W, U, O) {P, I, T, W, 0, U, O, false, 0, &launch_one<P, I, T, W, false, U, O>, nullptr}
#define NB_J(P, I, W) {P, I, 128, W, 1, 4, 0, false, 0, &launch_one_js<P, I, 128, W, false, 4, 0>, nullptr}
#define NB_K(P, K, I, T, W, U, E) {P, I, T, W, 0, U, 0, E, K, &launch_kind<P, K, I, T, W, E, U>, nullptr}
#define NB_KP(P)                                                                                          \
    NB_K(P, 1, 1, 64, 128, 4, false), NB_K(P, 1, 1, 128, 256, 4, false), NB_K(P, 1, 2, 128, 256, 4, false), \
    NB_K(P, 1, 1, 256, 256, 102, false), NB_K(P, 1, 2, 256, 256, 101, false),                              \
    NB_K(P, 1, 2, 256, 256, 4, false), NB_K(P, 1, 4, 256, 256, 4, false), NB_K(P, 1, 1, 128, 256, 4, true), \
    NB_K(P, 2, 1, 64, 128, 4, false), NB_K(P, 2, 1, 128, 256, 4, false), NB_K(P, 2, 1, 256, 256, 102, false), \
    NB_K(P, 2, 2, 256, 256, 101, false), NB_K(P, 2, 1, 128, 256, 4, true)
#define NB_VT(P, I, W)                                                                  \
    NB_V(P, I, 64, W, false), NB_V(P, I, 128, W, false), NB_V(P, I, 256, W, false)
#define NB_VW(P, I) NB_VT(P, I, 128), NB_VT(P, I, 256)
#define NB_VP(P) NB_VW(P, 1), NB_VW(P, 2), NB_VW(P, 4)

static const Variant kVariants[] = {
    NB_VP(0),
    NB_VP(1),
    // j records through the scalar data cache
    NB_J(0, 1, 64), NB_J(0, 2, 64), NB_J(0, 4, 64), NB_J(0, 1, 256), NB_J(0, 2, 256), NB_J(0, 4, 256),
    NB_J(1, 1, 64), NB_J(1, 2, 64), NB_J(1, 4, 64), NB_J(1, 1, 256), NB_J(1, 2, 256), NB_J(1, 4, 256),
    // unroll depth and occupancy experiments around the best LDS shapes
    NB_X(0, 1, 256, 256, 2, 0), NB_X(0, 1, 256, 256, 8, 0), NB_X(0, 1, 256, 256, 4, 6), NB_X(0, 1, 256, 256, 4, 8),
    NB_X(0, 2, 256, 256, 1, 0), NB_X(0, 2, 256, 256, 2, 0), NB_X(0, 2, 256, 256, 2, 5), NB_X(0, 2, 128, 256, 2, 4),
    NB_X(1, 1, 256, 256, 2, 0), NB_X(1, 1, 256, 256, 8, 0), NB_X(1, 1, 256, 256, 4, 6), NB_X(1, 1, 256, 256, 4, 8),
    NB_X(1, 2, 256, 256, 1, 0), NB_X(1, 2, 256, 256, 2, 0), NB_X(1, 2, 256, 256, 2, 5), NB_X(1, 2, 128, 256, 2, 4),
    // software-pipelined LDS reads (unroll = 100 + depth)
    NB_X(0, 1, 256, 256, 102, 0), NB_X(0, 1, 256, 256, 104, 0), NB_X(0, 2, 256, 256, 101, 0),
    NB_X(1, 1, 256, 256, 102, 0), NB_X(1, 1, 256, 256, 104, 0), NB_X(1, 2, 256, 256, 101, 0),
    NB_X(1, 1, 128, 256, 102, 0), NB_X(1, 1, 256, 128, 102, 0),
    // low-register forms (lo words in LDS, single-buffered tiles; 200 + d,
    // pipelined 300 + d)
    NB_X(1, 2, 256, 256, 202, 0), NB_X(1, 2, 256, 256, 301, 0), NB_X(1, 2, 128, 256, 202, 0),
    NB_X(1, 2, 128, 256, 301, 0), NB_X(0, 2, 256, 256, 202, 0), NB_X(0, 1, 256, 256, 302, 0),
    // short tiles for small, latency-bound sets (more j-ranges, shorter sweeps)
    NB_X(0, 1, 16, 64, 4, 0), NB_X(0, 1, 32, 64, 4, 0), NB_X(0, 1, 16, 128, 4, 0), NB_X(0, 1, 32, 128, 4, 0),
    NB_X(1, 1, 16, 64, 4, 0), NB_X(1, 1, 32, 64, 4, 0), NB_X(1, 1, 16, 128, 4, 0), NB_X(1, 1, 32, 128, 4, 0),
    // unsoftened (eps = 0) path: one shape per precision
    NB_V(0, 1, 128, 256, true), NB_V(0, 2, 128, 256, true),
    NB_V(1, 1, 128, 256, true), NB_V(1, 2, 128, 256, true),
    // force-only (kind 1) and nearest-neighbour (kind 2) evaluations
    NB_KP(0),
    NB_KP(1),
};

// unr / wpe of 0 select the default (unroll 4, no occupancy request)
static const Variant* find_variant(int prec, int ipt, int tj, int wg, int jsrc, int unr, int wpe, bool eps0,
                                   int kind = 0) {
    if (unr == 0) unr = 4;
    for (const Variant& v : kVariants)
        if (v.prec == prec && v.ipt == ipt && v.tj == tj && v.wg == wg && v.jsrc == jsrc && v.unr == unr &&
            v.wpe == wpe && v.eps0 == eps0 && v.kind == kind)
            return &v;
    return nullptr;
}

bool force_variant_exists(int prec, int ipt, int tj, int wg, int jsrc, int unr, int wpe, bool eps0, int kind) {
    return find_variant(prec, ipt, tj, wg, jsrc, unr, wpe, eps0, kind) != nullptr;
}

hipError_t launch_force(int prec, int ipt, int tj, int wg, int jsrc, int unr, int wpe, bool eps0, int nb, int S,
                        const ForceArgs& a, hipStream_t st, int kind) {
    const Variant* v = find_variant(prec, ipt, tj, wg, jsrc, unr, wpe, eps0, kind);
    if (!v) return hipErrorInvalidValue;
    return v->fn(nb, S, a, st);
}

hipError_t launch_force_batched(int prec, int ipt, int tj, int wg, int grid, const ForceArgs& a,
                                const BatchArgs& b, hipStream_t st) {
    const Variant* v = find_variant(prec, ipt, tj, wg, 0, 4, 0, false);
    if (!v || !v->bfn) return hipErrorInvalidValue;
    return v->bfn(grid, a, b, st);
}

int force_variant_count() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }

// plan-driven shapes (block steps)
template <int PREC>
static void launch_plan_pair(bool eps0, const ForceArgs& a, hipStream_t st) {
    if (eps0) {
        hipLaunchKernelGGL((force_kernel_plan<PREC, 1, kBlkSmallTile, kBlkSmallWG, true>), dim3(kBlkGrid),
                           dim3(kBlkSmallWG), 0, st, a);
        return;
    }
    hipLaunchKernelGGL((force_kernel_plan<PREC, 1, kBlkSmallTile, kBlkSmallWG, false, 4, 0>), dim3(kBlkGrid),
                       dim3(kBlkSmallWG), 0, st, a);
    if (kBlkBigMin > 0)
        hipLaunchKernelGGL((force_kernel_plan<PREC, 1, kBlkBigTile, kBlkBigWG, false, 102, 1>), dim3(kBlkGrid),
                           dim3(kBlkBigWG), 0, st, a);
}

hipError_t launch_force_plan(int prec, bool eps0, const ForceArgs& a, hipStream_t st) {
    if (prec == 0)
        launch_plan_pair<0>(eps0, a, st);
    else
        launch_plan_pair<1>(eps0, a, st);
    return hipGetLastError();
}

bool force_variant_at(int k, int* prec, int* ipt, int* tj, int* wg, int* jsrc, int* unr, int* wpe, bool* eps0,
                      int* kind) {
    if (k < 0 || k >= force_variant_count()) return false;
    const Variant& v = kVariants[k];
    *prec = v.prec; *ipt = v.ipt; *tj = v.tj; *wg = v.wg; *jsrc = v.jsrc; *unr = v.unr; *wpe = v.wpe; *eps0 = v.eps0;
    *kind = v.kind;
    return true;
}

}  // namespace nb

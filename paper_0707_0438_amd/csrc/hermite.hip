// Block time-step kernels (Section 3 and 3.1): active-block selection on
// integer ticks, the float64 Hermite corrector with the Aarseth step
// criterion and power-of-two step levels, first steps, and energy sums.
#include "nbody_internal.h"

namespace nb {

constexpr int kSelThreads = 1024;
constexpr int kSelWaves = kSelThreads / 64;

// One work-group scans the whole (t, dt) array: first the minimum of
// t + dt, then an order-preserving compaction of the indices that reach it.
// Integer work only, so the result is exact.
__global__ __launch_bounds__(kSelThreads) void select_kernel(int n, const int64_t* __restrict__ t,
                                                             const int64_t* __restrict__ dt,
                                                             int32_t* __restrict__ idx,
                                                             int64_t* __restrict__ out2) {
    __shared__ int64_t red[kSelWaves];
    __shared__ int wsum[kSelWaves];
    __shared__ int64_t tn_sh;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;

    int64_t m = INT64_MAX;
    for (int k = tid; k < n; k += kSelThreads) {
        const int64_t v = t[k] + dt[k];
        m = v < m ? v : m;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const int64_t o = __shfl_xor(m, off);
        m = o < m ? o : m;
    }
    if (lane == 0) red[w] = m;
    __syncthreads();
    if (tid == 0) {
        int64_t r = red[0];
        for (int k = 1; k < kSelWaves; ++k) r = red[k] < r ? red[k] : r;
        tn_sh = r;
    }
    __syncthreads();
    const int64_t tn = tn_sh;

    // compaction in chunks of 4 * kSelThreads consecutive elements; each lane
    // owns 4 consecutive entries so the output stays in ascending order
    int base = 0;
    for (int c0 = 0; c0 < n; c0 += 4 * kSelThreads) {
        const int k0 = c0 + 4 * tid;
        int f[4], cnt = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + u;
            f[u] = (k < n && t[k] + dt[k] == tn) ? 1 : 0;
            cnt += f[u];
        }
        // inclusive scan of cnt across the wave
        int incl = cnt;
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(incl, off);
            if (lane >= off) incl += o;
        }
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        int wbase = 0, total = 0;
        for (int k = 0; k < kSelWaves; ++k) {
            const int s = wsum[k];
            wbase += k < w ? s : 0;
            total += s;
        }
        int pos = base + wbase + incl - cnt;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (f[u]) idx[pos++] = k0 + u;
        base += total;
        __syncthreads();   // wsum is rewritten by the next chunk
    }
    if (tid == 0) {
        out2[0] = base;
        out2[1] = tn;
    }
}

// Larger sets: three passes over chunks of kSelChunk consecutive entries
// (one work-group each): group minima; the global minimum (every group
// reduces all group minima) and each group's count; then each group's
// offset (sum of the counts before it) and an ordered compaction.
constexpr int kSelChunk = 4096;
#ifndef NB_SEL_WG
#define NB_SEL_WG 256
#endif
constexpr int kSelWG = NB_SEL_WG;
constexpr int kSelPer = kSelChunk / kSelWG;   // consecutive entries per lane

__device__ __forceinline__ int64_t block_min_i64(int64_t m, int64_t* red) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int off = 32; off > 0; off >>= 1) {
        const int64_t o = __shfl_xor(m, off);
        m = o < m ? o : m;
    }
    if (lane == 0) red[w] = m;
    __syncthreads();
    int64_t r = red[0];
    for (int k = 1; k < kSelWG / 64; ++k) r = red[k] < r ? red[k] : r;
    __syncthreads();
    return r;
}

__device__ __forceinline__ int64_t block_sum_i64(int64_t v, int64_t* red) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) red[w] = v;
    __syncthreads();
    int64_t r = 0;
    for (int k = 0; k < kSelWG / 64; ++k) r += red[k];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kSelWG) void select_min_kernel(int n, const int64_t* __restrict__ t,
                                                            const int64_t* __restrict__ dt,
                                                            int64_t* __restrict__ gmin) {
    __shared__ int64_t red[kSelWG / 64];
    const int base = blockIdx.x * kSelChunk;
    const int end = min(n, base + kSelChunk);
    int64_t m = INT64_MAX;
    for (int k = base + threadIdx.x; k < end; k += kSelWG) {
        const int64_t v = t[k] + dt[k];
        m = v < m ? v : m;
    }
    m = block_min_i64(m, red);
    if (threadIdx.x == 0) gmin[blockIdx.x] = m;
}

__global__ __launch_bounds__(kSelWG) void select_count_kernel(int n, int G, const int64_t* __restrict__ t,
                                                              const int64_t* __restrict__ dt,
                                                              const int64_t* __restrict__ gmin,
                                                              int64_t* __restrict__ gcnt,
                                                              int64_t* __restrict__ out2) {
    __shared__ int64_t red[kSelWG / 64];
    int64_t m = INT64_MAX;
    for (int g = threadIdx.x; g < G; g += kSelWG) m = gmin[g] < m ? gmin[g] : m;
    const int64_t tn = block_min_i64(m, red);
    const int base = blockIdx.x * kSelChunk;
    const int end = min(n, base + kSelChunk);
    int64_t c = 0;
    for (int k = base + threadIdx.x; k < end; k += kSelWG) c += (t[k] + dt[k] == tn) ? 1 : 0;
    c = block_sum_i64(c, red);
    if (threadIdx.x == 0) {
        gcnt[blockIdx.x] = c;
        if (blockIdx.x == 0) out2[1] = tn;
    }
}

__global__ __launch_bounds__(kSelWG) void select_write_kernel(int n, int G, const int64_t* __restrict__ t,
                                                              const int64_t* __restrict__ dt,
                                                              const int64_t* __restrict__ gcnt,
                                                              int64_t* __restrict__ out2,
                                                              int32_t* __restrict__ idx) {
    __shared__ int64_t red[kSelWG / 64];
    __shared__ int wsum[kSelWG / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t tn = out2[1];
    int64_t before = 0, total = 0;
    for (int g = tid; g < G; g += kSelWG) {
        total += gcnt[g];
        before += g < (int)blockIdx.x ? gcnt[g] : 0;
    }
    before = block_sum_i64(before, red);
    total = block_sum_i64(total, red);
    const int k0 = blockIdx.x * kSelChunk + tid * kSelPer;
    int cnt = 0;
    for (int u = 0; u < kSelPer; ++u) {
        const int k = k0 + u;
        cnt += (k < n && t[k] + dt[k] == tn) ? 1 : 0;
    }
    int incl = cnt;
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(incl, off);
        if (lane >= off) incl += o;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int wbase = 0;
    for (int k = 0; k < w; ++k) wbase += wsum[k];
    int64_t pos = before + wbase + incl - cnt;
    for (int u = 0; u < kSelPer; ++u) {
        const int k = k0 + u;
        if (k < n && t[k] + dt[k] == tn) idx[pos++] = k;
    }
    if (blockIdx.x == 0 && tid == 0) out2[0] = total;
}

int select_scratch_words(int n) { return n > kSelChunk ? 2 * ((n + kSelChunk - 1) / kSelChunk) : 0; }

hipError_t launch_select(int n, const int64_t* t, const int64_t* dt, int32_t* idx, int64_t* out2,
                         int64_t* scratch, hipStream_t st) {
    if (n <= kSelChunk) {
        hipLaunchKernelGGL(select_kernel, dim3(1), dim3(kSelThreads), 0, st, n, t, dt, idx, out2);
        return hipGetLastError();
    }
    const int G = (n + kSelChunk - 1) / kSelChunk;
    int64_t* gmin = scratch;
    int64_t* gcnt = scratch + G;
    hipLaunchKernelGGL(select_min_kernel, dim3(G), dim3(kSelWG), 0, st, n, t, dt, gmin);
    hipLaunchKernelGGL(select_count_kernel, dim3(G), dim3(kSelWG), 0, st, n, G, t, dt, gmin, gcnt, out2);
    hipLaunchKernelGGL(select_write_kernel, dim3(G), dim3(kSelWG), 0, st, n, G, t, dt, gcnt, out2, idx);
    return hipGetLastError();
}

// ---- block-step front end ---------------------------------------------------
// The selection of a block step fused with the work that depends only on its
// result, in three passes over chunks of `ch` entries (a power of two chosen
// so that about kBlkGroups work-groups share the particles):
//   1. chunk minima of t + dt (only after the state was set or loaded:
//      afterwards pass 2 and the corrector keep them, see below);
//   2. the global minimum t_next, each chunk's count of particles due at
//      t_next, and the prediction of every particle of the chunk to t_next
//      packed into j records;
//   3. each chunk's offset and the ordered compaction of its due indices,
//      and (one thread) the block plan: size, launch geometry of the
//      pairwise kernel, statistics.
// A step whose t_next lies beyond the plan's end time changes nothing and
// marks the plan frozen.  Integer selection, so the block is exact.
#ifndef NB_BLK_GROUPS
#define NB_BLK_GROUPS 256
#endif
constexpr int kBlkGroups = NB_BLK_GROUPS;

__host__ __device__ inline int blk_chunk(int n) {
    int ch = kSelWG;
    while ((int64_t)ch * kBlkGroups < n) ch *= 2;
    return ch;
}

__global__ __launch_bounds__(kSelWG) void blk_min_kernel(int n, int ch, const int64_t* __restrict__ t,
                                                         const int64_t* __restrict__ dt, int64_t* __restrict__ gmin) {
    __shared__ int64_t red[kSelWG / 64];
    const int base = blockIdx.x * ch;
    const int end = min(n, base + ch);
    int64_t m = INT64_MAX;
    for (int k = base + threadIdx.x; k < end; k += kSelWG) {
        const int64_t v = t[k] + dt[k];
        m = v < m ? v : m;
    }
    m = block_min_i64(m, red);
    if (threadIdx.x == 0) gmin[blockIdx.x] = m;
}

constexpr int kFrontSpin = 1 << 20;

__device__ __forceinline__ void blk_plan_write(DevPlan* plan, int64_t total, int64_t tn, int n, int big_ok,
                                               int prec) {
    int nb, S, jc;
    const int big = blk_plan_geometry(total, n, big_ok, prec, &nb, &S, &jc);
    plan->shape = big;
    plan->n_act = total;
    plan->t_next = tn;
    plan->nb = nb;
    plan->S = S;
    plan->jchunk = jc;
    plan->steps += 1;
    plan->sum_active += total;
    plan->t_last = tn;
    if (TraceRec* r = plan->ring) {
        TraceRec& e = r[(plan->steps - 1) % kTraceCap];
        e.step = plan->steps;
        e.t_next = tn;
        e.n_act = total;
        e.shape = big;
        e.nb = nb;
        e.S = S;
        e.pad_ = 0;
    }
}

// gmin holds this step's chunk minima.  gmin_next receives, per chunk, the
// minimum of t + dt over the particles that are not due (the corrector then
// lowers it with the new t + dt of the due ones), so the next step needs no
// minimum pass; a step past the end time copies gmin unchanged.
template <int PREC>
__global__ __launch_bounds__(kSelWG) void blk_count_pack_kernel(int ch, int G, const int64_t* __restrict__ dt,
                                                                const int64_t* __restrict__ gmin,
                                                                int64_t* __restrict__ gmin_next,
                                                                int64_t* __restrict__ gcnt,
                                                                int64_t* __restrict__ sel2,
                                                                const DevPlan* __restrict__ plan, PackArgs pa) {
    __shared__ int64_t red[kSelWG / 64];
    int64_t m = INT64_MAX;
    for (int g = threadIdx.x; g < G; g += kSelWG) m = gmin[g] < m ? gmin[g] : m;
    const int64_t tn = block_min_i64(m, red);
    const int base = blockIdx.x * ch;
    const int end = min(pa.n, base + ch);
    int64_t c = 0, rest = INT64_MAX;
    for (int k = base + threadIdx.x; k < end; k += kSelWG) {
        const int64_t v = pa.t[k] + dt[k];
        c += v == tn ? 1 : 0;
        rest = (v != tn && v < rest) ? v : rest;
    }
    c = block_sum_i64(c, red);
    rest = block_min_i64(rest, red);
    const bool frozen = tn > plan->t_limit;
    if (threadIdx.x == 0) {
        gcnt[blockIdx.x] = c;
        gmin_next[blockIdx.x] = frozen ? gmin[blockIdx.x] : rest;
        if (blockIdx.x == 0) sel2[1] = tn;
    }
    if (frozen) return;
    for (int k = base + threadIdx.x; k < end; k += kSelWG) pack_one<PREC>(pa, k, tn);
}

__global__ __launch_bounds__(kSelWG) void blk_write_plan_kernel(int n, int ch, int G, const int64_t* __restrict__ t,
                                                                const int64_t* __restrict__ dt,
                                                                const int64_t* __restrict__ gcnt,
                                                                int64_t* __restrict__ sel2,
                                                                int32_t* __restrict__ idx, DevPlan* plan,
                                                                int big_ok, int prec) {
    __shared__ int64_t red[kSelWG / 64];
    __shared__ int wsum[kSelWG / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t tn = sel2[1];
    int64_t before = 0, total = 0;
    for (int g = tid; g < G; g += kSelWG) {
        total += gcnt[g];
        before += g < (int)blockIdx.x ? gcnt[g] : 0;
    }
    before = block_sum_i64(before, red);
    total = block_sum_i64(total, red);
    const bool go = total > 0 && tn <= plan->t_limit;
    if (go) {
        const int per = ch / kSelWG;   // consecutive entries per lane
        const int k0 = blockIdx.x * ch + tid * per;
        int cnt = 0;
        for (int u = 0; u < per; ++u) {
            const int k = k0 + u;
            cnt += (k < n && t[k] + dt[k] == tn) ? 1 : 0;
        }
        int incl = cnt;
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(incl, off);
            if (lane >= off) incl += o;
        }
        if (lane == 63) wsum[w] = incl;
        __syncthreads();
        int wbase = 0;
        for (int k = 0; k < w; ++k) wbase += wsum[k];
        int64_t pos = before + wbase + incl - cnt;
        for (int u = 0; u < per; ++u) {
            const int k = k0 + u;
            if (k < n && t[k] + dt[k] == tn) idx[pos++] = k;
        }
    }
    if (blockIdx.x == 0 && tid == 0) {
        sel2[0] = total;
        if (!go) {
            plan->n_act = 0;
            plan->frozen = 1;
        } else {
            // large blocks take the large direct evaluations' shape
            blk_plan_write(plan, total, tn, n, big_ok, prec);
        }
    }
}

// The whole front end in one launch.  Work-group b owns chunk b: it takes
// t_next from the kept chunk minima, counts its due particles, publishes
// that count in pub[b] tagged with this step's tag, then predicts and packs
// its chunk, and only then waits for the counts of the chunks before it to
// place its part of the ordered block list.  The published word is the only
// data passed between work-groups, so it is written and polled with relaxed
// device-scope atomics (no fences).  The tag is *tagp + 1 (never 0, the
// value the words start at); the last work-group stores it back only after
// the counts of every other work-group have arrived, each published after
// that work-group read *tagp, so every work-group of a launch sees the same
// tag and consecutive launches (also replays of a captured graph) never
// share one.  Lower-numbered work-groups are dispatched first and never
// wait for higher ones, so every wait ends; each wait is also bounded
// (kFrontSpin polls), after which the plan records the failure (frozen = 2)
// and the step does nothing.  A step past the end time (frozen) publishes
// and waits as well, but packs and places nothing.  The last work-group
// writes the plan.  The arithmetic of the count, the compaction and the pack
// is the same as blk_count_pack_kernel + blk_write_plan_kernel, so the same
// block list and records come out.
template <int PREC>
__global__ __launch_bounds__(kSelWG) void blk_front_kernel(int ch, int G, const int64_t* __restrict__ dt,
                                                           const int64_t* __restrict__ gmin,
                                                           int64_t* __restrict__ gmin_next,
                                                           uint64_t* __restrict__ pub, uint32_t* __restrict__ tagp,
                                                           int64_t* __restrict__ sel2, int32_t* __restrict__ idx,
                                                           DevPlan* plan, PackArgs pa, int big_ok) {
    __shared__ int64_t red[kSelWG / 64];
    __shared__ int wsum[kSelWG / 64];
    __shared__ int fail_sh;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int b = blockIdx.x;
    const int n = pa.n;
    // this lane's `per` consecutive entries of the chunk.  With one entry
    // per lane (n <= kBlkGroups x kSelWG) the entry's tick, next tick and
    // the pack's float64 inputs are loaded here, together with the chunk
    // minima, instead of one dependent load after another.
    const int per = ch / kSelWG;
    const int k0 = b * ch + tid * per;
    const bool one = per == 1;
    int64_t t1 = 0, v1 = 0;
    PackIn pre;
    if (one && k0 < n) {
        t1 = pa.t[k0];
        v1 = t1 + dt[k0];
        pack_load(pa, k0, true, pre);
    }
    const int64_t t_limit = plan->t_limit;
    uint32_t tag = *tagp + 1u;
    tag = tag ? tag : 1u;
    int64_t m = INT64_MAX;
    for (int g = tid; g < G; g += kSelWG) m = gmin[g] < m ? gmin[g] : m;
    const int64_t tn = block_min_i64(m, red);
    const bool frozen = tn > t_limit;
    // due particles among the lane's entries
    int cnt = 0;
    int64_t rest = INT64_MAX;
    for (int u = 0; u < per; ++u) {
        const int k = k0 + u;
        if (k < n) {
            const int64_t v = one ? v1 : pa.t[k] + dt[k];
            cnt += v == tn ? 1 : 0;
            rest = (v != tn && v < rest) ? v : rest;
        }
    }
    if (frozen) cnt = 0;
    int incl = cnt;
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(incl, off);
        if (lane >= off) incl += o;
    }
    if (lane == 63) wsum[w] = incl;
    if (tid == 0) fail_sh = 0;
    rest = block_min_i64(rest, red);   // (its barriers also publish wsum and fail_sh)
    int wbase = 0, c = 0;
    for (int k = 0; k < kSelWG / 64; ++k) {
        wbase += k < w ? wsum[k] : 0;
        c += wsum[k];
    }
    if (tid == 0) {
        gmin_next[b] = frozen ? gmin[b] : rest;
        if (b == 0) sel2[1] = tn;
        __hip_atomic_store(&pub[b], ((uint64_t)tag << 32) | (uint32_t)c, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!frozen) {
        if (one) {
            if (k0 < n) pack_write<PREC>(pa, k0, pre, true, (double)(tn - t1) * kTick);
        } else {
            for (int k = b * ch + tid; k < min(n, (b + 1) * ch); k += kSelWG) pack_one<PREC>(pa, k, tn);
        }
    }
    // counts of the chunks before this one
    int64_t before = 0;
    for (int g = tid; g < b; g += kSelWG) {
        uint64_t v = 0;
        int it = 0;
        for (;;) {
            // relaxed (coherent at device scope, no L2 invalidation per poll)
            v = __hip_atomic_load(&pub[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((uint32_t)(v >> 32) == tag) break;
            if (++it >= kFrontSpin) {
                fail_sh = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        before += (int64_t)(uint32_t)v;
    }
    before = block_sum_i64(before, red);
    const bool last = b == G - 1 && tid == 0;
    if (fail_sh || frozen) {
        // a void step (failed wait; the host reports it at the end of the
        // chunk) or one past the end time: no block, state untouched
        if (last) {
            sel2[0] = 0;
            plan->n_act = 0;
            plan->frozen = fail_sh ? 2 : 1;
            *tagp = tag;
        } else if (fail_sh && tid == 0) {
            plan->frozen = 2;
        }
        return;
    }
    int64_t pos = before + wbase + incl - cnt;
    for (int u = 0; u < per; ++u) {
        const int k = k0 + u;
        if (k < n && (one ? v1 : pa.t[k] + dt[k]) == tn) idx[pos++] = k;
    }
    if (last) {
        const int64_t total = before + c;
        sel2[0] = total;
        blk_plan_write(plan, total, tn, n, big_ok, PREC);
        *tagp = tag;
    }
}

hipError_t launch_blk_front_fused(const PackArgs& pa, const int64_t* dt, int32_t* idx, int64_t* sel2, DevPlan* plan,
                                  uint64_t* pub, uint32_t* tagp, int64_t* gmin, int64_t* gmin_next, bool need_min,
                                  bool big_ok, hipStream_t st) {
    const int n = pa.n;
    if (n <= 0) return hipErrorInvalidValue;
    const int ch = blk_chunk(n);
    const int G = (n + ch - 1) / ch;
    if (need_min) hipLaunchKernelGGL(blk_min_kernel, dim3(G), dim3(kSelWG), 0, st, n, ch, pa.t, dt, gmin);
    if (pa.prec == 0)
        hipLaunchKernelGGL(blk_front_kernel<0>, dim3(G), dim3(kSelWG), 0, st, ch, G, dt, gmin, gmin_next, pub, tagp,
                           sel2, idx, plan, pa, big_ok ? 1 : 0);
    else
        hipLaunchKernelGGL(blk_front_kernel<1>, dim3(G), dim3(kSelWG), 0, st, ch, G, dt, gmin, gmin_next, pub, tagp,
                           sel2, idx, plan, pa, big_ok ? 1 : 0);
    return hipGetLastError();
}

int blk_chunk_size(int n) { return blk_chunk(n); }

int blk_scratch_words(int n) {
    const int ch = blk_chunk(n);
    return 2 * ((n + ch - 1) / ch);
}

hipError_t launch_blk_front(const PackArgs& pa, const int64_t* dt, int32_t* idx, int64_t* sel2, DevPlan* plan,
                            int64_t* scratch, int64_t* gmin, int64_t* gmin_next, bool need_min, bool big_ok,
                            hipStream_t st) {
    const int n = pa.n;
    if (n <= 0) return hipErrorInvalidValue;
    const int ch = blk_chunk(n);
    const int G = (n + ch - 1) / ch;
    int64_t* gcnt = scratch;
    if (need_min) hipLaunchKernelGGL(blk_min_kernel, dim3(G), dim3(kSelWG), 0, st, n, ch, pa.t, dt, gmin);
    if (pa.prec == 0)
        hipLaunchKernelGGL(blk_count_pack_kernel<0>, dim3(G), dim3(kSelWG), 0, st, ch, G, dt, gmin, gmin_next, gcnt,
                           sel2, plan, pa);
    else
        hipLaunchKernelGGL(blk_count_pack_kernel<1>, dim3(G), dim3(kSelWG), 0, st, ch, G, dt, gmin, gmin_next, gcnt,
                           sel2, plan, pa);
    hipLaunchKernelGGL(blk_write_plan_kernel, dim3(G), dim3(kSelWG), 0, st, n, ch, G, pa.t, dt, gcnt, sel2, idx,
                       plan, big_ok ? 1 : 0, pa.prec);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void correct_kernel(CorrectArgs a) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n_act) return;
    correct_one(a, c);
}

hipError_t launch_correct(const CorrectArgs& a, hipStream_t st) {
    if (a.n_act <= 0) return hipSuccess;
    const int grid = (a.n_act + 255) / 256;
    hipLaunchKernelGGL(correct_kernel, dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void init_dt_kernel(InitDtArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    if (a.shared_log2 != 0) {
        a.dt[i] = (int64_t)1 << (a.shared_log2 + 20);
        return;
    }
    const double na = norm3(a.ax[i], a.ay[i], a.az[i]);
    const double nj = norm3(a.jx[i], a.jy[i], a.jz[i]);
    a.dt[i] = block_level(a.eta_s * na / nj, 0, 0, a.lmin, a.lmax);
}

// Block steps: the float64 reduction of the split partials fused with the
// corrector.  Without a split the pairwise kernel has written the forces and
// only the corrector runs.  Shared steps use it without a device plan, with
// the next step's prediction and packing fused in as well
// (CorrectArgs.pack_next).
__global__ __launch_bounds__(256) void blk_reduce_correct_kernel(ReduceArgs r, CorrectArgs ca) {
    const DevPlan* pl = r.plan;
    const int n = pl ? (int)pl->n_act : r.ni, S = pl ? pl->S : r.S;
    if (n <= 0) return;
    if (S <= 1) {
        for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) correct_one(ca, c);
        return;
    }
    // Split reduce, 16 particles per work-group (256 threads, as launched):
    // thread t takes particle p = t % 16 of the group and the ranges
    // s = t / 16, t / 16 + 16, ... in order, so that for every (s, q) the
    // group's 16 partial sums are one contiguous 128-byte line.  The 16
    // range-lanes of a particle then combine in a fixed order: two butterfly
    // steps inside each wave (lanes 16 and 32 apart), then the four waves in
    // order.  The result depends only on S.
    __shared__ double wpart[4][16][6];
    const int tid = threadIdx.x, p = tid & 15, l = tid >> 4, w = tid >> 6;
    const int ngroups = (n + 15) / 16;
    const size_t qs = (size_t)n, rs = 7 * (size_t)n;
    const int64_t tn = ca.tnext ? *ca.tnext : ca.tn;
    for (int g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const int c = g * 16 + p;
        // the corrector's inputs (threads 0-15, one particle each): the list
        // entry is loaded with the partials and the state right after it, so
        // that their latency overlaps the sums
        const bool corr = tid < 16 && c < n;
        int ci = 0;
        CorrIn pre;
        if (corr) ci = ca.idx ? ca.idx[c] : c;
        bool pending = corr;   // (S > 1, so the first range of threads 0-15 is read below)
        double f[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (c < n) {
            const float2* col = r.part + c;
            int sp = l;
            for (; sp + 48 < S; sp += 64) {
                float2 u[4][6];
#pragma unroll
                for (int h = 0; h < 4; ++h)
#pragma unroll
                    for (int q = 0; q < 6; ++q) u[h][q] = col[(size_t)(sp + 16 * h) * rs + q * qs];
                if (pending) {
                    corr_load(ca, ci, pre);
                    pending = false;
                }
#pragma unroll
                for (int h = 0; h < 4; ++h)
#pragma unroll
                    for (int q = 0; q < 6; ++q) {
                        f[q] += (double)u[h][q].x;
                        f[q] += (double)u[h][q].y;
                    }
            }
            for (; sp < S; sp += 16) {
                float2 u[6];
#pragma unroll
                for (int q = 0; q < 6; ++q) u[q] = col[(size_t)sp * rs + q * qs];
                if (pending) {
                    corr_load(ca, ci, pre);
                    pending = false;
                }
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    f[q] += (double)u[q].x;
                    f[q] += (double)u[q].y;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            f[q] += __shfl_xor(f[q], 16);
            f[q] += __shfl_xor(f[q], 32);
            if ((tid & 63) < 16) wpart[w][p][q] = f[q];
        }
        __syncthreads();
        if (corr) {
            double gq[6];
#pragma unroll
            for (int q = 0; q < 6; ++q)
                gq[q] = r.G * (((wpart[0][p][q] + wpart[1][p][q]) + wpart[2][p][q]) + wpart[3][p][q]);
            correct_apply(ca, c, ci, pre, tn, gq, gq + 3);
        }
        __syncthreads();   // wpart is rewritten by the next group
    }
}

hipError_t launch_blk_reduce_correct(const ReduceArgs& r, const CorrectArgs& ca, int grid, hipStream_t st) {
    hipLaunchKernelGGL(blk_reduce_correct_kernel, dim3(grid), dim3(256), 0, st, r, ca);
    return hipGetLastError();
}

hipError_t launch_init_dt(const InitDtArgs& a, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(init_dt_kernel, dim3((a.n + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

// Energy sums in float64 by one work-group in a fixed order (deterministic).
__global__ __launch_bounds__(1024) void energy_kernel(int n, const double* __restrict__ vx,
                                                      const double* __restrict__ vy,
                                                      const double* __restrict__ vz,
                                                      const double* __restrict__ m,
                                                      const double* __restrict__ pot,
                                                      double* __restrict__ out2) {
    __shared__ double sk[1024], sp[1024];
    const int tid = threadIdx.x;
    double k = 0.0, p = 0.0;
    for (int i = tid; i < n; i += 1024) {
        k += 0.5 * m[i] * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
        p += 0.5 * m[i] * pot[i];
    }
    sk[tid] = k;
    sp[tid] = p;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if (tid < s) {
            sk[tid] += sk[tid + s];
            sp[tid] += sp[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        out2[0] = sk[0];
        out2[1] = sp[0];
    }
}

hipError_t launch_energy(int n, const double* vx, const double* vy, const double* vz, const double* m,
                         const double* pot, double* out2, hipStream_t st) {
    hipLaunchKernelGGL(energy_kernel, dim3(1), dim3(1024), 0, st, n, vx, vy, vz, m, pot, out2);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void fill_i64_kernel(int64_t* p, int n, int64_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_i64(int64_t* p, int n, int64_t v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i64_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void fill_i32_kernel(int* p, int n, int v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(int* p, int n, int v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

}  // namespace nb

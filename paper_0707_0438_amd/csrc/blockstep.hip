// The pairwise launch of a block step (Section 3.1's block step, with the
// prediction and selection already done on the device): the sums of the
// plan's block for either launch shape, in one launch.  Shared steps of
// small sets use it too, with a plan written by the host.
#include <algorithm>

#include "force_block.h"

namespace nb {

// Small blocks (the plan's shape 0) are j-parallel: the kJparIG i-particles
// of a group are the same in every lane (uniform loads), and lane l of the
// work-group takes the j records jb + l + 256 k (k < kJparJPL) of its range,
// so that no lane idles however few particles are due.  Each lane adds its
// few pairs in float32; the 256 lane sums of each quantity are then added in
// float64 in a fixed order and stored as the range's (hi, lo) partial.
// Large blocks (shape 1) keep the tile loop of the large direct
// evaluations: one i per lane, 256-record LDS tiles, software-pipelined
// reads.  The self pair needs no mask here: an i record is its own j record,
// so its separation and relative velocity are exactly zero and it adds
// exactly nothing to the acceleration and jerk (the potential is not formed).
template <int PREC, bool EPS0, int IG = kJparIG, int JPL = kJparJPL>
__device__ __forceinline__ void jpar_block(const ForceArgs& a, int n_act, int g, int s, int jb, int je,
                                           float* smem) {
    constexpr int R = Rec<PREC>::R;
    constexpr int WG = kBlkStepWG;
    static_assert(IG * 6 * 8 <= WG, "the final reduce takes 8 threads per (i, quantity)");
    float* red = smem;                  // [IG * 6][WG]: high words of the lane sums
    float* losh = smem + IG * 6 * WG;   // [IG * 6][WG]: their low words
    const int tid = threadIdx.x;
    float ix[IG], iy[IG], iz[IG], iu[IG], iv[IG], iw[IG], lx[IG], ly[IG], lz[IG];
#pragma unroll
    for (int k = 0; k < IG; ++k) {
        const int c = g * IG + k;
        float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;
        if (c < n_act) {
            const int src = a.iidx ? a.iidx[c] : c;
            r0 = a.ipack[(size_t)src * R + 0];
            r1 = a.ipack[(size_t)src * R + 1];
            if (PREC == 1) r2 = a.ipack[(size_t)src * R + 2];
        }
        ix[k] = r0.x; iy[k] = r0.y; iz[k] = r0.z;
        iu[k] = r1.x; iv[k] = r1.y; iw[k] = r1.z;
        lx[k] = r2.x; ly[k] = r2.y; lz[k] = r2.z;
    }
    float eps2v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(eps2v) : "s"(a.eps2));
    float hi[IG][6];
#pragma unroll
    for (int k = 0; k < IG; ++k)
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            hi[k][q] = 0.f;
            losh[(k * 6 + q) * WG + tid] = 0.f;
        }
    // sweeps of WG x JPL records: lane l takes j0 + l + WG u (u < JPL), all
    // loads first; each sweep's float32 sums fold into a two-sum per lane
    for (int j0 = jb; j0 < je; j0 += WG * JPL) {
        float4 q0[JPL], q1[JPL], q2[JPL];
#pragma unroll
        for (int u = 0; u < JPL; ++u) {
            const int j = j0 + tid + WG * u;
            q0[u] = make_float4(kPadPos, kPadPos, kPadPos, 0.f);
            q1[u] = make_float4(0.f, 0.f, 0.f, 0.f);
            q2[u] = q1[u];
            if (j < je) {
                q0[u] = a.jpack[(size_t)j * R + 0];
                q1[u] = a.jpack[(size_t)j * R + 1];
                if (PREC == 1) q2[u] = a.jpack[(size_t)j * R + 2];
            }
        }
        float acc[IG][6];
#pragma unroll
        for (int k = 0; k < IG; ++k)
#pragma unroll
            for (int q = 0; q < 6; ++q) acc[k][q] = 0.f;
#pragma unroll
        for (int u = 0; u < JPL; ++u) {
#pragma unroll
            for (int k = 0; k < IG; ++k) {
                float dx, dy, dz;
                if (PREC == 1) {
                    dx = (q0[u].x - ix[k]) + (q2[u].x - lx[k]);
                    dy = (q0[u].y - iy[k]) + (q2[u].y - ly[k]);
                    dz = (q0[u].z - iz[k]) + (q2[u].z - lz[k]);
                } else {
                    dx = q0[u].x - ix[k];
                    dy = q0[u].y - iy[k];
                    dz = q0[u].z - iz[k];
                }
                const float sq = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2v)));
                float rinv = __builtin_amdgcn_rsqf(sq);
                if (EPS0) rinv = sq > 0.f ? rinv : 0.f;
                const float ux = q1[u].x - iu[k], uy = q1[u].y - iv[k], uz = q1[u].z - iw[k];
                const float rv = fmaf(dz, uz, fmaf(dy, uy, dx * ux));
                const float rinv2 = rinv * rinv;
                const float mr3 = (q0[u].w * rinv) * rinv2;
                const float al = 3.0f * rv * rinv2;
                acc[k][0] = fmaf(mr3, dx, acc[k][0]);
                acc[k][1] = fmaf(mr3, dy, acc[k][1]);
                acc[k][2] = fmaf(mr3, dz, acc[k][2]);
                acc[k][3] = fmaf(mr3, fmaf(-al, dx, ux), acc[k][3]);
                acc[k][4] = fmaf(mr3, fmaf(-al, dy, uy), acc[k][4]);
                acc[k][5] = fmaf(mr3, fmaf(-al, dz, uz), acc[k][5]);
            }
        }
#pragma unroll
        for (int k = 0; k < IG; ++k)
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                float lo = losh[(k * 6 + q) * WG + tid];
                two_sum_fold(hi[k][q], lo, acc[k][q]);
                losh[(k * 6 + q) * WG + tid] = lo;
            }
    }
    // lane sums -> LDS; then 8 threads per (i, quantity) add 32 lanes each in
    // float64, in lane order (high then low word), and a fixed butterfly
    // joins the 8
#pragma unroll
    for (int k = 0; k < IG; ++k)
#pragma unroll
        for (int q = 0; q < 6; ++q) red[(k * 6 + q) * WG + tid] = hi[k][q];
    __syncthreads();
    if (tid < IG * 6 * 8) {
        const int cq = tid >> 3, part = tid & 7;
        const int l0 = cq * WG + part * (WG / 8);
        double f = 0.0;
#pragma unroll 8
        for (int l = 0; l < WG / 8; ++l) {
            f += (double)red[l0 + l];
            f += (double)losh[l0 + l];
        }
        f += __shfl_xor(f, 1);
        f += __shfl_xor(f, 2);
        f += __shfl_xor(f, 4);
        const int k = cq / 6, q = cq - 6 * (cq / 6);
        const int c = g * IG + k;
        if (part == 0 && c < n_act) {
            if (a.partial) {
                const float h = (float)f;
                a.part[((size_t)s * 7 + q) * n_act + c] = make_float2(h, (float)(f - (double)h));
            } else {
                // (a select chain: a runtime index into the by-value array
                // of row pointers would place it in scratch memory)
                double* o = q == 0 ? a.out[0] : q == 1 ? a.out[1] : q == 2 ? a.out[2]
                          : q == 3 ? a.out[3] : q == 4 ? a.out[4] : a.out[5];
                o[c] = a.G * f;
            }
        }
    }
}

// The pairwise sums of the plan's block, either shape: the (group, range)
// items of the plan, strided over the grid.  The split partials (or, with
// one range, the final acceleration and jerk) go to a.part / a.out; the
// float64 split reduce and the corrector follow in blk_reduce_correct_kernel.
template <int PREC, bool EPS0>
__global__ __launch_bounds__(kBlkStepWG) __attribute__((amdgpu_waves_per_eu(kBlkStepWaves)))
void blk_step_kernel(ForceArgs a) {
    constexpr int R = Rec<PREC>::R;
    constexpr int kTileBytes = 2 * kBlkBigTile * R * (int)sizeof(float4);
    constexpr int kRedBytes = 2 * kJparIG * 6 * kBlkStepWG * (int)sizeof(float);
    __shared__ __align__(16) unsigned char smem[kTileBytes > kRedBytes ? kTileBytes : kRedBytes];
    const DevPlan* pl = a.plan;
    const int n = (int)pl->n_act;
    if (n <= 0) return;
    const int nb = pl->nb, S = pl->S, shape = pl->shape;
    ForceArgs b = a;
    b.ni = n;
    b.jchunk = pl->jchunk;
    b.partial = S > 1 ? 1 : 0;
    for (int v = blockIdx.x; v < nb * S; v += gridDim.x) {
        const int g = v % nb, s = v / nb;
        const int jb = s * b.jchunk;
        const int je = min(b.nj, jb + b.jchunk);
        if (!EPS0 && shape == 1) {
            constexpr int IPT = blk_big_ipt(PREC);
            force_block<PREC, IPT, kBlkBigTile, kBlkStepWG, false, false, IPT == 1 ? 2 : 1, true>(
                b, reinterpret_cast<float4(*)[kBlkBigTile * R]>(smem), g * kBlkStepWG * IPT, n, jb, je, b.eps2, s);
        }
        else
            jpar_block<PREC, EPS0>(b, n, g, s, jb, je, reinterpret_cast<float*>(smem));
        __syncthreads();   // LDS is rewritten by the next item
    }
}

// A shared step of a small set in one launch: work-group g sweeps all j for
// the kJparIG particles of group g (the j-parallel form with one range, so
// the group's forces are final in the work-group) and then corrects those
// particles.  Nothing passes between work-groups: each reads the current j
// records (a.jpack) and writes only its own particles' state and their
// next-step records, which go to another buffer (ca.pack_next must not be
// a.jpack).  The forces go through a.out, written and read inside the
// work-group, so the results equal the pairwise launch with one range
// followed by the corrector launch.
template <int PREC, bool EPS0, int JPL>
__global__ __launch_bounds__(kBlkStepWG) void shared_step_kernel(ForceArgs a, CorrectArgs ca) {
    __shared__ __align__(16) float smem[2 * kSharedIG * 6 * kBlkStepWG];
    const int n = a.ni;
    const int nb = (n + kSharedIG - 1) / kSharedIG;
    ForceArgs b = a;
    b.partial = 0;
    for (int g = blockIdx.x; g < nb; g += gridDim.x) {
        jpar_block<PREC, EPS0, kSharedIG, JPL>(b, n, g, 0, 0, n, smem);
        __syncthreads();   // the group's forces are in a.out
        const int c0 = g * kSharedIG, cnt = min(kSharedIG, n - c0);
        if ((int)threadIdx.x < cnt) correct_one(ca, c0 + threadIdx.x);
        __syncthreads();   // LDS is rewritten by the next group
    }
}

hipError_t launch_shared_step(int prec, bool eps0, const ForceArgs& a, const CorrectArgs& ca, hipStream_t st) {
    if (ca.pack_next && reinterpret_cast<const void*>(ca.pack_next) == reinterpret_cast<const void*>(a.jpack))
        return hipErrorInvalidValue;
    const int nb = (a.ni + kSharedIG - 1) / kSharedIG;
    const dim3 g(std::min(nb, kBlkStepGrid)), b(kBlkStepWG);
    // larger sets sweep 4 records per lane (half the dependent sweeps);
    // smaller ones keep the block steps' 2, whose sums the two-launch form
    // repeats bit for bit
    const bool wide = a.ni > kSharedJpl2Max;
    if (prec == 0) {
        if (eps0)
            hipLaunchKernelGGL(wide ? (shared_step_kernel<0, true, 4>) : (shared_step_kernel<0, true, kJparJPL>), g, b,
                               0, st, a, ca);
        else
            hipLaunchKernelGGL(wide ? (shared_step_kernel<0, false, 4>) : (shared_step_kernel<0, false, kJparJPL>), g,
                               b, 0, st, a, ca);
    } else {
        if (eps0)
            hipLaunchKernelGGL(wide ? (shared_step_kernel<1, true, 4>) : (shared_step_kernel<1, true, kJparJPL>), g, b,
                               0, st, a, ca);
        else
            hipLaunchKernelGGL(wide ? (shared_step_kernel<1, false, 4>) : (shared_step_kernel<1, false, kJparJPL>), g,
                               b, 0, st, a, ca);
    }
    return hipGetLastError();
}

hipError_t launch_blk_step(int prec, bool eps0, const ForceArgs& a, hipStream_t st) {
    const dim3 g(kBlkStepGrid), b(kBlkStepWG);
    if (prec == 0) {
        if (eps0)
            hipLaunchKernelGGL((blk_step_kernel<0, true>), g, b, 0, st, a);
        else
            hipLaunchKernelGGL((blk_step_kernel<0, false>), g, b, 0, st, a);
    } else {
        if (eps0)
            hipLaunchKernelGGL((blk_step_kernel<1, true>), g, b, 0, st, a);
        else
            hipLaunchKernelGGL((blk_step_kernel<1, false>), g, b, 0, st, a);
    }
    return hipGetLastError();
}

}  // namespace nb

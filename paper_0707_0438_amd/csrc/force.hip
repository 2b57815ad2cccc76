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

#include "nbody_internal.h"

namespace nb {

constexpr float kPadPos = 1.0e18f;   // far-away position of padding records

template <int PREC>
struct Rec;
template <>
struct Rec<0> { static constexpr int R = kRecFP32; };
template <>
struct Rec<1> { static constexpr int R = kRecDS; };

__device__ __forceinline__ void two_sum_fold(float& hi, float& lo, float p) {
    // Knuth's TwoSum: hi + p = s + e exactly; the error joins lo.
    const float s = hi + p;
    const float bb = s - hi;
    const float e = (hi - (s - bb)) + (p - bb);
    hi = s;
    lo += e;
}

// One work-group's share: i slots ibase + k*WG + tid (k < IPT) below iend,
// against j in [jb, je).  Results go to the float64 outputs or to split
// partial slot `split`.
// LOW (fewer registers, hence more resident waves): the low words of the
// compensated sums live in LDS (losh, 7 * IPT * WG floats: each lane
// touches its own words once per tile) and the j tiles are single-buffered
// (sh[0] only), so no staging registers stay live through the tile loop.
template <int PREC, int IPT, int TJ, int WG, bool EPS0, bool JS = false, int UNR = 4, bool PIPE = false,
          int KIND = 0, bool LOW = false>
__device__ __forceinline__ void force_block(const ForceArgs& a, float4 (*sh)[TJ * Rec<PREC>::R], int ibase,
                                            int iend, int jb, int je, float eps2, int split,
                                            float* __restrict__ losh = nullptr) {
    constexpr int R = Rec<PREC>::R;
    constexpr int NE = TJ * R;                  // float4 per tile
    constexpr int NLD = (NE + WG - 1) / WG;     // staging loads per lane

    const int tid = threadIdx.x;
    const int ntiles = je > jb ? (je - jb + TJ - 1) / TJ : 0;

    // i-particles of this lane
    float ix[IPT], iy[IPT], iz[IPT], iu[IPT], iv[IPT], iw[IPT];
    float lx[IPT], ly[IPT], lz[IPT];
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const int ii = ibase + k * WG + tid;
        float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;
        if (ii < iend) {
            const int src = a.iidx ? a.iidx[ii] : ii;
            r0 = a.ipack[(size_t)src * R + 0];
            r1 = a.ipack[(size_t)src * R + 1];
            if (PREC == 1) r2 = a.ipack[(size_t)src * R + 2];
        }
        ix[k] = r0.x; iy[k] = r0.y; iz[k] = r0.z;
        iu[k] = r1.x; iv[k] = r1.y; iw[k] = r1.z;
        lx[k] = r2.x; ly[k] = r2.y; lz[k] = r2.z;
    }
    // the j index of each i (-1: none) and the nearest-neighbour state
    // (KIND 2): best r^2 and its j.  With eps = 0 the self pair has s = 0
    // and drops out through the s > 0 select, so only the neighbour search
    // needs the index there.
    constexpr bool kSelf = !EPS0 || KIND == 2;
    float bnr[IPT];
    int bnj[IPT], selfk[IPT];
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const int ii = ibase + k * WG + tid;
        bnr[k] = __builtin_inff();
        bnj[k] = -1;
        selfk[k] = (kSelf && ii < iend) ? self_index(a.self_mode, a.iidx, a.iself, ii) : -1;
    }
    // Does the j range [j0, j0 + len) hold the own index of any lane of
    // this wave?  (One compare per i-slot per tile; the answer is uniform
    // over the wave, so the branch it drives does not diverge.)
    auto wave_has_self = [&](int j0, int len) {
        if (EPS0 || a.keep_self) return false;
        bool f = false;
#pragma unroll
        for (int k = 0; k < IPT; ++k) f |= (unsigned)(selfk[k] - j0) < (unsigned)len;
        return __ballot(f) != 0;
    };

    constexpr bool LO_LDS = LOW && PREC == 1;
    float acc[IPT][7];
    float chi[IPT][7], clo[LO_LDS ? 1 : IPT][7];
#pragma unroll
    for (int k = 0; k < IPT; ++k)
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            acc[k][q] = 0.f;
            chi[k][q] = 0.f;
            if (LO_LDS)
                losh[(k * 7 + q) * WG + tid] = 0.f;
            else
                clo[k][q] = 0.f;
        }

    float4 stg[NLD];
    auto load_tile = [&](int t) {
        const int j0 = jb + t * TJ;
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
            const int e = tid + q * WG;
            if (e < NE) {
                const int jj = e / R;
                const int c = e - jj * R;
                if (j0 + jj < je)
                    stg[q] = a.jpack[(size_t)j0 * R + e];
                else
                    stg[q] = c == 0 ? make_float4(kPadPos, kPadPos, kPadPos, 0.f)
                                    : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
    };
    auto store_tile = [&](int buf) {
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
            const int e = tid + q * WG;
            if (e < NE) sh[buf][e] = stg[q];
        }
    };

    // eps^2 lives in a VGPR: an SGPR operand would halve the issue rate of
    // the instruction that reads it
    float eps2v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(eps2v) : "s"(eps2));
    // MASK (a std::integral_constant): the self pair j == selfk[k] gets zero
    // mass, so it contributes exactly nothing to any sum.
    auto interact = [&](auto maskc, const float4& q0, const float4& q1, const float4& q2, int jidx) {
        constexpr bool MASK = decltype(maskc)::value;
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            const float mj = (MASK && !EPS0 && jidx == selfk[k]) ? 0.f : q0.w;
            float dx, dy, dz;
            if (PREC == 1) {
                dx = (q0.x - ix[k]) + (q2.x - lx[k]);
                dy = (q0.y - iy[k]) + (q2.y - ly[k]);
                dz = (q0.z - iz[k]) + (q2.z - lz[k]);
            } else {
                dx = q0.x - ix[k];
                dy = q0.y - iy[k];
                dz = q0.z - iz[k];
            }
            float s;
            if (KIND == 2) {
                const float r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                s = r2 + eps2v;
                const bool better = (r2 < bnr[k]) & (jidx != selfk[k]);
                bnr[k] = better ? r2 : bnr[k];
                bnj[k] = better ? jidx : bnj[k];
            } else {
                s = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2v)));
            }
            float rinv = __builtin_amdgcn_rsqf(s);
            if (EPS0) rinv = s > 0.f ? rinv : 0.f;
            if (KIND == 1) {
                const float mr = mj * rinv;
                const float mr3 = mr * (rinv * rinv);
                acc[k][0] = fmaf(mr3, dx, acc[k][0]);
                acc[k][1] = fmaf(mr3, dy, acc[k][1]);
                acc[k][2] = fmaf(mr3, dz, acc[k][2]);
                acc[k][6] += mr;
                continue;
            }
            const float ux = q1.x - iu[k], uy = q1.y - iv[k], uz = q1.z - iw[k];
            const float rv = fmaf(dz, uz, fmaf(dy, uy, dx * ux));
            const float rinv2 = rinv * rinv;
            const float mr = mj * rinv;
            const float mr3 = mr * rinv2;
            const float al = 3.0f * rv * rinv2;
            acc[k][0] = fmaf(mr3, dx, acc[k][0]);
            acc[k][1] = fmaf(mr3, dy, acc[k][1]);
            acc[k][2] = fmaf(mr3, dz, acc[k][2]);
            acc[k][3] = fmaf(mr3, fmaf(-al, dx, ux), acc[k][3]);
            acc[k][4] = fmaf(mr3, fmaf(-al, dy, uy), acc[k][4]);
            acc[k][5] = fmaf(mr3, fmaf(-al, dz, uz), acc[k][5]);
            acc[k][6] += mr;
        }
    };
    auto fold = [&]() {
        if (PREC == 1) {
#pragma unroll
            for (int k = 0; k < IPT; ++k)
#pragma unroll
                for (int q = 0; q < 7; ++q) {
                    if (LO_LDS) {
                        float lo = losh[(k * 7 + q) * WG + tid];
                        two_sum_fold(chi[k][q], lo, acc[k][q]);
                        losh[(k * 7 + q) * WG + tid] = lo;
                    } else {
                        two_sum_fold(chi[k][q], clo[k][q], acc[k][q]);
                    }
                    acc[k][q] = 0.f;
                }
        }
    };

    const std::integral_constant<bool, false> plain{};
    const std::integral_constant<bool, true> masked{};
    if (JS) {
        // j records read by wave-uniform loads (scalar data cache); chunks of
        // TJ j between compensated folds; no LDS, no barrier
        const float4* __restrict__ jp = a.jpack;
        auto chunk = [&](auto maskc, int j0, int j1) {
            constexpr int U = decltype(maskc)::value ? 1 : UNR;
#pragma unroll U
            for (int j = j0; j < j1; ++j) {
                const float4 q0 = jp[(size_t)j * R + 0];
                const float4 q1 = jp[(size_t)j * R + 1];
                float4 q2 = make_float4(0.f, 0.f, 0.f, 0.f);
                if (PREC == 1) q2 = jp[(size_t)j * R + 2];
                interact(maskc, q0, q1, q2, j);
            }
        };
        for (int j0 = jb; j0 < je; j0 += TJ) {
            const int j1 = min(je, j0 + TJ);
            if (wave_has_self(j0, j1 - j0))
                chunk(masked, j0, j1);
            else
                chunk(plain, j0, j1);
            fold();
        }
    } else {
        // one tile from LDS; jt is the j index of its first record.  The
        // masked copy (rare: the tiles that hold a lane's own index) is a
        // plain loop, so that it never sets the kernel's register count.
        auto sweep = [&](auto maskc, const float4* tile, int jt) {
            constexpr bool MASK = decltype(maskc)::value;
            if (MASK) {
#pragma unroll 1
                for (int jj = 0; jj < TJ; ++jj) {
                    const float4 q0 = tile[jj * R + 0];
                    const float4 q1 = tile[jj * R + 1];
                    float4 q2 = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (PREC == 1) q2 = tile[jj * R + 2];
                    interact(maskc, q0, q1, q2, jt + jj);
                }
            } else if (PIPE) {
                // software pipeline: the record of j+1 is read from LDS while
                // j is being computed
                float4 q0 = tile[0], q1 = tile[1];
                float4 q2 = make_float4(0.f, 0.f, 0.f, 0.f);
                if (PREC == 1) q2 = tile[2];
#pragma unroll UNR
                for (int jj = 0; jj < TJ; ++jj) {
                    const int jn = jj + 1 < TJ ? jj + 1 : jj;
                    const float4 n0 = tile[jn * R + 0];
                    const float4 n1 = tile[jn * R + 1];
                    float4 n2 = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (PREC == 1) n2 = tile[jn * R + 2];
                    interact(maskc, q0, q1, q2, jt + jj);
                    q0 = n0;
                    q1 = n1;
                    q2 = n2;
                }
            } else {
#pragma unroll UNR
                for (int jj = 0; jj < TJ; ++jj) {
                    const float4 q0 = tile[jj * R + 0];
                    const float4 q1 = tile[jj * R + 1];
                    float4 q2 = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (PREC == 1) q2 = tile[jj * R + 2];
                    interact(maskc, q0, q1, q2, jt + jj);
                }
            }
        };
        if (LOW) {
            // single buffer: stage, barrier, sweep, barrier
            for (int t = 0; t < ntiles; ++t) {
                load_tile(t);
                store_tile(0);
                __syncthreads();
                const int jt = jb + t * TJ;
                if (wave_has_self(jt, TJ))
                    sweep(masked, sh[0], jt);
                else
                    sweep(plain, sh[0], jt);
                fold();
                __syncthreads();
            }
        } else {
            if (ntiles > 0) {
                load_tile(0);
                store_tile(0);
            }
            __syncthreads();

            for (int t = 0; t < ntiles; ++t) {
                const int buf = t & 1;
                if (t + 1 < ntiles) load_tile(t + 1);
                const int jt = jb + t * TJ;
                if (wave_has_self(jt, TJ))
                    sweep(masked, sh[buf], jt);
                else
                    sweep(plain, sh[buf], jt);
                fold();
                if (t + 1 < ntiles) store_tile(buf ^ 1);
                __syncthreads();
            }
        }
    }

    // epilogue
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const int ii = ibase + k * WG + tid;
        if (ii >= iend) continue;
        float hi[7], lo[7];
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            hi[q] = PREC == 1 ? chi[k][q] : acc[k][q];
            lo[q] = PREC != 1 ? 0.f : LO_LDS ? losh[(k * 7 + q) * WG + tid] : clo[LO_LDS ? 0 : k][q];
        }
        int nnj = bnj[k];
        float nnr = bnr[k];
        if (nnj >= je) {   // a padding record: this range held no candidate
            nnj = -1;
            nnr = __builtin_inff();
        }
        if (a.partial) {
            const size_t base = (size_t)split * 7 * a.ni + ii;
#pragma unroll
            for (int q = 0; q < 7; ++q)
                if (KIND != 1 || q < 3 || q == 6) a.part[base + (size_t)q * a.ni] = make_float2(hi[q], lo[q]);
            if (KIND == 2) a.nnpart[(size_t)split * a.ni + ii] = make_float2(nnr, __int_as_float(nnj));
        } else {
            const double pot = (double)hi[6] + (double)lo[6];
#pragma unroll
            for (int q = 0; q < 6; ++q)
                if (KIND != 1 || q < 3) a.out[q][ii] = a.G * ((double)hi[q] + (double)lo[q]);
            a.out[6][ii] = -a.G * pot;
            if (KIND == 2) {
                a.nn[ii] = nnj;
                if (a.nn_r2) a.nn_r2[ii] = nnj >= 0 ? (double)nnr : (double)__builtin_inff();
            }
        }
    }
}

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

// ---- block steps: pairwise sums, split reduce and corrector in one launch ----
//
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
template <int PREC, bool EPS0>
__device__ __forceinline__ void jpar_block(const ForceArgs& a, int n_act, int g, int s, int jb, int je,
                                           float* smem) {
    constexpr int R = Rec<PREC>::R;
    constexpr int IG = kJparIG, JPL = kJparJPL, WG = kBlkStepWG;
    float* red = smem;                  // [IG * 6][WG]: high words of the lane sums
    float* losh = smem + IG * 6 * WG;   // [IG * 6][WG]: their low words
    const int tid = threadIdx.x;
    float ix[IG], iy[IG], iz[IG], iu[IG], iv[IG], iw[IG], lx[IG], ly[IG], lz[IG];
#pragma unroll
    for (int k = 0; k < IG; ++k) {
        const int c = g * IG + k;
        float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;
        if (c < n_act) {
            const int src = a.iidx[c];
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
            const float h = (float)f;
            a.part[((size_t)s * 7 + q) * n_act + c] = make_float2(h, (float)(f - (double)h));
        }
    }
}

template <int PREC, bool EPS0>
__global__ __launch_bounds__(kBlkStepWG) __attribute__((amdgpu_waves_per_eu(kBlkStepWaves)))
void blk_step_kernel(ForceArgs a, CorrectArgs ca,
                                                              unsigned* __restrict__ gcnt) {
    constexpr int R = Rec<PREC>::R;
    constexpr int kTileBytes = 2 * kBlkBigTile * R * (int)sizeof(float4);
    constexpr int kRedBytes = 2 * kJparIG * 6 * kBlkStepWG * (int)sizeof(float);
    __shared__ __align__(16) unsigned char smem[kTileBytes > kRedBytes ? kTileBytes : kRedBytes];
    __shared__ double gsum[kJparIG * 6];
    __shared__ int last_sh;
    const DevPlan* pl = a.plan;
    const int n = (int)pl->n_act;
    if (n <= 0) return;
    const int nb = pl->nb, S = pl->S, shape = pl->shape;
    ForceArgs b = a;
    b.ni = n;
    b.jchunk = pl->jchunk;
    b.partial = 1;
    const int tid = threadIdx.x;
    for (int v = blockIdx.x; v < nb * S; v += gridDim.x) {
        const int g = v % nb, s = v / nb;
        const int jb = s * b.jchunk;
        const int je = min(b.nj, jb + b.jchunk);
        int gbeg, gend;
        if (!EPS0 && shape == 1) {
            force_block<PREC, 1, kBlkBigTile, kBlkStepWG, false, false, 2, true>(
                b, reinterpret_cast<float4(*)[kBlkBigTile * R]>(smem), g * kBlkStepWG, n, jb, je, b.eps2, s);
            gbeg = g * kBlkStepWG;
            gend = min(n, gbeg + kBlkStepWG);
        } else {
            jpar_block<PREC, EPS0>(b, n, g, s, jb, je, reinterpret_cast<float*>(smem));
            gbeg = g * kJparIG;
            gend = min(n, gbeg + kJparIG);
        }
        // Every thread's partial stores are made visible device-wide before
        // one thread counts this range in; the work-group that brings the
        // count to S reads every range's partials after an acquire fence.
        __threadfence();
        __syncthreads();
        if (tid == 0) last_sh = atomicAdd(&gcnt[g], 1u) == (unsigned)(S - 1);
        __syncthreads();
        if (last_sh) {
            __threadfence();
            const size_t qs = (size_t)n;
            if (!EPS0 && shape == 1) {
                // one thread per particle, ranges s = 0 .. S-1 in order
                const int c = gbeg + tid;
                if (c < gend) {
                    double f[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                    for (int sp = 0; sp < S; ++sp) {
                        float2 u[6];
#pragma unroll
                        for (int q = 0; q < 6; ++q) u[q] = b.part[((size_t)sp * 7 + q) * qs + c];
#pragma unroll
                        for (int q = 0; q < 6; ++q) {
                            f[q] += (double)u[q].x;
                            f[q] += (double)u[q].y;
                        }
                    }
#pragma unroll
                    for (int q = 0; q < 6; ++q) f[q] *= b.G;
                    correct_core(ca, c, f, f + 3);
                }
            } else {
                // 8 threads per (particle, quantity): ranges s = part, part + 8,
                // ... in order, then a fixed butterfly over the 8
                if (tid < kJparIG * 6 * 8) {
                    const int cq = tid >> 3, part = tid & 7;
                    const int k = cq / 6, q = cq - 6 * (cq / 6);
                    const int c = gbeg + k;
                    double f = 0.0;
                    if (c < gend)
                        for (int sp = part; sp < S; sp += 8) {
                            const float2 u = b.part[((size_t)sp * 7 + q) * qs + c];
                            f += (double)u.x;
                            f += (double)u.y;
                        }
                    f += __shfl_xor(f, 1);
                    f += __shfl_xor(f, 2);
                    f += __shfl_xor(f, 4);
                    if (part == 0) gsum[cq] = b.G * f;
                }
                __syncthreads();
                if (tid < kJparIG && gbeg + tid < gend) {
                    const double* f = gsum + tid * 6;
                    correct_core(ca, gbeg + tid, f, f + 3);
                }
            }
            if (tid == 0) gcnt[g] = 0;   // ready for the next step
        }
        __syncthreads();   // LDS is rewritten by the next item
    }
}

hipError_t launch_blk_step(int prec, bool eps0, const ForceArgs& a, const CorrectArgs& ca, unsigned* gcnt,
                           hipStream_t st) {
    const dim3 g(kBlkGrid), b(kBlkStepWG);
    if (prec == 0) {
        if (eps0)
            hipLaunchKernelGGL((blk_step_kernel<0, true>), g, b, 0, st, a, ca, gcnt);
        else
            hipLaunchKernelGGL((blk_step_kernel<0, false>), g, b, 0, st, a, ca, gcnt);
    } else {
        if (eps0)
            hipLaunchKernelGGL((blk_step_kernel<1, true>), g, b, 0, st, a, ca, gcnt);
        else
            hipLaunchKernelGGL((blk_step_kernel<1, false>), g, b, 0, st, a, ca, gcnt);
    }
    return hipGetLastError();
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

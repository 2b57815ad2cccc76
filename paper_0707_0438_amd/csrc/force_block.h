// The pairwise tile loop (Section 3.1, Fig. 1, re-laid for CDNA4) as a
// device function shared by every kernel that sweeps j records against
// i-particles held in registers: the direct evaluations, the plan-driven
// block-step launches and the batched clusters.  See force.hip for the
// scheme.
#pragma once

#include <type_traits>

#include "nbody_internal.h"

namespace nb {

// Arguments of the pairwise kernel (passed by value).
struct ForceArgs {
    const float4* ipack;    // i records
    const int32_t* iidx;    // i -> record index in ipack (NULL: identity)
    int ni;
    const float4* jpack;    // j records
    int nj;
    int jchunk;             // j per split (multiple of the tile)
    float eps2;             // eps^2 rounded to float
    int partial;            // 0: final float64 outputs, 1: write split partials
    double G;
    const int32_t* iself;   // self j index per i (used when self_mode == 0; NULL: none)
    int self_mode;          // 0: iself[i], 1: iidx[i], 2: i itself
    int keep_self;          // 1: the self pair is not masked (its i row is a copy of its j
                            //    row, so a and jerk get exactly 0; the potential row is unused)
    double* out[7];         // ax ay az jx jy jz pot (final mode)
    float2* part;           // [S][7][ni] (hi, lo) partials (partial mode)
    const DevPlan* plan;    // plan-driven launch: ni, S, jchunk come from here
    int32_t* nn;            // nearest-neighbour evaluation: j index per i (final mode)
    double* nn_r2;          //   and its squared distance (final mode; NULL: not wanted)
    float2* nnpart;         //   [S][ni] (r^2, j bits) per range (partial mode)
};

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

}  // namespace nb

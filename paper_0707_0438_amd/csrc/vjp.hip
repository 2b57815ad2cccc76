// Adjoint (vector-Jacobian product) of the pairwise acceleration / jerk /
// potential sums with respect to positions, velocities and masses.
//
// Forward (Eq. 1 with Plummer softening, Section 3.3; jerk and potential,
// Section 3), per pair (i <- j), r = x_j - x_i, u = v_j - v_i,
// s = r.r + eps^2, A = s^-1/2, B = A^3, C = A^5:
//   a_i += G m_j B r,  jerk_i += G m_j (B u - 3C (r.u) r),  phi_i -= G m_j A.
// For output cotangents (ga_i, gj_i, gp_i) the pair contributes
//   g_r = G m_j [B ga - P r - 3C (gj.r) u - 3C (r.u) gj],
//         P = 3C (ga.r + gj.u - 5 (r.u)(gj.r)/s) - gp B,
//   g_u = G m_j [B gj - 3C (gj.r) r],
//   dL/dm_j = G [B (ga.r + gj.u) - 3C (r.u)(gj.r) - gp A],
// and x_j gets +g_r, x_i gets -g_r (v likewise); m_j gets dL/dm_j.
//
// One kernel serves three launch forms.  A lane holds particle k, the LDS
// tile holds particles p, and the pair geometry uses r = x_p - x_k:
//  * OWN     (lane = i, tile = j): the lane's own cotangents, partner mass;
//  * PARTNER (lane = j, tile = i): the tile's cotangents, the lane's mass;
//  * both at once when the i set and the j set are the same particles.
// Per-lane constant factors are pulled out of the sums (ga_k, gj_k enter
// only through the scalar sums sB = sum m_p B and sC = sum 3 m_p C (r.u)).
// A pair whose keys match (the self pair) or whose s is 0 contributes
// nothing.  Float32 pair arithmetic on double-single relative coordinates,
// per-tile partial sums folded into (hi, lo) two-sum accumulators.
#include "nbody_internal.h"

namespace nb {

constexpr int kVjpTile = 64;
constexpr int kVjpWG = 256;
constexpr int kVjpAcc = 9;   // X(3) V(3) M sB sC

__device__ __forceinline__ void two_sum_fold_v(float& hi, float& lo, float p) {
    const float s = hi + p;
    const float bb = s - hi;
    const float e = (hi - (s - bb)) + (p - bb);
    hi = s;
    lo += e;
}

// Record: {x_hi, y_hi, z_hi, m}, {vx, vy, vz, gp}, {x_lo, y_lo, z_lo, key},
//         {gax, gay, gaz, 0}, {gjx, gjy, gjz, 0}.
__global__ __launch_bounds__(256) void vjp_pack_kernel(VjpPackArgs a) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    const double px = a.x[k], py = a.y[k], pz = a.z[k];
    const float hx = (float)px, hy = (float)py, hz = (float)pz;
    float lx = 0.f, ly = 0.f, lz = 0.f;
    if (a.prec == 1) {
        lx = (float)(px - (double)hx);
        ly = (float)(py - (double)hy);
        lz = (float)(pz - (double)hz);
    }
    int key = k;
    if (a.key_mode == 1) key = a.iself ? (a.iself[k] >= 0 ? a.iself[k] : -1) : -1;
    const size_t n = (size_t)a.n;
    float4* o = a.out + 5 * (size_t)k;
    o[0] = make_float4(hx, hy, hz, a.m ? (float)a.m[k] : 0.f);
    o[1] = make_float4((float)a.vx[k], (float)a.vy[k], (float)a.vz[k], a.gp ? (float)a.gp[k] : 0.f);
    o[2] = make_float4(lx, ly, lz, __int_as_float(key));
    o[3] = a.ga ? make_float4((float)a.ga[k], (float)a.ga[n + k], (float)a.ga[2 * n + k], 0.f)
                : make_float4(0.f, 0.f, 0.f, 0.f);
    o[4] = a.gj ? make_float4((float)a.gj[k], (float)a.gj[n + k], (float)a.gj[2 * n + k], 0.f)
                : make_float4(0.f, 0.f, 0.f, 0.f);
}

hipError_t launch_vjp_pack(const VjpPackArgs& a, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(vjp_pack_kernel, dim3((a.n + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

// Final combination in float64: x_bar = G (X - ga sB + gj sC),
// v_bar = G (V - gj sB), m_bar = G M, from the lane's float64 cotangents.
__device__ __forceinline__ void vjp_finish(const VjpArgs& a, int k, const double v[kVjpAcc]) {
    const size_t n = (size_t)a.nl;
    double ga[3] = {0, 0, 0}, gj[3] = {0, 0, 0};
    if (a.own) {
        if (a.ga) { ga[0] = a.ga[k]; ga[1] = a.ga[n + k]; ga[2] = a.ga[2 * n + k]; }
        if (a.gj) { gj[0] = a.gj[k]; gj[1] = a.gj[n + k]; gj[2] = a.gj[2 * n + k]; }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (a.gx) a.gx[c * n + k] = a.G * (v[c] - ga[c] * v[7] + gj[c] * v[8]);
        if (a.gv) a.gv[c * n + k] = a.G * (v[3 + c] - gj[c] * v[7]);
    }
    if (a.gm) a.gm[k] = a.G * v[6];
}

template <int PREC, bool OWN, bool PARTNER>
__global__ __launch_bounds__(kVjpWG) void vjp_kernel(VjpArgs a) {
    constexpr int R = 5;
    constexpr int NE = kVjpTile * R;
    constexpr int NLD = (NE + kVjpWG - 1) / kVjpWG;
    __shared__ float4 sh[2][NE];

    const int tid = threadIdx.x;
    const int k = blockIdx.x * kVjpWG + tid;
    const int jb = blockIdx.y * a.jchunk;
    const int je = min(a.nt, jb + a.jchunk);
    const int ntiles = je > jb ? (je - jb + kVjpTile - 1) / kVjpTile : 0;

    float4 L0 = make_float4(0.f, 0.f, 0.f, 0.f), L1 = L0, L2 = L0, L3 = L0, L4 = L0;
    if (k < a.nl) {
        const float4* lr = a.lrec + (size_t)k * R;
        L0 = lr[0]; L1 = lr[1]; L2 = lr[2]; L3 = lr[3]; L4 = lr[4];
    } else {
        L2.w = __int_as_float(-7);   // never equal to a tile key
    }
    const int lkey = __float_as_int(L2.w);
    const float mk = L0.w;

    float acc[kVjpAcc], hi[kVjpAcc], lo[kVjpAcc];
#pragma unroll
    for (int q = 0; q < kVjpAcc; ++q) { acc[q] = 0.f; hi[q] = 0.f; lo[q] = 0.f; }

    float4 stg[NLD];
    auto load_tile = [&](int t) {
        const int j0 = jb + t * kVjpTile;
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
            const int e = tid + q * kVjpWG;
            if (e < NE) {
                const int jj = e / R;
                const int c = e - jj * R;
                if (j0 + jj < je) {
                    stg[q] = a.trec[(size_t)j0 * R + e];
                } else {
                    // massless, cotangent-free, far away, key that matches nothing
                    stg[q] = c == 0 ? make_float4(1.0e18f, 1.0e18f, 1.0e18f, 0.f)
                           : c == 2 ? make_float4(0.f, 0.f, 0.f, __int_as_float(-9))
                                    : make_float4(0.f, 0.f, 0.f, 0.f);
                }
            }
        }
    };
    auto store_tile = [&](int buf) {
#pragma unroll
        for (int q = 0; q < NLD; ++q) {
            const int e = tid + q * kVjpWG;
            if (e < NE) sh[buf][e] = stg[q];
        }
    };

    // eps^2 in a VGPR: an SGPR operand halves the issue rate of its instruction
    float eps2;
    asm volatile("v_mov_b32 %0, %1" : "=v"(eps2) : "s"(a.eps2));
    if (ntiles > 0) {
        load_tile(0);
        store_tile(0);
    }
    __syncthreads();
    for (int t = 0; t < ntiles; ++t) {
        const int buf = t & 1;
        if (t + 1 < ntiles) load_tile(t + 1);
        const float4* tile = sh[buf];
#pragma unroll 2
        for (int jj = 0; jj < kVjpTile; ++jj) {
            const float4 P0 = tile[jj * R + 0], P1 = tile[jj * R + 1], P2 = tile[jj * R + 2];
            float dx, dy, dz;
            if (PREC == 1) {
                dx = (P0.x - L0.x) + (P2.x - L2.x);
                dy = (P0.y - L0.y) + (P2.y - L2.y);
                dz = (P0.z - L0.z) + (P2.z - L2.z);
            } else {
                dx = P0.x - L0.x;
                dy = P0.y - L0.y;
                dz = P0.z - L0.z;
            }
            const float ux = P1.x - L1.x, uy = P1.y - L1.y, uz = P1.z - L1.z;
            const float s = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
            const bool live = (s > 0.f) && (__float_as_int(P2.w) != lkey);
            const float A = live ? __builtin_amdgcn_rsqf(s) : 0.f;
            const float q = A * A;
            const float B = A * q;
            const float C3 = 3.0f * B * q;
            const float ru = fmaf(dz, uz, fmaf(dy, uy, dx * ux));
            const float qru5 = 5.0f * q * ru;
            const float C3ru = C3 * ru;
            float cr = 0.f, cu = 0.f;
            if (OWN) {
                const float mp = P0.w;
                const float gar = fmaf(L3.z, dz, fmaf(L3.y, dy, L3.x * dx));
                const float gjr = fmaf(L4.z, dz, fmaf(L4.y, dy, L4.x * dx));
                const float gju = fmaf(L4.z, uz, fmaf(L4.y, uy, L4.x * ux));
                const float Pk = C3 * fmaf(-qru5, gjr, gar + gju);
                cr = mp * fmaf(-L1.w, B, Pk);
                cu = mp * (C3 * gjr);
                acc[7] = fmaf(mp, B, acc[7]);
                acc[8] = fmaf(mp, C3ru, acc[8]);
            }
            if (PARTNER) {
                const float4 P3 = tile[jj * R + 3], P4 = tile[jj * R + 4];
                const float garp = fmaf(P3.z, dz, fmaf(P3.y, dy, P3.x * dx));
                const float gjrp = fmaf(P4.z, dz, fmaf(P4.y, dy, P4.x * dx));
                const float gjup = fmaf(P4.z, uz, fmaf(P4.y, uy, P4.x * ux));
                const float sp = garp + gjup;
                const float Pp = C3 * fmaf(-qru5, gjrp, sp);
                cr = fmaf(-mk, fmaf(P1.w, B, Pp), cr);
                cu = fmaf(-mk, C3 * gjrp, cu);
                const float bk = mk * B;
                const float ck = -mk * C3ru;
                acc[0] = fmaf(bk, P3.x, acc[0]);
                acc[1] = fmaf(bk, P3.y, acc[1]);
                acc[2] = fmaf(bk, P3.z, acc[2]);
                acc[0] = fmaf(ck, P4.x, acc[0]);
                acc[1] = fmaf(ck, P4.y, acc[1]);
                acc[2] = fmaf(ck, P4.z, acc[2]);
                acc[3] = fmaf(bk, P4.x, acc[3]);
                acc[4] = fmaf(bk, P4.y, acc[4]);
                acc[5] = fmaf(bk, P4.z, acc[5]);
                acc[6] = fmaf(-B, sp, acc[6]);
                acc[6] = fmaf(C3ru, gjrp, acc[6]);
                acc[6] = fmaf(-P1.w, A, acc[6]);
            }
            acc[0] = fmaf(cr, dx, fmaf(cu, ux, acc[0]));
            acc[1] = fmaf(cr, dy, fmaf(cu, uy, acc[1]));
            acc[2] = fmaf(cr, dz, fmaf(cu, uz, acc[2]));
            acc[3] = fmaf(cu, dx, acc[3]);
            acc[4] = fmaf(cu, dy, acc[4]);
            acc[5] = fmaf(cu, dz, acc[5]);
        }
#pragma unroll
        for (int q = 0; q < kVjpAcc; ++q) {
            two_sum_fold_v(hi[q], lo[q], acc[q]);
            acc[q] = 0.f;
        }
        if (t + 1 < ntiles) store_tile(buf ^ 1);
        __syncthreads();
    }

    if (k >= a.nl) return;
    if (a.part) {
        const size_t base = (size_t)blockIdx.y * kVjpAcc * a.nl + k;
#pragma unroll
        for (int q = 0; q < kVjpAcc; ++q) a.part[base + (size_t)q * a.nl] = make_float2(hi[q], lo[q]);
    } else {
        double v[kVjpAcc];
#pragma unroll
        for (int q = 0; q < kVjpAcc; ++q) v[q] = (double)hi[q] + (double)lo[q];
        vjp_finish(a, k, v);
    }
}

__global__ __launch_bounds__(256) void vjp_reduce_kernel(VjpArgs a, int S) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.nl) return;
    double v[kVjpAcc];
#pragma unroll
    for (int q = 0; q < kVjpAcc; ++q) {
        double s = 0.0;
        for (int sp = 0; sp < S; ++sp) {
            const float2 p = a.part[((size_t)sp * kVjpAcc + q) * a.nl + k];
            s += (double)p.x;
            s += (double)p.y;
        }
        v[q] = s;
    }
    vjp_finish(a, k, v);
}

template <int PREC, bool OWN, bool PARTNER>
static void vjp_launch_t(int nb, int S, const VjpArgs& a, hipStream_t st) {
    hipLaunchKernelGGL((vjp_kernel<PREC, OWN, PARTNER>), dim3(nb, S), dim3(kVjpWG), 0, st, a);
}

hipError_t launch_vjp(int prec, bool own, bool partner, int S, const VjpArgs& a, hipStream_t st) {
    if (a.nl <= 0) return hipSuccess;
    const int nb = (a.nl + kVjpWG - 1) / kVjpWG;
    if (prec == 0) {
        if (own && partner) vjp_launch_t<0, true, true>(nb, S, a, st);
        else if (own) vjp_launch_t<0, true, false>(nb, S, a, st);
        else vjp_launch_t<0, false, true>(nb, S, a, st);
    } else {
        if (own && partner) vjp_launch_t<1, true, true>(nb, S, a, st);
        else if (own) vjp_launch_t<1, true, false>(nb, S, a, st);
        else vjp_launch_t<1, false, true>(nb, S, a, st);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !a.part) return e;
    hipLaunchKernelGGL(vjp_reduce_kernel, dim3((a.nl + 255) / 256), dim3(256), 0, st, a, S);
    return hipGetLastError();
}

int vjp_tile() { return kVjpTile; }
int vjp_wg() { return kVjpWG; }
int vjp_acc() { return kVjpAcc; }

}  // namespace nb

// Kick-drift-kick leapfrog on the force-only evaluation.
//
// Section 4 drives the library from a treecode, which integrates with the
// acceleration alone, so the jerk (and nearest-neighbour) work is switched
// off.  The matching direct-summation integrator is the second-order
// kick-drift-kick leapfrog:
//   v_h = v_0 + a_0 dt/2,  x_1 = x_0 + v_h dt,  a_1 = a(x_1),  v_1 = v_h + a_1 dt/2.
// The first kick and the drift are fused with the packing of the new
// positions into j records; the force evaluation between the two kernels is
// the KIND 1 pairwise kernel.  State is float64 rows of n: x, y, z (and
// likewise v, a), updated in place.
#include "nbody_internal.h"

namespace nb {

template <int PREC>
__global__ __launch_bounds__(256) void lf_kick_drift_pack_kernel(int n, double* __restrict__ x,
                                                                 double* __restrict__ v,
                                                                 const double* __restrict__ acc,
                                                                 const double* __restrict__ m, double h, double dt,
                                                                 float4* __restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double p[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const size_t o = (size_t)c * n + k;
        const double vh = v[o] + acc[o] * h;
        v[o] = vh;
        p[c] = x[o] + vh * dt;
        x[o] = p[c];
    }
    const float mk = (float)m[k];
    const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
    if (PREC == 0) {
        out[2 * (size_t)k] = make_float4((float)p[0], (float)p[1], (float)p[2], mk);
        out[2 * (size_t)k + 1] = zero;
    } else {
        const float hx = (float)p[0], hy = (float)p[1], hz = (float)p[2];
        out[3 * (size_t)k] = make_float4(hx, hy, hz, mk);
        out[3 * (size_t)k + 1] = zero;
        out[3 * (size_t)k + 2] = make_float4((float)(p[0] - (double)hx), (float)(p[1] - (double)hy),
                                             (float)(p[2] - (double)hz), 0.f);
    }
}

__global__ __launch_bounds__(256) void lf_kick_kernel(int64_t n3, double* __restrict__ v,
                                                      const double* __restrict__ acc, double h) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n3) v[k] += acc[k] * h;
}

hipError_t launch_lf_kick_drift_pack(int prec, int n, double* x, double* v, const double* acc, const double* m,
                                     double h, double dt, float4* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const dim3 g((n + 255) / 256), b(256);
    if (prec == 0)
        hipLaunchKernelGGL(lf_kick_drift_pack_kernel<0>, g, b, 0, st, n, x, v, acc, m, h, dt, out);
    else
        hipLaunchKernelGGL(lf_kick_drift_pack_kernel<1>, g, b, 0, st, n, x, v, acc, m, h, dt, out);
    return hipGetLastError();
}

hipError_t launch_lf_kick(int n, double* v, const double* acc, double h, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t n3 = 3 * (int64_t)n;
    hipLaunchKernelGGL(lf_kick_kernel, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, st, n3, v, acc, h);
    return hipGetLastError();
}

}  // namespace nb

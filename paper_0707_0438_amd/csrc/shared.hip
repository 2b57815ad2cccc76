// Shared-step Hermite integration of one self-gravitating set and its
// adjoint (float64 elementwise kernels; the forces and their adjoint come
// from force.hip and vjp.hip).
//
// Forward step over D (Section 3, Makino & Aarseth 1992 scheme):
//   x_p = x + v D + a D^2/2 + j D^3/6,  v_p = v + a D + j D^2/2
//   (a1, j1) = F(x_p, v_p, m)
//   a2 = (-6 (a - a1) - D (4 j + 2 j1)) / D^2,  a3 = (12 (a - a1) + 6 D (j + j1)) / D^3
//   x <- x_p + a2 D^4/24 + a3 D^5/120,  v <- v_p + a2 D^3/6 + a3 D^4/24,  a <- a1, j <- j1
// Backward step, for cotangents (X, V, Aa, Jj) of (x, v, a, j) after the step:
//   P2 = X D^4/24 + V D^3/6,  P3 = X D^5/120 + V D^4/24
//   force cotangents: ga = Aa + 6 P2/D^2 - 12 P3/D^3,  gj = Jj - 2 P2/D + 6 P3/D^2
//   (tx, tv, tm) = adjoint of F at (x_p, v_p, m) for (ga, gj)
//   gx_p = X + tx, gv_p = V + tv
//   X <- gx_p,  V <- D gx_p + gv_p,
//   Aa <- -6 P2/D^2 + 12 P3/D^3 + D^2/2 gx_p + D gv_p,
//   Jj <- -4 P2/D + 6 P3/D^2 + D^3/6 gx_p + D^2/2 gv_p.
// Vector fields are [3][n] float64 rows (one pointer, row stride n).
#include "nbody_internal.h"

namespace nb {

__global__ __launch_bounds__(256) void shared_predict_kernel(int n3, double D, const double* __restrict__ x,
                                                             const double* __restrict__ v,
                                                             const double* __restrict__ a,
                                                             const double* __restrict__ j,
                                                             double* __restrict__ xp, double* __restrict__ vp) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n3) return;
    predict1(x[q], v[q], a[q], j[q], D, xp[q], vp[q]);
}

__global__ __launch_bounds__(256) void shared_correct_kernel(int n3, double D, const double* __restrict__ xp,
                                                             const double* __restrict__ vp, double* x,
                                                             double* v, double* a, double* j,
                                                             const double* __restrict__ a1,
                                                             const double* __restrict__ j1) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n3) return;
    const double iD = 1.0 / D, iD2 = iD * iD, iD3 = iD2 * iD;
    const double da = a[q] - a1[q];
    const double a2 = (-6.0 * da - D * (4.0 * j[q] + 2.0 * j1[q])) * iD2;
    const double a3 = (12.0 * da + 6.0 * D * (j[q] + j1[q])) * iD3;
    const double D3 = D * D * D, D4 = D3 * D;
    x[q] = xp[q] + D4 * (a2 * (1.0 / 24.0) + D * a3 * (1.0 / 120.0));
    v[q] = vp[q] + D3 * (a2 * (1.0 / 6.0) + D * a3 * (1.0 / 24.0));
    a[q] = a1[q];
    j[q] = j1[q];
}

__global__ __launch_bounds__(256) void adj_correct_kernel(int n3, double D, const double* __restrict__ X,
                                                          const double* __restrict__ V, double* Aa,
                                                          double* Jj, double* __restrict__ ga,
                                                          double* __restrict__ gj) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n3) return;
    const double D2 = D * D, D3 = D2 * D, D4 = D3 * D, D5 = D4 * D;
    const double P2 = X[q] * (D4 / 24.0) + V[q] * (D3 / 6.0);
    const double P3 = X[q] * (D5 / 120.0) + V[q] * (D4 / 24.0);
    ga[q] = Aa[q] + 6.0 * P2 / D2 - 12.0 * P3 / D3;
    gj[q] = Jj[q] - 2.0 * P2 / D + 6.0 * P3 / D2;
    Aa[q] = -6.0 * P2 / D2 + 12.0 * P3 / D3;
    Jj[q] = -4.0 * P2 / D + 6.0 * P3 / D2;
}

__global__ __launch_bounds__(256) void adj_predict_kernel(int n3, double D, double* X, double* V, double* Aa,
                                                          double* Jj, const double* __restrict__ tx,
                                                          const double* __restrict__ tv) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n3) return;
    const double gxp = X[q] + tx[q], gvp = V[q] + tv[q];
    X[q] = gxp;
    V[q] = D * gxp + gvp;
    Aa[q] += (D * D / 2.0) * gxp + D * gvp;
    Jj[q] += (D * D * D / 6.0) * gxp + (D * D / 2.0) * gvp;
}

__global__ __launch_bounds__(256) void axpy_kernel(int n, double* y, const double* __restrict__ x) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) y[q] += x[q];
}

__global__ __launch_bounds__(256) void sum2_kernel(int n, double* out, const double* __restrict__ a,
                                                   const double* __restrict__ b) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) out[q] = a[q] + b[q];
}

__global__ __launch_bounds__(256) void fill_f64_kernel(int n, double* y, double v) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) y[q] = v;
}

static dim3 grid(int n) { return dim3((n + 255) / 256); }

hipError_t launch_shared_predict(int n, double D, const double* x, const double* v, const double* a,
                                 const double* j, double* xp, double* vp, hipStream_t st) {
    hipLaunchKernelGGL(shared_predict_kernel, grid(3 * n), dim3(256), 0, st, 3 * n, D, x, v, a, j, xp, vp);
    return hipGetLastError();
}
hipError_t launch_shared_correct(int n, double D, const double* xp, const double* vp, double* x, double* v,
                                 double* a, double* j, const double* a1, const double* j1, hipStream_t st) {
    hipLaunchKernelGGL(shared_correct_kernel, grid(3 * n), dim3(256), 0, st, 3 * n, D, xp, vp, x, v, a, j, a1, j1);
    return hipGetLastError();
}
hipError_t launch_adj_correct(int n, double D, const double* X, const double* V, double* Aa, double* Jj,
                              double* ga, double* gj, hipStream_t st) {
    hipLaunchKernelGGL(adj_correct_kernel, grid(3 * n), dim3(256), 0, st, 3 * n, D, X, V, Aa, Jj, ga, gj);
    return hipGetLastError();
}
hipError_t launch_adj_predict(int n, double D, double* X, double* V, double* Aa, double* Jj, const double* tx,
                              const double* tv, hipStream_t st) {
    hipLaunchKernelGGL(adj_predict_kernel, grid(3 * n), dim3(256), 0, st, 3 * n, D, X, V, Aa, Jj, tx, tv);
    return hipGetLastError();
}
hipError_t launch_axpy(int n, double* y, const double* x, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(axpy_kernel, grid(n), dim3(256), 0, st, n, y, x);
    return hipGetLastError();
}
hipError_t launch_sum2(int n, double* out, const double* a, const double* b, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(sum2_kernel, grid(n), dim3(256), 0, st, n, out, a, b);
    return hipGetLastError();
}
hipError_t launch_fill_f64(int n, double* y, double v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_f64_kernel, grid(n), dim3(256), 0, st, n, y, v);
    return hipGetLastError();
}

}  // namespace nb

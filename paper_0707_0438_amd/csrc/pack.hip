// Conversion of float64 particle rows into the float32 j records of the
// pairwise kernel (Section 3: the GPU works on single-precision particle
// data), optionally predicting every particle to the block time first
// (the Hermite predictor of Section 3, run for all j on the device), and the
// float64 prediction of all particles for the energy diagnostic.
#include "nbody_internal.h"

namespace nb {

template <int PREC>
__global__ __launch_bounds__(256) void pack_kernel(PackArgs a) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    pack_one<PREC>(a, k, a.t ? (a.tnext ? *a.tnext : a.tn) : 0);
}

hipError_t launch_pack(const PackArgs& a, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    const dim3 g((a.n + 255) / 256), b(256);
    if (a.prec == 0)
        hipLaunchKernelGGL(pack_kernel<0>, g, b, 0, st, a);
    else
        hipLaunchKernelGGL(pack_kernel<1>, g, b, 0, st, a);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void predict_all_kernel(int n, const double* __restrict__ x,
                                                          const double* __restrict__ y,
                                                          const double* __restrict__ z,
                                                          const double* __restrict__ vx,
                                                          const double* __restrict__ vy,
                                                          const double* __restrict__ vz,
                                                          const double* __restrict__ ax,
                                                          const double* __restrict__ ay,
                                                          const double* __restrict__ az,
                                                          const double* __restrict__ jx,
                                                          const double* __restrict__ jy,
                                                          const double* __restrict__ jz,
                                                          const int64_t* __restrict__ t,
                                                          const int64_t* __restrict__ tnext,
                                                          double* ox, double* oy, double* oz,
                                                          double* ovx, double* ovy, double* ovz) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double D = (double)(*tnext - t[k]) * kTick;
    predict1(x[k], vx[k], ax[k], jx[k], D, ox[k], ovx[k]);
    predict1(y[k], vy[k], ay[k], jy[k], D, oy[k], ovy[k]);
    predict1(z[k], vz[k], az[k], jz[k], D, oz[k], ovz[k]);
}

hipError_t launch_predict_all(int n, const double* const* s, const int64_t* t, const int64_t* tnext,
                              double* const* o, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(predict_all_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, s[0], s[1],
                       s[2], s[3], s[4], s[5], s[6], s[7], s[8], s[9], s[10], s[11], t, tnext, o[0],
                       o[1], o[2], o[3], o[4], o[5]);
    return hipGetLastError();
}

// Debug check of the self-pair contract: for every i with a self index s,
// the i record's position and velocity words must equal those of j record s
// bit for bit (the tile loop visits the pair and relies on it giving exactly
// zero).  Counts offending rows, and self indices beyond the j set.
__global__ __launch_bounds__(256) void self_check_kernel(int ni, int nj, int R, const float4* __restrict__ ip,
                                                         const int32_t* __restrict__ iself,
                                                         const float4* __restrict__ jp, int* __restrict__ bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ni) return;
    const int s = iself[i];
    if (s < 0) return;
    bool ok = s < nj;
    for (int r = 0; ok && r < R; ++r) {
        const float4 a = ip[(size_t)i * R + r], b = jp[(size_t)s * R + r];
        ok = __float_as_uint(a.x) == __float_as_uint(b.x) && __float_as_uint(a.y) == __float_as_uint(b.y) &&
             __float_as_uint(a.z) == __float_as_uint(b.z);
    }
    if (!ok) atomicAdd(bad, 1);
}

hipError_t launch_self_check(int ni, int nj, int prec, const float4* ip, const int32_t* iself, const float4* jp,
                             int* bad, hipStream_t st) {
    hipError_t e = launch_fill_i32(bad, 1, 0, st);
    if (e != hipSuccess || ni <= 0) return e;
    hipLaunchKernelGGL(self_check_kernel, dim3((ni + 255) / 256), dim3(256), 0, st, ni, nj,
                       prec == 0 ? kRecFP32 : kRecDS, ip, iself, jp, bad);
    return hipGetLastError();
}

}  // namespace nb

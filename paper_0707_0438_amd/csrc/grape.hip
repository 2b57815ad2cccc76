// GRAPE-6-style interface (Appendix A) on top of the library's C ABI.
//
// A cluster owns a library context, a non-blocking stream (default
// priority), host staging for the j-particles, device rows for the raw and
// the predicted j data, device and pinned host rows for one group of
// i-particles and its results.  GPU_set_ti sends the j data changed since
// the last call and predicts every j to the requested time in float64;
// GPUcalc_firsthalf sends the i group, substitutes the predicted j data of
// every i that is also a j (so that particle's pair with itself is
// bit-identical and contributes nothing), and enqueues nbody_force_nn (or
// nbody_force) plus the copies of the results into pinned memory;
// GPUcalc_lasthalf waits and scatters them into the caller's arrays.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "nbody.h"
#include "nbody_grape.h"
#include "nbody_internal.h"

namespace {

constexpr int kRaw = 14;           // j rows: x y z vx vy vz ax ay az jx jy jz m tj
constexpr int kPred = 6;           // predicted x y z vx vy vz
constexpr double kFar = 1.0e18;    // position of an unset j address (massless, never nearest)

__global__ __launch_bounds__(256) void grape_predict_kernel(int n, int64_t cap, const double* __restrict__ raw,
                                                            double ti, double* __restrict__ pred) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double D = ti - raw[13 * cap + k];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double xp, vp;
        nb::predict1(raw[c * cap + k], raw[(3 + c) * cap + k], raw[(6 + c) * cap + k], raw[(9 + c) * cap + k], D,
                     xp, vp);
        pred[c * cap + k] = xp;
        pred[(3 + c) * cap + k] = vp;
    }
}

// i rows of i-particles that are j-particles: the predicted j rows.
__global__ __launch_bounds__(256) void grape_gather_kernel(int ni, int64_t icap, const int32_t* __restrict__ addr,
                                                           int64_t cap, const double* __restrict__ pred,
                                                           double* __restrict__ irows) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ni) return;
    const int a = addr[k];
    if (a < 0) return;
#pragma unroll
    for (int c = 0; c < kPred; ++c) irows[c * icap + k] = pred[c * cap + a];
}

struct Slot {
    bool open = false;
    nbody_ctx* ctx = nullptr;
    hipStream_t st = nullptr;
    std::string err;
    int prec = NBODY_PREC_DS_COMP;
    bool nn = true;
    // host staging of the j set
    int64_t hcap = 0, nset = 0;
    std::vector<double> hj;              // kRaw rows of hcap
    std::vector<int> hindex;             // identity per address (-1: unset)
    std::unordered_map<int, int> addr_of;
    int64_t dirty_lo = 0, dirty_hi = 0;  // [lo, hi) changed since the last upload
    bool need_ti = false;
    // device j rows: kRaw raw + kPred predicted, each of dcap
    int64_t dcap = 0;
    double* dj = nullptr;
    // i group: device rows 6 in + 7 out; int rows addr, nn; pinned mirrors
    int64_t icap = 0;
    double* di = nullptr;
    int32_t* dint = nullptr;
    double* pin = nullptr;
    int32_t* pint = nullptr;
    bool pending = false;
    int pend_ni = 0;
    bool pend_nn = false;
};

Slot g_slot[NBODY_GRAPE_MAX_CLUSTERS];

int fail(Slot& s, int code, const std::string& what) {
    s.err = what;
    return code;
}

int lib_fail(Slot& s, int code, const char* what) {
    s.err = std::string(what) + ": " + (s.ctx ? nbody_last_error(s.ctx) : "");
    return code;
}

int hip_fail(Slot& s, hipError_t e, const char* what) {
    (void)hipGetLastError();
    s.err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? NBODY_ERR_NOMEM : NBODY_ERR_DEVICE;
}

Slot* slot(int id) {
    if (id < 0 || id >= NBODY_GRAPE_MAX_CLUSTERS) return nullptr;
    return &g_slot[id];
}

void free_device(Slot& s) {
    if (s.dj) (void)hipFree(s.dj);
    if (s.di) (void)hipFree(s.di);
    if (s.dint) (void)hipFree(s.dint);
    if (s.pin) (void)hipHostFree(s.pin);
    if (s.pint) (void)hipHostFree(s.pint);
    s.dj = nullptr;
    s.di = nullptr;
    s.dint = nullptr;
    s.pin = nullptr;
    s.pint = nullptr;
    s.dcap = s.icap = 0;
}

void host_grow(Slot& s, int64_t need) {
    if (need <= s.hcap) return;
    int64_t cap = s.hcap > 0 ? s.hcap : 1024;
    while (cap < need) cap *= 2;
    std::vector<double> nh((size_t)kRaw * cap, 0.0);
    for (int r = 0; r < kRaw; ++r)
        if (s.hcap) std::memcpy(&nh[(size_t)r * cap], &s.hj[(size_t)r * s.hcap], sizeof(double) * s.hcap);
    for (int64_t k = s.hcap; k < cap; ++k)
        for (int c = 0; c < 3; ++c) nh[(size_t)c * cap + k] = kFar;
    s.hj.swap(nh);
    s.hindex.resize(cap, -1);
    s.hcap = cap;
}

int device_j(Slot& s) {
    if (s.nset <= s.dcap) return NBODY_OK;
    hipError_t e = hipStreamSynchronize(s.st);
    if (e != hipSuccess) return hip_fail(s, e, "stream sync");
    if (s.dj) (void)hipFree(s.dj);
    s.dj = nullptr;
    s.dcap = 0;
    e = hipMalloc(&s.dj, sizeof(double) * (kRaw + kPred) * (size_t)s.hcap);
    if (e != hipSuccess) return hip_fail(s, e, "j buffers");
    s.dcap = s.hcap;
    s.dirty_lo = 0;
    s.dirty_hi = s.nset;
    return NBODY_OK;
}

int device_i(Slot& s, int ni) {
    if (ni <= s.icap) return NBODY_OK;
    hipError_t e = hipStreamSynchronize(s.st);
    if (e != hipSuccess) return hip_fail(s, e, "stream sync");
    if (s.di) (void)hipFree(s.di);
    if (s.dint) (void)hipFree(s.dint);
    if (s.pin) (void)hipHostFree(s.pin);
    if (s.pint) (void)hipHostFree(s.pint);
    s.di = nullptr;
    s.dint = nullptr;
    s.pin = nullptr;
    s.pint = nullptr;
    s.icap = 0;
    int64_t cap = 256;
    while (cap < ni) cap *= 2;
    e = hipMalloc(&s.di, sizeof(double) * 13 * (size_t)cap);
    if (e == hipSuccess) e = hipMalloc(&s.dint, sizeof(int32_t) * 2 * (size_t)cap);
    if (e == hipSuccess) e = hipHostMalloc(&s.pin, sizeof(double) * 13 * (size_t)cap, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&s.pint, sizeof(int32_t) * 2 * (size_t)cap, hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(s, e, "i buffers");
    s.icap = cap;
    return NBODY_OK;
}

bool finite3(const double* v) { return v && std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

int collect(int clusterid, int ni, double acc[][3], double jerk[][3], double pot[], int nnb[]) {
    Slot* sp = slot(clusterid);
    if (!sp || !sp->open) return NBODY_ERR_ARG;
    Slot& s = *sp;
    if (!s.pending) return fail(s, NBODY_ERR_STATE, "no calculation pending");
    if (ni != s.pend_ni) return fail(s, NBODY_ERR_ARG, "ni differs from the pending calculation");
    if (nnb && !s.pend_nn) return fail(s, NBODY_ERR_STATE, "nearest neighbour was not enabled");
    if (ni > 0 && (!acc || !jerk || !pot)) return fail(s, NBODY_ERR_ARG, "NULL result array");
    hipError_t e = hipStreamSynchronize(s.st);
    s.pending = false;
    if (e != hipSuccess) return hip_fail(s, e, "force calculation");
    const double* o = s.pin + 6 * s.icap;
    for (int k = 0; k < ni; ++k) {
        for (int c = 0; c < 3; ++c) {
            acc[k][c] = o[c * s.icap + k];
            jerk[k][c] = o[(3 + c) * s.icap + k];
        }
        pot[k] = o[6 * s.icap + k];
        if (nnb) {
            const int a = s.pint[s.icap + k];
            nnb[k] = (a >= 0 && a < s.nset) ? s.hindex[a] : -1;
        }
    }
    return NBODY_OK;
}

}  // namespace

extern "C" {

int GPU_open(int clusterid) {
    Slot* sp = slot(clusterid);
    if (!sp) return NBODY_ERR_ARG;
    Slot& s = *sp;
    if (s.open) return NBODY_OK;
    s = Slot();
    int rc = nbody_create(&s.ctx, clusterid, nullptr);
    if (rc != NBODY_OK) {
        s.err = "nbody_create failed";
        s.ctx = nullptr;
        return rc;
    }
    int prev = -1;
    (void)hipGetDevice(&prev);
    hipError_t e = hipSetDevice(clusterid);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking);
    if (prev >= 0) (void)hipSetDevice(prev);
    if (e != hipSuccess) {
        rc = hip_fail(s, e, "stream create");
        nbody_destroy(s.ctx);
        s.ctx = nullptr;
        return rc;
    }
    s.open = true;
    return NBODY_OK;
}

int GPU_close(int clusterid) {
    Slot* sp = slot(clusterid);
    if (!sp) return NBODY_ERR_ARG;
    Slot& s = *sp;
    if (!s.open) return NBODY_OK;
    (void)hipStreamSynchronize(s.st);
    free_device(s);
    (void)hipStreamDestroy(s.st);
    nbody_destroy(s.ctx);
    s = Slot();
    return NBODY_OK;
}

int GPU_npipes(void) {
    const char* v = std::getenv("NBODY_GRAPE_NPIPES");
    if (v) {
        const long n = std::strtol(v, nullptr, 10);
        if (n > 0 && n <= (1L << 30)) return (int)n;
    }
    return 2048;
}

int GPU_set_j_particle(int clusterid, int address, int index, double tj, double mass, const double x[3],
                       const double v[3], const double a[3], const double j[3]) {
    Slot* sp = slot(clusterid);
    if (!sp || !sp->open) return NBODY_ERR_ARG;
    Slot& s = *sp;
    if (address < 0 || address > 2147483646) return fail(s, NBODY_ERR_ARG, "address out of range");
    if (!finite3(x) || !finite3(v) || !finite3(a) || !finite3(j) || !std::isfinite(tj) || !std::isfinite(mass))
        return fail(s, NBODY_ERR_ARG, "NULL or non-finite j-particle data");
    host_grow(s, (int64_t)address + 1);
    const size_t cap = (size_t)s.hcap, k = (size_t)address;
    for (int c = 0; c < 3; ++c) {
        s.hj[c * cap + k] = x[c];
        s.hj[(3 + c) * cap + k] = v[c];
        s.hj[(6 + c) * cap + k] = a[c];
        s.hj[(9 + c) * cap + k] = j[c];
    }
    s.hj[12 * cap + k] = mass;
    s.hj[13 * cap + k] = tj;
    s.hindex[k] = index;
    s.addr_of[index] = address;
    if (s.dirty_hi <= s.dirty_lo) {
        s.dirty_lo = address;
        s.dirty_hi = (int64_t)address + 1;
    } else {
        s.dirty_lo = std::min<int64_t>(s.dirty_lo, address);
        s.dirty_hi = std::max<int64_t>(s.dirty_hi, (int64_t)address + 1);
    }
    s.nset = std::max<int64_t>(s.nset, (int64_t)address + 1);
    s.need_ti = true;
    return NBODY_OK;
}

int GPU_set_ti(int clusterid, double ti) {
    Slot* sp = slot(clusterid);
    if (!sp || !sp->open) return NBODY_ERR_ARG;
    Slot& s = *sp;
    if (!std::isfinite(ti)) return fail(s, NBODY_ERR_ARG, "ti must be finite");
    if (s.pending) return fail(s, NBODY_ERR_STATE, "a calculation is pending");
    s.need_ti = false;
    if (s.nset == 0) return NBODY_OK;
    int rc = device_j(s);
    if (rc) return rc;
    if (s.dirty_hi > s.dirty_lo) {
        const size_t n = (size_t)(s.dirty_hi - s.dirty_lo);
        for (int r = 0; r < kRaw; ++r) {
            hipError_t e = hipMemcpyAsync(s.dj + (size_t)r * s.dcap + s.dirty_lo,
                                          &s.hj[(size_t)r * s.hcap + s.dirty_lo], sizeof(double) * n,
                                          hipMemcpyHostToDevice, s.st);
            if (e != hipSuccess) return hip_fail(s, e, "j upload");
        }
        // the host rows may change as soon as this returns
        hipError_t e = hipStreamSynchronize(s.st);
        if (e != hipSuccess) return hip_fail(s, e, "j upload");
        s.dirty_lo = s.dirty_hi = 0;
    }
    const int n = (int)s.nset;
    hipLaunchKernelGGL(grape_predict_kernel, dim3((n + 255) / 256), dim3(256), 0, s.st, n, s.dcap, s.dj, ti,
                       s.dj + (size_t)kRaw * s.dcap);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(s, e, "predict launch");
    return NBODY_OK;
}

int GPUcalc_firsthalf(int clusterid, int nj, int ni, const int index[], const double xi[][3], const double vi[][3],
                      double eps2) {
    Slot* sp = slot(clusterid);
    if (!sp || !sp->open) return NBODY_ERR_ARG;
    Slot& s = *sp;
    if (s.pending) return fail(s, NBODY_ERR_STATE, "a calculation is pending");
    if (s.need_ti) return fail(s, NBODY_ERR_STATE, "j-particles changed since GPU_set_ti");
    if (nj < 0 || nj > s.nset) return fail(s, NBODY_ERR_ARG, "nj outside the j set");
    if (ni < 0) return fail(s, NBODY_ERR_ARG, "ni < 0");
    if (ni > 0 && (!index || !xi || !vi)) return fail(s, NBODY_ERR_ARG, "NULL i array");
    if (!std::isfinite(eps2) || eps2 < 0.0) return fail(s, NBODY_ERR_ARG, "eps2 must be finite and >= 0");
    s.pend_ni = ni;
    s.pend_nn = s.nn;
    if (ni == 0) {
        s.pending = true;
        return NBODY_OK;
    }
    int rc = device_i(s, ni);
    if (rc) return rc;
    const size_t ic = (size_t)s.icap;
    for (int k = 0; k < ni; ++k) {
        for (int c = 0; c < 3; ++c) {
            s.pin[c * ic + k] = xi[k][c];
            s.pin[(3 + c) * ic + k] = vi[k][c];
        }
        auto it = s.addr_of.find(index[k]);
        int a = it == s.addr_of.end() ? -1 : it->second;
        if (a >= nj || (a >= 0 && s.hindex[a] != index[k])) a = -1;
        s.pint[k] = a;
    }
    for (int r = 0; r < 6; ++r) {
        hipError_t e = hipMemcpyAsync(s.di + r * ic, s.pin + r * ic, sizeof(double) * ni, hipMemcpyHostToDevice, s.st);
        if (e != hipSuccess) return hip_fail(s, e, "i upload");
    }
    hipError_t e = hipMemcpyAsync(s.dint, s.pint, sizeof(int32_t) * ni, hipMemcpyHostToDevice, s.st);
    if (e != hipSuccess) return hip_fail(s, e, "i upload");
    if (nj > 0) {
        hipLaunchKernelGGL(grape_gather_kernel, dim3((ni + 255) / 256), dim3(256), 0, s.st, ni, (int64_t)ic, s.dint,
                           s.dcap, s.dj + (size_t)kRaw * s.dcap, s.di);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(s, e, "i gather launch");
    }
    const double* P = nj > 0 ? s.dj + (size_t)kRaw * s.dcap : nullptr;
    const size_t dc = (size_t)s.dcap;
    nbody_src I{s.di, s.di + ic, s.di + 2 * ic, s.di + 3 * ic, s.di + 4 * ic, s.di + 5 * ic, nullptr};
    nbody_src J{P, P ? P + dc : nullptr, P ? P + 2 * dc : nullptr, P ? P + 3 * dc : nullptr,
                P ? P + 4 * dc : nullptr, P ? P + 5 * dc : nullptr, nj > 0 ? s.dj + 12 * dc : nullptr};
    double* o = s.di + 6 * ic;
    nbody_out O{o, o + ic, o + 2 * ic, o + 3 * ic, o + 4 * ic, o + 5 * ic, o + 6 * ic};
    const nbody_prec prec = (nbody_prec)s.prec;
    const double eps = std::sqrt(eps2);
    const int32_t* self = nj > 0 ? s.dint : nullptr;
    rc = s.nn ? nbody_force_nn(s.ctx, s.st, prec, 1.0, eps, ni, I, self, nj, J, O, s.dint + ic, nullptr)
              : nbody_force(s.ctx, s.st, prec, 1.0, eps, ni, I, self, nj, J, O);
    if (rc) {
        // the i upload may still be reading the pinned rows the next call writes
        (void)hipStreamSynchronize(s.st);
        return lib_fail(s, rc, "force calculation");
    }
    e = hipMemcpyAsync(s.pin + 6 * ic, o, sizeof(double) * 7 * ic, hipMemcpyDeviceToHost, s.st);
    if (e == hipSuccess && s.nn)
        e = hipMemcpyAsync(s.pint + ic, s.dint + ic, sizeof(int32_t) * ni, hipMemcpyDeviceToHost, s.st);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(s.st);
        return hip_fail(s, e, "result download");
    }
    s.pending = true;
    return NBODY_OK;
}

int GPUcalc_lasthalf(int clusterid, int ni, double acc[][3], double jerk[][3], double pot[]) {
    return collect(clusterid, ni, acc, jerk, pot, nullptr);
}

int GPUcalc_lasthalf2(int clusterid, int ni, double acc[][3], double jerk[][3], double pot[], int nnb[]) {
    Slot* sp = slot(clusterid);
    if (sp && sp->open && ni > 0 && !nnb) return fail(*sp, NBODY_ERR_ARG, "NULL nnb");
    return collect(clusterid, ni, acc, jerk, pot, ni > 0 ? nnb : nullptr);
}

int GPU_set_nn(int clusterid, int enable) {
    Slot* sp = slot(clusterid);
    if (!sp || !sp->open) return NBODY_ERR_ARG;
    sp->nn = enable != 0;
    return NBODY_OK;
}

int GPU_set_precision(int clusterid, int prec) {
    Slot* sp = slot(clusterid);
    if (!sp || !sp->open) return NBODY_ERR_ARG;
    if (prec != NBODY_PREC_FP32 && prec != NBODY_PREC_DS_COMP) return fail(*sp, NBODY_ERR_ARG, "unknown precision");
    sp->prec = prec;
    return NBODY_OK;
}

const char* GPU_last_error(int clusterid) {
    Slot* sp = slot(clusterid);
    if (!sp) return "cluster id out of range";
    return sp->err.c_str();
}

}  // extern "C"

// Host side of the C ABI declared in include/nbody.h: argument checks,
// context-owned scratch memory, launch-shape choice and the Hermite
// block-step driver.  All particle arithmetic runs in the kernels of
// force.hip and hermite.hip.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "nbody.h"
#include "force_block.h"
#include "nbody_internal.h"
#include "tune.h"

using namespace nb;

namespace {

constexpr int64_t kMaxN = 2147483647LL;
// The differentiable run's elementwise kernels index [3][n] rows as one int32 range.
constexpr int64_t kMaxShared = kMaxN / 3;

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

// Caller-provided room for the split partial sums (the allocation-free
// entry point): run_force takes its partials from here, never allocates,
// and uses fewer j-ranges when the shape's partials would not fit.
struct FixedWS {
    float2* part = nullptr;
    size_t bytes = 0;
};

}  // namespace

// Device memory of the allocation-free evaluation (nbody_force_noalloc): one
// array per GPU, loaded with the library's code object and held until the
// process ends.  In host code `scratch` names a host-side stand-in, not a
// device address: the address on each device comes from
// hipGetSymbolAddress, taken once per device at context creation
// (scratch_setup) and kept in g_scratch.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};         // device address of `scratch` per device
hipError_t g_scratch_err[kMaxDevices] = {}; // result of the lookup (hipSuccess once found)
bool g_scratch_tried[kMaxDevices] = {};

// With `device` current: look up its copy of `scratch` once.
void scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_tried[device] && g_scratch_err[device] == hipSuccess) return;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_tried[device] = true;
    g_scratch_err[device] = e;
    g_scratch[device] = e == hipSuccess ? ptr : nullptr;
    if (e != hipSuccess) (void)hipGetLastError();
}

void* scratch_ptr(int device, hipError_t* err) {
    if (device < 0 || device >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    *err = g_scratch_tried[device] ? g_scratch_err[device] : hipErrorNotInitialized;
    return g_scratch[device];
}
}  // namespace

struct nbody_ctx {
    int device = -1;          // -1: argument-checking context without a device
    std::string err;
    DevBuf ipack, jpack, part, sel, scratch64, vrec_i, vrec_j, vpart, integ, hist, bplan, bstate, lf;
    // batched Hermite graph (captured on a context-owned stream)
    hipStream_t gstream = nullptr;
    hipEvent_t gev[2] = {nullptr, nullptr};
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    std::vector<uint64_t> gkey;
    bool have_override[2] = {false, false};
    nbody_tile override_tile[2];
    nb::TuneCache tune;
    int alloc_count = 0;
    int fail_alloc_at = 0;    // debug: NBODY_DEBUG_FAIL_ALLOC=k fails the k-th allocation
    bool self_check = false;  // debug: NBODY_DEBUG_SELF_CHECK=1 verifies self rows (synchronises)
    // NBODY_TRACE=<path>: one JSON line per Hermite step appended to that file
    std::string trace_path;
    FILE* trace = nullptr;
    // kernel timing: event pairs recorded around each pairwise-kernel launch
    bool timing = false;
    std::vector<hipEvent_t> ev;   // 2 per launch
    size_t ev_used = 0;
};

struct nbody_hermite {
    nbody_ctx* ctx = nullptr;
    int64_t n = 0;
    nbody_hermite_opts o{};
    bool has_state = false;
    // float64 state rows: x y z vx vy vz ax ay az jx jy jz m ; pot scratch
    double* s[13] = {};
    double* f[7] = {};        // block forces (a, jerk, pot) [n]
    double* pred[6] = {};     // predicted x, v for energy
    int64_t* t = nullptr;
    int64_t* dt = nullptr;
    int32_t* idx = nullptr;
    int64_t* sel2 = nullptr;  // device [2]: n_act, t_next
    int64_t* tnow = nullptr;  // device scalar: latest block time
    double* e2 = nullptr;     // device [2]
    DevPlan* plan = nullptr;  // device block-step plan and statistics
    float4* spack = nullptr;  // shared steps: records of all particles predicted to spack_tn
    float4* spack2 = nullptr; // shared steps: the next step's records while spack is being read
    int64_t spack_tn = -1;    // tick those records are valid for (-1: none)
    // shared steps of small sets: the sums and the corrector in one launch
    // (NBODY_FUSED_CORRECT=0: a pairwise launch and a corrector launch)
    bool fuse = true;
    int64_t* gmin2 = nullptr; // block steps: two arrays of chunk minima of t + dt (this step's, next)
    uint64_t* gpub = nullptr; // block steps: per-chunk published counts of the fused front end
    TraceRec* ring = nullptr; // block steps: per-step records for NBODY_TRACE (device)
    DevPlan* splan = nullptr; // shared steps of small sets: the j-parallel plan (device; written once)
    int splan_S = 0;          // its number of j-ranges (0: not written yet)
    bool part_checked = false; // block plans of every size checked against the partials' size
    uint32_t* ftag = nullptr; // block steps: the front end's last tag (device word after gpub)
    // block steps replayed as a captured graph of kBlkGraphSteps steps
    // (NBODY_BLOCK_GRAPH=1; measured slower than launching them)
    bool use_graph = false;
    hipGraph_t bgraph = nullptr;
    hipGraphExec_t bexec = nullptr;
    std::vector<uint64_t> bkey;
    int gpar = 0;             // which of the two holds this step's
    bool gmin_ok = false;     // false: recompute this step's before use
    int64_t t_ticks = 0;
    int64_t steps = 0, sum_active = 0;
    void* block = nullptr;    // single allocation holding everything above
};

static int set_err(nbody_ctx* c, int code, const char* fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

static int hip_err(nbody_ctx* c, hipError_t e, const char* what) {
    return set_err(c, NBODY_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Switch to the context's device for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (dev < 0) return;
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

static int dev_alloc(nbody_ctx* c, DevBuf& b, size_t bytes) {
    if (b.bytes >= bytes) return NBODY_OK;
    ++c->alloc_count;
    if (c->fail_alloc_at > 0 && c->alloc_count == c->fail_alloc_at)
        return set_err(c, NBODY_ERR_NOMEM, "device allocation of %zu bytes failed (injected)", bytes);
    if (b.p) {
        (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_err(c, NBODY_ERR_NOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    b.p = p;
    b.bytes = bytes;
    return NBODY_OK;
}

static bool aligned8(const void* p) { return ((uintptr_t)p & 7u) == 0; }

static int check_src(nbody_ctx* c, const nbody_src& s, bool need_m, const char* name, bool need_v = true) {
    const double* rows[7] = {s.x, s.y, s.z, s.vx, s.vy, s.vz, s.m};
    for (int k = 0; k < 7; ++k) {
        if (k == 6 && !need_m) continue;
        if (k >= 3 && k < 6 && !need_v) continue;
        if (!rows[k]) return set_err(c, NBODY_ERR_ARG, "%s: row %d is NULL", name, k);
        if (!aligned8(rows[k])) return set_err(c, NBODY_ERR_ARG, "%s: row %d is not 8-byte aligned", name, k);
    }
    return NBODY_OK;
}

static int check_out(nbody_ctx* c, const nbody_out& o, bool need_jerk = true) {
    double* rows[7] = {o.ax, o.ay, o.az, o.jx, o.jy, o.jz, o.pot};
    for (int k = 0; k < 7; ++k) {
        if (k >= 3 && k < 6 && !need_jerk) continue;
        if (!rows[k]) return set_err(c, NBODY_ERR_ARG, "out: row %d is NULL", k);
        if (!aligned8(rows[k])) return set_err(c, NBODY_ERR_ARG, "out: row %d is not 8-byte aligned", k);
    }
    return NBODY_OK;
}

static bool valid_tile(const nbody_tile& t) {
    if (t.split < 0 || t.split > 4096 || (t.jsrc != 0 && t.jsrc != 1)) return false;
    return force_variant_exists(0, t.ipt, t.tile_j, t.wg, t.jsrc, t.unroll, t.waves, false) ||
           force_variant_exists(1, t.ipt, t.tile_j, t.wg, t.jsrc, t.unroll, t.waves, false);
}

static nbody_tile pick_tile(nbody_ctx* c, int prec, int64_t ni, int64_t nj) {
    nbody_tile t;
    if (c->have_override[prec]) {
        t = c->override_tile[prec];
    } else if (!c->tune.lookup(prec, ni, nj, &t)) {
        t = default_tile(prec, ni, nj);
    }
    if (t.split <= 0) t.split = choose_split(ni, nj, t);
    return t;
}

// Core evaluation: i records (ipack, iidx) against j records (jpack).  kind 0
// writes all 7 rows of out; kind 1 (force only) rows 0-2 and 6; kind 2 all 7
// plus the nearest neighbour (nn, nn_r2).
static int run_force(nbody_ctx* c, hipStream_t st, int prec, double G, double eps, int64_t ni,
                     const float4* ipack, const int32_t* iidx, const int32_t* iself, int self_mode,
                     int64_t nj, const float4* jpack, double* const out[7], const nbody_tile* forced,
                     int kind = 0, int32_t* nn = nullptr, double* nn_r2 = nullptr,
                     int* defer_split = nullptr, const FixedWS* fixed = nullptr) {
    if (ni == 0) return NBODY_OK;
    if (fixed && (kind != 0 || defer_split)) return set_err(c, NBODY_ERR_ARG, "fixed workspace needs kind 0");
    if (defer_split && kind != 0) return set_err(c, NBODY_ERR_ARG, "deferred split reduce needs kind 0");
    nbody_tile t;
    if (forced) {
        t = *forced;
    } else if (kind == 0 || c->have_override[prec]) {
        t = pick_tile(c, prec, ni, nj);   // tuned entries hold kind-0 shapes only
    } else {
        t = default_tile_kind(kind, prec, ni, nj);
    }
    if (t.split <= 0) t.split = choose_split(ni, nj, t);
    const bool eps0 = eps == 0.0;
    int ipt = t.ipt, tj = t.tile_j, wg = t.wg, jsrc = t.jsrc, unr = t.unroll, wpe = t.waves;
    if (!force_variant_exists(prec, ipt, tj, wg, jsrc, unr, wpe, eps0, kind)) {
        if (eps0) {
            // the unsoftened path exists in few LDS shapes per precision
            ipt = (kind == 0 && ipt >= 2) ? 2 : 1;
            tj = 128;
            wg = 256;
        } else {
            // the other kinds fall back to their default shape for the size
            const nbody_tile d = default_tile_kind(kind, prec, ni, nj);
            ipt = d.ipt;
            tj = d.tile_j;
            wg = d.wg;
            unr = d.unroll;
        }
        jsrc = 0;
        if (eps0) unr = 0;
        wpe = 0;
        if (!forced) t.split = 0;
    }
    int nb, S, jchunk;
    split_plan(ni, nj, wg * ipt, tj, t.split, &nb, &S, &jchunk);
    if (fixed && S > 1) {
        // as many j-ranges as the fixed workspace holds partials for
        const int64_t fit = (int64_t)(fixed->bytes / (sizeof(float2) * 7 * (size_t)ni));
        if (fit < S) split_plan(ni, nj, wg * ipt, tj, (int)std::max<int64_t>(fit, 1), &nb, &S, &jchunk);
    }

    ForceArgs a{};
    a.ipack = ipack;
    a.iidx = iidx;
    a.ni = (int)ni;
    a.jpack = jpack;
    a.nj = (int)nj;
    a.jchunk = (int)jchunk;
    a.eps2 = (float)(eps * eps);
    a.G = G;
    a.iself = iself;
    a.self_mode = self_mode;
    for (int q = 0; q < 7; ++q) a.out[q] = out[q];
    if (kind == 1) a.out[3] = a.out[4] = a.out[5] = nullptr;
    a.nn = nn;
    a.nn_r2 = nn_r2;
    a.partial = S > 1 ? 1 : 0;
    if (S > 1) {
        const size_t rows = kind == 2 ? 8 : 7;
        const size_t need = sizeof(float2) * rows * (size_t)S * (size_t)ni;
        if (fixed) {
            if (need > fixed->bytes) return set_err(c, NBODY_ERR_ARG, "split partials exceed the fixed workspace");
            a.part = fixed->part;
        } else {
            int rc = dev_alloc(c, c->part, need);
            if (rc) return rc;
            a.part = (float2*)c->part.p;
        }
        if (kind == 2) a.nnpart = a.part + 7 * (size_t)S * (size_t)ni;
    }
    hipEvent_t tb = nullptr, te = nullptr;
    if (c->timing && !fixed) {
        while (c->ev.size() < c->ev_used + 2) {
            hipEvent_t x;
            if (hipEventCreate(&x) != hipSuccess) return set_err(c, NBODY_ERR_DEVICE, "event create");
            c->ev.push_back(x);
        }
        tb = c->ev[c->ev_used];
        te = c->ev[c->ev_used + 1];
        c->ev_used += 2;
        if (hipEventRecord(tb, st) != hipSuccess) return set_err(c, NBODY_ERR_DEVICE, "event record");
    }
    hipError_t e = launch_force(prec, ipt, tj, wg, jsrc, unr, wpe, eps0, nb, S, a, st, kind);
    if (e != hipSuccess) return hip_err(c, e, "force kernel launch");
    if (te && hipEventRecord(te, st) != hipSuccess) return set_err(c, NBODY_ERR_DEVICE, "event record");
    if (defer_split) {
        // the caller reduces the partials (kind 0 only) in a kernel of its own
        *defer_split = S;
        return NBODY_OK;
    }
    if (S > 1) {
        ReduceArgs r{};
        r.ni = (int)ni;
        r.S = S;
        r.part = a.part;
        r.G = G;
        for (int q = 0; q < 7; ++q) r.out[q] = a.out[q];
        e = launch_reduce(r, st);
        if (e != hipSuccess) return hip_err(c, e, "split reduce launch");
        if (kind == 2) {
            e = launch_nn_reduce((int)ni, S, a.nnpart, nn, nn_r2, st);
            if (e != hipSuccess) return hip_err(c, e, "nearest-neighbour reduce launch");
        }
    }
    return NBODY_OK;
}

static int pack_into(nbody_ctx* c, hipStream_t st, int prec, int64_t n, const nbody_src& s, bool with_m,
                     float4* dst) {
    PackArgs p{};
    p.n = (int)n;
    p.prec = prec;
    p.x = s.x; p.y = s.y; p.z = s.z;
    p.vx = s.vx; p.vy = s.vy; p.vz = s.vz;
    p.m = with_m ? s.m : nullptr;
    p.out = dst;
    hipError_t e = launch_pack(p, st);
    if (e != hipSuccess) return hip_err(c, e, "pack launch");
    return NBODY_OK;
}

static int pack_rows(nbody_ctx* c, hipStream_t st, int prec, int64_t n, const nbody_src& s,
                     bool with_m, DevBuf& dst) {
    const size_t bytes = sizeof(float4) * (size_t)rec_words(prec) * (size_t)std::max<int64_t>(n, 1);
    int rc = dev_alloc(c, dst, bytes);
    if (rc) return rc;
    return pack_into(c, st, prec, n, s, with_m, (float4*)dst.p);
}

static bool same_src(const nbody_src& a, const nbody_src& b) {
    return a.x == b.x && a.y == b.y && a.z == b.z && a.vx == b.vx && a.vy == b.vy && a.vz == b.vz;
}

// Debug mode (NBODY_DEBUG_SELF_CHECK=1): the packed i rows named by i_self
// must equal their j rows bit for bit; synchronises `st`.
static int debug_self_check(nbody_ctx* c, hipStream_t st, int prec, int64_t ni, const float4* ip,
                            const int32_t* iself, int64_t nj, const float4* jp) {
    if (!c->self_check || !iself || ni == 0) return NBODY_OK;
    int rc = dev_alloc(c, c->scratch64, sizeof(int64_t));
    if (rc) return rc;
    int* bad = (int*)c->scratch64.p;
    hipError_t e = launch_self_check((int)ni, (int)nj, prec, ip, iself, jp, bad, st);
    int h = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, bad, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_err(c, e, "self check");
    if (h) return set_err(c, NBODY_ERR_ARG, "i_self: %d i rows differ from their j rows or index beyond n_j", h);
    return NBODY_OK;
}

extern "C" {

int nbody_abi_version(void) { return NBODY_ABI_VERSION; }

int nbody_create(nbody_ctx** ctx, int device, const char* tune_cache_path) {
    if (!ctx) return NBODY_ERR_ARG;
    *ctx = nullptr;
    if (device < -1) return NBODY_ERR_ARG;
    nbody_ctx* c = new (std::nothrow) nbody_ctx();
    if (!c) return NBODY_ERR_NOMEM;
    if (const char* f = getenv("NBODY_DEBUG_FAIL_ALLOC")) c->fail_alloc_at = atoi(f);
    if (const char* f = getenv("NBODY_DEBUG_SELF_CHECK")) c->self_check = atoi(f) != 0;
    if (const char* f = getenv("NBODY_TRACE")) c->trace_path = f;
    if (const char* f = getenv("NBODY_FORCE_TILE")) {
        // tile_j,ipt,wg[,split[,jsrc[,unroll[,waves]]]]: the launch shape of
        // every evaluation of the precisions that compile it
        int v[7] = {0, 0, 0, 0, 0, 0, 0};
        const int got = sscanf(f, "%d,%d,%d,%d,%d,%d,%d", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &v[6]);
        const nbody_tile t{v[0], v[1], v[2], v[3], v[4], v[5], v[6]};
        bool any = false;
        if (got >= 3 && t.split >= 0 && t.split <= 4096)
            for (int prec = 0; prec < 2; ++prec)
                if (force_variant_exists(prec, t.ipt, t.tile_j, t.wg, t.jsrc, t.unroll, t.waves, false)) {
                    c->override_tile[prec] = t;
                    c->have_override[prec] = true;
                    any = true;
                }
        if (!any) {
            delete c;
            return NBODY_ERR_ARG;
        }
    }
    const char* path = tune_cache_path ? tune_cache_path : getenv("NBODY_TUNE_CACHE");
    if (path && *path) c->tune.set_path(path);
    if (device >= 0) {
        int count = 0;
        hipError_t e = hipGetDeviceCount(&count);
        if (e != hipSuccess || device >= count) {
            (void)hipGetLastError();
            delete c;
            return NBODY_ERR_DEVICE;
        }
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, device);
        if (e != hipSuccess) {
            delete c;
            return NBODY_ERR_DEVICE;
        }
        c->tune.set_arch(prop.gcnArchName);
        c->tune.load();
        DeviceGuard g(device);
        if (g.ok) scratch_setup(device);
    }
    c->device = device;
    *ctx = c;
    return NBODY_OK;
}

int nbody_destroy(nbody_ctx* c) {
    if (!c) return NBODY_OK;
    if (c->device >= 0) {
        DeviceGuard g(c->device);
        for (hipEvent_t x : c->ev) (void)hipEventDestroy(x);
        if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
        if (c->graph) (void)hipGraphDestroy(c->graph);
        for (hipEvent_t x : c->gev)
            if (x) (void)hipEventDestroy(x);
        if (c->gstream) (void)hipStreamDestroy(c->gstream);
        if (c->trace) fclose(c->trace);
        DevBuf* bufs[] = {&c->ipack, &c->jpack, &c->part, &c->sel, &c->scratch64,
                          &c->vrec_i, &c->vrec_j, &c->vpart, &c->integ, &c->hist, &c->bplan,
                          &c->bstate, &c->lf};
        for (DevBuf* b : bufs)
            if (b->p) (void)hipFree(b->p);
    }
    delete c;
    return NBODY_OK;
}

const char* nbody_last_error(const nbody_ctx* c) { return c ? c->err.c_str() : "null context"; }

static int need_device(nbody_ctx* c) {
    if (c->device < 0)
        return set_err(c, NBODY_ERR_UNSUPPORTED, "context has no device (created with device -1)");
    return NBODY_OK;
}

// Split-partial bytes of the shapes the next calls would take for up to
// max_i i-particles against max_j j: evaluated at max_i and at every power
// of two below it (the long-evaluation rule keeps S x n_i about constant, so
// the largest is near one of these).  Host arithmetic only.
static size_t reserve_part_bytes(nbody_ctx* c, int64_t max_i, int64_t max_j) {
    const int64_t ni = std::max<int64_t>(max_i, 1), nj = std::max<int64_t>(max_j, 1);
    size_t part = 0;
    for (int prec = 0; prec < 2; ++prec) {
        int64_t n = ni;
        for (;;) {
            const nbody_tile t = pick_tile(c, prec, n, nj);
            int nb, S, jc;
            split_plan(n, nj, t.wg * t.ipt, t.tile_j, t.split, &nb, &S, &jc);
            if (S > 1) part = std::max(part, sizeof(float2) * 8 * (size_t)S * (size_t)n);
            if (n <= 1) break;
            // the largest power of two below n (n strictly decreases)
            const int64_t p2 = (int64_t)1 << (63 - __builtin_clzll((unsigned long long)n));
            n = p2 < n ? p2 : n / 2;
        }
    }
    return part;
}

int nbody_reserve(nbody_ctx* c, int64_t max_i, int64_t max_j) {
    if (!c) return NBODY_ERR_ARG;
    if (max_i < 0 || max_j < 0 || max_i > kMaxN || max_j > kMaxN)
        return set_err(c, NBODY_ERR_ARG, "reserve: sizes must be in [0, 2^31-1]");
    const size_t part = reserve_part_bytes(c, max_i, max_j);
    if (int rc = need_device(c)) return rc;
    DeviceGuard g(c->device);
    const size_t ni = (size_t)std::max<int64_t>(max_i, 1), nj = (size_t)std::max<int64_t>(max_j, 1);
    int rc = dev_alloc(c, c->ipack, sizeof(float4) * kRecDS * ni);
    if (!rc) rc = dev_alloc(c, c->jpack, sizeof(float4) * kRecDS * nj);
    if (!rc && part > 0) rc = dev_alloc(c, c->part, part);
    return rc;
}

int nbody_sync(nbody_ctx* c, hipStream_t st) {
    if (!c) return NBODY_ERR_ARG;
    if (int rc = need_device(c)) return rc;
    DeviceGuard g(c->device);
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_err(c, e, "stream synchronize");
    return NBODY_OK;
}

int nbody_kernel_timing(nbody_ctx* c, int enable) {
    if (!c) return NBODY_ERR_ARG;
    if (enable != 0 && enable != 1) return set_err(c, NBODY_ERR_ARG, "enable must be 0 or 1");
    if (int rc = need_device(c)) return rc;
    c->timing = enable == 1;
    c->ev_used = 0;
    return NBODY_OK;
}

int nbody_kernel_time(nbody_ctx* c, double* total_ms, int64_t* launches) {
    if (!c) return NBODY_ERR_ARG;
    if (!total_ms || !launches) return set_err(c, NBODY_ERR_ARG, "NULL output");
    if (int rc = need_device(c)) return rc;
    DeviceGuard g(c->device);
    double tot = 0.0;
    for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
        hipError_t e = hipEventSynchronize(c->ev[k + 1]);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, c->ev[k], c->ev[k + 1]);
        if (e != hipSuccess) return hip_err(c, e, "kernel timing");
        tot += ms;
    }
    *total_ms = tot;
    *launches = (int64_t)(c->ev_used / 2);
    c->ev_used = 0;
    return NBODY_OK;
}

int nbody_set_tile(nbody_ctx* c, nbody_prec prec, const nbody_tile* t) {
    if (!c) return NBODY_ERR_ARG;
    if (prec != NBODY_PREC_FP32 && prec != NBODY_PREC_DS_COMP)
        return set_err(c, NBODY_ERR_ARG, "unknown precision %d", (int)prec);
    if (!t) {
        c->have_override[prec] = false;
        return NBODY_OK;
    }
    if (!valid_tile(*t))
        return set_err(c, NBODY_ERR_ARG, "tile (tile_j=%d ipt=%d wg=%d split=%d jsrc=%d unroll=%d waves=%d) not supported",
                       t->tile_j, t->ipt, t->wg, t->split, t->jsrc, t->unroll, t->waves);
    c->override_tile[prec] = *t;
    c->have_override[prec] = true;
    return NBODY_OK;
}

int nbody_get_tile(nbody_ctx* c, nbody_prec prec, int64_t ni, int64_t nj, nbody_tile* t) {
    if (!c || !t) return NBODY_ERR_ARG;
    if (prec != NBODY_PREC_FP32 && prec != NBODY_PREC_DS_COMP)
        return set_err(c, NBODY_ERR_ARG, "unknown precision %d", (int)prec);
    if (ni < 0 || nj < 0 || ni > kMaxN || nj > kMaxN) return set_err(c, NBODY_ERR_ARG, "bad sizes");
    *t = pick_tile(c, prec, ni, nj);
    return NBODY_OK;
}

static int check_common(nbody_ctx* c, nbody_prec prec, double G, double eps) {
    if (prec != NBODY_PREC_FP32 && prec != NBODY_PREC_DS_COMP)
        return set_err(c, NBODY_ERR_ARG, "unknown precision %d", (int)prec);
    if (!isfinite(G)) return set_err(c, NBODY_ERR_ARG, "G must be finite");
    if (!isfinite(eps) || eps < 0.0) return set_err(c, NBODY_ERR_ARG, "eps must be finite and >= 0");
    return NBODY_OK;
}

int nbody_force(nbody_ctx* c, hipStream_t st, nbody_prec prec, double G, double eps, int64_t n_i,
                nbody_src I, const int32_t* i_self, int64_t n_j, nbody_src J, nbody_out out) {
    if (!c) return NBODY_ERR_ARG;
    if (int rc = check_common(c, prec, G, eps)) return rc;
    if (n_i < 0 || n_j < 0) return set_err(c, NBODY_ERR_ARG, "n_i and n_j must be >= 0");
    if (n_i > kMaxN || n_j > kMaxN) return set_err(c, NBODY_ERR_ARG, "n_i and n_j must be <= 2^31-1");
    if (n_i > 0) {
        if (int rc = check_src(c, I, false, "I")) return rc;
        if (int rc = check_out(c, out)) return rc;
    }
    if (n_j > 0)
        if (int rc = check_src(c, J, true, "J")) return rc;
    if (n_i > 0 && n_j == 0 && i_self)
        return set_err(c, NBODY_ERR_ARG, "i_self given with an empty j set");
    if (int rc = need_device(c)) return rc;
    if (n_i == 0) return NBODY_OK;
    DeviceGuard g(c->device);
    if (!g.ok) return set_err(c, NBODY_ERR_DEVICE, "hipSetDevice(%d) failed", c->device);
    const int p = (int)prec;
    int rc = pack_rows(c, st, p, n_j, J, true, c->jpack);
    if (rc) return rc;
    const float4* ip = (const float4*)c->jpack.p;
    if (!(n_i == n_j && same_src(I, J))) {
        rc = pack_rows(c, st, p, n_i, I, false, c->ipack);
        if (rc) return rc;
        ip = (const float4*)c->ipack.p;
    }
    if ((rc = debug_self_check(c, st, p, n_i, ip, i_self, n_j, (const float4*)c->jpack.p))) return rc;
    double* o[7] = {out.ax, out.ay, out.az, out.jx, out.jy, out.jz, out.pot};
    return run_force(c, st, p, G, eps, n_i, ip, nullptr, i_self, 0, n_j, (const float4*)c->jpack.p, o,
                     nullptr);
}

int nbody_force_noalloc(nbody_ctx* c, hipStream_t st, nbody_prec prec, double G, double eps, int64_t n_i,
                        nbody_src I, const int32_t* i_self, int64_t n_j, nbody_src J, nbody_out out) {
    if (!c) return NBODY_ERR_ARG;
    if (int rc = check_common(c, prec, G, eps)) return rc;
    if (n_i < 0 || n_j < 0) return set_err(c, NBODY_ERR_ARG, "n_i and n_j must be >= 0");
    if (n_i > kMaxN || n_j > kMaxN) return set_err(c, NBODY_ERR_ARG, "n_i and n_j must be <= 2^31-1");
    if (n_i > 0) {
        if (int rc = check_src(c, I, false, "I")) return rc;
        if (int rc = check_out(c, out)) return rc;
    }
    if (n_j > 0)
        if (int rc = check_src(c, J, true, "J")) return rc;
    if (n_i > 0 && n_j == 0 && i_self)
        return set_err(c, NBODY_ERR_ARG, "i_self given with an empty j set");
    if (int rc = need_device(c)) return rc;
    const int p = (int)prec;
    const bool own = n_i == n_j && same_src(I, J);
    // packed records, each rounded up to 256 bytes, then the split partials
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t rec = sizeof(float4) * (size_t)rec_words(p);
    const size_t jb = up(rec * (size_t)n_j), ib = own ? 0 : up(rec * (size_t)n_i);
    if (jb + ib > kNoAllocBytes)
        return set_err(c, NBODY_ERR_ARG,
                       "nbody_force_noalloc: %lld i and %lld j records need %zu bytes, beyond its %zu-byte scratch",
                       (long long)n_i, (long long)n_j, jb + ib, kNoAllocBytes);
    if (n_i == 0) return NBODY_OK;
    DeviceGuard g(c->device);
    if (!g.ok) return set_err(c, NBODY_ERR_DEVICE, "hipSetDevice(%d) failed", c->device);
    hipError_t se;
    unsigned char* base = (unsigned char*)scratch_ptr(c->device, &se);
    if (!base) return hip_err(c, se, "nbody_force_noalloc: device address of the scratch array");
    float4* jp = (float4*)base;
    float4* ip = own ? jp : (float4*)(base + jb);
    int rc = pack_into(c, st, p, n_j, J, true, jp);
    if (!rc && !own) rc = pack_into(c, st, p, n_i, I, false, ip);
    if (rc) return rc;
    FixedWS ws;
    ws.part = (float2*)(base + jb + ib);
    ws.bytes = kNoAllocBytes - jb - ib;
    double* o[7] = {out.ax, out.ay, out.az, out.jx, out.jy, out.jz, out.pot};
    return run_force(c, st, p, G, eps, n_i, ip, nullptr, i_self, 0, n_j, jp, o, nullptr, 0, nullptr, nullptr,
                     nullptr, &ws);
}

// Shared argument checks and packing of nbody_force_acc / nbody_force_nn.
static int force_kind(nbody_ctx* c, hipStream_t st, nbody_prec prec, double G, double eps, int64_t n_i,
                      nbody_src I, const int32_t* i_self, int64_t n_j, nbody_src J, nbody_out out, int kind,
                      int32_t* nn, double* nn_r2) {
    if (!c) return NBODY_ERR_ARG;
    if (int rc = check_common(c, prec, G, eps)) return rc;
    if (n_i < 0 || n_j < 0) return set_err(c, NBODY_ERR_ARG, "n_i and n_j must be >= 0");
    if (n_i > kMaxN || n_j > kMaxN) return set_err(c, NBODY_ERR_ARG, "n_i and n_j must be <= 2^31-1");
    const bool vel = kind != 1;
    if (n_i > 0) {
        if (int rc = check_src(c, I, false, "I", vel)) return rc;
        if (int rc = check_out(c, out, vel)) return rc;
        if (kind == 2 && !nn) return set_err(c, NBODY_ERR_ARG, "nn is NULL");
        if (kind == 2 && !aligned8(nn_r2)) return set_err(c, NBODY_ERR_ARG, "nn_r2 is not 8-byte aligned");
    }
    if (n_j > 0)
        if (int rc = check_src(c, J, true, "J", vel)) return rc;
    if (n_i > 0 && n_j == 0 && i_self)
        return set_err(c, NBODY_ERR_ARG, "i_self given with an empty j set");
    if (int rc = need_device(c)) return rc;
    if (n_i == 0) return NBODY_OK;
    DeviceGuard g(c->device);
    if (!g.ok) return set_err(c, NBODY_ERR_DEVICE, "hipSetDevice(%d) failed", c->device);
    if (!vel) {
        // velocities are not read by the force-only evaluation
        I.vx = I.vy = I.vz = nullptr;
        J.vx = J.vy = J.vz = nullptr;
    }
    const int p = (int)prec;
    int rc = pack_rows(c, st, p, n_j, J, true, c->jpack);
    if (rc) return rc;
    const float4* ip = (const float4*)c->jpack.p;
    if (!(n_i == n_j && same_src(I, J))) {
        rc = pack_rows(c, st, p, n_i, I, false, c->ipack);
        if (rc) return rc;
        ip = (const float4*)c->ipack.p;
    }
    if ((rc = debug_self_check(c, st, p, n_i, ip, i_self, n_j, (const float4*)c->jpack.p))) return rc;
    double* o[7] = {out.ax, out.ay, out.az, vel ? out.jx : nullptr, vel ? out.jy : nullptr,
                    vel ? out.jz : nullptr, out.pot};
    return run_force(c, st, p, G, eps, n_i, ip, nullptr, i_self, 0, n_j, (const float4*)c->jpack.p, o, nullptr,
                     kind, nn, nn_r2);
}

int nbody_force_acc(nbody_ctx* c, hipStream_t st, nbody_prec prec, double G, double eps, int64_t n_i,
                    nbody_src I, const int32_t* i_self, int64_t n_j, nbody_src J, nbody_out out) {
    return force_kind(c, st, prec, G, eps, n_i, I, i_self, n_j, J, out, 1, nullptr, nullptr);
}

int nbody_force_nn(nbody_ctx* c, hipStream_t st, nbody_prec prec, double G, double eps, int64_t n_i,
                   nbody_src I, const int32_t* i_self, int64_t n_j, nbody_src J, nbody_out out, int32_t* nn,
                   double* nn_r2) {
    return force_kind(c, st, prec, G, eps, n_i, I, i_self, n_j, J, out, 2, nn, nn_r2);
}

int nbody_leapfrog(nbody_ctx* c, hipStream_t st, nbody_prec prec, double G, double eps, double dt, int nsteps,
                   int64_t n, double* x, double* v, const double* m, double* acc, double* pot, int have_acc) {
    if (!c) return NBODY_ERR_ARG;
    if (int rc = check_common(c, prec, G, eps)) return rc;
    if (!isfinite(dt)) return set_err(c, NBODY_ERR_ARG, "dt must be finite");
    if (nsteps < 0) return set_err(c, NBODY_ERR_ARG, "nsteps must be >= 0");
    if (n < 0 || n > kMaxN) return set_err(c, NBODY_ERR_ARG, "n must be in [0, 2^31-1]");
    if (n > 0) {
        const void* need[5] = {x, v, m, acc, pot};
        const char* names[5] = {"x", "v", "m", "acc", "pot"};
        for (int k = 0; k < 5; ++k) {
            if (!need[k] && k < 4) return set_err(c, NBODY_ERR_ARG, "%s is NULL", names[k]);
            if (!aligned8(need[k])) return set_err(c, NBODY_ERR_ARG, "%s is not 8-byte aligned", names[k]);
        }
    }
    if (int rc = need_device(c)) return rc;
    if (n == 0) return NBODY_OK;
    DeviceGuard g(c->device);
    if (!g.ok) return set_err(c, NBODY_ERR_DEVICE, "hipSetDevice(%d) failed", c->device);
    const int p = (int)prec;
    // scratch: a potential row when the caller wants none, and an
    // acceleration block for a potential-only evaluation
    int rc = dev_alloc(c, c->lf, sizeof(double) * 4 * (size_t)n);
    if (rc) return rc;
    double* pot_s = (double*)c->lf.p;
    double* acc_s = pot_s + n;
    rc = dev_alloc(c, c->jpack, sizeof(float4) * rec_words(p) * (size_t)n);
    if (rc) return rc;
    const float4* jp = (const float4*)c->jpack.p;
    double* const prow = pot ? pot : pot_s;
    auto eval = [&](double* a3) {
        double* o[7] = {a3, a3 + n, a3 + 2 * n, nullptr, nullptr, nullptr, prow};
        return run_force(c, st, p, G, eps, n, jp, nullptr, nullptr, 2, n, jp, o, nullptr, 1);
    };
    nbody_src P{x, x + n, x + 2 * n, nullptr, nullptr, nullptr, m};
    if (!have_acc || (nsteps == 0 && pot)) {
        if ((rc = pack_rows(c, st, p, n, P, true, c->jpack))) return rc;
        if ((rc = eval(have_acc ? acc_s : acc))) return rc;
    }
    for (int s = 0; s < nsteps; ++s) {
        hipError_t e = launch_lf_kick_drift_pack(p, (int)n, x, v, acc, m, 0.5 * dt, dt, (float4*)c->jpack.p, st);
        if (e != hipSuccess) return hip_err(c, e, "leapfrog kick-drift launch");
        if ((rc = eval(acc))) return rc;
        e = launch_lf_kick((int)n, v, acc, 0.5 * dt, st);
        if (e != hipSuccess) return hip_err(c, e, "leapfrog kick launch");
    }
    return NBODY_OK;
}

int nbody_select_active(nbody_ctx* c, hipStream_t st, int64_t n, const int64_t* t, const int64_t* dt,
                        int32_t* idx, int64_t* n_act, int64_t* t_next) {
    if (!c) return NBODY_ERR_ARG;
    if (n < 0 || n > kMaxN) return set_err(c, NBODY_ERR_ARG, "n must be in [0, 2^31-1]");
    if (!n_act || !t_next) return set_err(c, NBODY_ERR_ARG, "n_act and t_next must be host pointers");
    if (n > 0 && (!t || !dt || !idx)) return set_err(c, NBODY_ERR_ARG, "t, dt and idx must not be NULL");
    if (int rc = need_device(c)) return rc;
    if (n == 0) {
        *n_act = 0;
        *t_next = 0;
        return NBODY_OK;
    }
    DeviceGuard g(c->device);
    int rc = dev_alloc(c, c->sel, (2 + (size_t)select_scratch_words((int)n)) * sizeof(int64_t));
    if (rc) return rc;
    hipError_t e = launch_select((int)n, t, dt, idx, (int64_t*)c->sel.p, (int64_t*)c->sel.p + 2, st);
    if (e != hipSuccess) return hip_err(c, e, "select launch");
    int64_t h[2];
    e = hipMemcpyAsync(h, c->sel.p, sizeof h, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_err(c, e, "select readback");
    *n_act = h[0];
    *t_next = h[1];
    return NBODY_OK;
}

// ---- Hermite driver ---------------------------------------------------------

int nbody_hermite_create(nbody_ctx* c, nbody_hermite** hp, int64_t n, const nbody_hermite_opts* o) {
    if (!c) return NBODY_ERR_ARG;
    if (!hp || !o) return set_err(c, NBODY_ERR_ARG, "NULL argument");
    *hp = nullptr;
    if (n <= 0 || n > kMaxN) return set_err(c, NBODY_ERR_ARG, "n must be in [1, 2^31-1]");
    if (int rc = check_common(c, o->prec, o->G, o->eps)) return rc;
    if (!(o->eta > 0.0) || !isfinite(o->eta) || !(o->eta_start > 0.0) || !isfinite(o->eta_start))
        return set_err(c, NBODY_ERR_ARG, "eta and eta_start must be positive and finite");
    if (o->shared_dt_log2 != 0) {
        if (o->shared_dt_log2 < -20 || o->shared_dt_log2 > -1)
            return set_err(c, NBODY_ERR_ARG, "shared_dt_log2 must be in [-20, -1] (or 0 for block steps)");
    } else if (o->dt_min_log2 < -20 || o->dt_max_log2 > 0 || o->dt_min_log2 > o->dt_max_log2) {
        return set_err(c, NBODY_ERR_ARG, "need -20 <= dt_min_log2 <= dt_max_log2 <= 0");
    }
    if (int rc = need_device(c)) return rc;
    DeviceGuard g(c->device);
    nbody_hermite* h = new (std::nothrow) nbody_hermite();
    if (!h) return set_err(c, NBODY_ERR_NOMEM, "host allocation failed");
    h->ctx = c;
    h->n = n;
    h->o = *o;
    if (const char* f = getenv("NBODY_BLOCK_GRAPH")) h->use_graph = atoi(f) != 0;
    if (const char* f = getenv("NBODY_FUSED_CORRECT")) h->fuse = atoi(f) != 0;
    const size_t nn = (size_t)n;
    // every piece below starts on a 256-byte boundary
    auto r256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t bytes = (13 + 7 + 6) * r256(sizeof(double) * nn) + 2 * r256(sizeof(int64_t) * nn) +
                         r256(sizeof(int32_t) * nn) + r256(sizeof(int64_t) * 2) + r256(sizeof(int64_t)) +
                         r256(sizeof(double) * 2) + 2 * r256(sizeof(DevPlan)) +
                         (o->shared_dt_log2 != 0 ? 2 * r256(sizeof(float4) * kRecDS * nn) : 0) +
                         r256(sizeof(int64_t) * blk_scratch_words((int)n)) +
                         r256(sizeof(uint64_t) * (blk_scratch_words((int)n) / 2 + 1)) +
                         r256(sizeof(TraceRec) * kTraceCap);
    ++c->alloc_count;
    if (c->fail_alloc_at > 0 && c->alloc_count == c->fail_alloc_at) {
        delete h;
        return set_err(c, NBODY_ERR_NOMEM, "device allocation of %zu bytes failed (injected)", bytes);
    }
    hipError_t e = hipMalloc(&h->block, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete h;
        return set_err(c, NBODY_ERR_NOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    char* p = (char*)h->block;
    auto take = [&](size_t b) {
        char* r = p;
        p += (b + 255) & ~(size_t)255;
        return (void*)r;
    };
    for (int k = 0; k < 13; ++k) h->s[k] = (double*)take(sizeof(double) * nn);
    for (int k = 0; k < 7; ++k) h->f[k] = (double*)take(sizeof(double) * nn);
    for (int k = 0; k < 6; ++k) h->pred[k] = (double*)take(sizeof(double) * nn);
    h->t = (int64_t*)take(sizeof(int64_t) * nn);
    h->dt = (int64_t*)take(sizeof(int64_t) * nn);
    h->idx = (int32_t*)take(sizeof(int32_t) * nn);
    h->sel2 = (int64_t*)take(sizeof(int64_t) * 2);
    h->tnow = (int64_t*)take(sizeof(int64_t));
    h->e2 = (double*)take(sizeof(double) * 2);
    h->plan = (DevPlan*)take(sizeof(DevPlan));
    h->splan = (DevPlan*)take(sizeof(DevPlan));
    if (o->shared_dt_log2 != 0) {   // shared steps only
        h->spack = (float4*)take(sizeof(float4) * kRecDS * nn);
        h->spack2 = (float4*)take(sizeof(float4) * kRecDS * nn);
    }
    h->gmin2 = (int64_t*)take(sizeof(int64_t) * blk_scratch_words((int)n));
    h->gpub = (uint64_t*)take(sizeof(uint64_t) * (blk_scratch_words((int)n) / 2 + 1));
    h->ftag = (uint32_t*)(h->gpub + blk_scratch_words((int)n) / 2);
    h->ring = (TraceRec*)take(sizeof(TraceRec) * kTraceCap);
    // the published counts start untagged (tag 0 is never used)
    e = launch_fill_i64((int64_t*)h->gpub, blk_scratch_words((int)n) / 2 + 1, 0, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        (void)hipFree(h->block);
        delete h;
        return hip_err(c, e, "hermite scratch clear");
    }
    *hp = h;
    return NBODY_OK;
}

int nbody_hermite_destroy(nbody_hermite* h) {
    if (!h) return NBODY_OK;
    if (h->block) {
        DeviceGuard g(h->ctx->device);
        if (h->bexec) (void)hipGraphExecDestroy(h->bexec);
        if (h->bgraph) (void)hipGraphDestroy(h->bgraph);
        (void)hipFree(h->block);
    }
    delete h;
    return NBODY_OK;
}

static nbody_src state_src(nbody_hermite* h) {
    nbody_src s;
    s.x = h->s[0]; s.y = h->s[1]; s.z = h->s[2];
    s.vx = h->s[3]; s.vy = h->s[4]; s.vz = h->s[5];
    s.m = h->s[12];
    return s;
}

int nbody_hermite_set_state(nbody_hermite* h, hipStream_t st, nbody_src P) {
    if (!h) return NBODY_ERR_ARG;
    nbody_ctx* c = h->ctx;
    if (int rc = check_src(c, P, true, "P")) return rc;
    DeviceGuard g(c->device);
    const size_t b = sizeof(double) * (size_t)h->n;
    const double* src[7] = {P.x, P.y, P.z, P.vx, P.vy, P.vz, P.m};
    const int dst[7] = {0, 1, 2, 3, 4, 5, 12};
    for (int k = 0; k < 7; ++k) {
        hipError_t e = hipMemcpyAsync(h->s[dst[k]], src[k], b, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_err(c, e, "state copy");
    }
    hipError_t e = launch_fill_i64(h->t, (int)h->n, 0, st);
    if (e == hipSuccess) e = launch_fill_i64(h->tnow, 1, 0, st);
    if (e != hipSuccess) return hip_err(c, e, "state clear");
    // initial a, jerk of every particle (self excluded), then first steps
    const int p = (int)h->o.prec;
    int rc = pack_rows(c, st, p, h->n, state_src(h), true, c->jpack);
    if (rc) return rc;
    double* o[7] = {h->s[6], h->s[7], h->s[8], h->s[9], h->s[10], h->s[11], h->f[6]};
    rc = run_force(c, st, p, h->o.G, h->o.eps, h->n, (const float4*)c->jpack.p, nullptr, nullptr, 2,
                   h->n, (const float4*)c->jpack.p, o, nullptr);
    if (rc) return rc;
    InitDtArgs a{};
    a.n = (int)h->n;
    a.ax = h->s[6]; a.ay = h->s[7]; a.az = h->s[8];
    a.jx = h->s[9]; a.jy = h->s[10]; a.jz = h->s[11];
    a.t = h->t;
    a.dt = h->dt;
    a.eta_s = h->o.eta_start;
    a.lmin = h->o.dt_min_log2;
    a.lmax = h->o.dt_max_log2;
    a.shared_log2 = h->o.shared_dt_log2;
    e = launch_init_dt(a, st);
    if (e != hipSuccess) return hip_err(c, e, "init dt launch");
    h->has_state = true;
    h->spack_tn = -1;
    h->gmin_ok = false;
    h->t_ticks = 0;
    h->steps = 0;
    h->sum_active = 0;
    return NBODY_OK;
}


// NBODY_TRACE: append one JSON line per step to the trace file (opened on
// first use; a file that cannot be opened turns tracing off for the context).
static FILE* trace_file(nbody_ctx* c) {
    if (c->trace_path.empty()) return nullptr;
    if (!c->trace) {
        c->trace = fopen(c->trace_path.c_str(), "a");
        if (!c->trace) c->trace_path.clear();
    }
    return c->trace;
}

static void trace_line(nbody_ctx* c, const char* mode, int64_t step, int64_t t_next, int64_t n_act,
                       const char* shape, int groups, int ranges) {
    FILE* f = trace_file(c);
    if (!f) return;
    fprintf(f,
            "{\"mode\": \"%s\", \"step\": %lld, \"t_ticks\": %lld, \"t\": %.17g, \"n_act\": %lld, "
            "\"shape\": \"%s\", \"groups\": %d, \"ranges\": %d}\n",
            mode, (long long)step, (long long)t_next, (double)t_next * kTick, (long long)n_act, shape, groups,
            ranges);
}

// The block steps from `after` (exclusive) up to the plan's count, from the
// device ring (synchronises `st`; tracing only).
static int trace_block_steps(nbody_hermite* h, hipStream_t st, int64_t after, int64_t upto) {
    nbody_ctx* c = h->ctx;
    if (!trace_file(c) || upto <= after) return NBODY_OK;
    TraceRec r[kTraceCap];
    hipError_t e = hipMemcpyAsync(r, h->ring, sizeof r, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_err(c, e, "trace read");
    const int64_t from = std::max(after + 1, upto - kTraceCap + 1);
    for (int64_t k = from; k <= upto; ++k) {
        const TraceRec& x = r[(k - 1) % kTraceCap];
        if (x.step != k) continue;
        const bool small = x.shape == 0;
        trace_line(c, "block", x.step, x.t_next, x.n_act, small ? "small" : "large", x.nb, x.S);
    }
    fflush(c->trace);
    return NBODY_OK;
}

static int plan_reset(nbody_hermite* h, hipStream_t st, int64_t t_limit) {
    DevPlan p{};
    p.steps = h->steps;
    p.sum_active = h->sum_active;
    p.t_last = h->t_ticks;
    p.t_limit = t_limit;
    p.ring = h->ctx->trace_path.empty() ? nullptr : h->ring;
    hipError_t e = hipMemcpyAsync(h->plan, &p, sizeof p, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_err(h->ctx, e, "plan write");
    return NBODY_OK;
}

static int plan_read(nbody_hermite* h, hipStream_t st, DevPlan* p) {
    hipError_t e = hipMemcpyAsync(p, h->plan, sizeof *p, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_err(h->ctx, e, "plan read");
    h->steps = p->steps;
    h->sum_active = p->sum_active;
    h->t_ticks = p->t_last;
    return NBODY_OK;
}

// Predict every particle to tick tn and pack it, into `out` (NULL: the
// context's j-pack buffer).
static int pack_predicted(nbody_hermite* h, hipStream_t st, int64_t tn, float4* out = nullptr) {
    nbody_ctx* c = h->ctx;
    const int p = (int)h->o.prec;
    const int n = (int)h->n;
    if (!out) {
        int rc = dev_alloc(c, c->jpack, sizeof(float4) * rec_words(p) * (size_t)n);
        if (rc) return rc;
        out = (float4*)c->jpack.p;
    }
    PackArgs pa{};
    pa.n = n;
    pa.prec = p;
    pa.x = h->s[0]; pa.y = h->s[1]; pa.z = h->s[2];
    pa.vx = h->s[3]; pa.vy = h->s[4]; pa.vz = h->s[5];
    pa.m = h->s[12];
    pa.ax = h->s[6]; pa.ay = h->s[7]; pa.az = h->s[8];
    pa.jx = h->s[9]; pa.jy = h->s[10]; pa.jz = h->s[11];
    pa.t = h->t;
    pa.tnext = nullptr;
    pa.tn = tn;
    pa.out = out;
    hipError_t e = launch_pack(pa, st);
    if (e != hipSuccess) return hip_err(c, e, "predict/pack launch");
    return NBODY_OK;
}

static CorrectArgs correct_args(nbody_hermite* h, int n_act) {
    CorrectArgs ca{};
    ca.n_act = n_act;
    ca.idx = h->idx;
    ca.tnext = h->sel2 + 1;
    ca.x = h->s[0]; ca.y = h->s[1]; ca.z = h->s[2];
    ca.vx = h->s[3]; ca.vy = h->s[4]; ca.vz = h->s[5];
    ca.ax = h->s[6]; ca.ay = h->s[7]; ca.az = h->s[8];
    ca.jx = h->s[9]; ca.jy = h->s[10]; ca.jz = h->s[11];
    ca.t = h->t;
    ca.dt = h->dt;
    for (int k = 0; k < 6; ++k) ca.f[k] = h->f[k];
    ca.eta = h->o.eta;
    ca.lmin = h->o.dt_min_log2;
    ca.lmax = h->o.dt_max_log2;
    ca.shared = h->o.shared_dt_log2 != 0;
    ca.tnow = h->tnow;
    return ca;
}

// Shared steps: every particle is due every step, so the block (all n, in
// order) and its time are known on the host: no selection pass, the block
// time goes to the kernels by value, and the i-list is the identity.  Two
// kernels per step: the pairwise kernel, then split reduce + corrector +
// prediction and packing of every particle for the next step (its records
// live in h->spack; a pack pass runs only when they are not current).
static int hermite_step_shared(nbody_hermite* h, hipStream_t st, int64_t t_limit, bool* stopped) {
    nbody_ctx* c = h->ctx;
    const int n = (int)h->n;
    const int64_t dtk = (int64_t)1 << (h->o.shared_dt_log2 + 20);
    const int64_t tn = h->t_ticks + dtk;
    *stopped = tn > t_limit;
    if (*stopped) return NBODY_OK;
    if (h->spack_tn != tn) {
        int rc = pack_predicted(h, st, tn, h->spack);
        if (rc) return rc;
        h->spack_tn = tn;
    }
    const int p = (int)h->o.prec;
    int S = 1;
    if (n < kSharedJparMax) {
        // small sets: the j-parallel pairwise launch of the block steps, with
        // a plan written once from the host (the block is every particle)
        if (!h->splan_S) {
            DevPlan sp{};
            sp.n_act = n;
            sp.shape = 0;
            jpar_plan(n, n, &sp.nb, &sp.S, &sp.jchunk);
            if (n <= kSharedOneRangeMax) {
                // every group sweeps all j and writes its forces: the
                // corrector then reads them without a split reduce
                sp.S = 1;
                sp.jchunk = n;
            }
            int rc = dev_alloc(c, c->part, sizeof(float2) * 7 * (size_t)sp.S * (size_t)n);
            if (rc) return rc;
            hipError_t e = hipMemcpy(h->splan, &sp, sizeof sp, hipMemcpyHostToDevice);
            if (e != hipSuccess) return hip_err(c, e, "plan write");
            h->splan_S = sp.S;
        }
        S = h->splan_S;
        ForceArgs a{};
        a.ipack = h->spack;
        a.jpack = h->spack;
        a.ni = n;
        a.nj = n;
        a.eps2 = (float)(h->o.eps * h->o.eps);
        a.G = h->o.G;
        a.self_mode = 2;
        a.keep_self = 1;   // each i record is its own j record: the self pair adds exactly 0 to a and jerk
        for (int q = 0; q < 7; ++q) a.out[q] = h->f[q];
        a.part = (float2*)c->part.p;
        a.plan = h->splan;
        if (h->fuse && S == 1 && n <= kSharedOneLaunchMax) {
            // one launch: each work-group's group of particles gets its
            // forces and is corrected there; the next step's records go to
            // the second buffer, as this launch still reads the first
            CorrectArgs ca = correct_args(h, n);
            ca.idx = nullptr;
            ca.tnext = nullptr;
            ca.tn = tn;
            ca.m = h->s[12];
            ca.pack_next = h->spack2;
            ca.tn_next = tn + dtk;
            ca.pack_prec = p;
            h->spack_tn = -1;   // until the records are swapped in below
            hipError_t e = launch_shared_step(p, h->o.eps == 0.0, a, ca, st);
            if (e != hipSuccess) return hip_err(c, e, "force/corrector launch");
            std::swap(h->spack, h->spack2);
            h->spack_tn = tn + dtk;
            h->t_ticks = tn;
            h->steps += 1;
            h->sum_active += n;
            if (trace_file(c)) {
                trace_line(c, "shared", h->steps, tn, n, "direct", 0, S);
                fflush(c->trace);
            }
            return NBODY_OK;
        }
        hipError_t e = launch_blk_step(p, h->o.eps == 0.0, a, st);
        if (e != hipSuccess) return hip_err(c, e, "force launch");
    } else {
        int rc = run_force(c, st, p, h->o.G, h->o.eps, n, h->spack, nullptr, nullptr, 2, n, h->spack, h->f, nullptr,
                           0, nullptr, nullptr, &S);
        if (rc) return rc;
    }
    ReduceArgs r{};
    r.ni = n;
    r.S = S;
    r.part = (const float2*)c->part.p;
    r.G = h->o.G;
    r.plan = nullptr;
    CorrectArgs ca = correct_args(h, n);
    ca.idx = nullptr;
    ca.tnext = nullptr;
    ca.tn = tn;
    ca.m = h->s[12];
    ca.pack_next = h->spack;
    ca.tn_next = tn + dtk;
    ca.pack_prec = p;
    // a wave per particle for the split reduce, else a thread per particle
    const int64_t threads = S > 1 ? 64 * (int64_t)n : (int64_t)n;
    const int grid = (int)std::min<int64_t>(1024, (threads + 255) / 256);
    h->spack_tn = -1;   // the records are being rewritten
    hipError_t e = launch_blk_reduce_correct(r, ca, grid, st);
    if (e != hipSuccess) return hip_err(c, e, "reduce/corrector launch");
    h->spack_tn = tn + dtk;
    h->t_ticks = tn;
    h->steps += 1;
    h->sum_active += n;
    if (trace_file(c)) {
        trace_line(c, "shared", h->steps, tn, n, "direct", 0, S);
        fflush(c->trace);
    }
    return NBODY_OK;
}

// Block steps: select + predict/pack + plan (three passes), force, then
// reduce + correct, all driven by the device plan (block size, split,
// end-time gate); a step past the gate leaves every state untouched.  No
// host synchronisation.
static int hermite_enqueue_block(nbody_hermite* h, hipStream_t st) {
    nbody_ctx* c = h->ctx;
    const int n = (int)h->n;
    const int p = (int)h->o.prec;
    PackArgs pa{};
    pa.n = n;
    pa.prec = p;
    pa.x = h->s[0]; pa.y = h->s[1]; pa.z = h->s[2];
    pa.vx = h->s[3]; pa.vy = h->s[4]; pa.vz = h->s[5];
    pa.m = h->s[12];
    pa.ax = h->s[6]; pa.ay = h->s[7]; pa.az = h->s[8];
    pa.jx = h->s[9]; pa.jy = h->s[10]; pa.jz = h->s[11];
    pa.t = h->t;
    pa.out = (float4*)c->jpack.p;
    const int G = blk_scratch_words(n) / 2;
    int64_t* gmin = h->gmin2 + (size_t)h->gpar * G;
    int64_t* gmin_next = h->gmin2 + (size_t)(h->gpar ^ 1) * G;
    const bool need_min = !h->gmin_ok;
    h->gmin_ok = false;   // until every launch of this step is in
    const bool eps0 = h->o.eps == 0.0;
#if NB_BLK_FRONT_FUSED
    hipError_t e = launch_blk_front_fused(pa, h->dt, h->idx, h->sel2, h->plan, h->gpub, h->ftag, gmin,
                                          gmin_next, need_min, !eps0, st);
#else
    hipError_t e = launch_blk_front(pa, h->dt, h->idx, h->sel2, h->plan, (int64_t*)c->sel.p + 2, gmin, gmin_next,
                                    need_min, !eps0, st);
#endif
    if (e != hipSuccess) return hip_err(c, e, "select/pack/plan launch");
    ForceArgs a{};
    a.ipack = (const float4*)c->jpack.p;
    a.iidx = h->idx;
    a.ni = n;
    a.jpack = (const float4*)c->jpack.p;
    a.nj = n;
    a.jchunk = n;
    a.eps2 = (float)(h->o.eps * h->o.eps);
    a.G = h->o.G;
    a.self_mode = 1;
    a.keep_self = 1;   // the i rows are the j records themselves; the potential is not read
    for (int q = 0; q < 7; ++q) a.out[q] = h->f[q];
    a.part = (float2*)c->part.p;
    a.plan = h->plan;
#if NB_BLK_STEP_FUSED
    e = launch_blk_step(p, eps0, a, st);
#else
    e = launch_force_plan(p, eps0, a, st);
#endif
    if (e != hipSuccess) return hip_err(c, e, "force launch");
    ReduceArgs r{};
    r.ni = n;
    r.part = a.part;
    r.G = h->o.G;
    for (int q = 0; q < 7; ++q) r.out[q] = h->f[q];
    r.plan = h->plan;
    // kBlkRcGrid work-groups of 256 threads, 16 particles each in the split
    // reduce, one per thread for the corrector alone; both stride over
    // larger blocks
    CorrectArgs ca = correct_args(h, n);
    ca.gmin_next = gmin_next;
    ca.gch = blk_chunk_size(n);
    e = launch_blk_reduce_correct(r, ca, kBlkRcGrid, st);
    if (e != hipSuccess) return hip_err(c, e, "reduce/corrector launch");
    h->gpar ^= 1;
    h->gmin_ok = true;
    return NBODY_OK;
}

static int block_buffers(nbody_hermite* h) {
    nbody_ctx* c = h->ctx;
    const int64_t n = h->n;
    const int words = std::max(select_scratch_words((int)n), blk_scratch_words((int)n));
    int rc = dev_alloc(c, c->sel, (2 + (size_t)words) * sizeof(int64_t));
    // split partials of a block step of any size (blk_part_rows); checked
    // once per integrator against the plan of every block size up to 2^21
    const int64_t rows = blk_part_rows(n, (int)h->o.prec);
    if (!h->part_checked) {
        const int big_ok = h->o.eps != 0.0;
        for (int64_t tot = 1; tot <= std::min<int64_t>(n, (int64_t)1 << 21); ++tot) {
            int nb, S, jc;
            blk_plan_geometry(tot, (int)n, big_ok, (int)h->o.prec, &nb, &S, &jc);
            if ((int64_t)S * tot > rows)
                return set_err(c, NBODY_ERR_STATE, "block plan for %lld of %lld particles needs %lld partial rows > %lld",
                               (long long)tot, (long long)n, (long long)S * tot, (long long)rows);
        }
        h->part_checked = true;
    }
    if (!rc) rc = dev_alloc(c, c->part, sizeof(float2) * 7 * (size_t)rows);
    if (!rc) rc = dev_alloc(c, c->jpack, sizeof(float4) * rec_words((int)h->o.prec) * (size_t)n);
    return rc;
}

// Run block steps until the next block time would pass t_limit (or, with
// max_steps > 0, at most that many steps); chunks of steps are enqueued
// with one readback each.
// With NBODY_BLOCK_GRAPH=1, once the chunk size has reached kBlkGraphSteps,
// long runs replay the chunk from one captured hipGraph (on MI355X this
// measured about 2 us per step slower than launching the steps, so it is
// not the default): every launch of a block step is
// plan-driven (sizes, shapes and the end-time gate come from device memory)
// and its kernel arguments do not change from step to step, except the
// kept chunk minima, which alternate between two buffers (an even step
// count brings them back).  Captured on the context's graph stream and
// ordered against the caller's stream by two events.
constexpr int kBlkGraphSteps = 64;
// Launched block steps go in chunks of 1, 2, 4, ... up to this many, with
// one plan readback (a host synchronisation) per chunk.  An advance that
// ends inside a chunk runs its remaining steps as no-ops (the end-time
// gate), so the chunk bounds that waste too.
#ifndef NB_BLK_CHUNK_MAX
#define NB_BLK_CHUNK_MAX 256
#endif
constexpr int kBlkChunkMax = NB_BLK_CHUNK_MAX;

static int block_graph_launch(nbody_hermite* h, hipStream_t st) {
    nbody_ctx* c = h->ctx;
    hipError_t e = hipSuccess;
    if (!c->gstream) {
        e = hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->gev[0], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->gev[1], hipEventDisableTiming);
        if (e != hipSuccess) return hip_err(c, e, "graph stream setup");
    }
    const std::vector<uint64_t> key = {(uintptr_t)c->jpack.p, (uintptr_t)c->part.p, (uintptr_t)c->sel.p,
                                       (uint64_t)h->gpar};
    if (!h->bexec || h->bkey != key) {
        if (h->bexec) (void)hipGraphExecDestroy(h->bexec);
        if (h->bgraph) (void)hipGraphDestroy(h->bgraph);
        h->bexec = nullptr;
        h->bgraph = nullptr;
        e = hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_err(c, e, "begin capture");
        int rc = NBODY_OK;
        for (int k = 0; k < kBlkGraphSteps && !rc; ++k) rc = hermite_enqueue_block(h, c->gstream);
        hipGraph_t gr = nullptr;
        const hipError_t e2 = hipStreamEndCapture(c->gstream, &gr);
        if (rc) {
            if (gr) (void)hipGraphDestroy(gr);
            return rc;
        }
        if (e2 != hipSuccess) return hip_err(c, e2, "end capture");
        e = hipGraphInstantiate(&h->bexec, gr, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(gr);
            h->bexec = nullptr;
            return hip_err(c, e, "graph instantiate");
        }
        h->bgraph = gr;
        h->bkey = key;
    }
    e = hipEventRecord(c->gev[0], st);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->gstream, c->gev[0], 0);
    if (e == hipSuccess) e = hipGraphLaunch(h->bexec, c->gstream);
    if (e == hipSuccess) e = hipEventRecord(c->gev[1], c->gstream);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, c->gev[1], 0);
    if (e != hipSuccess) return hip_err(c, e, "graph launch");
    return NBODY_OK;
}

static int hermite_block_run(nbody_hermite* h, hipStream_t st, int64_t t_limit, int64_t max_steps,
                             int64_t* last_nact) {
    int rc = block_buffers(h);
    if (!rc) rc = plan_reset(h, st, t_limit);
    if (rc) return rc;
    int64_t done = 0;
    int chunk = 1;
    for (;;) {
        int k = chunk;
        if (max_steps > 0) k = (int)std::min<int64_t>(k, max_steps - done);
        if (h->use_graph && max_steps == 0 && k == kBlkGraphSteps && h->gmin_ok) {
            rc = block_graph_launch(h, st);
            if (rc) return rc;
        } else {
            for (int s = 0; s < k; ++s) {
                rc = hermite_enqueue_block(h, st);
                if (rc) return rc;
            }
        }
        done += k;
        DevPlan p;
        const int64_t before = h->steps;
        rc = plan_read(h, st, &p);
        if (rc) return rc;
        if ((rc = trace_block_steps(h, st, before, p.steps))) return rc;
        if (p.frozen == 2)
            return set_err(h->ctx, NBODY_ERR_DEVICE,
                           "block step: a wait for the chunk counts of the front end did not end");
        if (last_nact) *last_nact = p.frozen ? 0 : p.n_act;
        if (p.frozen || (max_steps > 0 && done >= max_steps)) break;
        // chunks of launched steps grow to kBlkChunkMax; a captured graph
        // replays kBlkGraphSteps, and the trace ring holds kTraceCap
        const int cap = h->use_graph ? kBlkGraphSteps : trace_file(h->ctx) ? kTraceCap : kBlkChunkMax;
        chunk = std::min(chunk * 2, cap);
    }
    return NBODY_OK;
}

int nbody_hermite_step(nbody_hermite* h, hipStream_t st, int64_t* n_active, int64_t* t_ticks) {
    if (!h) return NBODY_ERR_ARG;
    if (!h->has_state) return set_err(h->ctx, NBODY_ERR_STATE, "hermite: set_state or load first");
    DeviceGuard g(h->ctx->device);
    if (h->o.shared_dt_log2 != 0) {
        bool stopped = false;
        int rc = hermite_step_shared(h, st, INT64_MAX, &stopped);
        if (rc) return rc;
        if (n_active) *n_active = h->n;
        if (t_ticks) *t_ticks = h->t_ticks;
        return NBODY_OK;
    }
    int64_t na = 0;
    int rc = hermite_block_run(h, st, INT64_MAX, 1, &na);
    if (rc) return rc;
    if (n_active) *n_active = na;
    if (t_ticks) *t_ticks = h->t_ticks;
    return NBODY_OK;
}

int nbody_hermite_advance(nbody_hermite* h, hipStream_t st, int64_t t_end, nbody_hermite_stats* stats) {
    if (!h) return NBODY_ERR_ARG;
    if (!h->has_state) return set_err(h->ctx, NBODY_ERR_STATE, "hermite: set_state or load first");
    DeviceGuard g(h->ctx->device);
    if (h->o.shared_dt_log2 != 0) {
        for (;;) {
            bool stopped = false;
            int rc = hermite_step_shared(h, st, t_end, &stopped);
            if (rc) return rc;
            if (stopped) break;
        }
    } else {
        int rc = hermite_block_run(h, st, t_end, 0, nullptr);
        if (rc) return rc;
    }
    if (stats) {
        stats->steps = h->steps;
        stats->sum_active = h->sum_active;
        stats->t_ticks = h->t_ticks;
    }
    return NBODY_OK;
}

int nbody_hermite_get_state(nbody_hermite* h, hipStream_t st, nbody_src P, double* ax, double* ay,
                            double* az, double* jx, double* jy, double* jz, int64_t* t, int64_t* dt) {
    if (!h) return NBODY_ERR_ARG;
    nbody_ctx* c = h->ctx;
    if (!h->has_state) return set_err(c, NBODY_ERR_STATE, "hermite: no state");
    DeviceGuard g(c->device);
    const size_t b = sizeof(double) * (size_t)h->n;
    const void* src[15] = {h->s[0], h->s[1], h->s[2], h->s[3], h->s[4], h->s[5], h->s[12], h->s[6],
                           h->s[7], h->s[8], h->s[9], h->s[10], h->s[11], h->t, h->dt};
    void* dst[15] = {(void*)P.x, (void*)P.y, (void*)P.z, (void*)P.vx, (void*)P.vy, (void*)P.vz,
                     (void*)P.m, ax, ay, az, jx, jy, jz, t, dt};
    for (int k = 0; k < 15; ++k) {
        if (!dst[k]) continue;
        hipError_t e = hipMemcpyAsync(dst[k], src[k], b, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_err(c, e, "state copy out");
    }
    return NBODY_OK;
}

int nbody_hermite_energy(nbody_hermite* h, hipStream_t st, double* ekin, double* epot) {
    if (!h) return NBODY_ERR_ARG;
    nbody_ctx* c = h->ctx;
    if (!ekin || !epot) return set_err(c, NBODY_ERR_ARG, "ekin and epot must be host pointers");
    if (!h->has_state) return set_err(c, NBODY_ERR_STATE, "hermite: no state");
    DeviceGuard g(c->device);
    const int n = (int)h->n;
    const double* s[12];
    for (int k = 0; k < 12; ++k) s[k] = h->s[k];
    hipError_t e = launch_predict_all(n, s, h->t, h->tnow, h->pred, st);
    if (e != hipSuccess) return hip_err(c, e, "predict launch");
    nbody_src P;
    P.x = h->pred[0]; P.y = h->pred[1]; P.z = h->pred[2];
    P.vx = h->pred[3]; P.vy = h->pred[4]; P.vz = h->pred[5];
    P.m = h->s[12];
    const int p = (int)h->o.prec;
    int rc = pack_rows(c, st, p, n, P, true, c->jpack);
    if (rc) return rc;
    double* o[7] = {h->f[0], h->f[1], h->f[2], h->f[3], h->f[4], h->f[5], h->f[6]};
    rc = run_force(c, st, p, h->o.G, h->o.eps, n, (const float4*)c->jpack.p, nullptr, nullptr, 2, n,
                   (const float4*)c->jpack.p, o, nullptr);
    if (rc) return rc;
    e = launch_energy(n, h->pred[3], h->pred[4], h->pred[5], h->s[12], h->f[6], h->e2, st);
    if (e != hipSuccess) return hip_err(c, e, "energy launch");
    double r[2];
    e = hipMemcpyAsync(r, h->e2, sizeof r, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_err(c, e, "energy readback");
    *ekin = r[0];
    *epot = r[1];
    return NBODY_OK;
}

// Checkpoint layout: header (n, t_ticks, steps, sum_active), then 13 float64
// rows (x y z vx vy vz ax ay az jx jy jz m), then t and dt int64 rows.
int64_t nbody_hermite_state_bytes(const nbody_hermite* h) {
    if (!h) return 0;
    return (int64_t)(4 * sizeof(int64_t) + (13 * sizeof(double) + 2 * sizeof(int64_t)) * (size_t)h->n);
}

int nbody_hermite_save(nbody_hermite* h, hipStream_t st, void* buf) {
    if (!h) return NBODY_ERR_ARG;
    nbody_ctx* c = h->ctx;
    if (!buf) return set_err(c, NBODY_ERR_ARG, "NULL buffer");
    if (!h->has_state) return set_err(c, NBODY_ERR_STATE, "hermite: no state");
    DeviceGuard g(c->device);
    int64_t* hdr = (int64_t*)buf;
    hdr[0] = h->n;
    hdr[1] = h->t_ticks;
    hdr[2] = h->steps;
    hdr[3] = h->sum_active;
    char* p = (char*)buf + 4 * sizeof(int64_t);
    const size_t b = sizeof(double) * (size_t)h->n;
    for (int k = 0; k < 13; ++k, p += b) {
        hipError_t e = hipMemcpyAsync(p, h->s[k], b, hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return hip_err(c, e, "save copy");
    }
    hipError_t e = hipMemcpyAsync(p, h->t, b, hipMemcpyDeviceToHost, st);
    p += b;
    if (e == hipSuccess) e = hipMemcpyAsync(p, h->dt, b, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_err(c, e, "save copy");
    return NBODY_OK;
}

int nbody_hermite_load(nbody_hermite* h, hipStream_t st, const void* buf) {
    if (!h) return NBODY_ERR_ARG;
    nbody_ctx* c = h->ctx;
    if (!buf) return set_err(c, NBODY_ERR_ARG, "NULL buffer");
    const int64_t* hdr = (const int64_t*)buf;
    if (hdr[0] != h->n) return set_err(c, NBODY_ERR_ARG, "checkpoint holds %lld particles, driver %lld",
                                       (long long)hdr[0], (long long)h->n);
    DeviceGuard g(c->device);
    const char* p = (const char*)buf + 4 * sizeof(int64_t);
    const size_t b = sizeof(double) * (size_t)h->n;
    for (int k = 0; k < 13; ++k, p += b) {
        hipError_t e = hipMemcpyAsync(h->s[k], p, b, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_err(c, e, "load copy");
    }
    hipError_t e = hipMemcpyAsync(h->t, p, b, hipMemcpyHostToDevice, st);
    p += b;
    if (e == hipSuccess) e = hipMemcpyAsync(h->dt, p, b, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(h->tnow, &hdr[1], sizeof(int64_t), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_err(c, e, "load copy");
    h->t_ticks = hdr[1];
    h->steps = hdr[2];
    h->sum_active = hdr[3];
    h->has_state = true;
    h->spack_tn = -1;
    h->gmin_ok = false;
    return NBODY_OK;
}

// ---- adjoint ----------------------------------------------------------------

static int vjp_split(int64_t nl, int64_t nt) {
    const int64_t nblk = (nl + vjp_wg() - 1) / vjp_wg();
    const int64_t target = 2048;
    if (nblk <= 0 || nblk >= target / 2) return 1;
    int64_t S = (target + nblk - 1) / nblk;
    S = std::min<int64_t>(S, std::max<int64_t>(1, nt / (2 * (int64_t)vjp_tile())));
    return (int)std::max<int64_t>(1, S);
}

static int pack_vjp(nbody_ctx* c, hipStream_t st, int prec, int64_t n, const nbody_src& s,
                    const double* ga, const double* gj, const double* gp, int key_mode,
                    const int32_t* iself, DevBuf& dst) {
    int rc = dev_alloc(c, dst, sizeof(float4) * 5 * (size_t)std::max<int64_t>(n, 1));
    if (rc) return rc;
    VjpPackArgs p{};
    p.n = (int)n;
    p.prec = prec;
    p.x = s.x; p.y = s.y; p.z = s.z;
    p.vx = s.vx; p.vy = s.vy; p.vz = s.vz;
    p.m = s.m;
    p.ga = ga; p.gj = gj; p.gp = gp;
    p.key_mode = key_mode;
    p.iself = iself;
    p.out = (float4*)dst.p;
    hipError_t e = launch_vjp_pack(p, st);
    if (e != hipSuccess) return hip_err(c, e, "adjoint pack launch");
    return NBODY_OK;
}

static int run_vjp(nbody_ctx* c, hipStream_t st, int prec, bool own, bool partner, double G, double eps,
                   int64_t nl, const float4* lrec, int64_t nt, const float4* trec, const double* ga,
                   const double* gj, double* gx, double* gv, double* gm) {
    if (nl == 0) return NBODY_OK;
    const int Sreq = vjp_split(nl, nt);
    int64_t jchunk = (nt + Sreq - 1) / Sreq;
    jchunk = ((jchunk + vjp_tile() - 1) / vjp_tile()) * vjp_tile();
    if (jchunk <= 0) jchunk = vjp_tile();
    const int S = (int)std::max<int64_t>(1, (nt + jchunk - 1) / jchunk);
    VjpArgs a{};
    a.lrec = lrec;
    a.nl = (int)nl;
    a.trec = trec;
    a.nt = (int)nt;
    a.jchunk = (int)jchunk;
    a.eps2 = (float)(eps * eps);
    a.G = G;
    a.own = own ? 1 : 0;
    a.ga = ga;
    a.gj = gj;
    a.gx = gx;
    a.gv = gv;
    a.gm = gm;
    if (S > 1) {
        int rc = dev_alloc(c, c->vpart, sizeof(float2) * (size_t)vjp_acc() * (size_t)S * (size_t)nl);
        if (rc) return rc;
        a.part = (float2*)c->vpart.p;
    }
    hipError_t e = launch_vjp(prec, own, partner, S, a, st);
    if (e != hipSuccess) return hip_err(c, e, "adjoint kernel launch");
    return NBODY_OK;
}

static int check_rows3(nbody_ctx* c, const void* p, const char* name) {
    if (p && !aligned8(p)) return set_err(c, NBODY_ERR_ARG, "%s is not 8-byte aligned", name);
    return NBODY_OK;
}

int nbody_force_vjp(nbody_ctx* c, hipStream_t st, nbody_prec prec, double G, double eps, int64_t n_i,
                    nbody_src I, const int32_t* i_self, int64_t n_j, nbody_src J, const double* ga,
                    const double* gj, const double* gp, double* gxi, double* gvi, double* gxj, double* gvj,
                    double* gmj) {
    if (!c) return NBODY_ERR_ARG;
    if (int rc = check_common(c, prec, G, eps)) return rc;
    if (n_i < 0 || n_j < 0 || n_i > kMaxN || n_j > kMaxN)
        return set_err(c, NBODY_ERR_ARG, "n_i and n_j must be in [0, 2^31-1]");
    if (n_i > 0 && !ga) return set_err(c, NBODY_ERR_ARG, "ga must not be NULL");
    const void* rows[8] = {ga, gj, gp, gxi, gvi, gxj, gvj, gmj};
    const char* names[8] = {"ga", "gj", "gp", "gxi", "gvi", "gxj", "gvj", "gmj"};
    for (int k = 0; k < 8; ++k)
        if (int rc = check_rows3(c, rows[k], names[k])) return rc;
    if (n_i > 0)
        if (int rc = check_src(c, I, false, "I")) return rc;
    if (n_j > 0)
        if (int rc = check_src(c, J, true, "J")) return rc;
    if (int rc = need_device(c)) return rc;
    DeviceGuard g(c->device);
    if (!g.ok) return set_err(c, NBODY_ERR_DEVICE, "hipSetDevice(%d) failed", c->device);
    const int p = (int)prec;
    const bool want_i = n_i > 0 && (gxi || gvi);
    const bool want_j = n_j > 0 && (gxj || gvj || gmj);
    if (n_i == 0 && want_j == false) return NBODY_OK;
    int rc = NBODY_OK;
    if (n_i > 0) rc = pack_vjp(c, st, p, n_i, I, ga, gj, gp, 1, i_self, c->vrec_i);
    if (!rc && n_j > 0) rc = pack_vjp(c, st, p, n_j, J, nullptr, nullptr, nullptr, 0, nullptr, c->vrec_j);
    if (rc) return rc;
    if (want_i)
        rc = run_vjp(c, st, p, true, false, G, eps, n_i, (const float4*)c->vrec_i.p, n_j,
                     (const float4*)c->vrec_j.p, ga, gj, gxi, gvi, nullptr);
    if (!rc && want_j)
        rc = run_vjp(c, st, p, false, true, G, eps, n_j, (const float4*)c->vrec_j.p, n_i,
                     (const float4*)c->vrec_i.p, nullptr, nullptr, gxj, gvj, gmj);
    // (an empty partner set gives a launch with no tiles, which writes zeros)
    return rc;
}

int nbody_force_vjp_self(nbody_ctx* c, hipStream_t st, nbody_prec prec, double G, double eps, int64_t n,
                         nbody_src P, const double* ga, const double* gj, const double* gp, double* gx,
                         double* gv, double* gm) {
    if (!c) return NBODY_ERR_ARG;
    if (int rc = check_common(c, prec, G, eps)) return rc;
    if (n < 0 || n > kMaxN) return set_err(c, NBODY_ERR_ARG, "n must be in [0, 2^31-1]");
    if (n > 0 && !ga) return set_err(c, NBODY_ERR_ARG, "ga must not be NULL");
    const void* rows[6] = {ga, gj, gp, gx, gv, gm};
    const char* names[6] = {"ga", "gj", "gp", "gx", "gv", "gm"};
    for (int k = 0; k < 6; ++k)
        if (int rc = check_rows3(c, rows[k], names[k])) return rc;
    if (n > 0)
        if (int rc = check_src(c, P, true, "P")) return rc;
    if (int rc = need_device(c)) return rc;
    if (n == 0 || !(gx || gv || gm)) return NBODY_OK;
    DeviceGuard g(c->device);
    if (!g.ok) return set_err(c, NBODY_ERR_DEVICE, "hipSetDevice(%d) failed", c->device);
    const int p = (int)prec;
    int rc = pack_vjp(c, st, p, n, P, ga, gj, gp, 0, nullptr, c->vrec_i);
    if (rc) return rc;
    return run_vjp(c, st, p, true, true, G, eps, n, (const float4*)c->vrec_i.p, n, (const float4*)c->vrec_i.p,
                   ga, gj, gx, gv, gm);
}

// ---- shared-step run and its adjoint -------------------------------------------

namespace {
struct SharedWS {
    double *x, *v, *a, *j, *f, *X, *V, *Aa, *Jj, *ga, *gj, *tx, *tv, *tm;
};
}  // namespace

static int shared_ws(nbody_ctx* c, int64_t n, SharedWS* w) {
    const size_t n3 = 3 * (size_t)n, nn = (size_t)n;
    const size_t per = 12 * n3 + 8 * nn;   // x v a j X V Aa Jj ga gj tx tv (3n each), f (7n), tm (n)
    int rc = dev_alloc(c, c->integ, sizeof(double) * per);
    if (rc) return rc;
    double* p = (double*)c->integ.p;
    double** v3[] = {&w->x, &w->v, &w->a, &w->j, &w->X, &w->V, &w->Aa, &w->Jj, &w->ga, &w->gj, &w->tx, &w->tv};
    for (double** q : v3) {
        *q = p;
        p += n3;
    }
    w->f = p;
    p += 7 * nn;
    w->tm = p;
    return NBODY_OK;
}

static int copy_src3(nbody_ctx* c, hipStream_t st, int64_t n, const double* r0, const double* r1,
                     const double* r2, double* dst) {
    const size_t b = sizeof(double) * (size_t)n;
    const double* rows[3] = {r0, r1, r2};
    for (int k = 0; k < 3; ++k) {
        hipError_t e = hipMemcpyAsync(dst + k * (size_t)n, rows[k], b, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_err(c, e, "state copy");
    }
    return NBODY_OK;
}

static nbody_src rows_src(const double* x, const double* v, const double* m, int64_t n) {
    nbody_src s;
    s.x = x; s.y = x + n; s.z = x + 2 * n;
    s.vx = v; s.vy = v + n; s.vz = v + 2 * n;
    s.m = m;
    return s;
}

// a, j (and pot into f + 6n) of the set (x, v, m) with self excluded.
static int shared_force(nbody_ctx* c, hipStream_t st, int prec, double G, double eps, int64_t n,
                        const double* x, const double* v, const double* m, double* a3, double* j3,
                        double* pot) {
    int rc = pack_rows(c, st, prec, n, rows_src(x, v, m, n), true, c->jpack);
    if (rc) return rc;
    double* o[7] = {a3, a3 + n, a3 + 2 * n, j3, j3 + n, j3 + 2 * n, pot};
    return run_force(c, st, prec, G, eps, n, (const float4*)c->jpack.p, nullptr, nullptr, 2, n,
                     (const float4*)c->jpack.p, o, nullptr);
}

// One step from (w.x, w.v, w.a, w.j); the predicted state goes to xp, vp.
static int shared_step(nbody_ctx* c, hipStream_t st, int prec, double G, double eps, double D, int64_t n,
                       const double* m, SharedWS& w, double* xp, double* vp) {
    hipError_t e = launch_shared_predict((int)n, D, w.x, w.v, w.a, w.j, xp, vp, st);
    if (e != hipSuccess) return hip_err(c, e, "predict launch");
    int rc = shared_force(c, st, prec, G, eps, n, xp, vp, m, w.f, w.f + 3 * n, w.f + 6 * n);
    if (rc) return rc;
    e = launch_shared_correct((int)n, D, xp, vp, w.x, w.v, w.a, w.j, w.f, w.f + 3 * n, st);
    if (e != hipSuccess) return hip_err(c, e, "corrector launch");
    return NBODY_OK;
}

static int check_shared(nbody_ctx* c, nbody_prec prec, double G, double eps, double dt, int nsteps, int64_t n,
                        int every) {
    if (int rc = check_common(c, prec, G, eps)) return rc;
    if (!(dt > 0.0) || !isfinite(dt)) return set_err(c, NBODY_ERR_ARG, "dt must be positive and finite");
    if (nsteps < 0) return set_err(c, NBODY_ERR_ARG, "nsteps must be >= 0");
    if (n < 1 || n > kMaxShared)
        return set_err(c, NBODY_ERR_ARG, "n must be in [1, %lld] (3n vector entries are indexed in int32)",
                       (long long)kMaxShared);
    if (every < 1) return set_err(c, NBODY_ERR_ARG, "ckpt_every must be >= 1");
    return NBODY_OK;
}

int64_t nbody_shared_ckpt_bytes(int64_t n, int nsteps, int every) {
    if (n < 1 || n > kMaxShared || nsteps < 0 || every < 1) return -1;
    const int64_t nseg = (nsteps + every - 1) / every;
    return std::max<int64_t>(nseg, 1) * 12 * n * (int64_t)sizeof(double);
}

int nbody_shared_run(nbody_ctx* c, hipStream_t st, nbody_prec prec, double G, double eps, double dt, int nsteps,
                     int64_t n, nbody_src P0, double* x_out, double* v_out, double* ckpt, int every) {
    if (!c) return NBODY_ERR_ARG;
    if (int rc = check_shared(c, prec, G, eps, dt, nsteps, n, every)) return rc;
    if (int rc = check_src(c, P0, true, "P0")) return rc;
    if (!x_out || !v_out || !aligned8(x_out) || !aligned8(v_out) || (ckpt && !aligned8(ckpt)))
        return set_err(c, NBODY_ERR_ARG, "x_out and v_out must be 8-byte aligned device pointers");
    if (int rc = need_device(c)) return rc;
    DeviceGuard g(c->device);
    SharedWS w;
    int rc = shared_ws(c, n, &w);
    if (rc) return rc;
    const int p = (int)prec;
    rc = copy_src3(c, st, n, P0.x, P0.y, P0.z, w.x);
    if (!rc) rc = copy_src3(c, st, n, P0.vx, P0.vy, P0.vz, w.v);
    if (!rc) rc = shared_force(c, st, p, G, eps, n, w.x, w.v, P0.m, w.a, w.j, w.f + 6 * n);
    if (rc) return rc;
    const size_t n3 = 3 * (size_t)n;
    // predicted states of a step land in the tx / tv scratch rows
    for (int s = 0; s < nsteps; ++s) {
        if (ckpt && s % every == 0) {
            double* cp = ckpt + (size_t)(s / every) * 4 * n3;
            const double* src[4] = {w.x, w.v, w.a, w.j};
            for (int k = 0; k < 4; ++k) {
                hipError_t e = hipMemcpyAsync(cp + k * n3, src[k], sizeof(double) * n3, hipMemcpyDeviceToDevice, st);
                if (e != hipSuccess) return hip_err(c, e, "checkpoint copy");
            }
        }
        rc = shared_step(c, st, p, G, eps, dt, n, P0.m, w, w.tx, w.tv);
        if (rc) return rc;
    }
    hipError_t e = hipMemcpyAsync(x_out, w.x, sizeof(double) * n3, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(v_out, w.v, sizeof(double) * n3, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_err(c, e, "state copy out");
    return NBODY_OK;
}

int nbody_shared_adjoint(nbody_ctx* c, hipStream_t st, nbody_prec prec, double G, double eps, double dt,
                         int nsteps, int64_t n, nbody_src P0, const double* ckpt, int every, const double* gx_end,
                         const double* gv_end, double* gx0, double* gv0, double* gm) {
    if (!c) return NBODY_ERR_ARG;
    if (int rc = check_shared(c, prec, G, eps, dt, nsteps, n, every)) return rc;
    if (int rc = check_src(c, P0, true, "P0")) return rc;
    if (nsteps > 0 && !ckpt) return set_err(c, NBODY_ERR_ARG, "ckpt must hold the forward checkpoints");
    if (!gx_end || !gx0 || !gv0 || !gm) return set_err(c, NBODY_ERR_ARG, "NULL gradient pointer");
    const void* al[6] = {ckpt, gx_end, gv_end, gx0, gv0, gm};
    for (const void* q : al)
        if (q && !aligned8(q)) return set_err(c, NBODY_ERR_ARG, "pointer not 8-byte aligned");
    if (int rc = need_device(c)) return rc;
    DeviceGuard g(c->device);
    SharedWS w;
    int rc = shared_ws(c, n, &w);
    if (rc) return rc;
    const int p = (int)prec;
    const size_t n3 = 3 * (size_t)n;
    const int every_eff = std::min(every, std::max(nsteps, 1));
    rc = dev_alloc(c, c->hist, sizeof(double) * 2 * n3 * (size_t)every_eff);
    if (rc) return rc;
    double* hist = (double*)c->hist.p;
    hipError_t e = hipMemcpyAsync(w.X, gx_end, sizeof(double) * n3, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_err(c, e, "cotangent copy");
    if (gv_end) {
        e = hipMemcpyAsync(w.V, gv_end, sizeof(double) * n3, hipMemcpyDeviceToDevice, st);
    } else {
        e = launch_fill_f64((int)n3, w.V, 0.0, st);
    }
    if (e == hipSuccess) e = launch_fill_f64((int)n3, w.Aa, 0.0, st);
    if (e == hipSuccess) e = launch_fill_f64((int)n3, w.Jj, 0.0, st);
    if (e == hipSuccess) e = launch_fill_f64((int)n, gm, 0.0, st);
    if (e != hipSuccess) return hip_err(c, e, "adjoint clear");
    const int nseg = (nsteps + every - 1) / every;
    for (int seg = nseg - 1; seg >= 0; --seg) {
        const int s0 = seg * every, s1 = std::min(nsteps, s0 + every);
        const double* cp = ckpt + (size_t)seg * 4 * n3;
        double* dst[4] = {w.x, w.v, w.a, w.j};
        for (int k = 0; k < 4; ++k) {
            e = hipMemcpyAsync(dst[k], cp + k * n3, sizeof(double) * n3, hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return hip_err(c, e, "checkpoint restore");
        }
        for (int s = s0; s < s1; ++s) {
            double* xp = hist + (size_t)(s - s0) * 2 * n3;
            rc = shared_step(c, st, p, G, eps, dt, n, P0.m, w, xp, xp + n3);
            if (rc) return rc;
        }
        for (int s = s1 - 1; s >= s0; --s) {
            const double* xp = hist + (size_t)(s - s0) * 2 * n3;
            e = launch_adj_correct((int)n, dt, w.X, w.V, w.Aa, w.Jj, w.ga, w.gj, st);
            if (e != hipSuccess) return hip_err(c, e, "corrector adjoint launch");
            rc = pack_vjp(c, st, p, n, rows_src(xp, xp + n3, P0.m, n), w.ga, w.gj, nullptr, 0, nullptr, c->vrec_i);
            if (!rc)
                rc = run_vjp(c, st, p, true, true, G, eps, n, (const float4*)c->vrec_i.p, n,
                             (const float4*)c->vrec_i.p, w.ga, w.gj, w.tx, w.tv, w.tm);
            if (rc) return rc;
            e = launch_axpy((int)n, gm, w.tm, st);
            if (e == hipSuccess) e = launch_adj_predict((int)n, dt, w.X, w.V, w.Aa, w.Jj, w.tx, w.tv, st);
            if (e != hipSuccess) return hip_err(c, e, "predictor adjoint launch");
        }
    }
    // initial evaluation (a0, j0) = F(x0, v0, m)
    rc = copy_src3(c, st, n, P0.x, P0.y, P0.z, w.x);
    if (!rc) rc = copy_src3(c, st, n, P0.vx, P0.vy, P0.vz, w.v);
    if (!rc) rc = pack_vjp(c, st, p, n, rows_src(w.x, w.v, P0.m, n), w.Aa, w.Jj, nullptr, 0, nullptr, c->vrec_i);
    if (!rc)
        rc = run_vjp(c, st, p, true, true, G, eps, n, (const float4*)c->vrec_i.p, n, (const float4*)c->vrec_i.p,
                     w.Aa, w.Jj, w.tx, w.tv, w.tm);
    if (rc) return rc;
    e = launch_axpy((int)n, gm, w.tm, st);
    if (e == hipSuccess) e = launch_sum2((int)n3, gx0, w.X, w.tx, st);
    if (e == hipSuccess) e = launch_sum2((int)n3, gv0, w.V, w.tv, st);
    if (e != hipSuccess) return hip_err(c, e, "adjoint final launch");
    return NBODY_OK;
}

// ---- batched clusters -----------------------------------------------------------

static nbody_tile batched_tile(nbody_ctx* c, int prec, int64_t n_total, int32_t n_clusters) {
    nbody_tile t;
    if (c->have_override[prec]) {
        t = c->override_tile[prec];
    } else if (!c->tune.lookup(prec + 2, n_total, n_clusters, &t)) {
        t.tile_j = 64;
        t.ipt = 1;
        t.wg = 128;
        t.split = 1;
        t.jsrc = 0;
    }
    if (t.jsrc != 0 || t.unroll != 0 || t.waves != 0 || !force_variant_exists(prec, t.ipt, t.tile_j, t.wg, 0, 4, 0, false)) {
        t.tile_j = 128;
        t.jsrc = 0;
        if (t.wg != 128 && t.wg != 256) t.wg = 256;
    }
    t.unroll = 0;
    t.waves = 0;
    t.split = 1;
    return t;
}

namespace {
struct BatchWS {
    int *cbeg, *cend, *order, *start, *n_items, *counters;
    int2* items;
    int64_t cap;
};
}  // namespace

static int batch_ws(nbody_ctx* c, int32_t C, int64_t n_total, int nsteps, BatchWS* w) {
    const int64_t cap = n_total / 64 + (int64_t)C + 1;
    const size_t ints = 4 * (size_t)std::max(C, 1) + 1 + (size_t)std::max(nsteps, 1);
    const size_t bytes = sizeof(int2) * (size_t)cap + sizeof(int) * ints + 256;
    int rc = dev_alloc(c, c->bplan, bytes);
    if (rc) return rc;
    int2* it = (int2*)c->bplan.p;
    int* p = (int*)(it + cap);
    const size_t Cn = (size_t)std::max(C, 1);
    w->items = it;
    w->cap = cap;
    w->cbeg = p;
    w->cend = p + Cn;
    w->order = p + 2 * Cn;
    w->start = p + 3 * Cn;
    w->n_items = p + 4 * Cn;
    w->counters = p + 4 * Cn + 1;
    return NBODY_OK;
}

static int batch_plan(nbody_ctx* c, hipStream_t st, int32_t C, const int64_t* offsets, int64_t n_total,
                      const nbody_tile& t, BatchWS& w) {
    PlanArgs p{};
    p.n_clusters = C;
    p.offsets = offsets;
    p.n_total = (int)n_total;
    p.per = t.wg * t.ipt;
    p.cap = w.cap;
    p.cbeg = w.cbeg;
    p.cend = w.cend;
    p.order = w.order;
    p.start = w.start;
    p.n_items = w.n_items;
    p.items = w.items;
    hipError_t e = launch_batch_plan(p, st);
    if (e != hipSuccess) return hip_err(c, e, "batch plan launch");
    return NBODY_OK;
}

static int batch_force(nbody_ctx* c, hipStream_t st, int prec, double G, const nbody_tile& t, int64_t n_total,
                       const double* eps, const BatchWS& w, int* counter, double* const out[7]) {
    ForceArgs a{};
    a.ipack = (const float4*)c->jpack.p;
    a.iidx = nullptr;
    a.ni = (int)n_total;
    a.jpack = (const float4*)c->jpack.p;
    a.nj = (int)n_total;
    a.jchunk = (int)n_total;
    a.eps2 = 0.f;
    a.partial = 0;
    a.G = G;
    a.iself = nullptr;
    a.self_mode = 2;
    for (int q = 0; q < 7; ++q) a.out[q] = out[q];
    BatchArgs b{};
    b.items = w.items;
    b.n_items = w.n_items;
    b.counter = counter;
    b.cbeg = w.cbeg;
    b.cend = w.cend;
    b.eps = eps;
    const int per = t.wg * t.ipt;
    const int64_t bound = n_total / per + 1 + (int64_t)(w.cap - n_total / 64 - 1);   // <= items
    const int resident = 1024 * (256 / t.wg);
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(bound, resident));
    hipError_t e = launch_fill_i32(counter, 1, 0, st);
    if (e == hipSuccess) e = launch_force_batched(prec, t.ipt, t.tile_j, t.wg, grid, a, b, st);
    if (e != hipSuccess) return hip_err(c, e, "batched force launch");
    return NBODY_OK;
}

static int check_batched(nbody_ctx* c, nbody_prec prec, double G, int32_t C, const int64_t* offsets,
                         const double* eps, int64_t n_total) {
    if (prec != NBODY_PREC_FP32 && prec != NBODY_PREC_DS_COMP)
        return set_err(c, NBODY_ERR_ARG, "unknown precision %d", (int)prec);
    if (!isfinite(G)) return set_err(c, NBODY_ERR_ARG, "G must be finite");
    if (C < 0 || C > (1 << 20)) return set_err(c, NBODY_ERR_ARG, "n_clusters must be in [0, 2^20]");
    if (n_total < 0 || n_total > kMaxN) return set_err(c, NBODY_ERR_ARG, "n_total must be in [0, 2^31-1]");
    if (C > 0 && (!offsets || !eps)) return set_err(c, NBODY_ERR_ARG, "offsets and eps must not be NULL");
    if (!aligned8(offsets) || !aligned8(eps)) return set_err(c, NBODY_ERR_ARG, "offsets/eps not 8-byte aligned");
    return NBODY_OK;
}

int nbody_force_batched(nbody_ctx* c, hipStream_t st, nbody_prec prec, double G, int32_t n_clusters,
                        const int64_t* offsets, const double* eps, int64_t n_total, nbody_src P, nbody_out out) {
    if (!c) return NBODY_ERR_ARG;
    if (int rc = check_batched(c, prec, G, n_clusters, offsets, eps, n_total)) return rc;
    if (n_total > 0) {
        if (int rc = check_src(c, P, true, "P")) return rc;
        if (int rc = check_out(c, out)) return rc;
    }
    if (int rc = need_device(c)) return rc;
    if (n_total == 0) return NBODY_OK;
    DeviceGuard g(c->device);
    const int p = (int)prec;
    const nbody_tile t = batched_tile(c, p, n_total, n_clusters);
    BatchWS w;
    int rc = batch_ws(c, n_clusters, n_total, 1, &w);
    if (!rc) rc = dev_alloc(c, c->jpack, sizeof(float4) * rec_words(p) * (size_t)n_total);
    if (rc) return rc;
    // zero output for particles outside every cluster
    double* o[7] = {out.ax, out.ay, out.az, out.jx, out.jy, out.jz, out.pot};
    for (int q = 0; q < 7; ++q) {
        hipError_t e = launch_fill_f64((int)n_total, o[q], 0.0, st);
        if (e != hipSuccess) return hip_err(c, e, "output clear");
    }
    rc = pack_rows(c, st, p, n_total, P, true, c->jpack);
    if (!rc) rc = batch_plan(c, st, n_clusters, offsets, n_total, t, w);
    if (!rc && n_clusters > 0) rc = batch_force(c, st, p, G, t, n_total, eps, w, w.counters, o);
    return rc;
}

// the step sequence of nbody_batch_hermite (kernels only: capturable)
static int batch_hermite_enqueue(nbody_ctx* c, hipStream_t st, int p, double G, int32_t C, const int64_t* offsets,
                                 const double* eps, int64_t n, double dt, int nsteps, double* x, double* v,
                                 double* a3, double* j3, const double* m, const nbody_tile& t, BatchWS& w) {
    const size_t n3 = 3 * (size_t)n;
    double* xp = (double*)c->bstate.p;
    double* vp = xp + n3;
    double* f = vp + n3;
    double* o[7] = {f, f + n, f + 2 * n, f + 3 * n, f + 4 * n, f + 5 * n, f + 6 * n};
    int rc = batch_plan(c, st, C, offsets, n, t, w);
    if (rc) return rc;
    for (int s = 0; s < nsteps; ++s) {
        hipError_t e = launch_shared_predict((int)n, dt, x, v, a3, j3, xp, vp, st);
        if (e != hipSuccess) return hip_err(c, e, "predict launch");
        PackArgs pa{};
        pa.n = (int)n;
        pa.prec = p;
        pa.x = xp; pa.y = xp + n; pa.z = xp + 2 * n;
        pa.vx = vp; pa.vy = vp + n; pa.vz = vp + 2 * n;
        pa.m = m;
        pa.out = (float4*)c->jpack.p;
        e = launch_pack(pa, st);
        if (e != hipSuccess) return hip_err(c, e, "pack launch");
        rc = batch_force(c, st, p, G, t, n, eps, w, w.counters + s, o);
        if (rc) return rc;
        e = launch_shared_correct((int)n, dt, xp, vp, x, v, a3, j3, f, f + 3 * n, st);
        if (e != hipSuccess) return hip_err(c, e, "corrector launch");
    }
    return NBODY_OK;
}

int nbody_batch_hermite(nbody_ctx* c, hipStream_t st, nbody_prec prec, double G, int32_t n_clusters,
                        const int64_t* offsets, const double* eps, int64_t n_total, double dt, int nsteps, double* x,
                        double* v, double* a3, double* j3, const double* m, int use_graph) {
    if (!c) return NBODY_ERR_ARG;
    if (int rc = check_batched(c, prec, G, n_clusters, offsets, eps, n_total)) return rc;
    if (!(dt > 0.0) || !isfinite(dt)) return set_err(c, NBODY_ERR_ARG, "dt must be positive and finite");
    if (nsteps < 0 || nsteps > 1000000) return set_err(c, NBODY_ERR_ARG, "nsteps must be in [0, 10^6]");
    if (use_graph != 0 && use_graph != 1) return set_err(c, NBODY_ERR_ARG, "use_graph must be 0 or 1");
    const void* ptrs[5] = {x, v, a3, j3, m};
    for (const void* q : ptrs)
        if (n_total > 0 && (!q || !aligned8(q))) return set_err(c, NBODY_ERR_ARG, "state rows must be aligned, non-NULL");
    if (int rc = need_device(c)) return rc;
    if (n_total == 0 || nsteps == 0 || n_clusters == 0) return NBODY_OK;
    DeviceGuard g(c->device);
    const int p = (int)prec;
    const nbody_tile t = batched_tile(c, p, n_total, n_clusters);
    BatchWS w;
    int rc = batch_ws(c, n_clusters, n_total, nsteps, &w);
    if (!rc) rc = dev_alloc(c, c->jpack, sizeof(float4) * rec_words(p) * (size_t)n_total);
    if (!rc) rc = dev_alloc(c, c->bstate, sizeof(double) * 13 * (size_t)n_total);
    if (rc) return rc;
    if (!use_graph)
        return batch_hermite_enqueue(c, st, p, G, n_clusters, offsets, eps, n_total, dt, nsteps, x, v, a3, j3, m, t, w);
    // graph: capture once per argument signature, replay afterwards
    uint64_t dtb;
    memcpy(&dtb, &dt, sizeof dtb);
    uint64_t Gb;
    memcpy(&Gb, &G, sizeof Gb);
    std::vector<uint64_t> key = {(uint64_t)p, Gb, (uint64_t)n_clusters, (uintptr_t)offsets, (uintptr_t)eps,
                                 (uint64_t)n_total, dtb, (uint64_t)nsteps, (uintptr_t)x, (uintptr_t)v,
                                 (uintptr_t)a3, (uintptr_t)j3, (uintptr_t)m, (uint64_t)t.tile_j,
                                 (uint64_t)t.ipt, (uint64_t)t.wg, (uintptr_t)c->jpack.p, (uintptr_t)c->bplan.p,
                                 (uintptr_t)c->bstate.p};
    hipError_t e = hipSuccess;
    if (!c->gstream) {
        e = hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->gev[0], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->gev[1], hipEventDisableTiming);
        if (e != hipSuccess) return hip_err(c, e, "graph stream setup");
    }
    if (!c->gexec || c->gkey != key) {
        if (c->gexec) {
            (void)hipGraphExecDestroy(c->gexec);
            c->gexec = nullptr;
        }
        if (c->graph) {
            (void)hipGraphDestroy(c->graph);
            c->graph = nullptr;
        }
        e = hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_err(c, e, "begin capture");
        rc = batch_hermite_enqueue(c, c->gstream, p, G, n_clusters, offsets, eps, n_total, dt, nsteps, x, v, a3, j3,
                                   m, t, w);
        hipGraph_t gr = nullptr;
        hipError_t e2 = hipStreamEndCapture(c->gstream, &gr);
        if (rc) {
            if (gr) (void)hipGraphDestroy(gr);
            return rc;
        }
        if (e2 != hipSuccess) return hip_err(c, e2, "end capture");
        e = hipGraphInstantiate(&c->gexec, gr, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(gr);
            return hip_err(c, e, "graph instantiate");
        }
        c->graph = gr;
        c->gkey = key;
    }
    e = hipEventRecord(c->gev[0], st);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->gstream, c->gev[0], 0);
    if (e == hipSuccess) e = hipGraphLaunch(c->gexec, c->gstream);
    if (e == hipSuccess) e = hipEventRecord(c->gev[1], c->gstream);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, c->gev[1], 0);
    if (e != hipSuccess) return hip_err(c, e, "graph launch");
    return NBODY_OK;
}

int nbody_autotune_batched(nbody_ctx* c, hipStream_t st, nbody_prec prec, double G, int32_t n_clusters,
                           const int64_t* offsets, const double* eps, int64_t n_total, nbody_src P, nbody_out out,
                           int reps, nbody_tile* best, double* best_ms) {
    if (!c) return NBODY_ERR_ARG;
    if (reps < 1 || reps > 100) return set_err(c, NBODY_ERR_ARG, "reps must be in [1, 100]");
    if (n_total <= 0 || n_clusters <= 0) return set_err(c, NBODY_ERR_ARG, "need clusters and particles");
    if (int rc = check_batched(c, prec, G, n_clusters, offsets, eps, n_total)) return rc;
    if (int rc = check_src(c, P, true, "P")) return rc;
    if (int rc = check_out(c, out)) return rc;
    if (int rc = need_device(c)) return rc;
    DeviceGuard g(c->device);
    const int p = (int)prec;
    const bool had = c->have_override[p];
    const nbody_tile saved = c->override_tile[p];
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return set_err(c, NBODY_ERR_DEVICE, "event create");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_err(c, NBODY_ERR_DEVICE, "event create");
    }
    const int tjs[3] = {64, 128, 256}, ipts[3] = {1, 2, 4}, wgs[2] = {128, 256};
    nbody_tile bt{};
    double bms = 1e300;
    int rc = NBODY_OK;
    for (int a = 0; a < 3 && !rc; ++a)
        for (int b = 0; b < 3 && !rc; ++b)
            for (int wi = 0; wi < 2 && !rc; ++wi) {
                nbody_tile t{tjs[a], ipts[b], wgs[wi], 1, 0, 0, 0};
                c->override_tile[p] = t;
                c->have_override[p] = true;
                rc = nbody_force_batched(c, st, prec, G, n_clusters, offsets, eps, n_total, P, out);
                if (rc) break;
                hipError_t e = hipEventRecord(e0, st);
                for (int r = 0; r < reps && e == hipSuccess && !rc; ++r)
                    rc = nbody_force_batched(c, st, prec, G, n_clusters, offsets, eps, n_total, P, out);
                if (rc) break;
                if (e == hipSuccess) e = hipEventRecord(e1, st);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) {
                    rc = hip_err(c, e, "autotune timing");
                    break;
                }
                if (ms / reps < bms) {
                    bms = ms / reps;
                    bt = t;
                }
            }
    c->have_override[p] = had;
    c->override_tile[p] = saved;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    c->tune.store(p + 2, n_total, n_clusters, bt, bms);
    if (!c->tune.save()) return set_err(c, NBODY_ERR_ARG, "cannot write tune cache %s", c->tune.path().c_str());
    if (best) *best = bt;
    if (best_ms) *best_ms = bms;
    return NBODY_OK;
}

int nbody_autotune(nbody_ctx* c, hipStream_t st, nbody_prec prec, double G, double eps, int64_t n_i,
                   nbody_src I, int64_t n_j, nbody_src J, nbody_out out, int reps, nbody_tile* best,
                   double* best_ms) {
    if (!c) return NBODY_ERR_ARG;
    if (int rc = check_common(c, prec, G, eps)) return rc;
    if (n_i <= 0 || n_j <= 0 || n_i > kMaxN || n_j > kMaxN)
        return set_err(c, NBODY_ERR_ARG, "autotune needs 1 <= n_i, n_j <= 2^31-1");
    if (reps < 1 || reps > 100) return set_err(c, NBODY_ERR_ARG, "reps must be in [1, 100]");
    if (int rc = check_src(c, I, false, "I")) return rc;
    if (int rc = check_src(c, J, true, "J")) return rc;
    if (int rc = check_out(c, out)) return rc;
    if (int rc = need_device(c)) return rc;
    DeviceGuard g(c->device);
    const int p = (int)prec;
    int rc = pack_rows(c, st, p, n_j, J, true, c->jpack);
    if (rc) return rc;
    const float4* ip = (const float4*)c->jpack.p;
    if (!(n_i == n_j && same_src(I, J))) {
        rc = pack_rows(c, st, p, n_i, I, false, c->ipack);
        if (rc) return rc;
        ip = (const float4*)c->ipack.p;
    }
    double* o[7] = {out.ax, out.ay, out.az, out.jx, out.jy, out.jz, out.pot};
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return set_err(c, NBODY_ERR_DEVICE, "event create");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_err(c, NBODY_ERR_DEVICE, "event create");
    }
    std::vector<nbody_tile> cand;
    for (int k = 0; k < force_variant_count(); ++k) {
        int vp, vi, vt, vw, vj, vu, vo, vk;
        bool ve;
        if (force_variant_at(k, &vp, &vi, &vt, &vw, &vj, &vu, &vo, &ve, &vk) && vk == 0 && vp == p &&
            ve == (eps == 0.0))
            cand.push_back(nbody_tile{vt, vi, vw, 0, vj, vu, vo});
    }
    nbody_tile bt{};
    double bms = 1e300;
    for (size_t ci = 0; ci < cand.size() && !rc; ++ci) {
            {
                nbody_tile t = cand[ci];

                t.split = choose_split(n_i, n_j, t);
                rc = run_force(c, st, p, G, eps, n_i, ip, nullptr, nullptr, 0, n_j, (const float4*)c->jpack.p, o, &t);
                if (rc) break;
                hipError_t e = hipEventRecord(e0, st);
                for (int r = 0; r < reps && e == hipSuccess && !rc; ++r)
                    rc = run_force(c, st, p, G, eps, n_i, ip, nullptr, nullptr, 0, n_j, (const float4*)c->jpack.p, o, &t);
                if (rc) break;
                if (e == hipSuccess) e = hipEventRecord(e1, st);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) {
                    rc = hip_err(c, e, "autotune timing");
                    break;
                }
                const double per = (double)ms / reps;
                if (per < bms) {
                    bms = per;
                    bt = t;
                }
            }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    c->tune.store(p, n_i, n_j, bt, bms);
    if (!c->tune.save()) return set_err(c, NBODY_ERR_ARG, "cannot write tune cache %s", c->tune.path().c_str());
    if (best) *best = bt;
    if (best_ms) *best_ms = bms;
    return NBODY_OK;
}

// Host copy of the step-level rule the corrector kernel applies (for
// host-side checks of the integer rule; no device work).
int64_t nbody_block_level(double crit, int64_t dt_old, int64_t t_new, int lmin, int lmax) {
    if (lmin < -20 || lmax > 0 || lmin > lmax) return -1;
    return block_level(crit, dt_old, t_new, lmin, lmax);
}

}  // extern "C"

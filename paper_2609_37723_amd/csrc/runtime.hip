// Host runtime of the nucleon-correlator library: the C ABI of include/nucleon.h,
// argument checks, host-side FP64 profile evaluation, the context's HBM
// workspace and the kernel launch sequence.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/nucleon.h"
#include "nuc_internal.h"

#define NUC_VERSION "nucleon-mi355x 0.1 (gfx950)"

using namespace nuc;

struct nuc_ctx_s {
    int device = 0;
    size_t budget = 0;
    void* ws = nullptr;
    size_t ws_size = 0;
    hipEvent_t done = nullptr;      // recorded at the end of every call
    bool have_done = false;
    void* staging = nullptr;        // pinned host staging for small constants
    size_t staging_size = 0;
    hipEvent_t staged = nullptr;    // recorded after the last staging copy
    bool have_staged = false;
    std::string err;
    std::mutex mu;
    // per-kernel timing
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    struct Timed { int id; hipEvent_t a, b; };
    std::vector<Timed> timed;
};

namespace {

thread_local std::string g_thread_err;

nuc_status fail(nuc_ctx ctx, nuc_status s, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
nuc_status fail(nuc_ctx ctx, nuc_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_thread_err = buf;
    if (ctx) ctx->err = buf;
    return s;
}

nuc_status hip_fail(nuc_ctx ctx, hipError_t e, const char* what) {
    return fail(ctx, NUC_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(ctx, expr)                                              \
    do {                                                               \
        hipError_t e_ = (expr);                                        \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, #expr);       \
    } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

hipEvent_t pool_get(nuc_ctx ctx) {
    if (!ctx->ev_pool.empty()) {
        hipEvent_t e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

// Launch `fn` on stream s; with timing on, bracket it with events on s.
template <class F>
hipError_t timed_launch(nuc_ctx ctx, int id, hipStream_t s, F&& fn) {
    if (!ctx->timing) return fn();
    hipEvent_t a = pool_get(ctx), b = pool_get(ctx);
    if (!a || !b) return fn();
    hipError_t e = hipEventRecord(a, s);
    if (e != hipSuccess) return e;
    e = fn();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, s);
    if (e != hipSuccess) return e;
    ctx->timed.push_back({id, a, b});
    return hipSuccess;
}

long long choose3(long long n) { return n * (n - 1) * (n - 2) / 6; }

int pad16(int n) { return (n + 15) / 16 * 16; }

// ------------------------------------------------------------- argument checks

nuc_status check_geom(nuc_ctx ctx, const nuc_geom* g) {
    if (!g) return fail(ctx, NUC_ERR_INVALID, "geom is NULL");
    if (g->L < 1 || g->L > 256) return fail(ctx, NUC_ERR_INVALID, "L=%d out of range [1,256]", g->L);
    if (g->T < 1) return fail(ctx, NUC_ERR_INVALID, "T=%d must be >= 1", g->T);
    if (g->nvec < 3 || g->nvec > kMaxNvec)
        return fail(ctx, NUC_ERR_INVALID, "nvec=%d out of range [3,%d]", g->nvec, kMaxNvec);
    if (g->t0 < 0 || g->t0 >= g->T) return fail(ctx, NUC_ERR_INVALID, "t0=%d outside [0,T)", g->t0);
    return NUC_OK;
}

nuc_status check_moms(nuc_ctx ctx, const nuc_geom* g, int nmom, const int32_t* mom) {
    if (nmom < 1 || nmom > 64) return fail(ctx, NUC_ERR_INVALID, "nmom=%d out of range [1,64]", nmom);
    if (!mom) return fail(ctx, NUC_ERR_INVALID, "mom is NULL");
    for (int p = 0; p < nmom; ++p)
        for (int d = 0; d < 3; ++d)
            if (mom[3 * p + d] <= -g->L || mom[3 * p + d] >= g->L)
                return fail(ctx, NUC_ERR_INVALID, "momentum %d component %d = %d needs |n| < L=%d", p, d,
                            mom[3 * p + d], g->L);
    return NUC_OK;
}

nuc_status check_profiles(nuc_ctx ctx, const nuc_geom* g, const double* evals, int nprof,
                          const nuc_profile* prof) {
    if (nprof < 1 || nprof > kMaxProf)
        return fail(ctx, NUC_ERR_INVALID, "nprof=%d out of range [1,%d]", nprof, kMaxProf);
    if (!prof) return fail(ctx, NUC_ERR_INVALID, "prof is NULL");
    for (int a = 0; a < nprof; ++a) {
        switch (prof[a].kind) {
            case NUC_PROF_GAUSS:
                if (!(prof[a].sigma > 0.0) || !isfinite(prof[a].sigma))
                    return fail(ctx, NUC_ERR_INVALID, "profile %d: sigma=%g must be finite and > 0", a,
                                prof[a].sigma);
                if (!evals) return fail(ctx, NUC_ERR_INVALID, "profile %d is Gaussian but evals is NULL", a);
                break;
            case NUC_PROF_LINEAR:
            case NUC_PROF_ONE:
                break;
            case NUC_PROF_EXPLICIT:
                if (!prof[a].values) return fail(ctx, NUC_ERR_INVALID, "profile %d: values is NULL", a);
                break;
            default:
                return fail(ctx, NUC_ERR_INVALID, "profile %d: unknown kind %d", a, prof[a].kind);
        }
    }
    return NUC_OK;
}

nuc_status check_prec(nuc_ctx ctx, nuc_precision p) {
    if (p == NUC_FP32 || p == NUC_BF16X3) return NUC_OK;
    return fail(ctx, NUC_ERR_INVALID, "unknown precision %d", (int)p);
}

// BF16x3 is implemented for the perambulator chain at nvec <= 32.
nuc_status check_prec_shape(nuc_ctx ctx, nuc_precision p, const nuc_geom* g) {
    if (p == NUC_BF16X3 && pad16(g->nvec) > 32)
        return fail(ctx, NUC_ERR_UNSUPPORTED, "BF16x3 contraction is implemented for nvec <= 32 (got %d)",
                    g->nvec);
    return NUC_OK;
}

// Section 2.1 profile functions, evaluated in FP64 on the host.
void eval_profiles(const nuc_geom* g, const double* evals, int nprof, const nuc_profile* prof,
                   double* out) {
    const int T = g->T, N = g->nvec;
    for (int a = 0; a < nprof; ++a)
        for (int t = 0; t < T; ++t)
            for (int i = 0; i < N; ++i) {
                double v = 1.0;
                const double sig = prof[a].sigma;
                switch (prof[a].kind) {
                    case NUC_PROF_GAUSS: {
                        const double lam = evals[(size_t)t * N + i];
                        v = exp(-(lam * lam) / (2.0 * sig * sig));
                        break;
                    }
                    case NUC_PROF_LINEAR: v = 1.0 - (double)i / (double)N; break;
                    case NUC_PROF_ONE: v = 1.0; break;
                    case NUC_PROF_EXPLICIT: v = prof[a].values[(size_t)t * N + i]; break;
                }
                out[((size_t)a * T + t) * N + i] = v;
            }
}

SpinFold make_fold() { return kFold; }

// ------------------------------------------------------------------ planning

struct ElemPlan {
    int N, npairs, nwork, nsplit, C3, Tc;
    std::vector<int2> pairs, work;
    size_t part_bytes, packed_bytes;
    size_t scratch() const { return align_up(part_bytes, 256) + packed_bytes; }
};

ElemPlan plan_elementals(const nuc_geom* g, int nmom) {
    ElemPlan P;
    const int N = g->nvec;
    P.N = N;
    for (int j = 0; j < N; ++j)
        for (int k = j + 1; k < N; ++k) P.pairs.push_back(make_int2(j, k));
    P.npairs = (int)P.pairs.size();
    P.C3 = (int)choose3(N);
    const int nit = (N + 15) / 16, npb = (P.npairs + 63) / 64;
    for (int it = 0; it < nit; ++it)
        for (int pb = 0; pb < npb; ++pb) {
            bool any = false;
            for (int wv = 0; wv < 4; ++wv) {
                const int q0 = pb * 64 + wv * 16;
                if (q0 >= P.npairs) break;
                const int ql = std::min(q0 + 15, P.npairs - 1);
                if (it * 16 < P.pairs[ql].x) any = true;
            }
            if (any) P.work.push_back(make_int2(it, pb));
        }
    P.nwork = (int)P.work.size();
    const int V3 = g->L * g->L * g->L;
    // Each workgroup sums about 256 sites in FP32; the site ranges are combined in
    // FP64. The FP64 partials of one launch stay under 1 GiB (timeslice chunks,
    // then longer site ranges if one timeslice alone would exceed it).
    const size_t per_ts = (size_t)nmom * P.C3 * sizeof(double2);  // one t, one split
    const size_t cap = (size_t)1 << 30;
    int ns = std::max(1, (V3 + 255) / 256);
    ns = std::min<int>(ns, (int)std::max<size_t>(1, cap / per_ts));
    P.nsplit = ns;
    P.Tc = (int)std::max<size_t>(1, std::min<size_t>((size_t)g->T, cap / (per_ts * ns)));
    P.part_bytes = per_ts * ns * P.Tc;
    P.packed_bytes = (size_t)P.Tc * nmom * P.C3 * sizeof(float2);
    return P;
}

struct CorrPlan {
    int Np, Tc;
    size_t x_bytes, part_bytes;
};

CorrPlan plan_correlator(const nuc_geom* g, int nmom, int nprof, size_t cap) {
    CorrPlan P;
    const int N = g->nvec;
    P.Np = pad16(N);
    const size_t per_t_x = (size_t)nmom * nprof * 2 * 4 * (size_t)P.Np * P.Np * P.Np * sizeof(float2);
    const size_t per_t_p = (size_t)nmom * nprof * 2 * N * nprof * sizeof(double2);
    P.Tc = (int)std::max<size_t>(1, std::min<size_t>((size_t)g->T, cap / (per_t_x + per_t_p)));
    P.x_bytes = per_t_x * P.Tc;
    P.part_bytes = per_t_p * P.Tc;
    return P;
}

const size_t kCorrCap = (size_t)4 << 30;

struct Layout {
    size_t consts = 0, phi = 0, scratch = 0, total = 0;
};

// Byte counts of the small constant block copied to the device for a call.
struct Consts {
    std::vector<char> host;
    size_t off_mom = 0, off_pairs = 0, off_work = 0, off_gsnk = 0, off_gsrc = 0;
};

void consts_add(Consts& c, size_t& off, const void* src, size_t n) {
    off = align_up(c.host.size(), 256);
    c.host.resize(off + n);
    if (n) memcpy(c.host.data() + off, src, n);
}

nuc_status ensure_workspace(nuc_ctx ctx, size_t bytes, hipStream_t s) {
    if (ctx->budget && bytes > ctx->budget)
        return fail(ctx, NUC_ERR_NOMEM, "workspace of %zu bytes exceeds the HBM budget of %zu bytes", bytes,
                    ctx->budget);
    if (bytes <= ctx->ws_size) return NUC_OK;
    if (ctx->ws) {
        HIPCHK(ctx, hipStreamSynchronize(s));
        if (ctx->have_done) HIPCHK(ctx, hipEventSynchronize(ctx->done));
        HIPCHK(ctx, hipFree(ctx->ws));
        ctx->ws = nullptr;
        ctx->ws_size = 0;
    }
    const size_t want = align_up(bytes, (size_t)1 << 20);
    hipError_t e = hipMalloc(&ctx->ws, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        ctx->ws = nullptr;
        return fail(ctx, NUC_ERR_NOMEM, "hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
    }
    ctx->ws_size = want;
    return NUC_OK;
}

nuc_status upload_consts(nuc_ctx ctx, const Consts& c, void* dst, hipStream_t s) {
    const size_t n = c.host.size();
    if (n == 0) return NUC_OK;
    if (ctx->have_staged) HIPCHK(ctx, hipEventSynchronize(ctx->staged));
    if (n > ctx->staging_size) {
        if (ctx->staging) HIPCHK(ctx, hipHostFree(ctx->staging));
        ctx->staging = nullptr;
        ctx->staging_size = 0;
        const size_t want = align_up(n, 65536);
        HIPCHK(ctx, hipHostMalloc(&ctx->staging, want, hipHostMallocDefault));
        ctx->staging_size = want;
    }
    memcpy(ctx->staging, c.host.data(), n);
    HIPCHK(ctx, hipMemcpyAsync(dst, ctx->staging, n, hipMemcpyHostToDevice, s));
    HIPCHK(ctx, hipEventRecord(ctx->staged, s));
    ctx->have_staged = true;
    return NUC_OK;
}

// Order this call after the previous call of the context (which may have used
// another stream) so the shared workspace is never used by two calls at once.
nuc_status begin_call(nuc_ctx ctx, hipStream_t s) {
    HIPCHK(ctx, hipSetDevice(ctx->device));
    if (ctx->have_done) HIPCHK(ctx, hipStreamWaitEvent(s, ctx->done, 0));
    return NUC_OK;
}

nuc_status end_call(nuc_ctx ctx, hipStream_t s) {
    HIPCHK(ctx, hipEventRecord(ctx->done, s));
    ctx->have_done = true;
    return NUC_OK;
}

struct DeviceGuard {
    int prev = -1;
    DeviceGuard() { (void)hipGetDevice(&prev); }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// Enqueue the elementals of every timeslice into phi (dense c64).
nuc_status run_elementals(nuc_ctx ctx, const nuc_geom* g, const void* evecs, int nmom, const ElemPlan& P,
                          const int* d_mom, const int2* d_pairs, const int2* d_work, void* scratch,
                          void* phi, hipStream_t s) {
    ElemLaunch a;
    a.evecs = (const float2*)evecs;
    a.mom = d_mom;
    a.pairs = d_pairs;
    a.work = d_work;
    a.part = (double2*)scratch;
    a.packed = (float2*)((char*)scratch + align_up(P.part_bytes, 256));
    a.phi = (float2*)phi;
    a.T = g->T;
    a.N = g->nvec;
    a.L = g->L;
    a.V3 = g->L * g->L * g->L;
    a.nmom = nmom;
    a.npairs = P.npairs;
    a.nwork = P.nwork;
    a.nsplit = P.nsplit;
    a.C3 = P.C3;
    a.precision = 0;
    for (int t0 = 0; t0 < g->T; t0 += P.Tc) {
        a.t_off = t0;
        a.Tc = std::min(P.Tc, g->T - t0);
        HIPCHK(ctx, timed_launch(ctx, NUC_K_ELEMENTALS, s, [&] { return launch_elementals(a, s); }));
        HIPCHK(ctx, timed_launch(ctx, NUC_K_ELEM_EXPAND, s, [&] { return launch_elem_expand(a, s); }));
    }
    return NUC_OK;
}

nuc_status run_correlator(nuc_ctx ctx, const nuc_geom* g, const void* phi, int nmom, int nprof,
                          const CorrPlan& P, const double* d_gsnk, const double* d_gsrc, const void* peramb,
                          void* scratch, void* corr, nuc_precision prec, hipStream_t s) {
    CorrLaunch a;
    a.phi = (const float2*)phi;
    a.tau = (const float2*)peramb;
    a.gsnk = d_gsnk;
    a.gsrc = d_gsrc;
    a.X = (float2*)scratch;
    a.part = (double2*)((char*)scratch + align_up(P.x_bytes, 256));
    a.corr = (double2*)corr;
    a.fold = make_fold();
    a.T = g->T;
    a.N = g->nvec;
    a.Np = P.Np;
    a.nmom = nmom;
    a.nprof = nprof;
    a.t0 = g->t0;
    a.precision = prec == NUC_BF16X3 ? 1 : 0;
    for (int t0 = 0; t0 < g->T; t0 += P.Tc) {
        a.t_off = t0;
        a.Tc = std::min(P.Tc, g->T - t0);
        HIPCHK(ctx, timed_launch(ctx, NUC_K_CORR_STEP1, s, [&] { return launch_corr_step1(a, s); }));
        HIPCHK(ctx, timed_launch(ctx, NUC_K_CORR_CHAIN, s, [&] { return launch_corr_chain(a, s); }));
        HIPCHK(ctx, timed_launch(ctx, NUC_K_CORR_REDUCE, s, [&] { return launch_corr_reduce(a, s); }));
    }
    return NUC_OK;
}

}  // namespace

// ======================================================================== ABI

extern "C" {

const char* nuc_version(void) { return NUC_VERSION; }

const char* nuc_status_string(nuc_status s) {
    switch (s) {
        case NUC_OK: return "ok";
        case NUC_ERR_INVALID: return "invalid argument";
        case NUC_ERR_NOMEM: return "out of workspace memory";
        case NUC_ERR_DEVICE: return "device error";
        case NUC_ERR_UNSUPPORTED: return "unsupported";
        case NUC_ERR_BUSY: return "busy";
        case NUC_ERR_INTERNAL: return "internal error";
    }
    return "unknown status";
}

const char* nuc_last_error(nuc_ctx ctx) { return ctx ? ctx->err.c_str() : g_thread_err.c_str(); }

nuc_status nuc_create(nuc_ctx* out, int device, size_t hbm_budget_bytes) {
    if (!out) return fail(nullptr, NUC_ERR_INVALID, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        return fail(nullptr, NUC_ERR_DEVICE, "no HIP device available");
    }
    if (device < 0 || device >= ndev)
        return fail(nullptr, NUC_ERR_INVALID, "device %d outside [0,%d)", device, ndev);
    DeviceGuard guard;
    nuc_ctx c = new nuc_ctx_s();
    c->device = device;
    c->budget = hbm_budget_bytes;
    if ((e = hipSetDevice(device)) != hipSuccess || (e = hipEventCreateWithFlags(&c->done, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->staged, hipEventDisableTiming)) != hipSuccess) {
        nuc_status st = hip_fail(nullptr, e, "context setup");
        delete c;
        return st;
    }
    *out = c;
    return NUC_OK;
}

nuc_status nuc_destroy(nuc_ctx ctx) {
    if (!ctx) return NUC_OK;
    DeviceGuard guard;
    (void)hipSetDevice(ctx->device);
    if (ctx->have_done) (void)hipEventSynchronize(ctx->done);
    if (ctx->have_staged) (void)hipEventSynchronize(ctx->staged);
    for (auto& t : ctx->timed) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->staging) (void)hipHostFree(ctx->staging);
    if (ctx->done) (void)hipEventDestroy(ctx->done);
    if (ctx->staged) (void)hipEventDestroy(ctx->staged);
    delete ctx;
    return NUC_OK;
}

const char* nuc_kernel_name(int id) {
    static const char* names[NUC_K_COUNT] = {"elementals", "elem_expand", "corr_step1", "corr_chain",
                                             "corr_reduce"};
    return (id >= 0 && id < NUC_K_COUNT) ? names[id] : "?";
}

nuc_status nuc_timing_enable(nuc_ctx ctx, int on) {
    if (!ctx) return fail(nullptr, NUC_ERR_INVALID, "ctx is NULL");
    std::lock_guard<std::mutex> lock(ctx->mu);
    DeviceGuard guard;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    for (auto& t : ctx->timed) {
        HIPCHK(ctx, hipEventSynchronize(t.b));
        ctx->ev_pool.push_back(t.a);
        ctx->ev_pool.push_back(t.b);
    }
    ctx->timed.clear();
    ctx->timing = on != 0;
    return NUC_OK;
}

nuc_status nuc_timing_read(nuc_ctx ctx, double* ms, int* launches) {
    if (!ctx) return fail(nullptr, NUC_ERR_INVALID, "ctx is NULL");
    if (!ms || !launches) return fail(ctx, NUC_ERR_INVALID, "ms or launches is NULL");
    std::lock_guard<std::mutex> lock(ctx->mu);
    DeviceGuard guard;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    for (int k = 0; k < NUC_K_COUNT; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    for (auto& t : ctx->timed) {
        HIPCHK(ctx, hipEventSynchronize(t.b));
        float e = 0.f;
        HIPCHK(ctx, hipEventElapsedTime(&e, t.a, t.b));
        ms[t.id] += e;
        launches[t.id] += 1;
        ctx->ev_pool.push_back(t.a);
        ctx->ev_pool.push_back(t.b);
    }
    ctx->timed.clear();
    return NUC_OK;
}

nuc_status nuc_profiles_eval(const nuc_geom* geom, const double* evals, int nprof, const nuc_profile* prof,
                             double* g_out) {
    nuc_status st;
    if ((st = check_geom(nullptr, geom)) != NUC_OK) return st;
    if ((st = check_profiles(nullptr, geom, evals, nprof, prof)) != NUC_OK) return st;
    if (!g_out) return fail(nullptr, NUC_ERR_INVALID, "g_out is NULL");
    eval_profiles(geom, evals, nprof, prof, g_out);
    return NUC_OK;
}

static size_t consts_bytes_upper(const nuc_geom* g, int nmom, int nprof) {
    const size_t N = g->nvec;
    return 5 * 256 + nmom * 3 * sizeof(int) + N * N / 2 * sizeof(int2) + 4096 * sizeof(int2) +
           (size_t)nprof * g->T * N * sizeof(double) + (size_t)nprof * N * sizeof(double);
}

nuc_status nuc_workspace_query(const nuc_geom* geom, int nmom, int nprof, nuc_precision prec, size_t* bytes) {
    nuc_status st;
    if ((st = check_geom(nullptr, geom)) != NUC_OK) return st;
    if (nmom < 1 || nmom > 64) return fail(nullptr, NUC_ERR_INVALID, "nmom=%d out of range [1,64]", nmom);
    if (nprof < 1 || nprof > kMaxProf) return fail(nullptr, NUC_ERR_INVALID, "nprof=%d out of range", nprof);
    if ((st = check_prec(nullptr, prec)) != NUC_OK) return st;
    if (!bytes) return fail(nullptr, NUC_ERR_INVALID, "bytes is NULL");
    ElemPlan E = plan_elementals(geom, nmom);
    CorrPlan C = plan_correlator(geom, nmom, nprof, kCorrCap);
    *bytes = align_up(consts_bytes_upper(geom, nmom, nprof), 256) +
             std::max(E.scratch(), align_up(C.x_bytes, 256) + C.part_bytes);
    return NUC_OK;
}

static nuc_status run_impl(nuc_ctx ctx, const nuc_geom* g, const void* evecs, const double* evals, int nprof,
                           const nuc_profile* prof, int nmom, const int32_t* mom, const void* peramb,
                           nuc_precision prec, void* phi, void* corr, void* stream, bool do_elem, bool do_corr) {
    if (!ctx) return fail(nullptr, NUC_ERR_INVALID, "ctx is NULL");
    std::lock_guard<std::mutex> lock(ctx->mu);
    nuc_status st;
    if ((st = check_geom(ctx, g)) != NUC_OK) return st;
    if ((st = check_prec(ctx, prec)) != NUC_OK) return st;
    if (do_corr && (st = check_prec_shape(ctx, prec, g)) != NUC_OK) return st;
    if (nmom < 1 || nmom > 64) return fail(ctx, NUC_ERR_INVALID, "nmom=%d out of range [1,64]", nmom);
    if (do_elem) {
        if (!evecs) return fail(ctx, NUC_ERR_INVALID, "evecs is NULL");
        if ((st = check_moms(ctx, g, nmom, mom)) != NUC_OK) return st;
        if (!do_corr && !phi) return fail(ctx, NUC_ERR_INVALID, "phi is NULL");
    }
    if (do_corr) {
        if (!do_elem && !phi) return fail(ctx, NUC_ERR_INVALID, "phi is NULL");
        if ((st = check_profiles(ctx, g, evals, nprof, prof)) != NUC_OK) return st;
        if (!peramb) return fail(ctx, NUC_ERR_INVALID, "peramb is NULL");
        if (!corr) return fail(ctx, NUC_ERR_INVALID, "corr is NULL");
    }
    DeviceGuard guard;
    hipStream_t s = (hipStream_t)stream;
    if ((st = begin_call(ctx, s)) != NUC_OK) return st;

    const int N = g->nvec;
    Consts c;
    ElemPlan E;
    CorrPlan C;
    std::vector<double> gs, g0;
    if (do_elem) {
        E = plan_elementals(g, nmom);
        consts_add(c, c.off_mom, mom, (size_t)nmom * 3 * sizeof(int));
        consts_add(c, c.off_pairs, E.pairs.data(), E.pairs.size() * sizeof(int2));
        consts_add(c, c.off_work, E.work.data(), E.work.size() * sizeof(int2));
    }
    if (do_corr) {
        C = plan_correlator(g, nmom, nprof, ctx->budget ? std::min(kCorrCap, ctx->budget / 2) : kCorrCap);
        gs.resize((size_t)nprof * g->T * N);
        eval_profiles(g, evals, nprof, prof, gs.data());
        g0.resize((size_t)nprof * N);
        for (int a = 0; a < nprof; ++a)
            memcpy(&g0[(size_t)a * N], &gs[((size_t)a * g->T + g->t0) * N], N * sizeof(double));
        consts_add(c, c.off_gsnk, gs.data(), gs.size() * sizeof(double));
        consts_add(c, c.off_gsrc, g0.data(), g0.size() * sizeof(double));
    }
    const size_t phi_bytes = (size_t)g->T * nmom * N * N * N * sizeof(float2);
    const bool phi_internal = do_elem && do_corr && !phi;
    Layout L;
    L.consts = 0;
    L.phi = align_up(c.host.size(), 256);
    L.scratch = L.phi + (phi_internal ? align_up(phi_bytes, 256) : 0);
    size_t scratch = 0;
    if (do_elem) scratch = std::max(scratch, E.scratch());
    if (do_corr) scratch = std::max(scratch, align_up(C.x_bytes, 256) + C.part_bytes);
    L.total = L.scratch + scratch;
    if ((st = ensure_workspace(ctx, L.total, s)) != NUC_OK) return st;
    char* ws = (char*)ctx->ws;
    if ((st = upload_consts(ctx, c, ws, s)) != NUC_OK) return st;
    void* phi_buf = phi_internal ? (void*)(ws + L.phi) : phi;
    if (do_elem) {
        st = run_elementals(ctx, g, evecs, nmom, E, (const int*)(ws + c.off_mom), (const int2*)(ws + c.off_pairs),
                            (const int2*)(ws + c.off_work), ws + L.scratch, phi_buf, s);
        if (st != NUC_OK) return st;
    }
    if (do_corr) {
        st = run_correlator(ctx, g, phi_buf, nmom, nprof, C, (const double*)(ws + c.off_gsnk),
                            (const double*)(ws + c.off_gsrc), peramb, ws + L.scratch, corr, prec, s);
        if (st != NUC_OK) return st;
    }
    return end_call(ctx, s);
}

nuc_status nuc_elementals(nuc_ctx ctx, const nuc_geom* geom, const void* evecs, int nmom, const int32_t* mom,
                          nuc_precision prec, void* phi, void* stream) {
    return run_impl(ctx, geom, evecs, nullptr, 0, nullptr, nmom, mom, nullptr, prec, phi, nullptr, stream, true,
                    false);
}

nuc_status nuc_correlator(nuc_ctx ctx, const nuc_geom* geom, const void* phi, const double* evals, int nprof,
                          const nuc_profile* prof, int nmom, const void* peramb, nuc_precision prec, void* corr,
                          void* stream) {
    return run_impl(ctx, geom, nullptr, evals, nprof, prof, nmom, nullptr, peramb, prec, (void*)phi, corr, stream,
                    false, true);
}

nuc_status nuc_run(nuc_ctx ctx, const nuc_geom* geom, const void* evecs, const double* evals, int nprof,
                   const nuc_profile* prof, int nmom, const int32_t* mom, const void* peramb, nuc_precision prec,
                   void* phi, void* corr, void* stream) {
    return run_impl(ctx, geom, evecs, evals, nprof, prof, nmom, mom, peramb, prec, phi, corr, stream, true, true);
}

}  // extern "C"

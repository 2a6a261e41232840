// Host-runtime internals shared by the one-shot/batch entry points and the
// serving loop: the context, the job/program model and the planner.
#pragma once

#include <string.h>

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/nucleon.h"
#include "nuc_internal.h"

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
    int graphs_alive = 0;           // captured graphs referencing the workspace
    // launch parameters chosen by nuc_autotune, per job shape
    std::map<std::vector<int>, std::pair<int, int>> tuned;
};

struct nuc_graph_s {
    nuc_ctx ctx = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void* staging = nullptr;        // pinned copy of the constants the graph uploads
};

namespace nuc {
namespace rt {

nuc_status fail(nuc_ctx ctx, nuc_status s, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
nuc_status hip_fail(nuc_ctx ctx, hipError_t e, const char* what);

#define HIPCHK(ctx, expr)                                              \
    do {                                                               \
        hipError_t e_ = (expr);                                        \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, #expr);       \
    } while (0)

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// The value of an enum argument as an int, read byte-wise: a C caller may pass a value
// outside the enum's range, and reading it as the enum type would be undefined.
template <class E>
inline int raw_enum(const E& e) {
    static_assert(sizeof(E) == sizeof(int), "enum arguments are int-sized");
    int v;
    memcpy(&v, &e, sizeof v);
    return v;
}

struct DeviceGuard {
    int prev = -1;
    DeviceGuard() { (void)hipGetDevice(&prev); }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

struct Job {
    nuc_geom g;
    const void* evecs = nullptr;
    const void* peramb = nullptr;
    void* phi = nullptr;
    void* corr = nullptr;
    int nmom = 0, nprof = 0, prec = 0;
    int ld = 0;  // leading nvec dimension of evecs and tau (>= nvec)
    int elem_mp = 0, s1_target = 0;  // tunable launch shapes (0 = defaults)
    bool do_elem = false, do_corr = false;
    std::vector<int32_t> mom;
    std::vector<double> gsnk, gsrc;
    std::vector<float> gsrc_f;
    std::vector<int2> pairs, work;
    int C3 = 0, nsplit = 1, elem_tc = 1;
    int Np = 16, corr_tc = 1;
    size_t off_mom = 0, off_pairs = 0, off_work = 0, off_gsnk = 0, off_gsrc = 0, off_gsrc_f = 0, off_phi = 0;
    bool phi_internal = false;
    // Sink timeslices [t_begin, t_end) of this call (0 / 0 = all T). Internal
    // elementals hold only this range.
    int t_begin = 0, t_end = 0;
    // Source elementals Phi(t0) [nmom][N^3] at a separate DEVICE address (NULL:
    // inside phi, which then must cover t0). With src_compute, this call also
    // computes them there (one extra elementals piece at t0).
    void* src_phi = nullptr;
    bool src_compute = false;
};

struct Piece {
    int job, t_off, Tc;
    size_t scratch_off;  // relative to the scratch region
    bool src = false;    // elementals piece that writes the source block src_phi
};

struct Stage {
    int kid, cls, prec;
    std::vector<Piece> pcs;
    size_t off_descs = 0, off_offs = 0, off_offs2 = 0;
    int nitems = 0, nitems2 = 0;
};

struct HostBlock {
    std::vector<char> bytes;
    size_t add(const void* src, size_t n) {
        const size_t off = align_up(bytes.size(), 256);
        bytes.resize(off + n);
        if (n) memcpy(bytes.data() + off, src, n);
        return off;
    }
    size_t reserve(size_t n) {
        const size_t off = align_up(bytes.size(), 256);
        bytes.resize(off + n, 0);
        return off;
    }
};

struct Program {
    std::vector<Job> jobs;
    HostBlock block;
    std::vector<Stage> stages;
    size_t scratch_off = 0, scratch_bytes = 0, total_bytes = 0;
};

// Scratch caps: of one piece's elementals partials, of one piece's contraction
// intermediates, and of one round of pieces (a call's workspace, unless the context's
// budget is lower). A round of 64 GiB lets a batch of many jobs run in few rounds
// (the 64-job batched workload holds about 450 GB of X in all) next to ~80 GB of inputs
// on a 288 GB MI355X.
const size_t kElemCap = (size_t)1 << 30;
const size_t kCorrCap = (size_t)4 << 30;
const size_t kBatchCap = (size_t)64 << 30;
// Static device scratch of nuc_correlator_noalloc and the pinned staging buffer
// every context allocates at creation (launch constants of that call go through it).
const size_t kStaticScratchBytes = NUC_STATIC_SCRATCH_BYTES;
const size_t kStaticStagingBytes = (size_t)1 << 20;

void eval_profiles(const nuc_geom* g, const double* evals, int nprof, const nuc_profile* prof, double* out);
nuc_status make_job(nuc_ctx ctx, const nuc_geom* g, const void* evecs, const double* evals, int nprof,
                    const nuc_profile* prof, int nmom, const int32_t* mom, const void* peramb, nuc_precision prec,
                    void* phi, void* corr, int stage, Job& J, int ld = 0);
// Plan pieces, rounds and stages; ws_cap bounds the scratch of one round.
nuc_status plan_program(nuc_ctx ctx, Program& P, size_t ws_cap);
// Plan, upload and enqueue P on stream s in ctx's workspace (ordered after ctx's previous call).
nuc_status run_program(nuc_ctx ctx, Program& P, hipStream_t s);
nuc_status ensure_workspace(nuc_ctx ctx, size_t bytes, hipStream_t s);
// Order a call after ctx's previous call (begin) and mark its end (end); copy a
// host block to device memory through ctx's pinned staging buffer.
nuc_status begin_call(nuc_ctx ctx, hipStream_t s);
nuc_status end_call(nuc_ctx ctx, hipStream_t s);
nuc_status upload_block(nuc_ctx ctx, const HostBlock& hb, void* dst, hipStream_t s, bool may_grow = true);
nuc_status check_geom(nuc_ctx ctx, const nuc_geom* g);
nuc_status check_moms(nuc_ctx ctx, const nuc_geom* g, int nmom, const int32_t* mom);
nuc_status check_profiles(nuc_ctx ctx, const nuc_geom* g, const double* evals, int nprof, const nuc_profile* prof);

hipEvent_t pool_get(nuc_ctx ctx);

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


}  // namespace rt
}  // namespace nuc

// Serving loop of the nucleon-correlator library (include/nucleon_server.h):
// resident gauge configurations, admission of jobs into a fixed device arena,
// and continuous batching of timeslice chunks of the admitted jobs into
// iterations that run on several HIP streams at once. The scheduler is written
// against an executor interface with two implementations: the HIP executor
// (slot contexts of the batch runtime) and a fake one with a cost model and a
// virtual clock, which runs the same scheduler with no device.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/nucleon_server.h"
#include "runtime_internal.h"

using namespace nuc;

namespace {

// ------------------------------------------------------------------ arena
// First-fit allocator over [0, size) with coalescing of free neighbours.
class Arena {
   public:
    explicit Arena(size_t size = 0) { reset(size); }
    void reset(size_t size) {
        size_ = size;
        used_ = peak_ = 0;
        free_.clear();
        if (size) free_[0] = size;
    }
    // Returns the offset, or SIZE_MAX if no free range is large enough.
    size_t alloc(size_t bytes) {
        bytes = rt::align_up(std::max<size_t>(bytes, 1), 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > bytes) free_[off + bytes] = len - bytes;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return off;
        }
        return SIZE_MAX;
    }
    void release(size_t off, size_t bytes) {
        bytes = rt::align_up(std::max<size_t>(bytes, 1), 256);
        used_ -= bytes;
        auto next = free_.lower_bound(off);
        size_t start = off, len = bytes;
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        if (next != free_.end() && next->first == off + bytes) {
            len += next->second;
            free_.erase(next);
        }
        free_[start] = len;
    }
    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

   private:
    size_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

// ------------------------------------------------------------- data model

struct Conf {
    nuc_geom g{};                 // nvec = nvec_max
    void* evecs = nullptr;        // DEVICE c64 [T][nmax][V3][3] (HIP executor)
    void* tau = nullptr;          // DEVICE c64 [T][4 nmax][4 nmax]
    std::vector<double> evals;    // HOST [T][nmax], empty if not given
    size_t bytes = 0;
    int users = 0;                // queued or admitted jobs
};

enum JobState { kQueued, kActive, kDone };

struct SJob {
    uint64_t ticket = 0, conf_id = 0;
    rt::Job tmpl;                 // validated job with the profiles evaluated
    int T = 0, nvec = 0, nmom = 0, nprof = 0;
    double flops_t = 0.0;         // algorithmic flops of one sink timeslice
    double flops_src = 0.0;       // elementals of the source timeslice
    double flops = 0.0;           // whole job
    size_t bytes_src = 0, bytes_corr = 0, arena_off = SIZE_MAX;
    int next_t = 0, t_done = 0, inflight = 0;
    bool src_done = false, src_inflight = false, cancelled = false;
    int status = NUC_OK;
    JobState state = kQueued;
    double submit_s = 0, admit_s = -1, start_s = -1, done_s = -1;
    double service = 0.0;         // flops launched so far
    int iterations = 0;
    std::vector<double2> result;  // HOST [nmom][T][nprof][nprof]
};
using JobPtr = std::shared_ptr<SJob>;

struct Chunk {
    JobPtr job;
    int tb, te;
    bool src;
    double flops;
};

struct Iteration {
    std::vector<Chunk> chunks;
    double flops = 0.0;
};

double choose(double n, int k) {
    double r = 1.0;
    for (int i = 0; i < k; ++i) r = r * (n - i) / (i + 1);
    return r;
}

// Algorithmic flops (elementals: 24 V3 C(N,3) per (t, p) plus 42 V3 C(N,2) per t
// of colour cross products; contraction: 768 N^4 per (t, p, b) for the three
// tau steps of both spin components, plus the sink dots).
double flops_elem_t(int L, int N, int nmom) {
    const double V3 = (double)L * L * L;
    return 24.0 * V3 * choose(N, 3) * nmom + 42.0 * V3 * choose(N, 2);
}
double flops_corr_t(int N, int nmom, int nprof) {
    const double n = N;
    return nmom * (768.0 * nprof * n * n * n * n + nprof * 2.0 * (8.0 * n * n * n + nprof * 4.0 * n * n * n));
}

// ------------------------------------------------------------- executors

class Executor {
   public:
    virtual ~Executor() {}
    virtual bool virtual_time() const = 0;
    virtual double now() = 0;
    // Enqueue an iteration on slot; err gets the detail of a failure.
    virtual nuc_status launch(int slot, const Iteration& it, std::string& err) = 0;
    // 1 done, 0 running, < 0 the iteration failed (a nuc_status)
    virtual int poll(int slot, const Iteration& it) = 0;
    // Earliest completion among busy slots (virtual time only).
    virtual double next_done() { return 0.0; }
    virtual void advance_to(double) {}
    // Bring a finished job's result to host memory.
    virtual nuc_status fetch(SJob& j, std::string& err) = 0;
    virtual nuc_status add_conf(Conf& c, const void* ev, const void* tau, std::string& err) = 0;
    virtual void drop_conf(Conf& c) = 0;
    virtual char* arena_base() = 0;
    virtual const void* conf_ptr_evecs(const Conf& c) = 0;
    virtual const void* conf_ptr_tau(const Conf& c) = 0;
};

class FakeExecutor : public Executor {
   public:
    FakeExecutor(int slots, double rate, double fixed, int fault_at)
        : done_at_(slots, 0.0), busy_(slots, false), rate_(rate), fixed_(fixed), fault_at_(fault_at) {}
    bool virtual_time() const override { return true; }
    double now() override { return clock_; }
    nuc_status launch(int slot, const Iteration& it, std::string&) override {
        ++launches_;
        const double start = std::max(clock_, device_free_);
        device_free_ = start + fixed_ + it.flops / rate_;
        done_at_[slot] = device_free_;
        busy_[slot] = true;
        fail_[slot] = (launches_ == fault_at_);
        return NUC_OK;
    }
    int poll(int slot, const Iteration& it) override {
        if (!busy_[slot] || clock_ < done_at_[slot]) return 0;
        busy_[slot] = false;
        if (fail_[slot]) return NUC_ERR_DEVICE;
        for (const Chunk& c : it.chunks) {
            SJob& j = *c.job;
            for (int p = 0; p < j.nmom; ++p)
                for (int t = c.tb; t < c.te; ++t)
                    for (int ab = 0; ab < j.nprof * j.nprof; ++ab) {
                        double2& v = j.result[((size_t)p * j.T + t) * j.nprof * j.nprof + ab];
                        v.x += 1.0;
                        v.y = (double)j.ticket;
                    }
        }
        return 1;
    }
    double next_done() override {
        double t = 1e300;
        for (size_t s = 0; s < busy_.size(); ++s)
            if (busy_[s]) t = std::min(t, done_at_[s]);
        return t;
    }
    void advance_to(double t) override { clock_ = std::max(clock_, t); }
    nuc_status fetch(SJob&, std::string&) override { return NUC_OK; }
    nuc_status add_conf(Conf&, const void*, const void*, std::string&) override { return NUC_OK; }
    void drop_conf(Conf&) override {}
    char* arena_base() override { return nullptr; }
    const void* conf_ptr_evecs(const Conf&) override { return nullptr; }
    const void* conf_ptr_tau(const Conf&) override { return nullptr; }

   private:
    std::vector<double> done_at_;
    std::vector<bool> busy_;
    std::map<int, bool> fail_;
    double clock_ = 0.0, device_free_ = 0.0, rate_, fixed_;
    long long launches_ = 0, fault_at_;
};

class HipExecutor : public Executor {
   public:
    ~HipExecutor() override { release(); }

    nuc_status init(int device, int slots, size_t slot_ws, size_t arena_bytes, std::string& err) {
        device_ = device;
        t_start_ = std::chrono::steady_clock::now();
        rt::DeviceGuard guard;
        hipError_t e = hipSetDevice(device);
        if (e != hipSuccess) return hfail(e, "hipSetDevice", err);
        if ((e = hipStreamCreateWithFlags(&copy_, hipStreamNonBlocking)) != hipSuccess)
            return hfail(e, "hipStreamCreateWithFlags", err);
        if ((e = hipMalloc(&arena_, std::max<size_t>(arena_bytes, 256))) != hipSuccess) {
            arena_ = nullptr;
            (void)hipGetLastError();
            err = "arena: hipMalloc failed";
            return NUC_ERR_NOMEM;
        }
        for (int s = 0; s < slots; ++s) {
            Slot sl;
            nuc_status st = nuc_create(&sl.ctx, device, slot_ws);
            if (st != NUC_OK) {
                err = nuc_last_error(nullptr);
                return st;
            }
            slots_.push_back(sl);
            Slot& S = slots_.back();
            if ((e = hipStreamCreateWithFlags(&S.stream, hipStreamNonBlocking)) != hipSuccess)
                return hfail(e, "hipStreamCreateWithFlags", err);
            if ((e = hipEventCreateWithFlags(&S.done, hipEventDisableTiming)) != hipSuccess)
                return hfail(e, "hipEventCreateWithFlags", err);
            // full-size workspace up front: no reallocation (and no implicit
            // device synchronisation of hipFree) while serving
            st = rt::ensure_workspace(S.ctx, slot_ws, S.stream);
            if (st != NUC_OK) {
                err = S.ctx->err;
                return st;
            }
        }
        return NUC_OK;
    }

    bool virtual_time() const override { return false; }
    double now() override {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start_).count();
    }

    void set_confs(const std::map<uint64_t, Conf>* confs) { confs_ = confs; }

    nuc_status launch(int slot, const Iteration& it, std::string& err) override {
        Slot& S = slots_[slot];
        rt::DeviceGuard guard;
        hipError_t e = hipSetDevice(device_);
        if (e != hipSuccess) return hfail(e, "hipSetDevice", err);
        rt::Program P;
        for (const Chunk& c : it.chunks) P.jobs.push_back(chunk_job(c, (char*)arena_));
        nuc_status st;
        {
            std::lock_guard<std::mutex> lock(S.ctx->mu);
            st = rt::run_program(S.ctx, P, S.stream);
            if (st != NUC_OK) err = S.ctx->err;
        }
        if (st != NUC_OK) return st;
        if ((e = hipEventRecord(S.done, S.stream)) != hipSuccess) return hfail(e, "hipEventRecord", err);
        return NUC_OK;
    }

    int poll(int slot, const Iteration&) override {
        hipError_t e = hipEventQuery(slots_[slot].done);
        if (e == hipSuccess) return 1;
        if (e == hipErrorNotReady) return 0;
        (void)hipGetLastError();
        return NUC_ERR_DEVICE;
    }

    nuc_status fetch(SJob& j, std::string& err) override {
        rt::DeviceGuard guard;
        hipError_t e = hipSetDevice(device_);
        if (e == hipSuccess)
            e = hipMemcpyAsync(j.result.data(), (char*)arena_ + j.arena_off + j.bytes_src,
                               j.result.size() * sizeof(double2), hipMemcpyDeviceToHost, copy_);
        if (e == hipSuccess) e = hipStreamSynchronize(copy_);
        if (e != hipSuccess) return hfail(e, "result copy", err);
        return NUC_OK;
    }

    nuc_status add_conf(Conf& c, const void* ev, const void* tau, std::string& err) override {
        rt::DeviceGuard guard;
        hipError_t e = hipSetDevice(device_);
        if (e != hipSuccess) return hfail(e, "hipSetDevice", err);
        const size_t V3 = (size_t)c.g.L * c.g.L * c.g.L, N = c.g.nvec;
        const size_t bev = (size_t)c.g.T * N * V3 * 3 * sizeof(float2);
        const size_t btau = (size_t)c.g.T * 16 * N * N * sizeof(float2);
        if ((e = hipMalloc(&c.evecs, bev)) != hipSuccess || (e = hipMalloc(&c.tau, btau)) != hipSuccess) {
            (void)hipGetLastError();
            drop_conf(c);
            err = "resident data: hipMalloc failed";
            return NUC_ERR_NOMEM;
        }
        // the caller's buffers may still be written by work on any stream
        if ((e = hipDeviceSynchronize()) != hipSuccess ||
            (e = hipMemcpyAsync(c.evecs, ev, bev, hipMemcpyDeviceToDevice, copy_)) != hipSuccess ||
            (e = hipMemcpyAsync(c.tau, tau, btau, hipMemcpyDeviceToDevice, copy_)) != hipSuccess ||
            (e = hipStreamSynchronize(copy_)) != hipSuccess) {
            drop_conf(c);
            return hfail(e, "resident copy", err);
        }
        return NUC_OK;
    }

    void drop_conf(Conf& c) override {
        rt::DeviceGuard guard;
        (void)hipSetDevice(device_);
        if (c.evecs) (void)hipFree(c.evecs);
        if (c.tau) (void)hipFree(c.tau);
        c.evecs = c.tau = nullptr;
    }

    char* arena_base() override { return (char*)arena_; }
    const void* conf_ptr_evecs(const Conf& c) override { return c.evecs; }
    const void* conf_ptr_tau(const Conf& c) override { return c.tau; }

    void release() {
        rt::DeviceGuard guard;
        (void)hipSetDevice(device_);
        for (Slot& S : slots_) {
            if (S.stream) (void)hipStreamSynchronize(S.stream);
            if (S.ctx) (void)nuc_destroy(S.ctx);
            if (S.done) (void)hipEventDestroy(S.done);
            if (S.stream) (void)hipStreamDestroy(S.stream);
        }
        slots_.clear();
        if (copy_) (void)hipStreamDestroy(copy_);
        copy_ = nullptr;
        if (arena_) (void)hipFree(arena_);
        arena_ = nullptr;
    }

    // The batch-runtime job of one chunk: sink timeslices [tb, te) of the job,
    // elementals in the slot workspace, source block and result in the arena.
    rt::Job chunk_job(const Chunk& c, char* base) const {
        const SJob& j = *c.job;
        rt::Job J = j.tmpl;
        const Conf& cf = confs_->at(j.conf_id);
        J.evecs = cf.evecs;
        J.peramb = cf.tau;
        J.ld = cf.g.nvec;
        J.phi = nullptr;
        J.t_begin = c.tb;
        J.t_end = c.te;
        J.src_phi = base ? base + j.arena_off : nullptr;
        J.src_compute = c.src;
        J.corr = base ? base + j.arena_off + j.bytes_src : nullptr;
        return J;
    }

   private:
    struct Slot {
        nuc_ctx ctx = nullptr;
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
    };
    nuc_status hfail(hipError_t e, const char* what, std::string& err) {
        char buf[256];
        snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
        err = buf;
        (void)hipGetLastError();
        return NUC_ERR_DEVICE;
    }
    int device_ = 0;
    std::chrono::steady_clock::time_point t_start_;
    hipStream_t copy_ = nullptr;
    void* arena_ = nullptr;
    std::vector<Slot> slots_;
    const std::map<uint64_t, Conf>* confs_ = nullptr;
};

thread_local std::string g_server_err;

}  // namespace

// ------------------------------------------------------------------ server

struct nuc_server_s {
    nuc_server_config cfg{};
    std::unique_ptr<Executor> exec;
    HipExecutor* hip = nullptr;  // == exec.get() for the HIP executor
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread thread;
    bool stop = false, paused = false;
    std::string err;

    std::map<uint64_t, Conf> confs;
    std::map<uint64_t, JobPtr> jobs;  // not yet retired by nuc_server_wait
    std::deque<JobPtr> queue;
    std::vector<JobPtr> active;
    std::vector<Iteration> slot_it;
    std::vector<bool> slot_busy;
    Arena arena;
    uint64_t next_ticket = 1;
    size_t bytes_resident = 0;

    // metrics
    long long n_submitted = 0, n_completed = 0, n_failed = 0, n_cancelled = 0, n_iterations = 0;
    int max_outstanding = 0;
    std::vector<double> lat_ms;
    double first_submit = -1.0, last_done = -1.0, flops_done = 0.0;

    nuc_status set_err(nuc_status s, const char* fmt, ...) __attribute__((format(printf, 3, 4))) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        err = buf;
        g_server_err = buf;
        return s;
    }

    size_t slot_cap() const { return std::min(rt::kBatchCap, cfg.slot_workspace / 2); }

    // Workspace a set of chunks needs in one slot (host planning only).
    size_t plan_bytes(const std::vector<Chunk>& cs, nuc_status* st) const {
        rt::Program P;
        for (const Chunk& c : cs) {
            rt::Job J = c.job->tmpl;
            J.phi = nullptr;
            J.t_begin = c.tb;
            J.t_end = c.te;
            J.src_phi = (void*)256;  // planning only: any non-null address
            J.src_compute = c.src;
            P.jobs.push_back(J);
        }
        *st = rt::plan_program(nullptr, P, slot_cap());
        return P.total_bytes;
    }

    void finish(const JobPtr& j) {
        // called with mu held, when the job has no chunk in flight
        if (j->state == kDone) return;
        if (j->status == NUC_OK && j->cancelled) j->status = NUC_ERR_CANCELLED;
        if (j->status == NUC_OK) {
            std::string e;
            nuc_status st = exec->fetch(*j, e);
            if (st != NUC_OK) {
                j->status = st;
                set_err(st, "ticket %llu: %s", (unsigned long long)j->ticket, e.c_str());
            }
        }
        if (j->arena_off != SIZE_MAX) {
            arena.release(j->arena_off, j->bytes_src + j->bytes_corr);
            j->arena_off = SIZE_MAX;
        }
        confs[j->conf_id].users -= 1;
        j->state = kDone;
        j->done_s = exec->now();
        if (j->status == NUC_OK) {
            n_completed += 1;
            lat_ms.push_back(1e3 * (j->done_s - j->submit_s));
            last_done = std::max(last_done, j->done_s);
            flops_done += j->flops;
        } else if (j->status == NUC_ERR_CANCELLED) {
            n_cancelled += 1;
        } else {
            n_failed += 1;
        }
        active.erase(std::remove(active.begin(), active.end(), j), active.end());
        cv_done.notify_all();
    }

    void maybe_finish(const JobPtr& j) {
        if (j->state != kActive || j->inflight > 0) return;
        if (j->status != NUC_OK || j->cancelled || j->t_done == j->T) finish(j);
    }

    bool admit() {
        bool any = false;
        while (!queue.empty() && (int)active.size() < cfg.max_active) {
            JobPtr j = queue.front();
            if (j->cancelled) {
                queue.pop_front();
                j->status = NUC_ERR_CANCELLED;
                j->state = kActive;  // finish() expects an admitted job
                active.push_back(j);
                finish(j);
                any = true;
                continue;
            }
            const size_t off = arena.alloc(j->bytes_src + j->bytes_corr);
            if (off == SIZE_MAX) break;  // FIFO: later jobs wait behind the head
            queue.pop_front();
            j->arena_off = off;
            j->state = kActive;
            j->admit_s = exec->now();
            active.push_back(j);
            any = true;
        }
        return any;
    }

    // Next iteration for a free slot: chunks of the admitted jobs in order of
    // least service received, each sized to the remaining flop quantum.
    bool build(Iteration& it) {
        std::vector<JobPtr> cand;
        for (const JobPtr& j : active)
            if (!j->cancelled && j->status == NUC_OK && j->next_t < j->T && !j->src_inflight &&
                (j->src_done || j->inflight == 0))
                cand.push_back(j);
        if (cand.empty()) return false;
        std::stable_sort(cand.begin(), cand.end(), [](const JobPtr& a, const JobPtr& b) {
            return a->service != b->service ? a->service < b->service : a->ticket < b->ticket;
        });
        double remaining = cfg.quantum_flops;
        it.chunks.clear();
        it.flops = 0.0;
        for (const JobPtr& j : cand) {
            if (!it.chunks.empty() && j->flops_t > remaining) continue;
            int k = (int)std::floor(remaining / std::max(j->flops_t, 1.0));
            k = std::max(1, std::min(k, j->T - j->next_t));
            const bool src = !j->src_done;
            for (;;) {
                Chunk c{j, j->next_t, j->next_t + k, src, k * j->flops_t + (src ? j->flops_src : 0.0)};
                it.chunks.push_back(c);
                nuc_status st;
                const size_t b = plan_bytes(it.chunks, &st);
                if (st == NUC_OK && b <= cfg.slot_workspace) break;
                it.chunks.pop_back();
                if (k > 1) {
                    k /= 2;
                    continue;
                }
                if (it.chunks.empty()) {  // one timeslice alone does not fit
                    j->status = set_err(NUC_ERR_NOMEM, "ticket %llu: one timeslice exceeds the slot workspace",
                                        (unsigned long long)j->ticket);
                    maybe_finish(j);
                }
                k = 0;
                break;
            }
            if (k == 0) continue;
            const Chunk& c = it.chunks.back();
            it.flops += c.flops;
            remaining -= c.flops;
            if (remaining <= 0.0) break;
        }
        return !it.chunks.empty();
    }

    void launch(int slot, Iteration& it) {
        const double now = exec->now();
        for (Chunk& c : it.chunks) {
            SJob& j = *c.job;
            j.next_t = c.te;
            j.inflight += 1;
            if (c.src) j.src_inflight = true;
            j.service += c.flops;
            j.iterations += 1;
            if (j.start_s < 0) j.start_s = now;
        }
        std::string e;
        nuc_status st = exec->launch(slot, it, e);
        n_iterations += 1;
        if (st != NUC_OK) {
            set_err(st, "iteration launch: %s", e.c_str());
            complete(it, st);
            return;
        }
        slot_it[slot] = it;
        slot_busy[slot] = true;
    }

    void complete(Iteration& it, int r) {
        for (Chunk& c : it.chunks) {
            JobPtr j = c.job;
            j->inflight -= 1;
            if (c.src) j->src_inflight = false;
            if (r < 0) {
                if (j->status == NUC_OK) j->status = r;
            } else {
                j->t_done += c.te - c.tb;
                if (c.src) j->src_done = true;
            }
            maybe_finish(j);
        }
    }

    void loop() {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            bool progress = false, inflight = false;
            for (size_t s = 0; s < slot_busy.size(); ++s) {
                if (!slot_busy[s]) continue;
                const int r = exec->poll((int)s, slot_it[s]);
                if (r == 0) {
                    inflight = true;
                    continue;
                }
                if (r < 0) set_err((nuc_status)r, "iteration on slot %zu failed", s);
                slot_busy[s] = false;
                Iteration it = std::move(slot_it[s]);
                slot_it[s] = Iteration();
                complete(it, r);
                progress = true;
            }
            if (stop && !inflight && !progress) break;
            if (!paused && !stop) {
                progress |= admit();
                for (size_t s = 0; s < slot_busy.size(); ++s) {
                    if (slot_busy[s]) continue;
                    Iteration it;
                    if (!build(it)) break;
                    launch((int)s, it);
                    inflight |= slot_busy[s];
                    progress = true;
                }
            }
            if (progress) continue;
            if (inflight) {
                if (exec->virtual_time())
                    exec->advance_to(exec->next_done());
                else
                    cv_work.wait_for(lk, std::chrono::microseconds(200));
            } else {
                cv_work.wait(lk);
            }
        }
    }
};

namespace {

nuc_status srv_fail(nuc_server s, nuc_status st, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
nuc_status srv_fail(nuc_server s, nuc_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_server_err = buf;
    if (s) s->err = buf;
    return st;
}

double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    // nearest rank: the smallest value with at least q of the samples at or below it
    size_t r = (size_t)std::ceil(q * (double)v.size());
    r = std::max<size_t>(1, std::min(r, v.size()));
    return v[r - 1];
}

}  // namespace

extern "C" {

nuc_status nuc_server_create(const nuc_server_config* cfg_in, nuc_server* out) {
    if (!out) return srv_fail(nullptr, NUC_ERR_INVALID, "out is NULL");
    *out = nullptr;
    nuc_server_config cfg{};
    if (cfg_in) cfg = *cfg_in;
    if (cfg.executor != NUC_EXEC_HIP && cfg.executor != NUC_EXEC_FAKE)
        return srv_fail(nullptr, NUC_ERR_INVALID, "executor=%d is not a nuc_executor_kind", cfg.executor);
    if (cfg.slots == 0) cfg.slots = 2;
    if (cfg.slots < 1 || cfg.slots > 8) return srv_fail(nullptr, NUC_ERR_INVALID, "slots=%d out of [1,8]", cfg.slots);
    if (cfg.max_active == 0) cfg.max_active = 64;
    if (cfg.max_active < 1 || cfg.max_active > 4096)
        return srv_fail(nullptr, NUC_ERR_INVALID, "max_active=%d out of [1,4096]", cfg.max_active);
    if (cfg.job_arena == 0) cfg.job_arena = (size_t)4 << 30;
    if (cfg.slot_workspace == 0) cfg.slot_workspace = (size_t)16 << 30;
    if (cfg.slot_workspace < ((size_t)64 << 20))
        return srv_fail(nullptr, NUC_ERR_INVALID, "slot_workspace=%zu below 64 MiB", cfg.slot_workspace);
    if (!(cfg.quantum_flops >= 0.0)) return srv_fail(nullptr, NUC_ERR_INVALID, "quantum_flops is negative or NaN");
    if (cfg.quantum_flops == 0.0) cfg.quantum_flops = 4e12;
    if (cfg.fake_flops_per_s == 0.0) cfg.fake_flops_per_s = 5e13;
    if (cfg.fake_fixed_s == 0.0) cfg.fake_fixed_s = 1e-4;
    if (!(cfg.fake_flops_per_s > 0.0) || !(cfg.fake_fixed_s >= 0.0))
        return srv_fail(nullptr, NUC_ERR_INVALID, "fake cost model must be positive");
    const size_t fixed = cfg.job_arena + (size_t)cfg.slots * cfg.slot_workspace;
    if (cfg.hbm_budget && fixed > cfg.hbm_budget)
        return srv_fail(nullptr, NUC_ERR_NOMEM, "arena + slot workspaces (%zu bytes) exceed hbm_budget (%zu bytes)",
                        fixed, cfg.hbm_budget);
    std::unique_ptr<nuc_server_s> s(new nuc_server_s());
    s->cfg = cfg;
    s->paused = cfg.start_paused != 0;
    s->arena.reset(cfg.job_arena);
    s->slot_it.resize(cfg.slots);
    s->slot_busy.assign(cfg.slots, false);
    if (cfg.executor == NUC_EXEC_FAKE) {
        const char* f = getenv("NUC_FAULT_INJECT");
        s->exec.reset(new FakeExecutor(cfg.slots, cfg.fake_flops_per_s, cfg.fake_fixed_s, f ? atoi(f) : 0));
    } else {
        HipExecutor* h = new HipExecutor();
        s->exec.reset(h);
        s->hip = h;
        std::string e;
        nuc_status st = h->init(cfg.device, cfg.slots, cfg.slot_workspace, cfg.job_arena, e);
        if (st != NUC_OK) return srv_fail(nullptr, st, "server create: %s", e.c_str());
        h->set_confs(&s->confs);
    }
    nuc_server srv = s.release();
    srv->thread = std::thread([srv] { srv->loop(); });
    *out = srv;
    return NUC_OK;
}

nuc_status nuc_server_destroy(nuc_server s) {
    if (!s) return NUC_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        for (const JobPtr& j : s->active) j->cancelled = true;
        while (!s->queue.empty()) {
            JobPtr j = s->queue.front();
            s->queue.pop_front();
            j->status = NUC_ERR_CANCELLED;
            j->state = kActive;
            s->active.push_back(j);
            s->finish(j);
        }
    }
    s->cv_work.notify_all();
    if (s->thread.joinable()) s->thread.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (JobPtr j : std::vector<JobPtr>(s->active)) s->maybe_finish(j);
        for (auto& kv : s->confs) s->exec->drop_conf(kv.second);
    }
    s->exec.reset();
    delete s;
    return NUC_OK;
}

nuc_status nuc_server_register(nuc_server s, uint64_t conf_id, const nuc_geom* g, const void* evecs,
                               const double* evals, const void* peramb) {
    if (!s) return srv_fail(nullptr, NUC_ERR_INVALID, "server is NULL");
    if (!g) return srv_fail(s, NUC_ERR_INVALID, "geom is NULL");
    if (g->L < 1 || g->L > 256 || g->T < 1 || g->nvec < 3 || g->nvec > kMaxNvec || g->t0 < 0 || g->t0 >= g->T)
        return srv_fail(s, NUC_ERR_INVALID, "geometry L=%d T=%d nvec=%d t0=%d out of range", g->L, g->T, g->nvec,
                        g->t0);
    const bool fake = s->cfg.executor == NUC_EXEC_FAKE;
    if (!fake && (!evecs || !peramb)) return srv_fail(s, NUC_ERR_INVALID, "evecs or peramb is NULL");
    const size_t V3 = (size_t)g->L * g->L * g->L, N = g->nvec;
    const size_t bytes = (size_t)g->T * N * V3 * 3 * sizeof(float2) + (size_t)g->T * 16 * N * N * sizeof(float2);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->confs.count(conf_id)) return srv_fail(s, NUC_ERR_BUSY, "conf_id %llu already registered",
                                                 (unsigned long long)conf_id);
    const size_t fixed = s->cfg.job_arena + (size_t)s->cfg.slots * s->cfg.slot_workspace;
    if (s->cfg.hbm_budget && fixed + s->bytes_resident + bytes > s->cfg.hbm_budget)
        return srv_fail(s, NUC_ERR_NOMEM, "conf_id %llu (%zu bytes) would exceed hbm_budget (%zu bytes in use of %zu)",
                        (unsigned long long)conf_id, bytes, fixed + s->bytes_resident, s->cfg.hbm_budget);
    Conf c;
    c.g = *g;
    c.bytes = bytes;
    if (evals) c.evals.assign(evals, evals + (size_t)g->T * N);
    std::string e;
    nuc_status st = s->exec->add_conf(c, evecs, peramb, e);
    if (st != NUC_OK) return srv_fail(s, st, "register: %s", e.c_str());
    s->confs[conf_id] = std::move(c);
    s->bytes_resident += bytes;
    return NUC_OK;
}

nuc_status nuc_server_unregister(nuc_server s, uint64_t conf_id) {
    if (!s) return srv_fail(nullptr, NUC_ERR_INVALID, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->confs.find(conf_id);
    if (it == s->confs.end())
        return srv_fail(s, NUC_ERR_INVALID, "conf_id %llu not registered", (unsigned long long)conf_id);
    if (it->second.users > 0)
        return srv_fail(s, NUC_ERR_BUSY, "conf_id %llu is used by %d job(s)", (unsigned long long)conf_id,
                        it->second.users);
    s->exec->drop_conf(it->second);
    s->bytes_resident -= it->second.bytes;
    s->confs.erase(it);
    return NUC_OK;
}

nuc_status nuc_server_submit(nuc_server s, const nuc_request* r, uint64_t* ticket) {
    if (!s) return srv_fail(nullptr, NUC_ERR_INVALID, "server is NULL");
    if (!r || !ticket) return srv_fail(s, NUC_ERR_INVALID, "request or ticket is NULL");
    *ticket = 0;
    JobPtr j = std::make_shared<SJob>();
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->confs.find(r->conf_id);
    if (it == s->confs.end())
        return srv_fail(s, NUC_ERR_INVALID, "conf_id %llu not registered", (unsigned long long)r->conf_id);
    Conf& cf = it->second;
    if (r->nvec < 3 || r->nvec > cf.g.nvec)
        return srv_fail(s, NUC_ERR_INVALID, "nvec=%d outside [3, %d] of conf_id %llu", r->nvec, cf.g.nvec,
                        (unsigned long long)r->conf_id);
    nuc_geom g = cf.g;
    g.nvec = r->nvec;
    std::vector<double> ev;
    if (!cf.evals.empty()) {
        ev.resize((size_t)g.T * g.nvec);
        for (int t = 0; t < g.T; ++t)
            memcpy(&ev[(size_t)t * g.nvec], &cf.evals[(size_t)t * cf.g.nvec], g.nvec * sizeof(double));
    }
    // validation and FP64 profile evaluation; device addresses are set per chunk
    void* dummy = (void*)256;
    nuc_status st = rt::make_job(nullptr, &g, dummy, ev.empty() ? nullptr : ev.data(), r->nprof, r->prof, r->nmom,
                                 r->mom, dummy, (nuc_precision)r->precision, nullptr, dummy, 3, j->tmpl, cf.g.nvec);
    if (st != NUC_OK) return srv_fail(s, st, "request: %s", nuc_last_error(nullptr));
    j->conf_id = r->conf_id;
    j->T = g.T;
    j->nvec = g.nvec;
    j->nmom = r->nmom;
    j->nprof = r->nprof;
    j->flops_t = flops_elem_t(g.L, g.nvec, r->nmom) + flops_corr_t(g.nvec, r->nmom, r->nprof);
    j->flops_src = flops_elem_t(g.L, g.nvec, r->nmom);
    j->flops = g.T * j->flops_t;
    const size_t n3 = (size_t)g.nvec * g.nvec * g.nvec;
    j->bytes_src = rt::align_up((size_t)r->nmom * n3 * sizeof(float2), 256);
    j->bytes_corr = rt::align_up((size_t)r->nmom * g.T * r->nprof * r->nprof * sizeof(double2), 256);
    if (j->bytes_src + j->bytes_corr > s->arena.size())
        return srv_fail(s, NUC_ERR_BUSY, "job buffers (%zu bytes) exceed the job arena (%zu bytes)",
                        j->bytes_src + j->bytes_corr, s->arena.size());
    {
        std::vector<Chunk> one{Chunk{j, 0, 1, true, 0.0}};
        const size_t b = s->plan_bytes(one, &st);
        if (st != NUC_OK || b > s->cfg.slot_workspace)
            return srv_fail(s, NUC_ERR_BUSY, "one timeslice needs %zu bytes of workspace, a slot has %zu", b,
                            s->cfg.slot_workspace);
    }
    j->result.assign((size_t)r->nmom * g.T * r->nprof * r->nprof, double2{0.0, 0.0});
    j->ticket = s->next_ticket++;
    j->submit_s = s->exec->now();
    if (s->first_submit < 0) s->first_submit = j->submit_s;
    cf.users += 1;
    s->jobs[j->ticket] = j;
    s->queue.push_back(j);
    s->n_submitted += 1;
    s->max_outstanding = std::max(s->max_outstanding, (int)(s->queue.size() + s->active.size()));
    *ticket = j->ticket;
    lk.unlock();
    s->cv_work.notify_all();
    return NUC_OK;
}

nuc_status nuc_server_wait(nuc_server s, uint64_t ticket, int timeout_ms, void* corr_host, nuc_job_info* info) {
    if (!s) return srv_fail(nullptr, NUC_ERR_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end())
        return srv_fail(s, NUC_ERR_INVALID, "ticket %llu unknown or retired", (unsigned long long)ticket);
    JobPtr j = it->second;
    auto done = [&] { return j->state == kDone; };
    if (timeout_ms < 0)
        s->cv_done.wait(lk, done);
    else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done))
        return NUC_ERR_TIMEOUT;
    if (corr_host && j->status == NUC_OK)
        memcpy(corr_host, j->result.data(), j->result.size() * sizeof(double2));
    if (info) {
        info->status = j->status;
        info->submit_s = j->submit_s;
        info->admit_s = j->admit_s;
        info->start_s = j->start_s;
        info->done_s = j->done_s;
        info->flops = j->flops;
        info->iterations = j->iterations;
    }
    s->jobs.erase(it);
    return (nuc_status)j->status;
}

nuc_status nuc_server_cancel(nuc_server s, uint64_t ticket) {
    if (!s) return srv_fail(nullptr, NUC_ERR_INVALID, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end())
        return srv_fail(s, NUC_ERR_INVALID, "ticket %llu unknown or retired", (unsigned long long)ticket);
    JobPtr j = it->second;
    if (j->state == kDone) return NUC_OK;
    j->cancelled = true;
    if (j->state == kQueued) {
        s->queue.erase(std::remove(s->queue.begin(), s->queue.end(), j), s->queue.end());
        j->state = kActive;
        s->active.push_back(j);
    }
    s->maybe_finish(j);
    lk.unlock();
    s->cv_work.notify_all();
    return NUC_OK;
}

nuc_status nuc_server_resume(nuc_server s) {
    if (!s) return srv_fail(nullptr, NUC_ERR_INVALID, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->paused = false;
    }
    s->cv_work.notify_all();
    return NUC_OK;
}

nuc_status nuc_server_stats(nuc_server s, nuc_server_metrics* m) {
    if (!s) return srv_fail(nullptr, NUC_ERR_INVALID, "server is NULL");
    if (!m) return srv_fail(s, NUC_ERR_INVALID, "metrics is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    memset(m, 0, sizeof *m);
    m->submitted = s->n_submitted;
    m->completed = s->n_completed;
    m->failed = s->n_failed;
    m->cancelled = s->n_cancelled;
    m->iterations = s->n_iterations;
    m->queued = (int)s->queue.size();
    m->active = (int)s->active.size();
    m->max_outstanding = s->max_outstanding;
    m->p50_ms = percentile(s->lat_ms, 0.50);
    m->p99_ms = percentile(s->lat_ms, 0.99);
    double sum = 0.0, mx = 0.0;
    for (double v : s->lat_ms) {
        sum += v;
        mx = std::max(mx, v);
    }
    m->mean_ms = s->lat_ms.empty() ? 0.0 : sum / s->lat_ms.size();
    m->max_ms = mx;
    m->window_s = (s->first_submit >= 0 && s->last_done >= 0) ? s->last_done - s->first_submit : 0.0;
    m->jobs_per_s = m->window_s > 0 ? s->n_completed / m->window_s : 0.0;
    m->flops_per_s = m->window_s > 0 ? s->flops_done / m->window_s : 0.0;
    m->bytes_resident = s->bytes_resident;
    m->bytes_arena_used = s->arena.used();
    m->bytes_arena_peak = s->arena.peak();
    m->bytes_arena = s->arena.size();
    m->bytes_total = s->bytes_resident + s->arena.size() + (size_t)s->cfg.slots * s->cfg.slot_workspace;
    return NUC_OK;
}

const char* nuc_server_last_error(nuc_server s) { return s ? s->err.c_str() : g_server_err.c_str(); }

}  // extern "C"

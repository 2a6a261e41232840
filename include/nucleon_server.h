/*
 * nucleon_server.h - serving loop of the MI355X nucleon-correlator library.
 *
 * A server takes correlator jobs (a gauge configuration, a number of
 * distillation vectors, a momentum set and a profile basis) while earlier jobs
 * are still running, and produces for each the N_B x N_B matrix C_ab(t) of
 * Section 2.1 for every sink time and momentum, exactly as nuc_run would
 * (include/nucleon.h; same kernels, same per-(t, p) arithmetic, same reduction
 * order).
 *
 * Model
 *   - Residency: the eigenvectors (at nvec_max), eigenvalues and perambulators
 *     of each gauge configuration are copied once into server-owned device
 *     memory by nuc_server_register. A job uses the first nvec vectors and the
 *     matching sub-blocks of tau (distillation with fewer vectors).
 *   - Admission by HBM budget: an admitted job holds its source elementals
 *     Phi(t0) (c64 [nmom][nvec^3]) and its result (c128 [nmom][T][nprof][nprof])
 *     in a fixed device arena of job_arena bytes; a job waits in the queue until
 *     its buffers fit and fewer than max_active jobs are admitted. Everything the
 *     server allocates (resident data, arena, slot workspaces) is counted against
 *     hbm_budget.
 *   - Continuous batching: a job is split into chunks of sink timeslices. One
 *     iteration is one batched launch sequence (elementals, contraction) over
 *     chunks of several admitted jobs; iterations run on `slots` HIP streams,
 *     each with its own workspace of slot_workspace bytes, so their work overlaps
 *     on the device. Whenever a slot is free the scheduler builds the next
 *     iteration from the admitted jobs in order of least device work received so
 *     far (ties: submission order), giving each a chunk sized to the iteration's
 *     flop quantum; jobs that arrive meanwhile join the next iteration. A job's
 *     first chunk also computes its source elementals Phi(t0); its other chunks
 *     start after that one completed.
 *   - Latency of a job: from nuc_server_submit to its result being in host
 *     memory. Times are seconds on the server's clock (0 at creation; with the
 *     fake executor a virtual clock advanced by the cost model).
 *
 * Executors: NUC_EXEC_HIP runs on a GPU. NUC_EXEC_FAKE runs the same scheduler
 * with no device at all: an iteration "takes" fixed_s + flops / flops_per_s of
 * virtual time and marks, for each chunk, every (p, t) block of the job's result
 * with re += 1 and im = ticket (so tests can check that every block was computed
 * exactly once, for the right job). With environment variable
 * NUC_FAULT_INJECT=n the fake executor fails its n-th iteration (1-based) and the
 * jobs in it end with NUC_ERR_DEVICE.
 *
 * Thread safety: every call may be made from any thread; nuc_server_wait blocks
 * only the calling thread. nuc_server_destroy must not race other calls on the
 * same server.
 */
#ifndef NUCLEON_SERVER_H
#define NUCLEON_SERVER_H

#include "nucleon.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nuc_server_s* nuc_server;

typedef enum { NUC_EXEC_HIP = 0, NUC_EXEC_FAKE = 1 } nuc_executor_kind;

typedef struct {
    int executor;            /* nuc_executor_kind                                             */
    int device;              /* HIP device (NUC_EXEC_HIP)                                     */
    size_t hbm_budget;       /* cap on all server device memory; 0 = no cap                   */
    size_t job_arena;        /* bytes for admitted jobs' buffers; 0 = 4 GiB                   */
    size_t slot_workspace;   /* workspace of one slot; 0 = 16 GiB                             */
    int slots;               /* iterations in flight at once, 1..8; 0 = 2                     */
    int max_active;          /* admitted jobs at once, 1..4096; 0 = 64                        */
    double quantum_flops;    /* algorithmic flops one iteration aims at; 0 = 4e12             */
    int start_paused;        /* nonzero: schedule nothing until nuc_server_resume             */
    double fake_flops_per_s; /* NUC_EXEC_FAKE cost model; 0 = 5e13                            */
    double fake_fixed_s;     /* NUC_EXEC_FAKE cost of one iteration beyond its flops; 0 = 1e-4 */
} nuc_server_config;

/* One correlator job. HOST arrays are copied during nuc_server_submit. */
typedef struct {
    uint64_t conf_id;          /* a registered gauge configuration                       */
    int nvec;                  /* 3 <= nvec <= the configuration's nvec_max               */
    int nmom;                  /* 1..64                                                   */
    const int32_t* mom;        /* HOST [nmom][3], units of 2 pi / L                        */
    int nprof;                 /* 1..16                                                   */
    const nuc_profile* prof;   /* HOST [nprof]; NUC_PROF_EXPLICIT values are [T][nvec]    */
    int precision;             /* nuc_precision                                           */
} nuc_request;

typedef struct {
    int status;          /* nuc_status of the job                                        */
    double submit_s;     /* server clock at submission                                   */
    double admit_s;      /* ... when its buffers were reserved                            */
    double start_s;      /* ... when its first chunk was launched                         */
    double done_s;       /* ... when its result reached host memory                       */
    double flops;        /* algorithmic flops of the job (bench.py's convention)          */
    int iterations;      /* iterations the job took part in                               */
} nuc_job_info;

typedef struct {
    long long submitted, completed, failed, cancelled, iterations;
    int queued;                 /* submitted, not yet admitted                           */
    int active;                 /* admitted, not yet done                                */
    int max_outstanding;        /* peak of queued + active                               */
    double p50_ms, p99_ms;      /* latency percentiles (nearest rank) of completed jobs  */
    double mean_ms, max_ms;
    double window_s;            /* first submission to last completion                   */
    double jobs_per_s;          /* completed / window_s                                  */
    double flops_per_s;         /* algorithmic flops of completed jobs / window_s        */
    size_t bytes_resident;      /* registered configurations                             */
    size_t bytes_arena_used, bytes_arena_peak, bytes_arena;
    size_t bytes_total;         /* resident + arena + slot workspaces                    */
} nuc_server_metrics;

/* Create a server (and for NUC_EXEC_HIP its streams, arena and workspaces).
 * cfg may be NULL (all defaults). NUC_ERR_NOMEM if the arena and workspaces
 * exceed hbm_budget or cannot be allocated. */
nuc_status nuc_server_create(const nuc_server_config* cfg, nuc_server* out);

/* Cancel queued jobs, wait for iterations in flight, release everything.
 * NULL is ignored. */
nuc_status nuc_server_destroy(nuc_server srv);

/* Make a gauge configuration resident. geom->nvec is nvec_max, geom->t0 the
 * source timeslice of its perambulators. evecs: DEVICE c64 [T][nvec_max][L^3][3];
 * evals: HOST [T][nvec_max] (may be NULL if jobs use no NUC_PROF_GAUSS profile);
 * peramb: DEVICE c64 [T][4 nvec_max][4 nvec_max], tau(t, t0). The call waits for
 * all work on the device, then copies the data (the caller may free its buffers
 * after it returns); with NUC_EXEC_FAKE
 * only the geometry is kept and the pointers may be NULL. NUC_ERR_BUSY if conf_id
 * is already registered, NUC_ERR_NOMEM if it would exceed hbm_budget. */
nuc_status nuc_server_register(nuc_server srv, uint64_t conf_id, const nuc_geom* geom, const void* evecs,
                               const double* evals, const void* peramb);

/* Release a resident configuration. NUC_ERR_BUSY while a job that uses it is
 * queued or running. */
nuc_status nuc_server_unregister(nuc_server srv, uint64_t conf_id);

/* Queue a job; never waits for the device. *ticket identifies it. NUC_ERR_BUSY
 * if the job could never run under this server's limits (its buffers exceed the
 * arena, or one timeslice of it exceeds a slot workspace); NUC_ERR_INVALID for
 * bad arguments or an unknown conf_id. */
nuc_status nuc_server_submit(nuc_server srv, const nuc_request* req, uint64_t* ticket);

/* Wait up to timeout_ms (< 0: forever) for a job. On completion copy its result
 * to corr_host (HOST c128 [nmom][T][nprof][nprof], may be NULL), fill info (may
 * be NULL), retire the ticket and return the job's status (NUC_OK, or the error
 * that ended it, or NUC_ERR_CANCELLED). NUC_ERR_TIMEOUT if it is still running
 * (the ticket stays valid); NUC_ERR_INVALID for an unknown or retired ticket. */
nuc_status nuc_server_wait(nuc_server srv, uint64_t ticket, int timeout_ms, void* corr_host, nuc_job_info* info);

/* Cancel a job: a queued job ends at once, an admitted one gets no further
 * chunks and ends when its chunks in flight have. NUC_ERR_INVALID for an unknown
 * ticket; completed jobs are not affected. */
nuc_status nuc_server_cancel(nuc_server srv, uint64_t ticket);

/* Start scheduling on a server created with start_paused. */
nuc_status nuc_server_resume(nuc_server srv);

/* Counters and latency percentiles over all jobs completed so far. */
nuc_status nuc_server_stats(nuc_server srv, nuc_server_metrics* out);

/* Detail of the last failure on srv (or of nuc_server_create, with NULL). */
const char* nuc_server_last_error(nuc_server srv);

#ifdef __cplusplus
}
#endif

#endif /* NUCLEON_SERVER_H */

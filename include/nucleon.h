/*
 * nucleon.h - C ABI of the MI355X (gfx950) library for profiled-distillation
 * nucleon correlators.
 *
 * The library computes, on one GPU, the three steps of the nucleon part of the
 * paper's Section 2.1 ("Improved nucleon operators"):
 *   1. baryon elementals  Phi[p,t]_ijk = sum_x exp(-i p.x) eps_abc v_i^a v_j^b v_k^c
 *      built from the Laplacian eigenvectors v_i(t) (distillation vectors);
 *   2. the per-profile weighting of Section 2.1's only displayed equation,
 *      Phi^(a)_ijk = g_i^(a)[t] g_j^(a)[t] g_k^(a)[t] Phi_ijk (no sum over a,i,j,k),
 *      with profiles g that are functions of the Laplacian eigenvalues or of the
 *      distillation index;
 *   3. the N_B x N_B correlation matrix C_ab(t) that Section 2.1 feeds to its GEVP:
 *      profiled sink elementals Phi^(a)(t,p) contracted with profiled source
 *      elementals conj(Phi^(b)(t0,p)) through three spin-by-distillation
 *      perambulators tau(t,t0), direct minus u-quark exchange Wick term, nucleon
 *      spin structure (C gamma5)_{alpha beta} delta_{gamma sigma}, parity projector
 *      P+ = (1 + gamma4)/2 in the Dirac-Pauli basis.
 *
 * Conventions shared by every call
 *   - Complex numbers are interleaved {re, im}; "c64" is two floats, "c128" two doubles.
 *   - Arrays are dense and row-major with the shapes given per argument.
 *   - Pointers marked DEVICE are device (HBM) addresses owned by the caller
 *     (e.g. torch tensors); pointers marked HOST are host addresses owned by the
 *     caller and only read during the call. The library owns only its workspace.
 *   - Lattice sites are x = x0 + L*(x1 + L*x2) on an L^3 spatial lattice; momenta
 *     are integer triples n in units of 2*pi/L, with |n_d| < L.
 *   - Perambulator rows/columns are (spin * nvec + i): row = sink, column = source.
 *   - Calls that take a stream enqueue work on it (hipStream_t passed as void*,
 *     NULL = default stream) and return without waiting. NUC_OK means enqueued.
 *   - Argument checks are synchronous, host-side and happen before anything is
 *     enqueued; a failed check returns a negative status and leaves a message for
 *     nuc_last_error(). No call aborts the process or throws across the ABI.
 */
#ifndef NUCLEON_H
#define NUCLEON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nuc_ctx_s* nuc_ctx;

typedef enum {
    NUC_OK = 0,
    NUC_ERR_INVALID = -1,     /* bad argument (null pointer, size, range)          */
    NUC_ERR_NOMEM = -2,       /* workspace would exceed the context's HBM budget   */
    NUC_ERR_DEVICE = -3,      /* HIP runtime error (also latched for the next call) */
    NUC_ERR_UNSUPPORTED = -4, /* valid request this build does not implement        */
    NUC_ERR_BUSY = -5,        /* resource temporarily unavailable                   */
    NUC_ERR_INTERNAL = -6,
    NUC_ERR_TIMEOUT = -7,     /* a bounded wait ended before the work did           */
    NUC_ERR_CANCELLED = -8    /* the work was cancelled before it completed         */
} nuc_status;

/* Arithmetic of the elemental and contraction GEMMs. Cross-block site sums and the
 * final N^3 accumulation are FP64 in every mode; in the FP32 and split modes the
 * elementals and the first (k') step of the contraction are FP32 MFMA. */
typedef enum {
    NUC_FP32 = 0,   /* FP32 MFMA, FP32 accumulation inside a tile                   */
    NUC_BF16X3 = 1, /* perambulator chain with each FP32 operand split x = hi + lo in
                       bfloat16 (round to nearest even); products hi*hi + hi*lo +
                       lo*hi on bf16 MFMA with FP32 accumulation. For nvec <= 32,
                       and for nvec a multiple of 16 (>= 48) with an even storage
                       nvec; other nvec return NUC_ERR_UNSUPPORTED                 */
    NUC_FP16X3 = 2, /* the same split in IEEE half precision with power-of-two scales:
                       tau(t) per timeslice and X per contraction unit scaled so that
                       their largest |value| is near 2^14, the intermediate R by a
                       fixed power of two from its bound; 3 more mantissa bits than
                       bfloat16. Same nvec support as NUC_BF16X3                    */
    NUC_FP64 = 3    /* every GEMM (elementals, first step, chain) on FP64 MFMA over the
                       c64 data: a product of two FP32 values is exact in FP64, so
                       rounding happens only in FP64 accumulation and where the
                       intermediates X and phi are stored as c64. The form that holds
                       the relative error of C per block below 1e-6 on the
                       FP32-accumulated forms' worst blocks (the two Wick terms
                       cancelling); FP64 MFMA peaks at half the FP32 rate. Same nvec
                       support as NUC_BF16X3                                          */
} nuc_precision;

/* Distillation profile g_i[t] of Section 2.1 (a function of the Laplacian
 * eigenvalue lambda_i[t] or of the distillation index i). */
typedef enum {
    NUC_PROF_GAUSS = 0,    /* g_i[t] = exp(-lambda_i[t]^2 / (2 sigma^2)), sigma > 0 */
    NUC_PROF_LINEAR = 1,   /* g_i[t] = 1 - i / nvec (i zero-based)                 */
    NUC_PROF_ONE = 2,      /* g_i[t] = 1: standard (un-profiled) distillation       */
    NUC_PROF_EXPLICIT = 3  /* g_i[t] = values[t * nvec + i] (HOST, [T][nvec])       */
} nuc_prof_kind;

typedef struct {
    int L;     /* spatial extent: L^3 sites, L >= 1                              */
    int T;     /* number of timeslices, T >= 1                                     */
    int nvec;  /* distillation vectors per timeslice, 3 <= nvec <= 128             */
    int t0;    /* source timeslice, 0 <= t0 < T                                    */
} nuc_geom;

typedef struct {
    int kind;              /* nuc_prof_kind                                         */
    double sigma;          /* width for NUC_PROF_GAUSS                              */
    const double* values;  /* HOST [T][nvec] for NUC_PROF_EXPLICIT, else ignored    */
} nuc_profile;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`. hbm_budget_bytes caps the library's
 * own workspace (0 = no cap). *out receives the handle (NULL on failure). */
nuc_status nuc_create(nuc_ctx* out, int device, size_t hbm_budget_bytes);

/* Wait for the context's outstanding work, free its workspace and the handle.
 * NULL is accepted and ignored. */
nuc_status nuc_destroy(nuc_ctx ctx);

/* Static text for a status code. Never NULL. */
const char* nuc_status_string(nuc_status s);

/* Detail of the last failure on ctx; with ctx == NULL, of the last failure on
 * this thread (including failures of calls that had no valid context). */
const char* nuc_last_error(nuc_ctx ctx);

/* Version string of the library build. */
const char* nuc_version(void);

/* --------------------------------------------------------------- host-only */

/* Evaluate profiles on the host in FP64 (Section 2.1 profile functions).
 * evals: HOST [T][nvec] Laplacian eigenvalues (needed for NUC_PROF_GAUSS, may be
 * NULL otherwise); prof: HOST [nprof]; g_out: HOST [nprof][T][nvec]. */
nuc_status nuc_profiles_eval(const nuc_geom* geom, const double* evals, int nprof,
                             const nuc_profile* prof, double* g_out);

/* Bytes of library workspace nuc_run needs for this problem (elementals and
 * correlator together, phi supplied by the caller). Pure host computation. */
nuc_status nuc_workspace_query(const nuc_geom* geom, int nmom, int nprof,
                               nuc_precision prec, size_t* bytes);

/* ---------------------------------------------------------------- compute */

/* Baryon elementals of Section 2.1 for every timeslice and momentum:
 *   phi[t][p][i][j][k] = sum_x exp(-2 pi i n_p.x / L)
 *                        sum_abc eps_abc v_i^a(x,t) v_j^b(x,t) v_k^c(x,t).
 * evecs: DEVICE c64 [T][nvec][L^3][3] (colour innermost).
 * mom:   HOST int32 [nmom][3].
 * phi:   DEVICE c64 [T][nmom][nvec][nvec][nvec], fully written; exactly
 *        antisymmetric (one value per i<j<k, signed copies, zeros on repeated
 *        indices). The site sum is accumulated in FP32 within blocks of sites and
 *        in FP64 across blocks. */
nuc_status nuc_elementals(nuc_ctx ctx, const nuc_geom* geom, const void* evecs, int nmom,
                          const int32_t* mom, nuc_precision prec, void* phi, void* stream);

/* Nucleon correlation matrix of Section 2.1 for every sink time t and momentum:
 *   corr[p][t][a][b] = C_ab(t) = D_ab(t) - E_ab(t),
 *   D_ab(t) = sum_{sigma} sum A^(a)[sigma]_{IJK} tau_{II'} tau_{JJ'} tau_{KK'} B^(b)[sigma]_{I'J'K'},
 *   E_ab(t) = the same with tau_{IK'} tau_{JJ'} tau_{KI'} (u quarks exchanged),
 * A^(a)[sigma]_{(alpha i)(beta j)(gamma k)} = Phi^(a)(t,p)_ijk (C g5)_{alpha beta} delta_{gamma sigma},
 * B^(b)[sigma] = conj(Phi^(b)(t0,p)) conj(S), sigma summed over the P+ components {0,1},
 * tau = tau(t,t0). Profiles g^(a)[t] weight the sink, g^(b)[t0] the source.
 * phi:    DEVICE c64 [T][nmom][nvec][nvec][nvec] as produced by nuc_elementals
 *         (must be totally antisymmetric in (i,j,k); phi[t0] is the source).
 * evals:  HOST [T][nvec] (may be NULL if no profile is NUC_PROF_GAUSS).
 * prof:   HOST [nprof], 1 <= nprof <= 16.
 * peramb: DEVICE c64 [T][4 nvec][4 nvec], tau(t, t0) for every t.
 * corr:   DEVICE c128 [nmom][T][nprof][nprof]. The final sum over the N^3
 *         distillation indices is accumulated in FP64. */
nuc_status nuc_correlator(nuc_ctx ctx, const nuc_geom* geom, const void* phi,
                          const double* evals, int nprof, const nuc_profile* prof, int nmom,
                          const void* peramb, nuc_precision prec, void* corr, void* stream);

/* nuc_elementals followed by nuc_correlator. phi may be NULL, in which case the
 * elementals live in library workspace and are not returned. */
nuc_status nuc_run(nuc_ctx ctx, const nuc_geom* geom, const void* evecs, const double* evals,
                   int nprof, const nuc_profile* prof, int nmom, const int32_t* mom,
                   const void* peramb, nuc_precision prec, void* phi, void* corr, void* stream);

/* ---------------------------------------------------- no-allocation variant */

/* Size of the static device array behind nuc_correlator_noalloc. */
#define NUC_STATIC_SCRATCH_BYTES ((size_t)128 << 20)

/* nuc_correlator for callers that cannot allocate during the call: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc. Same
 * arguments, kernels and result (bitwise) as nuc_correlator; it calls no
 * allocating routine. Intermediates (X and the FP64 unit partials) live in a
 * file-scope device array of NUC_STATIC_SCRATCH_BYTES that each GPU the library
 * runs on holds from the first nuc_create on it until the process ends; the
 * launch constants go through the context's pinned staging buffer (1 MiB,
 * allocated by nuc_create). Sink timeslices are processed in rounds that fit the
 * array; NUC_ERR_NOMEM if one timeslice does not fit (its X takes
 * 64 nmom nprof Np^3 bytes, Np = nvec rounded up to 16: nvec <= 32 with 7 momenta
 * and 4 profiles fits, nvec = 64 with 3 momenta and 6 profiles does not).
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents (nothing in it needs to start at zero): calls that overlap on one GPU
 * -- from different contexts, or on streams not ordered with each other -- race
 * and give wrong results. Calls on one context are ordered by the context. */
nuc_status nuc_correlator_noalloc(nuc_ctx ctx, const nuc_geom* geom, const void* phi, const double* evals,
                                  int nprof, const nuc_profile* prof, int nmom, const void* peramb,
                                  nuc_precision prec, void* corr, void* stream);

/* ------------------------------------------------------ general spin tensors */

/* Spin structure of a three-quark operator over the rows sigma of an irrep:
 * S[sigma][alpha][beta][gamma] multiplies u_alpha^i d_beta^j u_gamma^k (i, j, k the
 * distillation indices of the elemental). The nucleon of nuc_correlator is
 * S[sigma] = (C gamma5)_{alpha beta} delta_{gamma sigma} for sigma in {0, 1} (P+); the
 * same diquark with sigma in {2, 3} is the P- projection, and moving-frame G1 rows
 * (Section 2.1's nonzero-momentum operators) or other diquarks are further choices. */
typedef struct {
    int nrow;            /* rows sigma, 1..4                                              */
    const double* snk;   /* HOST c128 [nrow][4][4][4]: the sink tensor S                  */
    const double* src;   /* HOST c128 [nrow][4][4][4]: S', the source operator uses conj(S') */
} nuc_spin;

/* The nucleon rows of nuc_spin for either parity projection (Section 2.1's nucleon
 * operators; at nonzero momentum the G1 basis holds both): S[r][alpha][beta][gamma] =
 * (C gamma5)_{alpha beta} delta_{gamma sigma_r}, C = gamma2 gamma4 in the Euclidean
 * Dirac-Pauli basis, sigma = (0, 1) for parity +1 (P+ = (1 + gamma4)/2) and (2, 3) for
 * parity -1 (P-). out: HOST c128 [2][4][4][4], fully written. Host only. */
nuc_status nuc_spin_nucleon(int parity, double* out);

/* Correlation matrix of profiled three-quark operators with general spin tensors:
 *   C_ab(t) = sum_sigma [D - E],  D = sum A_{IJK} tau_{II'} tau_{JJ'} tau_{KK'} B_{I'J'K'},
 *   E = the same with tau_{IK'} tau_{JJ'} tau_{KI'} (u quarks exchanged),
 *   A^(a)[sigma]_{(alpha i)(beta j)(gamma k)} = g_i g_j g_k Phi(t,p)_ijk S[sigma]_{alpha beta gamma},
 *   B^(b)[sigma]_{(alpha' i')(beta' j')(gamma' k')} = conj(g_i' g_j' g_k' Phi(t0,p)_i'j'k' S'[sigma]_{alpha' beta' gamma'}).
 * Arguments as nuc_correlator (phi need not be antisymmetric), plus spin (HOST).
 * FP32 MFMA tau products, FP64 sink sums. With the nucleon tensors it equals
 * nuc_correlator's result (a slower, general path). */
nuc_status nuc_correlator_spin(nuc_ctx ctx, const nuc_geom* geom, const void* phi, const double* evals, int nprof,
                               const nuc_profile* prof, int nmom, const void* peramb, const nuc_spin* spin, void* corr,
                               void* stream);

/* --------------------------------------------------------------- batching */

/* One correlator job: the arguments of nuc_run for one gauge configuration. */
typedef struct {
    nuc_geom geom;
    const void* evecs;          /* DEVICE c64 [T][nvec][L^3][3]                          */
    const double* evals;        /* HOST [T][nvec] (NULL if no profile is NUC_PROF_GAUSS)  */
    int nprof;                  /* 1..16                                                  */
    const nuc_profile* prof;    /* HOST [nprof]                                           */
    int nmom;                   /* 1..64                                                  */
    const int32_t* mom;         /* HOST [nmom][3]                                         */
    const void* peramb;         /* DEVICE c64 [T][4 nvec][4 nvec], tau(t, t0)             */
    void* phi;                  /* DEVICE c64 [T][nmom][nvec^3] or NULL (workspace)       */
    void* corr;                 /* DEVICE c128 [nmom][T][nprof][nprof]                    */
    int ld_nvec;                /* 0, or the nvec the inputs are stored with (>= nvec):
                                   evecs [T][ld][L^3][3] and peramb [T][4 ld][4 ld], of which
                                   the first nvec vectors / each block's first nvec rows and
                                   columns are used (distillation with fewer vectors)     */
} nuc_job;

/* Run many jobs (different lattices, nvec, momenta, profiles) together: every
 * stage is one launch per shape class over the work items of all jobs (the
 * perambulator-chain kernels are persistent, one workgroup per CU walking a
 * contiguous range of items). Pieces are packed into rounds that fit the
 * workspace. Each job's results equal those of nuc_run on that job alone
 * (same kernels, same per-job plan, fixed reduction order). HOST arrays are read
 * during the call only. */
nuc_status nuc_batch_run(nuc_ctx ctx, int njobs, const nuc_job* jobs, nuc_precision prec, void* stream);

/* Autotuner: time the tunable launch shapes of one job -- momenta (row tiles) per
 * wave of the elemental GEMM (1, 2 or 4) and the rows per workgroup of the first
 * contraction step (about 768, 1536 or 3072 workgroups) -- on that job, keep the
 * fastest for every later call on ctx whose job has the same shape (L, nvec,
 * ld_nvec, nmom, nprof, precision; any T), and write them to best[2] (HOST, may be
 * NULL). Results do not depend on these shapes. Blocks until the timing runs end;
 * the job's outputs are overwritten. */
nuc_status nuc_autotune(nuc_ctx ctx, const nuc_job* job, nuc_precision prec, void* stream, int* best);

typedef struct nuc_graph_s* nuc_graph;

/* Capture the work of nuc_batch_run(jobs) into a HIP graph that can be replayed
 * with nuc_graph_launch. The graph keeps its own copy of the host inputs and
 * refers to the device buffers of `jobs` and to the context workspace: while a
 * graph exists, calls that would need a larger workspace return NUC_ERR_BUSY. */
nuc_status nuc_batch_graph(nuc_ctx ctx, int njobs, const nuc_job* jobs, nuc_precision prec, nuc_graph* out);

/* Replay a captured batch on `stream` (ordered after the context's previous work). */
nuc_status nuc_graph_launch(nuc_graph g, void* stream);

/* Wait for the context's outstanding work and release the graph. NULL is ignored. */
nuc_status nuc_graph_destroy(nuc_graph g);

/* ----------------------------------------------------- analysis (host FP64) */

/* Generalised eigenvalue problem of Section 2.1's correlation matrix, in FP64 on
 * the host: for every t, C(t) v_n = lambda_n(t) C(t0) v_n, with each C(t)
 * Hermitised, (C + C^H) / 2, first. The eigenvectors combine the N_B profiled
 * operators into the optimised ones; their eigenvalues give effective masses.
 * corr:       HOST c128 [T][nb][nb], C_ab(t) of one momentum (a slice of nuc_run's output).
 * lambda_out: HOST [T][nb], eigenvalues in descending order per t.
 * vecs_out:   HOST c128 [T][nb][nb] or NULL; column n of block t is v_n(t), normalised
 *             to v^H C(t0) v = 1 (phase arbitrary).
 * 1 <= nb <= 64, 0 <= t0 < T. NUC_ERR_INVALID for bad arguments or if the Hermitised
 * C(t0) is not positive definite. */
nuc_status nuc_gevp(const void* corr, int T, int nb, int t0, double* lambda_out, void* vecs_out);

/* Effective masses m_n(t) = log(lambda_n(t) / lambda_n(t+1)), t = 0 .. T-2, from
 * nuc_gevp's eigenvalues (HOST [T][nb] in, HOST [T-1][nb] out; NaN where a ratio
 * is not positive). */
nuc_status nuc_effective_mass(const double* lambda, int T, int nb, double* meff_out);

/* ------------------------------------------- meson operators (charmonium study) */

/* Profiled single-meson operators qbar Gamma q of Section 3 ("Improved charmonium
 * operators"), built from distillation vectors, gauge-covariant derivatives and
 * bilinear profiles g_i g_j:
 *   (nabla_d f)(x) = 1/2 [U_d(x) f(x + d) - U_d(x - d)^H f(x - d)],  d = 0, 1, 2
 *     (periodic spatial lattice, U_d(x) the SU(3) link from x to x + d);
 *   B_i = eps_ijk nabla_j nabla_k:  B_0 = nabla_1 nabla_2 - nabla_2 nabla_1, and cyclic.
 * Meson elementals for D = (1, nabla_0, nabla_1, nabla_2, B_0, B_1, B_2), index 0..6:
 *   Phi^D[t][p]_ij = sum_x exp(-2 pi i n_p.x / L) v_i(x,t)^H (D v_j)(x,t).
 * Operators (Dirac-Pauli basis: gamma_k = [[0, -i sigma_k], [i sigma_k, 0]],
 * gamma_4 = diag(1,1,-1,-1) the time direction, gamma_5 = g1 g2 g3 g4):
 *   family 0: Gamma = g4 g5 with D = 1;   family 1: sum_k g4 g5 g_k (x) nabla_k;
 *   family 2: sum_k g_k (x) B_k;
 * each with the profile weight g_i^(a) g_j^(a); operator index A = family * nprof + a:
 *   M_A(t)[(alpha,i),(beta,j)] = sum_(Gamma,D) Gamma[alpha][beta] g_i g_j Phi^D_ij(t).
 * Correlation matrix (connected part, tau = tau(t, t0); the minus sign is the closed
 * quark loop's):
 *   C_AB(t) = -Tr[ M_A(t) tau Mbar_B(t0) g5 tau^H g5 ],   Mbar = g4 M^H g4.
 * Arithmetic: FP32 MFMA with FP64 sums across 64-term stretches of the site sum and
 * FP64 accumulation of the trace; nvec = N with 1 <= N <= 512. */

/* Meson elementals for every timeslice and momentum.
 * evecs: DEVICE c64 [T][nvec][L^3][3].
 * links: DEVICE c64 [T][L^3][3][3][3], U_d(x,t)[a][b] at [t][x][d][a][b].
 * mom:   HOST int32 [nmom][3] (|n_d| < L), 1 <= nmom <= 64.
 * phi:   DEVICE c64 [T][nmom][7][nvec][nvec], fully written. */
nuc_status nuc_meson_elementals(nuc_ctx ctx, const nuc_geom* geom, const void* evecs, const void* links, int nmom,
                                const int32_t* mom, void* phi, void* stream);

/* Meson correlation matrix of the 3 nprof profiled operators for every sink time t.
 * phi:    DEVICE c64 [T][nmom][7][nvec][nvec] from nuc_meson_elementals (phi[t0] is the source).
 * evals:  HOST [T][nvec] (may be NULL if no profile is NUC_PROF_GAUSS).
 * prof:   HOST [nprof], 1 <= nprof <= 16; sink profiles at t, source profiles at t0.
 * peramb: DEVICE c64 [T][4 nvec][4 nvec], tau(t, t0), rows/columns spin * nvec + i.
 * corr:   DEVICE c128 [nmom][T][3 nprof][3 nprof]. */
nuc_status nuc_meson_correlator(nuc_ctx ctx, const nuc_geom* geom, const void* phi, const double* evals, int nprof,
                                const nuc_profile* prof, int nmom, const void* peramb, void* corr, void* stream);

/* nuc_meson_elementals followed by nuc_meson_correlator. phi may be NULL (the
 * elementals then live in library workspace and are not returned). */
nuc_status nuc_meson_run(nuc_ctx ctx, const nuc_geom* geom, const void* evecs, const void* links,
                         const double* evals, int nprof, const nuc_profile* prof, int nmom, const int32_t* mom,
                         const void* peramb, void* phi, void* corr, void* stream);

/* Pruning of a correlation matrix before its GEVP (Section 3): the m left singular
 * vectors U_m of C(t_p) with the largest singular values (eigenvectors of
 * C(t_p) C(t_p)^H in FP64 on the host) project every C(t) to U_m^H C(t) U_m.
 * corr:  HOST c128 [T][n][n];  out: HOST c128 [T][m][m];  basis: HOST c128 [n][m] or
 * NULL. Each basis column is scaled so that its largest-modulus component (the first
 * one on ties) is real and positive. 1 <= m <= n <= 64, 0 <= t_p < T. */
nuc_status nuc_svd_prune(const void* corr, int T, int n, int t_p, int m, void* out, void* basis);

/* ------------------------------------------- two-meson operators (Section 3) */

/* The I=2 A1++ two-meson correlator of the charmonium study, built from an optimal
 * one-meson operator at zero total momentum and back-to-back momenta:
 *   M_w(t, p) = sum_A w_A M_A(t, p)   (M_A the profiled operators of nuc_meson_correlator;
 *     for a GEVP eigenvector v of C(t) v = lambda C(t0) v use w = conj(v), after SVD
 *     pruning with basis U_m w = conj(U_m v));
 *   O(t) = sum_k pi+(p_k, t) pi+(-p_k, t),  pi+(p, t) = dbar M_w(t, p) u;
 *   P_kl(t) = M_w(t, p_k) tau Mbar_w(t0, p_l) g5 tau^H g5,  Mbar = g4 M^H g4;
 *   C(t) = <O(t) O(t0)^H> = D - X,
 *   D = 2 sum_{k,l} Tr P_kl Tr P_kbar,lbar   (direct: two closed quark loops),
 *   X = 2 sum_{k,l} Tr[P_kl P_kbar,lbar]     (crossed: one loop),
 * kbar the index of -p_k in the list.
 * phi:     DEVICE c64 [T][nmom][7][nvec][nvec] from nuc_meson_elementals at these momenta.
 * evals, nprof, prof: as nuc_meson_correlator (sink profiles at t, source at t0).
 * weights: HOST c128 [3 nprof], the coefficients w_A (A = family * nprof + a).
 * mom:     HOST int32 [nmom][3], 1 <= nmom <= 48, distinct, closed under negation
 *          (the star of a momentum; a single zero momentum is the threshold operator).
 * peramb:  DEVICE c64 [T][4 nvec][4 nvec], tau(t, t0).
 * corr:    DEVICE c128 [T][3]: (C, D, X) for every sink time t.
 * FP32 MFMA products (tau, the operators and the two-meson products), FP64 traces and
 * sums. Library workspace holds the operators and products of a block of timeslices. */
/* Coefficients of the optimal one-meson operator from a GEVP eigenvector v of the
 * (pruned) correlation matrix (Section 3): w = conj(v), or with the pruning basis U_m of
 * nuc_svd_prune w = conj(U_m v), so that v^H C v is the correlator of sum_A w_A O_A.
 * vec: HOST c128 [m]; basis: HOST c128 [n][m] or NULL; w_out: HOST c128 [n] (or [m]
 * without a basis). 1 <= m <= n <= 64. Host only. */
nuc_status nuc_twomeson_weights(const void* vec, int m, const void* basis, int n, void* w_out);

nuc_status nuc_twomeson_correlator(nuc_ctx ctx, const nuc_geom* geom, const void* phi, const double* evals,
                                   int nprof, const nuc_profile* prof, const double* weights, int nmom,
                                   const int32_t* mom, const void* peramb, void* corr, void* stream);

/* ------------------------------------------- glueball operators (Section 3) */

/* The five A1^{-+} glueball operators of Section 3 ("Improved glueball operators")
 * per timeslice of many gauge configurations, built from the chromo-magnetic field
 * B_i = eps_ijk F_jk (clover F, made anti-Hermitian and traceless:
 * F_mn = (Q_mn - Q_mn^H)/8 minus its trace, Q_mn the sum of the four plaquette leaves
 * at x in the (m, n) plane, each oriented m then n) and the adjoint gauge-covariant
 * symmetric difference (D_j X)(x) = 1/2 [U_j(x) X(x+j) U_j(x)^H - U_j(x-j)^H X(x-j) U_j(x-j)]:
 *   O1 = sum_x Tr(eps_ijk B_i D_j B_k)        O2 = sum_x Tr(eps_ijk eps_ilm B_j B_k D_l B_m)
 *   O3 = sum_x Tr(eps_ijk B_i D_j^3 B_k)      O4 = sum_x Tr(eps_ijk B_i D_j^2 D_k B_j)
 *   O5 = sum_x Tr(eps_ijk B_i D_j D_i^2 B_k)  (repeated indices summed, D acting right to left).
 * links: DEVICE c64 [nconf][T][L^3][3][3][3], U_d(x,t)[a][b] (spatial directions d = 0..2),
 *        SU(3): only the first two rows are read, the third is taken as the complex
 *        conjugate of their cross product.
 * ops:   DEVICE c128 [nconf][T][5]. FP32 fields (each stored as the 8 reals of a traceless
 *        anti-Hermitian matrix), FP64 site sums. 2 <= L <= 256. */
nuc_status nuc_glueball_operators(nuc_ctx ctx, int L, int T, int nconf, const void* links, void* ops, void* stream);

/* Correlation matrix of one configuration's operators, time-averaged with the vacuum
 * part removed (host FP64):
 *   C_nm(dt) = 1/T sum_t O_n(t+dt) conj(O_m(t)) - Obar_n conj(Obar_m),  Obar = 1/T sum_t O(t),
 * t + dt taken modulo T. ops: HOST c128 [T][nop]; corr: HOST c128 [T][nop][nop]. */
nuc_status nuc_glueball_correlator(const void* ops, int T, int nop, void* corr);

/* ---------------------------------------------------------- instrumentation */

/* Kernels of the library, for per-kernel timing. */
typedef enum {
    NUC_K_ELEMENTALS = 0,   /* cross-product MFMA GEMM over sites (FP64 split partials) */
    NUC_K_ELEM_EXPAND = 1,  /* FP64 split reduction + antisymmetric expansion to dense  */
    NUC_K_CORR_STEP1 = 2,   /* source elemental times tau on the third index            */
    NUC_K_CORR_CHAIN = 3,   /* per-k tau sandwiches and FP64 sink dot                  */
    NUC_K_CORR_REDUCE = 4,  /* FP64 sum over k and sigma into C_ab(t)                   */
    NUC_K_CORR_SCALE = 5,   /* split forms: FP16x3 power-of-two scales, BF16x3 tau planes */
    NUC_K_MESON_DERIV = 6,  /* meson: covariant derivatives nabla_k v and B_k v         */
    NUC_K_MESON_ELEM = 7,   /* meson: elemental GEMM over sites (FP64 split partials)   */
    NUC_K_MESON_ELEM_REDUCE = 8, /* meson: FP64 split sum into Phi^D                     */
    NUC_K_MESON_GEMM = 9,   /* meson: spin-sparse operator products M tau, tau M        */
    NUC_K_MESON_TRACE = 10, /* meson: FP64 traces C_AB                                  */
    NUC_K_MESON_SUM = 11,   /* meson: FP64 sum of trace partials                        */
    NUC_K_MESON_WEIGHT = 12, /* meson: profile-weighted elementals g_i g_j Phi^D         */
    NUC_K_MESON_PHASE = 13, /* meson: phase-weighted conjugate vectors (GEMM operands)  */
    NUC_K_GLUE_STENCIL = 14, /* glueball: link layout, clover B_i, adjoint differences   */
    NUC_K_GLUE_CONTRACT = 15, /* glueball: operator densities and FP64 site sums         */
    NUC_K_SPIN_SOURCE = 16, /* general spin: folded dense source tensors                */
    NUC_K_SPIN_GEMM = 17,   /* general spin: the three tau products (complex GEMMs)     */
    NUC_K_SPIN_SINK = 18,   /* general spin: FP64 sink dots and their sum               */
    NUC_K_TM_OPERATOR = 19, /* two-meson: optimal operators M_w and Mbar_w               */
    NUC_K_TM_GEMM = 20,     /* two-meson: g5 tau^H g5, L = M tau, R = Mbar g5 tau^H g5   */
    NUC_K_TM_PAIR = 21,     /* two-meson: paired products and their traces               */
    NUC_K_TM_SUM = 22,      /* two-meson: FP64 sum into (C, D, X)                        */
    NUC_K_COUNT = 23
} nuc_kernel_id;

/* Enable (on != 0) or disable per-kernel timing on ctx. While enabled, every
 * kernel launch of ctx is bracketed by HIP events recorded on the launch stream.
 * Enabling clears the accumulated figures. */
nuc_status nuc_timing_enable(nuc_ctx ctx, int on);

/* Wait for the timed launches and return, per nuc_kernel_id, the summed kernel
 * milliseconds (ms[NUC_K_COUNT], HOST) and launch counts (launches[NUC_K_COUNT],
 * HOST) since timing was enabled or last read; then clear them. */
nuc_status nuc_timing_read(nuc_ctx ctx, double* ms, int* launches);

/* Static name of a kernel id ("?" if out of range). */
const char* nuc_kernel_name(int id);

#ifdef __cplusplus
}
#endif

#endif /* NUCLEON_H */

/*
 * FP64 CPU oracle for profiled-distillation nucleon correlators.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load this file's library. The HIP library never links,
 * includes or calls it, and it includes nothing from the HIP library.
 *
 * Plain loops in double precision (C99 double _Complex), written from the
 * definitions of the paper's Section 2.1 ("Improved nucleon operators") and the
 * standard distillation construction it builds on:
 *
 *   elemental   Phi[p,t]_ijk = sum_x exp(-i p.x) eps_abc v_i^a(x,t) v_j^b(x,t) v_k^c(x,t)
 *   profiled    Phi^(a)[p,t]_ijk = g_i^(a)[t] g_j^(a)[t] g_k^(a)[t] Phi[p,t]_ijk   (no sums)
 *   correlator  C_ab(t) = D_ab(t) - E_ab(t), the N_B x N_B matrix of Section 2.1,
 *               contracting profiled sink and source elementals through three
 *               perambulators tau(t,t0), direct (D) and u-quark exchange (E) terms.
 *
 * Readings where the paper is silent (it omits spin, see the remark after the
 * profile equation of Section 2.1):
 *   - Euclidean Dirac-Pauli gammas, C = gamma2 gamma4, nucleon spin structure
 *     (C gamma5)_{alpha beta} delta_{gamma sigma}, parity projector P+ = (1+gamma4)/2,
 *     so sigma = sigma' in {0,1}.
 *   - sink uses Phi^(a)(t,p), source uses conj(Phi^(b)(t0,p)) with conj(S).
 *   - momenta are integers n in units of 2 pi / L, site x = x0 + L (x1 + L x2).
 *   - profiles: Gaussian g_i = exp(-lambda_i^2 / (2 sigma^2)); linear g_i = 1 - i/N.
 *
 * Parity status: pinned (brute force, closed forms and invariants in the test suite).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double _Complex cplx;

#define ORACLE_OK 0
#define ORACLE_EINVAL -1
#define ORACLE_ENOMEM -2

/* (C gamma5) in the Dirac-Pauli basis: real, antisymmetric, four nonzeros. */
static const double CG5[4][4] = {
    {0.0, -1.0, 0.0, 0.0},
    {1.0, 0.0, 0.0, 0.0},
    {0.0, 0.0, 0.0, -1.0},
    {0.0, 0.0, 1.0, 0.0},
};

void oracle_cg5(double* out16) {
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) out16[a * 4 + b] = CG5[a][b];
}

/* ------------------------------------------------------------------ profiles */
/* Distillation profiles (Section 2.1: functions of the Laplacian eigenvalues or
 * of the distillation index). kind 0: exp(-lambda^2/(2 sigma^2)); kind 1: 1 - i/N;
 * kind 2: 1 (standard distillation, no profile).
 * g is [nprof][T][N]. */
int oracle_profiles(int T, int N, const double* evals, int nprof, const int* kind,
                    const double* sigma, double* g) {
    if (T <= 0 || N <= 0 || nprof <= 0) return ORACLE_EINVAL;
    for (int a = 0; a < nprof; ++a) {
        for (int t = 0; t < T; ++t) {
            for (int i = 0; i < N; ++i) {
                double v;
                if (kind[a] == 0) {
                    double lam = evals[(size_t)t * N + i];
                    v = exp(-(lam * lam) / (2.0 * sigma[a] * sigma[a]));
                } else if (kind[a] == 1) {
                    v = 1.0 - (double)i / (double)N;
                } else if (kind[a] == 2) {
                    v = 1.0;
                } else {
                    return ORACLE_EINVAL;
                }
                g[((size_t)a * T + t) * N + i] = v;
            }
        }
    }
    return ORACLE_OK;
}

/* ---------------------------------------------------------------- elementals */
/* exp(-i 2 pi (n . x) / L) at site x = x0 + L (x1 + L x2). */
static cplx site_phase(int L, const int* n, int x) {
    int x0 = x % L, x1 = (x / L) % L, x2 = x / (L * L);
    long m = (long)n[0] * x0 + (long)n[1] * x1 + (long)n[2] * x2;
    m %= L;
    if (m < 0) m += L;
    double ang = 2.0 * M_PI * (double)m / (double)L;
    return cos(ang) - I * sin(ang);
}

/* eps_abc u^a v^b w^c summed over the six permutations of (0,1,2). */
static cplx eps_contract(const cplx* u, const cplx* v, const cplx* w) {
    return u[0] * v[1] * w[2] - u[0] * v[2] * w[1] + u[1] * v[2] * w[0]
         - u[1] * v[0] * w[2] + u[2] * v[0] * w[1] - u[2] * v[1] * w[0];
}

/* Phi[t][p][i][j][k] for the nt timeslices given.
 * evecs: [nt][N][V3][3]; mom: [nmom][3]; phi: [nt][nmom][N][N][N].
 * For each i<j<k the site sum runs in increasing x; the other five orderings
 * take the same value with the sign of the permutation (eps is totally
 * antisymmetric), and entries with a repeated index are zero. */
int oracle_elementals(int L, int N, int nt, const cplx* evecs, int nmom, const int* mom,
                      cplx* phi) {
    if (L <= 0 || N <= 0 || nt <= 0 || nmom <= 0) return ORACLE_EINVAL;
    const int V3 = L * L * L;
    const size_t N3 = (size_t)N * N * N;
    int nunit = nt * nmom;
#pragma omp parallel for schedule(dynamic, 1)
    for (int u = 0; u < nunit; ++u) {
        int t = u / nmom, p = u % nmom;
        const cplx* v = evecs + (size_t)t * N * V3 * 3;
        cplx* out = phi + ((size_t)t * nmom + p) * N3;
        memset(out, 0, N3 * sizeof(cplx));
        for (int i = 0; i < N; ++i)
            for (int j = i + 1; j < N; ++j)
                for (int k = j + 1; k < N; ++k) {
                    cplx acc = 0.0;
                    for (int x = 0; x < V3; ++x) {
                        cplx ph = site_phase(L, mom + 3 * p, x);
                        acc += ph * eps_contract(v + ((size_t)i * V3 + x) * 3,
                                                 v + ((size_t)j * V3 + x) * 3,
                                                 v + ((size_t)k * V3 + x) * 3);
                    }
#define PHI(a, b, c) out[((size_t)(a) * N + (b)) * N + (c)]
                    PHI(i, j, k) = acc;
                    PHI(j, k, i) = acc;
                    PHI(k, i, j) = acc;
                    PHI(j, i, k) = -acc;
                    PHI(i, k, j) = -acc;
                    PHI(k, j, i) = -acc;
#undef PHI
                }
    }
    return ORACLE_OK;
}

/* Selected elemental entries: phi_out[n] = Phi[p_n]_{i_n j_n k_n} for one timeslice,
 * the same site sum as above for arbitrary (i,j,k) (zero if two indices coincide).
 * evecs: [N][V3][3] of that timeslice; idx: [count][4] = (p, i, j, k). */
int oracle_elemental_entries(int L, int N, const cplx* evecs, const int* mom, int count,
                             const int* idx, cplx* out) {
    if (L <= 0 || N <= 0 || count < 0) return ORACLE_EINVAL;
    const int V3 = L * L * L;
#pragma omp parallel for schedule(dynamic, 1)
    for (int n = 0; n < count; ++n) {
        const int p = idx[4 * n], i = idx[4 * n + 1], j = idx[4 * n + 2], k = idx[4 * n + 3];
        cplx acc = 0.0;
        if (i != j && j != k && i != k) {
            for (int x = 0; x < V3; ++x)
                acc += site_phase(L, mom + 3 * p, x) *
                       eps_contract(evecs + ((size_t)i * V3 + x) * 3, evecs + ((size_t)j * V3 + x) * 3,
                                    evecs + ((size_t)k * V3 + x) * 3);
        }
        out[n] = acc;
    }
    return ORACLE_OK;
}

/* --------------------------------------------------------------- correlator */
/* One perambulator contraction with a general real source spin tensor w[a'][b'][c'],
 * evaluated only on the sink spin blocks the nucleon sink touches:
 *
 *   Z_(a b)[i][j][k] = sum_{a'b'c'} w[a'][b'][c'] sum_{i'j'k'}
 *        tau[aN+i][a'N+i'] tau[bN+j][b'N+j'] tau[sN+k][c'N+k'] src[i'][j'][k']
 *
 * for the four sink pairs (a,b) with (C gamma5)_{ab} != 0 and sink spin c = s.
 * The three tau factors are applied one index at a time (k, then j, then i).
 * For each of the nsnk sink tensors snk[n] ([N][N][N]) it adds
 *   sum_{(a,b)} (C gamma5)_{ab} sum_{ijk} snk[n][i][j][k] Z_(ab)[i][j][k]
 * to out[n]. */
static void contract_one(int N, const cplx* tau, int s, const double w[4][4][4],
                         const cplx* src, int nsnk, const cplx* snk, cplx* out,
                         cplx* X, cplx* Y, cplx* Z) {
    const int N4 = 4 * N;
    const size_t N3 = (size_t)N * N * N;
#define TAU(r, c) tau[(size_t)(r) * N4 + (c)]
    int cused[4] = {0, 0, 0, 0};
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
            for (int c = 0; c < 4; ++c)
                if (w[a][b][c] != 0.0) cused[c] = 1;
    /* index k' -> k (sink spin s) */
    for (int c = 0; c < 4; ++c) {
        if (!cused[c]) continue;
        cplx* Xc = X + (size_t)c * N3;
#pragma omp parallel for
        for (int ip = 0; ip < N; ++ip)
            for (int jp = 0; jp < N; ++jp)
                for (int k = 0; k < N; ++k) {
                    cplx acc = 0.0;
                    for (int kp = 0; kp < N; ++kp)
                        acc += TAU(s * N + k, c * N + kp) * src[((size_t)ip * N + jp) * N + kp];
                    Xc[((size_t)ip * N + jp) * N + k] = acc;
                }
    }
    /* index j' -> j, all four sink spins b; source spins (b', c') summed with w.
     * For each (i', j) the k values are carried side by side (k innermost, so the
     * rows of X are read in order); each entry is still summed over j' in order,
     * then over (b', c') in order. */
    for (int ap = 0; ap < 4; ++ap)
        for (int b = 0; b < 4; ++b) {
            cplx* Yab = Y + ((size_t)ap * 4 + b) * N3;
#pragma omp parallel for
            for (int ip = 0; ip < N; ++ip) {
                cplx acc[N], part[N];
                for (int j = 0; j < N; ++j) {
                    for (int k = 0; k < N; ++k) acc[k] = 0.0;
                    for (int bp = 0; bp < 4; ++bp)
                        for (int c = 0; c < 4; ++c) {
                            if (w[ap][bp][c] == 0.0) continue;
                            const cplx* Xc = X + (size_t)c * N3;
                            for (int k = 0; k < N; ++k) part[k] = 0.0;
                            for (int jp = 0; jp < N; ++jp) {
                                const cplx t = TAU(b * N + j, bp * N + jp);
                                const cplx* xr = Xc + ((size_t)ip * N + jp) * N;
                                for (int k = 0; k < N; ++k) part[k] += t * xr[k];
                            }
                            for (int k = 0; k < N; ++k) acc[k] += w[ap][bp][c] * part[k];
                        }
                    for (int k = 0; k < N; ++k) Yab[((size_t)ip * N + j) * N + k] = acc[k];
                }
            }
        }
    /* index i' -> i for the sink pairs, then the sink dots */
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            if (CG5[a][b] == 0.0) continue;
#pragma omp parallel for
            for (int i = 0; i < N; ++i) {
                cplx acc[N];
                for (int j = 0; j < N; ++j) {
                    /* k innermost as above; each entry summed over a', then i', in order */
                    for (int k = 0; k < N; ++k) acc[k] = 0.0;
                    for (int ap = 0; ap < 4; ++ap) {
                        const cplx* Yab = Y + ((size_t)ap * 4 + b) * N3;
                        for (int ip = 0; ip < N; ++ip) {
                            const cplx t = TAU(a * N + i, ap * N + ip);
                            const cplx* yr = Yab + ((size_t)ip * N + j) * N;
                            for (int k = 0; k < N; ++k) acc[k] += t * yr[k];
                        }
                    }
                    for (int k = 0; k < N; ++k) Z[((size_t)i * N + j) * N + k] = acc[k];
                }
            }
            for (int n = 0; n < nsnk; ++n) {
                const cplx* sn = snk + (size_t)n * N3;
                cplx dot = 0.0;
                for (size_t q = 0; q < N3; ++q) dot += sn[q] * Z[q];
                out[n] += CG5[a][b] * dot;
            }
        }
#undef TAU
}

/* C_ab(t) = D_ab(t) - E_ab(t) for every (t, p) of the nt sink times given.
 *   phi_snk [nt][nmom][N][N][N]  elementals at the sink times
 *   phi_src [nmom][N][N][N]      elementals at the source time t0
 *   tau     [nt][4N][4N]         tau(t, t0), row = sink (spin*N + i), column = source
 *   g_snk   [nprof][nt][N]       profiles at the sink times
 *   g_src   [nprof][N]           profiles at t0
 *   corr    [nmom][nt][nprof][nprof]; dterm, eterm (same shape) may be NULL.
 * Direct term: source spin tensor (C gamma5)_{a'b'} delta_{c' s}.
 * Exchange term: the two u quarks (slots 1 and 3) swapped at the source, i.e.
 * the source tensor with (i',a') and (k',c') exchanged; built explicitly. */
int oracle_correlator(int N, int nt, int nmom, int nprof, const cplx* phi_snk,
                      const cplx* phi_src, const cplx* tau, const double* g_snk,
                      const double* g_src, cplx* corr, cplx* dterm, cplx* eterm) {
    if (N <= 0 || nt <= 0 || nmom <= 0 || nprof <= 0) return ORACLE_EINVAL;
    const size_t N3 = (size_t)N * N * N;
    const int N4 = 4 * N;
    cplx* X = malloc(4 * N3 * sizeof(cplx));
    cplx* Y = malloc(16 * N3 * sizeof(cplx));
    cplx* Z = malloc(N3 * sizeof(cplx));
    cplx* A = malloc((size_t)nprof * N3 * sizeof(cplx));
    cplx* B = malloc(N3 * sizeof(cplx));
    cplx* BX = malloc(N3 * sizeof(cplx));
    cplx* dsum = malloc((size_t)nprof * sizeof(cplx));
    cplx* esum = malloc((size_t)nprof * sizeof(cplx));
    if (!X || !Y || !Z || !A || !B || !BX || !dsum || !esum) {
        free(X); free(Y); free(Z); free(A); free(B); free(BX); free(dsum); free(esum);
        return ORACLE_ENOMEM;
    }
    for (int t = 0; t < nt; ++t)
        for (int p = 0; p < nmom; ++p) {
            const cplx* ph_t = phi_snk + ((size_t)t * nmom + p) * N3;
            const cplx* ph_0 = phi_src + (size_t)p * N3;
            const cplx* tau_t = tau + (size_t)t * N4 * N4;
            /* profiled sinks Phi^(a)(t,p) */
            for (int a = 0; a < nprof; ++a) {
                const double* ga = g_snk + ((size_t)a * nt + t) * N;
                for (int i = 0; i < N; ++i)
                    for (int j = 0; j < N; ++j)
                        for (int k = 0; k < N; ++k) {
                            size_t q = ((size_t)i * N + j) * N + k;
                            A[(size_t)a * N3 + q] = ga[i] * ga[j] * ga[k] * ph_t[q];
                        }
            }
            for (int b = 0; b < nprof; ++b) {
                const double* gb = g_src + (size_t)b * N;
                /* profiled source conj(Phi^(b)(t0,p)) */
                for (int i = 0; i < N; ++i)
                    for (int j = 0; j < N; ++j)
                        for (int k = 0; k < N; ++k) {
                            size_t q = ((size_t)i * N + j) * N + k;
                            B[q] = conj(gb[i] * gb[j] * gb[k] * ph_0[q]);
                        }
                /* exchange source: BX[i'][j'][k'] = B[k'][j'][i'] */
                for (int i = 0; i < N; ++i)
                    for (int j = 0; j < N; ++j)
                        for (int k = 0; k < N; ++k)
                            BX[((size_t)i * N + j) * N + k] = B[((size_t)k * N + j) * N + i];
                for (int a = 0; a < nprof; ++a) dsum[a] = esum[a] = 0.0;
                for (int s = 0; s < 2; ++s) { /* P+ = diag(1,1,0,0): sigma = sigma' in {0,1} */
                    double wd[4][4][4], we[4][4][4];
                    memset(wd, 0, sizeof wd);
                    memset(we, 0, sizeof we);
                    for (int x = 0; x < 4; ++x)
                        for (int y = 0; y < 4; ++y) {
                            wd[x][y][s] = CG5[x][y]; /* S_{a'b'c'} = Cg5_{a'b'} delta_{c's} */
                            we[s][y][x] = CG5[x][y]; /* S_{c'b'a'}: a' = s, (c',b') a Cg5 pair */
                        }
                    contract_one(N, tau_t, s, wd, B, nprof, A, dsum, X, Y, Z);
                    contract_one(N, tau_t, s, we, BX, nprof, A, esum, X, Y, Z);
                }
                for (int a = 0; a < nprof; ++a) {
                    size_t o = (((size_t)p * nt + t) * nprof + a) * nprof + b;
                    corr[o] = dsum[a] - esum[a];
                    if (dterm) dterm[o] = dsum[a];
                    if (eterm) eterm[o] = esum[a];
                }
            }
        }
    free(X); free(Y); free(Z); free(A); free(B); free(BX); free(dsum); free(esum);
    return ORACLE_OK;
}

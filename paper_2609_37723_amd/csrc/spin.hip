// Nucleon-type correlation matrices with general spin tensors on gfx950: the sink
// operator A^(a)[s]_{(alpha i)(beta j)(gamma k)} = g_i g_j g_k Phi(t,p)_ijk S[s]_{alpha beta gamma}
// and the source B^(b)[s] = conj(g g g Phi(t0,p) S'[s]) over the rows s of an irrep
// (moving-frame G1 operators, other parity projections, other three-quark spin
// structures), C_ab(t) = sum_s D - E with D and E the direct and u-quark exchange terms
// of the perambulator contraction (the paper's Section 2.1 correlator, generalised).
//
// Method. The exchange term is the direct term of the source with its first and third
// (spin, index) slots swapped, so C = sum_s A (tau (x) tau (x) tau) Bt with
// Bt = B - B^{T13}, built densely ((4N)^3 per (p, b, s)) once per call. Per timeslice
// the three tau products are FP32 MFMA complex GEMMs with uniform batch strides:
//   Y1 = tau Bt               ([4N] x [4N] times [4N] x [16N^2])
//   Y2[I] = tau Y1[I]         (batched over I, [4N] x [4N] times [4N] x [4N])
//   Y3 = Y2 tau^T             ([16N^2] x [4N] times [4N] x [4N])
// and the sink dot sum_{(alpha beta gamma) nonzero} S sum_ijk g g g Phi Y3 runs in FP64
// for every sink profile at once.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <complex>
#include <vector>

#include "../../include/nucleon.h"
#include "nuc_internal.h"
#include "cgemm.h"
#include "meson_spin.h"
#include "runtime_internal.h"

namespace nuc {
namespace spin {

constexpr size_t kSpinCap = (size_t)16 << 30;
constexpr int kMaxRow = 4;

// ------------------------------------------------------------ batched complex GEMM

// C[b] = A[b] B[b], row-major, complex, FP32; A [M][K] (lda), B [K][N] (ldb), C [M][N] (ldc),
// batch b at A + ((b / dA) % mA) sA, B + ((b / dB) % mB) sB, C + b sC.
struct CGemm {
    const float2* A;
    const float2* B;
    float2* C;
    int M, N, K, lda, ldb, ldc;
    long long sA, sB, sC;
    int tiles_m, tiles_n;
    int dA, mA, dB, mB;
};

constexpr int SKC = 32;   // complex K per LDS stage
constexpr int SAP = SKC + 2;  // A tile [64][SKC] pitch
constexpr int SBP = 80;   // B tile [SKC][64] pitch
constexpr int kAQ = SKC / 4;    // A tile elements per thread (256 threads): rows ar + kAS q
constexpr int kAS = 256 / SKC;
constexpr int kBQ = SKC / 8;    // B tile K rows per thread (two columns each): rows bk + 8 q

// MFMAs of one staged K block for a wave's 32 x 32 quadrant, complex products in Gauss's
// three-multiplication form: t1 = sum ar br, t2 = sum ai bi, t3 = sum (ar + ai)(br + bi),
// the product being (t1 - t2) + i (t3 - t1 - t2).
template <bool GUARD>
__device__ __forceinline__ void cgemm_stage(const float2* As, const float2* Bs, int wm, int wn, int lr, int lk, bool m1,
                                            bool n1, floatx4 (&t1)[2][2], floatx4 (&t2)[2][2], floatx4 (&t3)[2][2]) {
    float2 av[SKC / 4][2], bv[SKC / 4][2];
#pragma unroll
    for (int ks = 0; ks < SKC / 4; ++ks) {
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) av[ks][mb] = As[(wm + 16 * mb + lr) * SAP + 4 * ks + lk];
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) bv[ks][nb] = Bs[(4 * ks + lk) * SBP + wn + 16 * nb + lr];
    }
#pragma unroll
    for (int ks = 0; ks < SKC / 4; ++ks)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                if (GUARD && ((mb == 1 && !m1) || (nb == 1 && !n1))) continue;
                t1[mb][nb] = mfma16x4(av[ks][mb].x, bv[ks][nb].x, t1[mb][nb]);
                t2[mb][nb] = mfma16x4(av[ks][mb].y, bv[ks][nb].y, t2[mb][nb]);
                t3[mb][nb] = mfma16x4(av[ks][mb].x + av[ks][mb].y, bv[ks][nb].x + bv[ks][nb].y, t3[mb][nb]);
            }
}

__global__ __launch_bounds__(256, 2) void spin_cgemm_kernel(CGemm g) {
    __shared__ float2 As[2][64 * SAP];
    __shared__ float2 Bs[2][SKC * SBP];
    const int ntile = g.tiles_m * g.tiles_n;
    const int bid = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int batch = bid / ntile, tile = bid - batch * ntile;
    const int tm = tile % g.tiles_m, tn = tile / g.tiles_m;
    const int m0 = tm * 64, n0 = tn * 64;
    const float2* A = g.A + (batch / g.dA % g.mA) * g.sA;
    const float2* B = g.B + (batch / g.dB % g.mB) * g.sB;
    float2* C = g.C + batch * g.sC;
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    // A loads: rows ar + kAS q at K column ak; B loads: K rows bk + 8 q' at columns bc + 32 q
    const int ak = tid % SKC, ar = tid / SKC, bc = tid & 31, bk = tid >> 5;
    int arow[kAQ], bcol[2];
#pragma unroll
    for (int q = 0; q < kAQ; ++q) arow[q] = min(m0 + ar + kAS * q, g.M - 1);  // rows past the end are never written
#pragma unroll
    for (int q = 0; q < 2; ++q) bcol[q] = min(n0 + bc + 32 * q, g.N - 1);
    const int nchunks = (g.K + SKC - 1) / SKC;
    float2 ra[kAQ], rbv[kBQ][2];
    float am = 0.f;
    floatx4 t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            t1[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
            t2[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
            t3[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
    const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;
    const bool any = m0 + wm < g.M && n0 + wn < g.N;
    const bool m1 = m0 + wm + 16 < g.M, n1 = n0 + wn + 16 < g.N;
    const bool full = any && m1 && n1;
    int buf = 0;
    for (int c = 0; c <= nchunks; ++c) {
        if (c < nchunks) {  // stage c into registers; K past the end contributes zero
            const int qa = c * SKC + ak;
            am = qa < g.K ? 1.f : 0.f;
            const int qac = min(qa, g.K - 1);
#pragma unroll
            for (int q = 0; q < kAQ; ++q) ra[q] = gld(A + (size_t)arow[q] * g.lda + qac);
#pragma unroll
            for (int q1 = 0; q1 < kBQ; ++q1) {
                const int qb = min(c * SKC + bk + 8 * q1, g.K - 1);
#pragma unroll
                for (int q = 0; q < 2; ++q) rbv[q1][q] = gld(B + (size_t)qb * g.ldb + bcol[q]);
            }
        }
        if (c > 0) {  // MFMAs of stage c - 1
            if (full)
                cgemm_stage<false>(As[buf], Bs[buf], wm, wn, lr, lk, true, true, t1, t2, t3);
            else if (any)
                cgemm_stage<true>(As[buf], Bs[buf], wm, wn, lr, lk, m1, n1, t1, t2, t3);
            buf ^= 1;
        }
        if (c < nchunks) {
#pragma unroll
            for (int q = 0; q < kAQ; ++q) As[buf][(ar + kAS * q) * SAP + ak] = make_float2(ra[q].x * am, ra[q].y * am);
#pragma unroll
            for (int q1 = 0; q1 < kBQ; ++q1)
#pragma unroll
                for (int q = 0; q < 2; ++q) Bs[buf][(bk + 8 * q1) * SBP + bc + 32 * q] = rbv[q1][q];
        }
        __syncthreads();
    }
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm + 16 * mb + 4 * lk + v, col = n0 + wn + 16 * nb + lr;
                if (row < g.M && col < g.N) {
                    const float r1 = t1[mb][nb][v], r2 = t2[mb][nb][v];
                    C[(size_t)row * g.ldc + col] = make_float2(r1 - r2, t3[mb][nb][v] - r1 - r2);
                }
            }
}

// ------------------------------------------------------------------ elementwise

struct SpinArgs {
    const float2* phi;     // [T][nmom][N^3]
    const float2* tau;     // [T][4N][4N]
    float2* tauT;          // [4N][4N] transpose of tau(t)
    float2* Bt;            // [nu][(4N)^3] folded source per unit
    float2* Y3;            // [nu][(4N)^3]
    double2* part;         // [nu][ntrip][nblk][nprof]
    double2* corr;         // [nmom][T][nprof][nprof]
    const float* gsnk;     // [nprof][T][N]
    const float* gsrc;     // [nprof][N] at t0
    const float2* ssnk;    // [nrow][64] sink spin tensor
    const float2* ssrc;    // [nrow][64] source spin tensor
    const int4* trip;      // [nrow][64]: (alpha, beta, gamma, index into ssnk) of the nonzero sink entries
    const int* ntrip;      // [nrow]
    int N, T, nmom, nprof, nrow, t0, t, pb0, nu, nblk, maxtrip;
};

// unit u of the round: (p, b) = pb0 + u / nrow, row s = u % nrow
__device__ __forceinline__ void unit_of(const SpinArgs& a, int u, int& p, int& b, int& s) {
    const int pb = a.pb0 + u / a.nrow;
    s = u - (u / a.nrow) * a.nrow;
    p = pb / a.nprof;
    b = pb - p * a.nprof;
}

// Bt[(al i)(be j)(ga k)] = conj(w_ijk Phi0_ijk S'[al be ga]) - conj(w_kji Phi0_kji S'[ga be al]),
// w the source profile weights g_i g_j g_k (symmetric in the three indices)
__global__ __launch_bounds__(256) void spin_source_kernel(SpinArgs a) {
    const int N = a.N, N4 = 4 * N;
    const size_t per = (size_t)N4 * N4 * N4;
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (size_t)a.nu * per) return;
    const int u = (int)(e / per);
    size_t r = e - (size_t)u * per;
    const int K = (int)(r % N4), J = (int)((r / N4) % N4), I = (int)(r / ((size_t)N4 * N4));
    const int al = I / N, i = I - al * N, be = J / N, j = J - be * N, ga = K / N, k = K - ga * N;
    int p, b, s;
    unit_of(a, u, p, b, s);
    const float* g = a.gsrc + (size_t)b * N;
    const float w = gld(g + i) * gld(g + j) * gld(g + k);
    const float2* ph = a.phi + ((size_t)a.t0 * a.nmom + p) * N * N * N;
    const float2 x = gld(ph + ((size_t)i * N + j) * N + k), y = gld(ph + ((size_t)k * N + j) * N + i);
    const float2 s1 = gld(a.ssrc + s * 64 + (al * 4 + be) * 4 + ga), s2 = gld(a.ssrc + s * 64 + (ga * 4 + be) * 4 + al);
    const float2 d = cmul(x, s1), f = cmul(y, s2);
    a.Bt[e] = make_float2(w * (d.x - f.x), -w * (d.y - f.y));  // conj(w x s1 - w y s2)
}

__global__ __launch_bounds__(256) void spin_transpose_kernel(SpinArgs a) {
    const int N4 = 4 * a.N;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= N4 * N4) return;
    const int r = e / N4, c = e - r * N4;
    a.tauT[(size_t)c * N4 + r] = gld(a.tau + (size_t)a.t * N4 * N4 + e);
}

// Sink dot at timeslice t: one workgroup per (unit, nonzero sink triple, block of 256
// (i, j) pairs); FP64 sums over k in each lane, over the workgroup in a fixed order,
// for every sink profile.
__global__ __launch_bounds__(256) void spin_sink_kernel(SpinArgs a) {
    // One workgroup: a unit, a sink triple and a block of 256 (i, j) pairs. The block's
    // 256 N terms (i, j, k) go to consecutive threads k fastest, so the reads of the
    // elementals (contiguous over (i, j, k)) and of Y3 (runs of N over k) are coalesced;
    // the sink profile weights g_q(t) are staged in LDS.
    __shared__ double2 red[4][kMaxProf];
    __shared__ float gw[kMaxProf * kMaxNvec];
    const int blk = blockIdx.x, tr = blockIdx.y, u = blockIdx.z;
    int p, b, s;
    unit_of(a, u, p, b, s);
    const int N = a.N, N4 = 4 * N;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int e = tid; e < a.nprof * N; e += 256) {
        const int q = e / N, i = e - q * N;
        gw[e] = a.gsnk[((size_t)q * a.T + a.t) * N + i];
    }
    __syncthreads();
    double2 acc[kMaxProf];
#pragma unroll
    for (int q = 0; q < kMaxProf; ++q) acc[q] = make_double2(0.0, 0.0);
    if (tr < a.ntrip[s]) {
        const int4 T4 = a.trip[s * 64 + tr];
        const float2 sv = gld(a.ssnk + s * 64 + T4.w);
        const int ij0 = blk * 256, nij = min(256, N * N - ij0);
        const float2* ph = a.phi + (((size_t)a.t * a.nmom + p) * N * N + ij0) * N;
        const float2* y3 = a.Y3 + (size_t)u * N4 * N4 * N4 + (size_t)T4.z * N;
        // term e = tid + 256 m is (i, j, k) with i N + j = ij0 + e / N, k = e % N,
        // advanced by 256 terms per step without division
        const int dl = 256 / N, dk = 256 - dl * N;
        int k = tid % N, i = (ij0 + tid / N) / N, j = (ij0 + tid / N) % N;
        for (int e = tid; e < nij * N; e += 256) {
            const float2* y = y3 + ((size_t)(T4.x * N + i) * N4 + T4.y * N + j) * N4;
            const float2 py = cmul(cmul(gld(ph + e), gld(y + k)), sv);
#pragma unroll
            for (int q = 0; q < kMaxProf; ++q) {  // fixed trip count: acc stays in registers
                if (q < a.nprof) {
                    const double wq = (double)gw[q * N + i] * gw[q * N + j] * gw[q * N + k];
                    acc[q].x += wq * py.x;
                    acc[q].y += wq * py.y;
                }
            }
            k += dk;
            j += dl;
            if (k >= N) {
                k -= N;
                ++j;
            }
            while (j >= N) {
                j -= N;
                ++i;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < kMaxProf; ++q) {
        const double x = wave_sum(acc[q].x), y = wave_sum(acc[q].y);
        if (lane == 0) red[w][q] = make_double2(x, y);
    }
    __syncthreads();
    if (tid < a.nprof) {
        double2 sum = make_double2(0.0, 0.0);
        for (int ww = 0; ww < 4; ++ww) {
            sum.x += red[ww][tid].x;
            sum.y += red[ww][tid].y;
        }
        a.part[(((size_t)u * a.maxtrip + tr) * a.nblk + blk) * a.nprof + tid] = sum;
    }
}

// C[p][t][a][b] for the round's (p, b): sum over rows, triples and blocks in a fixed order
__global__ __launch_bounds__(256) void spin_sum_kernel(SpinArgs a) {
    const int e = blockIdx.x * 256 + threadIdx.x;  // over [pb in round][nprof a]
    const int npb = a.nu / a.nrow;
    if (e >= npb * a.nprof) return;
    const int q = e % a.nprof, pbl = e / a.nprof;
    double2 sum = make_double2(0.0, 0.0);
    for (int s = 0; s < a.nrow; ++s) {
        const int u = pbl * a.nrow + s;
        for (int tr = 0; tr < a.maxtrip; ++tr)
            for (int blk = 0; blk < a.nblk; ++blk) {
                const double2 v = a.part[(((size_t)u * a.maxtrip + tr) * a.nblk + blk) * a.nprof + q];
                sum.x += v.x;
                sum.y += v.y;
            }
    }
    const int pb = a.pb0 + pbl, p = pb / a.nprof, b = pb - p * a.nprof;
    a.corr[(((size_t)p * a.T + a.t) * a.nprof + q) * a.nprof + b] = sum;
}

// ================================================================ host side

using namespace nuc::rt;

hipError_t gemm(const float2* A, const float2* B, float2* C, int M, int N, int K, int lda, int ldb, int ldc,
                long long sA, long long sB, long long sC, int batch, hipStream_t s, int dA, int mA, int dB, int mB) {
    CGemm g{A, B, C, M, N, K, lda, ldb, ldc, sA, sB, sC, (M + 63) / 64, (N + 63) / 64, dA, mA, dB, mB};
    const long long nblk = (long long)g.tiles_m * g.tiles_n * batch;
    hipLaunchKernelGGL(spin_cgemm_kernel, dim3((unsigned)nblk), dim3(256), 0, s, g);
    return hipGetLastError();
}

nuc_status spin_run(nuc_ctx ctx, const nuc_geom* g, const void* phi, const double* evals, int nprof,
                    const nuc_profile* prof, int nmom, const void* peramb, const nuc_spin* sp, void* corr,
                    hipStream_t s) {
    nuc_status st;
    if ((st = check_geom(ctx, g)) != NUC_OK) return st;
    if (nmom < 1 || nmom > 64) return fail(ctx, NUC_ERR_INVALID, "nmom=%d out of range [1,64]", nmom);
    if ((st = check_profiles(ctx, g, evals, nprof, prof)) != NUC_OK) return st;
    if (!phi || !peramb || !corr) return fail(ctx, NUC_ERR_INVALID, "phi, peramb or corr is NULL");
    if (!sp || !sp->snk || !sp->src) return fail(ctx, NUC_ERR_INVALID, "spin tensors are NULL");
    if (sp->nrow < 1 || sp->nrow > kMaxRow) return fail(ctx, NUC_ERR_INVALID, "nrow=%d out of range [1,4]", sp->nrow);
    const int N = g->nvec, T = g->T, N4 = 4 * N, nrow = sp->nrow;
    const size_t cube = (size_t)N4 * N4 * N4;
    // host tables: spin tensors (FP32), the nonzero sink triples per row, profiles
    std::vector<float2> ssnk((size_t)nrow * 64), ssrc((size_t)nrow * 64);
    std::vector<int4> trip((size_t)nrow * 64, make_int4(0, 0, 0, 0));
    std::vector<int> ntrip(nrow, 0);
    int maxtrip = 1;
    for (int r = 0; r < nrow; ++r) {
        for (int e = 0; e < 64; ++e) {
            const double sr = sp->snk[2 * (r * 64 + e)], si = sp->snk[2 * (r * 64 + e) + 1];
            const double tr = sp->src[2 * (r * 64 + e)], ti = sp->src[2 * (r * 64 + e) + 1];
            if (!isfinite(sr) || !isfinite(si) || !isfinite(tr) || !isfinite(ti))
                return fail(ctx, NUC_ERR_INVALID, "spin tensor entry (%d, %d) is not finite", r, e);
            ssnk[r * 64 + e] = make_float2((float)sr, (float)si);
            ssrc[r * 64 + e] = make_float2((float)tr, (float)ti);
            if (sr != 0.0 || si != 0.0) trip[r * 64 + ntrip[r]++] = make_int4(e / 16, (e / 4) % 4, e % 4, e);
        }
        maxtrip = std::max(maxtrip, ntrip[r]);
    }
    std::vector<double> gall((size_t)nprof * T * N);
    eval_profiles(g, evals, nprof, prof, gall.data());
    std::vector<float> gs(gall.size()), g0((size_t)nprof * N);
    for (size_t i = 0; i < gall.size(); ++i) gs[i] = (float)gall[i];
    for (int a = 0; a < nprof; ++a)
        for (int i = 0; i < N; ++i) g0[(size_t)a * N + i] = (float)gall[((size_t)a * T + g->t0) * N + i];
    HostBlock hb;
    const size_t o_ssnk = hb.add(ssnk.data(), ssnk.size() * sizeof(float2));
    const size_t o_ssrc = hb.add(ssrc.data(), ssrc.size() * sizeof(float2));
    const size_t o_trip = hb.add(trip.data(), trip.size() * sizeof(int4));
    const size_t o_ntrip = hb.add(ntrip.data(), ntrip.size() * sizeof(int));
    const size_t o_gs = hb.add(gs.data(), gs.size() * sizeof(float));
    const size_t o_g0 = hb.add(g0.data(), g0.size() * sizeof(float));
    // rounds of whole (p, b) pairs: Bt, Y1, Y2 (Y3 reuses Y1's buffer) per unit
    const int nblk = (N * N + 255) / 256;
    const size_t per_unit = 3 * cube * sizeof(float2) + (size_t)maxtrip * nblk * nprof * sizeof(double2);
    const size_t cap = ctx->budget ? std::min(kSpinCap, ctx->budget / 2) : kSpinCap;
    const int npb_total = nmom * nprof;
    const int npb = (int)std::max<long long>(1, std::min<long long>(npb_total, (long long)(cap / (per_unit * nrow))));
    const size_t o_tauT = align_up(hb.bytes.size(), 256);
    const size_t o_Bt = o_tauT + align_up((size_t)N4 * N4 * sizeof(float2), 256);
    const size_t o_Y1 = o_Bt + align_up((size_t)npb * nrow * cube * sizeof(float2), 256);
    const size_t o_Y2 = o_Y1 + align_up((size_t)npb * nrow * cube * sizeof(float2), 256);
    const size_t o_part = o_Y2 + align_up((size_t)npb * nrow * cube * sizeof(float2), 256);
    const size_t total = o_part + align_up((size_t)npb * nrow * maxtrip * nblk * nprof * sizeof(double2), 256);
    if ((st = begin_call(ctx, s)) != NUC_OK) return st;
    if ((st = ensure_workspace(ctx, total, s)) != NUC_OK) return st;
    char* base = (char*)ctx->ws;
    if ((st = upload_block(ctx, hb, base, s)) != NUC_OK) return st;
    SpinArgs a{};
    a.phi = (const float2*)phi;
    a.tau = (const float2*)peramb;
    a.tauT = (float2*)(base + o_tauT);
    a.Bt = (float2*)(base + o_Bt);
    a.Y3 = (float2*)(base + o_Y1);
    a.part = (double2*)(base + o_part);
    a.corr = (double2*)corr;
    a.gsnk = (const float*)(base + o_gs);
    a.gsrc = (const float*)(base + o_g0);
    a.ssnk = (const float2*)(base + o_ssnk);
    a.ssrc = (const float2*)(base + o_ssrc);
    a.trip = (const int4*)(base + o_trip);
    a.ntrip = (const int*)(base + o_ntrip);
    a.N = N;
    a.T = T;
    a.nmom = nmom;
    a.nprof = nprof;
    a.nrow = nrow;
    a.t0 = g->t0;
    a.nblk = nblk;
    a.maxtrip = maxtrip;
    float2* Y1 = (float2*)(base + o_Y1);
    float2* Y2 = (float2*)(base + o_Y2);
    for (int pb0 = 0; pb0 < npb_total; pb0 += npb) {
        const int np = std::min(npb, npb_total - pb0), nu = np * nrow;
        a.pb0 = pb0;
        a.nu = nu;
        const size_t nsrc = (size_t)nu * cube;
        HIPCHK(ctx, timed_launch(ctx, NUC_K_SPIN_SOURCE, s, [&] {
                   hipLaunchKernelGGL(spin_source_kernel, dim3((unsigned)((nsrc + 255) / 256)), dim3(256), 0, s, a);
                   return hipGetLastError();
               }));
        for (int t = 0; t < T; ++t) {
            a.t = t;
            const float2* tau_t = (const float2*)peramb + (size_t)t * N4 * N4;
            HIPCHK(ctx, timed_launch(ctx, NUC_K_SPIN_GEMM, s, [&] {
                       hipLaunchKernelGGL(spin_transpose_kernel, dim3((N4 * N4 + 255) / 256), dim3(256), 0, s, a);
                       return hipGetLastError();
                   }));
            HIPCHK(ctx, timed_launch(ctx, NUC_K_SPIN_GEMM, s, [&] {  // Y1 = tau Bt
                       return gemm(tau_t, a.Bt, Y1, N4, N4 * N4, N4, N4, N4 * N4, N4 * N4, 0, (long long)cube,
                                   (long long)cube, nu, s);
                   }));
            HIPCHK(ctx, timed_launch(ctx, NUC_K_SPIN_GEMM, s, [&] {  // Y2[I] = tau Y1[I]
                       return gemm(tau_t, Y1, Y2, N4, N4, N4, N4, N4, N4, 0, (long long)N4 * N4, (long long)N4 * N4,
                                   nu * N4, s);
                   }));
            HIPCHK(ctx, timed_launch(ctx, NUC_K_SPIN_GEMM, s, [&] {  // Y3 = Y2 tau^T
                       return gemm(Y2, a.tauT, Y1, N4 * N4, N4, N4, N4, N4, N4, (long long)cube, 0, (long long)cube,
                                   nu, s);
                   }));
            HIPCHK(ctx, timed_launch(ctx, NUC_K_SPIN_SINK, s, [&] {
                       hipLaunchKernelGGL(spin_sink_kernel, dim3(nblk, maxtrip, nu), dim3(256), 0, s, a);
                       return hipGetLastError();
                   }));
            HIPCHK(ctx, timed_launch(ctx, NUC_K_SPIN_SINK, s, [&] {
                       hipLaunchKernelGGL(spin_sum_kernel, dim3((np * nprof + 255) / 256), dim3(256), 0, s, a);
                       return hipGetLastError();
                   }));
        }
    }
    return end_call(ctx, s);
}

}  // namespace spin
}  // namespace nuc

extern "C" nuc_status nuc_correlator_spin(nuc_ctx ctx, const nuc_geom* geom, const void* phi, const double* evals,
                                          int nprof, const nuc_profile* prof, int nmom, const void* peramb,
                                          const nuc_spin* spin, void* corr, void* stream) {
    if (!ctx) return nuc::rt::fail(nullptr, NUC_ERR_INVALID, "ctx is NULL");
    std::lock_guard<std::mutex> lock(ctx->mu);
    nuc::rt::DeviceGuard guard;
    return nuc::spin::spin_run(ctx, geom, phi, evals, nprof, prof, nmom, peramb, spin, corr, (hipStream_t)stream);
}

extern "C" nuc_status nuc_spin_nucleon(int parity, double* out) {
    if (parity != 1 && parity != -1)
        return nuc::rt::fail(nullptr, NUC_ERR_INVALID, "parity=%d must be +1 or -1", parity);
    if (!out) return nuc::rt::fail(nullptr, NUC_ERR_INVALID, "out is NULL");
    // C = gamma2 gamma4 in the Euclidean Dirac-Pauli basis, then C gamma5
    const nuc::meson::Gammas G = nuc::meson::dirac_pauli();
    const nuc::meson::Mat4 cg5 = nuc::meson::mul(nuc::meson::mul(G.g[1], G.g4), G.g5);
    memset(out, 0, sizeof(double) * 2 * 2 * 64);
    for (int r = 0; r < 2; ++r) {
        const int sigma = parity > 0 ? r : 2 + r;  // the rows (1 + parity gamma4) / 2 keeps
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                double* e = out + 2 * (((r * 4 + a) * 4 + b) * 4 + sigma);
                e[0] = cg5.m[a][b].real();
                e[1] = cg5.m[a][b].imag();
            }
    }
    return NUC_OK;
}

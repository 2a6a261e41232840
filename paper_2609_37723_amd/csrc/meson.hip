// Profiled single-meson operators of the charmonium study (paper Section 3): the
// gauge-covariant derivatives of the distillation vectors, the meson elementals
// Phi^D_ij = sum_x exp(-ip.x) v_i^H (D v_j) for D in (1, nabla_k, B_k), and the
// correlation matrix of the profiled operators qbar Gamma q with
// Gamma in {g4 g5, g4 g5 g_k nabla_k, g_k B_k}, on gfx950, with the host runtime of
// the nuc_meson_* entry points.
//
// Kernels (FP32 arithmetic in HBM, FP64 where a long sum is taken):
//   meson_deriv    nabla_d v (pass 0) and B_i = nabla_j nabla_k - nabla_k nabla_j
//                  (pass 1): a site stencil, one thread per site, links in registers.
//   meson_elem     the site sum as one complex GEMM per (t, p): rows i (conj(v_i)
//                  times the momentum phase), columns (D, j), K = 3 L^3 (site, colour);
//                  FP32 MFMA 16x16x4, 64x64 complex tiles, LDS double buffer, FP32
//                  inside every 64-term stretch of K and FP64 across them; split K with
//                  FP64 partials.
//   meson_reduce   FP64 sum of the K splits into c64 Phi[t][p][D][i][j].
//   meson_gemm     the spin-sparse operator products Y_A = M_A tau and
//                  Z_B = (g5 tau g5)(g4 M_B(t0) g4) as lists of complex GEMMs whose K
//                  dimension concatenates up to three (Gamma, D) terms, profile weights
//                  applied on the fly.
//   meson_trace    Tr[Y_A Z_B^H] = sum Y_A conj(Z_B), FP64 accumulation.
//   meson_sum      FP64 sum of the trace partials into C_AB = -Tr[..] (the quark loop's sign).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <complex>
#include <vector>

#include "../../include/nucleon.h"
#include "nuc_internal.h"
#include "runtime_internal.h"

namespace nuc {
namespace meson {

constexpr int kMaxNvecMeson = 512;
constexpr int kND = 7;       // D = 1, nabla_0..2, B_0..2
constexpr int kNFam = 3;     // g4 g5; g4 g5 g_k nabla_k; g_k B_k
constexpr size_t kMesonCap = (size_t)16 << 30;

// ------------------------------------------------------------------ derivatives

struct DerivArgs {
    const float2* v;  // distillation vectors from timeslice t_off on: [.][N][V3][3]
    const float2* U;  // links from timeslice t_off on: [.][V3][3 dir][3][3]
    float2* F;        // [Tc][6][N][Kp]: nabla_0..2 v, then B_0..2 v (K = 3 V3 values, zero pad)
    int L, V3, N, Tc, jchunk, Kp;
};

// 1/2 [U_d(x) f(x+d) - U_d(x-d)^H f(x-d)] for one colour vector
__device__ __forceinline__ void cov_diff(const float2* uf, const float2* ub, const float2* ff, const float2* fb,
                                         float2* out) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        float sx = 0.f, sy = 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float2 u = uf[r * 3 + c], f = ff[c];
            sx += u.x * f.x - u.y * f.y;
            sy += u.x * f.y + u.y * f.x;
            const float2 w = ub[c * 3 + r], g = fb[c];  // conj(U[c][r]) g
            sx -= w.x * g.x + w.y * g.y;
            sy -= w.x * g.y - w.y * g.x;
        }
        out[r] = make_float2(0.5f * sx, 0.5f * sy);
    }
}

__device__ __forceinline__ void load3(const float2* base, int x, float2* f) {
#pragma unroll
    for (int c = 0; c < 3; ++c) f[c] = gld(base + (size_t)x * 3 + c);
}

// Grid: (site block, vector chunk, timeslice) flattened with the site block fastest and
// mapped so every XCD walks a contiguous range: the neighbour planes a block reads are
// the neighbouring blocks' own sites, which then sit in the same L2.
template <int PASS>
__global__ __launch_bounds__(256) void meson_deriv_kernel(DerivArgs a) {
    const int nxb = (a.V3 + 255) / 256, njc = (a.N + a.jchunk - 1) / a.jchunk;
    int r = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int xblk = r % nxb;
    r /= nxb;
    const int jc = r % njc;
    const int tc = r / njc;
    const int x = xblk * 256 + threadIdx.x;
    if (x >= a.V3) return;
    const int L = a.L;
    const int c[3] = {x % L, (x / L) % L, x / (L * L)};
    int xf[3], xb[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        int cf[3] = {c[0], c[1], c[2]}, cb[3] = {c[0], c[1], c[2]};
        cf[d] = c[d] + 1 == L ? 0 : c[d] + 1;
        cb[d] = c[d] == 0 ? L - 1 : c[d] - 1;
        xf[d] = cf[0] + L * (cf[1] + L * cf[2]);
        xb[d] = cb[0] + L * (cb[1] + L * cb[2]);
    }
    const float2* Ut = a.U + (size_t)tc * a.V3 * 27;
    float2 uf[3][9], ub[3][9];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            uf[d][e] = gld(Ut + ((size_t)x * 3 + d) * 9 + e);
            ub[d][e] = gld(Ut + ((size_t)xb[d] * 3 + d) * 9 + e);
        }
    const size_t vstride = (size_t)a.V3 * 3;  // one vector
    const size_t fstride = a.Kp;               // one field of one vector
    const int j0 = jc * a.jchunk, j1 = min(a.N, j0 + a.jchunk);
    const bool pad = x == a.V3 - 1 && a.Kp > 3 * a.V3;
    for (int j = j0; j < j1; ++j) {
        if (pad)
#pragma unroll
            for (int d = 0; d < 3; ++d)
                a.F[(((size_t)tc * 6 + 3 * PASS + d) * a.N + j) * fstride + 3 * a.V3] = make_float2(0.f, 0.f);
        if (PASS == 0) {
            const float2* vj = a.v + ((size_t)tc * a.N + j) * vstride;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                float2 ff[3], fb[3], o[3];
                load3(vj, xf[d], ff);
                load3(vj, xb[d], fb);
                cov_diff(uf[d], ub[d], ff, fb, o);
                float2* out = a.F + (((size_t)tc * 6 + d) * a.N + j) * fstride + (size_t)x * 3;
#pragma unroll
                for (int r = 0; r < 3; ++r) out[r] = o[r];
            }
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int jj = (i + 1) % 3, kk = (i + 2) % 3;
                const float2* wk = a.F + (((size_t)tc * 6 + kk) * a.N + j) * fstride;
                const float2* wj = a.F + (((size_t)tc * 6 + jj) * a.N + j) * fstride;
                float2 ff[3], fb[3], o1[3], o2[3];
                load3(wk, xf[jj], ff);
                load3(wk, xb[jj], fb);
                cov_diff(uf[jj], ub[jj], ff, fb, o1);
                load3(wj, xf[kk], ff);
                load3(wj, xb[kk], fb);
                cov_diff(uf[kk], ub[kk], ff, fb, o2);
                float2* out = a.F + (((size_t)tc * 6 + 3 + i) * a.N + j) * fstride + (size_t)x * 3;
#pragma unroll
                for (int r = 0; r < 3; ++r) out[r] = make_float2(o1[r].x - o2[r].x, o1[r].y - o2[r].y);
            }
        }
    }
}

// ------------------------------------------------------------ elemental GEMM

// Phase-weighted conjugate vectors A_p[i][(x,a)] = conj(v_i^a(x)) exp(-2 pi i n_p.x / L),
// the left operand of the site sum, and a copy of v, both with rows padded to an
// even length Kp (zero pad) so every 16-byte segment is aligned: slot p < nmom of
// the output is A_p, slot nmom the copy.
struct PhaseArgs {
    const float2* v;   // from timeslice t_off on: [.][N][K]
    const float2* ph;  // [nmom][V3]
    float2* A;         // [Tc][nmom][N][Kp]
    float2* V;         // [Tc][N][Kp]
    int N, K, Kp, nmom, Tc;
};

__global__ __launch_bounds__(256) void meson_phase_kernel(PhaseArgs a) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    const size_t per_p = (size_t)a.N * a.Kp;
    if (e >= (size_t)a.Tc * (a.nmom + 1) * per_p) return;
    const size_t r = e % per_p, tp = e / per_p;
    const int p = (int)(tp % (a.nmom + 1)), tc = (int)(tp / (a.nmom + 1));
    const int k = (int)(r % a.Kp), i = (int)(r / a.Kp);
    float2 y = make_float2(0.f, 0.f);
    if (k < a.K) {
        const float2 x = gld(a.v + ((size_t)tc * a.N + i) * a.K + k);
        if (p == a.nmom) {
            y = x;
        } else {
            const float2 f = gld(a.ph + (size_t)p * (a.K / 3) + k / 3);
            y = make_float2(x.x * f.x + x.y * f.y, x.x * f.y - x.y * f.x);  // conj(x) f
        }
    }
    if (p == a.nmom)
        a.V[(size_t)tc * per_p + r] = y;
    else
        a.A[((size_t)tc * a.nmom + p) * per_p + r] = y;
}

// Site sum Phi[i][(D,j)] = sum_K A_p[i][K] (D v_j)[K] as an NT GEMM: both operands are
// K-contiguous rows, staged into LDS with global_load_lds_dwordx4 in stages of 32
// complex (one row = 256 B = sixteen 16-byte segments; lane L of an instruction
// writes segment L % 16 of row L / 16 of its four rows and fetches logical segment
// (L % 16) ^ (row % 16), so the operand reads of 16 consecutive rows hit 16 different
// segment positions). The stage s+1 streams into one half of a double buffer while
// the MFMAs read stage s from the other; one barrier per stage. A workgroup owns a
// 64 x 64 complex output tile (four waves of 2 x 2 blocks of 16 x 16) and a range of
// stages (split K); FP32 accumulation inside every EFOLD stages, FP64 across them.
constexpr int EKC = 32;    // complex K values per stage (one staged row)
constexpr int EFOLD = 2;   // stages per FP32 stretch before the FP64 fold

__device__ float4 g_meson_zero[1];  // source of the zeros past the end of K

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void gbl_void_t;

struct ElemArgs {
    const float2* A;   // [Tc][nmom][N][Kp] phase-weighted conjugate vectors
    const float2* V;   // [Tc][N][Kp] the vectors (D = 1)
    const float2* F;   // [Tc][6][N][Kp] the derivative fields (D = nabla_k, B_k)
    double2* part;     // [nsplit][Tc][nmom][N][7N]
    int N, K, Kp, nmom, Tc, nsplit, cps, nchunks, mt, nt;
};

// Complex k..k+3 (k a multiple of 4) of staged row r as re[4], im[4].
__device__ __forceinline__ void elem_read4(const float2* arr, int r, int k, float (&re)[4], float (&im)[4]) {
    const int s0 = (k >> 1) ^ (r & 15);
    const float4 a01 = *reinterpret_cast<const float4*>(arr + r * EKC + 2 * s0);
    const float4 a23 = *reinterpret_cast<const float4*>(arr + r * EKC + 2 * (s0 ^ 1));
    re[0] = a01.x;
    re[1] = a01.z;
    re[2] = a23.x;
    re[3] = a23.z;
    im[0] = a01.y;
    im[1] = a01.w;
    im[2] = a23.y;
    im[3] = a23.w;
}

// The MFMAs of one stage for one wave (2 x NB blocks of 16 x 16 complex outputs): per
// group of 16 K values, operand reads of 4 consecutive K per lane, then 4 K steps.
// With GUARD, blocks outside the output (second row block unless m1, column blocks
// from nbv on) are skipped.
template <int NB, bool GUARD>
__device__ __forceinline__ void elem_stage(const float2* sA, const float2* sB, int wm, int wn, int lr, int lg, bool m1,
                                           int nbv, floatx4 (&cr)[2][NB], floatx4 (&ci)[2][NB]) {
#pragma unroll
    for (int kb = 0; kb < EKC; kb += 16) {
        float ar[2][4], ai[2][4], br[NB][4], bi[NB][4];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) elem_read4(sA, wm + 16 * mb + lr, kb + 4 * lg, ar[mb], ai[mb]);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) elem_read4(sB, wn + 16 * nb + lr, kb + 4 * lg, br[nb], bi[nb]);
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    if (GUARD && ((mb == 1 && !m1) || nb >= nbv)) continue;
                    cmfma16x4(ar[mb][v], ai[mb][v], br[nb][v], bi[nb][v], cr[mb][nb], ci[mb][nb]);
                }
    }
}

// Workgroup tile: 64 rows (i) x ETN columns ((D, j)), four waves as 2 x 2, each wave
// 32 x (16 NB) complex outputs.
template <int NB>
struct ElemTile {
    static constexpr int TN = 2 * 16 * NB;            // columns per workgroup
    static constexpr int ROWS = 64 + TN;              // staged rows per stage (A then B)
    static constexpr int SMEM = 2 * ROWS * EKC;       // float2, double buffer
};

template <int NB>
__global__ __launch_bounds__(256, NB <= 2 ? 2 : 1) void meson_elem_kernel(ElemArgs a) {
    using TL = ElemTile<NB>;
    __shared__ __attribute__((aligned(16))) float2 sm[TL::SMEM];  // [buf][A rows | B rows][32]
    int r = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int tm = r % a.mt;
    r /= a.mt;
    const int tn = r % a.nt;
    r /= a.nt;
    const int p = r % a.nmom;
    r /= a.nmom;
    const int s = r % a.nsplit;
    const int tc = r / a.nsplit;
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int N = a.N, K = a.K, N7 = kND * N;
    const int m0 = tm * 64, n0 = tn * TL::TN;

    // DMA sources of this lane: four-row groups 4 q + w (A: q < 4, B: q < TN / 16),
    // row 4 (4 q + w) + lane / 16 of the operand
    constexpr int QA = 4, QB = TL::TN / 16;
    const int rsub = lane >> 4, pos = lane & 15;
    const float2* src[QA + QB];
#pragma unroll
    for (int q = 0; q < QA; ++q) {
        const int i = min(m0 + 4 * (4 * q + w) + rsub, N - 1);  // rows past the end are never written
        src[q] = a.A + (((size_t)tc * a.nmom + p) * N + i) * a.Kp;
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
        const int n = min(n0 + 4 * (4 * q + w) + rsub, N7 - 1);
        const int D = n / N, j = n - D * N;
        src[QA + q] = D == 0 ? a.V + ((size_t)tc * N + j) * a.Kp : a.F + (((size_t)tc * 6 + D - 1) * N + j) * a.Kp;
    }
    const int swz = (4 * w + rsub) & 15;  // (row & 15) of every row this lane stages
    auto issue = [&](int chunk, int buf) __attribute__((always_inline)) {
        float2* d = sm + buf * TL::ROWS * EKC;
        const int k = chunk * EKC + 2 * (pos ^ swz);
#pragma unroll
        for (int q = 0; q < QA + QB; ++q) {
            const int r4 = q < QA ? 4 * q + w : 16 + 4 * (q - QA) + w;  // four-row group in [A | B]
            const void* gp = k < K ? (const void*)(src[q] + k) : (const void*)g_meson_zero;
            __builtin_amdgcn_global_load_lds((gbl_void_t*)gp, (lds_void_t*)(d + r4 * 4 * EKC), 16, 0, 0);
        }
    };

    floatx4 cr[2][NB], ci[2][NB];
    double dr[2][NB][4], di[2][NB][4];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            cr[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
            ci[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int v = 0; v < 4; ++v) dr[mb][nb][v] = di[mb][nb][v] = 0.0;
        }
    auto fold = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    dr[mb][nb][v] += (double)cr[mb][nb][v];
                    di[mb][nb][v] += (double)ci[mb][nb][v];
                }
                cr[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
                ci[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
            }
    };
    const int wm = (w & 1) * 32, wn = (w >> 1) * 16 * NB;
    const int lr = lane & 15, lg = lane >> 4;
    // 16 x 16 blocks of this wave inside the output (the rest of a tail tile is skipped)
    const bool m1 = m0 + wm + 16 < N;
    const int nbv = max(0, min(NB, (N7 - (n0 + wn) + 15) / 16));
    const bool any = m0 + wm < N && nbv > 0;
    const bool full = m1 && nbv == NB;

    const int c_begin = s * a.cps, c_end = min(a.nchunks, c_begin + a.cps);
    int nf = 0;
    if (c_begin < c_end) issue(c_begin, 0);
    for (int c = c_begin; c < c_end; ++c) {
        const int buf = (c - c_begin) & 1;
        __builtin_amdgcn_s_waitcnt(0);  // this lane's DMA of stage c has landed
        __syncthreads();                // ... every lane's, and stage c-1's buffer is free
        if (c + 1 < c_end) issue(c + 1, buf ^ 1);
        const float2* sA = sm + buf * TL::ROWS * EKC;
        const float2* sB = sA + 64 * EKC;
        if (full)
            elem_stage<NB, false>(sA, sB, wm, wn, lr, lg, true, NB, cr, ci);
        else if (any)
            elem_stage<NB, true>(sA, sB, wm, wn, lr, lg, m1, nbv, cr, ci);
        if (++nf == EFOLD) {
            fold();
            nf = 0;
        }
    }
    fold();
    double2* out = a.part + (((size_t)s * a.Tc + tc) * a.nmom + p) * (size_t)N * N7;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm + 16 * mb + 4 * lg + v, col = n0 + wn + 16 * nb + lr;
                if (row < N && col < N7) out[(size_t)row * N7 + col] = make_double2(dr[mb][nb][v], di[mb][nb][v]);
            }
}

constexpr int kElemNB = 2;  // column blocks per wave of the elemental GEMM

struct ElemReduceArgs {
    const double2* part;  // [nsplit][Tc][nmom][N][7N]
    float2* phi;          // [T][nmom][7][N][N]
    int N, nmom, Tc, nsplit, t_off;
};

__global__ __launch_bounds__(256) void meson_elem_reduce_kernel(ElemReduceArgs a) {
    const int N = a.N, N7 = kND * N;
    const size_t per = (size_t)a.Tc * a.nmom * N * N7;
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= per) return;
    double sr = 0.0, si = 0.0;
    for (int s = 0; s < a.nsplit; ++s) {
        const double2 v = a.part[(size_t)s * per + e];
        sr += v.x;
        si += v.y;
    }
    const int n = (int)(e % N7);
    size_t r = e / N7;
    const int i = (int)(r % N);
    r /= N;  // tc * nmom + p
    const int p = (int)(r % a.nmom), tc = (int)(r / a.nmom);
    const int D = n / N, j = n - D * N;
    a.phi[((((size_t)(a.t_off + tc) * a.nmom + p) * kND + D) * N + i) * N + j] = make_float2((float)sr, (float)si);
}

// --------------------------------------------------------- profile weighting

// Weighted elementals g_i^(a) g_j^(a) Phi^D_ij, the per-profile bilinear weighting,
// in the two layouts the operator products read:
//   sink  (SRC mode 0): Ps[tc][p][D][a][i][j] with the profiles at t = t_off + tc;
//   source (mode 1):    Pt[p][D][i][b][j]     with the profiles at t0.
struct WeightArgs {
    const float2* phi;  // [T][nmom][7][N][N]
    float2* out;
    const float* g;     // FP32 profiles: [nprof][T][N] (sink) or [nprof][N] (source, at t0)
    int N, T, nmom, nprof, t0, t_off, Tc, mode;
};

__global__ __launch_bounds__(256) void meson_weight_kernel(WeightArgs a) {
    const int N = a.N;
    const size_t N2 = (size_t)N * N;
    const size_t per_tp = (size_t)kND * a.nprof * N2;
    const size_t nt = a.mode == 0 ? (size_t)a.Tc : 1;
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= nt * a.nmom * per_tp) return;
    const int j = (int)(e % N);
    size_t r = e / N;
    int i, pr;
    if (a.mode == 0) {  // [.][D][a][i][j]
        i = (int)(r % N);
        r /= N;
        pr = (int)(r % a.nprof);
        r /= a.nprof;
    } else {            // [.][D][i][b][j]
        pr = (int)(r % a.nprof);
        r /= a.nprof;
        i = (int)(r % N);
        r /= N;
    }
    const int D = (int)(r % kND);
    r /= kND;
    const int p = (int)(r % a.nmom), tc = (int)(r / a.nmom);
    const int t = a.mode == 0 ? a.t_off + tc : a.t0;
    const float* g = a.mode == 0 ? a.g + ((size_t)pr * a.T + t) * N : a.g + (size_t)pr * N;
    const float w = gld(g + i) * gld(g + j);
    const float2 v = gld(a.phi + (((size_t)t * a.nmom + p) * kND + D) * N2 + (size_t)i * N + j);
    a.out[e] = make_float2(v.x * w, v.y * w);
}

// --------------------------------------------------------- operator products

// Operand sources, resolved per (t, p) inside the kernel.
enum { SRC_PS = 0, SRC_PT = 1, SRC_TAU = 2, SRC_Y = 3, SRC_Z = 4 };

struct GemmSeg {
    int a_src, a_off, lda;   // A_s [M][Kseg] at a_off, row stride lda
    int b_src, b_off, ldb;   // B_s [Kseg][Nc] at b_off, row stride ldb
    float2 coef;             // spin-matrix element of the term
};

// out(m, n) = sum_s coef_s sum_q A_s[m][q] B_s[q][n], stored at
//   out_off + (m / rb) rbs + (m % rb) ldo + (n / cb) cbs + n % cb
// (rb, cb: rows / columns per block of the output, rbs, cbs: their strides).
struct GemmItem {
    int out_src, out_off, ldo;
    int M, Nc, Kseg, nseg;
    int rb, rbs, cb, cbs;
    int tiles_m, tiles_n;
    GemmSeg seg[3];
};

struct GemmArgs {
    const GemmItem* items;
    const int* offs;        // [nitems + 1] first tile of each item
    int nitems, tiles_per_tp;
    const float2* Ps;       // [Tc][nmom][7][nprof][N][N] weighted sink elementals
    const float2* Pt;       // [nmom][7][N][nprof][N]    weighted source elementals
    const float2* tau;      // [T][4N][4N]
    float2* Y;              // [Tc][nmom][nop][4N][4N]
    float2* Z;              // [Tc][nmom][nop][4N][4N]
    int N, nmom, nprof, nop, t_off;
};

constexpr int GKC = 16;   // complex K values per LDS stage (segments start on a stage)
constexpr int GAP = 18;   // A tile [64][GKC] row pitch
constexpr int GBP = 80;   // B tile [GKC][64] row pitch

// One LDS stage of the operator GEMM for one wave (2 x 2 blocks of 16 x 16 complex):
// operand reads first, then the MFMAs; GUARD skips blocks outside the output.
template <bool GUARD>
__device__ __forceinline__ void gemm_stage(const float2* As, const float2* Bs, int wm, int wn, int lr, int lk, bool m1,
                                           bool n1, floatx4 (&cr)[2][2], floatx4 (&ci)[2][2]) {
    float2 av[GKC / 4][2], bv[GKC / 4][2];
#pragma unroll
    for (int ks = 0; ks < GKC / 4; ++ks) {
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) av[ks][mb] = As[(wm + 16 * mb + lr) * GAP + 4 * ks + lk];
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) bv[ks][nb] = Bs[(4 * ks + lk) * GBP + wn + 16 * nb + lr];
    }
#pragma unroll
    for (int ks = 0; ks < GKC / 4; ++ks)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                if (GUARD && ((mb == 1 && !m1) || (nb == 1 && !n1))) continue;
                cmfma16x4(av[ks][mb].x, av[ks][mb].y, bv[ks][nb].x, bv[ks][nb].y, cr[mb][nb], ci[mb][nb]);
            }
}

// Global -> register loads of one K stage: A rows arow[0..3] at K column q0 + akc
// (scaled by the term's coefficient, 0 past the segment's end), B row q0 + arb at
// columns bcol[0..3].
__device__ __forceinline__ void gemm_load(const float2* A, int lda, const float2* B, int ldb, float2 cf, int q0,
                                          int akc, int arb, int Kseg, const int (&arow)[4], const int (&bcol)[4],
                                          float2 (&ra)[4], float2 (&rbv)[4], float2& af) {
    const int qa = q0 + akc, qb = min(q0 + arb, Kseg - 1);
    const float m = qa < Kseg ? 1.f : 0.f;
    af = make_float2(cf.x * m, cf.y * m);
    const int qac = min(qa, Kseg - 1);
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) {
        ra[qq] = gld(A + (size_t)arow[qq] * lda + qac);
        rbv[qq] = gld(B + (size_t)qb * ldb + bcol[qq]);
    }
}

__global__ __launch_bounds__(256, 2) void meson_gemm_kernel(GemmArgs a) {
    __shared__ float2 As[2][64 * GAP];
    __shared__ float2 Bs[2][GKC * GBP];
    const int g = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int tp = g / a.tiles_per_tp, tile = g - tp * a.tiles_per_tp;
    const int tc = tp / a.nmom, p = tp - tc * a.nmom, t = a.t_off + tc;
    const int N = a.N;
    const size_t N2 = (size_t)N * N, N16 = 16 * N2;
    const size_t wsz = (size_t)kND * a.nprof * N2;  // weighted elementals of one (t, p)
    const int it = find_inst(a.offs, a.nitems, tile);
    const GemmItem I = a.items[it];
    const int local = tile - a.offs[it];
    const int tm = local % I.tiles_m, tn = local / I.tiles_m;
    const int m0 = tm * 64, n0 = tn * 64;
    const float2* bases[5] = {a.Ps + ((size_t)tc * a.nmom + p) * wsz, a.Pt + (size_t)p * wsz, a.tau + (size_t)t * N16,
                              a.Y + ((size_t)tc * a.nmom + p) * a.nop * N16,
                              a.Z + ((size_t)tc * a.nmom + p) * a.nop * N16};
    // per-segment operands, resolved once into named scalars (the item's source ids
    // are the same in every lane)
    const float2* pa0 = bases[I.seg[0].a_src] + I.seg[0].a_off;
    const float2* pa1 = bases[I.seg[1].a_src] + I.seg[1].a_off;
    const float2* pa2 = bases[I.seg[2].a_src] + I.seg[2].a_off;
    const float2* pb0 = bases[I.seg[0].b_src] + I.seg[0].b_off;
    const float2* pb1 = bases[I.seg[1].b_src] + I.seg[1].b_off;
    const float2* pb2 = bases[I.seg[2].b_src] + I.seg[2].b_off;
    float2* out = (float2*)bases[I.out_src] + I.out_off;

    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int Kseg = I.Kseg;
    const int cps = (Kseg + GKC - 1) / GKC;  // stages per segment
    const int nchunks = I.nseg * cps;
    // A loads: rows (tid >> 4) + 16 q, K offset tid & 15; B loads: K row tid >> 4, columns (tid & 15) + 16 q
    const int akc = tid & 15, arb = tid >> 4;
    int arow[4], bcol[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        arow[q] = min(m0 + arb + 16 * q, I.M - 1);
        bcol[q] = min(n0 + akc + 16 * q, I.Nc - 1);
    }
    float2 ra[4], rbv[4], af;

    floatx4 cr[2][2], ci[2][2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            cr[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
            ci[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
    const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;
    // 16 x 16 blocks of this wave inside the output (the rest of a tail tile is skipped)
    const bool any = m0 + wm < I.M && n0 + wn < I.Nc;
    const bool m1 = m0 + wm + 16 < I.M, n1 = n0 + wn + 16 < I.Nc;
    const bool full = any && m1 && n1;
    int buf = 0;
    for (int c = 0; c <= nchunks; ++c) {
        if (c < nchunks) {  // stage c into registers (the segment is the same in every lane)
            const int sg = c / cps;
            const int q0 = (c - sg * cps) * GKC;
            if (sg == 0)
                gemm_load(pa0, I.seg[0].lda, pb0, I.seg[0].ldb, I.seg[0].coef, q0, akc, arb, Kseg, arow, bcol, ra, rbv, af);
            else if (sg == 1)
                gemm_load(pa1, I.seg[1].lda, pb1, I.seg[1].ldb, I.seg[1].coef, q0, akc, arb, Kseg, arow, bcol, ra, rbv, af);
            else
                gemm_load(pa2, I.seg[2].lda, pb2, I.seg[2].ldb, I.seg[2].coef, q0, akc, arb, Kseg, arow, bcol, ra, rbv, af);
        }
        if (c > 0) {  // MFMAs of stage c - 1
            if (full)
                gemm_stage<false>(As[buf], Bs[buf], wm, wn, lr, lk, true, true, cr, ci);
            else if (any)
                gemm_stage<true>(As[buf], Bs[buf], wm, wn, lr, lk, m1, n1, cr, ci);
            buf ^= 1;
        }
        if (c < nchunks) {  // registers -> LDS buffer of stage c
#pragma unroll
            for (int qq = 0; qq < 4; ++qq) {
                As[buf][(arb + 16 * qq) * GAP + akc] = cmul(ra[qq], af);
                Bs[buf][arb * GBP + akc + 16 * qq] = rbv[qq];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            const int col = n0 + wn + 16 * nb + lr;
            const size_t co = (size_t)(col / I.cb) * I.cbs + col % I.cb;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm + 16 * mb + 4 * lk + v;
                if (row < I.M && col < I.Nc)
                    out[(size_t)(row / I.rb) * I.rbs + (size_t)(row % I.rb) * I.ldo + co] =
                        make_float2(cr[mb][nb][v], ci[mb][nb][v]);
            }
        }
}

// ------------------------------------------------------------------ trace

constexpr int TCH = 64;        // elements per LDS stage
constexpr int TCP = TCH + 1;   // LDS row pitch (complex)
constexpr int kMaxOp = 3 * kMaxProf;

struct TraceArgs {
    const float2* Y;   // [Tc][nmom][nop][4N][4N]
    const float2* Z;
    double2* part;     // [Tc][nmom][nwg][nop][nop]
    int N, nop, nmom, nwg, cpb;  // cpb: stages per row block of N x 4N elements
    int pi5[4];        // Z row block paired with Y row block gamma
    float2 s5[4];      // and its factor: C += Y conj(s5 Z)
};

__global__ __launch_bounds__(256) void meson_trace_kernel(TraceArgs a) {
    __shared__ double2 lds_raw[kMaxOp * TCP];  // Ys and Zs (float2 each), then the group partials
    float2* Ys = (float2*)lds_raw;
    float2* Zs = Ys + kMaxOp * TCP;
    const int tp = blockIdx.y, wg = blockIdx.x, tid = threadIdx.x;
    const int nop = a.nop;
    const size_t E = (size_t)4 * a.N * a.N;  // elements of one row block (N rows of 4N)
    const float2* Yb = a.Y + (size_t)tp * nop * 4 * E;
    const float2* Zb = a.Z + (size_t)tp * nop * 4 * E;
    const int nta = (nop + 2) / 3, ntiles = nta * nta;
    const int ngrp = 256 / ntiles;
    const int grp = tid / ntiles, tl = tid - grp * ntiles;
    const int ta = tl % nta, tb = tl / nta;
    double ar[3][3], ai[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) ar[i][j] = ai[i][j] = 0.0;
    const int nch = 4 * a.cpb;
    const int c0 = (int)((long long)wg * nch / a.nwg), c1 = (int)((long long)(wg + 1) * nch / a.nwg);
    for (int c = c0; c < c1; ++c) {
        const int gam = c / a.cpb;
        const size_t e0 = (size_t)(c - gam * a.cpb) * TCH;
        const int ne = (int)min((size_t)TCH, E - e0);
        const float2 f = a.s5[gam];
        const size_t yo = (size_t)gam * E + e0, zo = (size_t)a.pi5[gam] * E + e0;
        for (int idx = tid; idx < nop * TCH; idx += 256) {
            const int A = idx / TCH, e = idx - A * TCH;
            const int ec = min(e, ne - 1);
            const float m = e < ne ? 1.f : 0.f;
            const float2 y = gld(Yb + (size_t)A * 4 * E + yo + ec);
            const float2 z = gld(Zb + (size_t)A * 4 * E + zo + ec);
            Ys[A * TCP + e] = make_float2(y.x * m, y.y * m);
            const float2 zs = cmul(f, z);
            Zs[A * TCP + e] = make_float2(zs.x * m, zs.y * m);
        }
        __syncthreads();
        if (grp < ngrp) {
            for (int e = grp; e < TCH; e += ngrp) {
                double yr[3], yi[3], zr[3], zi[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const int A = min(3 * ta + i, nop - 1), B = min(3 * tb + i, nop - 1);
                    const float2 y = Ys[A * TCP + e], z = Zs[B * TCP + e];
                    yr[i] = y.x;
                    yi[i] = y.y;
                    zr[i] = z.x;
                    zi[i] = z.y;
                }
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) {  // y conj(z)
                        ar[i][j] = fma(yr[i], zr[j], fma(yi[i], zi[j], ar[i][j]));
                        ai[i][j] = fma(yi[i], zr[j], fma(-yr[i], zi[j], ai[i][j]));
                    }
            }
        }
        __syncthreads();
    }
    // group partials into LDS, then a fixed-order sum over groups
    double2* red = lds_raw;  // [ngrp][nop][nop]: ngrp * nop^2 <= 256 * 9 entries
    if (grp < ngrp) {
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int A = 3 * ta + i, B = 3 * tb + j;
                if (A < nop && B < nop) red[((size_t)grp * nop + A) * nop + B] = make_double2(ar[i][j], ai[i][j]);
            }
    }
    __syncthreads();
    double2* out = a.part + ((size_t)tp * a.nwg + wg) * nop * nop;
    for (int pr = tid; pr < nop * nop; pr += 256) {
        double sr = 0.0, si = 0.0;
        for (int gg = 0; gg < ngrp; ++gg) {
            const double2 v = red[(size_t)gg * nop * nop + pr];
            sr += v.x;
            si += v.y;
        }
        out[pr] = make_double2(sr, si);
    }
}

struct SumArgs {
    const double2* part;  // [Tc][nmom][nwg][nop][nop]
    double2* corr;        // [nmom][T][nop][nop]
    int T, nop, nmom, nwg, Tc, t_off;
};

__global__ __launch_bounds__(256) void meson_sum_kernel(SumArgs a) {
    const int npair = a.nop * a.nop;
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= a.Tc * a.nmom * npair) return;
    const int pr = e % npair, tp = e / npair;
    const int tc = tp / a.nmom, p = tp - tc * a.nmom;
    double sr = 0.0, si = 0.0;
    for (int wg = 0; wg < a.nwg; ++wg) {
        const double2 v = a.part[((size_t)tp * a.nwg + wg) * npair + pr];
        sr += v.x;
        si += v.y;
    }
    a.corr[((size_t)p * a.T + a.t_off + tc) * npair + pr] = make_double2(-sr, -si);  // quark loop: -1
}

// ================================================================ host side

using namespace nuc::rt;
typedef std::complex<double> cd;

struct Mat4 {
    cd m[4][4];
};

Mat4 mul(const Mat4& x, const Mat4& y) {
    Mat4 r{};
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
            for (int k = 0; k < 4; ++k) r.m[i][j] += x.m[i][k] * y.m[k][j];
    return r;
}

// Euclidean Dirac-Pauli matrices: gamma_k = [[0, -i sigma_k], [i sigma_k, 0]],
// gamma_4 = diag(1, 1, -1, -1), gamma_5 = g1 g2 g3 g4.
struct Gammas {
    Mat4 g[3], g4, g5;
};

Gammas dirac_pauli() {
    const cd I(0.0, 1.0);
    const cd sig[3][2][2] = {{{0.0, 1.0}, {1.0, 0.0}}, {{0.0, -I}, {I, 0.0}}, {{1.0, 0.0}, {0.0, -1.0}}};
    Gammas G{};
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                G.g[k].m[a][2 + b] = -I * sig[k][a][b];
                G.g[k].m[2 + a][b] = I * sig[k][a][b];
            }
    for (int a = 0; a < 4; ++a) G.g4.m[a][a] = a < 2 ? 1.0 : -1.0;
    G.g5 = mul(mul(mul(G.g[0], G.g[1]), G.g[2]), G.g4);
    return G;
}

// A matrix with exactly one nonzero per row and per column: col[r] and val[r] of row r.
struct Perm {
    int col[4];
    cd val[4];
    int row_of_col[4];
};

bool as_perm(const Mat4& x, Perm& p) {
    int cnt_col[4] = {0, 0, 0, 0};
    for (int r = 0; r < 4; ++r) {
        int n = 0;
        for (int c = 0; c < 4; ++c)
            if (std::abs(x.m[r][c]) > 1e-12) {
                p.col[r] = c;
                p.val[r] = x.m[r][c];
                p.row_of_col[c] = r;
                ++n;
                ++cnt_col[c];
            }
        if (n != 1) return false;
    }
    for (int c = 0; c < 4; ++c)
        if (cnt_col[c] != 1) return false;
    return true;
}

struct Term {
    Perm G;
    int D;
};

// The three operator families: (Gamma, D) terms.
bool operator_terms(std::vector<std::vector<Term>>& fam, Perm& g5p, double g4d[4]) {
    const Gammas G = dirac_pauli();
    const Mat4 g45 = mul(G.g4, G.g5);
    fam.assign(kNFam, {});
    Term t;
    if (!as_perm(g45, t.G)) return false;
    t.D = 0;
    fam[0].push_back(t);
    for (int k = 0; k < 3; ++k) {
        if (!as_perm(mul(g45, G.g[k]), t.G)) return false;
        t.D = 1 + k;
        fam[1].push_back(t);
    }
    for (int k = 0; k < 3; ++k) {
        if (!as_perm(G.g[k], t.G)) return false;
        t.D = 4 + k;
        fam[2].push_back(t);
    }
    if (!as_perm(G.g5, g5p)) return false;
    for (int a = 0; a < 4; ++a) g4d[a] = G.g4.m[a][a].real();
    return true;
}

float2 f2(cd z) { return make_float2((float)z.real(), (float)z.imag()); }

nuc_status check_meson_geom(nuc_ctx ctx, const nuc_geom* g) {
    if (!g) return fail(ctx, NUC_ERR_INVALID, "geom is NULL");
    if (g->L < 1 || g->L > 256) return fail(ctx, NUC_ERR_INVALID, "L=%d out of range [1,256]", g->L);
    if (g->T < 1) return fail(ctx, NUC_ERR_INVALID, "T=%d must be >= 1", g->T);
    if (g->nvec < 1 || g->nvec > kMaxNvecMeson)
        return fail(ctx, NUC_ERR_INVALID, "nvec=%d out of range [1,%d] for meson operators", g->nvec,
                    kMaxNvecMeson);
    if (g->t0 < 0 || g->t0 >= g->T) return fail(ctx, NUC_ERR_INVALID, "t0=%d outside [0,T)", g->t0);
    if ((long long)g->L * g->L * g->L * 3 > INT32_MAX / 2)
        return fail(ctx, NUC_ERR_INVALID, "L=%d too large", g->L);
    return NUC_OK;
}

// ------------------------------------------------------------ elementals plan

struct ElemPlan {
    int Tc = 1, nsplit = 1, cps = 1, nchunks = 1, mt = 1, nt = 1, Kp = 2;
    size_t off_ph = 0, off_A = 0, off_V = 0, off_F = 0, off_part = 0, bytes = 0;
};

ElemPlan plan_elem(const nuc_geom& g, int nmom, size_t cap) {
    ElemPlan P;
    const size_t N = g.nvec, V3 = (size_t)g.L * g.L * g.L, K = 3 * V3;
    P.Kp = (int)((K + 1) / 2 * 2);
    P.nchunks = (int)((K + EKC - 1) / EKC);
    P.mt = (int)((N + 63) / 64);
    P.nt = (int)((kND * N + ElemTile<kElemNB>::TN - 1) / ElemTile<kElemNB>::TN);
    // derivative fields, phase-weighted vectors and the vector copy, all with rows of Kp
    const size_t fields_t = (6 + nmom + 1) * N * P.Kp * sizeof(float2);
    const size_t part_t = (size_t)nmom * N * kND * N * sizeof(double2);
    const size_t ph = (size_t)nmom * V3 * sizeof(float2);
    // timeslices per launch Tc and K splits: a launch is tc nmom mt nt nsplit workgroups
    // of equal work (proportional to 1 / nsplit), run in rounds of `slots`. Pick the
    // pair whose workspace fits and whose summed rounds over all launches (the last one
    // may hold fewer timeslices) take the least time; a little extra for each split's
    // partials; ties go to the larger Tc.
    const long long slots = kElemNB <= 2 ? 512 : 256;
    const int max_split = std::max(1, std::min(16, P.nchunks / 16));
    const long long X = (long long)nmom * P.mt * P.nt;
    double best = 1e300;
    P.Tc = 1;
    P.nsplit = 1;
    for (int tc = g.T; tc >= 1; --tc)
        for (int ns = 1; ns <= max_split; ++ns) {
            if ((fields_t + part_t * ns) * tc > cap && !(tc == 1 && ns == 1)) continue;
            double rounds = 0.0;
            for (int t0c = 0; t0c < g.T; t0c += tc) {
                const long long items = (long long)std::min(tc, g.T - t0c) * X * ns;
                rounds += (double)((items + slots - 1) / slots);
            }
            const double cost = rounds / ns * (1.0 + 0.01 * ns);
            if (cost < best * (1.0 - 1e-9)) {
                best = cost;
                P.Tc = tc;
                P.nsplit = ns;
            }
        }
    P.cps = (P.nchunks + P.nsplit - 1) / P.nsplit;
    P.nsplit = (P.nchunks + P.cps - 1) / P.cps;
    P.off_ph = 0;
    P.off_A = align_up(ph, 256);
    P.off_V = P.off_A + align_up((size_t)nmom * N * P.Kp * sizeof(float2) * P.Tc, 256);
    P.off_F = P.off_V + align_up(N * P.Kp * sizeof(float2) * P.Tc, 256);
    P.off_part = P.off_F + align_up(6 * N * P.Kp * sizeof(float2) * P.Tc, 256);
    P.bytes = P.off_part + align_up(part_t * P.nsplit * P.Tc, 256);
    return P;
}

// --------------------------------------------------------- correlator plan

struct CorrPlan {
    int Tc = 1, nwg = 1, cpb = 1, nop = 3, tiles_per_tp = 0, nitems = 0;
    size_t off_items = 0, off_offs = 0, off_gsnk = 0, off_gsrc = 0, block_bytes = 0;
    size_t off_Pt = 0, off_Ps = 0, off_Y = 0, off_Z = 0, off_part = 0, bytes = 0;
    HostBlock block;
    int pi5[4];
    float2 s5[4];
};

nuc_status plan_corr(nuc_ctx ctx, const nuc_geom& g, int nmom, int nprof, const double* gall, size_t cap,
                     CorrPlan& P) {
    const int N = g.nvec, T = g.T;
    std::vector<std::vector<Term>> fam;
    Perm g5p;
    double g4d[4];
    if (!operator_terms(fam, g5p, g4d)) return fail(ctx, NUC_ERR_INTERNAL, "spin matrices are not permutations");
    P.nop = kNFam * nprof;
    const size_t N2 = (size_t)N * N, N16 = 16 * N2;
    const size_t wsz = (size_t)kND * nprof * N2;  // weighted elementals per (t, p)
    std::vector<GemmItem> items;
    auto tiles = [](int n) { return (n + 63) / 64; };
    // Y_(f,a) = M_(f,a) tau for all profiles a of family f at once, row block alpha:
    //   rows (a, i): sum_k Gamma_k[alpha][pi_k(alpha)] (g^a g^a Phi^{D_k})[i][.] tau[pi_k(alpha) block][.]
    for (int f = 0; f < kNFam; ++f)
        for (int al = 0; al < 4; ++al) {
            GemmItem I{};
            I.out_src = SRC_Y;
            I.out_off = (int)((size_t)f * nprof * N16 + (size_t)al * N * 4 * N);
            I.ldo = 4 * N;
            I.M = nprof * N;
            I.Nc = 4 * N;
            I.Kseg = N;
            I.nseg = (int)fam[f].size();
            I.rb = N;
            I.rbs = (int)N16;
            I.cb = I.Nc;
            I.cbs = 0;
            I.tiles_m = tiles(I.M);
            I.tiles_n = tiles(I.Nc);
            for (int k = 0; k < I.nseg; ++k) {
                const Term& tm = fam[f][k];
                GemmSeg& sg = I.seg[k];
                sg.a_src = SRC_PS;
                sg.a_off = (int)(tm.D * nprof * N2);
                sg.lda = N;
                sg.b_src = SRC_TAU;
                sg.b_off = (int)((size_t)tm.G.col[al] * N * 4 * N);
                sg.ldb = 4 * N;
                sg.coef = f2(tm.G.val[al]);
            }
            items.push_back(I);
        }
    // Z~_(f,b) for all profiles b of family f at once, column block beta: columns (b, j):
    //   sum_k s5'(alpha) g4(alpha) g4(beta) Gamma_k[alpha][beta] tau[:, rho5(alpha) block] (g^b g^b Phi^{D_k}(t0)),
    // alpha = the row of Gamma_k's nonzero in column beta. Z_B = (g5 tau g5)(g4 M_B(t0) g4) has
    // row block gamma equal to s5(gamma) times row block pi5(gamma) of Z~_B.
    for (int f = 0; f < kNFam; ++f)
        for (int be = 0; be < 4; ++be) {
            GemmItem I{};
            I.out_src = SRC_Z;
            I.out_off = (int)((size_t)f * nprof * N16 + (size_t)be * N);
            I.ldo = 4 * N;
            I.M = 4 * N;
            I.Nc = nprof * N;
            I.Kseg = N;
            I.nseg = (int)fam[f].size();
            I.rb = I.M;
            I.rbs = 0;
            I.cb = N;
            I.cbs = (int)N16;
            I.tiles_m = tiles(I.M);
            I.tiles_n = tiles(I.Nc);
            for (int k = 0; k < I.nseg; ++k) {
                const Term& tm = fam[f][k];
                const int al = tm.G.row_of_col[be];
                const int rho = g5p.row_of_col[al];
                const cd s5c = g5p.val[rho];  // g5[rho][al]
                GemmSeg& sg = I.seg[k];
                sg.a_src = SRC_TAU;
                sg.a_off = rho * N;
                sg.lda = 4 * N;
                sg.b_src = SRC_PT;
                sg.b_off = (int)(tm.D * nprof * N2);
                sg.ldb = nprof * N;
                sg.coef = f2(s5c * g4d[al] * g4d[be] * tm.G.val[al]);
            }
            items.push_back(I);
        }
    for (int gm = 0; gm < 4; ++gm) {
        P.pi5[gm] = g5p.col[gm];
        P.s5[gm] = f2(g5p.val[gm]);
    }
    // every operand and output element of every item inside its buffer
    auto src_size = [&](int src) -> size_t {
        switch (src) {
            case SRC_PS:
            case SRC_PT: return wsz;
            case SRC_TAU: return N16;
            case SRC_Y:
            case SRC_Z: return (size_t)P.nop * N16;
        }
        return 0;
    };
    for (const GemmItem& I : items) {
        bool ok = I.nseg >= 1 && I.nseg <= 3 && I.rb >= 1 && I.cb >= 1;
        size_t rmax = 0, cmax = 0;
        for (int r = 0; ok && r < I.M; ++r) rmax = std::max(rmax, (size_t)(r / I.rb) * I.rbs + (size_t)(r % I.rb) * I.ldo);
        for (int c = 0; ok && c < I.Nc; ++c) cmax = std::max(cmax, (size_t)(c / I.cb) * I.cbs + c % I.cb);
        ok = ok && (size_t)I.out_off + rmax + cmax < src_size(I.out_src);
        for (int k = 0; ok && k < I.nseg; ++k) {
            const GemmSeg& sg = I.seg[k];
            ok = ok && (size_t)sg.a_off + (size_t)(I.M - 1) * sg.lda + I.Kseg <= src_size(sg.a_src);
            ok = ok && (size_t)sg.b_off + (size_t)(I.Kseg - 1) * sg.ldb + I.Nc <= src_size(sg.b_src);
        }
        if (!ok) return fail(ctx, NUC_ERR_INTERNAL, "meson GEMM item out of bounds");
    }
    std::vector<int> offs(1, 0);
    for (const GemmItem& I : items) offs.push_back(offs.back() + I.tiles_m * I.tiles_n);
    P.nitems = (int)items.size();
    P.tiles_per_tp = offs.back();
    // FP32 profile values: sink [nprof][T][N], source (t0) [nprof][N]
    std::vector<float> gs((size_t)nprof * T * N), g0((size_t)nprof * N);
    for (size_t i = 0; i < gs.size(); ++i) gs[i] = (float)gall[i];
    for (int a = 0; a < nprof; ++a)
        for (int i = 0; i < N; ++i) g0[(size_t)a * N + i] = (float)gall[((size_t)a * T + g.t0) * N + i];
    P.off_items = P.block.add(items.data(), items.size() * sizeof(GemmItem));
    P.off_offs = P.block.add(offs.data(), offs.size() * sizeof(int));
    P.off_gsnk = P.block.add(gs.data(), gs.size() * sizeof(float));
    P.off_gsrc = P.block.add(g0.data(), g0.size() * sizeof(float));
    P.block_bytes = align_up(P.block.bytes.size(), 256);
    // timeslices per round
    P.cpb = (int)((4 * N2 + TCH - 1) / TCH);
    const size_t yz_tp = 2 * (size_t)P.nop * N16 * sizeof(float2) + wsz * sizeof(float2);
    auto part_tp = [&](int nwg) { return (size_t)nwg * P.nop * P.nop * sizeof(double2); };
    for (P.Tc = T; P.Tc > 1; --P.Tc)
        if ((yz_tp + part_tp(256)) * P.Tc * nmom <= cap) break;
    P.nwg = std::max(1, std::min({256, 4 * P.cpb, 2048 / std::max(1, P.Tc * nmom)}));
    P.off_Pt = P.block_bytes;
    P.off_Ps = P.off_Pt + align_up((size_t)nmom * wsz * sizeof(float2), 256);
    P.off_Y = P.off_Ps + align_up((size_t)P.Tc * nmom * wsz * sizeof(float2), 256);
    P.off_Z = P.off_Y + align_up((size_t)P.Tc * nmom * P.nop * N16 * sizeof(float2), 256);
    P.off_part = P.off_Z + align_up((size_t)P.Tc * nmom * P.nop * N16 * sizeof(float2), 256);
    P.bytes = P.off_part + align_up(part_tp(P.nwg) * P.Tc * nmom, 256);
    return NUC_OK;
}

// ------------------------------------------------------------------ calls

struct MesonCall {
    const nuc_geom* g;
    const void* evecs;
    const void* links;
    const double* evals;
    int nprof;
    const nuc_profile* prof;
    int nmom;
    const int32_t* mom;
    const void* peramb;
    void* phi;
    void* corr;
    int stage;  // 1 elementals, 2 correlator, 3 both
};

nuc_status meson_call(nuc_ctx ctx, const MesonCall& c, hipStream_t s) {
    nuc_status st;
    if ((st = check_meson_geom(ctx, c.g)) != NUC_OK) return st;
    const nuc_geom g = *c.g;
    const bool do_elem = c.stage & 1, do_corr = (c.stage & 2) != 0;
    if (c.nmom < 1 || c.nmom > 64) return fail(ctx, NUC_ERR_INVALID, "nmom=%d out of range [1,64]", c.nmom);
    if (do_elem) {
        if (!c.evecs) return fail(ctx, NUC_ERR_INVALID, "evecs is NULL");
        if (!c.links) return fail(ctx, NUC_ERR_INVALID, "links is NULL");
        if ((st = check_moms(ctx, &g, c.nmom, c.mom)) != NUC_OK) return st;
    }
    if (!c.phi && c.stage != 3) return fail(ctx, NUC_ERR_INVALID, "phi is NULL");
    std::vector<double> gall;
    if (do_corr) {
        if (!c.peramb) return fail(ctx, NUC_ERR_INVALID, "peramb is NULL");
        if (!c.corr) return fail(ctx, NUC_ERR_INVALID, "corr is NULL");
        if ((st = check_profiles(ctx, &g, c.evals, c.nprof, c.prof)) != NUC_OK) return st;
        gall.resize((size_t)c.nprof * g.T * g.nvec);
        eval_profiles(&g, c.evals, c.nprof, c.prof, gall.data());
    }
    const size_t cap = ctx->budget ? std::min(kMesonCap, ctx->budget / 2) : kMesonCap;
    const int N = g.nvec, V3 = g.L * g.L * g.L, K = 3 * V3;
    const size_t phi_bytes = (size_t)g.T * c.nmom * kND * N * N * sizeof(float2);
    const size_t off_phase = c.phi ? 0 : align_up(phi_bytes, 256);  // internal phi first
    ElemPlan EP;
    CorrPlan CP;
    if (do_elem) EP = plan_elem(g, c.nmom, cap);
    if (do_corr && (st = plan_corr(ctx, g, c.nmom, c.nprof, gall.data(), cap, CP)) != NUC_OK) return st;
    const size_t total = off_phase + std::max(do_elem ? EP.bytes : 0, do_corr ? CP.bytes : 0);

    if ((st = begin_call(ctx, s)) != NUC_OK) return st;
    if ((st = ensure_workspace(ctx, total, s)) != NUC_OK) return st;
    char* base = (char*)ctx->ws;
    float2* phi = c.phi ? (float2*)c.phi : (float2*)base;
    char* scr = base + off_phase;

    if (do_elem) {
        HostBlock hb;
        std::vector<float2> ph((size_t)c.nmom * V3);
        for (int p = 0; p < c.nmom; ++p)
            for (int x = 0; x < V3; ++x) {
                const int x0 = x % g.L, x1 = (x / g.L) % g.L, x2 = x / (g.L * g.L);
                long long nx = (long long)c.mom[3 * p] * x0 + (long long)c.mom[3 * p + 1] * x1 +
                               (long long)c.mom[3 * p + 2] * x2;
                nx = ((nx % g.L) + g.L) % g.L;
                const double ang = -2.0 * M_PI * (double)nx / g.L;
                ph[(size_t)p * V3 + x] = make_float2((float)cos(ang), (float)sin(ang));
            }
        hb.add(ph.data(), ph.size() * sizeof(float2));
        if ((st = upload_block(ctx, hb, scr + EP.off_ph, s)) != NUC_OK) return st;
        for (int t0c = 0; t0c < g.T; t0c += EP.Tc) {
            const int Tc = std::min(EP.Tc, g.T - t0c);
            DerivArgs da;
            da.v = (const float2*)c.evecs + (size_t)t0c * N * K;
            da.U = (const float2*)c.links + (size_t)t0c * V3 * 27;
            da.F = (float2*)(scr + EP.off_F);
            da.L = g.L;
            da.V3 = V3;
            da.N = N;
            da.Tc = Tc;
            da.jchunk = 8;
            da.Kp = EP.Kp;
            const dim3 dg(((V3 + 255) / 256) * ((N + da.jchunk - 1) / da.jchunk) * Tc);
            HIPCHK(ctx, timed_launch(ctx, NUC_K_MESON_DERIV, s, [&] {
                       hipLaunchKernelGGL(meson_deriv_kernel<0>, dg, dim3(256), 0, s, da);
                       return hipGetLastError();
                   }));
            HIPCHK(ctx, timed_launch(ctx, NUC_K_MESON_DERIV, s, [&] {
                       hipLaunchKernelGGL(meson_deriv_kernel<1>, dg, dim3(256), 0, s, da);
                       return hipGetLastError();
                   }));
            PhaseArgs pa;
            pa.v = da.v;
            pa.ph = (const float2*)(scr + EP.off_ph);
            pa.A = (float2*)(scr + EP.off_A);
            pa.V = (float2*)(scr + EP.off_V);
            pa.N = N;
            pa.K = K;
            pa.Kp = EP.Kp;
            pa.nmom = c.nmom;
            pa.Tc = Tc;
            const size_t nph = (size_t)Tc * (c.nmom + 1) * N * EP.Kp;
            HIPCHK(ctx, timed_launch(ctx, NUC_K_MESON_PHASE, s, [&] {
                       hipLaunchKernelGGL(meson_phase_kernel, dim3((unsigned)((nph + 255) / 256)), dim3(256), 0, s,
                                          pa);
                       return hipGetLastError();
                   }));
            ElemArgs ea;
            ea.A = pa.A;
            ea.V = pa.V;
            ea.F = da.F;
            ea.part = (double2*)(scr + EP.off_part);
            ea.N = N;
            ea.K = K;
            ea.Kp = EP.Kp;
            ea.nmom = c.nmom;
            ea.Tc = Tc;
            ea.nsplit = EP.nsplit;
            ea.cps = EP.cps;
            ea.nchunks = EP.nchunks;
            ea.mt = EP.mt;
            ea.nt = EP.nt;
            const int nblk = Tc * EP.nsplit * c.nmom * EP.mt * EP.nt;
            HIPCHK(ctx, timed_launch(ctx, NUC_K_MESON_ELEM, s, [&] {
                       hipLaunchKernelGGL(meson_elem_kernel<kElemNB>, dim3(nblk), dim3(256), 0, s, ea);
                       return hipGetLastError();
                   }));
            ElemReduceArgs ra;
            ra.part = ea.part;
            ra.phi = phi;
            ra.N = N;
            ra.nmom = c.nmom;
            ra.Tc = Tc;
            ra.nsplit = EP.nsplit;
            ra.t_off = t0c;
            const size_t nel = (size_t)Tc * c.nmom * N * kND * N;
            HIPCHK(ctx, timed_launch(ctx, NUC_K_MESON_ELEM_REDUCE, s, [&] {
                       hipLaunchKernelGGL(meson_elem_reduce_kernel, dim3((unsigned)((nel + 255) / 256)), dim3(256), 0,
                                          s, ra);
                       return hipGetLastError();
                   }));
        }
    }
    if (do_corr) {
        if ((st = upload_block(ctx, CP.block, scr, s)) != NUC_OK) return st;
        const size_t wsz = (size_t)kND * c.nprof * N * N;
        WeightArgs wa;
        wa.phi = phi;
        wa.N = N;
        wa.T = g.T;
        wa.nmom = c.nmom;
        wa.nprof = c.nprof;
        wa.t0 = g.t0;
        {  // source elementals, once per call
            wa.out = (float2*)(scr + CP.off_Pt);
            wa.g = (const float*)(scr + CP.off_gsrc);
            wa.t_off = 0;
            wa.Tc = 1;
            wa.mode = 1;
            const size_t nel = (size_t)c.nmom * wsz;
            HIPCHK(ctx, timed_launch(ctx, NUC_K_MESON_WEIGHT, s, [&] {
                       hipLaunchKernelGGL(meson_weight_kernel, dim3((unsigned)((nel + 255) / 256)), dim3(256), 0, s,
                                          wa);
                       return hipGetLastError();
                   }));
        }
        for (int t0c = 0; t0c < g.T; t0c += CP.Tc) {
            const int Tc = std::min(CP.Tc, g.T - t0c);
            wa.out = (float2*)(scr + CP.off_Ps);
            wa.g = (const float*)(scr + CP.off_gsnk);
            wa.t_off = t0c;
            wa.Tc = Tc;
            wa.mode = 0;
            const size_t nel = (size_t)Tc * c.nmom * wsz;
            HIPCHK(ctx, timed_launch(ctx, NUC_K_MESON_WEIGHT, s, [&] {
                       hipLaunchKernelGGL(meson_weight_kernel, dim3((unsigned)((nel + 255) / 256)), dim3(256), 0, s,
                                          wa);
                       return hipGetLastError();
                   }));
            GemmArgs ga;
            ga.items = (const GemmItem*)(scr + CP.off_items);
            ga.offs = (const int*)(scr + CP.off_offs);
            ga.nitems = CP.nitems;
            ga.tiles_per_tp = CP.tiles_per_tp;
            ga.Ps = (const float2*)(scr + CP.off_Ps);
            ga.Pt = (const float2*)(scr + CP.off_Pt);
            ga.tau = (const float2*)c.peramb;
            ga.Y = (float2*)(scr + CP.off_Y);
            ga.Z = (float2*)(scr + CP.off_Z);
            ga.N = N;
            ga.nmom = c.nmom;
            ga.nprof = c.nprof;
            ga.nop = CP.nop;
            ga.t_off = t0c;
            const unsigned nblk = (unsigned)CP.tiles_per_tp * Tc * c.nmom;
            HIPCHK(ctx, timed_launch(ctx, NUC_K_MESON_GEMM, s, [&] {
                       hipLaunchKernelGGL(meson_gemm_kernel, dim3(nblk), dim3(256), 0, s, ga);
                       return hipGetLastError();
                   }));
            TraceArgs ta;
            ta.Y = ga.Y;
            ta.Z = ga.Z;
            ta.part = (double2*)(scr + CP.off_part);
            ta.N = N;
            ta.nop = CP.nop;
            ta.nmom = c.nmom;
            ta.nwg = CP.nwg;
            ta.cpb = CP.cpb;
            for (int gm = 0; gm < 4; ++gm) {
                ta.pi5[gm] = CP.pi5[gm];
                ta.s5[gm] = CP.s5[gm];
            }
            HIPCHK(ctx, timed_launch(ctx, NUC_K_MESON_TRACE, s, [&] {
                       hipLaunchKernelGGL(meson_trace_kernel, dim3(CP.nwg, Tc * c.nmom), dim3(256), 0, s, ta);
                       return hipGetLastError();
                   }));
            SumArgs sa;
            sa.part = ta.part;
            sa.corr = (double2*)c.corr;
            sa.T = g.T;
            sa.nop = CP.nop;
            sa.nmom = c.nmom;
            sa.nwg = CP.nwg;
            sa.Tc = Tc;
            sa.t_off = t0c;
            const int nsum = Tc * c.nmom * CP.nop * CP.nop;
            HIPCHK(ctx, timed_launch(ctx, NUC_K_MESON_SUM, s, [&] {
                       hipLaunchKernelGGL(meson_sum_kernel, dim3((nsum + 255) / 256), dim3(256), 0, s, sa);
                       return hipGetLastError();
                   }));
        }
    }
    return end_call(ctx, s);
}

nuc_status meson_entry(nuc_ctx ctx, const MesonCall& c, void* stream) {
    if (!ctx) return fail(nullptr, NUC_ERR_INVALID, "ctx is NULL");
    std::lock_guard<std::mutex> lock(ctx->mu);
    DeviceGuard guard;
    return meson_call(ctx, c, (hipStream_t)stream);
}

}  // namespace meson
}  // namespace nuc

using nuc::meson::MesonCall;

extern "C" {

nuc_status nuc_meson_elementals(nuc_ctx ctx, const nuc_geom* geom, const void* evecs, const void* links, int nmom,
                                const int32_t* mom, void* phi, void* stream) {
    MesonCall c{geom, evecs, links, nullptr, 0, nullptr, nmom, mom, nullptr, phi, nullptr, 1};
    return nuc::meson::meson_entry(ctx, c, stream);
}

nuc_status nuc_meson_correlator(nuc_ctx ctx, const nuc_geom* geom, const void* phi, const double* evals, int nprof,
                                const nuc_profile* prof, int nmom, const void* peramb, void* corr, void* stream) {
    MesonCall c{geom, nullptr, nullptr, evals, nprof, prof, nmom, nullptr, peramb, (void*)phi, corr, 2};
    return nuc::meson::meson_entry(ctx, c, stream);
}

nuc_status nuc_meson_run(nuc_ctx ctx, const nuc_geom* geom, const void* evecs, const void* links,
                         const double* evals, int nprof, const nuc_profile* prof, int nmom, const int32_t* mom,
                         const void* peramb, void* phi, void* corr, void* stream) {
    MesonCall c{geom, evecs, links, evals, nprof, prof, nmom, mom, peramb, phi, corr, 3};
    return nuc::meson::meson_entry(ctx, c, stream);
}

}  // extern "C"

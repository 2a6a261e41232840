// Meson elementals on gfx950 (paper Section 3): the gauge-covariant derivatives of the
// distillation vectors (nabla_k and B_k = eps_kij nabla_i nabla_j as site stencils), the
// phase-weighted conjugate vectors, and the site sum
// Phi^D[t][p]_ij = sum_x exp(-ip.x) v_i^H (D v_j) as an FP32 MFMA GEMM with FP64 sums
// across 64-term stretches of the site index, staged through LDS by DMA.
#include "meson_internal.h"

namespace nuc {
namespace meson {

// ------------------------------------------------------------------ derivatives


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
constexpr int EFOLD = 2;   // stages per FP32 stretch before the FP64 fold

__device__ float4 g_meson_zero[1];  // source of the zeros past the end of K

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void gbl_void_t;


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
// group of 16 K values, operand reads of 4 consecutive K per lane, then 4 K steps,
// complex products in Gauss's three-multiplication form (t1 = sum ar br, t2 = sum ai bi,
// t3 = sum (ar + ai)(br + bi); the product is (t1 - t2) + i (t3 - t1 - t2)).
// With GUARD, blocks outside the output (second row block unless m1, column blocks
// from nbv on) are skipped.
// With Z (the first stage after an FP64 fold) the stage's first MFMA of each accumulator
// takes a zero accumulator operand, so the fold needs no clearing.
template <int NB, bool GUARD, bool Z>
__device__ __forceinline__ void elem_stage(const float2* sA, const float2* sB, int wm, int wn, int lr, int lg, bool m1,
                                           int nbv, floatx4 (&t1)[2][NB], floatx4 (&t2)[2][NB],
                                           floatx4 (&t3)[2][NB]) {
    const floatx4 z4 = floatx4{0.f, 0.f, 0.f, 0.f};
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
                    const bool first = Z && kb == 0 && v == 0;
                    t1[mb][nb] = mfma16x4(ar[mb][v], br[nb][v], first ? z4 : t1[mb][nb]);
                    t2[mb][nb] = mfma16x4(ai[mb][v], bi[nb][v], first ? z4 : t2[mb][nb]);
                    t3[mb][nb] = mfma16x4(ar[mb][v] + ai[mb][v], br[nb][v] + bi[nb][v], first ? z4 : t3[mb][nb]);
                }
    }
}


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

    floatx4 t1[2][NB], t2[2][NB], t3[2][NB];
    double dr[2][NB][4], di[2][NB][4];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            t1[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
            t2[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
            t3[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
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
                    const float r1 = t1[mb][nb][v], r2 = t2[mb][nb][v];
                    dr[mb][nb][v] += (double)(r1 - r2);
                    di[mb][nb][v] += (double)(t3[mb][nb][v] - r1 - r2);
                }
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
        if (full) {
            if (nf == 0)
                elem_stage<NB, false, true>(sA, sB, wm, wn, lr, lg, true, NB, t1, t2, t3);
            else
                elem_stage<NB, false, false>(sA, sB, wm, wn, lr, lg, true, NB, t1, t2, t3);
        } else if (any) {
            if (nf == 0)
                elem_stage<NB, true, true>(sA, sB, wm, wn, lr, lg, m1, nbv, t1, t2, t3);
            else
                elem_stage<NB, true, false>(sA, sB, wm, wn, lr, lg, m1, nbv, t1, t2, t3);
        }
        if (++nf == EFOLD) {
            fold();
            nf = 0;
        }
    }
    if (nf != 0) fold();  // the stages since the last fold (the accumulators are not cleared)
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

// ------------------------------------------------------------------ launchers

hipError_t launch_deriv(int pass, const DerivArgs& a, hipStream_t s) {
    const dim3 g(((a.V3 + 255) / 256) * ((a.N + a.jchunk - 1) / a.jchunk) * a.Tc);
    if (pass == 0)
        hipLaunchKernelGGL(meson_deriv_kernel<0>, g, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(meson_deriv_kernel<1>, g, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_phase(const PhaseArgs& a, hipStream_t s) {
    const size_t n = (size_t)a.Tc * (a.nmom + 1) * a.N * a.Kp;
    hipLaunchKernelGGL(meson_phase_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_elem(const ElemArgs& a, hipStream_t s) {
    const int nblk = a.Tc * a.nsplit * a.nmom * a.mt * a.nt;
    hipLaunchKernelGGL(meson_elem_kernel<kElemNB>, dim3(nblk), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_elem_reduce(const ElemReduceArgs& a, hipStream_t s) {
    const size_t n = (size_t)a.Tc * a.nmom * a.N * kND * a.N;
    hipLaunchKernelGGL(meson_elem_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace meson
}  // namespace nuc

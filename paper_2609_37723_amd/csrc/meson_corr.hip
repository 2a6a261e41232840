// Meson correlation matrix on gfx950 (paper Section 3): per-profile weighting
// g_i g_j Phi^D, the spin-sparse operator products Y_A = M_A tau and
// Z_B = (g5 tau g5)(g4 M_B(t0) g4) as stacked FP32 MFMA GEMMs, and the FP64 traces
// C_AB = -Tr[Y_A Z_B^H].
#include "meson_internal.h"

namespace nuc {
namespace meson {

// --------------------------------------------------------- profile weighting


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





constexpr int GKC = 16;   // complex K values per LDS stage (segments start on a stage)
constexpr int GAP = 18;   // A tile [64][GKC] row pitch
constexpr int GBP = 80;   // B tile [GKC][64] row pitch

// One LDS stage of the operator GEMM for one wave (2 x 2 blocks of 16 x 16 complex):
// operand reads first, then the MFMAs; GUARD skips blocks outside the output.
// MFMAs of one staged K block for a wave's 32 x 32 quadrant, complex products in Gauss's
// three-multiplication form: t1 = sum ar br, t2 = sum ai bi, t3 = sum (ar + ai)(br + bi),
// the product being (t1 - t2) + i (t3 - t1 - t2).
template <bool GUARD>
__device__ __forceinline__ void gemm_stage(const float2* As, const float2* Bs, int wm, int wn, int lr, int lk, bool m1,
                                           bool n1, floatx4 (&t1)[2][2], floatx4 (&t2)[2][2], floatx4 (&t3)[2][2]) {
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
                t1[mb][nb] = mfma16x4(av[ks][mb].x, bv[ks][nb].x, t1[mb][nb]);
                t2[mb][nb] = mfma16x4(av[ks][mb].y, bv[ks][nb].y, t2[mb][nb]);
                t3[mb][nb] = mfma16x4(av[ks][mb].x + av[ks][mb].y, bv[ks][nb].x + bv[ks][nb].y, t3[mb][nb]);
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
    // 16 x 16 blocks of this wave inside the output (the rest of a tail tile is skipped)
    const bool any = m0 + wm < I.M && n0 + wn < I.Nc;
    const bool m1 = m0 + wm + 16 < I.M, n1 = n0 + wn + 16 < I.Nc;
    const bool full = any && m1 && n1;
    int buf = 0;
    int sg = 0, q0 = 0;  // segment and K offset of stage c, advanced without division
    for (int c = 0; c <= nchunks; ++c) {
        if (c < nchunks) {  // stage c into registers (the segment is the same in every lane)
            if (sg == 0)
                gemm_load(pa0, I.seg[0].lda, pb0, I.seg[0].ldb, I.seg[0].coef, q0, akc, arb, Kseg, arow, bcol, ra, rbv, af);
            else if (sg == 1)
                gemm_load(pa1, I.seg[1].lda, pb1, I.seg[1].ldb, I.seg[1].coef, q0, akc, arb, Kseg, arow, bcol, ra, rbv, af);
            else
                gemm_load(pa2, I.seg[2].lda, pb2, I.seg[2].ldb, I.seg[2].coef, q0, akc, arb, Kseg, arow, bcol, ra, rbv, af);
            q0 += GKC;
            if (q0 >= cps * GKC) {
                q0 = 0;
                ++sg;
            }
        }
        if (c > 0) {  // MFMAs of stage c - 1
            if (full)
                gemm_stage<false>(As[buf], Bs[buf], wm, wn, lr, lk, true, true, t1, t2, t3);
            else if (any)
                gemm_stage<true>(As[buf], Bs[buf], wm, wn, lr, lk, m1, n1, t1, t2, t3);
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
    // output offsets: one division for the wave's first row and column, then carries
    const int row0 = m0 + wm + 4 * lk, col0 = n0 + wn + lr;
    const int rq0 = row0 / I.rb, rr0 = row0 - rq0 * I.rb;
    const int cq0 = col0 / I.cb, cr0 = col0 - cq0 * I.cb;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            const int col = col0 + 16 * nb;
            int cq = cq0, cr = cr0 + 16 * nb;
            while (cr >= I.cb) {
                cr -= I.cb;
                ++cq;
            }
            const size_t co = (size_t)cq * I.cbs + cr;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = row0 + 16 * mb + v;
                int rq = rq0, rr = rr0 + 16 * mb + v;
                while (rr >= I.rb) {
                    rr -= I.rb;
                    ++rq;
                }
                if (row < I.M && col < I.Nc) {
                    const float r1 = t1[mb][nb][v], r2 = t2[mb][nb][v];
                    out[(size_t)rq * I.rbs + (size_t)rr * I.ldo + co] = make_float2(r1 - r2, t3[mb][nb][v] - r1 - r2);
                }
            }
        }
}

// ------------------------------------------------------------------ trace

constexpr int TCP = TCH + 1;   // LDS row pitch (complex)
constexpr int kMaxOp = 3 * kMaxProf;


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

// ------------------------------------------------------------------ launchers

hipError_t launch_weight(const WeightArgs& a, size_t nel, hipStream_t s) {
    hipLaunchKernelGGL(meson_weight_kernel, dim3((unsigned)((nel + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs& a, unsigned nblk, hipStream_t s) {
    hipLaunchKernelGGL(meson_gemm_kernel, dim3(nblk), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_trace(const TraceArgs& a, int ntp, hipStream_t s) {
    hipLaunchKernelGGL(meson_trace_kernel, dim3(a.nwg, ntp), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sum(const SumArgs& a, int nsum, hipStream_t s) {
    hipLaunchKernelGGL(meson_sum_kernel, dim3((nsum + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace meson
}  // namespace nuc

// Glueball operators of the paper's Section 3 ("Improved glueball operators") on
// gfx950: the chromo-magnetic field B_i = eps_ijk F_jk from the clover F, adjoint
// gauge-covariant symmetric differences D_j, and the five A1^{-+} operators
//   O1 = sum_x Tr(eps_ijk B_i D_j B_k)             O2 = sum_x Tr(eps_ijk eps_ilm B_j B_k D_l B_m)
//   O3 = sum_x Tr(eps_ijk B_i D_j^3 B_k)           O4 = sum_x Tr(eps_ijk B_i D_j^2 D_k B_j)
//   O5 = sum_x Tr(eps_ijk B_i D_j D_i^2 B_k)
// per timeslice of many gauge configurations, with the host entry points.
//
// Data flow (every field is a 3 x 3 complex matrix per site, stored component-major,
// [9][V3] per (configuration, timeslice), so a wave's loads of one component are
// contiguous):
//   glue_links   links [c][t][V3][3][3][3] -> [c][t][3][9][V3]
//   glue_clover  B_0..2 (fields 0..2) from the four-leaf clover of each plane
//   glue_deriv   two levels of D_j applications, a task list per level:
//                DB_jk = D_j B_k; S1_ab = D_a D_a B_b, S2_ab = D_a D_b B_a
//   glue_contract the third D on the fly (D_j S1_jk for O3, D_j S2_jk for O4,
//                D_j S1_ik for O5, i the third index) and the five densities per
//                site, FP64 sums per workgroup
//   glue_sum      FP64 sum of the workgroup partials into O[c][t][5]
// FP32 arithmetic for the fields, FP64 for every site sum.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/nucleon.h"
#include "nuc_internal.h"
#include "runtime_internal.h"

namespace nuc {
namespace glue {

constexpr int kNOp = 5;
constexpr int kNField = 21;   // B (3), DB (6), S1 (6), S2 (6)
constexpr int F_B = 0, F_DB = 3, F_S1 = 9, F_S2 = 15;
constexpr size_t kGlueCap = (size_t)16 << 30;

// index of an ordered pair (a, b), a != b, in 0..5
__host__ __device__ constexpr int pair_index(int a, int b) { return 2 * a + (b > a ? b - 1 : b); }

// ------------------------------------------------------------ 3 x 3 complex algebra

struct M3 {
    float2 e[9];
};

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cfma(float2 a, float2 b, float2 c) {  // c + a b
    return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, c.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, c.y)));
}
__device__ __forceinline__ float2 cfma_conj_b(float2 a, float2 b, float2 c) {  // c + a conj(b)
    return make_float2(fmaf(a.x, b.x, fmaf(a.y, b.y, c.x)), fmaf(a.y, b.x, fmaf(-a.x, b.y, c.y)));
}
__device__ __forceinline__ float2 cfma_conj_a(float2 a, float2 b, float2 c) {  // c + conj(a) b
    return make_float2(fmaf(a.x, b.x, fmaf(a.y, b.y, c.x)), fmaf(a.x, b.y, fmaf(-a.y, b.x, c.y)));
}

__device__ __forceinline__ M3 mul(const M3& a, const M3& b) {  // a b
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            float2 s = make_float2(0.f, 0.f);
#pragma unroll
            for (int k = 0; k < 3; ++k) s = cfma(a.e[3 * i + k], b.e[3 * k + j], s);
            r.e[3 * i + j] = s;
        }
    return r;
}
__device__ __forceinline__ M3 mul_h(const M3& a, const M3& b) {  // a b^H
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            float2 s = make_float2(0.f, 0.f);
#pragma unroll
            for (int k = 0; k < 3; ++k) s = cfma_conj_b(a.e[3 * i + k], b.e[3 * j + k], s);
            r.e[3 * i + j] = s;
        }
    return r;
}
__device__ __forceinline__ M3 hmul(const M3& a, const M3& b) {  // a^H b
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            float2 s = make_float2(0.f, 0.f);
#pragma unroll
            for (int k = 0; k < 3; ++k) s = cfma_conj_a(a.e[3 * k + i], b.e[3 * k + j], s);
            r.e[3 * i + j] = s;
        }
    return r;
}
// Tr(a b) in FP64
__device__ __forceinline__ double2 trace_prod(const M3& a, const M3& b) {
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float2 x = a.e[3 * i + k], y = b.e[3 * k + i];
            re += (double)x.x * y.x - (double)x.y * y.y;
            im += (double)x.x * y.y + (double)x.y * y.x;
        }
    return make_double2(re, im);
}

// field component-major: base [9][V3]
__device__ __forceinline__ M3 ld(const float2* base, size_t V3, int x) {
    M3 m;
#pragma unroll
    for (int e = 0; e < 9; ++e) m.e[e] = gld(base + (size_t)e * V3 + x);
    return m;
}
__device__ __forceinline__ void st(float2* base, size_t V3, int x, const M3& m) {
#pragma unroll
    for (int e = 0; e < 9; ++e) base[(size_t)e * V3 + x] = m.e[e];
}

__device__ __forceinline__ int nbr(int x, int L, int d, int step) {
    int c[3] = {x % L, (x / L) % L, x / (L * L)};
    c[d] += step;
    c[d] = c[d] < 0 ? c[d] + L : (c[d] >= L ? c[d] - L : c[d]);
    return c[0] + L * (c[1] + L * c[2]);
}

// ------------------------------------------------------------------ kernels

struct GlueArgs {
    const float2* links;  // [nc][T][V3][3][3][3] (caller's layout)
    float2* U;            // [nct][3][9][V3]
    float2* F;            // [nct][kNField][9][V3]
    double2* part;        // [nct][nblk][5]
    double2* ops;         // [nc][T][5]
    const int4* tasks;    // (in field, direction, out field, 0)
    int ntask;
    int L, V3, nct, nblk;
};

__global__ __launch_bounds__(256) void glue_links_kernel(GlueArgs a) {
    const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;  // over [nct][V3][27]
    if (e >= (size_t)a.nct * a.V3 * 27) return;
    const int comp = (int)(e % 27);
    const size_t r = e / 27;
    const int x = (int)(r % a.V3), ct = (int)(r / a.V3);
    const int d = comp / 9, el = comp % 9;
    a.U[(((size_t)ct * 3 + d) * 9 + el) * a.V3 + x] = gld(a.links + e);
}

// F_mn(x) = (Q - Q^H) / 8, traceless; Q the sum of the four leaves in the (m, n) plane
__device__ M3 clover(const float2* U, int L, size_t V3, int x, int m, int n) {
    const float2* Um = U + (size_t)m * 9 * V3;
    const float2* Un = U + (size_t)n * 9 * V3;
    const int xpm = nbr(x, L, m, 1), xpn = nbr(x, L, n, 1), xmm = nbr(x, L, m, -1), xmn = nbr(x, L, n, -1);
    const int xmm_pn = nbr(xmm, L, n, 1), xmm_mn = nbr(xmm, L, n, -1), xpm_mn = nbr(xpm, L, n, -1);
    // x -> x+m -> x+m+n -> x+n -> x:  U_m(x) U_n(x+m) U_m(x+n)^H U_n(x)^H
    const M3 q = mul_h(mul_h(mul(ld(Um, V3, x), ld(Un, V3, xpm)), ld(Um, V3, xpn)), ld(Un, V3, x));
    // x -> x+n -> x-m+n -> x-m -> x:  U_n(x) U_m(x-m+n)^H U_n(x-m)^H U_m(x-m)
    const M3 l2 = mul(mul_h(mul_h(ld(Un, V3, x), ld(Um, V3, xmm_pn)), ld(Un, V3, xmm)), ld(Um, V3, xmm));
    // x -> x-m -> x-m-n -> x-n -> x:  U_m(x-m)^H U_n(x-m-n)^H U_m(x-m-n) U_n(x-n)
    //                                = (U_n(x-m-n) U_m(x-m))^H U_m(x-m-n) U_n(x-n)
    const M3 l3 = mul(hmul(mul(ld(Un, V3, xmm_mn), ld(Um, V3, xmm)), ld(Um, V3, xmm_mn)), ld(Un, V3, xmn));
    // x -> x-n -> x+m-n -> x+m -> x:  U_n(x-n)^H U_m(x-n) U_n(x+m-n) U_m(x)^H
    const M3 l4 = mul_h(mul(hmul(ld(Un, V3, xmn), ld(Um, V3, xmn)), ld(Un, V3, xpm_mn)), ld(Um, V3, x));
    M3 f;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const float2 s = cadd(cadd(q.e[3 * i + j], l2.e[3 * i + j]), cadd(l3.e[3 * i + j], l4.e[3 * i + j]));
            const float2 t = cadd(cadd(q.e[3 * j + i], l2.e[3 * j + i]), cadd(l3.e[3 * j + i], l4.e[3 * j + i]));
            // (s - conj(t)) / 8
            f.e[3 * i + j] = make_float2((s.x - t.x) * 0.125f, (s.y + t.y) * 0.125f);
        }
    const float2 tr3 = make_float2((f.e[0].x + f.e[4].x + f.e[8].x) / 3.f, (f.e[0].y + f.e[4].y + f.e[8].y) / 3.f);
#pragma unroll
    for (int i = 0; i < 3; ++i) f.e[4 * i] = csub(f.e[4 * i], tr3);
    return f;
}

__global__ __launch_bounds__(256) void glue_clover_kernel(GlueArgs a) {
    const int x = blockIdx.x * 256 + threadIdx.x, ct = blockIdx.y;
    if (x >= a.V3) return;
    const size_t V3 = a.V3;
    const float2* U = a.U + (size_t)ct * 27 * V3;
    float2* F = a.F + (size_t)ct * kNField * 9 * V3;
    // B_0 = 2 F_12, B_1 = 2 F_20, B_2 = 2 F_01
    const int pl[3][2] = {{1, 2}, {2, 0}, {0, 1}};
#pragma unroll 1
    for (int i = 0; i < 3; ++i) {
        M3 f = clover(U, a.L, V3, x, pl[i][0], pl[i][1]);
#pragma unroll
        for (int e = 0; e < 9; ++e) f.e[e] = make_float2(2.f * f.e[e].x, 2.f * f.e[e].y);
        st(F + (size_t)(F_B + i) * 9 * V3, V3, x, f);
    }
}

// (D_j X)(x) = 1/2 [U_j(x) X(x+j) U_j(x)^H - U_j(x-j)^H X(x-j) U_j(x-j)] for the field X
// ([9][V3]) and the links Uj ([9][V3]) of direction j
__device__ __forceinline__ M3 adjoint_diff(const float2* Uj, const float2* X, size_t V3, int L, int x, int j) {
    const int xf = nbr(x, L, j, 1), xb = nbr(x, L, j, -1);
    const M3 u = ld(Uj, V3, x);
    const M3 up = mul_h(mul(u, ld(X, V3, xf)), u);
    const M3 ub = ld(Uj, V3, xb);
    const M3 dn = mul(hmul(ub, ld(X, V3, xb)), ub);
    M3 r;
#pragma unroll
    for (int e = 0; e < 9; ++e) r.e[e] = make_float2(0.5f * (up.e[e].x - dn.e[e].x), 0.5f * (up.e[e].y - dn.e[e].y));
    return r;
}

// One task per blockIdx.y (in field, direction, out field), all sites, configurations
// and timeslices.
__global__ __launch_bounds__(256) void glue_deriv_kernel(GlueArgs a) {
    const int x = blockIdx.x * 256 + threadIdx.x, ct = blockIdx.z;
    if (x >= a.V3) return;
    const int4 tk = a.tasks[blockIdx.y];
    const size_t V3 = a.V3;
    const float2* Uj = a.U + ((size_t)ct * 3 + tk.y) * 9 * V3;
    const float2* X = a.F + ((size_t)ct * kNField + tk.x) * 9 * V3;
    st(a.F + ((size_t)ct * kNField + tk.z) * 9 * V3, V3, x, adjoint_diff(Uj, X, V3, a.L, x, tk.y));
}

__device__ __forceinline__ double2 dadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 dscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }

__global__ __launch_bounds__(256, 2) void glue_contract_kernel(GlueArgs a) {
    __shared__ double2 red[256 / 64][kNOp];
    const int x = blockIdx.x * 256 + threadIdx.x, ct = blockIdx.y;
    const size_t V3 = a.V3;
    const float2* F = a.F + (size_t)ct * kNField * 9 * V3;
    const float2* U = a.U + (size_t)ct * 27 * V3;
    double2 o[kNOp];
#pragma unroll
    for (int n = 0; n < kNOp; ++n) o[n] = make_double2(0.0, 0.0);
    if (x < a.V3) {
        // loops kept rolled: one B in registers at a time (reloaded from cache), the
        // loop indices only ever address memory
#pragma unroll 1
        for (int i = 0; i < 3; ++i) {
            const M3 Bi = ld(F + (size_t)(F_B + i) * 9 * V3, V3, x);
#pragma unroll 1
            for (int s = 0; s < 2; ++s) {  // (j, k) = (i+1, i+2) with eps +1, then swapped with eps -1
                const int j = s == 0 ? (i + 1) % 3 : (i + 2) % 3, k = s == 0 ? (i + 2) % 3 : (i + 1) % 3;
                const double e = s == 0 ? 1.0 : -1.0;
                const int pjk = pair_index(j, k);
                const float2* Uj = U + (size_t)j * 9 * V3;
                o[0] = dadd(o[0], dscale(e, trace_prod(Bi, ld(F + (size_t)(F_DB + pjk) * 9 * V3, V3, x))));
                // the third D on the fly: D_j^3 B_k, D_j^2 D_k B_j, D_j D_i^2 B_k
                o[2] = dadd(o[2], dscale(e, trace_prod(Bi, adjoint_diff(Uj, F + (size_t)(F_S1 + pjk) * 9 * V3, V3,
                                                                        a.L, x, j))));
                o[3] = dadd(o[3], dscale(e, trace_prod(Bi, adjoint_diff(Uj, F + (size_t)(F_S2 + pjk) * 9 * V3, V3,
                                                                        a.L, x, j))));
                o[4] = dadd(o[4], dscale(e, trace_prod(Bi, adjoint_diff(Uj, F + (size_t)(F_S1 + pair_index(i, k)) * 9 * V3,
                                                                        V3, a.L, x, j))));
            }
        }
        // O2 through eps_ijk eps_ilm = d_jl d_km - d_jm d_kl:
        //   sum_{j != k} Tr(B_j B_k D_j B_k) - Tr(B_j B_k D_k B_j)
#pragma unroll 1
        for (int j = 0; j < 3; ++j) {
            const M3 Bj = ld(F + (size_t)(F_B + j) * 9 * V3, V3, x);
#pragma unroll 1
            for (int k = 0; k < 3; ++k) {
                if (k == j) continue;
                const M3 bb = mul(Bj, ld(F + (size_t)(F_B + k) * 9 * V3, V3, x));
                const double2 t1 = trace_prod(bb, ld(F + (size_t)(F_DB + pair_index(j, k)) * 9 * V3, V3, x));
                const double2 t2 = trace_prod(bb, ld(F + (size_t)(F_DB + pair_index(k, j)) * 9 * V3, V3, x));
                o[1] = dadd(o[1], make_double2(t1.x - t2.x, t1.y - t2.y));
            }
        }
    }
    // workgroup sum in a fixed order: waves, then lanes
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int n = 0; n < kNOp; ++n) {
        o[n].x = wave_sum(o[n].x);
        o[n].y = wave_sum(o[n].y);
        if (lane == 0) red[w][n] = o[n];
    }
    __syncthreads();
    if (threadIdx.x < kNOp) {
        double2 s = make_double2(0.0, 0.0);
        for (int ww = 0; ww < 256 / 64; ++ww) s = dadd(s, red[ww][threadIdx.x]);
        a.part[((size_t)ct * a.nblk + blockIdx.x) * kNOp + threadIdx.x] = s;
    }
}

__global__ __launch_bounds__(256) void glue_sum_kernel(GlueArgs a) {
    const int e = blockIdx.x * 256 + threadIdx.x;  // over [nct][5]
    if (e >= a.nct * kNOp) return;
    const int n = e % kNOp, ct = e / kNOp;
    double2 s = make_double2(0.0, 0.0);
    for (int b = 0; b < a.nblk; ++b) s = dadd(s, a.part[((size_t)ct * a.nblk + b) * kNOp + n]);
    a.ops[e] = s;
}

// ================================================================ host side

using namespace nuc::rt;

// The derivative tasks of the two stored levels (the third D is taken in the contraction).
void make_tasks(std::vector<int4>& l1, std::vector<int4>& l2) {
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) {
            if (j == k) continue;
            const int p = pair_index(j, k);
            l1.push_back(make_int4(F_B + k, j, F_DB + p, 0));                         // D_j B_k
            l2.push_back(make_int4(F_DB + p, j, F_S1 + p, 0));                       // D_j D_j B_k
            l2.push_back(make_int4(F_DB + pair_index(k, j), j, F_S2 + p, 0));        // D_j D_k B_j
        }
}

nuc_status glue_run(nuc_ctx ctx, int L, int T, int nconf, const void* links, void* ops, hipStream_t s) {
    if (L < 2 || L > 256) return fail(ctx, NUC_ERR_INVALID, "L=%d out of range [2,256]", L);
    if (T < 1) return fail(ctx, NUC_ERR_INVALID, "T=%d must be >= 1", T);
    if (nconf < 1) return fail(ctx, NUC_ERR_INVALID, "nconf=%d must be >= 1", nconf);
    if (!links || !ops) return fail(ctx, NUC_ERR_INVALID, "links or ops is NULL");
    if ((long long)L * L * L > (1LL << 28)) return fail(ctx, NUC_ERR_INVALID, "L=%d too large", L);
    const int V3 = L * L * L;
    const int nblk = (V3 + 255) / 256;
    const size_t per_ct = (size_t)(27 + kNField * 9) * V3 * sizeof(float2) + (size_t)nblk * kNOp * sizeof(double2);
    const size_t cap = ctx->budget ? std::min(kGlueCap, ctx->budget / 2) : kGlueCap;
    const long long total_ct = (long long)nconf * T;
    // (configuration, timeslice) pairs per round: within the workspace cap and the
    // grid's y / z limit
    const long long fit = std::max<long long>(1, std::min<long long>({total_ct, (long long)(cap / per_ct), 65535LL}));
    const long long rounds = (total_ct + fit - 1) / fit;  // equal rounds, no small last one
    const int nct_max = (int)((total_ct + rounds - 1) / rounds);
    std::vector<int4> l1, l2;
    make_tasks(l1, l2);
    HostBlock hb;
    const size_t off1 = hb.add(l1.data(), l1.size() * sizeof(int4));
    const size_t off2 = hb.add(l2.data(), l2.size() * sizeof(int4));
    const size_t off_U = align_up(hb.bytes.size(), 256);
    const size_t off_F = off_U + align_up((size_t)nct_max * 27 * V3 * sizeof(float2), 256);
    const size_t off_P = off_F + align_up((size_t)nct_max * kNField * 9 * V3 * sizeof(float2), 256);
    const size_t total = off_P + align_up((size_t)nct_max * nblk * kNOp * sizeof(double2), 256);
    nuc_status st;
    if ((st = begin_call(ctx, s)) != NUC_OK) return st;
    if ((st = ensure_workspace(ctx, total, s)) != NUC_OK) return st;
    char* base = (char*)ctx->ws;
    if ((st = upload_block(ctx, hb, base, s)) != NUC_OK) return st;
    for (long long c0 = 0; c0 < total_ct; c0 += nct_max) {
        const int nct = (int)std::min<long long>(nct_max, total_ct - c0);
        GlueArgs a;
        a.links = (const float2*)links + (size_t)c0 * V3 * 27;
        a.U = (float2*)(base + off_U);
        a.F = (float2*)(base + off_F);
        a.part = (double2*)(base + off_P);
        a.ops = (double2*)ops + (size_t)c0 * kNOp;
        a.L = L;
        a.V3 = V3;
        a.nct = nct;
        a.nblk = nblk;
        const size_t nl = (size_t)nct * V3 * 27;
        HIPCHK(ctx, timed_launch(ctx, NUC_K_GLUE_STENCIL, s, [&] {
                   hipLaunchKernelGGL(glue_links_kernel, dim3((unsigned)((nl + 255) / 256)), dim3(256), 0, s, a);
                   return hipGetLastError();
               }));
        HIPCHK(ctx, timed_launch(ctx, NUC_K_GLUE_STENCIL, s, [&] {
                   hipLaunchKernelGGL(glue_clover_kernel, dim3(nblk, nct), dim3(256), 0, s, a);
                   return hipGetLastError();
               }));
        const std::vector<int4>* lv[2] = {&l1, &l2};
        const size_t offs[2] = {off1, off2};
        for (int l = 0; l < 2; ++l) {
            a.tasks = (const int4*)(base + offs[l]);
            a.ntask = (int)lv[l]->size();
            HIPCHK(ctx, timed_launch(ctx, NUC_K_GLUE_STENCIL, s, [&] {
                       hipLaunchKernelGGL(glue_deriv_kernel, dim3(nblk, a.ntask, nct), dim3(256), 0, s, a);
                       return hipGetLastError();
                   }));
        }
        HIPCHK(ctx, timed_launch(ctx, NUC_K_GLUE_CONTRACT, s, [&] {
                   hipLaunchKernelGGL(glue_contract_kernel, dim3(nblk, nct), dim3(256), 0, s, a);
                   return hipGetLastError();
               }));
        HIPCHK(ctx, timed_launch(ctx, NUC_K_GLUE_CONTRACT, s, [&] {
                   hipLaunchKernelGGL(glue_sum_kernel, dim3((nct * kNOp + 255) / 256), dim3(256), 0, s, a);
                   return hipGetLastError();
               }));
    }
    return end_call(ctx, s);
}

}  // namespace glue
}  // namespace nuc

extern "C" {

nuc_status nuc_glueball_operators(nuc_ctx ctx, int L, int T, int nconf, const void* links, void* ops, void* stream) {
    if (!ctx) return nuc::rt::fail(nullptr, NUC_ERR_INVALID, "ctx is NULL");
    std::lock_guard<std::mutex> lock(ctx->mu);
    nuc::rt::DeviceGuard guard;
    return nuc::glue::glue_run(ctx, L, T, nconf, links, ops, (hipStream_t)stream);
}

nuc_status nuc_glueball_correlator(const void* ops, int T, int nop, void* corr) {
    if (!ops || !corr || T < 1 || nop < 1) return NUC_ERR_INVALID;
    const double* o = (const double*)ops;  // [T][nop] complex
    double* c = (double*)corr;             // [T][nop][nop] complex
    std::vector<double> mr(nop, 0.0), mi(nop, 0.0);
    for (int t = 0; t < T; ++t)
        for (int n = 0; n < nop; ++n) {
            mr[n] += o[2 * ((size_t)t * nop + n)] / T;
            mi[n] += o[2 * ((size_t)t * nop + n) + 1] / T;
        }
    for (int dt = 0; dt < T; ++dt)
        for (int n = 0; n < nop; ++n)
            for (int m = 0; m < nop; ++m) {
                double sr = 0.0, si = 0.0;
                for (int t = 0; t < T; ++t) {
                    const size_t a = 2 * ((size_t)((t + dt) % T) * nop + n), b = 2 * ((size_t)t * nop + m);
                    // O_n(t+dt) conj(O_m(t))
                    sr += o[a] * o[b] + o[a + 1] * o[b + 1];
                    si += o[a + 1] * o[b] - o[a] * o[b + 1];
                }
                const size_t k = 2 * (((size_t)dt * nop + n) * nop + m);
                c[k] = sr / T - (mr[n] * mr[m] + mi[n] * mi[m]);
                c[k + 1] = si / T - (mi[n] * mr[m] - mr[n] * mi[m]);
            }
    return NUC_OK;
}

}  // extern "C"

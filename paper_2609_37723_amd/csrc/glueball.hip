// Glueball operators of the paper's Section 3 ("Improved glueball operators") on
// gfx950: the chromo-magnetic field B_i = eps_ijk F_jk from the clover F, adjoint
// gauge-covariant symmetric differences D_j, and the five A1^{-+} operators
//   O1 = sum_x Tr(eps_ijk B_i D_j B_k)             O2 = sum_x Tr(eps_ijk eps_ilm B_j B_k D_l B_m)
//   O3 = sum_x Tr(eps_ijk B_i D_j^3 B_k)           O4 = sum_x Tr(eps_ijk B_i D_j^2 D_k B_j)
//   O5 = sum_x Tr(eps_ijk B_i D_j D_i^2 B_k)
// per timeslice of many gauge configurations, with the host entry points.
//
// Data flow (stored component-major per (configuration, timeslice), so a wave's loads
// of one component are contiguous; every stored field is traceless anti-Hermitian,
// the clover B_i and all its adjoint differences, and is kept as the 8 reals of that
// algebra, [8][V3] floats; the SU(3) links keep their first two rows, [6][V3] complex,
// the third being the conjugated cross product of the two):
//   glue_links   links [c][t][V3][3][3][3] -> [c][t][3][6][V3]
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

// Traceless anti-Hermitian field, component-major [8][V3] floats:
// (Im X00, Im X11, Re X01, Im X01, Re X02, Im X02, Re X12, Im X12).
__device__ __forceinline__ M3 ldA(const float* base, size_t V3, int x) {
    float c[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) c[e] = gld(base + (size_t)e * V3 + x);
    M3 m;
    m.e[0] = make_float2(0.f, c[0]);
    m.e[4] = make_float2(0.f, c[1]);
    m.e[8] = make_float2(0.f, -c[0] - c[1]);
    m.e[1] = make_float2(c[2], c[3]);
    m.e[2] = make_float2(c[4], c[5]);
    m.e[5] = make_float2(c[6], c[7]);
    m.e[3] = make_float2(-c[2], c[3]);
    m.e[6] = make_float2(-c[4], c[5]);
    m.e[7] = make_float2(-c[6], c[7]);
    return m;
}
// Stores the traceless anti-Hermitian part (M - M^H)/2 - Tr/3 of m (m itself for the
// fields here, up to rounding).
__device__ __forceinline__ void stA(float* base, size_t V3, int x, const M3& m) {
    const float ti = (m.e[0].y + m.e[4].y + m.e[8].y) * (1.f / 3.f);
    float c[8];
    c[0] = m.e[0].y - ti;
    c[1] = m.e[4].y - ti;
    c[2] = 0.5f * (m.e[1].x - m.e[3].x);
    c[3] = 0.5f * (m.e[1].y + m.e[3].y);
    c[4] = 0.5f * (m.e[2].x - m.e[6].x);
    c[5] = 0.5f * (m.e[2].y + m.e[6].y);
    c[6] = 0.5f * (m.e[5].x - m.e[7].x);
    c[7] = 0.5f * (m.e[5].y + m.e[7].y);
#pragma unroll
    for (int e = 0; e < 8; ++e) base[(size_t)e * V3 + x] = c[e];
}
// SU(3) link from its first two rows ([6][V3] complex): row 2 = conj(row 0 x row 1).
__device__ __forceinline__ M3 ldU(const float2* base, size_t V3, int x) {
    M3 m;
#pragma unroll
    for (int e = 0; e < 6; ++e) m.e[e] = gld(base + (size_t)e * V3 + x);
    auto cross = [](float2 a, float2 b, float2 c, float2 d) {  // conj(a b - c d)
        return make_float2(a.x * b.x - a.y * b.y - c.x * d.x + c.y * d.y, -(a.x * b.y + a.y * b.x - c.x * d.y - c.y * d.x));
    };
    m.e[6] = cross(m.e[1], m.e[5], m.e[2], m.e[4]);
    m.e[7] = cross(m.e[2], m.e[3], m.e[0], m.e[5]);
    m.e[8] = cross(m.e[0], m.e[4], m.e[1], m.e[3]);
    return m;
}

__device__ __forceinline__ int nbr(int x, int L, int d, int step) {
    int c[3] = {x % L, (x / L) % L, x / (L * L)};
    c[d] += step;
    c[d] = c[d] < 0 ? c[d] + L : (c[d] >= L ? c[d] - L : c[d]);
    return c[0] + L * (c[1] + L * c[2]);
}

// ------------------------------------------------------------ su(3) algebra level

// The 8 components of a traceless anti-Hermitian matrix, ordered as stored.
struct A8 {
    float c[8];
};

__device__ __forceinline__ A8 ldA8(const float* base, size_t V3, int x) {
    A8 a;
#pragma unroll
    for (int e = 0; e < 8; ++e) a.c[e] = gld(base + (size_t)e * V3 + x);
    return a;
}
__device__ __forceinline__ void stA8(float* base, size_t V3, int x, const A8& a) {
#pragma unroll
    for (int e = 0; e < 8; ++e) base[(size_t)e * V3 + x] = a.c[e];
}

// Components of w v^H (CONJ_RIGHT) or w v for a product that is traceless anti-Hermitian
// in exact arithmetic (u X u^H and u^H X u for X in su(3)): the imaginary diagonal, the
// three upper entries, trace removed; the lower entries are not formed.
template <bool CONJ_RIGHT>
__device__ __forceinline__ A8 alg_of_product(const M3& w, const M3& v) {
    auto entry = [&](int i, int j) {
        float2 r = make_float2(0.f, 0.f);
#pragma unroll
        for (int k = 0; k < 3; ++k) r = CONJ_RIGHT ? cfma_conj_b(w.e[3 * i + k], v.e[3 * j + k], r)
                                                   : cfma(w.e[3 * i + k], v.e[3 * k + j], r);
        return r;
    };
    auto diag_im = [&](int i) {
        float r = 0.f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float2 a = w.e[3 * i + k];
            const float2 b = CONJ_RIGHT ? make_float2(v.e[3 * i + k].x, -v.e[3 * i + k].y) : v.e[3 * k + i];
            r += a.x * b.y + a.y * b.x;
        }
        return r;
    };
    const float y0 = diag_im(0), y1 = diag_im(1), y2 = diag_im(2);
    const float t = (y0 + y1 + y2) * (1.f / 3.f);
    const float2 e01 = entry(0, 1), e02 = entry(0, 2), e12 = entry(1, 2);
    return A8{{y0 - t, y1 - t, e01.x, e01.y, e02.x, e02.y, e12.x, e12.y}};
}

// (D_j X)(x) at the algebra level for X stored as components ([8][V3]):
// 1/2 [U_j(x) X(x+j) U_j(x)^H - U_j(x-j)^H X(x-j) U_j(x-j)], with the links u = U_j(x),
// ub = U_j(x-j) and the neighbours xf = x+j, xb = x-j given (callers take every
// difference along one direction from one load of its two links).
__device__ __forceinline__ A8 adjoint_diff_links(const M3& u, const M3& ub, const float* X, size_t V3, int xf,
                                                 int xb) {
    const A8 up = alg_of_product<true>(mul(u, ldA(X, V3, xf)), u);
    const A8 dn = alg_of_product<false>(hmul(ub, ldA(X, V3, xb)), ub);
    A8 r;
#pragma unroll
    for (int e = 0; e < 8; ++e) r.c[e] = 0.5f * (up.c[e] - dn.c[e]);
    return r;
}


// Tr(B Y) of two traceless anti-Hermitian matrices (real): with B_ii = i b_i and
// B_ji = -conj(B_ij), Tr(B Y) = -sum_i b_i y_i - 2 sum_{i<j} Re(B_ij conj(Y_ij)).
__device__ __forceinline__ double trace_alg(const A8& b, const A8& y) {
    const double b0 = b.c[0], b1 = b.c[1], y0 = y.c[0], y1 = y.c[1];
    double r = -(b0 * y0 + b1 * y1 + (b0 + b1) * (y0 + y1));
#pragma unroll
    for (int e = 2; e < 8; e += 2) r -= 2.0 * ((double)b.c[e] * y.c[e] + (double)b.c[e + 1] * y.c[e + 1]);
    return r;
}

// ------------------------------------------------------------------ kernels

struct GlueArgs {
    const float2* links;  // [nc][T][V3][3][3][3] (caller's layout)
    float2* U;            // [nct][3][6][V3]: the first two rows of each link
    float* F;             // [nct][kNField][8][V3]: the algebra components of each field
    double2* part;        // [nct][nblk][5]
    double2* ops;         // [nc][T][5]
    const int4* tasks;    // (in field, direction, out field, 0)
    int ntask;
    int L, V3, nct, nblk;
};

// The caller's links, [V3][3][3][3] per (configuration, timeslice), to the 18 planes
// [3][6][V3] of their first two rows (the third is rebuilt where it is used). One
// workgroup moves kLinkSites sites through LDS: the sites' 27 values each are read as
// one contiguous run, and each plane is written as a run of consecutive sites.
constexpr int kLinkSites = 64;

__global__ __launch_bounds__(256) void glue_links_kernel(GlueArgs a) {
    __shared__ float2 st[kLinkSites * 27];  // site stride 27 (odd): conflict-free column reads
    const int nb = (a.V3 + kLinkSites - 1) / kLinkSites;
    const int ct = blockIdx.x / nb;
    const int x0 = (blockIdx.x - ct * nb) * kLinkSites;
    const int ns = min(kLinkSites, a.V3 - x0);
    const float2* src = a.links + ((size_t)ct * a.V3 + x0) * 27;
    for (int i = threadIdx.x; i < ns * 27; i += 256) st[i] = gld(src + i);
    __syncthreads();
    for (int i = threadIdx.x; i < 18 * kLinkSites; i += 256) {
        const int q = i / kLinkSites, sx = i - q * kLinkSites;  // plane q = 6 d + el
        if (sx < ns) {
            const int d = q / 6, el = q - 6 * d;
            a.U[((size_t)ct * 18 + q) * a.V3 + x0 + sx] = st[sx * 27 + 9 * d + el];
        }
    }
}

// F_mn(x) = (Q - Q^H) / 8, traceless; Q the sum of the four leaves in the (m, n) plane
__device__ M3 clover(const float2* U, int L, size_t V3, int x, int m, int n) {
    const float2* Um = U + (size_t)m * 6 * V3;
    const float2* Un = U + (size_t)n * 6 * V3;
    const int xpm = nbr(x, L, m, 1), xpn = nbr(x, L, n, 1), xmm = nbr(x, L, m, -1), xmn = nbr(x, L, n, -1);
    const int xmm_pn = nbr(xmm, L, n, 1), xmm_mn = nbr(xmm, L, n, -1), xpm_mn = nbr(xpm, L, n, -1);
    // x -> x+m -> x+m+n -> x+n -> x:  U_m(x) U_n(x+m) U_m(x+n)^H U_n(x)^H
    const M3 q = mul_h(mul_h(mul(ldU(Um, V3, x), ldU(Un, V3, xpm)), ldU(Um, V3, xpn)), ldU(Un, V3, x));
    // x -> x+n -> x-m+n -> x-m -> x:  U_n(x) U_m(x-m+n)^H U_n(x-m)^H U_m(x-m)
    const M3 l2 = mul(mul_h(mul_h(ldU(Un, V3, x), ldU(Um, V3, xmm_pn)), ldU(Un, V3, xmm)), ldU(Um, V3, xmm));
    // x -> x-m -> x-m-n -> x-n -> x:  U_m(x-m)^H U_n(x-m-n)^H U_m(x-m-n) U_n(x-n)
    //                                = (U_n(x-m-n) U_m(x-m))^H U_m(x-m-n) U_n(x-n)
    const M3 l3 = mul(hmul(mul(ldU(Un, V3, xmm_mn), ldU(Um, V3, xmm)), ldU(Um, V3, xmm_mn)), ldU(Un, V3, xmn));
    // x -> x-n -> x+m-n -> x+m -> x:  U_n(x-n)^H U_m(x-n) U_n(x+m-n) U_m(x)^H
    const M3 l4 = mul_h(mul(hmul(ldU(Un, V3, xmn), ldU(Um, V3, xmn)), ldU(Un, V3, xpm_mn)), ldU(Um, V3, x));
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

// The stencil kernels run 1D grids over (configuration-timeslice, site block[, task]) in
// that order, remapped so each XCD takes one contiguous range: the neighbour blocks a
// site block reads (x +- e_2 lies 2-3 blocks away at L = 24) are then in the same L2.
__global__ __launch_bounds__(256) void glue_clover_kernel(GlueArgs a) {
    const int bid = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int ct = bid / a.nblk, x = (bid - ct * a.nblk) * 256 + threadIdx.x;
    if (x >= a.V3) return;
    const size_t V3 = a.V3;
    const float2* U = a.U + (size_t)ct * 18 * V3;
    float* F = a.F + (size_t)ct * kNField * 8 * V3;
    // B_0 = 2 F_12, B_1 = 2 F_20, B_2 = 2 F_01
    const int pl[3][2] = {{1, 2}, {2, 0}, {0, 1}};
#pragma unroll 1
    for (int i = 0; i < 3; ++i) {
        M3 f = clover(U, a.L, V3, x, pl[i][0], pl[i][1]);
#pragma unroll
        for (int e = 0; e < 9; ++e) f.e[e] = make_float2(2.f * f.e[e].x, 2.f * f.e[e].y);
        stA(F + (size_t)(F_B + i) * 8 * V3, V3, x, f);
    }
}

// One work item per (configuration-timeslice, site block, direction); a task is (in
// field, direction, out field), and a level's tasks are listed direction by direction,
// ntask / 3 each. A thread loads the two links of its direction (rebuilding their third
// rows) once and takes every task of that direction at its site.
__global__ __launch_bounds__(256) void glue_deriv_kernel(GlueArgs a) {
    const int bid = (int)xcd_remap(blockIdx.x, gridDim.x);  // (ct, site block, direction)
    const int dir = bid % 3, r = bid / 3;
    const int ct = r / a.nblk, x = (r - ct * a.nblk) * 256 + threadIdx.x;
    if (x >= a.V3) return;
    const size_t V3 = a.V3;
    const float2* Uj = a.U + ((size_t)ct * 3 + dir) * 6 * V3;
    const int xf = nbr(x, a.L, dir, 1), xb = nbr(x, a.L, dir, -1);
    const M3 u = ldU(Uj, V3, x);
    const M3 ub = ldU(Uj, V3, xb);
    const int per = a.ntask / 3;
    for (int t = dir * per; t < (dir + 1) * per; ++t) {
        const int4 tk = a.tasks[t];
        const float* X = a.F + ((size_t)ct * kNField + tk.x) * 8 * V3;
        stA8(a.F + ((size_t)ct * kNField + tk.z) * 8 * V3, V3, x, adjoint_diff_links(u, ub, X, V3, xf, xb));
    }
}

__device__ __forceinline__ double2 dadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 dscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }

__global__ __launch_bounds__(256, 2) void glue_contract_kernel(GlueArgs a) {
    __shared__ double2 red[256 / 64][kNOp];
    const int bid = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int ct = bid / a.nblk, xb = bid - ct * a.nblk, x = xb * 256 + threadIdx.x;
    const size_t V3 = a.V3;
    const float* F = a.F + (size_t)ct * kNField * 8 * V3;
    const float2* U = a.U + (size_t)ct * 18 * V3;
    double2 o[kNOp];
#pragma unroll
    for (int n = 0; n < kNOp; ++n) o[n] = make_double2(0.0, 0.0);
    if (x < a.V3) {
        // loops kept rolled, the loop indices only ever address memory. By direction j of
        // the third D: its two links are loaded (third rows rebuilt) once for the six
        // differences taken along it
#pragma unroll 1
        for (int j = 0; j < 3; ++j) {
            const float2* Uj = U + (size_t)j * 6 * V3;
            const int xf = nbr(x, a.L, j, 1), xbk = nbr(x, a.L, j, -1);
            const M3 u = ldU(Uj, V3, x);
            const M3 ub = ldU(Uj, V3, xbk);
#pragma unroll 1
            for (int s = 0; s < 2; ++s) {  // eps_ijk = +1 for (i, k) = (j+2, j+1), -1 for (j+1, j+2)
                const int i = s == 0 ? (j + 2) % 3 : (j + 1) % 3, k = s == 0 ? (j + 1) % 3 : (j + 2) % 3;
                const double e = s == 0 ? 1.0 : -1.0;
                const int pjk = pair_index(j, k);
                const A8 Bi = ldA8(F + (size_t)(F_B + i) * 8 * V3, V3, x);
                // traces of two su(3) fields are real
                o[0].x += e * trace_alg(Bi, ldA8(F + (size_t)(F_DB + pjk) * 8 * V3, V3, x));
                // the third D on the fly: D_j^3 B_k, D_j^2 D_k B_j, D_j D_i^2 B_k
                o[2].x += e * trace_alg(Bi, adjoint_diff_links(u, ub, F + (size_t)(F_S1 + pjk) * 8 * V3, V3, xf, xbk));
                o[3].x += e * trace_alg(Bi, adjoint_diff_links(u, ub, F + (size_t)(F_S2 + pjk) * 8 * V3, V3, xf, xbk));
                o[4].x += e * trace_alg(Bi, adjoint_diff_links(u, ub, F + (size_t)(F_S1 + pair_index(i, k)) * 8 * V3,
                                                               V3, xf, xbk));
            }
        }
        // O2 through eps_ijk eps_ilm = d_jl d_km - d_jm d_kl:
        //   sum_{j != k} Tr(B_j B_k D_j B_k) - Tr(B_j B_k D_k B_j)
#pragma unroll 1
        for (int j = 0; j < 3; ++j) {
            const M3 Bj = ldA(F + (size_t)(F_B + j) * 8 * V3, V3, x);
#pragma unroll 1
            for (int k = 0; k < 3; ++k) {
                if (k == j) continue;
                const M3 bb = mul(Bj, ldA(F + (size_t)(F_B + k) * 8 * V3, V3, x));
                const double2 t1 = trace_prod(bb, ldA(F + (size_t)(F_DB + pair_index(j, k)) * 8 * V3, V3, x));
                const double2 t2 = trace_prod(bb, ldA(F + (size_t)(F_DB + pair_index(k, j)) * 8 * V3, V3, x));
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
        a.part[((size_t)ct * a.nblk + xb) * kNOp + threadIdx.x] = s;
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

// The derivative tasks of the two stored levels (the third D is taken in the contraction),
// direction by direction: 2 per direction at the first level, 4 at the second.
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
    const size_t per_ct = (size_t)18 * V3 * sizeof(float2) + (size_t)kNField * 8 * V3 * sizeof(float) +
                          (size_t)nblk * kNOp * sizeof(double2);
    const size_t cap = ctx->budget ? std::min(kGlueCap, ctx->budget / 2) : kGlueCap;
    const long long total_ct = (long long)nconf * T;
    // (configuration, timeslice) pairs per round: within the workspace cap and the 1D
    // grid of the difference kernel (site blocks x 12 tasks x pairs below 2^31)
    const long long grid_cap = (long long)(INT32_MAX / (12LL * nblk));
    const long long fit =
        std::max<long long>(1, std::min<long long>({total_ct, (long long)(cap / per_ct), grid_cap, 65535LL}));
    const long long rounds = (total_ct + fit - 1) / fit;  // equal rounds, no small last one
    const int nct_max = (int)((total_ct + rounds - 1) / rounds);
    std::vector<int4> l1, l2;
    make_tasks(l1, l2);
    for (const std::vector<int4>* lv : {&l1, &l2})  // the difference kernel reads them by direction
        for (size_t t = 0; t < lv->size(); ++t)
            if (lv->size() % 3 != 0 || (*lv)[t].y != (int)(t / (lv->size() / 3)))
                return fail(ctx, NUC_ERR_INTERNAL, "difference tasks not grouped by direction");
    HostBlock hb;
    const size_t off1 = hb.add(l1.data(), l1.size() * sizeof(int4));
    const size_t off2 = hb.add(l2.data(), l2.size() * sizeof(int4));
    const size_t off_U = align_up(hb.bytes.size(), 256);
    const size_t off_F = off_U + align_up((size_t)nct_max * 18 * V3 * sizeof(float2), 256);
    const size_t off_P = off_F + align_up((size_t)nct_max * kNField * 8 * V3 * sizeof(float), 256);
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
        a.F = (float*)(base + off_F);
        a.part = (double2*)(base + off_P);
        a.ops = (double2*)ops + (size_t)c0 * kNOp;
        a.L = L;
        a.V3 = V3;
        a.nct = nct;
        a.nblk = nblk;
        const size_t nl = (size_t)nct * ((V3 + kLinkSites - 1) / kLinkSites);
        HIPCHK(ctx, timed_launch(ctx, NUC_K_GLUE_STENCIL, s, [&] {
                   hipLaunchKernelGGL(glue_links_kernel, dim3((unsigned)nl), dim3(256), 0, s, a);
                   return hipGetLastError();
               }));
        HIPCHK(ctx, timed_launch(ctx, NUC_K_GLUE_STENCIL, s, [&] {
                   hipLaunchKernelGGL(glue_clover_kernel, dim3((unsigned)((size_t)nblk * nct)), dim3(256), 0, s, a);
                   return hipGetLastError();
               }));
        const std::vector<int4>* lv[2] = {&l1, &l2};
        const size_t offs[2] = {off1, off2};
        for (int l = 0; l < 2; ++l) {
            a.tasks = (const int4*)(base + offs[l]);
            a.ntask = (int)lv[l]->size();
            HIPCHK(ctx, timed_launch(ctx, NUC_K_GLUE_STENCIL, s, [&] {
                       hipLaunchKernelGGL(glue_deriv_kernel, dim3((unsigned)((size_t)nblk * 3 * nct)), dim3(256),
                                          0, s, a);
                       return hipGetLastError();
                   }));
        }
        HIPCHK(ctx, timed_launch(ctx, NUC_K_GLUE_CONTRACT, s, [&] {
                   hipLaunchKernelGGL(glue_contract_kernel, dim3((unsigned)((size_t)nblk * nct)), dim3(256), 0, s, a);
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

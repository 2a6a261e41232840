// Baryon elementals on CDNA4 MFMA (paper Section 2.1: the nucleon elementals
// Phi[p,t]_ijk that the distillation profiles then reweight).
//
//   Phi[p,t]_ijk = sum_{x,a} v_i^a(x) B_p[(x,a), jk],
//   B_p[(x,a), jk] = exp(-i p.x) W_jk^a(x),   W_jk^a(x) = eps_abc v_j^b(x) v_k^c(x)   (j < k)
//
// is a complex GEMM with rows i, columns the pairs j<k and the reduction over
// (site, colour). Only i < j < k is wanted. A workgroup owns 64 consecutive
// pairs of the job's pair list (16 per wave) and up to four row tiles of 16 i.
// Below 20 vectors the list holds every pair in lexicographic order and a wave
// takes the row tiles below the largest j of its pairs. From 20 vectors on it is
// the block pair set (elem_block_pairs), ordered by the row tiles each pair needs:
// pairs inside a 16-index block with every row tile (a row beyond the block is
// then the triple's largest index, Phi_rjk = Phi_jkr) and pairs across blocks
// with the tiles below j's block only, which leaves out the idle half of the
// diagonal tiles and about half the cross products. Each colour cross product
// is built once per (site, colour, pair, momentum) and feeds those row tiles;
// the momentum phase rides on that operand, and the eigenvectors v_i are read
// from LDS as they are. Neither operand is stored in HBM: each workgroup stages
// the eigenvectors of a block of 16 sites in LDS (prefetching the next block
// into registers while the current one is consumed). The K order is (site
// group of 4, colour), so every LDS address is a per-lane base plus a
// compile-time offset.
//
// Each block of 16 sites is summed in FP32 MFMA accumulators (for 17..32 vectors
// with three real products per complex one, Gauss's form) and folded into
// per-lane FP64 sums; a workgroup stores the canonical entries (i<j<k) of its
// range of sites in FP64, the reduce kernel adds the ranges in FP64 (fixed
// order) and the expand kernel writes the dense, exactly antisymmetric output.
#include <type_traits>

#include "nuc_internal.h"

namespace nuc {
namespace {

constexpr int CS = 16;              // sites per LDS block
constexpr int ROW3 = CS * 3;        // (site, colour) values per vector and block
// LDS row pitch of a vector (complex): 2 mod 32 in 8-byte units, so the 32
// lanes of a half-wave reading rows col (0..15) at offsets 3 g (g = 0, 1) hit
// 32 different 8-byte slots of the 256-byte bank row (a pitch of 48 puts 16
// rows on 2 slots)
constexpr int RS = ROW3 + 2;
constexpr int MAXP = 4;             // most momenta sharing one cross-product operand
constexpr int MAXNIT = 4;           // row tiles per workgroup (i chunks of 64 beyond that)

__device__ __forceinline__ long long choose3(long long k) { return k * (k - 1) * (k - 2) / 6; }
__device__ __forceinline__ long long choose2(long long j) { return j * (j - 1) / 2; }

// Momenta per workgroup a row-tile count allows (accumulators grow with both).
constexpr int mp_max(int nit) { return nit <= 1 ? MAXP : nit <= 3 ? 2 : 1; }

// Complex products in Gauss's three-multiplication form (t1 = sum vr wr, t2 = sum vi wi,
// t3 = sum (vr + vi)(wr + wi); Phi = (t1 - t2) + i (t3 - t1 - t2), combined in FP64 at the
// fold) for the 17..32-vector class (two row tiles), where the third accumulator set keeps
// two waves per SIMD without spilling; the other classes keep four real products.
constexpr bool gauss3(int nit) { return nit == 2; }

// One colour term of the cross product, jb kc - jc kb, as two four-operation FMA chains.
__device__ __forceinline__ float2 cross_term(float2 jb, float2 kc, float2 jc, float2 kb) {
    const float re = fmaf(jb.x, kc.x, fmaf(-jb.y, kc.y, fmaf(-jc.x, kb.x, jc.y * kb.y)));
    const float im = fmaf(jb.x, kc.y, fmaf(jb.y, kc.x, fmaf(-jc.x, kb.y, -(jc.y * kb.x))));
    return make_float2(re, im);
}

// MFMAs of one staged block of CS sites for a wave with NI row tiles and NP momenta
// (compile-time, so the loop carries no per-tile or per-momentum branches). The colour
// cross product of the wave's pair is formed once per (site, colour) and multiplied by
// each momentum's phase; vi is read from LDS as staged.
template <int NIT, int MP, int NI, int NP>
__device__ __forceinline__ void elem_block(const float2* bj, const float2* bk, const float2* bi, const float2* sph,
                                           int g, floatx4 (&cr)[NIT][MP], floatx4 (&ci)[NIT][MP],
                                           floatx4 (&c3)[NIT][MP]) {
    // one site group; with zero, the block's first MFMA of each accumulator takes a zero
    // accumulator operand, so the accumulators need no clearing between blocks
    auto group = [&](int sg, auto zero) __attribute__((always_inline)) {
        constexpr bool Z = decltype(zero)::value;
        const floatx4 z4 = floatx4{0.f, 0.f, 0.f, 0.f};
        float2 ph[NP];
#pragma unroll
        for (int r = 0; r < NP; ++r) ph[r] = sph[r * CS + 4 * sg + g];
#pragma unroll
        for (int ca = 0; ca < 3; ++ca) {
            const int cb = (ca + 1) % 3, cc = (ca + 2) % 3;
            const int o = 12 * sg;
            const float2 jb = bj[o + cb], kc = bk[o + cc], jc = bj[o + cc], kb = bk[o + cb];
            const float2 wjk = cross_term(jb, kc, jc, kb);
            float2 bw[NP];
#pragma unroll
            for (int r = 0; r < NP; ++r) bw[r] = cmul(ph[r], wjk);
            float2 vi[NI];
#pragma unroll
            for (int it = 0; it < NI; ++it) vi[it] = bi[it * 16 * RS + o + ca];
            if constexpr (gauss3(NIT)) {
#pragma unroll
                for (int it = 0; it < NI; ++it) {
                    const float vs = vi[it].x + vi[it].y;
#pragma unroll
                    for (int r = 0; r < NP; ++r) {
                        cr[it][r] = mfma16x4(vi[it].x, bw[r].x, Z && ca == 0 ? z4 : cr[it][r]);
                        ci[it][r] = mfma16x4(vi[it].y, bw[r].y, Z && ca == 0 ? z4 : ci[it][r]);
                        c3[it][r] = mfma16x4(vs, bw[r].x + bw[r].y, Z && ca == 0 ? z4 : c3[it][r]);
                    }
                }
            } else {
                // two passes, so that an accumulator's second MFMA comes 2 NI NP MFMAs after its
                // first instead of right behind it (each accumulator sums its terms in the
                // same order as a single pass)
#pragma unroll
                for (int it = 0; it < NI; ++it)
#pragma unroll
                    for (int r = 0; r < NP; ++r) {
                        cr[it][r] = mfma16x4(vi[it].x, bw[r].x, Z && ca == 0 ? z4 : cr[it][r]);
                        ci[it][r] = mfma16x4(vi[it].x, bw[r].y, Z && ca == 0 ? z4 : ci[it][r]);
                    }
#pragma unroll
                for (int it = 0; it < NI; ++it)
#pragma unroll
                    for (int r = 0; r < NP; ++r) {
                        cr[it][r] = mfma16x4(-vi[it].y, bw[r].y, cr[it][r]);
                        ci[it][r] = mfma16x4(vi[it].y, bw[r].x, ci[it][r]);
                    }
            }
        }
    };
    group(0, std::true_type{});
#pragma unroll 1
    for (int sg = 1; sg < CS / 4; ++sg) group(sg, std::false_type{});
}

// The same block with the wave's row tiles nit taken at run time and every momentum
// slot of the group computed (a short last group leaves its extra accumulators unused):
// for the larger tile counts, where one specialisation per (nit, np) would raise
// register use past the point of spilling.
template <int NIT, int MP>
__device__ __forceinline__ void elem_block_generic(int nit, int, const float2* bj, const float2* bk,
                                                   const float2* bi, const float2* sph, int g,
                                                   floatx4 (&cr)[NIT][MP], floatx4 (&ci)[NIT][MP],
                                                   floatx4 (&c3)[NIT][MP]) {
#pragma unroll 1
    for (int sg = 0; sg < CS / 4; ++sg) {
        float2 ph[MP];
#pragma unroll
        for (int r = 0; r < MP; ++r) ph[r] = sph[r * CS + 4 * sg + g];
#pragma unroll
        for (int ca = 0; ca < 3; ++ca) {
            const int cb = (ca + 1) % 3, cc = (ca + 2) % 3;
            const int o = 12 * sg;
            const float2 jb = bj[o + cb], kc = bk[o + cc], jc = bj[o + cc], kb = bk[o + cb];
            const float2 wjk = cross_term(jb, kc, jc, kb);
            float2 bw[MP];
#pragma unroll
            for (int r = 0; r < MP; ++r) bw[r] = cmul(ph[r], wjk);
            if constexpr (gauss3(NIT)) {
#pragma unroll
                for (int it = 0; it < NIT; ++it) {
                    if (it >= nit) break;
                    const float2 vi = bi[it * 16 * RS + o + ca];
                    const float vs = vi.x + vi.y;
#pragma unroll
                    for (int r = 0; r < MP; ++r) {
                        cr[it][r] = mfma16x4(vi.x, bw[r].x, cr[it][r]);
                        ci[it][r] = mfma16x4(vi.y, bw[r].y, ci[it][r]);
                        c3[it][r] = mfma16x4(vs, bw[r].x + bw[r].y, c3[it][r]);
                    }
                }
            } else {
                // two passes, as in elem_block (v_i read from LDS in each)
#pragma unroll
                for (int it = 0; it < NIT; ++it) {
                    if (it >= nit) break;
                    const float vx = bi[it * 16 * RS + o + ca].x;
#pragma unroll
                    for (int r = 0; r < MP; ++r) {
                        cr[it][r] = mfma16x4(vx, bw[r].x, cr[it][r]);
                        ci[it][r] = mfma16x4(vx, bw[r].y, ci[it][r]);
                    }
                }
#pragma unroll
                for (int it = 0; it < NIT; ++it) {
                    if (it >= nit) break;
                    const float vy = bi[it * 16 * RS + o + ca].y;
#pragma unroll
                    for (int r = 0; r < MP; ++r) {
                        cr[it][r] = mfma16x4(-vy, bw[r].y, cr[it][r]);
                        ci[it][r] = mfma16x4(vy, bw[r].x, ci[it][r]);
                    }
                }
            }
        }
    }
}

// The FP64 form of one staged block: the colour cross product and its phase in FP64
// (a product of two FP32 eigenvector components is exact there), FP64 MFMAs on the
// FP32 vectors, and the accumulators carried over the workgroup's whole site range.
template <int NIT, int MP>
__device__ __forceinline__ void elem_block_f64(int nit, const float2* bj, const float2* bk, const float2* bi,
                                               const double2* sph, int g, doublex4 (&xr)[NIT][MP],
                                               doublex4 (&xi)[NIT][MP]) {
#pragma unroll 1
    for (int sg = 0; sg < CS / 4; ++sg) {
        double2 ph[MP];
#pragma unroll
        for (int r = 0; r < MP; ++r) ph[r] = sph[r * CS + 4 * sg + g];
#pragma unroll
        for (int ca = 0; ca < 3; ++ca) {
            const int cb = (ca + 1) % 3, cc = (ca + 2) % 3;
            const int o = 12 * sg;
            const float2 jb = bj[o + cb], kc = bk[o + cc], jc = bj[o + cc], kb = bk[o + cb];
            const double wr = ((double)jb.x * kc.x - (double)jb.y * kc.y) - ((double)jc.x * kb.x - (double)jc.y * kb.y);
            const double wi = ((double)jb.x * kc.y + (double)jb.y * kc.x) - ((double)jc.x * kb.y + (double)jc.y * kb.x);
            double br[MP], bim[MP];
#pragma unroll
            for (int r = 0; r < MP; ++r) {
                br[r] = ph[r].x * wr - ph[r].y * wi;
                bim[r] = ph[r].x * wi + ph[r].y * wr;
            }
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                if (it >= nit) break;
                const float2 vi = bi[it * 16 * RS + o + ca];
#pragma unroll
                for (int r = 0; r < MP; ++r) cmac((double)vi.x, (double)vi.y, br[r], bim[r], xr[it][r], xi[it][r]);
            }
        }
    }
}

// Select the specialisation for the wave's row tiles nit (1..NIT) and the group's
// momenta np (1..MP); both are wave-uniform.
template <int NIT, int MP, int NI, int NP>
__device__ __forceinline__ void elem_dispatch_np(int np, const float2* bj, const float2* bk, const float2* bi,
                                                 const float2* sph, int g, floatx4 (&cr)[NIT][MP],
                                                 floatx4 (&ci)[NIT][MP], floatx4 (&c3)[NIT][MP]) {
    if constexpr (NP > 1) {
        if (np < NP) {
            elem_dispatch_np<NIT, MP, NI, NP - 1>(np, bj, bk, bi, sph, g, cr, ci, c3);
            return;
        }
    }
    elem_block<NIT, MP, NI, NP>(bj, bk, bi, sph, g, cr, ci, c3);
}

template <int NIT, int MP, int NI>
__device__ __forceinline__ void elem_dispatch_ni(int nit, int np, const float2* bj, const float2* bk, const float2* bi,
                                                 const float2* sph, int g, floatx4 (&cr)[NIT][MP],
                                                 floatx4 (&ci)[NIT][MP], floatx4 (&c3)[NIT][MP]) {
    if constexpr (NI > 1) {
        if (nit < NI) {
            elem_dispatch_ni<NIT, MP, NI - 1>(nit, np, bj, bk, bi, sph, g, cr, ci, c3);
            return;
        }
    }
    elem_dispatch_np<NIT, MP, NI, MP>(np, bj, bk, bi, sph, g, cr, ci, c3);
}

// F64: the FP64 form (elem_block_f64), whose phases are FP64 too.
template <int NPF, int NIT, int MP, bool F64>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void elem_kernel(BatchRef bt) {
    // NPF: prefetch registers, N ROW3 values / 256 threads rounded up
    typedef std::conditional_t<F64, double2, float2> Ph;
    extern __shared__ float2 smem[];
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    const int inst = find_inst(bt.offs, bt.ninst, item);
    const ElemLaunch a = reinterpret_cast<const ElemLaunch*>(bt.descs)[inst];  // by value: read once
    float2* sv = smem;                    // [256 NPF / ROW3][RS]
    Ph* sph = reinterpret_cast<Ph*>(sv + 256 * NPF / ROW3 * RS);  // [MP][CS]
    Ph* tab = sph + MP * CS;              // [L]  exp(-2 pi i m / L)
    float2* zrow = reinterpret_cast<float2*>(tab + 256);  // [RS] zeros: the vectors of lanes past the last pair

    unsigned bid = item - bt.offs[inst];
    const int w = bid % a.nwork;
    bid /= a.nwork;
    const int pg = bid % a.npgroup;
    bid /= a.npgroup;
    const int split = bid % a.nsplit;
    bid /= a.nsplit;
    const int tl = bid;
    const int t = a.t_off + tl;

    const int ichunk = a.work[w].x, pblock = a.work[w].y;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 15, g = lane >> 4;
    const int q = pblock * 64 + wv * 16 + col;
    const bool qok = q < a.npairs;
    const int2 pr = a.pairs[qok ? q : 0];
    // row tiles of this wave: from the smallest first tile of its 16 pairs to their
    // largest end (the pairs are ordered by row range, so a wave mostly has one), in
    // chunks of MAXNIT; a pair stores only the rows it owns
    const int q0 = pblock * 64 + wv * 16;
    int it0 = 0, nit = 0;
    if (q0 < a.npairs) {
        int rb = 1 << 30, re = 0;
        for (int i = 0; i < 16; ++i) {
            const int2 r = elem_row_range(a.N, a.pairs[min(q0 + i, a.npairs - 1)]);
            rb = min(rb, r.x);
            re = max(re, r.y);
        }
        it0 = rb + ichunk * MAXNIT;
        nit = min(NIT, re - it0);
    }
    it0 = __builtin_amdgcn_readfirstlane(it0);
    nit = __builtin_amdgcn_readfirstlane(max(nit, 0));
    const int p0 = pg * MP;
    const int np = __builtin_amdgcn_readfirstlane(min(MP, a.nmom - p0));  // momenta in this group

    for (int m = threadIdx.x; m < a.L; m += 256) {
        double sn, cs;
        sincospi(2.0 * (double)m / (double)a.L, &sn, &cs);
        if constexpr (F64)
            tab[m] = make_double2(cs, -sn);
        else
            tab[m] = make_float2((float)cs, (float)(-sn));
    }

    // accumulators of one site block: real and imaginary parts, or t1, t2, t3 (gauss3)
    floatx4 cr[NIT][MP], ci[NIT][MP], c3[NIT][MP];
    double dr[NIT][MP][4], di[NIT][MP][4];
    doublex4 xr[NIT][MP], xi[NIT][MP];  // F64: accumulators over the whole site range
#pragma unroll
    for (int it = 0; it < NIT; ++it)
#pragma unroll
        for (int r = 0; r < MP; ++r) {
            xr[it][r] = doublex4{0.0, 0.0, 0.0, 0.0};
            xi[it][r] = doublex4{0.0, 0.0, 0.0, 0.0};
            cr[it][r] = floatx4{0.f, 0.f, 0.f, 0.f};
            ci[it][r] = floatx4{0.f, 0.f, 0.f, 0.f};
            c3[it][r] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int v = 0; v < 4; ++v) dr[it][r][v] = di[it][r][v] = 0.0;
        }

    const int s_begin = split * a.sites_per_split;
    const int s_end = min(a.V3, s_begin + a.sites_per_split);
    const float2* vt = a.evecs + (size_t)t * a.ev_tstride;
    const int nval = a.N * ROW3;

    // prefetch of one site block: element idx = threadIdx.x + 256 r is value
    // e = idx % ROW3 (site e / 3, colour e % 3) of vector idx / ROW3. Loads are
    // unconditional (clamped index); the mask is applied at the LDS write.
    float2 pf[NPF];
    int pf_off[NPF];
#pragma unroll
    for (int r = 0; r < NPF; ++r) {
        const int idx = threadIdx.x + 256 * r;
        const int n = idx / ROW3, e = idx - n * ROW3;
        pf_off[r] = (idx < nval) ? n * a.V3 * 3 + e : -1;
    }
#define NUC_PREFETCH(c0_)                                                             \
    {                                                                                 \
        const int ns3_ = min(CS, s_end - (c0_)) * 3;                                  \
        _Pragma("unroll") for (int r = 0; r < NPF; ++r) {                             \
            const int e_ = (threadIdx.x + 256 * r) % ROW3;                            \
            const bool ok_ = pf_off[r] >= 0 && e_ < ns3_;                             \
            pf[r] = gld(vt + (ok_ ? pf_off[r] + 3 * (c0_) : 0));                      \
        }                                                                             \
    }
    if (s_begin < s_end) NUC_PREFETCH(s_begin);

    // per-lane LDS bases: site 4*sg + g, colour c  ->  offset 12*sg + 3*g + c
    for (int m = threadIdx.x; m < RS; m += 256) zrow[m] = make_float2(0.f, 0.f);
    const float2* bj = (qok ? sv + pr.x * RS : zrow) + 3 * g;
    const float2* bk = (qok ? sv + pr.y * RS : zrow) + 3 * g;
    const float2* bi = sv + (16 * it0 + arow(col, F64)) * RS + 3 * g;  // row tile it adds 16 it RS

    for (int c0 = s_begin; c0 < s_end; c0 += CS) {
        const int ns = min(CS, s_end - c0);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NPF; ++r) {
            const int idx = threadIdx.x + 256 * r;
            const int n = idx / ROW3, e = idx - n * ROW3;
            const float m = (pf_off[r] >= 0 && e < 3 * ns) ? 1.f : 0.f;  // finite inputs: zero outside
            sv[n * RS + e] = make_float2(pf[r].x * m, pf[r].y * m);
        }
        if (threadIdx.x < MP * CS) {
            const int r = threadIdx.x / CS, s = threadIdx.x % CS;
            Ph ph{};
            if (r < np && s < ns) {
                const int x = c0 + s;
                const int x0 = x % a.L, x1 = (x / a.L) % a.L, x2 = x / (a.L * a.L);
                const int* n = a.mom + 3 * (p0 + r);
                int m = (n[0] * x0 + n[1] * x1 + n[2] * x2) % a.L;
                if (m < 0) m += a.L;
                ph = tab[m];
            }
            sph[threadIdx.x] = ph;
        }
        __syncthreads();
        if (c0 + CS < s_end) NUC_PREFETCH(c0 + CS);
        if (nit == 0) continue;
        // per-(nit, np) bodies: faster for N <= 32 and N = 64 (measured), but for the
        // 48-vector and the deep-prefetch classes they spill, so those keep one body
        if constexpr (F64) {
            elem_block_f64<NIT, MP>(nit, bj, bk, bi, sph, g, xr, xi);
            continue;
        } else if constexpr (NPF <= 12 && NIT != 3) {
            elem_dispatch_ni<NIT, MP, NIT>(nit, np, bj, bk, bi, sph, g, cr, ci, c3);
        } else {
            elem_block_generic<NIT, MP>(nit, np, bj, bk, bi, sph, g, cr, ci, c3);
        }
        // fold each block of sites (48 FP32 terms per lane) into the FP64 sums
        if constexpr (!F64) {
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                if (it >= nit) break;
#pragma unroll
                for (int r = 0; r < MP; ++r) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        if constexpr (gauss3(NIT)) {
                            const double t1 = cr[it][r][v], t2 = ci[it][r][v];
                            dr[it][r][v] += t1 - t2;
                            di[it][r][v] += ((double)c3[it][r][v] - t1) - t2;
                        } else {
                            dr[it][r][v] += (double)cr[it][r][v];
                            di[it][r][v] += (double)ci[it][r][v];
                        }
                    }
                    if constexpr (!(NPF <= 12 && NIT != 3)) {  // the per-case bodies start from zero
                        cr[it][r] = floatx4{0.f, 0.f, 0.f, 0.f};
                        ci[it][r] = floatx4{0.f, 0.f, 0.f, 0.f};
                        c3[it][r] = floatx4{0.f, 0.f, 0.f, 0.f};
                    }
                }
            }
        }
    }
#undef NUC_PREFETCH
    if (!qok) return;
    const int2 rg = elem_row_range(a.N, pr);
#pragma unroll
    for (int r = 0; r < MP; ++r) {
        if (r >= np) break;
        double2* out = a.part + ((size_t)(split * a.Tc + tl) * a.nmom + p0 + r) * a.C3;
        const long long base = choose3(pr.y) + choose2(pr.x);
        const long long above = choose2(pr.y) + pr.x;  // + choose3(row) for a row beyond k
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            if (it >= nit) break;
            const int tile = it0 + it;
            if (tile < rg.x || tile >= rg.y) continue;  // a tile of the wave's range this pair does not own
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = tile * 16 + 4 * g + v;
                const double2 val = F64 ? make_double2(xr[it][r][v], xi[it][r][v]) : make_double2(dr[it][r][v], di[it][r][v]);
                if (row >= a.N || (tile == (pr.x >> 4) && row >= pr.x)) continue;
                // the row is the smallest index, or (a tile beyond k's) the largest:
                // Phi_{row,j,k} = Phi_{j,k,row}
                if (row < pr.x)
                    out[base + row] = val;
                else
                    out[choose3(row) + above] = val;
            }
        }
    }
}

// FP64 sum of the per-split partials of every canonical entry (fixed split order).
// One item = 256 canonical entries.
__global__ __launch_bounds__(256) void elem_reduce_kernel(BatchRef bt) {
    const int item = blockIdx.x;
    const int inst = find_inst(bt.offs, bt.ninst, item);
    const ElemLaunch a = reinterpret_cast<const ElemLaunch*>(bt.descs)[inst];
    const size_t per_split = (size_t)a.Tc * a.nmom * a.C3;
    const size_t idx = (size_t)(item - bt.offs[inst]) * 256 + threadIdx.x;
    if (idx >= per_split) return;
    double sr = 0.0, si = 0.0;
    for (int s = 0; s < a.nsplit; ++s) {
        const double2 v = a.part[s * per_split + idx];
        sr += v.x;
        si += v.y;
    }
    a.packed[idx] = make_float2((float)sr, (float)si);
}

// Dense output: value of the sorted triple with the sign of the permutation,
// zero when two indices coincide. One item = 256 dense entries.
__global__ __launch_bounds__(256) void elem_expand_kernel(BatchRef bt) {
    const int item = blockIdx.x;
    const int inst = find_inst(bt.offs, bt.ninst, item);
    const ElemLaunch a = reinterpret_cast<const ElemLaunch*>(bt.descs)[inst];
    const size_t n3 = (size_t)a.N * a.N * a.N;
    const size_t total = (size_t)a.Tc * a.nmom * n3;
    const size_t idx = (size_t)(item - bt.offs[inst]) * 256 + threadIdx.x;
    if (idx >= total) return;
    const size_t tp = idx / n3;
    const int r = (int)(idx - tp * n3);
    int x = r / (a.N * a.N), y = (r / a.N) % a.N, z = r % a.N;
    float2 out = make_float2(0.f, 0.f);
    if (x != y && y != z && x != z) {
        bool neg = false;
        int tmp;
        if (x > y) { tmp = x; x = y; y = tmp; neg = !neg; }
        if (y > z) { tmp = y; y = z; z = tmp; neg = !neg; }
        if (x > y) { tmp = x; x = y; y = tmp; neg = !neg; }
        const float2 v = a.packed[tp * a.C3 + choose3(z) + choose2(y) + x];
        out = neg ? make_float2(-v.x, -v.y) : v;
    }
    a.phi[(size_t)(a.t_off - a.phi_t) * a.nmom * n3 + idx] = out;
}

template <int NPF, int NIT, int MP, bool F64>
hipError_t launch_elem_t(const BatchRef& b, hipStream_t s) {
    const size_t ph = F64 ? sizeof(double2) : sizeof(float2);
    const size_t lds = (size_t)(256 * NPF / ROW3 * RS + RS) * sizeof(float2) + (size_t)(MP * CS + 256) * ph;
    static std::atomic<unsigned long long> lds_set{0};
    const hipError_t lds_err = lds_limit_once((const void*)elem_kernel<NPF, NIT, MP, F64>, lds, lds_set);
    if (lds_err != hipSuccess) return lds_err;
    hipLaunchKernelGGL((elem_kernel<NPF, NIT, MP, F64>), dim3(b.nitems), dim3(256), lds, s, b);
    return hipGetLastError();
}

// Shape class: row tiles (from N) and momenta per workgroup (tuned, else from
// nmom), the latter capped by what the row-tile count allows.
int nit_of(int N) { return std::min(MAXNIT, (N + 15) / 16); }
int mp_of(int nmom) { return nmom <= 1 ? 1 : nmom <= 2 ? 2 : MAXP; }
int mp_sel(const ElemLaunch& a) {
    const int want = a.mp == 1 || a.mp == 2 || a.mp == MAXP ? a.mp : mp_of(a.nmom);
    return a.N > 64 ? 1 : std::min(want, mp_max(nit_of(a.N)));  // N > 64: deepest prefetch, one momentum
}

}  // namespace

void elem_finalize(ElemLaunch& a) {
    const int mp = mp_sel(a);
    a.npgroup = (a.nmom + mp - 1) / mp;
    int sps = (a.V3 + a.nsplit - 1) / a.nsplit;
    a.sites_per_split = ((sps + CS - 1) / CS) * CS;
}

int elem_items(const ElemLaunch& a) { return a.nwork * a.npgroup * a.nsplit * a.Tc; }
int elem_reduce_items(const ElemLaunch& a) { return (int)(((size_t)a.Tc * a.nmom * a.C3 + 255) / 256); }
int elem_expand_items(const ElemLaunch& a) {
    return (int)(((size_t)a.Tc * a.nmom * a.N * a.N * a.N + 255) / 256);
}
int n_bucket(int N) { return N <= 64 ? (N + 15) / 16 : 8; }
int elem_class(const ElemLaunch& a) { return n_bucket(a.N) * 16 + mp_sel(a) + (a.f64 ? kElemF64 : 0); }

// Class = 16 * (N bucket) + MP; the bucket fixes the prefetch depth NPF and the
// row tiles per workgroup: N <= 16 (NPF 3, 1 tile), <= 32 (6, 2), <= 48 (9, 3),
// <= 64 (12, 4), <= 128 (24, 4).
template <bool F64>
hipError_t launch_elem_f(int cls, const BatchRef& b, hipStream_t s) {
    const int nb = cls / 16, mp = cls % 16;
#define NUC_ELEM_CASE(NB_, NPF_, NIT_)                                                                \
    if (nb == NB_) {                                                                                  \
        if (mp == 1) return launch_elem_t<NPF_, NIT_, 1, F64>(b, s);                                  \
        if (mp == 2) return launch_elem_t<NPF_, NIT_, mp_max(NIT_) >= 2 ? 2 : 1, F64>(b, s);          \
        if (mp == MAXP) return launch_elem_t<NPF_, NIT_, mp_max(NIT_) >= MAXP ? MAXP : 1, F64>(b, s); \
        return hipErrorInvalidValue;                                                                  \
    }
    NUC_ELEM_CASE(1, 3, 1)
    NUC_ELEM_CASE(2, 6, 2)
    NUC_ELEM_CASE(3, 9, 3)
    NUC_ELEM_CASE(4, 12, 4)
    if (nb == 8) return mp == 1 ? launch_elem_t<24, 4, 1, F64>(b, s) : hipErrorInvalidValue;
#undef NUC_ELEM_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_elementals(int cls, const BatchRef& b, hipStream_t s) {
    if (b.nitems == 0) return hipSuccess;
    return (cls & kElemF64) ? launch_elem_f<true>(cls & ~kElemF64, b, s) : launch_elem_f<false>(cls, b, s);
}

hipError_t launch_elem_reduce(const BatchRef& b, hipStream_t s) {
    if (b.nitems == 0) return hipSuccess;
    hipLaunchKernelGGL(elem_reduce_kernel, dim3(b.nitems), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_elem_expand(const BatchRef& b, hipStream_t s) {
    if (b.nitems == 0) return hipSuccess;
    hipLaunchKernelGGL(elem_expand_kernel, dim3(b.nitems), dim3(256), 0, s, b);
    return hipGetLastError();
}

}  // namespace nuc

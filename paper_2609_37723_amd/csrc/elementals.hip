// Baryon elementals on CDNA4 MFMA (paper Section 2.1: the nucleon elementals
// Phi[p,t]_ijk that the distillation profiles then reweight).
//
//   Phi[p,t]_ijk = sum_{x,a} v_i^a(x) B_p[(x,a), jk],
//   B_p[(x,a), jk] = exp(-i p.x) W_jk^a(x),   W_jk^a(x) = eps_abc v_j^b(x) v_k^c(x)   (j < k)
//
// is a complex GEMM with rows i, columns the pairs j<k and the reduction over
// (site, colour). Only i < j < k is wanted. A workgroup (four waves up to 32 vectors,
// eight beyond) owns 16 consecutive pairs of the job's pair list per wave and up to
// four row tiles of 16 i per wave. Below 20 vectors the list holds every pair in lexicographic
// order and a wave takes the row tiles below the largest j of its pairs. From 20 vectors
// on it is the block pair set (elem_pair_in_set, elem_row_range): pairs inside a
// 16-index block with every row tile, pairs across two blocks of the lower half of the
// blocks with the tiles above k's block (Phi_rjk = Phi_jkr for a row past k), and pairs
// across two blocks of the upper half with the tiles below j's block; ordered by row
// range. Each colour cross product is built once per (site, colour,
// pair, momentum) and feeds those row tiles; the momentum phase rides on that operand,
// and the eigenvectors v_i are read from LDS as they are. Neither operand is stored in
// HBM: the workgroup stages the eigenvectors of a block of 16 sites in LDS by
// global_load_lds, double buffered (the next block streams in while the current one is
// multiplied). The K order is (site group of 4, colour), so every LDS address is a
// per-lane base plus a compile-time offset.
//
// Each block of 16 sites is summed in FP32 MFMA accumulators (three real products per
// complex one, Gauss's form, except for 48 vectors with two momenta per workgroup) and
// folded into per-lane FP64 sums; a workgroup stores the canonical entries (i<j<k) of its
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
// fold): three real MFMAs per complex product instead of four, wherever the third
// accumulator set fits two waves per SIMD without spilling (at most four row-tile x
// momentum products per wave; the 48-vector class with two momenta keeps four products).
constexpr bool gauss3(int nit, int mp) { return nit * mp <= 4; }

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
            if constexpr (gauss3(NIT, MP)) {
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

// The FP64 form of one staged block: the colour cross product and its phase in FP64
// (a product of two FP32 eigenvector components is exact there), FP64 MFMAs on the
// FP32 vectors, and the accumulators carried over the workgroup's whole site range. The
// complex products are in Gauss's three-multiplication form: xr, xi, x3 accumulate
// t1 = sum vr br, t2 = sum vi bi, t3 = sum (vr + vi)(br + bi), and the sum is
// (t1 - t2) + i (t3 - t1 - t2).
template <int NIT, int MP>
__device__ __forceinline__ void elem_block_f64(int nit, const float2* bj, const float2* bk, const float2* bi,
                                               const double2* sph, int g, doublex4 (&xr)[NIT][MP],
                                               doublex4 (&xi)[NIT][MP], doublex4 (&x3)[NIT][MP]) {
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
            double br[MP], bim[MP], bs[MP];
#pragma unroll
            for (int r = 0; r < MP; ++r) {
                br[r] = ph[r].x * wr - ph[r].y * wi;
                bim[r] = ph[r].x * wi + ph[r].y * wr;
                bs[r] = br[r] + bim[r];
            }
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                if (it >= nit) break;
                const float2 vi = bi[it * 16 * RS + o + ca];
                const double vs = (double)vi.x + vi.y;  // exact
#pragma unroll
                for (int r = 0; r < MP; ++r) {
                    xr[it][r] = dmfma16x4((double)vi.x, br[r], xr[it][r]);
                    xi[it][r] = dmfma16x4((double)vi.y, bim[r], xi[it][r]);
                    x3[it][r] = dmfma16x4(vs, bs[r], x3[it][r]);
                }
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

// One site block (sites c0 .. c0 + CS - 1 of vectors 0 .. N-1) into an LDS buffer of
// rows of RS complex, by global_load_lds. With 16-byte copies (evecs 16-byte aligned,
// an even number of complex per vector), slot s of the buffer is 16-byte segment
// s % 25 of row s / 25: segments 0..23 hold the row's 48 values, 24 is the row's
// padding (it receives a copy of segment 23). Otherwise 4-byte copies: slot s is float
// s % 100 of row s / 100, floats 96..99 the padding. Values past the end of a vector's
// sites are read from its first site instead; they, and the sites past the
// workgroup's range, meet a zero phase, so they add nothing (inputs are finite).
template <int WAVES>
__device__ __forceinline__ void elem_dma(float2* dst, const float2* vt, int N, int V3, int c0, bool x4, int wv,
                                         int lane) {
    const int row3 = 3 * V3;  // complex per vector
    if (x4) {
        const int nslot = N * (RS / 2);
        for (int i = wv; i * 64 < nslot; i += WAVES) {
            const int s = i * 64 + lane;
            const int n = s / (RS / 2), seg = min(s - n * (RS / 2), ROW3 / 2 - 1);
            const int e = 3 * c0 + 2 * seg;
            const float2* src = vt + (size_t)min(n, N - 1) * row3 + (e + 1 < row3 ? e : 0);
            if (s < nslot)
                __builtin_amdgcn_global_load_lds((gbl_void_t*)src, (lds_void_t*)(dst + 128 * i), 16, 0, 0);
        }
    } else {
        const int nslot = N * (2 * RS);
        for (int i = wv; i * 64 < nslot; i += WAVES) {
            const int s = i * 64 + lane;
            const int n = s / (2 * RS), f = min(s - n * (2 * RS), 2 * ROW3 - 1);
            const int e = 6 * c0 + f;  // float index within the vector
            const float* src =
                reinterpret_cast<const float*>(vt + (size_t)min(n, N - 1) * row3) + (e < 2 * row3 ? e : 0);
            if (s < nslot)
                __builtin_amdgcn_global_load_lds((gbl_void_t*)src, (lds_void_t*)(dst + 32 * i), 4, 0, 0);
        }
    }
}

// Phases exp(-i p.x) of the group's momenta at the sites of one block ([MP][CS]); zero
// for the sites past the workgroup's range and for momenta past the group's last.
template <int MP, class Ph>
__device__ __forceinline__ void elem_phases(Ph* sph, const Ph* tab, const ElemLaunch& a, int p0, int np, int c0,
                                            int ns) {
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
}

// F64: the FP64 form (elem_block_f64), whose phases are FP64 too.
// The workgroup's waves (elem_waves) share the staged vectors. Blocks of CS sites are
// double buffered: block m + 1 streams into LDS (global_load_lds) while block m is
// multiplied, with one barrier per block.
template <int NPF, int NIT, int MP, bool F64>
__global__ __launch_bounds__(64 * elem_waves(16 * NPF / 3)) __attribute__((amdgpu_waves_per_eu(2))) void elem_kernel(
    BatchRef bt) {
    // NPF: the vector class, 16 NPF / 3 staged rows (N rounded up to 16, 32, 48, 64 or 128)
    typedef std::conditional_t<F64, double2, float2> Ph;
    constexpr int WAVES = elem_waves(16 * NPF / 3), THREADS = 64 * WAVES;
    constexpr int ROWS = 16 * NPF / 3;
    constexpr int BUF = (ROWS + 1) * RS;  // complex per buffer: ROWS vector rows, then a zero row
    extern __shared__ float2 smem[];
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    const int inst = find_inst(bt.offs, bt.ninst, item);
    const ElemLaunch a = reinterpret_cast<const ElemLaunch*>(bt.descs)[inst];  // by value: read once
    float2* sv = smem;                              // [2][ROWS + 1][RS]
    Ph* sph = reinterpret_cast<Ph*>(sv + 2 * BUF);  // [2][MP][CS]
    Ph* tab = sph + 2 * MP * CS;                    // [L]  exp(-2 pi i m / L)

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
    const int q = pblock * 16 * WAVES + wv * 16 + col;
    const bool qok = q < a.npairs;
    const int2 pr = a.pairs[qok ? q : 0];
    // row tiles of this wave: from the smallest first tile of its 16 pairs to their
    // largest end (the pairs are ordered by row range, so a wave mostly has one), in
    // chunks of MAXNIT; a pair stores only the rows it owns
    const int q0 = pblock * 16 * WAVES + wv * 16;
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

    for (int m = threadIdx.x; m < a.L; m += THREADS) {
        double sn, cs;
        sincospi(2.0 * (double)m / (double)a.L, &sn, &cs);
        if constexpr (F64)
            tab[m] = make_double2(cs, -sn);
        else
            tab[m] = make_float2((float)cs, (float)(-sn));
    }
    // the zero rows of both buffers (the vectors of lanes past the last pair)
    for (int m = threadIdx.x; m < 2 * RS; m += THREADS)
        sv[(m / RS) * BUF + ROWS * RS + m % RS] = make_float2(0.f, 0.f);

    // accumulators of one site block: real and imaginary parts, or t1, t2, t3 (gauss3)
    floatx4 cr[NIT][MP], ci[NIT][MP], c3[NIT][MP];
    double dr[NIT][MP][4], di[NIT][MP][4];
    doublex4 xr[NIT][MP], xi[NIT][MP], x3[NIT][MP];  // F64: t1, t2, t3 over the whole site range
#pragma unroll
    for (int it = 0; it < NIT; ++it)
#pragma unroll
        for (int r = 0; r < MP; ++r) {
            xr[it][r] = doublex4{0.0, 0.0, 0.0, 0.0};
            xi[it][r] = doublex4{0.0, 0.0, 0.0, 0.0};
            x3[it][r] = doublex4{0.0, 0.0, 0.0, 0.0};
            cr[it][r] = floatx4{0.f, 0.f, 0.f, 0.f};
            ci[it][r] = floatx4{0.f, 0.f, 0.f, 0.f};
            c3[it][r] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int v = 0; v < 4; ++v) dr[it][r][v] = di[it][r][v] = 0.0;
        }

    const int s_begin = split * a.sites_per_split;
    const int s_end = min(a.V3, s_begin + a.sites_per_split);
    const float2* vt = a.evecs + (size_t)t * a.ev_tstride;
    const bool x4 = (reinterpret_cast<uintptr_t>(a.evecs) & 15) == 0 && a.V3 % 2 == 0 && a.ev_tstride % 2 == 0;

    // per-lane LDS bases in buffer 0 (buffer 1 adds BUF): site 4*sg + g, colour c  ->
    // offset 12*sg + 3*g + c
    const float2* bj = sv + (qok ? pr.x : ROWS) * RS + 3 * g;
    const float2* bk = sv + (qok ? pr.y : ROWS) * RS + 3 * g;
    const float2* bi = sv + (16 * it0 + arow(col, F64)) * RS + 3 * g;  // row tile it adds 16 it RS

    if (s_begin < s_end) elem_dma<WAVES>(sv, vt, a.N, a.V3, s_begin, x4, wv, lane);
    __syncthreads();  // the phase table
    elem_phases<MP>(sph, tab, a, p0, np, s_begin, min(CS, s_end - s_begin));
    int buf = 0;
    for (int c0 = s_begin; c0 < s_end; c0 += CS, buf ^= 1) {
        __builtin_amdgcn_s_waitcnt(0);  // this wave's copies of block c0
        __syncthreads();  // every wave's copies and phases of block c0; every wave done with the other buffer
        if (c0 + CS < s_end) {
            elem_dma<WAVES>(sv + (buf ^ 1) * BUF, vt, a.N, a.V3, c0 + CS, x4, wv, lane);
            elem_phases<MP>(sph + (buf ^ 1) * MP * CS, tab, a, p0, np, c0 + CS, min(CS, s_end - c0 - CS));
        }
        const int boff = buf * BUF;
        const Ph* ph_b = sph + buf * MP * CS;
        if (nit == 0) continue;
        // per-(nit, np) bodies (each starts its accumulators from zero)
        if constexpr (F64) {
            elem_block_f64<NIT, MP>(nit, bj + boff, bk + boff, bi + boff, ph_b, g, xr, xi, x3);
            continue;
        } else {
            elem_dispatch_ni<NIT, MP, NIT>(nit, np, bj + boff, bk + boff, bi + boff, ph_b, g, cr, ci, c3);
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
                        if constexpr (gauss3(NIT, MP)) {
                            const double t1 = cr[it][r][v], t2 = ci[it][r][v];
                            dr[it][r][v] += t1 - t2;
                            di[it][r][v] += ((double)c3[it][r][v] - t1) - t2;
                        } else {
                            dr[it][r][v] += (double)cr[it][r][v];
                            di[it][r][v] += (double)ci[it][r][v];
                        }
                    }
                }
            }
        }
    }
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
                const double2 val = F64 ? make_double2(xr[it][r][v] - xi[it][r][v], (x3[it][r][v] - xr[it][r][v]) - xi[it][r][v])
                                        : make_double2(dr[it][r][v], di[it][r][v]);
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
    const size_t lds = (size_t)2 * (16 * NPF / 3 + 1) * RS * sizeof(float2) + (size_t)(2 * MP * CS + 256) * ph;
    static std::atomic<unsigned long long> lds_set{0};
    const hipError_t lds_err = lds_limit_once((const void*)elem_kernel<NPF, NIT, MP, F64>, lds, lds_set);
    if (lds_err != hipSuccess) return lds_err;
    hipLaunchKernelGGL((elem_kernel<NPF, NIT, MP, F64>), dim3(b.nitems), dim3(64 * elem_waves(16 * NPF / 3)), lds, s,
                       b);
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

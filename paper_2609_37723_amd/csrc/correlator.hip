// Profiled nucleon correlation matrix C_ab(t) on CDNA4 MFMA (paper Section 2.1:
// the N_B x N_B matrix built from the profiled elementals Phi^(a)).
//
// Both Wick terms are folded into one contraction: because Phi is totally
// antisymmetric, D - E equals the direct contraction with the source spin
// tensor s'_{a'b'c'} = (C g5)_{a'b'} d_{c' sigma} + (C g5)_{c'b'} d_{a' sigma}.
// For each source profile b and sigma in {0,1} (P+):
//
//   step 1   X^{c'}[k] = D_b conj(Phi(t0))[k'-contracted] D_b,
//            X^{c'}[k]_{i'j'} = g_i' g_j' sum_k' tau[sN+k][c'N+k'] g_k' conj(Phi0_{i'j'k'})
// (tau may be an nvec-prefix of perambulators stored with block size Nt >= N.)
//   chain    W[k] = sum_beta cg5_beta sum_a' tau^{alpha(beta) a'}
//                     ( sum_{e in a'} s_e X^{c'_e}[k] (tau^{beta b'_e})^T )
//   sink     C_ab += g_k sum_ij g_i g_j Phi(t)_{ijk} W[k]_{ij}      (FP64 accumulation)
//
// The profile weights of the source (g^(b)[t0]) enter as diagonal scalings of
// X; those of the sink (g^(a)[t]) are applied in the FP64 dot, so one chain per
// source profile serves every sink profile. Step 1 is a GEMM over k'; the chain
// is a sequence of small complex GEMMs per sink index k whose first product's
// MFMA accumulators are fed straight back as the B operand of the second.
#include <math.h>

#include <type_traits>

#include "nuc_internal.h"

namespace nuc {
namespace {

// Step 1 as one complex GEMM per momentum p:
//   X[(tl,b,sp,c',k)][(i',j')] = g_i' g_j' sum_k' A[(tl,b,sp,c',k)][k'] conj(Phi0)[k'][(i',j')],
//   A[...][k'] = tau(t)[sp N + k][c' N + k'] g_k'   (source profile b at t0),
// with Phi0 = Phi(t0, p) stored [k'][i'][j'] (cyclic symmetry of Phi). A
// workgroup keeps one BN-column block of conj(Phi0) in LDS for the whole K and
// streams 64-row blocks of A past it, so the kernel runs at the rate of its
// output (X) writes.
constexpr int S1_BM = 64;

// Plane layout of BF16x3 operands split ahead of the chain. One row-chunk (32 complex
// along the contracted index) is 256 bytes: planes re_hi, re_lo, im_hi, im_lo of 32
// bf16, each in slot order: slot 8 g + e holds chunk position 4 g + e (e < 4) or
// 16 + 4 g + (e - 4). A lane of group g of a 16x16x32 MFMA reads slots 8g..8g+7 (16
// contiguous bytes per plane): those are the K positions of the rows of R it holds in
// its accumulators (tiles 2kc, 2kc + 1), the order the on-the-fly split path uses too.
__host__ __device__ inline int pre_slot(int q) { return 8 * ((q & 15) >> 2) + (q & 3) + (q & 16 ? 4 : 0); }
constexpr int kPreChunkBf16 = 128;  // bf16 per row-chunk (4 planes x 32)

__device__ __forceinline__ void split_bf16(float x, uint16_t& hi, uint16_t& lo) {
    const __bf16 h = (__bf16)x;
    const __bf16 l = (__bf16)(x - (float)h);
    hi = __builtin_bit_cast(uint16_t, h);
    lo = __builtin_bit_cast(uint16_t, l);
}

// tau values and source profile weights of one 64-row block of A, loaded into
// registers while the previous block is being multiplied; they are combined
// (and masked to zero outside N) only when the block is written to LDS.
// Waves of a step-1 workgroup: four (two workgroups per CU) up to Np = 64; eight beyond,
// where the LDS of one 64 x 64 block leaves room for one workgroup per CU and the
// eight waves keep two per SIMD.
constexpr int step1_waves(int KP) { return KP <= 64 ? 4 : 8; }

template <int KP, int TH = 64 * step1_waves(KP)>
struct Step1Block {
    static constexpr int PER = S1_BM * KP / TH;
    float2 v[PER];
    float g[PER];
};

// Row r of the block and its column kk for the q-th element of this thread;
// ok is false in the zero padding past N.
template <int KP, int TH = 64 * step1_waves(KP)>
__device__ __forceinline__ bool step1_elem(int rr0, int q, int N, int& r, int& kk, int& k, int& cp) {
    const int e = threadIdx.x + TH * q;
    r = e / KP;
    kk = e - r * KP;
    const int rr = rr0 + r;
    cp = rr / KP;
    k = rr - cp * KP;
    return k < N && kk < N;
}

template <int KP, int TH = 64 * step1_waves(KP)>
__device__ __forceinline__ void step1_fetch(const CorrLaunch& a, int r0, Step1Block<KP, TH>& blk) {
    const int N = a.N, Nt = a.Nt, N4t = 4 * Nt;
    int tmp = r0 / (4 * KP);
    const int sp = tmp % 2;
    tmp /= 2;
    const int b = tmp % a.nprof;
    const int t = a.t_off + tmp / a.nprof;
    const int rr0 = r0 % (4 * KP);
    const float* gb = a.gsrc_f + (size_t)b * N;
    const float2* tau_t = a.tau + (size_t)t * N4t * N4t + (size_t)sp * Nt * N4t;
#pragma unroll
    for (int q = 0; q < Step1Block<KP, TH>::PER; ++q) {
        int r, kk, k, cp;
        // unconditional loads from a clamped (in-bounds) index: a branch around
        // each load would serialise them
        const bool ok = step1_elem<KP, TH>(rr0, q, N, r, kk, k, cp);
        blk.v[q] = gld(tau_t + (ok ? (size_t)k * N4t + cp * Nt + kk : 0));
        blk.g[q] = gld(gb + (ok ? kk : 0));
    }
}

// For KP <= 32 the complex products take Gauss's three-multiplication form (three
// real MFMAs per complex step instead of four), which fits two waves per SIMD
// there; the larger tiles keep four products, where the third accumulator set
// would spill.
// F64: the FP64 form, FP64 MFMAs on the staged FP32 operands (exact products) with
// FP64 accumulation and the g_i' g_j' scaling in FP64 before X is rounded to FP32.
template <int KP, int BN, bool F64>
__global__ __launch_bounds__(64 * step1_waves(KP), KP <= 64 ? 2 : 1) void corr_step1_kernel(BatchRef bt) {
    constexpr bool G3 = KP <= 32 && !F64;
    typedef std::conditional_t<F64, doublex4, floatx4> Acc;
    typedef std::conditional_t<F64, double, float> Real;
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    const int inst = find_inst(bt.offs, bt.ninst, item);
    const CorrLaunch a = reinterpret_cast<const CorrLaunch*>(bt.descs)[inst];  // by value: read once
    const int row_chunk = a.row_chunk;
    constexpr int LD = KP + 2;  // complex row stride in LDS (16 bytes of padding)
    constexpr int WAVES = step1_waves(KP), THREADS = 64 * WAVES;
    constexpr int NCT = BN / 8 / WAVES;  // column tiles per wave (two row tiles each)
    constexpr int Np = KP;
    extern __shared__ float2 s1[];
    float2* sB = s1;             // [BN][LD]  conj(Phi0) transposed: [col][k']
    float2* sA = s1 + BN * LD;   // [S1_BM][LD]
    const int N = a.N;
    const int rows = a.Tc * a.nprof * 2 * 4 * Np;
    constexpr int ncols = Np * Np;
    constexpr int ncb = (ncols + BN - 1) / BN;
    const int nrc = (rows + row_chunk - 1) / row_chunk;
    unsigned bid = item - bt.offs[inst];
    const int cb = bid % ncb;
    bid /= ncb;
    const int rc = bid % nrc;
    const int p = bid / nrc;
    const float2* phi0 = a.phi0 + (size_t)p * N * N * N;

    const int r_beg = rc * row_chunk;
    const int r_end = min(rows, (rc + 1) * row_chunk);
    Step1Block<KP> blk;
    if (r_beg < r_end) step1_fetch<KP>(a, r_beg, blk);

    for (int e = threadIdx.x; e < KP * BN; e += THREADS) {
        const int kk = e / BN, c = e - kk * BN;
        const int cc = cb * BN + c;
        const int ip = cc / Np, jp = cc - ip * Np;
        const bool ok = cc < ncols && kk < N && ip < N && jp < N;
        const float2 f = phi0[ok ? ((size_t)kk * N + ip) * N + jp : 0];
        sB[c * LD + kk] = ok ? make_float2(f.x, -f.y) : make_float2(0.f, 0.f);
    }

    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 15, g = lane >> 4;
    const int wr = (wv / (WAVES / 2)) * 32, wc = (wv % (WAVES / 2)) * 16 * NCT;
    for (int r0 = r_beg; r0 < r_end; r0 += S1_BM) {
        // the 64 rows of a block share (tl, b, sp) because 64 divides 4 Np
        int tmp = r0 / (4 * Np);
        const int sp = tmp % 2;
        tmp /= 2;
        const int b = tmp % a.nprof;
        const int tl = tmp / a.nprof;
        const int rr0 = r0 % (4 * Np);
        const double* gb = a.gsrc + (size_t)b * N;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Step1Block<KP>::PER; ++q) {
            int r, kk, k, cp;
            const bool ok = step1_elem<KP>(rr0, q, N, r, kk, k, cp);
            const float w = blk.g[q] * (ok ? 1.f : 0.f);  // finite inputs: zero outside N
            sA[r * LD + kk] = make_float2(blk.v[q].x * w, blk.v[q].y * w);
        }
        __syncthreads();
        if (r0 + S1_BM < r_end) step1_fetch<KP>(a, r0 + S1_BM, blk);
        // G3: t1 = sum ar br, t2 = sum ai bi, t3 = sum (ar + ai)(br + bi), and
        // X = (t1 - t2) + i (t3 - t1 - t2); otherwise t1, t2 hold X's real and
        // imaginary parts
        Acc t1[2][NCT], t2[2][NCT], t3[2][NCT];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < NCT; ++y) {
                t1[x][y] = Acc{0, 0, 0, 0};
                t2[x][y] = Acc{0, 0, 0, 0};
                t3[x][y] = Acc{0, 0, 0, 0};
            }
#pragma unroll
        for (int kb = 0; kb < KP; kb += 16) {
            float4 av[2][2], bv[NCT][2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                const float4* pa =
                    reinterpret_cast<const float4*>(sA + (wr + 16 * x + arow(col, F64)) * LD + kb + 4 * g);
                av[x][0] = pa[0];
                av[x][1] = pa[1];
            }
#pragma unroll
            for (int y = 0; y < NCT; ++y) {
                const float4* pb = reinterpret_cast<const float4*>(sB + (wc + 16 * y + col) * LD + kb + 4 * g);
                bv[y][0] = pb[0];
                bv[y][1] = pb[1];
            }
            if constexpr (G3) {
                float as[2][4], bs[NCT][4];
#pragma unroll
                for (int x = 0; x < 2; ++x) {
                    as[x][0] = av[x][0].x + av[x][0].y;
                    as[x][1] = av[x][0].z + av[x][0].w;
                    as[x][2] = av[x][1].x + av[x][1].y;
                    as[x][3] = av[x][1].z + av[x][1].w;
                }
#pragma unroll
                for (int y = 0; y < NCT; ++y) {
                    bs[y][0] = bv[y][0].x + bv[y][0].y;
                    bs[y][1] = bv[y][0].z + bv[y][0].w;
                    bs[y][2] = bv[y][1].x + bv[y][1].y;
                    bs[y][3] = bv[y][1].z + bv[y][1].w;
                }
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int y = 0; y < NCT; ++y) {
                        t1[x][y] = mfma16x4(av[x][0].x, bv[y][0].x, t1[x][y]);
                        t2[x][y] = mfma16x4(av[x][0].y, bv[y][0].y, t2[x][y]);
                        t3[x][y] = mfma16x4(as[x][0], bs[y][0], t3[x][y]);
                        t1[x][y] = mfma16x4(av[x][0].z, bv[y][0].z, t1[x][y]);
                        t2[x][y] = mfma16x4(av[x][0].w, bv[y][0].w, t2[x][y]);
                        t3[x][y] = mfma16x4(as[x][1], bs[y][1], t3[x][y]);
                        t1[x][y] = mfma16x4(av[x][1].x, bv[y][1].x, t1[x][y]);
                        t2[x][y] = mfma16x4(av[x][1].y, bv[y][1].y, t2[x][y]);
                        t3[x][y] = mfma16x4(as[x][2], bs[y][2], t3[x][y]);
                        t1[x][y] = mfma16x4(av[x][1].z, bv[y][1].z, t1[x][y]);
                        t2[x][y] = mfma16x4(av[x][1].w, bv[y][1].w, t2[x][y]);
                        t3[x][y] = mfma16x4(as[x][3], bs[y][3], t3[x][y]);
                    }
            } else {
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int y = 0; y < NCT; ++y) {
                        cmac((Real)av[x][0].x, (Real)av[x][0].y, (Real)bv[y][0].x, (Real)bv[y][0].y, t1[x][y],
                             t2[x][y]);
                        cmac((Real)av[x][0].z, (Real)av[x][0].w, (Real)bv[y][0].z, (Real)bv[y][0].w, t1[x][y],
                             t2[x][y]);
                        cmac((Real)av[x][1].x, (Real)av[x][1].y, (Real)bv[y][1].x, (Real)bv[y][1].y, t1[x][y],
                             t2[x][y]);
                        cmac((Real)av[x][1].z, (Real)av[x][1].w, (Real)bv[y][1].z, (Real)bv[y][1].w, t1[x][y],
                             t2[x][y]);
                    }
            }
        }
        // epilogue: scale by g_i' g_j' and store rows of X[u][c'][k][(i',j')]; the
        // stores are nontemporal (X is read back only by the chain kernels)
        Real sc[NCT];
        int ccs[NCT];
#pragma unroll
        for (int y = 0; y < NCT; ++y) {
            const int cc = cb * BN + wc + 16 * y + col;
            const int ip = cc / Np, jp = cc - ip * Np;
            ccs[y] = cc;
            sc[y] = (cc < ncols && ip < N && jp < N) ? (Real)(gb[ip] * gb[jp]) : (Real)0;
        }
        const size_t u = (((size_t)tl * a.nmom + p) * a.nprof + b) * 2 + sp;
        float2* Xu = a.X + u * 4 * (size_t)Np * ncols;
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rr = rr0 + wr + 16 * x + 4 * g + v;  // (c', k) row within the unit
                float2* Xr = Xu + (size_t)rr * ncols;
#pragma unroll
                for (int y = 0; y < NCT; ++y)
                    if (ccs[y] < ncols) {
                        const Real r1 = t1[x][y][v], r2 = t2[x][y][v];
                        const float2 xv = G3 ? make_float2((r1 - r2) * sc[y], (t3[x][y][v] - r1 - r2) * sc[y])
                                             : make_float2((float)(r1 * sc[y]), (float)(r2 * sc[y]));
                        __builtin_nontemporal_store(*reinterpret_cast<const double*>(&xv),
                                                    reinterpret_cast<double*>(Xr + ccs[y]));
                    }
            }
    }
}

template <int KP, int BN, bool F64>
hipError_t launch_step1_t(const BatchRef& b, hipStream_t s) {
    const size_t lds = (size_t)(BN + S1_BM) * (KP + 2) * sizeof(float2);
    static std::atomic<unsigned long long> lds_set{0};
    const hipError_t lds_err = lds_limit_once((const void*)corr_step1_kernel<KP, BN, F64>, lds, lds_set);
    if (lds_err != hipSuccess) return lds_err;
    hipLaunchKernelGGL((corr_step1_kernel<KP, BN, F64>), dim3(b.nitems), dim3(64 * step1_waves(KP)), lds, s, b);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Step 1 for Np >= 48 over the triangle of (i', j'). X^{c'}[k]_{i'j'} is antisymmetric in
// (i', j') because Phi(t0) is, so only the column tiles of 8 i' x 8 j' with i'-block <=
// j'-block are multiplied; a tile below the diagonal is the negated transpose of one above
// it, and the kernel fed that tile's exactly negated conj(Phi0) columns would produce
// exactly these values, negated. A workgroup multiplies 64 rows (t, b, sigma', c', k) by one
// tile, K = k', in the K order of corr_step1_kernel; each wave takes 16 rows and all four
// 16-column MFMA tiles (two of them with eight waves, from Np = 80). Column c = 16 y + l of a tile is i' = 8 A + 2 y + (l >> 3),
// j' = 8 B + (l & 7): a lane's four values of one row of X are i' = 8 A + h, 8 A + 2 + h, ...
// (h = l >> 3) at one j'. The direct values leave as rows of 8 consecutive j' (64 bytes
// from 8 lanes); for the transposed ones (tiles off the diagonal) lanes l and l ^ 8 swap
// two values, so that each holds 4 consecutive i' (32 bytes) and the pair a 64-byte run.
template <int KP, bool F64>
__global__ __launch_bounds__(64 * step1_waves(KP), KP <= 64 ? 2 : 1) void corr_step1_tri_kernel(BatchRef bt) {
    typedef std::conditional_t<F64, doublex4, floatx4> Acc;
    typedef std::conditional_t<F64, double, float> Real;
    // Gauss's three-multiplication form, as corr_step1_kernel's (FP64 at Np = 48 would spill)
    constexpr bool G3 = !F64 || KP >= 64;
    // four waves (two workgroups per CU) up to Np = 64; eight from Np = 80, where one
    // block's LDS fills a CU: wave w takes row tile w % 4 and MFMA column tiles
    // NCT (w / 4) .. + NCT - 1
    constexpr int WAVES = step1_waves(KP), THREADS = 64 * WAVES, NCT = 16 / WAVES;
    constexpr int BN = 64, LD = KP + 2, Np = KP, NB8 = KP / 8;
    constexpr int ncols = Np * Np;
    constexpr int ncb = NB8 * (NB8 + 1) / 2;
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    const int inst = find_inst(bt.offs, bt.ninst, item);
    const CorrLaunch a = reinterpret_cast<const CorrLaunch*>(bt.descs)[inst];  // by value: read once
    const int row_chunk = a.row_chunk;
    extern __shared__ float2 s1t[];
    float2* sB = s1t;            // [BN][LD]  conj(Phi0) columns of the tile: [c][k']
    float2* sA = s1t + BN * LD;  // [S1_BM][LD]
    const int N = a.N;
    const int rows = a.Tc * a.nprof * 2 * 4 * Np;
    const int nrc = (rows + row_chunk - 1) / row_chunk;
    unsigned bid = item - bt.offs[inst];
    int cb = bid % ncb;
    bid /= ncb;
    const int rc = bid % nrc;
    const int p = bid / nrc;
    const float2* phi0 = a.phi0 + (size_t)p * N * N * N;
    int A = 0;  // tile -> 8-index blocks A <= B
    while (cb >= NB8 - A) {
        cb -= NB8 - A;
        ++A;
    }
    const int B = A + cb;

    const int r_beg = rc * row_chunk;
    const int r_end = min(rows, (rc + 1) * row_chunk);
    Step1Block<KP, THREADS> blk;
    if (r_beg < r_end) step1_fetch<KP, THREADS>(a, r_beg, blk);

    for (int e = threadIdx.x; e < KP * BN; e += THREADS) {
        const int kk = e / BN, c = e - kk * BN;
        const int ip = 8 * A + 2 * (c >> 4) + ((c & 15) >> 3), jp = 8 * B + (c & 7);
        const bool ok = kk < N && ip < N && jp < N;
        const float2 f = phi0[ok ? ((size_t)kk * N + ip) * N + jp : 0];
        sB[c * LD + kk] = ok ? make_float2(f.x, -f.y) : make_float2(0.f, 0.f);
    }

    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 15, g = lane >> 4, h = col >> 3;
    const int jp = 8 * B + (col & 7);
    const int rt = wv & 3, ys = NCT * (wv >> 2);  // row tile; first MFMA column tile
    for (int r0 = r_beg; r0 < r_end; r0 += S1_BM) {
        // the 64 rows of a block share (tl, b, sp) because 64 divides 4 Np
        int tmp = r0 / (4 * Np);
        const int sp = tmp % 2;
        tmp /= 2;
        const int b = tmp % a.nprof;
        const int tl = tmp / a.nprof;
        const int rr0 = r0 % (4 * Np);
        const double* gb = a.gsrc + (size_t)b * N;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Step1Block<KP, THREADS>::PER; ++q) {
            int r, kk, k, cp;
            const bool ok = step1_elem<KP, THREADS>(rr0, q, N, r, kk, k, cp);
            const float w = blk.g[q] * (ok ? 1.f : 0.f);  // finite inputs: zero outside N
            sA[r * LD + kk] = make_float2(blk.v[q].x * w, blk.v[q].y * w);
        }
        __syncthreads();
        if (r0 + S1_BM < r_end) step1_fetch<KP, THREADS>(a, r0 + S1_BM, blk);
        Acc t1[NCT], t2[NCT], t3[NCT];
#pragma unroll
        for (int y = 0; y < NCT; ++y) {
            t1[y] = Acc{0, 0, 0, 0};
            t2[y] = Acc{0, 0, 0, 0};
            t3[y] = Acc{0, 0, 0, 0};
        }
#pragma unroll
        for (int kb = 0; kb < KP; kb += 16) {
            float4 av[2], bv[NCT][2];
            const float4* pa = reinterpret_cast<const float4*>(sA + (16 * rt + arow(col, F64)) * LD + kb + 4 * g);
            av[0] = pa[0];
            av[1] = pa[1];
#pragma unroll
            for (int y = 0; y < NCT; ++y) {
                const float4* pb = reinterpret_cast<const float4*>(sB + (16 * (ys + y) + col) * LD + kb + 4 * g);
                bv[y][0] = pb[0];
                bv[y][1] = pb[1];
            }
            if constexpr (G3) {
                const Real as[4] = {(Real)av[0].x + av[0].y, (Real)av[0].z + av[0].w, (Real)av[1].x + av[1].y,
                                   (Real)av[1].z + av[1].w};
#pragma unroll
                for (int y = 0; y < NCT; ++y) {
                    const Real bs[4] = {(Real)bv[y][0].x + bv[y][0].y, (Real)bv[y][0].z + bv[y][0].w,
                                        (Real)bv[y][1].x + bv[y][1].y, (Real)bv[y][1].z + bv[y][1].w};
                    t1[y] = rmfma((Real)av[0].x, (Real)bv[y][0].x, t1[y]);
                    t2[y] = rmfma((Real)av[0].y, (Real)bv[y][0].y, t2[y]);
                    t3[y] = rmfma(as[0], bs[0], t3[y]);
                    t1[y] = rmfma((Real)av[0].z, (Real)bv[y][0].z, t1[y]);
                    t2[y] = rmfma((Real)av[0].w, (Real)bv[y][0].w, t2[y]);
                    t3[y] = rmfma(as[1], bs[1], t3[y]);
                    t1[y] = rmfma((Real)av[1].x, (Real)bv[y][1].x, t1[y]);
                    t2[y] = rmfma((Real)av[1].y, (Real)bv[y][1].y, t2[y]);
                    t3[y] = rmfma(as[2], bs[2], t3[y]);
                    t1[y] = rmfma((Real)av[1].z, (Real)bv[y][1].z, t1[y]);
                    t2[y] = rmfma((Real)av[1].w, (Real)bv[y][1].w, t2[y]);
                    t3[y] = rmfma(as[3], bs[3], t3[y]);
                }
            } else {
#pragma unroll
                for (int y = 0; y < NCT; ++y) {
                    cmac((Real)av[0].x, (Real)av[0].y, (Real)bv[y][0].x, (Real)bv[y][0].y, t1[y], t2[y]);
                    cmac((Real)av[0].z, (Real)av[0].w, (Real)bv[y][0].z, (Real)bv[y][0].w, t1[y], t2[y]);
                    cmac((Real)av[1].x, (Real)av[1].y, (Real)bv[y][1].x, (Real)bv[y][1].y, t1[y], t2[y]);
                    cmac((Real)av[1].z, (Real)av[1].w, (Real)bv[y][1].z, (Real)bv[y][1].w, t1[y], t2[y]);
                }
            }
        }
        // epilogue: scale by g_i' g_j'; direct rows X_{i'j'}, then (off the diagonal)
        // X_{j'i'} = -X_{i'j'}; nontemporal (X is read back only by the chain kernels)
        Real sc[NCT];
#pragma unroll
        for (int y = 0; y < NCT; ++y) {
            const int ip = 8 * A + 2 * (ys + y) + h;
            sc[y] = (ip < N && jp < N) ? (Real)(gb[ip] * gb[jp]) : (Real)0;
        }
        const size_t u = (((size_t)tl * a.nmom + p) * a.nprof + b) * 2 + sp;
        float2* Xu = a.X + u * 4 * (size_t)Np * ncols;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int rr = rr0 + 16 * rt + 4 * g + v;  // (c', k) row within the unit
            float2* Xr = Xu + (size_t)rr * ncols;
            float2 xv[NCT];
#pragma unroll
            for (int y = 0; y < NCT; ++y) {
                const Real r1 = t1[y][v], r2 = t2[y][v];
                xv[y] = G3 ? make_float2((r1 - r2) * sc[y], (t3[y][v] - r1 - r2) * sc[y])
                           : make_float2((float)(r1 * sc[y]), (float)(r2 * sc[y]));
                __builtin_nontemporal_store(*reinterpret_cast<const double*>(&xv[y]),
                                            reinterpret_cast<double*>(Xr + (8 * A + 2 * (ys + y) + h) * Np + jp));
            }
            if (A < B) {  // wave-uniform
                if constexpr (NCT == 4) {
                    const float2 s0 = h ? xv[0] : xv[2], s1 = h ? xv[1] : xv[3];
                    const float2 q0 = make_float2(__shfl_xor(s0.x, 8), __shfl_xor(s0.y, 8));
                    const float2 q1 = make_float2(__shfl_xor(s1.x, 8), __shfl_xor(s1.y, 8));
                    // i' = 8 A + 4 h + 0..3: h = 0 holds 0 and 2, gets 1 and 3; h = 1 holds 5 and 7,
                    // gets 4 and 6
                    const float2 o0 = h ? q0 : xv[0], o1 = h ? xv[2] : q0, o2 = h ? q1 : xv[1], o3 = h ? xv[3] : q1;
                    const floatx4 w0 = {-o0.x, -o0.y, -o1.x, -o1.y}, w1 = {-o2.x, -o2.y, -o3.x, -o3.y};
                    floatx4* dst = reinterpret_cast<floatx4*>(Xr + jp * Np + 8 * A + 4 * h);
                    __builtin_nontemporal_store(w0, dst);
                    __builtin_nontemporal_store(w1, dst + 1);
                } else {
                    // i' = 8 A + 2 ys + 2 h + 0..1: h = 0 holds 0 and 2, gives 2 and gets 1; h = 1
                    // holds 1 and 3, gives 1 and gets 2 (the other column half's wave writes the
                    // rest of the 64-byte run)
                    const float2 s0 = h ? xv[0] : xv[1];
                    const float2 q0 = make_float2(__shfl_xor(s0.x, 8), __shfl_xor(s0.y, 8));
                    const float2 o0 = h ? q0 : xv[0], o1 = h ? xv[1] : q0;
                    const floatx4 w0 = {-o0.x, -o0.y, -o1.x, -o1.y};
                    __builtin_nontemporal_store(w0, reinterpret_cast<floatx4*>(Xr + jp * Np + 8 * A + 2 * ys + 2 * h));
                }
            }
        }
    }
}

template <int KP, bool F64>
hipError_t launch_step1_tri_t(const BatchRef& b, hipStream_t s) {
    const size_t lds = (size_t)(64 + S1_BM) * (KP + 2) * sizeof(float2);
    static std::atomic<unsigned long long> lds_set{0};
    const hipError_t lds_err = lds_limit_once((const void*)corr_step1_tri_kernel<KP, F64>, lds, lds_set);
    if (lds_err != hipSuccess) return lds_err;
    hipLaunchKernelGGL((corr_step1_tri_kernel<KP, F64>), dim3(b.nitems), dim3(64 * step1_waves(KP)), lds, s, b);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Step 1 of the BF16x3 form with the chain's operands split ahead (N = Np = KP in
// {64, 96, 128}): the blocks of corr_step1_kernel (64 columns (i', j') by 64 rows
// (t, b, sigma', c', k), K = k'), with both operands staged in LDS as bf16 planes
// (re_hi, re_lo, im_hi, im_lo along k') and multiplied on 16x16x32 bf16 MFMA, three
// products per real product. The conj(Phi0) block is the MFMA's A operand and the tau
// block its B operand, so the accumulators hold X transposed: lane (c, g) of a tile
// pair (y = 0, 1) ends with positions 16 y + 4 g + v (v < 4) of one 32-position chunk
// of X's row c, i.e. slots 8 g .. 8 g + 7 of that chunk in the chain's slot order, and
// writes each plane as one 16-byte store.
constexpr int kS1PreBN = 64;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int KP>
struct Step1PreBlock {
    static constexpr int NG = S1_BM * KP / 8;  // groups of 8 k' per block
    static constexpr int G = (NG + 64 * step1_waves(KP) - 1) / (64 * step1_waves(KP));  // per thread (the last may be partial)
    float4 v[G][4];                                  // tau values
    float4 w[G][2];                                  // source weights g_k'
};

template <int KP>
__device__ __forceinline__ void step1_pre_fetch(const CorrLaunch& a, int r0, Step1PreBlock<KP>& blk) {
    const int Nt = a.Nt, N4t = 4 * Nt;
    int tmp = r0 / (4 * KP);
    const int sp = tmp % 2;
    tmp /= 2;
    const int b = tmp % a.nprof;
    const int t = a.t_off + tmp / a.nprof;
    const int rr0 = r0 % (4 * KP);
    const float* gb = a.gsrc_f + (size_t)b * KP;
    const float2* tau_t = a.tau + (size_t)t * N4t * N4t + (size_t)sp * Nt * N4t;
#pragma unroll
    for (int q = 0; q < Step1PreBlock<KP>::G; ++q) {
        const int e = min(threadIdx.x + 64 * step1_waves(KP) * q, Step1PreBlock<KP>::NG - 1);
        const int r = e / (KP / 8), kg = e - r * (KP / 8);
        const int rr = rr0 + r;
        const int cp = rr / KP, k = rr - cp * KP;
        const float4* src = reinterpret_cast<const float4*>(tau_t + (size_t)k * N4t + cp * Nt + 8 * kg);
#pragma unroll
        for (int i = 0; i < 4; ++i) blk.v[q][i] = src[i];
        const float4* gw = reinterpret_cast<const float4*>(gb + 8 * kg);
        blk.w[q][0] = gw[0];
        blk.w[q][1] = gw[1];
    }
}

template <int KP>
__global__ __launch_bounds__(64 * step1_waves(KP), KP <= 64 ? 2 : 1) void corr_step1_pre_kernel(BatchRef bt) {
    constexpr int BN = kS1PreBN;
    constexpr int WAVES = step1_waves(KP), THREADS = 64 * WAVES;
    constexpr int NX = 4 / (WAVES / 2);  // row tiles per wave; each wave has one 32-column chunk
    constexpr int PW = 4 * KP + 8;  // LDS row pitch in bf16: four planes of KP, then 16 bytes
    constexpr int ncols = KP * KP;
    constexpr int ncb = ncols / BN;
    constexpr int NKC = KP / 32;
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    const int inst = find_inst(bt.offs, bt.ninst, item);
    const CorrLaunch a = reinterpret_cast<const CorrLaunch*>(bt.descs)[inst];  // by value: read once
    extern __shared__ uint16_t s1pre[];
    uint16_t* sB = s1pre;            // [BN][PW]     conj(Phi0): rows (i', j'), planes along k'
    uint16_t* sA = s1pre + BN * PW;  // [S1_BM][PW]  g_k' tau: rows (c', k), planes along k'
    const int rows = a.Tc * a.nprof * 2 * 4 * KP;
    const int nrc = (rows + a.row_chunk - 1) / a.row_chunk;
    unsigned bid = item - bt.offs[inst];
    const int cb = bid % ncb;
    bid /= ncb;
    const int rc = bid % nrc;
    const int p = bid / nrc;
    const float2* phi0 = a.phi0 + (size_t)p * KP * KP * KP;

    const int r_beg = rc * a.row_chunk;
    const int r_end = min(rows, (rc + 1) * a.row_chunk);
    Step1PreBlock<KP> blk;
    if (r_beg < r_end) step1_pre_fetch<KP>(a, r_beg, blk);

    // conj(Phi0) block, two consecutive k' per thread and element
    for (int e = threadIdx.x; e < (KP / 2) * BN; e += THREADS) {
        const int k2 = e / BN, c = e - k2 * BN;
        const int cc = cb * BN + c;
        const int ip = cc / KP, jp = cc - ip * KP;
        const float2 f0 = phi0[((size_t)(2 * k2) * KP + ip) * KP + jp];
        const float2 f1 = phi0[((size_t)(2 * k2 + 1) * KP + ip) * KP + jp];
        uint16_t h[4][2];
        split_bf16(f0.x, h[0][0], h[1][0]);
        split_bf16(f1.x, h[0][1], h[1][1]);
        split_bf16(-f0.y, h[2][0], h[3][0]);
        split_bf16(-f1.y, h[2][1], h[3][1]);
#pragma unroll
        for (int pl = 0; pl < 4; ++pl)
            *reinterpret_cast<uint32_t*>(sB + c * PW + pl * KP + 2 * k2) = (uint32_t)h[pl][0] | ((uint32_t)h[pl][1] << 16);
    }

    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 15, g = lane >> 4;
    const int wr = (wv >> 1) * 16 * NX, wc = (wv & 1) * 32;
    // the wave's 32 columns are one 32-position chunk of one row i' of X
    const int cc0 = cb * BN + wc;
    const int ip = cc0 / KP, chunk = (cc0 - ip * KP) >> 5;
    const uint16_t* pa = sB + (wc + col) * PW + 8 * g;
    const uint16_t* pb = sA + (wr + col) * PW + 8 * g;
    for (int r0 = r_beg; r0 < r_end; r0 += S1_BM) {
        // the 64 rows of a block share (tl, b, sp) because 64 divides 4 Np
        int tmp = r0 / (4 * KP);
        const int sp = tmp % 2;
        tmp /= 2;
        const int b = tmp % a.nprof;
        const int tl = tmp / a.nprof;
        const int rr0 = r0 % (4 * KP);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Step1PreBlock<KP>::G; ++q) {
            const int e = threadIdx.x + THREADS * q;
            if (Step1PreBlock<KP>::NG % THREADS != 0 && e >= Step1PreBlock<KP>::NG) break;
            const int r = e / (KP / 8), kg = e - r * (KP / 8);
            const float* v = reinterpret_cast<const float*>(blk.v[q]);
            const float* w = reinterpret_cast<const float*>(blk.w[q]);
            floatx8 fr, fi;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                fr[j] = v[2 * j] * w[j];
                fi[j] = v[2 * j + 1] * w[j];
            }
            bf16x8 rh, rl, ih, il;
            split8(fr, rh, rl);
            split8(fi, ih, il);
            uint16_t* d = sA + r * PW + 8 * kg;
            *reinterpret_cast<bf16x8*>(d) = rh;
            *reinterpret_cast<bf16x8*>(d + KP) = rl;
            *reinterpret_cast<bf16x8*>(d + 2 * KP) = ih;
            *reinterpret_cast<bf16x8*>(d + 3 * KP) = il;
        }
        __syncthreads();
        if (r0 + S1_BM < r_end) step1_pre_fetch<KP>(a, r0 + S1_BM, blk);

        floatx4 cr[2][NX], ci[2][NX];  // [y: columns][x: rows]
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int x = 0; x < NX; ++x) {
                cr[y][x] = floatx4{0.f, 0.f, 0.f, 0.f};
                ci[y][x] = floatx4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
        for (int kc = 0; kc < NKC; ++kc) {
            bf16x8 av[2][4], bv[NX][4], nbh[NX], nbl[NX];
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int pl = 0; pl < 4; ++pl)
                    av[y][pl] = *reinterpret_cast<const bf16x8*>(pa + 16 * y * PW + pl * KP + 32 * kc);
#pragma unroll
            for (int x = 0; x < NX; ++x) {
#pragma unroll
                for (int pl = 0; pl < 4; ++pl)
                    bv[x][pl] = *reinterpret_cast<const bf16x8*>(pb + 16 * x * PW + pl * KP + 32 * kc);
                nbh[x] = bneg(bv[x][2]);
                nbl[x] = bneg(bv[x][3]);
            }
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int x = 0; x < NX; ++x)
                    cmfma_bf16x3(av[y][0], av[y][1], av[y][2], av[y][3], bv[x][0], bv[x][1], bv[x][2], bv[x][3],
                                 nbh[x], nbl[x], cr[y][x], ci[y][x]);
        }
        // epilogue: scale by g_i' g_j', split, and store slots 8 g .. 8 g + 7 of each plane
        const double* gbd = a.gsrc + (size_t)b * KP;
        const double gi = gbd[ip];
        float sc[2][4];
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) sc[y][v] = (float)(gi * gbd[32 * chunk + 16 * y + 4 * g + v]);
        const size_t u = (((size_t)tl * a.nmom + p) * a.nprof + b) * 2 + sp;
        uint16_t* Xu = reinterpret_cast<uint16_t*>(a.X + u * 4 * (size_t)KP * ncols);
#pragma unroll
        for (int x = 0; x < NX; ++x) {
            const int rr = rr0 + wr + 16 * x + col;  // (c', k) row within the unit
            floatx8 fr, fi;
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    fr[4 * y + v] = cr[y][x][v] * sc[y][v];
                    fi[4 * y + v] = ci[y][x][v] * sc[y][v];
                }
            bf16x8 o[4];
            split8(fr, o[0], o[1]);
            split8(fi, o[2], o[3]);
            uint16_t* dst = Xu + (size_t)rr * ncols * 4 + (size_t)ip * KP * 4 + chunk * kPreChunkBf16 + 8 * g;
#pragma unroll
            for (int pl = 0; pl < 4; ++pl)
                __builtin_nontemporal_store(__builtin_bit_cast(u32x4, o[pl]), reinterpret_cast<u32x4*>(dst + 32 * pl));
        }
    }
}

template <int KP>
hipError_t launch_step1_pre_t(const BatchRef& b, hipStream_t s) {
    const size_t lds = (size_t)(kS1PreBN + S1_BM) * (4 * KP + 8) * sizeof(uint16_t);
    static std::atomic<unsigned long long> lds_set{0};
    const hipError_t lds_err = lds_limit_once((const void*)corr_step1_pre_kernel<KP>, lds, lds_set);
    if (lds_err != hipSuccess) return lds_err;
    hipLaunchKernelGGL((corr_step1_pre_kernel<KP>), dim3(b.nitems), dim3(64 * step1_waves(KP)), lds, s, b);
    return hipGetLastError();
}

// Columns per workgroup: 128 up to Np = 32; 64 beyond, which keeps two workgroups per CU
// (LDS and registers) up to Np = 64.
int step1_bn(int Np) { return Np <= 32 ? 128 : 64; }

// ---------------------------------------------------------------------------
// Fused chain for Np <= 32. A workgroup (4 waves, one per SIMD) shares
// (t, p, b, sigma') and takes 4 consecutive sink indices k, one per wave. tau(t) is staged once in LDS
// (spin blocks padded to Np, rows padded by 16 bytes against bank conflicts);
// each wave keeps its four X^{c'}[k] slices in registers as ready-made MFMA A
// operands and its W[k] accumulator for all N_p columns. The spin structure is
// compile-time (kFold), so every register index is static.
template <int NRT>
struct FusedGeom {
    static constexpr int Np = NRT * 16;
    static constexpr int RS = 8 * Np + 4;  // LDS row stride in floats (4 Np complex + 16 B)
};

// FP32 operand as the MFMA's input type. Widening to FP64 goes through an empty asm
// statement so that the conversions of the register-resident X operands stay next to
// their MFMAs instead of being hoisted out of the beta loop (256 more live registers).
template <class Real>
__device__ __forceinline__ Real widen(float x) {
    if constexpr (std::is_same<Real, double>::value) asm volatile("" : "+v"(x));
    return (Real)x;
}

// Real/Acc: float/floatx4 (FP32 MFMA) or double/doublex4 (the FP64 form: the FP32
// operands are widened, R and W are FP64 and R feeds the second product unrounded).
template <int NRT, int SP, class Real, class Acc>
__device__ __forceinline__ void fused_unit(const float* __restrict__ lt, const float4 (&xa)[4][NRT][NRT][2],
                                           Acc (&Wr)[NRT][NRT], Acc (&Wi)[NRT][NRT], int col, int g) {
    constexpr int Np = FusedGeom<NRT>::Np, RS = FusedGeom<NRT>::RS;
    constexpr bool F64 = std::is_same<Real, double>::value;  // xa holds rows arow(col, F64)
    for (int beta = 0; beta < 4; ++beta) {
        const int al = kFold.sink_a[beta];
        const float cb = kFold.sink_c[beta];
#pragma unroll
        for (int ap = 0; ap < 4; ++ap) {
            Acc Rr[NRT][NRT], Ri[NRT][NRT];
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
                for (int ct = 0; ct < NRT; ++ct) {
                    Rr[rt][ct] = Acc{0, 0, 0, 0};
                    Ri[rt][ct] = Acc{0, 0, 0, 0};
                }
            // R = cg5_beta sum_e s_e X^{c'_e}[k] (tau^{beta b'_e})^T
#pragma unroll
            for (int e = 0; e < kFold.n[SP][ap]; ++e) {
                const int bp = kFold.bp[SP][ap][e], cp = kFold.cp[SP][ap][e];
                const float we = kFold.w[SP][ap][e] * cb;
#pragma unroll
                for (int ct = 0; ct < NRT; ++ct) {
                    const float* trow = lt + (beta * Np + 16 * ct + col) * RS + 2 * (bp * Np + 4 * g);
#pragma unroll
                    for (int kt = 0; kt < NRT; ++kt) {
                        const float4 b01 = *reinterpret_cast<const float4*>(trow + 32 * kt);
                        const float4 b23 = *reinterpret_cast<const float4*>(trow + 32 * kt + 4);
                        const float br[4] = {b01.x * we, b01.z * we, b23.x * we, b23.z * we};
                        const float bi[4] = {b01.y * we, b01.w * we, b23.y * we, b23.w * we};
#pragma unroll
                        for (int rt = 0; rt < NRT; ++rt) {
                            const float4 x01 = xa[cp][rt][kt][0], x23 = xa[cp][rt][kt][1];
                            const float ar[4] = {x01.x, x01.z, x23.x, x23.z};
                            const float ai[4] = {x01.y, x01.w, x23.y, x23.w};
#pragma unroll
                            for (int v = 0; v < 4; ++v)
                                cmac(widen<Real>(ar[v]), widen<Real>(ai[v]), widen<Real>(br[v]), widen<Real>(bi[v]),
                                     Rr[rt][ct], Ri[rt][ct]);
                        }
                    }
                }
            }
            // W += tau^{alpha a'} R: the accumulator rows of R are the K index
#pragma unroll
            for (int rt2 = 0; rt2 < NRT; ++rt2) {
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt) {
                    const float* ap0 = lt + (al * Np + 16 * rt + arow(col, F64)) * RS + 2 * (ap * Np + 16 * rt2 + 4 * g);
                    const float4 a01 = *reinterpret_cast<const float4*>(ap0);
                    const float4 a23 = *reinterpret_cast<const float4*>(ap0 + 4);
                    const float ar[4] = {a01.x, a01.z, a23.x, a23.z};
                    const float ai[4] = {a01.y, a01.w, a23.y, a23.w};
#pragma unroll
                    for (int ct = 0; ct < NRT; ++ct) {
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            cmac(widen<Real>(ar[v]), widen<Real>(ai[v]), Rr[rt2][ct][v], Ri[rt2][ct][v], Wr[rt][ct],
                                 Wi[rt][ct]);
                    }
                }
            }
        }
    }
}

constexpr int kFusedWaves = 4;

// Sink of one unit: C_ab += g_k sum_ij g_i g_j Phi(t)_{kij} W_ij, FP32 products
// accumulated in FP64, reduced over the wave, stored per (unit, sink profile).
template <int NRT, class Acc>
__device__ __forceinline__ void sink_dot(const CorrLaunch& a, const Acc (&Wr)[NRT][NRT], const Acc (&Wi)[NRT][NRT],
                                         int t, int p, int k, size_t ucore, int col, int g, int lane) {
    typedef std::conditional_t<std::is_same<Acc, doublex4>::value, double2, float2> C2;
    const int N = a.N;
    const float2* ph = a.phi + ((size_t)(t - a.phi_t) * a.nmom + p) * N * N * N + (size_t)k * N * N;
    C2 qv[NRT][NRT][4];
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
        for (int ct = 0; ct < NRT; ++ct)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * rt + 4 * g + v, j = 16 * ct + col;
                float2 f = make_float2(0.f, 0.f);
                if (i < N && j < N) f = ph[(size_t)i * N + j];
                const auto wr = Wr[rt][ct][v], wi = Wi[rt][ct][v];
                qv[rt][ct][v] = C2{f.x * wr - f.y * wi, f.x * wi + f.y * wr};
            }
    for (int pa = 0; pa < a.nprof; ++pa) {
        const double* ga = a.gsnk + ((size_t)pa * a.T + t) * N;
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int ct = 0; ct < NRT; ++ct) {
            const int j = 16 * ct + col;
            const double gj = j < N ? ga[j] : 0.0;
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = 16 * rt + 4 * g + v;
                    const double wgt = (i < N ? ga[i] : 0.0) * gj;
                    sr += wgt * (double)qv[rt][ct][v].x;
                    si += wgt * (double)qv[rt][ct][v].y;
                }
        }
        sr = wave_sum(sr);
        si = wave_sum(si);
        if (lane == 0) {
            const double gk = ga[k];
            a.part[(ucore * N + k) * a.nprof + pa] = make_double2(sr * gk, si * gk);
        }
    }
}

template <int NRT>
__device__ __forceinline__ void fused_load_x(const CorrLaunch& a, size_t ucore, int k, int col, int g,
                                             float4 (&xa)[4][NRT][NRT][2]) {
    constexpr int Np = FusedGeom<NRT>::Np;
    const size_t np2 = (size_t)Np * Np;
    const float2* Xu = a.X + ucore * 4 * np2 * Np;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
            for (int kt = 0; kt < NRT; ++kt) {
                const float4* src = reinterpret_cast<const float4*>(
                    Xu + ((size_t)c * Np + k) * np2 + (size_t)(16 * rt + col) * Np + 16 * kt + 4 * g);
                xa[c][rt][kt][0] = src[0];
                xa[c][rt][kt][1] = src[1];
            }
}

// One workgroup runs G consecutive unit groups that share the sink time t, so
// tau(t) is staged once; the next unit's X slices are loaded into registers as
// soon as the current chain is done, while the sink dot runs.
// ---------------------------------------------------------------------------
// BF16x3 form of the fused chain (Np <= 32). Same unit structure as the FP32
// kernel; tau(t) is staged in LDS already split into bf16 planes (re_hi,
// re_lo, im_hi, im_lo), each wave keeps X^{c'}[k] split in registers, and the
// FP32 accumulator R of the first product is split on the fly to serve as the B
// operand of the second. MFMA: 16x16x32 bf16 with FP32 accumulation. The K
// index of the first product is j' = 8 g + e; that of the second is
// i' = 16 (e/4) + 4 g + (e%4), matching the accumulator rows of R.
// Split arithmetic of the two split forms (FORM 1: BF16x3, FORM 2: scaled
// FP16x3): element vectors, hi/lo split, sign flip, complex 3-product MFMA.
template <int FORM>
struct SplitT;
template <>
struct SplitT<1> {
    typedef bf16x8 V;
    static __device__ __forceinline__ void split(floatx8 f, V& hi, V& lo) { split8(f, hi, lo); }
    static __device__ __forceinline__ V neg(V x) { return bneg(x); }
    static __device__ __forceinline__ void cmfma(V arh, V arl, V aih, V ail, V brh, V brl, V bih, V bil, V nbih,
                                                 V nbil, floatx4& cr, floatx4& ci) {
        cmfma_bf16x3(arh, arl, aih, ail, brh, brl, bih, bil, nbih, nbil, cr, ci);
    }
};
template <>
struct SplitT<2> {
    typedef f16x8 V;
    static __device__ __forceinline__ void split(floatx8 f, V& hi, V& lo) { split8h(f, hi, lo); }
    static __device__ __forceinline__ V neg(V x) { return hneg(x); }
    static __device__ __forceinline__ void cmfma(V arh, V arl, V aih, V ail, V brh, V brl, V bih, V bil, V nbih,
                                                 V nbil, floatx4& cr, floatx4& ci) {
        cmfma_f16x3(arh, arl, aih, ail, brh, brl, bih, bil, nbih, nbil, cr, ci);
    }
};

template <int FORM>
struct SplitOp {
    typename SplitT<FORM>::V rh, rl, ih, il;
};

// q of the FP16x3 scheme: 2^q >= 5 N 2^29 / 2^15
__device__ __forceinline__ int f16_rshift(int N) {
    int e;
    frexpf(5.f * (float)N, &e);  // 5 N < 2^e
    return e + 14;
}

template <int NRT>
struct Bf16Geom {
    static constexpr int Np = NRT * 16;
    static constexpr int RSB = 4 * Np + 8;        // LDS row stride in bf16 (4 Np + 16 bytes)
    static constexpr int PLANE = 4 * Np * RSB;    // bf16 per plane
};

template <int NRT, int FORM>
__device__ __forceinline__ void split_load_x(const CorrLaunch& a, size_t ucore, int k, int col, int g, float sx,
                                             SplitOp<FORM> (&xs)[4][NRT]) {
    constexpr int Np = Bf16Geom<NRT>::Np;
    const size_t np2 = (size_t)Np * Np;
    const float2* Xu = a.X + ucore * 4 * np2 * Np;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int rt = 0; rt < NRT; ++rt) {
            floatx8 re, im;
            if (NRT == 1 && g >= 2) {
                re = floatx8{0, 0, 0, 0, 0, 0, 0, 0};
                im = re;
            } else {
                const float4* src = reinterpret_cast<const float4*>(Xu + ((size_t)c * Np + k) * np2 +
                                                                    (size_t)(16 * rt + col) * Np + 8 * g);
                const float4 q0 = src[0], q1 = src[1], q2 = src[2], q3 = src[3];
                re = floatx8{q0.x, q0.z, q1.x, q1.z, q2.x, q2.z, q3.x, q3.z} * sx;
                im = floatx8{q0.y, q0.w, q1.y, q1.w, q2.y, q2.w, q3.y, q3.w} * sx;
            }
            SplitT<FORM>::split(re, xs[c][rt].rh, xs[c][rt].rl);
            SplitT<FORM>::split(im, xs[c][rt].ih, xs[c][rt].il);
        }
}

// rq: power of two applied to R before its split (FP16x3; 1 for BF16x3).
template <int NRT, int SP, int FORM>
__device__ __forceinline__ void split_unit(const uint16_t* __restrict__ lt, const SplitOp<FORM> (&xs)[4][NRT],
                                           floatx4 (&Wr)[NRT][NRT], floatx4 (&Wi)[NRT][NRT], int col, int g,
                                           float rq) {
    using S = SplitT<FORM>;
    typedef typename S::V V;
    typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
    constexpr int Np = Bf16Geom<NRT>::Np, RSB = Bf16Geom<NRT>::RSB, PL = Bf16Geom<NRT>::PLANE;
    const V zero8 = {};
    for (int beta = 0; beta < 4; ++beta) {
        const int al = kFold.sink_a[beta];
        const bool cneg = kFold.sink_c[beta] < 0.f;
#pragma unroll
        for (int ap = 0; ap < 4; ++ap) {
            floatx4 Rr[NRT][NRT], Ri[NRT][NRT];
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
                for (int ct = 0; ct < NRT; ++ct) {
                    Rr[rt][ct] = floatx4{0.f, 0.f, 0.f, 0.f};
                    Ri[rt][ct] = floatx4{0.f, 0.f, 0.f, 0.f};
                }
#pragma unroll
            for (int e = 0; e < kFold.n[SP][ap]; ++e) {
                const int bp = kFold.bp[SP][ap][e], cp = kFold.cp[SP][ap][e];
                const float wf = kFold.w[SP][ap][e];
                const bool wneg = (wf < 0.f) != cneg;
                const int reps = (wf == 2.f || wf == -2.f) ? 2 : 1;
#pragma unroll
                for (int ct = 0; ct < NRT; ++ct) {
                    // B[j'][j] = tau[beta Np + j][b' Np + j'], j' = 8 g + e
                    V brh = zero8, brl = zero8, bih = zero8, bil = zero8;
                    if (NRT > 1 || g < 2) {
                        const int off = (beta * Np + 16 * ct + col) * RSB + bp * Np + 8 * g;
                        brh = *reinterpret_cast<const V*>(lt + off);
                        brl = *reinterpret_cast<const V*>(lt + PL + off);
                        bih = *reinterpret_cast<const V*>(lt + 2 * PL + off);
                        bil = *reinterpret_cast<const V*>(lt + 3 * PL + off);
                    }
                    if (wneg) {
                        brh = S::neg(brh);
                        brl = S::neg(brl);
                        bih = S::neg(bih);
                        bil = S::neg(bil);
                    }
                    const V nbih = S::neg(bih), nbil = S::neg(bil);
#pragma unroll
                    for (int r = 0; r < reps; ++r)
#pragma unroll
                        for (int rt = 0; rt < NRT; ++rt)
                            S::cmfma(xs[cp][rt].rh, xs[cp][rt].rl, xs[cp][rt].ih, xs[cp][rt].il, brh, brl, bih,
                                     bil, nbih, nbil, Rr[rt][ct], Ri[rt][ct]);
                }
            }
            // W += tau^{alpha a'} R with R split on the fly; K slot (g, e) is row
            // 16 (e/4) + 4 g + (e%4) of R
#pragma unroll
            for (int ct = 0; ct < NRT; ++ct) {
                floatx8 fr, fi;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int rt2 = e / 4, v = e % 4;
                    fr[e] = rt2 < NRT ? Rr[rt2 < NRT ? rt2 : 0][ct][v] * rq : 0.f;
                    fi[e] = rt2 < NRT ? Ri[rt2 < NRT ? rt2 : 0][ct][v] * rq : 0.f;
                }
                V brh, brl, bih, bil;
                S::split(fr, brh, brl);
                S::split(fi, bih, bil);
                const V nbih = S::neg(bih), nbil = S::neg(bil);
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt) {
                    const int off = (al * Np + 16 * rt + col) * RSB + ap * Np + 4 * g;
                    V arh, arl, aih, ail;
                    {
                        const u16x4 z4 = {};
                        const u16x4* p0 = reinterpret_cast<const u16x4*>(lt + off);
                        const u16x4* p1 = reinterpret_cast<const u16x4*>(lt + off + 16);
                        const u16x4 r0 = p0[0], l0 = p0[PL / 4], i0 = p0[PL / 2], m0 = p0[3 * PL / 4];
                        const u16x4 r1 = NRT > 1 ? p1[0] : z4, l1 = NRT > 1 ? p1[PL / 4] : z4;
                        const u16x4 i1 = NRT > 1 ? p1[PL / 2] : z4, m1 = NRT > 1 ? p1[3 * PL / 4] : z4;
                        arh = __builtin_bit_cast(V, __builtin_shufflevector(r0, r1, 0, 1, 2, 3, 4, 5, 6, 7));
                        arl = __builtin_bit_cast(V, __builtin_shufflevector(l0, l1, 0, 1, 2, 3, 4, 5, 6, 7));
                        aih = __builtin_bit_cast(V, __builtin_shufflevector(i0, i1, 0, 1, 2, 3, 4, 5, 6, 7));
                        ail = __builtin_bit_cast(V, __builtin_shufflevector(m0, m1, 0, 1, 2, 3, 4, 5, 6, 7));
                    }
                    S::cmfma(arh, arl, aih, ail, brh, brl, bih, bil, nbih, nbil, Wr[rt][ct], Wi[rt][ct]);
                }
            }
        }
    }
}


// ---------------------------------------------------------------------------
// Persistent driver of the Np <= 32 chain (FORM 0: FP32, FORM 1: BF16x3). The
// grid is one workgroup per CU; each takes a contiguous range of unit groups
// (4 sink indices k of one (instance, t, p, b, sigma')) across all instances of
// the batch, restaging tau(t) only when the instance or the sink time changes,
// and loading the next unit's X slices while the current sink dot runs.
template <int NRT, int FORM>
struct XRegs;
template <int NRT>
struct XRegs<NRT, 0> {
    float4 v[4][NRT][NRT][2];
};
template <int NRT>
struct XRegs<NRT, 1> {
    SplitOp<1> v[4][NRT];
    float sx;
};
template <int NRT>
struct XRegs<NRT, 2> {
    SplitOp<2> v[4][NRT];
    float sx;  // power-of-two scale of these X blocks
};

// Stage tau(t) in LDS: FP32 rows, or (split forms) four planes of tau st split
// into hi/lo, st = 1 for BF16x3 and the timeslice's power-of-two scale for FP16x3.
template <int NRT, int FORM>
__device__ __forceinline__ void small_stage_tau(float* lds, const CorrLaunch& a, int t) {
    constexpr int Np = NRT * 16;
    const int N = a.N, Nt = a.Nt, N4t = 4 * Nt;
    const float2* tau_t = a.tau + (size_t)t * N4t * N4t;
    const float st = FORM == 2 ? a.tscale[t - a.t_off] : 1.f;
    for (int e = threadIdx.x; e < 16 * Np * Np; e += kFusedWaves * 64) {
        const int r = e / (4 * Np), c = e - r * (4 * Np);
        const int rs = r / Np, ri = r - rs * Np, cs = c / Np, ci = c - cs * Np;
        float2 v = make_float2(0.f, 0.f);
        if (ri < N && ci < N) v = tau_t[(size_t)(rs * Nt + ri) * N4t + cs * Nt + ci];
        if constexpr (FORM == 0 || FORM == 3) {
            *reinterpret_cast<float2*>(lds + r * FusedGeom<NRT>::RS + 2 * c) = v;
        } else if constexpr (FORM == 1) {
            __bf16* ltb = reinterpret_cast<__bf16*>(lds);
            constexpr int RSB = Bf16Geom<NRT>::RSB, PL = Bf16Geom<NRT>::PLANE;
            const __bf16 rh = (__bf16)v.x, ih = (__bf16)v.y;
            const __bf16 rl = (__bf16)(v.x - (float)rh), il = (__bf16)(v.y - (float)ih);
            const int o = r * RSB + c;
            ltb[o] = rh;
            ltb[PL + o] = rl;
            ltb[2 * PL + o] = ih;
            ltb[3 * PL + o] = il;
        } else {
            _Float16* lth = reinterpret_cast<_Float16*>(lds);
            constexpr int RSB = Bf16Geom<NRT>::RSB, PL = Bf16Geom<NRT>::PLANE;
            const float xr = v.x * st, xi = v.y * st;
            const _Float16 rh = (_Float16)xr, ih = (_Float16)xi;
            const _Float16 rl = (_Float16)(xr - (float)rh), il = (_Float16)(xi - (float)ih);
            const int o = r * RSB + c;
            lth[o] = rh;
            lth[PL + o] = rl;
            lth[2 * PL + o] = ih;
            lth[3 * PL + o] = il;
        }
    }
}

template <int NRT>
struct XRegs<NRT, 3> : XRegs<NRT, 0> {};

template <int NRT, int FORM>
__device__ __forceinline__ void small_load_x(const CorrLaunch& a, size_t ucore, int k, int col, int g,
                                             XRegs<NRT, FORM>& x) {
    if constexpr (FORM == 0 || FORM == 3) {
        fused_load_x<NRT>(a, ucore, k, arow(col, FORM == 3), g, x.v);  // the A rows of the first product
    } else {
        x.sx = FORM == 2 ? a.xscale[ucore * a.N + k] : 1.f;
        split_load_x<NRT, FORM>(a, ucore, k, col, g, x.sx, x.v);
    }
}

template <int NRT, int FORM>
__global__ __launch_bounds__(kFusedWaves * 64) __attribute__((amdgpu_waves_per_eu(1, 1)))
void corr_chain_small_kernel(BatchRef bt) {
    extern __shared__ float lsm[];
    const CorrLaunch* descs = reinterpret_cast<const CorrLaunch*>(bt.descs);
    const int nwg = gridDim.x;
    const int wg = xcd_remap(blockIdx.x, nwg);
    const int i0 = (int)((long)wg * bt.nitems / nwg), i1 = (int)((long)(wg + 1) * bt.nitems / nwg);
    if (i0 >= i1) return;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 15, g = lane >> 4;

    struct Cur {
        int inst, t, p, k;
        size_t ucore;
    };
    auto decode = [&](int item) {
        Cur c;
        c.inst = find_inst(bt.offs, bt.ninst, item);
        const CorrLaunch& a = descs[c.inst];
        const int nkg = (a.N + kFusedWaves - 1) / kFusedWaves;
        const int gpt = a.nmom * a.nprof * 2 * nkg;
        const int li = item - bt.offs[c.inst];
        const int tl = li / gpt;
        int tmp = li - tl * gpt;
        const int kg = tmp % nkg;
        tmp /= nkg;
        const int sp = tmp % 2;
        tmp /= 2;
        const int b = tmp % a.nprof;
        c.p = tmp / a.nprof;
        c.t = a.t_off + tl;
        c.ucore = (((size_t)tl * a.nmom + c.p) * a.nprof + b) * 2 + sp;
        c.k = kg * kFusedWaves + wv;
        return c;
    };

    Cur cur = decode(i0);
    small_stage_tau<NRT, FORM>(lsm, descs[cur.inst], cur.t);
    XRegs<NRT, FORM> xr;
    {
        const CorrLaunch& a = descs[cur.inst];
        small_load_x<NRT, FORM>(a, cur.ucore, cur.k < a.N ? cur.k : 0, col, g, xr);
    }
    __syncthreads();

    for (int it = i0; it < i1; ++it) {
        const bool has_next = it + 1 < i1;
        const Cur nxt = has_next ? decode(it + 1) : cur;
        const CorrLaunch& a = descs[cur.inst];
        const CorrLaunch& an = descs[nxt.inst];
        if (cur.k < a.N) {
            const int sp = (int)(cur.ucore & 1);
            typedef typename AccT<FORM>::type Acc;
            Acc Wr[NRT][NRT], Wi[NRT][NRT];
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
                for (int ct = 0; ct < NRT; ++ct) {
                    Wr[rt][ct] = Acc{0, 0, 0, 0};
                    Wi[rt][ct] = Acc{0, 0, 0, 0};
                }
            if constexpr (FORM == 0 || FORM == 3) {
                typedef std::conditional_t<FORM == 3, double, float> Real;
                if (sp == 0)
                    fused_unit<NRT, 0, Real, Acc>(lsm, xr.v, Wr, Wi, col, g);
                else
                    fused_unit<NRT, 1, Real, Acc>(lsm, xr.v, Wr, Wi, col, g);
            } else {
                const uint16_t* lth = reinterpret_cast<const uint16_t*>(lsm);
                // FP16x3: R sx st enters the second product times rq; W then carries sx st^2 rq
                const float rq = FORM == 2 ? ldexpf(1.f, -f16_rshift(a.N)) : 1.f;
                if (sp == 0)
                    split_unit<NRT, 0, FORM>(lth, xr.v, Wr, Wi, col, g, rq);
                else
                    split_unit<NRT, 1, FORM>(lth, xr.v, Wr, Wi, col, g, rq);
                if constexpr (FORM == 2) {
                    const float st = a.tscale[cur.t - a.t_off];
                    const float u = 1.f / (xr.sx * st * st * rq);
#pragma unroll
                    for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
                        for (int ct = 0; ct < NRT; ++ct) {
                            Wr[rt][ct] *= u;
                            Wi[rt][ct] *= u;
                        }
                }
            }
            if (has_next) small_load_x<NRT, FORM>(an, nxt.ucore, nxt.k < an.N ? nxt.k : 0, col, g, xr);
            sink_dot<NRT, Acc>(a, Wr, Wi, cur.t, cur.p, cur.k, cur.ucore, col, g, lane);
        } else if (has_next) {
            small_load_x<NRT, FORM>(an, nxt.ucore, nxt.k < an.N ? nxt.k : 0, col, g, xr);
        }
        if (has_next && (nxt.inst != cur.inst || nxt.t != cur.t)) {
            __syncthreads();
            small_stage_tau<NRT, FORM>(lsm, an, nxt.t);
            __syncthreads();
        }
        cur = nxt;
    }
}

int device_cus() {
    static int ncu = 0;
    if (ncu == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
            ncu = 256;
    }
    return ncu;
}

template <int NRT, int FORM>
hipError_t launch_small_t(const BatchRef& b, hipStream_t s) {
    const size_t lds = FORM == 0 || FORM == 3 ? (size_t)4 * FusedGeom<NRT>::Np * FusedGeom<NRT>::RS * sizeof(float)
                                              : (size_t)4 * Bf16Geom<NRT>::PLANE * sizeof(__bf16);
    static std::atomic<unsigned long long> lds_set{0};
    const hipError_t lds_err = lds_limit_once((const void*)corr_chain_small_kernel<NRT, FORM>, lds, lds_set);
    if (lds_err != hipSuccess) return lds_err;
    const int grid = std::min(b.nitems, device_cus());
    hipLaunchKernelGGL((corr_chain_small_kernel<NRT, FORM>), dim3(grid), dim3(kFusedWaves * 64), lds, s, b);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Chain for 32 < Np <= 128 (FP32). One workgroup (4 waves, one per SIMD) per
// (t, p, b, sigma', k) unit; wave w owns the 16-column strips w, w+4, ... of R
// and W. The first product streams 32-wide K chunks of X^{c'}[k] and of the
// weighted tau^{beta b'} block through LDS (the spin weight is applied while
// staging); the second product stages the whole tau^{alpha a'} block so the K
// index (the accumulator rows of R) stays compile-time.
constexpr int kLargeWaves = 4;

template <int NRT>
struct LargeGeom {
    static constexpr int Np = NRT * 16;
    static constexpr int CT = (NRT + kLargeWaves - 1) / kLargeWaves;  // strips per wave
    static constexpr int KC = 32, LDC = KC + 2;   // chunk width and its LDS row stride (complex)
    static constexpr int LDL = Np + 2;            // row stride of the staged tau^{alpha a'} block
    static constexpr int CHUNK = 2 * Np * LDC;    // complex in sX + sT
    static constexpr int FULL = Np * LDL;
    static constexpr int LDS = (CHUNK > FULL ? CHUNK : FULL);
};

template <int NRT, int SP>
__device__ __forceinline__ void large_unit(const CorrLaunch& a, float2* __restrict__ sm, const float2* Xu, int k,
                                           const float2* tau_t, floatx4 (&Wr)[NRT][LargeGeom<NRT>::CT],
                                           floatx4 (&Wi)[NRT][LargeGeom<NRT>::CT], int wv, int col, int g) {
    using G = LargeGeom<NRT>;
    constexpr int Np = G::Np, KC = G::KC, LDC = G::LDC, LDL = G::LDL, CT = G::CT;
    const int N = a.N, Nt = a.Nt, N4t = 4 * Nt;
    constexpr int nthr = kLargeWaves * 64;
    const size_t np2 = (size_t)Np * Np;
    float2* sX = sm;
    float2* sT = sm + Np * LDC;
    for (int beta = 0; beta < 4; ++beta) {
        const int al = kFold.sink_a[beta];
        const float cb = kFold.sink_c[beta];
#pragma unroll
        for (int ap = 0; ap < 4; ++ap) {
            floatx4 Rr[NRT][CT], Ri[NRT][CT];
#pragma unroll
            for (int r = 0; r < NRT; ++r)
#pragma unroll
                for (int c = 0; c < CT; ++c) {
                    Rr[r][c] = floatx4{0.f, 0.f, 0.f, 0.f};
                    Ri[r][c] = floatx4{0.f, 0.f, 0.f, 0.f};
                }
#pragma unroll
            for (int e = 0; e < kFold.n[SP][ap]; ++e) {
                const int bp = kFold.bp[SP][ap][e], cp = kFold.cp[SP][ap][e];
                const float we = kFold.w[SP][ap][e] * cb;
                const float2* Xs = Xu + ((size_t)cp * Np + k) * np2;  // [i'][j']
                for (int k0 = 0; k0 < Np; k0 += KC) {
                    __syncthreads();
                    for (int q = threadIdx.x; q < Np * KC; q += nthr) {
                        const int r = q / KC, kk = q - r * KC;
                        const int jp = k0 + kk;
                        float2 xv = make_float2(0.f, 0.f), tv = make_float2(0.f, 0.f);
                        if (jp < Np) xv = Xs[(size_t)r * Np + jp];
                        if (r < N && jp < N) {
                            const float2 t0 = tau_t[(size_t)(beta * Nt + r) * N4t + bp * Nt + jp];
                            tv = make_float2(t0.x * we, t0.y * we);
                        }
                        sX[r * LDC + kk] = xv;
                        sT[r * LDC + kk] = tv;
                    }
                    __syncthreads();
#pragma unroll
                    for (int kb = 0; kb < KC; kb += 16) {
                        if (k0 + kb >= Np) break;
                        float br[CT][4], bi[CT][4];
#pragma unroll
                        for (int c = 0; c < CT; ++c) {
                            const int j = 16 * (wv + kLargeWaves * c) + col;
                            const int jj = j < Np ? j : 0;
                            const float4* pb = reinterpret_cast<const float4*>(sT + jj * LDC + kb + 4 * g);
                            const float4 b01 = pb[0], b23 = pb[1];
                            br[c][0] = b01.x; br[c][1] = b01.z; br[c][2] = b23.x; br[c][3] = b23.z;
                            bi[c][0] = b01.y; bi[c][1] = b01.w; bi[c][2] = b23.y; bi[c][3] = b23.w;
                        }
#pragma unroll
                        for (int rt = 0; rt < NRT; ++rt) {
                            const float4* pa = reinterpret_cast<const float4*>(sX + (16 * rt + col) * LDC + kb + 4 * g);
                            const float4 a01 = pa[0], a23 = pa[1];
                            const float ar[4] = {a01.x, a01.z, a23.x, a23.z};
                            const float ai[4] = {a01.y, a01.w, a23.y, a23.w};
#pragma unroll
                            for (int c = 0; c < CT; ++c)
#pragma unroll
                                for (int v = 0; v < 4; ++v) {
                                    Rr[rt][c] = mfma16x4(ar[v], br[c][v], Rr[rt][c]);
                                    Rr[rt][c] = mfma16x4(-ai[v], bi[c][v], Rr[rt][c]);
                                    Ri[rt][c] = mfma16x4(ar[v], bi[c][v], Ri[rt][c]);
                                    Ri[rt][c] = mfma16x4(ai[v], br[c][v], Ri[rt][c]);
                                }
                        }
                    }
                }
            }
            // W += tau^{alpha a'} R with the whole tau block in LDS
            __syncthreads();
            for (int q = threadIdx.x; q < Np * Np; q += nthr) {
                const int r = q / Np, c = q - r * Np;
                float2 tv = make_float2(0.f, 0.f);
                if (r < N && c < N) tv = tau_t[(size_t)(al * Nt + r) * N4t + ap * Nt + c];
                sm[r * LDL + c] = tv;
            }
            __syncthreads();
#pragma unroll
            for (int rt2 = 0; rt2 < NRT; ++rt2) {
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt) {
                    const float4* pa = reinterpret_cast<const float4*>(sm + (16 * rt + col) * LDL + 16 * rt2 + 4 * g);
                    const float4 a01 = pa[0], a23 = pa[1];
                    const float ar[4] = {a01.x, a01.z, a23.x, a23.z};
                    const float ai[4] = {a01.y, a01.w, a23.y, a23.w};
#pragma unroll
                    for (int c = 0; c < CT; ++c)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const float brr = Rr[rt2][c][v], bri = Ri[rt2][c][v];
                            Wr[rt][c] = mfma16x4(ar[v], brr, Wr[rt][c]);
                            Wr[rt][c] = mfma16x4(-ai[v], bri, Wr[rt][c]);
                            Wi[rt][c] = mfma16x4(ar[v], bri, Wi[rt][c]);
                            Wi[rt][c] = mfma16x4(ai[v], brr, Wi[rt][c]);
                        }
                }
            }
        }
    }
}

template <int NRT>
__global__ __launch_bounds__(kLargeWaves * 64) __attribute__((amdgpu_waves_per_eu(1, 1)))
void corr_chain_large_kernel(BatchRef bt) {
    using G = LargeGeom<NRT>;
    constexpr int Np = G::Np, CT = G::CT;
    extern __shared__ float2 smL[];
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    const int inst = find_inst(bt.offs, bt.ninst, item);
    const CorrLaunch a = reinterpret_cast<const CorrLaunch*>(bt.descs)[inst];
    const int N = a.N, N4t = 4 * a.Nt;
    unsigned bid = item - bt.offs[inst];
    int tmp = bid;
    const int k = tmp % N;
    tmp /= N;
    const int sp = tmp % 2;
    tmp /= 2;
    const int b = tmp % a.nprof;
    tmp /= a.nprof;
    const int p = tmp % a.nmom;
    const int tl = tmp / a.nmom;
    const int t = a.t_off + tl;
    const size_t ucore = (((size_t)tl * a.nmom + p) * a.nprof + b) * 2 + sp;
    const float2* Xu = a.X + ucore * 4 * (size_t)Np * Np * Np;
    const float2* tau_t = a.tau + (size_t)t * N4t * N4t;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 15, g = lane >> 4;

    floatx4 Wr[NRT][CT], Wi[NRT][CT];
#pragma unroll
    for (int r = 0; r < NRT; ++r)
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            Wr[r][c] = floatx4{0.f, 0.f, 0.f, 0.f};
            Wi[r][c] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
    if (sp == 0)
        large_unit<NRT, 0>(a, smL, Xu, k, tau_t, Wr, Wi, wv, col, g);
    else
        large_unit<NRT, 1>(a, smL, Xu, k, tau_t, Wr, Wi, wv, col, g);

    // sink dot (FP64), waves combined through LDS
    __syncthreads();
    double2* red = reinterpret_cast<double2*>(smL);  // [kLargeWaves][kMaxProf]
    const float2* ph = a.phi + ((size_t)(t - a.phi_t) * a.nmom + p) * N * N * N + (size_t)k * N * N;
    float2 qv[NRT][CT][4];
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
        for (int c = 0; c < CT; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * rt + 4 * g + v, j = 16 * (wv + kLargeWaves * c) + col;
                float2 f = make_float2(0.f, 0.f);
                if (i < N && j < N) f = ph[(size_t)i * N + j];
                const float wr = Wr[rt][c][v], wi = Wi[rt][c][v];
                qv[rt][c][v] = make_float2(f.x * wr - f.y * wi, f.x * wi + f.y * wr);
            }
    for (int pa = 0; pa < a.nprof; ++pa) {
        const double* ga = a.gsnk + ((size_t)pa * a.T + t) * N;
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int c = 0; c < CT; ++c) {
            const int j = 16 * (wv + kLargeWaves * c) + col;
            const double gj = j < N ? ga[j] : 0.0;
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = 16 * rt + 4 * g + v;
                    const double wgt = (i < N ? ga[i] : 0.0) * gj;
                    sr += wgt * (double)qv[rt][c][v].x;
                    si += wgt * (double)qv[rt][c][v].y;
                }
        }
        sr = wave_sum(sr);
        si = wave_sum(si);
        if (lane == 0) red[wv * kMaxProf + pa] = make_double2(sr, si);
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)a.nprof) {
        const int pa = threadIdx.x;
        double sr = 0.0, si = 0.0;
        for (int w = 0; w < kLargeWaves; ++w) {
            sr += red[w * kMaxProf + pa].x;
            si += red[w * kMaxProf + pa].y;
        }
        const double gk = a.gsnk[((size_t)pa * a.T + t) * N + k];
        a.part[(ucore * N + k) * a.nprof + pa] = make_double2(sr * gk, si * gk);
    }
}


// ------------------------------------------------ large N, LDS-DMA pipeline
//
// Same unit and arithmetic as corr_chain_large_kernel, for N = Np (a multiple
// of 16) and an even tau block size. Every operand reaches LDS through
// global_load_lds_dwordx4 in chunks of 32 complex along the contracted index:
// the chunk of step s+1 streams into one half of a double buffer while the
// MFMAs consume step s from the other half (one barrier per step). The
// tau^{alpha a'} product W += tau R is cut into the same chunks, its B operand
// being the R accumulators of the chunk's row tiles.
//
// A staged array is Np rows of 32 complex (256 B, sixteen 16-byte segments).
// Lane L of a DMA instruction writes segment L%16 of row L/16 of the
// instruction's four rows; it fetches logical segment (L%16) ^ (row%16), so
// the MFMA operand reads (16 consecutive rows, one segment each) touch 16
// different segment positions.
constexpr int kDmaKC = 32;
constexpr int kDmaRow = kDmaKC;  // complex per staged row

__device__ float4 g_dma_zero[1];  // zeros for the tail of a chunk past Np


// Stage rows [0, ROWS) x complex [k0, k0 + 32) of a row-major source (row stride
// `stride` complex, rows start at src) into dst; columns at or past kend are zero.
// W waves: instruction m stages rows m * 4W + 4 wv + lane / 16; since 16 divides 4W, their
// swizzle (row % 16) is the same for every m, so the lane's column and its mask are
// computed once. When 4W does not divide ROWS (a multiple of 16), the last instruction
// is issued by the waves whose four rows exist (a wave-uniform test).
template <int ROWS, int W = kLargeWaves>
__device__ __forceinline__ void dma_rows(float2* dst, const float2* src, size_t stride, int k0, int kend, int wv,
                                         int lane) {
    static_assert(ROWS % 16 == 0 && (4 * W) % 16 == 0, "row groups of 16");
    const int rsub = lane >> 4, pos = lane & 15;
    const int row0 = wv * 4 + rsub;  // < 4W
    const int k = k0 + 2 * (pos ^ (row0 & 15));
    const bool ok = k < kend;
    const float2* g0 = src + (size_t)row0 * stride + k;
#pragma unroll
    for (int m = 0; m < (ROWS + 4 * W - 1) / (4 * W); ++m) {
        if (ROWS % (4 * W) != 0 && m * 4 * W + 4 * wv >= ROWS) break;
        const void* g = ok ? (const void*)(g0 + (size_t)m * 4 * W * stride) : (const void*)g_dma_zero;
        __builtin_amdgcn_global_load_lds((gbl_void_t*)g, (lds_void_t*)(dst + ((size_t)m * W + wv) * 4 * kDmaRow), 16,
                                         0, 0);
    }
}

// Operand fetch from a staged array: complex k..k+3 (k = kb + 4g, kb a multiple
// of 16) of row r as re[4], im[4].
__device__ __forceinline__ void dma_read4(const float2* arr, int r, int k, float (&re)[4], float (&im)[4]) {
    const int s0 = (k >> 1) ^ (r & 15);
    const float4 a01 = *reinterpret_cast<const float4*>(arr + r * kDmaRow + 2 * s0);
    const float4 a23 = *reinterpret_cast<const float4*>(arr + r * kDmaRow + 2 * (s0 ^ 1));
    re[0] = a01.x; re[1] = a01.z; re[2] = a23.x; re[3] = a23.z;
    im[0] = a01.y; im[1] = a01.w; im[2] = a23.y; im[3] = a23.w;
}

// One step of a unit's schedule. Per beta and source spin a' (ap) the schedule
// is n[SP][ap] * CH R-steps (e, chunk) followed by CH W-steps (chunk).
template <int SP, int CH>
struct DmaStep {
    int ap, e, kc;
    bool w;
};

template <int SP, int CH>
__device__ __forceinline__ DmaStep<SP, CH> dma_step(int idx) {
    DmaStep<SP, CH> d{0, 0, 0, false};
#pragma unroll
    for (int ap = 0; ap < 4; ++ap) {
        const int nr = kFold.n[SP][ap] * CH;
        if (idx < nr) {
            d.ap = ap;
            d.e = idx / CH;
            d.kc = idx - d.e * CH;
            return d;
        }
        idx -= nr;
        if (idx < CH) {
            d.ap = ap;
            d.kc = idx;
            d.w = true;
            return d;
        }
        idx -= CH;
    }
    return d;
}

template <int NRT, int SP, int W = kLargeWaves>
__device__ __forceinline__ void dma_issue(const CorrLaunch& a, float2* buf, const float2* Xu, int k,
                                          const float2* tau_t, int beta, int idx, int wv, int lane) {
    constexpr int Np = NRT * 16, CH = (Np + kDmaKC - 1) / kDmaKC;
    const int Nt = a.Nt, N4t = 4 * Nt;
    const DmaStep<SP, CH> d = dma_step<SP, CH>(idx);
    const int k0 = d.kc * kDmaKC;
    float2* sA = buf;
    float2* sB = buf + Np * kDmaRow;
    if (d.w) {
        const int al = kFold.sink_a[beta];
        dma_rows<Np, W>(sA, tau_t + (size_t)al * Nt * N4t + (size_t)d.ap * Nt, N4t, k0, Np, wv, lane);
    } else {
        const int bp = kFold.bp[SP][d.ap][d.e], cp = kFold.cp[SP][d.ap][d.e];
        const size_t np2 = (size_t)Np * Np;
        dma_rows<Np, W>(sA, Xu + ((size_t)cp * Np + k) * np2, Np, k0, Np, wv, lane);
        dma_rows<Np, W>(sB, tau_t + (size_t)beta * Nt * N4t + (size_t)bp * Nt, N4t, k0, Np, wv, lane);
    }
}

template <int NRT, int SP, int W = kLargeWaves>
__device__ __forceinline__ const float2* dma_advance(const CorrLaunch& a, float2* sm, const float2* Xu, int k,
                                                     const float2* tau_t, int s, int wv, int lane) {
    constexpr int Np = NRT * 16, CH = (Np + kDmaKC - 1) / kDmaKC, L = 11 * CH, BUF = 2 * Np * kDmaRow;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (s + 1 < 4 * L) {
        const int b1 = (s + 1) / L;
        dma_issue<NRT, SP, W>(a, sm + ((s + 1) & 1) * BUF, Xu, k, tau_t, b1, s + 1 - b1 * L, wv, lane);
    }
    return sm + (s & 1) * BUF;
}

// Real/Acc as in fused_unit; the wave (of W) owns the CTX column strips wv + W (c + cs),
// c < CTX (cs = 0 and CTX = CT when one workgroup takes the whole unit).
// GR, GW: the first (R) and the second (W) product in Gauss's three-multiplication form,
// t1 = sum ar br, t2 = sum ai bi, t3 = sum (ar + ai)(br + bi), the product
// (t1 - t2) + i (t3 - t1 - t2); R is formed that way before it enters the second product,
// W once at the end of the unit. Each takes a third accumulator set, so they are used
// where that fits the kernel's waves per SIMD without spilling.
template <int NRT, int SP, class Real, class Acc, int CTX, bool GR = false, bool GW = false, int W = kLargeWaves>
__device__ __forceinline__ void dma_unit(const CorrLaunch& a, float2* __restrict__ sm, const float2* Xu, int k,
                                         const float2* tau_t, Acc (&Wr)[NRT][CTX], Acc (&Wi)[NRT][CTX], int wv,
                                         int lane, int cs) {
    constexpr int Np = NRT * 16, CH = (Np + kDmaKC - 1) / kDmaKC;
    constexpr bool F64 = std::is_same<Real, double>::value;
    const int col = lane & 15, g = lane >> 4;
    Acc W3[NRT][CTX];  // GW: t3 of W (Wr, Wi hold t1, t2 until the end)
#pragma unroll
    for (int r = 0; r < NRT; ++r)
#pragma unroll
        for (int c = 0; c < CTX; ++c) W3[r][c] = Acc{0, 0, 0, 0};
    dma_issue<NRT, SP, W>(a, sm, Xu, k, tau_t, 0, 0, wv, lane);
    int s = 0;
    for (int beta = 0; beta < 4; ++beta) {
        const float cb = kFold.sink_c[beta];
        for (int ap = 0; ap < 4; ++ap) {
            Acc Rr[NRT][CTX], Ri[NRT][CTX], R3[NRT][CTX];
#pragma unroll
            for (int r = 0; r < NRT; ++r)
#pragma unroll
                for (int c = 0; c < CTX; ++c) {
                    Rr[r][c] = Acc{0, 0, 0, 0};
                    Ri[r][c] = Acc{0, 0, 0, 0};
                    R3[r][c] = Acc{0, 0, 0, 0};
                }
            const int ne = kFold.n[SP][ap];
            for (int e = 0; e < ne; ++e) {
                const float we = kFold.w[SP][ap][e] * cb;
                for (int kc = 0; kc < CH; ++kc, ++s) {
                    const float2* sA = dma_advance<NRT, SP, W>(a, sm, Xu, k, tau_t, s, wv, lane);
                    const float2* sB = sA + Np * kDmaRow;
#pragma unroll
                    for (int kb = 0; kb < kDmaKC; kb += 16) {
                        if (kc * kDmaKC + kb >= Np) break;
                        float br[CTX][4], bi[CTX][4], bs[CTX][4];
#pragma unroll
                        for (int c = 0; c < CTX; ++c) {
                            const int j = 16 * (wv + W * (c + cs)) + col;
                            dma_read4(sB, j < Np ? j : 0, kb + 4 * g, br[c], bi[c]);
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                br[c][v] *= we;
                                bi[c][v] *= we;
                                bs[c][v] = br[c][v] + bi[c][v];
                            }
                        }
#pragma unroll
                        for (int rt = 0; rt < NRT; ++rt) {
                            float ar[4], ai[4];
                            dma_read4(sA, 16 * rt + arow(col, F64), kb + 4 * g, ar, ai);
#pragma unroll
                            for (int c = 0; c < CTX; ++c)
#pragma unroll
                                for (int v = 0; v < 4; ++v) {
                                    if constexpr (GR) {
                                        Rr[rt][c] = rmfma((Real)ar[v], (Real)br[c][v], Rr[rt][c]);
                                        Ri[rt][c] = rmfma((Real)ai[v], (Real)bi[c][v], Ri[rt][c]);
                                        R3[rt][c] = rmfma((Real)ar[v] + (Real)ai[v], (Real)br[c][v] + (Real)bi[c][v],
                                                          R3[rt][c]);
                                    } else {
                                        cmac((Real)ar[v], (Real)ai[v], (Real)br[c][v], (Real)bi[c][v], Rr[rt][c],
                                             Ri[rt][c]);
                                    }
                                }
                        }
                    }
                }
            }
            // GR: R = (t1 - t2) + i (t3 - t1 - t2); GW: R3 then holds Rr + Ri for the second product
#pragma unroll
            for (int r = 0; r < NRT; ++r)
#pragma unroll
                for (int c = 0; c < CTX; ++c)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        if constexpr (GR) {
                            const Real t1 = Rr[r][c][v], t2 = Ri[r][c][v], t3 = R3[r][c][v];
                            Rr[r][c][v] = t1 - t2;
                            Ri[r][c][v] = t3 - t1 - t2;
                        }
                        if constexpr (GW) R3[r][c][v] = Rr[r][c][v] + Ri[r][c][v];
                    }
            // W += tau^{alpha a'} R, chunk by chunk over the rows of R
#pragma unroll
            for (int kc = 0; kc < CH; ++kc, ++s) {
                const float2* sA = dma_advance<NRT, SP, W>(a, sm, Xu, k, tau_t, s, wv, lane);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int rt2 = 2 * kc + h;
                    if (rt2 >= NRT) break;
#pragma unroll
                    for (int rt = 0; rt < NRT; ++rt) {
                        float ar[4], ai[4];
                        dma_read4(sA, 16 * rt + arow(col, F64), 16 * h + 4 * g, ar, ai);
#pragma unroll
                        for (int c = 0; c < CTX; ++c)
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                if constexpr (GW) {
                                    Wr[rt][c] = rmfma((Real)ar[v], Rr[rt2][c][v], Wr[rt][c]);
                                    Wi[rt][c] = rmfma((Real)ai[v], Ri[rt2][c][v], Wi[rt][c]);
                                    W3[rt][c] = rmfma((Real)ar[v] + (Real)ai[v], R3[rt2][c][v], W3[rt][c]);
                                } else {
                                    cmac((Real)ar[v], (Real)ai[v], Rr[rt2][c][v], Ri[rt2][c][v], Wr[rt][c],
                                         Wi[rt][c]);
                                }
                            }
                    }
                }
            }
        }
    }
    if constexpr (GW) {
#pragma unroll
        for (int r = 0; r < NRT; ++r)
#pragma unroll
            for (int c = 0; c < CTX; ++c)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const Real t1 = Wr[r][c][v], t2 = Wi[r][c][v], t3 = W3[r][c][v];
                    Wr[r][c][v] = t1 - t2;
                    Wi[r][c][v] = t3 - t1 - t2;
                }
    }
}

// BF16x3 with operands split ahead (kernel form 4): X^{c'}[k] and tau(t) arrive as bf16
// planes (pre_slot layout) and are staged as they are, 256 bytes per row-chunk with the
// same 16-byte XOR swizzle as the FP32 path; the MFMAs read their operands straight from
// LDS (16 bytes per plane and lane). Only R, an FP32 accumulator, is split on the fly.
// The source weights are signs, applied by negating planes, and 2, applied by reading the
// doubled tau block (exact either way).
// Row m * 16 + 4 wv + lane / 16 of instruction m; since 16 divides m * 16, the row's
// swizzle (row % 16) and so the lane's byte offset inside its row group are the same
// for every m: one per-lane offset, plus a wave-uniform m * 16 * stride.
template <int ROWS, int W>
__device__ __forceinline__ void dma_rows_pre(char* dst, const char* src, size_t stride, int wv, int lane) {
    // W waves: instruction m of wave wv stages rows m 4W + 4 wv .. + 3 (row0 + 4W m)
    const int rsub = lane >> 4, pos = lane & 15;
    const int row0 = wv * 4 + rsub;  // < 4 W; rows of one swizzle share row0 % 16
    const char* g0 = src + (size_t)row0 * stride + 16 * (pos ^ (row0 & 15));
#pragma unroll
    for (int m = 0; m < ROWS / (4 * W); ++m)
        __builtin_amdgcn_global_load_lds((gbl_void_t*)(g0 + (size_t)m * 4 * W * stride),
                                         (lds_void_t*)(dst + ((size_t)m * W + wv) * 4 * 256), 16, 0, 0);
}

// Byte offsets, inside a 16-row tile of a staged pre-split array, of the four planes a
// lane (column col, group g) reads: row col, logical segment 4 p + g.
struct PreLane {
    int off[4];
};
__device__ __forceinline__ PreLane pre_lane(int col, int g) {
    PreLane o;
#pragma unroll
    for (int p = 0; p < 4; ++p) o.off[p] = col * 256 + 16 * ((4 * p + g) ^ col);
    return o;
}
__device__ __forceinline__ bf16x8 pre_read(const char* tile, const PreLane& o, int p) {
    return *reinterpret_cast<const bf16x8*>(tile + o.off[p]);
}

template <int NRT, int SP, int W>
__device__ __forceinline__ void dma_issue_pre(const CorrLaunch& a, char* buf, const char* Xu, int k, const char* tt,
                                              int beta, int idx, int wv, int lane) {
    constexpr int Np = NRT * 16, CH = Np / kDmaKC;
    constexpr size_t trow = (size_t)kTauBlocks * CH * 256;  // bytes per row of tau's planes
    const DmaStep<SP, CH> d = dma_step<SP, CH>(idx);
    char* sA = buf;
    char* sB = buf + Np * 256;
    if (d.w) {
        const int al = kFold.sink_a[beta];
        dma_rows_pre<Np, W>(sA, tt + (size_t)al * Np * trow + ((size_t)d.ap * CH + d.kc) * 256, trow, wv, lane);
    } else {
        const int bp = kFold.bp[SP][d.ap][d.e], cp = kFold.cp[SP][d.ap][d.e];
        const float wf = kFold.w[SP][d.ap][d.e];
        const int blk = (wf == 2.f || wf == -2.f) ? 4 + bp : bp;  // weight 2: the doubled block
        dma_rows_pre<Np, W>(sA, Xu + (((size_t)cp * Np + k) * Np * CH + d.kc) * 256, (size_t)CH * 256, wv, lane);
        dma_rows_pre<Np, W>(sB, tt + (size_t)beta * Np * trow + ((size_t)blk * CH + d.kc) * 256, trow, wv, lane);
    }
}

template <int NRT, int SP, int W>
__device__ __forceinline__ const char* dma_advance_pre(const CorrLaunch& a, char* sm, const char* Xu, int k,
                                                       const char* tt, int s, int wv, int lane) {
    constexpr int Np = NRT * 16, CH = Np / kDmaKC, L = 11 * CH, BUF = 2 * Np * 256;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (s + 1 < 4 * L) {
        const int b1 = (s + 1) / L;
        dma_issue_pre<NRT, SP, W>(a, sm + ((s + 1) & 1) * BUF, Xu, k, tt, b1, s + 1 - b1 * L, wv, lane);
    }
    return sm + (s & 1) * BUF;
}

// FENCE: keep each row tile's operand reads next to its MFMAs (a scheduling barrier per
// tile), so the reads of all tiles are not hoisted ahead into live registers.
template <int NRT, int CT, bool FENCE = false>
__device__ __forceinline__ void pre_first_product(const char* sA, const SplitOp<1> (&bo)[CT], const bf16x8 (&nbh)[CT],
                                                  const bf16x8 (&nbl)[CT], const PreLane& pl,
                                                  floatx4 (&Rr)[NRT][CT], floatx4 (&Ri)[NRT][CT]) {
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt) {
        const char* tile = sA + rt * 16 * 256;
        const bf16x8 arh = pre_read(tile, pl, 0), arl = pre_read(tile, pl, 1);
        const bf16x8 aih = pre_read(tile, pl, 2), ail = pre_read(tile, pl, 3);
#pragma unroll
        for (int c = 0; c < CT; ++c)
            cmfma_bf16x3(arh, arl, aih, ail, bo[c].rh, bo[c].rl, bo[c].ih, bo[c].il, nbh[c], nbl[c], Rr[rt][c],
                         Ri[rt][c]);
        if constexpr (FENCE) __builtin_amdgcn_sched_barrier(0);
    }
}

template <int NRT, int SP, int W>
__device__ __forceinline__ void dma_unit_pre(const CorrLaunch& a, char* __restrict__ sm, const char* Xu, int k,
                                             const char* tt, floatx4 (&Wr)[NRT][(NRT + W - 1) / W],
                                             floatx4 (&Wi)[NRT][(NRT + W - 1) / W], int wv, int lane) {
    constexpr int Np = NRT * 16, CT = (NRT + W - 1) / W, CH = Np / kDmaKC;
    const int col = lane & 15, g = lane >> 4;
    const PreLane pl = pre_lane(col, g);
    dma_issue_pre<NRT, SP, W>(a, sm, Xu, k, tt, 0, 0, wv, lane);
    int s = 0;
    for (int beta = 0; beta < 4; ++beta) {
        const bool cneg = kFold.sink_c[beta] < 0.f;
        for (int ap = 0; ap < 4; ++ap) {
            floatx4 Rr[NRT][CT], Ri[NRT][CT];
#pragma unroll
            for (int r = 0; r < NRT; ++r)
#pragma unroll
                for (int c = 0; c < CT; ++c) {
                    Rr[r][c] = floatx4{0.f, 0.f, 0.f, 0.f};
                    Ri[r][c] = floatx4{0.f, 0.f, 0.f, 0.f};
                }
            const int ne = kFold.n[SP][ap];
            for (int e = 0; e < ne; ++e) {
                const float wf = kFold.w[SP][ap][e];
                const bool neg = (wf < 0.f) != cneg;  // |wf| = 2 is in the doubled tau block
                for (int kc = 0; kc < CH; ++kc, ++s) {
                    const char* sA = dma_advance_pre<NRT, SP, W>(a, sm, Xu, k, tt, s, wv, lane);
                    const char* sB = sA + Np * 256;
                    SplitOp<1> bo[CT];
                    bf16x8 nbh[CT], nbl[CT];
#pragma unroll
                    for (int c = 0; c < CT; ++c) {
                        const int jt = wv + W * c;  // column strip (tile of 16 rows of sB)
                        const char* tile = sB + (jt < NRT ? jt : 0) * 16 * 256;
                        bo[c].rh = pre_read(tile, pl, 0);
                        bo[c].rl = pre_read(tile, pl, 1);
                        bo[c].ih = pre_read(tile, pl, 2);
                        bo[c].il = pre_read(tile, pl, 3);
                        if (neg) {
                            bo[c].rh = bneg(bo[c].rh);
                            bo[c].rl = bneg(bo[c].rl);
                            bo[c].ih = bneg(bo[c].ih);
                            bo[c].il = bneg(bo[c].il);
                        }
                        nbh[c] = bneg(bo[c].ih);
                        nbl[c] = bneg(bo[c].il);
                    }
                    pre_first_product<NRT, CT, (W > 4)>(sA, bo, nbh, nbl, pl, Rr, Ri);
                }
            }
            // W += tau^{alpha a'} R, chunk by chunk over the rows of R (R split on the fly)
#pragma unroll
            for (int kc = 0; kc < CH; ++kc, ++s) {
                const char* sA = dma_advance_pre<NRT, SP, W>(a, sm, Xu, k, tt, s, wv, lane);
                SplitOp<1> bo[CT];
                bf16x8 nbh[CT], nbl[CT];
#pragma unroll
                for (int c = 0; c < CT; ++c) {
                    floatx8 fr, fi;
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int rt2 = 2 * kc + e / 4, v = e % 4;
                        fr[e] = Rr[rt2][c][v];
                        fi[e] = Ri[rt2][c][v];
                    }
                    split8(fr, bo[c].rh, bo[c].rl);
                    split8(fi, bo[c].ih, bo[c].il);
                    nbh[c] = bneg(bo[c].ih);
                    nbl[c] = bneg(bo[c].il);
                }
                pre_first_product<NRT, CT, (W > 4)>(sA, bo, nbh, nbl, pl, Wr, Wi);
            }
        }
    }
}

// Split forms of dma_unit (FORM 1: BF16x3, FORM 2: scaled FP16x3): the same
// chunk schedule and DMA staging; operands are split into hi/lo as they leave
// LDS. K slot j of lane group g of a 32-wide chunk is chunk column 4g + j (j < 4)
// or 16 + 4g + (j - 4): for the second product those are exactly the rows of R a
// lane holds in its accumulators (R tiles 2kc and 2kc+1), and the first product
// uses the same order for both of its operands.
//
// FP16x3 scales: X by sx (per unit) and tau by st (per timeslice) bring their
// largest components near 2^14, so R's accumulator holds R sx st; R enters the
// second product as R sx st 2^-q with q from the bound |R sx st| <= 5 N 2^29
// (at most weight 5 summed over the e terms, N products of components below
// 2^14 * sqrt 2), which keeps it below 2^15. W's accumulator then holds
// W sx st^2 2^-q, one power of two per unit, removed before the sink dot.
template <int FORM>
__device__ __forceinline__ void dma_split_row(const float2* arr, int r, int g, float w, SplitOp<FORM>& o) {
    float re0[4], im0[4], re1[4], im1[4];
    dma_read4(arr, r, 4 * g, re0, im0);
    dma_read4(arr, r, 16 + 4 * g, re1, im1);
    const floatx8 fr = {re0[0] * w, re0[1] * w, re0[2] * w, re0[3] * w, re1[0] * w, re1[1] * w, re1[2] * w, re1[3] * w};
    const floatx8 fi = {im0[0] * w, im0[1] * w, im0[2] * w, im0[3] * w, im1[0] * w, im1[1] * w, im1[2] * w, im1[3] * w};
    SplitT<FORM>::split(fr, o.rh, o.rl);
    SplitT<FORM>::split(fi, o.ih, o.il);
}

template <int NRT, int SP, int FORM>
__device__ __forceinline__ void dma_unit_split(const CorrLaunch& a, float2* __restrict__ sm, const float2* Xu, int k,
                                               const float2* tau_t, float sx, float st,
                                               floatx4 (&Wr)[NRT][LargeGeom<NRT>::CT],
                                               floatx4 (&Wi)[NRT][LargeGeom<NRT>::CT], int wv, int lane) {
    using G = LargeGeom<NRT>;
    using S = SplitT<FORM>;
    constexpr int Np = G::Np, CT = G::CT, CH = (Np + kDmaKC - 1) / kDmaKC;
    const int col = lane & 15, g = lane >> 4;
    const float rq = FORM == 2 ? ldexpf(1.f, -f16_rshift(a.N)) : 1.f;  // scale of R in the second product
    dma_issue<NRT, SP>(a, sm, Xu, k, tau_t, 0, 0, wv, lane);
    int s = 0;
    for (int beta = 0; beta < 4; ++beta) {
        const float cb = kFold.sink_c[beta];
        for (int ap = 0; ap < 4; ++ap) {
            floatx4 Rr[NRT][CT], Ri[NRT][CT];
#pragma unroll
            for (int r = 0; r < NRT; ++r)
#pragma unroll
                for (int c = 0; c < CT; ++c) {
                    Rr[r][c] = floatx4{0.f, 0.f, 0.f, 0.f};
                    Ri[r][c] = floatx4{0.f, 0.f, 0.f, 0.f};
                }
            const int ne = kFold.n[SP][ap];
            for (int e = 0; e < ne; ++e) {
                const float we = kFold.w[SP][ap][e] * cb * st;  // weight +-1 or +-2 and a power of two
                for (int kc = 0; kc < CH; ++kc, ++s) {
                    const float2* sA = dma_advance<NRT, SP>(a, sm, Xu, k, tau_t, s, wv, lane);
                    const float2* sB = sA + Np * kDmaRow;
                    SplitOp<FORM> bo[CT];
#pragma unroll
                    for (int c = 0; c < CT; ++c) {
                        const int j = 16 * (wv + kLargeWaves * c) + col;
                        dma_split_row<FORM>(sB, j < Np ? j : 0, g, we, bo[c]);
                    }
#pragma unroll
                    for (int rt = 0; rt < NRT; ++rt) {
                        SplitOp<FORM> ao;
                        dma_split_row<FORM>(sA, 16 * rt + col, g, sx, ao);
#pragma unroll
                        for (int c = 0; c < CT; ++c)
                            S::cmfma(ao.rh, ao.rl, ao.ih, ao.il, bo[c].rh, bo[c].rl, bo[c].ih, bo[c].il,
                                     S::neg(bo[c].ih), S::neg(bo[c].il), Rr[rt][c], Ri[rt][c]);
                    }
                }
            }
            // W += tau^{alpha a'} R, chunk by chunk over the rows of R
#pragma unroll
            for (int kc = 0; kc < CH; ++kc, ++s) {
                const float2* sA = dma_advance<NRT, SP>(a, sm, Xu, k, tau_t, s, wv, lane);
                SplitOp<FORM> bo[CT];
#pragma unroll
                for (int c = 0; c < CT; ++c) {
                    floatx8 fr, fi;
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int rt2 = 2 * kc + e / 4, v = e % 4;
                        fr[e] = rt2 < NRT ? Rr[rt2 < NRT ? rt2 : 0][c][v] * rq : 0.f;
                        fi[e] = rt2 < NRT ? Ri[rt2 < NRT ? rt2 : 0][c][v] * rq : 0.f;
                    }
                    S::split(fr, bo[c].rh, bo[c].rl);
                    S::split(fi, bo[c].ih, bo[c].il);
                }
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt) {
                    SplitOp<FORM> ao;
                    dma_split_row<FORM>(sA, 16 * rt + col, g, st, ao);
#pragma unroll
                    for (int c = 0; c < CT; ++c)
                        S::cmfma(ao.rh, ao.rl, ao.ih, ao.il, bo[c].rh, bo[c].rl, bo[c].ih, bo[c].il,
                                 S::neg(bo[c].ih), S::neg(bo[c].il), Wr[rt][c], Wi[rt][c]);
                }
            }
        }
    }
    if constexpr (FORM == 2) {  // W sx st^2 2^-q -> W
        const float u = 1.f / (sx * st * st * rq);
#pragma unroll
        for (int r = 0; r < NRT; ++r)
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                Wr[r][c] *= u;
                Wi[r][c] *= u;
            }
    }
}

// FORM 3 (FP64): one column strip per wave (CTX = 1) and ncs workgroups per unit, each
// taking strips wv + 4 cs, so that R and W fit in registers as FP64.
// Up to Np = 64 (four row tiles) every form fits two waves per SIMD (two workgroups per
// CU, 64 KB of LDS each; the FP64 form's one strip per wave within 256 registers), so one
// unit's barrier and chunk wait overlap with the other's MFMAs.
// From Np = 80 (FP32) and at 128 (pre-split BF16x3), where the double-buffered chunks
// leave room for one workgroup per CU, the chains run eight waves, one 16-column strip each
// (waves past the last strip compute a copy of strip 0 that meets zero sink weight), so that
// each SIMD still has two waves (and FP32 room for Gauss's third accumulator set).
template <int NRT, int FORM>
constexpr int dma_waves() { return (FORM == 4 && NRT >= 8) || (FORM == 0 && NRT >= 5) ? 8 : kLargeWaves; }
template <int NRT, int FORM>
constexpr int dma_waves_per_simd() { return dma_waves<NRT, FORM>() == 8 || NRT <= 4 ? 2 : 1; }

template <int NRT, int FORM>
__global__ __launch_bounds__((dma_waves<NRT, FORM>() * 64))
__attribute__((amdgpu_waves_per_eu(dma_waves_per_simd<NRT, FORM>(), dma_waves_per_simd<NRT, FORM>())))
void corr_chain_dma_kernel(BatchRef bt) {
    using G = LargeGeom<NRT>;
    constexpr int W = dma_waves<NRT, FORM>();
    constexpr int CTX = FORM == 3 ? 1 : (NRT + W - 1) / W;
    typedef typename AccT<FORM>::type Acc;
    typedef std::conditional_t<FORM == 3, double, float> Real;
    extern __shared__ float2 smD[];
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    const int inst = find_inst(bt.offs, bt.ninst, item);
    const CorrLaunch a = reinterpret_cast<const CorrLaunch*>(bt.descs)[inst];
    const int N = a.N, N4t = 4 * a.Nt, ncs = a.ncs;
    unsigned bid = item - bt.offs[inst];
    int tmp = bid;
    const int cs = tmp % ncs;
    tmp /= ncs;
    const int k = tmp % N;
    tmp /= N;
    const int sp = tmp % 2;
    tmp /= 2;
    const int b = tmp % a.nprof;
    tmp /= a.nprof;
    const int p = tmp % a.nmom;
    const int tl = tmp / a.nmom;
    const int t = a.t_off + tl;
    const size_t ucore = (((size_t)tl * a.nmom + p) * a.nprof + b) * 2 + sp;
    constexpr int Np = G::Np;
    const float2* Xu = a.X + ucore * 4 * (size_t)Np * Np * Np;
    const float2* tau_t = a.tau + (size_t)t * N4t * N4t;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 15, g = lane >> 4;

    Acc Wr[NRT][CTX], Wi[NRT][CTX];
#pragma unroll
    for (int r = 0; r < NRT; ++r)
#pragma unroll
        for (int c = 0; c < CTX; ++c) {
            Wr[r][c] = Acc{0, 0, 0, 0};
            Wi[r][c] = Acc{0, 0, 0, 0};
        }
    if constexpr (FORM == 4) {
        const char* Xp = reinterpret_cast<const char*>(a.X) + ucore * 4 * (size_t)Np * Np * Np * sizeof(float2);
        const char* tt = reinterpret_cast<const char*>(a.tau16) + (size_t)tl * 4 * kTauBlocks * Np * Np * sizeof(float2);
        if (sp == 0)
            dma_unit_pre<NRT, 0, W>(a, reinterpret_cast<char*>(smD), Xp, k, tt, Wr, Wi, wv, lane);
        else
            dma_unit_pre<NRT, 1, W>(a, reinterpret_cast<char*>(smD), Xp, k, tt, Wr, Wi, wv, lane);
    } else if constexpr (FORM == 1 || FORM == 2) {
        const float sx = FORM == 2 ? a.xscale[ucore * N + k] : 1.f;
        const float st = FORM == 2 ? a.tscale[tl] : 1.f;
        if (sp == 0)
            dma_unit_split<NRT, 0, FORM>(a, smD, Xu, k, tau_t, sx, st, Wr, Wi, wv, lane);
        else
            dma_unit_split<NRT, 1, FORM>(a, smD, Xu, k, tau_t, sx, st, Wr, Wi, wv, lane);
    } else {
        // Gauss's form where its third accumulator set fits without spilling: FP32 in both
        // products (at Np = 112 in the first only); FP64 up to 48 in both and at 64, 80 and
        // 96 in the first (which takes most of the MFMAs)
        constexpr bool GR = (NRT <= 4 || W == 8 || (FORM == 3 && NRT <= 6)) && (FORM == 0 || FORM == 3);
        constexpr bool GW = (NRT <= (FORM == 3 ? 3 : 4) || (W == 8 && NRT != 7)) && (FORM == 0 || FORM == 3);
        if (sp == 0)
            dma_unit<NRT, 0, Real, Acc, CTX, GR, GW, W>(a, smD, Xu, k, tau_t, Wr, Wi, wv, lane, cs);
        else
            dma_unit<NRT, 1, Real, Acc, CTX, GR, GW, W>(a, smD, Xu, k, tau_t, Wr, Wi, wv, lane, cs);
    }

    // sink dot (FP64), waves combined through LDS
    typedef std::conditional_t<FORM == 3, double2, float2> C2;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    double2* red = reinterpret_cast<double2*>(smD);  // [W][kMaxProf]
    const float2* ph = a.phi + ((size_t)(t - a.phi_t) * a.nmom + p) * N * N * N + (size_t)k * N * N;
    C2 qv[NRT][CTX][4];
#pragma unroll
    for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
        for (int c = 0; c < CTX; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = 16 * rt + 4 * g + v, j = 16 * (wv + W * (c + cs)) + col;
                float2 f = make_float2(0.f, 0.f);
                if (i < N && j < N) f = ph[(size_t)i * N + j];
                const Real wr = Wr[rt][c][v], wi = Wi[rt][c][v];
                qv[rt][c][v] = C2{f.x * wr - f.y * wi, f.x * wi + f.y * wr};
            }
    for (int pa = 0; pa < a.nprof; ++pa) {
        const double* ga = a.gsnk + ((size_t)pa * a.T + t) * N;
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int c = 0; c < CTX; ++c) {
            const int j = 16 * (wv + W * (c + cs)) + col;
            const double gj = j < N ? ga[j] : 0.0;
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = 16 * rt + 4 * g + v;
                    const double wgt = (i < N ? ga[i] : 0.0) * gj;
                    sr += wgt * (double)qv[rt][c][v].x;
                    si += wgt * (double)qv[rt][c][v].y;
                }
        }
        sr = wave_sum(sr);
        si = wave_sum(si);
        if (lane == 0) red[wv * kMaxProf + pa] = make_double2(sr, si);
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)a.nprof) {
        const int pa = threadIdx.x;
        double sr = 0.0, si = 0.0;
        for (int w = 0; w < W; ++w) {
            sr += red[w * kMaxProf + pa].x;
            si += red[w * kMaxProf + pa].y;
        }
        const double gk = a.gsnk[((size_t)pa * a.T + t) * N + k];
        a.part[((ucore * N + k) * ncs + cs) * a.nprof + pa] = make_double2(sr * gk, si * gk);
    }
}

template <int NRT, int FORM>
hipError_t launch_dma_t(const BatchRef& b, hipStream_t s) {
    constexpr int Np = NRT * 16;
    const size_t lds = std::max<size_t>((size_t)4 * Np * kDmaRow * sizeof(float2),
                                        (size_t)dma_waves<NRT, FORM>() * kMaxProf * sizeof(double2));
    static std::atomic<unsigned long long> lds_set{0};
    const hipError_t lds_err = lds_limit_once((const void*)corr_chain_dma_kernel<NRT, FORM>, lds, lds_set);
    if (lds_err != hipSuccess) return lds_err;
    hipLaunchKernelGGL((corr_chain_dma_kernel<NRT, FORM>), dim3(b.nitems), dim3(dma_waves<NRT, FORM>() * 64), lds, s,
                       b);
    return hipGetLastError();
}

template <int NRT>
hipError_t launch_large_t(const BatchRef& b, hipStream_t s) {
    const size_t lds = std::max<size_t>((size_t)LargeGeom<NRT>::LDS * sizeof(float2),
                                        (size_t)kLargeWaves * kMaxProf * sizeof(double2));
    static std::atomic<unsigned long long> lds_set{0};
    const hipError_t lds_err = lds_limit_once((const void*)corr_chain_large_kernel<NRT>, lds, lds_set);
    if (lds_err != hipSuccess) return lds_err;
    hipLaunchKernelGGL(corr_chain_large_kernel<NRT>, dim3(b.nitems), dim3(kLargeWaves * 64), lds, s, b);
    return hipGetLastError();
}

// FP16x3 scales. Items [0, Tc): tau(t) of the piece (the N x N blocks in use);
// items [Tc, Tc + units): the four X^{c'}[k] blocks of one unit. Each writes the
// power of two that brings its block's largest |component| into [2^13, 2^14).
__device__ __forceinline__ float block_max(float m) {
    __shared__ float red[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    return fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

__global__ __launch_bounds__(256) void corr_scale_kernel(BatchRef bt) {
    const int item = blockIdx.x;
    const int inst = find_inst(bt.offs, bt.ninst, item);
    const CorrLaunch a = reinterpret_cast<const CorrLaunch*>(bt.descs)[inst];
    const int local = item - bt.offs[inst];
    const int N = a.N, Np = a.Np, Nt = a.Nt, N4t = 4 * Nt;
    float m = 0.f;
    if (local < a.Tc) {
        const float2* tau_t = a.tau + (size_t)(a.t_off + local) * N4t * N4t;
        const int n4 = 4 * N;
        for (int e = threadIdx.x; e < n4 * n4; e += 256) {
            const int r = e / n4, c = e - r * n4;
            const float2 v = tau_t[(size_t)((r / N) * Nt + r % N) * N4t + (c / N) * Nt + c % N];
            m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
        }
        m = block_max(m);
        if (threadIdx.x == 0) a.tscale[local] = f16_scale(m);
    } else {
        const int u = local - a.Tc;  // ucore * N + k
        const size_t ucore = u / N;
        const int k = u - (int)ucore * N;
        const size_t np2 = (size_t)Np * Np;
        const float2* Xu = a.X + ucore * 4 * np2 * Np;
        for (int c = 0; c < 4; ++c) {
            const float4* blk = reinterpret_cast<const float4*>(Xu + ((size_t)c * Np + k) * np2);
            for (size_t e = threadIdx.x; e < np2 / 2; e += 256) {
                const float4 v = blk[e];
                m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
            }
        }
        m = block_max(m);
        if (threadIdx.x == 0) a.xscale[u] = f16_scale(m);
    }
}

// tau(t) of each timeslice of the piece as bf16 hi/lo planes for the pre-split chain:
// [tl][row 4 Np][source spin block][Np / 32 chunks][4 planes][32 slots], blocks 4 and 5
// holding blocks 0 and 1 times 2 (kTauBlocks). One item = one row; the N x N spin blocks
// in use are read, zeros past N.
__global__ __launch_bounds__(256) void corr_split_tau_kernel(BatchRef bt) {
    const int item = blockIdx.x;
    const int inst = find_inst(bt.offs, bt.ninst, item);
    const CorrLaunch a = reinterpret_cast<const CorrLaunch*>(bt.descs)[inst];
    const int local = item - bt.offs[inst];
    const int N = a.N, Np = a.Np, Nt = a.Nt, N4t = 4 * Nt, CH = Np / kDmaKC;
    const int tl = local / (4 * Np), r = local - tl * 4 * Np;
    const int rs = r / Np, ri = r - rs * Np;
    const float2* trow = a.tau + (size_t)(a.t_off + tl) * N4t * N4t + (size_t)(rs * Nt + ri) * N4t;
    uint16_t* dst = a.tau16 + ((size_t)tl * 4 * Np + r) * kTauBlocks * CH * kPreChunkBf16;
    for (int e = threadIdx.x; e < kTauBlocks * Np; e += 256) {
        const int cs = e / Np, ci = e - cs * Np;
        const int src = cs < 4 ? cs : cs - 4;
        const float f = cs < 4 ? 1.f : 2.f;
        const float2 v0 = (ri < N && ci < N) ? trow[src * Nt + ci] : make_float2(0.f, 0.f);
        const float2 v = make_float2(f * v0.x, f * v0.y);
        uint16_t rh, rl, ih, il;
        split_bf16(v.x, rh, rl);
        split_bf16(v.y, ih, il);
        uint16_t* o = dst + (cs * CH + (ci >> 5)) * kPreChunkBf16 + pre_slot(ci & 31);
        o[0] = rh;
        o[32] = rl;
        o[64] = ih;
        o[96] = il;
    }
}

// C[p][t][a][b] = sum over sigma' and k of the unit partials (FP64, fixed order).
// One item = 256 outputs.
__global__ __launch_bounds__(256) void corr_reduce_kernel(BatchRef bt) {
    const int item = blockIdx.x;
    const int inst = find_inst(bt.offs, bt.ninst, item);
    const CorrLaunch a = reinterpret_cast<const CorrLaunch*>(bt.descs)[inst];
    const int total = a.Tc * a.nmom * a.nprof * a.nprof;
    const int idx = (item - bt.offs[inst]) * 256 + threadIdx.x;
    if (idx >= total) return;
    int tmp = idx;
    const int b = tmp % a.nprof;
    tmp /= a.nprof;
    const int pa = tmp % a.nprof;
    tmp /= a.nprof;
    const int p = tmp % a.nmom;
    const int tl = tmp / a.nmom;
    double sr = 0.0, si = 0.0;
    for (int sp = 0; sp < 2; ++sp) {
        const size_t ucore = (((size_t)tl * a.nmom + p) * a.nprof + b) * 2 + sp;
        for (int k = 0; k < a.N; ++k)
            for (int c = 0; c < a.ncs; ++c) {
                const double2 v = a.part[((ucore * a.N + k) * a.ncs + c) * a.nprof + pa];
                sr += v.x;
                si += v.y;
            }
    }
    const int t = a.t_off + tl;
    a.corr[(((size_t)p * a.T + t) * a.nprof + pa) * a.nprof + b] = make_double2(sr, si);
}

}  // namespace

// Column blocks of a step-1 launch: 64-column blocks for the pre-split kernel, the
// triangle of 8 x 8 tiles from Np = 48, Np^2 / 128 below.
int step1_ncb(const CorrLaunch& a) {
    if (a.pre) return a.Np * a.Np / kS1PreBN;
    if (a.Np >= 48) return (a.Np / 8) * (a.Np / 8 + 1) / 2;
    return (a.Np * a.Np + step1_bn(a.Np) - 1) / step1_bn(a.Np);
}

int corr_step1_items(const CorrLaunch& a) {
    const int rows = a.Tc * a.nprof * 2 * 4 * a.Np;
    const int ncb = step1_ncb(a);
    const int nrc = (rows + a.row_chunk - 1) / a.row_chunk;
    return a.nmom * nrc * ncb;
}

int corr_chain_items(const CorrLaunch& a) {
    if (a.Np <= 32) return a.Tc * a.nmom * a.nprof * 2 * ((a.N + kFusedWaves - 1) / kFusedWaves);
    return a.Tc * a.nmom * a.nprof * 2 * a.N * a.ncs;
}

bool corr_pre_split(int N, int Np, int Nt, int precision) {
    return precision == 1 && Np >= 64 && Np % kDmaKC == 0 && N == Np && Nt % 2 == 0;
}

int corr_split_tau_items(const CorrLaunch& a) { return a.Tc * 4 * a.Np; }

hipError_t launch_corr_split_tau(const BatchRef& b, hipStream_t s) {
    if (b.nitems == 0) return hipSuccess;
    hipLaunchKernelGGL(corr_split_tau_kernel, dim3(b.nitems), dim3(256), 0, s, b);
    return hipGetLastError();
}

int corr_col_splits(int N, int Np, int Nt, int precision) {
    return precision == 3 && (corr_chain_class(N, Np, Nt, precision) & kChainDma) && Np >= 80 ? 2 : 1;
}

int corr_reduce_items(const CorrLaunch& a) { return (a.Tc * a.nmom * a.nprof * a.nprof + 255) / 256; }
int corr_scale_items(const CorrLaunch& a) { return a.Tc + a.Tc * a.nmom * a.nprof * 2 * a.N; }

hipError_t launch_corr_scale(const BatchRef& b, hipStream_t s) {
    if (b.nitems == 0) return hipSuccess;
    hipLaunchKernelGGL(corr_scale_kernel, dim3(b.nitems), dim3(256), 0, s, b);
    return hipGetLastError();
}

// Step-1 rows per workgroup: a multiple of 64 that gives the instance about
// s1_target workgroups (fewer for small instances).
void corr_finalize(CorrLaunch& a, int s1_target) {
    const long target = s1_target > 0 ? s1_target : 3072;
    const int rows = a.Tc * a.nprof * 2 * 4 * a.Np;
    const long ncb = step1_ncb(a);
    const long per = (long)rows * ncb * a.nmom;
    a.row_chunk = (int)std::max<long>(S1_BM, (per / target + S1_BM - 1) / S1_BM * S1_BM);
}

template <bool F64>
hipError_t launch_step1_f(int Np, const BatchRef& b, hipStream_t s) {
    switch (Np) {
        case 16: return launch_step1_t<16, 128, F64>(b, s);
        case 32: return launch_step1_t<32, 128, F64>(b, s);
        case 48: return launch_step1_tri_t<48, F64>(b, s);
        case 64: return launch_step1_tri_t<64, F64>(b, s);
        case 80: return launch_step1_tri_t<80, F64>(b, s);
        case 96: return launch_step1_tri_t<96, F64>(b, s);
        case 112: return launch_step1_tri_t<112, F64>(b, s);
        case 128: return launch_step1_tri_t<128, F64>(b, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_corr_step1(int cls, const BatchRef& b, hipStream_t s) {
    if (b.nitems == 0) return hipSuccess;
    if (cls & kStep1Pre) {
        switch (cls & ~kStep1Pre) {
            case 64: return launch_step1_pre_t<64>(b, s);
            case 96: return launch_step1_pre_t<96>(b, s);
            case 128: return launch_step1_pre_t<128>(b, s);
            default: return hipErrorInvalidValue;
        }
    }
    return (cls & kStep1F64) ? launch_step1_f<true>(cls & ~kStep1F64, b, s) : launch_step1_f<false>(cls, b, s);
}

int corr_chain_class(int N, int Np, int Nt, int precision) {
    if (corr_pre_split(N, Np, Nt, precision)) return Np | kChainDma | kChainPre;
    if (Np >= 48 && N == Np && Nt % 2 == 0) return Np | kChainDma;
    return Np;
}

bool corr_bf16x3_supported(int N, int Nt) { return N <= 32 || (N >= 48 && N % 16 == 0 && Nt % 2 == 0); }

hipError_t launch_corr_chain(int cls, int precision, const BatchRef& b, hipStream_t s) {
    if (b.nitems == 0) return hipSuccess;
    const int Np = cls & ~(kChainDma | kChainPre);
    if (cls & kChainPre) {
        switch (Np / 16) {
            case 4: return launch_dma_t<4, 4>(b, s);
            case 6: return launch_dma_t<6, 4>(b, s);
            case 8: return launch_dma_t<8, 4>(b, s);
            default: return hipErrorInvalidValue;
        }
    }
    if (cls & kChainDma) {
#define NUC_DMA_CASE(NRT_)                                                      \
    case NRT_:                                                                  \
        return precision == 3   ? launch_dma_t<NRT_, 3>(b, s)                   \
               : precision == 2 ? launch_dma_t<NRT_, 2>(b, s)                   \
               : precision == 1 ? launch_dma_t<NRT_, 1>(b, s)                   \
                                : launch_dma_t<NRT_, 0>(b, s);
        switch (Np / 16) {
            NUC_DMA_CASE(3)
            NUC_DMA_CASE(4)
            NUC_DMA_CASE(5)
            NUC_DMA_CASE(6)
            NUC_DMA_CASE(7)
            NUC_DMA_CASE(8)
            default: return hipErrorInvalidValue;
        }
#undef NUC_DMA_CASE
    }
    if (Np == 16)
        return precision == 3   ? launch_small_t<1, 3>(b, s)
               : precision == 2 ? launch_small_t<1, 2>(b, s)
               : precision == 1 ? launch_small_t<1, 1>(b, s)
                                : launch_small_t<1, 0>(b, s);
    if (Np == 32)
        return precision == 3   ? launch_small_t<2, 3>(b, s)
               : precision == 2 ? launch_small_t<2, 2>(b, s)
               : precision == 1 ? launch_small_t<2, 1>(b, s)
                                : launch_small_t<2, 0>(b, s);
    if (precision != 0) return hipErrorInvalidValue;
    switch (Np / 16) {
        case 3: return launch_large_t<3>(b, s);
        case 4: return launch_large_t<4>(b, s);
        case 5: return launch_large_t<5>(b, s);
        case 6: return launch_large_t<6>(b, s);
        case 7: return launch_large_t<7>(b, s);
        case 8: return launch_large_t<8>(b, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_corr_reduce(const BatchRef& b, hipStream_t s) {
    if (b.nitems == 0) return hipSuccess;
    hipLaunchKernelGGL(corr_reduce_kernel, dim3(b.nitems), dim3(256), 0, s, b);
    return hipGetLastError();
}

}  // namespace nuc

// Internal declarations shared by the HIP kernels and the host runtime of the
// nucleon-correlator library (gfx950 / CDNA4 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <atomic>

namespace nuc {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kMaxNvec = 128;

// Raise a kernel's dynamic-LDS limit to `bytes` on the current device, once per device
// (the attribute is per device; `done` holds one bit per device ordinal, one flag set
// per kernel instantiation whose LDS size is fixed by its template parameters).
inline hipError_t lds_limit_once(const void* fn, size_t bytes, std::atomic<unsigned long long>& done) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const unsigned long long bit = 1ull << (dev & 63);
    if (done.load(std::memory_order_acquire) & bit) return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) done.fetch_or(bit, std::memory_order_acq_rel);
    return e;
}
constexpr int kMaxProf = 16;

// ---------------------------------------------------------------- device helpers
// Pointer types of global_load_lds (global source, LDS destination).
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void gbl_void_t;

// 16x16x4 FP32 MFMA. Lane l supplies A[l%16][l/16] and B[l/16][l%16]; the
// accumulator holds D[4*(l/16)+v][l%16] in element v.
__device__ __forceinline__ floatx4 mfma16x4(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Complex multiply-accumulate of one 16x16x4 step with four real MFMAs:
// (cr + i ci) += (ar + i ai)(br + i bi).
__device__ __forceinline__ void cmfma16x4(float ar, float ai, float br, float bi, floatx4& cr,
                                          floatx4& ci) {
    cr = mfma16x4(ar, br, cr);
    cr = mfma16x4(-ai, bi, cr);
    ci = mfma16x4(ar, bi, ci);
    ci = mfma16x4(ai, br, ci);
}

// 16x16x4 FP64 MFMA. Lane l supplies A[l%16][l/16] and B[l/16][l%16] as in mfma16x4,
// but element v of the accumulator holds D[4*v+l/16][l%16] (rows interleaved, not
// blocked). A product of two FP32 values is exact in FP64, so on FP32 data it rounds
// only in the accumulation.
typedef double doublex4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ doublex4 dmfma16x4(double a, double b, doublex4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Row of its tile that lane column `col` feeds into an MFMA's A operand. The FP64 form
// feeds row (col%4)*4 + col/4 in place of row col: the accumulator's element v then holds
// logical row 4*(l/16)+v, the FP32 layout, so every consumer of the accumulators
// (stores, sink dots, accumulators reused as the next product's B operand) is shared.
__device__ __forceinline__ int arow(int col, bool f64) { return f64 ? ((col & 3) << 2) | (col >> 2) : col; }

// The accumulator of a precision form: FP64 for the FP64 form (3), FP32 otherwise.
template <int FORM>
struct AccT {
    typedef floatx4 type;
};
template <>
struct AccT<3> {
    typedef doublex4 type;
};

// Complex multiply-accumulate of one 16x16x4 step in either precision:
// (cr + i ci) += (ar + i ai)(br + i bi), four real MFMAs.
__device__ __forceinline__ void cmac(float ar, float ai, float br, float bi, floatx4& cr, floatx4& ci) {
    cmfma16x4(ar, ai, br, bi, cr, ci);
}
// One real MFMA step of the accumulator's precision.
__device__ __forceinline__ floatx4 rmfma(float a, float b, floatx4 c) { return mfma16x4(a, b, c); }
__device__ __forceinline__ doublex4 rmfma(double a, double b, doublex4 c) { return dmfma16x4(a, b, c); }

__device__ __forceinline__ void cmac(double ar, double ai, double br, double bi, doublex4& cr, doublex4& ci) {
    cr = dmfma16x4(ar, br, cr);
    cr = dmfma16x4(-ai, bi, cr);
    ci = dmfma16x4(ar, bi, ci);
    ci = dmfma16x4(ai, br, ci);
}

// ------------------------------------------------------------- split bfloat16
// x = hi + lo with hi = bf16(x) (round to nearest even) and lo = bf16(x - hi);
// products hi*hi + hi*lo + lo*hi on bf16 MFMA with FP32 accumulation ("BF16x3").
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void split8(floatx8 f, bf16x8& hi, bf16x8& lo) {
    hi = __builtin_convertvector(f, bf16x8);
    const floatx8 fh = __builtin_convertvector(hi, floatx8);
    lo = __builtin_convertvector(f - fh, bf16x8);
}

__device__ __forceinline__ bf16x8 bneg(bf16x8 x) {
    uint4 u = __builtin_bit_cast(uint4, x);
    u.x ^= 0x80008000u;
    u.y ^= 0x80008000u;
    u.z ^= 0x80008000u;
    u.w ^= 0x80008000u;
    return __builtin_bit_cast(bf16x8, u);
}

__device__ __forceinline__ floatx4 mfma16x32bf(bf16x8 a, bf16x8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// (cr + i ci) += (ar + i ai)(br + i bi), every real product as hi*hi + hi*lo + lo*hi.
// nbi_* are the negated imaginary parts of b.
__device__ __forceinline__ void cmfma_bf16x3(bf16x8 arh, bf16x8 arl, bf16x8 aih, bf16x8 ail, bf16x8 brh,
                                             bf16x8 brl, bf16x8 bih, bf16x8 bil, bf16x8 nbih, bf16x8 nbil,
                                             floatx4& cr, floatx4& ci) {
    cr = mfma16x32bf(arh, brh, cr);
    cr = mfma16x32bf(arh, brl, cr);
    cr = mfma16x32bf(arl, brh, cr);
    cr = mfma16x32bf(aih, nbih, cr);
    cr = mfma16x32bf(aih, nbil, cr);
    cr = mfma16x32bf(ail, nbih, cr);
    ci = mfma16x32bf(arh, bih, ci);
    ci = mfma16x32bf(arh, bil, ci);
    ci = mfma16x32bf(arl, bih, ci);
    ci = mfma16x32bf(aih, brh, ci);
    ci = mfma16x32bf(aih, brl, ci);
    ci = mfma16x32bf(ail, brh, ci);
}

// --------------------------------------------------------- scaled split FP16
// x s = hi + lo with hi = fp16(x s), lo = fp16(x s - hi) (round to nearest even),
// s a power of two that brings the block's largest |x| near 2^14 ("FP16x3":
// products hi*hi + hi*lo + lo*hi on fp16 MFMA with FP32 accumulation).
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void split8h(floatx8 f, f16x8& hi, f16x8& lo) {
    hi = __builtin_convertvector(f, f16x8);
    const floatx8 fh = __builtin_convertvector(hi, floatx8);
    lo = __builtin_convertvector(f - fh, f16x8);
}

__device__ __forceinline__ f16x8 hneg(f16x8 x) {
    uint4 u = __builtin_bit_cast(uint4, x);
    u.x ^= 0x80008000u;
    u.y ^= 0x80008000u;
    u.z ^= 0x80008000u;
    u.w ^= 0x80008000u;
    return __builtin_bit_cast(f16x8, u);
}

__device__ __forceinline__ floatx4 mfma16x32h(f16x8 a, f16x8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void cmfma_f16x3(f16x8 arh, f16x8 arl, f16x8 aih, f16x8 ail, f16x8 brh, f16x8 brl,
                                            f16x8 bih, f16x8 bil, f16x8 nbih, f16x8 nbil, floatx4& cr,
                                            floatx4& ci) {
    cr = mfma16x32h(arh, brh, cr);
    cr = mfma16x32h(arh, brl, cr);
    cr = mfma16x32h(arl, brh, cr);
    cr = mfma16x32h(aih, nbih, cr);
    cr = mfma16x32h(aih, nbil, cr);
    cr = mfma16x32h(ail, nbih, cr);
    ci = mfma16x32h(arh, bih, ci);
    ci = mfma16x32h(arh, bil, ci);
    ci = mfma16x32h(arl, bih, ci);
    ci = mfma16x32h(aih, brh, ci);
    ci = mfma16x32h(aih, brl, ci);
    ci = mfma16x32h(ail, brh, ci);
}

// Power of two s with max_abs * s in [2^13, 2^14) (1 for a zero block).
__device__ __forceinline__ float f16_scale(float max_abs) {
    if (!(max_abs > 0.f)) return 1.f;
    int e;
    frexpf(max_abs, &e);  // max_abs = m 2^e, m in [0.5, 1)
    return ldexpf(1.f, 14 - e);
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Workgroups are dispatched round-robin over the 8 XCDs (bid % 8). Map them so
// each XCD works through one contiguous range of logical work items, which keeps
// the data those items share inside that XCD's L2. Bijective on [0, n).
__device__ __forceinline__ unsigned xcd_remap(unsigned bid, unsigned n) {
    unsigned q = n / 8u, r = n % 8u, x = bid % 8u, loc = bid / 8u;
    return x * q + (x < r ? x : r) + loc;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ---------------------------------------------------------------- kernel launchers
//
// Every kernel is launched over the work items of one or more instances of the
// same shape class (a batch). The per-instance launch structs live in device
// memory; offs[i] is the first item of instance i (offs[ninst] = nitems), and a
// workgroup finds its instance with find_inst().

struct BatchRef {
    const void* descs;  // device array of ElemLaunch or CorrLaunch
    const int* offs;    // device [ninst + 1]
    int ninst;
    int nitems;
};

// item is the same in every lane of a workgroup, so is the result; saying so
// lets the compiler fetch the instance's launch struct with scalar loads.
__device__ __forceinline__ int find_inst(const int* offs, int ninst, int item) {
    int lo = 0, hi = ninst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (offs[mid] <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

// Load through a global-address-space pointer (a global_load rather than a
// flat load, which also waits on the LDS counter).
__device__ __forceinline__ float gld(const float* p) { return *(const __attribute__((address_space(1))) float*)p; }
__device__ __forceinline__ double gld(const double* p) { return *(const __attribute__((address_space(1))) double*)p; }
__device__ __forceinline__ float2 gld(const float2* p) {
    typedef float f2v __attribute__((ext_vector_type(2)));
    const f2v x = *(const __attribute__((address_space(1))) f2v*)p;
    return make_float2(x.x, x.y);
}

// Pair set of the elementals. With 16-index blocks, a triple i<j<k either has two
// indices in one block or lies in three blocks. The pairs inside one block take every
// row tile (rows below the pair's block, or below j in it, as the smallest index; rows
// beyond the pair's block as the largest, Phi_rjk = Phi_jkr by cyclic symmetry). For
// the triples in three blocks the blocks are cut into a lower half [0, h) and an upper
// half [h, nb): a pair across two lower blocks takes the row tiles above its k's block
// (the row is the largest index), a pair across two upper blocks the tiles below its
// j's block (the row is the smallest), and pairs with one index in each half are not
// built. Two of a triple's three blocks lie in one half, so exactly one of its pairs
// is in the set and reaches it. With half the blocks on each side this needs the
// fewest cross-block pairs for which every three-block triple still has one (the
// block pairs left out form the complete bipartite graph between the halves, the
// largest graph on nb blocks without a triangle): 512 instead of 768 at N = 64 and
// 3072 instead of 5376 at N = 128, for the same MFMA tiles. Used from 20 vectors on; below
// that the plain set of all pairs j<k with the rows below j.
__host__ __device__ inline bool elem_block_pairs(int N) { return N >= 20; }
// Elementals workgroup: waves of 16 pairs each; four (two workgroups per CU) up to 32
// vectors, eight (one workgroup per CU, two waves per SIMD, half the staging per pair)
// beyond (measured: 32 vectors run faster with four, 64 and more with eight).
__host__ __device__ constexpr int elem_waves(int N) { return N > 32 ? 8 : 4; }
__host__ __device__ inline int elem_half(int N) { return (((N + 15) >> 4) + 1) >> 1; }
__host__ __device__ inline bool elem_pair_in_set(int N, int j, int k) {
    if (!elem_block_pairs(N)) return true;
    const int bj = j >> 4, bk = k >> 4, h = elem_half(N);
    return bj == bk || bk < h || bj >= h;
}

// Row tiles [x, y) of 16 rows a pair (j, k) of the set needs. The rows of a tile that
// the pair owns: all of them, except in j's own tile (rows below j only) and past N.
__host__ __device__ inline int2 elem_row_range(int N, int2 p) {
    const int nb = (N + 15) >> 4;
    if (!elem_block_pairs(N)) return make_int2(0, (p.x + 15) >> 4);
    const int bj = p.x >> 4, bk = p.y >> 4;
    if (bj == bk) return make_int2(0, nb);
    return bk < elem_half(N) ? make_int2(bk + 1, nb) : make_int2(0, bj);
}

struct ElemLaunch {
    const float2* evecs;  // [T][N][V3][3]
    const int* mom;       // [nmom][3]
    const int2* pairs;    // [npairs] (j,k), j<k: all, lexicographic; or the block pair set (elem_block_pairs), by row range
    const int2* work;     // [nwork] (chunk of 4 row tiles from the wave's first, pair-block)
    double2* part;        // [nsplit][Tc][nmom][C3] canonical FP64 partial sums
    float2* packed;       // [Tc][nmom][C3] canonical entries after the FP64 split sum
    float2* phi;          // [..][nmom][N^3], timeslice t at row t - phi_t
    int phi_t;
    int T, N, L, V3, nmom, npairs, nwork, nsplit, C3;
    int t_off, Tc;        // timeslices [t_off, t_off+Tc) in this launch
    int sites_per_split, npgroup;
    size_t ev_tstride;    // complex elements between timeslices of evecs (N_ld * V3 * 3)
    int mp;               // momenta (row tiles) per wave: 1, 2 or 4; 0 = by nmom
    int f64;              // 1: FP64 MFMA on the FP32 inputs, the whole site range in FP64
};

// Items per instance of each elementals kernel, and the shape class (template
// parameters) an instance belongs to.
int elem_items(const ElemLaunch& a);
int elem_reduce_items(const ElemLaunch& a);
int elem_expand_items(const ElemLaunch& a);
int elem_class(const ElemLaunch& a);
constexpr int kElemF64 = 0x400;  // elementals class bit of the FP64 form
void elem_finalize(ElemLaunch& a);  // fills sites_per_split and npgroup
hipError_t launch_elementals(int cls, const BatchRef& b, hipStream_t s);
hipError_t launch_elem_reduce(const BatchRef& b, hipStream_t s);
hipError_t launch_elem_expand(const BatchRef& b, hipStream_t s);

// Source spin tensor of the Wick-folded contraction, grouped by source spin a':
// for sigma' in {0,1}, a' in 0..3: n entries (b', c', weight), where
//   s'_{a'b'c'} = (C g5)_{a'b'} delta_{c' sigma'} + (C g5)_{c'b'} delta_{a' sigma'},
// and the sink pairs (alpha(beta), beta) with (C g5)_{alpha beta} != 0.
// (C gamma5) in the Dirac-Pauli basis is real and antisymmetric with nonzeros
// (0,1) = -1, (1,0) = 1, (2,3) = -1, (3,2) = 1.
struct SpinFold {
    int n[2][4];
    int bp[2][4][4];
    int cp[2][4][4];
    float w[2][4][4];
    int sink_a[4];    // sink pair partner alpha(beta) of each beta
    float sink_c[4];  // (C gamma5)_{alpha(beta) beta}
};

constexpr float kCg5[4][4] = {{0, -1, 0, 0}, {1, 0, 0, 0}, {0, 0, 0, -1}, {0, 0, 1, 0}};

constexpr SpinFold make_spin_fold() {
    SpinFold f{};
    for (int s = 0; s < 2; ++s)
        for (int ap = 0; ap < 4; ++ap)
            for (int bp = 0; bp < 4; ++bp)
                for (int cp = 0; cp < 4; ++cp) {
                    const float w = kCg5[ap][bp] * (cp == s ? 1.f : 0.f) + kCg5[cp][bp] * (ap == s ? 1.f : 0.f);
                    if (w != 0.f) {
                        const int n = f.n[s][ap]++;
                        f.bp[s][ap][n] = bp;
                        f.cp[s][ap][n] = cp;
                        f.w[s][ap][n] = w;
                    }
                }
    for (int beta = 0; beta < 4; ++beta)
        for (int al = 0; al < 4; ++al)
            if (kCg5[al][beta] != 0.f) {
                f.sink_a[beta] = al;
                f.sink_c[beta] = kCg5[al][beta];
            }
    return f;
}

constexpr SpinFold kFold = make_spin_fold();

// Source-spin blocks per row of the pre-split tau planes: the four blocks of tau(t), then
// blocks 0 and 1 again times 2. A fold entry of weight +-2 has c' = a' = sigma' and b' the
// partner of sigma' in C gamma5 (1 - sigma'), so it reads block 4 + b' instead of issuing its
// products twice (doubling a bf16 value is exact).
constexpr int kTauBlocks = 6;
constexpr bool fold_doubles_fit() {
    for (int s = 0; s < 2; ++s)
        for (int ap = 0; ap < 4; ++ap)
            for (int e = 0; e < kFold.n[s][ap]; ++e) {
                const float w = kFold.w[s][ap][e];
                if ((w == 2.f || w == -2.f) && kFold.bp[s][ap][e] >= kTauBlocks - 4) return false;
                if (w != 1.f && w != -1.f && w != 2.f && w != -2.f) return false;
            }
    return true;
}
static_assert(fold_doubles_fit(), "every fold weight is +-1 or +-2, the latter on a doubled block");

struct CorrLaunch {
    const float2* phi;    // sink elementals [..][nmom][N^3], timeslice t at row t - phi_t
    const float2* phi0;   // source elementals Phi(t0) [nmom][N^3]
    int phi_t;
    const float2* tau;    // [T][4N][4N]
    const double* gsnk;   // [nprof][T][N]
    const double* gsrc;   // [nprof][N]   (profiles at t0)
    const float* gsrc_f;  // the same rounded to FP32 (the precision step 1 applies them in)
    float2* X;            // [Tc][nmom][nprof][2][4][Np][Np][Np]
    double2* part;        // [Tc][nmom][nprof][2][N][ncs][nprof]
    double2* corr;        // [nmom][T][nprof][nprof]
    int T, N, Np, nmom, nprof, t0, t_off, Tc;
    int Nt;               // block size of tau ([T][4 Nt][4 Nt]); the first N of each block are used
    int precision;        // 0 FP32, 1 BF16x3, 2 FP16x3 (scaled), 3 FP64
    int ncs;              // workgroups sharing one chain unit's columns (FP64 chains at Np >= 80: 2)
    float* tscale;        // FP16x3: [Tc] power-of-two scale of tau(t)
    float* xscale;        // FP16x3: [Tc][nmom][nprof][2][N] power-of-two scale of a unit's X blocks
    int row_chunk;        // step 1: rows per workgroup (multiple of 64)
    int pre;              // BF16x3 with operands split ahead (corr_pre_split): X holds bf16 planes
    uint16_t* tau16;      // pre: [Tc][4 Np][kTauBlocks][Np/32][4 planes][32] bf16 planes of tau(t)
};

// BF16x3 operands split ahead of the chain: for the LDS-DMA chain with Np a multiple
// of 32, step 1 writes X and a prep kernel writes tau(t) as bf16 hi/lo planes, so the
// chain's MFMA operands come from LDS ready-made.
bool corr_pre_split(int N, int Np, int Nt, int precision);
constexpr int kChainPre = 0x200;  // chain class bit of that path
int corr_split_tau_items(const CorrLaunch& a);
hipError_t launch_corr_split_tau(const BatchRef& b, hipStream_t s);

int corr_step1_items(const CorrLaunch& a);
int corr_chain_items(const CorrLaunch& a);
int corr_reduce_items(const CorrLaunch& a);
void corr_finalize(CorrLaunch& a, int s1_target);  // row_chunk for ~s1_target step-1 workgroups (0 = 3072)
// Chain shape class of an instance: Np, plus kChainDma when the LDS-DMA kernel
// applies (N = Np >= 48, even tau block size, FP32). Step-1 class: Np.
constexpr int kChainDma = 0x100;
int corr_chain_class(int N, int Np, int Nt, int precision);
// BF16x3, FP16x3 and FP64 chains exist for N <= 32 and for N = Np >= 48 with an even
// tau block size.
bool corr_bf16x3_supported(int N, int Nt);
// Workgroups per chain unit: 2 for the FP64 LDS-DMA chain at Np >= 80 (each takes
// half of the unit's 16-column strips, which keeps its FP64 accumulators in
// registers), else 1.
int corr_col_splits(int N, int Np, int Nt, int precision);
// Step-1 shape class: Np, plus kStep1F64 for the FP64 form or kStep1Pre for the
// pre-split BF16x3 path (X written as bf16 planes).
constexpr int kStep1F64 = 0x200;
constexpr int kStep1Pre = 0x400;
hipError_t launch_corr_step1(int Np, const BatchRef& b, hipStream_t s);
hipError_t launch_corr_chain(int cls, int precision, const BatchRef& b, hipStream_t s);
hipError_t launch_corr_reduce(const BatchRef& b, hipStream_t s);
// FP16x3 scales: one item per timeslice (tau) and per unit (X), in one launch.
int corr_scale_items(const CorrLaunch& a);
hipError_t launch_corr_scale(const BatchRef& b, hipStream_t s);

}  // namespace nuc

// Internals of the meson-operator path shared by its kernel files
// (meson_elem.hip: derivatives, phase-weighted vectors, elemental GEMM; meson_corr.hip:
// profile weighting, operator products, traces) and its host runtime (meson.hip):
// launch argument structs, tile constants and the launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nuc_internal.h"

namespace nuc {
namespace meson {

constexpr int kMaxNvecMeson = 512;
constexpr int kND = 7;       // D = 1, nabla_0..2, B_0..2
constexpr int kNFam = 3;     // g4 g5; g4 g5 g_k nabla_k; g_k B_k
constexpr int EKC = 32;    // complex K values per stage (one staged row)
constexpr int kElemNB = 2;  // column blocks per wave of the elemental GEMM
constexpr int TCH = 64;        // elements per LDS stage

// Operand sources, resolved per (t, p) inside the kernel.
enum { SRC_PS = 0, SRC_PT = 1, SRC_TAU = 2, SRC_Y = 3, SRC_Z = 4 };

struct DerivArgs {
    const float2* v;  // distillation vectors from timeslice t_off on: [.][N][V3][3]
    const float2* U;  // links from timeslice t_off on: [.][V3][3 dir][3][3]
    float2* F;        // [Tc][6][N][Kp]: nabla_0..2 v, then B_0..2 v (K = 3 V3 values, zero pad)
    int L, V3, N, Tc, jchunk, Kp;
};


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


struct ElemArgs {
    const float2* A;   // [Tc][nmom][N][Kp] phase-weighted conjugate vectors
    const float2* V;   // [Tc][N][Kp] the vectors (D = 1)
    const float2* F;   // [Tc][6][N][Kp] the derivative fields (D = nabla_k, B_k)
    double2* part;     // [nsplit][Tc][nmom][N][7N]
    int N, K, Kp, nmom, Tc, nsplit, cps, nchunks, mt, nt;
};


// Workgroup tile: 64 rows (i) x ETN columns ((D, j)), four waves as 2 x 2, each wave
// 32 x (16 NB) complex outputs.
template <int NB>
struct ElemTile {
    static constexpr int TN = 2 * 16 * NB;            // columns per workgroup
    static constexpr int ROWS = 64 + TN;              // staged rows per stage (A then B)
    static constexpr int SMEM = 2 * ROWS * EKC;       // float2, double buffer
};


struct ElemReduceArgs {
    const double2* part;  // [nsplit][Tc][nmom][N][7N]
    float2* phi;          // [T][nmom][7][N][N]
    int N, nmom, Tc, nsplit, t_off;
};


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


struct TraceArgs {
    const float2* Y;   // [Tc][nmom][nop][4N][4N]
    const float2* Z;
    double2* part;     // [Tc][nmom][nwg][nop][nop]
    int N, nop, nmom, nwg, cpb;  // cpb: stages per row block of N x 4N elements
    int pi5[4];        // Z row block paired with Y row block gamma
    float2 s5[4];      // and its factor: C += Y conj(s5 Z)
};


struct SumArgs {
    const double2* part;  // [Tc][nmom][nwg][nop][nop]
    double2* corr;        // [nmom][T][nop][nop]
    int T, nop, nmom, nwg, Tc, t_off;
};


// Launchers (each computes its grid from the arguments).
hipError_t launch_deriv(int pass, const DerivArgs& a, hipStream_t s);
hipError_t launch_phase(const PhaseArgs& a, hipStream_t s);
hipError_t launch_elem(const ElemArgs& a, hipStream_t s);
hipError_t launch_elem_reduce(const ElemReduceArgs& a, hipStream_t s);
hipError_t launch_weight(const WeightArgs& a, size_t nel, hipStream_t s);
hipError_t launch_gemm(const GemmArgs& a, unsigned nblk, hipStream_t s);
hipError_t launch_trace(const TraceArgs& a, int ntp, hipStream_t s);
hipError_t launch_sum(const SumArgs& a, int nsum, hipStream_t s);

}  // namespace meson
}  // namespace nuc

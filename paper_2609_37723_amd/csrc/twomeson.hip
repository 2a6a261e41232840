// Two-meson correlators on gfx950: the I=2 A1++ operator of the charmonium study
// (paper Section 3) built from an optimal one-meson operator, at zero total momentum
// with back-to-back momenta, O(t) = sum_k pi+(p_k, t) pi+(-p_k, t).
//
//   M_w(t, p) = sum_A w_A M_A(t, p),  Mbar_l = g4 M_w(t0, p_l)^H g4,  tau~ = g5 tau^H g5,
//   L_k = M_w(t, p_k) tau,  R_l = Mbar_l tau~,  P_kl = L_k R_l,
//   C(t) = 2 sum_{k,l} (Tr P_kl Tr P_kbar,lbar - Tr[P_kl P_kbar,lbar])
// (direct minus crossed Wick terms; kbar is the index of -p_k).
//
// Method. The operator kernel forms the dense optimal operators from the elementals
// (profile weights and spin terms applied on the fly), L and R are batched FP32 MFMA
// complex GEMMs, and the pair kernel never stores P: a workgroup computes tile (I, J)
// of A = L_a R_b and tile (I, J) of B^T = (L_c R_d)^T (the second with the operand roles
// swapped: rows from R_d's columns, columns from L_c's rows), so the tiles line up
// element by element in the MFMA output layout and Tr[A B] = sum A .* B^T reduces in
// registers in FP64, with Tr A and Tr B from the diagonal tiles (complex products in
// Gauss's three-multiplication form: three real MFMAs per complex step). The pair (k, l) and
// its partner (kbar, lbar) are one work item; a self-partnered pair (p = 0 on both
// sides) computes only the tiles I <= J, the off-diagonal ones counted twice.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <complex>
#include <vector>

#include "../../include/nucleon.h"
#include "cgemm.h"
#include "meson_spin.h"
#include "runtime_internal.h"

namespace nuc {
namespace twomeson {

constexpr size_t kTmCap = (size_t)16 << 30;
constexpr int kMaxMom = 48;
constexpr int kMaxTerm = 7;   // (Gamma, D) terms that can meet one spin block
constexpr int kGroupI = 4;    // tile rows per group of the pair work list

// ------------------------------------------------------------------ operators

struct SpinTable {
    float2 coef[16][kMaxTerm];  // Gamma[alpha][beta] of each term meeting block (alpha, beta)
    int fd[16][kMaxTerm];       // family * 8 + D of the term
    int nterm[16];
    float g4[4];                // gamma_4 diagonal
    int col5[4];                // gamma_5 as a signed permutation: column of row alpha
    float v5[4];                // and its (real) value
};

struct OpArgs {
    const float2* phi;   // [T][nmom][7][N][N]
    const float* g;      // [nprof][T][N]
    const float2* w;     // [3][nprof]
    float2* out;         // sink: [tc][nmom][4N][4N]; source: [nmom][4N][4N]
    int N, T, nmom, nprof, t_off, t0;
    SpinTable tab;
};

// One thread per (unit, i, j): the three profile weights W_f = sum_a w_fa g_i g_j, the
// seven elementals at (i, j), then all 16 spin blocks. SOURCE writes
// Mbar[(alpha, j), (beta, i)] = g4_alpha g4_beta conj(M[(beta, i), (alpha, j)]).
template <bool SOURCE>
__global__ __launch_bounds__(256) void tm_operator_kernel(OpArgs a) {
    const int unit = blockIdx.y;  // sink: tl * nmom + p; source: p
    const int e = blockIdx.x * 256 + threadIdx.x;
    const int N = a.N, N4 = 4 * N;
    if (e >= N * N) return;
    const int i = e / N, j = e - i * N;
    const int t = SOURCE ? a.t0 : a.t_off + unit / a.nmom;
    const int p = SOURCE ? unit : unit % a.nmom;
    float2 W[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) W[f] = make_float2(0.f, 0.f);
    for (int b = 0; b < a.nprof; ++b) {
        const float gg = a.g[((size_t)b * a.T + t) * N + i] * a.g[((size_t)b * a.T + t) * N + j];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const float2 wf = a.w[f * a.nprof + b];
            W[f].x += wf.x * gg;
            W[f].y += wf.y * gg;
        }
    }
    const float2* ph = a.phi + ((size_t)t * a.nmom + p) * 7 * N * N + e;
    float2 G[3][7];  // W_f * Phi^D, only the (f, D) pairs the families use are read
#pragma unroll
    for (int d = 0; d < 7; ++d) {
        const float2 v = gld(ph + (size_t)d * N * N);
#pragma unroll
        for (int f = 0; f < 3; ++f) G[f][d] = cmul(W[f], v);
    }
    float2* out = a.out + (size_t)unit * N4 * N4;
#pragma unroll
    for (int ab = 0; ab < 16; ++ab) {
        const int al = ab >> 2, be = ab & 3;
        float2 s = make_float2(0.f, 0.f);
        for (int q = 0; q < a.tab.nterm[ab]; ++q) {
            const int fd = a.tab.fd[ab][q];
            float2 gv = G[0][0];
#pragma unroll
            for (int f = 0; f < 3; ++f)
#pragma unroll
                for (int d = 0; d < 7; ++d)
                    if (fd == f * 8 + d) gv = G[f][d];
            const float2 c = cmul(a.tab.coef[ab][q], gv);
            s.x += c.x;
            s.y += c.y;
        }
        if (SOURCE) {
            const float sg = a.tab.g4[al] * a.tab.g4[be];
            out[(size_t)(be * N + j) * N4 + al * N + i] = make_float2(sg * s.x, -sg * s.y);
        } else {
            out[(size_t)(al * N + i) * N4 + be * N + j] = s;
        }
    }
}

// tau~(t) = g5 tau(t)^H g5: tau~[(al, i), (be, j)] = v5[al] v5[be'] conj(tau[(be', j), (col5[al], i)])
// with be' the row of gamma_5 whose column is be. A 32 x 32 output tile per workgroup,
// transposed through LDS so reads and writes are both row-contiguous.
struct BackArgs {
    const float2* tau;  // [T][4N][4N]
    float2* out;        // [tc][4N][4N]
    int N, t_off;
    SpinTable tab;
};

__global__ __launch_bounds__(256) void tm_back_kernel(BackArgs a) {
    __shared__ float2 tile[32][33];
    const int N4 = 4 * a.N;
    const int tl = blockIdx.z;
    const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
    const float2* tau = a.tau + (size_t)(a.t_off + tl) * N4 * N4;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    // read: output column c = c0 + (ty + 8 m) maps to source row; output row r = r0 + tx to source column
    const int r = r0 + tx;
    int srccol = 0;
    float vr = 0.f;
    if (r < N4) {
        const int al = r / a.N, i = r - al * a.N;
        srccol = a.tab.col5[al] * a.N + i;
        vr = a.tab.v5[al];
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int c = c0 + ty + 8 * m;
        if (r < N4 && c < N4) {
            const int be = c / a.N, j = c - be * a.N;
            int bp = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (a.tab.col5[q] == be) bp = q;
            const float2 v = gld(tau + (size_t)(bp * a.N + j) * N4 + srccol);
            const float sg = vr * a.tab.v5[bp];
            tile[tx][ty + 8 * m] = make_float2(sg * v.x, -sg * v.y);
        }
    }
    __syncthreads();
    float2* out = a.out + (size_t)tl * N4 * N4;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int rr = r0 + ty + 8 * m, cc = c0 + tx;
        if (rr < N4 && cc < N4) out[(size_t)rr * N4 + cc] = tile[ty + 8 * m][tx];
    }
}

// ------------------------------------------------------------------ pair GEMM

constexpr int PKC = 32;   // complex K per LDS stage
constexpr int PAP = PKC + 2;  // row-major panel [64][PKC] pitch
constexpr int PBP = 80;   // K-major panel [PKC][64] pitch
constexpr int kRQ = PKC / 8;    // row-major panel elements per thread (512 threads)
constexpr int kRS = 512 / PKC;  // row stride between them
constexpr int kKQ = PKC / 16;   // K rows per thread of a K-major panel (two columns each)
constexpr int PXP = 65;   // exchange tile [64][64] pitch
constexpr int kPanelRM = 64 * PAP, kPanelKM = PKC * PBP;
constexpr int kPairSmem = 2 * 2 * kPanelRM + 2 * 2 * kPanelKM;  // float2; >= 64 PXP
static_assert(kPairSmem >= 64 * PXP, "exchange tile must fit the staging buffers");

struct PairArgs {
    const float2* L;     // [tc][nmom][n][n]
    const float2* R;     // [tc][nmom][n][n]
    const int4* items;   // [nitems]: (pair, I, J, weight)
    const int4* pairs;   // [npair]: (a, b, c, d): A = L_a R_b, B = L_c R_d
    double2* part;       // [tc][nitems][3]: (weight Tr-block of A B, Tr-block A, Tr-block B)
    int n, nmom, nitems;
};

// MFMAs of one staged K block for one wave's 32 x 32 quadrant, complex products in
// Gauss's three-multiplication form: with t1 = sum ar br, t2 = sum ai bi and
// t3 = sum (ar + ai)(br + bi), the product is (t1 - t2) + i (t3 - t1 - t2).
// AKM: the row operand comes from a K-major panel (R_d's columns, for B^T) and the
// column operand from a row-major one (L_c's rows); otherwise the reverse.
template <bool AKM, bool GUARD>
__device__ __forceinline__ void pair_stage(const float2* Xa, const float2* Xb, int wm, int wn, int lr, int lk,
                                           bool m1, bool n1, floatx4 (&t1)[2][2], floatx4 (&t2)[2][2],
                                           floatx4 (&t3)[2][2]) {
#pragma unroll
    for (int ks = 0; ks < PKC / 4; ++ks) {
        float2 av[2], bv[2];
        float as[2], bs[2];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            av[mb] = AKM ? Xa[(4 * ks + lk) * PBP + wm + 16 * mb + lr] : Xa[(wm + 16 * mb + lr) * PAP + 4 * ks + lk];
            as[mb] = av[mb].x + av[mb].y;
        }
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            bv[nb] = AKM ? Xb[(wn + 16 * nb + lr) * PAP + 4 * ks + lk] : Xb[(4 * ks + lk) * PBP + wn + 16 * nb + lr];
            bs[nb] = bv[nb].x + bv[nb].y;
        }
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                if (GUARD && ((mb == 1 && !m1) || (nb == 1 && !n1))) continue;
                t1[mb][nb] = mfma16x4(av[mb].x, bv[nb].x, t1[mb][nb]);
                t2[mb][nb] = mfma16x4(av[mb].y, bv[nb].y, t2[mb][nb]);
                t3[mb][nb] = mfma16x4(as[mb], bs[nb], t3[mb][nb]);
            }
    }
}

// One work item = tile (I, J) of A = L_a R_b (waves 0-3, one 32 x 32 quadrant each) and
// tile (I, J) of B^T = (L_c R_d)^T (waves 4-7, the same quadrants), 512 threads. After
// the K loop waves 4-7 hand their tile to waves 0-3 through LDS, which form the FP64
// sums of A .* B^T over the tile and, on a diagonal tile, of both diagonals.
__global__ __launch_bounds__(512, 2) void tm_pair_kernel(PairArgs g) {
    __shared__ float2 smem[kPairSmem];
    __shared__ double red[4][6];
    float2* Al = smem;                       // [2][64][PAP]  L_a rows of I
    float2* Ac = Al + 2 * kPanelRM;          // [2][64][PAP]  L_c rows of J
    float2* Bl = Ac + 2 * kPanelRM;          // [2][PKC][PBP] R_b columns of J
    float2* Bd = Bl + 2 * kPanelKM;          // [2][PKC][PBP] R_d columns of I
    const int bid = (int)xcd_remap(blockIdx.x, gridDim.x);
    const int tl = bid / g.nitems, it = bid - tl * g.nitems;
    const int4 item = g.items[it];
    const int4 pr = g.pairs[item.x];
    const int n = g.n;
    const size_t nn = (size_t)n * n;
    const float2* La = g.L + ((size_t)tl * g.nmom + pr.x) * nn;
    const float2* Rb = g.R + ((size_t)tl * g.nmom + pr.y) * nn;
    const float2* Lc = g.L + ((size_t)tl * g.nmom + pr.z) * nn;
    const float2* Rd = g.R + ((size_t)tl * g.nmom + pr.w) * nn;
    const int i0 = item.y * 64, j0 = item.z * 64;
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const bool second = w >= 4;              // wave-uniform: this wave computes B^T
    // staging: row-major panels 64 x PKC (rows rr + kRS q, column rk), K-major panels PKC x 64
    // (rows kk + 16 q, columns kc + 32 q'); rows and columns past n are clamped and never
    // counted
    const int rk = tid % PKC, rr = tid / PKC, kc = tid & 31, kk = tid >> 5;
    int ra_i[kRQ], ra_j[kRQ], kb_j[2], kb_i[2];
#pragma unroll
    for (int q = 0; q < kRQ; ++q) {
        ra_i[q] = min(i0 + rr + kRS * q, n - 1);
        ra_j[q] = min(j0 + rr + kRS * q, n - 1);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        kb_j[q] = min(j0 + kc + 32 * q, n - 1);
        kb_i[q] = min(i0 + kc + 32 * q, n - 1);
    }
    const int nchunks = (n + PKC - 1) / PKC;
    float2 la[kRQ], lc[kRQ], rb[kKQ][2], rd[kKQ][2];
    float am = 0.f;
    floatx4 t1[2][2], t2[2][2], t3[2][2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            t1[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
            t2[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
            t3[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
    const int wq = w & 3, wm = (wq & 1) * 32, wn = (wq >> 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;
    const bool any = i0 + wm < n && j0 + wn < n;
    const bool m1 = i0 + wm + 16 < n, n1 = j0 + wn + 16 < n;
    const bool full = any && m1 && n1;
    int buf = 0;
    for (int c = 0; c <= nchunks; ++c) {
        if (c < nchunks) {  // stage c into registers; K past the end contributes zero
            const int qa = c * PKC + rk;
            am = qa < n ? 1.f : 0.f;
            const int qac = min(qa, n - 1);
#pragma unroll
            for (int q = 0; q < kRQ; ++q) {  // offsets below n^2 <= 2^22: 32-bit
                la[q] = gld(La + (unsigned)(ra_i[q] * n + qac));
                lc[q] = gld(Lc + (unsigned)(ra_j[q] * n + qac));
            }
#pragma unroll
            for (int q1 = 0; q1 < kKQ; ++q1) {
                const int qb = min(c * PKC + kk + 16 * q1, n - 1);
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    rb[q1][q] = gld(Rb + (unsigned)(qb * n + kb_j[q]));
                    rd[q1][q] = gld(Rd + (unsigned)(qb * n + kb_i[q]));
                }
            }
        }
        if (c > 0) {  // MFMAs of stage c - 1
            const int o_rm = buf * kPanelRM, o_km = buf * kPanelKM;
            if (!second) {
                if (full)
                    pair_stage<false, false>(Al + o_rm, Bl + o_km, wm, wn, lr, lk, true, true, t1, t2, t3);
                else if (any)
                    pair_stage<false, true>(Al + o_rm, Bl + o_km, wm, wn, lr, lk, m1, n1, t1, t2, t3);
            } else {
                if (full)
                    pair_stage<true, false>(Bd + o_km, Ac + o_rm, wm, wn, lr, lk, true, true, t1, t2, t3);
                else if (any)
                    pair_stage<true, true>(Bd + o_km, Ac + o_rm, wm, wn, lr, lk, m1, n1, t1, t2, t3);
            }
            buf ^= 1;
        }
        if (c < nchunks) {
            const int o_rm = buf * kPanelRM, o_km = buf * kPanelKM;
#pragma unroll
            for (int q = 0; q < kRQ; ++q) {
                Al[o_rm + (rr + kRS * q) * PAP + rk] = make_float2(la[q].x * am, la[q].y * am);
                Ac[o_rm + (rr + kRS * q) * PAP + rk] = make_float2(lc[q].x * am, lc[q].y * am);
            }
#pragma unroll
            for (int q1 = 0; q1 < kKQ; ++q1)
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    Bl[o_km + (kk + 16 * q1) * PBP + kc + 32 * q] = rb[q1][q];
                    Bd[o_km + (kk + 16 * q1) * PBP + kc + 32 * q] = rd[q1][q];
                }
        }
        __syncthreads();
    }
    // hand B^T to waves 0-3 (the staging buffers are free after the loop's last barrier)
    float2* xch = smem;  // [64][PXP]
    if (second) {
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const float r1 = t1[mb][nb][v], r2 = t2[mb][nb][v];
                    xch[(wm + 16 * mb + 4 * lk + v) * PXP + wn + 16 * nb + lr] =
                        make_float2(r1 - r2, t3[mb][nb][v] - r1 - r2);
                }
    }
    __syncthreads();
    double xr = 0.0, xi = 0.0, tar = 0.0, tai = 0.0, tbr = 0.0, tbi = 0.0;
    if (!second) {
        const bool diag = item.y == item.z;
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int lrow = wm + 16 * mb + 4 * lk + v, lcol = wn + 16 * nb + lr;
                    if (i0 + lrow < n && j0 + lcol < n) {
                        const float r1 = t1[mb][nb][v], r2 = t2[mb][nb][v];
                        const double a_r = r1 - r2, a_i = t3[mb][nb][v] - r1 - r2;
                        const float2 bt = xch[lrow * PXP + lcol];
                        const double b_r = bt.x, b_i = bt.y;
                        xr += a_r * b_r - a_i * b_i;
                        xi += a_r * b_i + a_i * b_r;
                        if (diag && lrow == lcol) {
                            tar += a_r;
                            tai += a_i;
                            tbr += b_r;
                            tbi += b_i;
                        }
                    }
                }
        xr = wave_sum(xr);
        xi = wave_sum(xi);
        tar = wave_sum(tar);
        tai = wave_sum(tai);
        tbr = wave_sum(tbr);
        tbi = wave_sum(tbi);
        if (lane == 0) {
            red[w][0] = xr;
            red[w][1] = xi;
            red[w][2] = tar;
            red[w][3] = tai;
            red[w][4] = tbr;
            red[w][5] = tbi;
        }
    }
    __syncthreads();
    if (tid == 0) {
        double s[6];
        for (int k = 0; k < 6; ++k) s[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
        const double wt = (double)item.w;
        double2* out = g.part + ((size_t)tl * g.nitems + it) * 3;
        out[0] = make_double2(wt * s[0], wt * s[1]);
        out[1] = make_double2(s[2], s[3]);
        out[2] = make_double2(s[4], s[5]);
    }
}

// ------------------------------------------------------------------ sum

struct SumArgs {
    const double2* part;     // [tc][nitems][3]
    const int* pair_begin;   // [npair + 1]: items of pair q are [pair_begin[q], pair_begin[q + 1])
    const int* pair_mult;    // [npair]: 2 when the pair and its partner are distinct, else 1
    double2* corr;           // [T][3]: (C, direct, crossed)
    int nitems, npair, t_off;
};

// One workgroup per timeslice; thread q handles pairs q, q + 256, ... in order, then a
// fixed-order tree over the threads (deterministic).
__global__ __launch_bounds__(256) void tm_sum_kernel(SumArgs a) {
    __shared__ double sd[256][4];
    const int tl = blockIdx.x;
    const double2* part = a.part + (size_t)tl * a.nitems * 3;
    double dr = 0.0, di = 0.0, xr = 0.0, xi = 0.0;
    for (int q = threadIdx.x; q < a.npair; q += 256) {
        double cr = 0.0, ci = 0.0, ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
        for (int it = a.pair_begin[q]; it < a.pair_begin[q + 1]; ++it) {
            const double2 x = part[(size_t)it * 3], ta = part[(size_t)it * 3 + 1], tb = part[(size_t)it * 3 + 2];
            cr += x.x;
            ci += x.y;
            ar += ta.x;
            ai += ta.y;
            br += tb.x;
            bi += tb.y;
        }
        const double m = (double)a.pair_mult[q];
        dr += m * (ar * br - ai * bi);
        di += m * (ar * bi + ai * br);
        xr += m * cr;
        xi += m * ci;
    }
    sd[threadIdx.x][0] = dr;
    sd[threadIdx.x][1] = di;
    sd[threadIdx.x][2] = xr;
    sd[threadIdx.x][3] = xi;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int k = 0; k < 4; ++k) sd[threadIdx.x][k] += sd[threadIdx.x + s][k];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // C = 2 sum_{k,l} (Tr P_kl Tr P_kbar,lbar - Tr[P_kl P_kbar,lbar])
        const double Dr = 2.0 * sd[0][0], Di = 2.0 * sd[0][1], Xr = 2.0 * sd[0][2], Xi = 2.0 * sd[0][3];
        double2* out = a.corr + (size_t)(a.t_off + tl) * 3;
        out[0] = make_double2(Dr - Xr, Di - Xi);
        out[1] = make_double2(Dr, Di);
        out[2] = make_double2(Xr, Xi);
    }
}

// ================================================================ host side

using namespace nuc::rt;
using meson::cd;

struct Plan {
    std::vector<int4> items, pairs;
    std::vector<int> pair_begin, pair_mult;
};

// Unique pairs {(k, l), (kbar, lbar)} and their tiles.
Plan plan_pairs(int nmom, const std::vector<int>& kbar, int ntile) {
    Plan P;
    for (int k = 0; k < nmom; ++k)
        for (int l = 0; l < nmom; ++l) {
            const int kb = kbar[k], lb = kbar[l];
            if (std::make_pair(k, l) > std::make_pair(kb, lb)) continue;  // the partner carries it
            const bool self = k == kb && l == lb;
            const int q = (int)P.pairs.size();
            P.pairs.push_back(make_int4(k, l, kb, lb));
            P.pair_begin.push_back((int)P.items.size());
            P.pair_mult.push_back(self ? 1 : 2);
            // groups of kGroupI tile rows, columns outer within a group: the workgroups in
            // flight at once share their row panels and a window of column panels in L2
            for (int I0 = 0; I0 < ntile; I0 += kGroupI)
                for (int J = 0; J < ntile; ++J)
                    for (int I = I0; I < std::min(ntile, I0 + kGroupI); ++I) {
                        if (self && J < I) continue;
                        P.items.push_back(make_int4(q, I, J, self && I != J ? 2 : 1));
                    }
        }
    P.pair_begin.push_back((int)P.items.size());
    return P;
}

nuc_status tm_run(nuc_ctx ctx, const nuc_geom* geom, const void* phi, const double* evals, int nprof,
                  const nuc_profile* prof, const double* weights, int nmom, const int32_t* mom, const void* peramb,
                  void* corr, hipStream_t s) {
    nuc_status st;
    if ((st = meson::check_meson_geom(ctx, geom)) != NUC_OK) return st;
    const nuc_geom g = *geom;
    if (nmom < 1 || nmom > kMaxMom) return fail(ctx, NUC_ERR_INVALID, "nmom=%d out of range [1,%d]", nmom, kMaxMom);
    if (!phi || !peramb || !corr) return fail(ctx, NUC_ERR_INVALID, "phi, peramb or corr is NULL");
    if (!weights) return fail(ctx, NUC_ERR_INVALID, "weights is NULL");
    if ((st = check_moms(ctx, &g, nmom, mom)) != NUC_OK) return st;
    if ((st = check_profiles(ctx, &g, evals, nprof, prof)) != NUC_OK) return st;
    std::vector<int> kbar(nmom, -1);
    for (int k = 0; k < nmom; ++k)
        for (int q = 0; q < nmom; ++q) {
            const bool same = mom[3 * k] == mom[3 * q] && mom[3 * k + 1] == mom[3 * q + 1] &&
                              mom[3 * k + 2] == mom[3 * q + 2];
            if (same && q != k)
                return fail(ctx, NUC_ERR_INVALID, "momenta %d and %d are equal", k, q);
            if (mom[3 * k] == -mom[3 * q] && mom[3 * k + 1] == -mom[3 * q + 1] && mom[3 * k + 2] == -mom[3 * q + 2])
                kbar[k] = q;
        }
    for (int k = 0; k < nmom; ++k)
        if (kbar[k] < 0)
            return fail(ctx, NUC_ERR_INVALID, "momentum %d (%d,%d,%d) has no partner of opposite sign", k,
                        mom[3 * k], mom[3 * k + 1], mom[3 * k + 2]);
    std::vector<float2> wf((size_t)3 * nprof);
    for (int A = 0; A < 3 * nprof; ++A) {
        if (!isfinite(weights[2 * A]) || !isfinite(weights[2 * A + 1]))
            return fail(ctx, NUC_ERR_INVALID, "weight %d is not finite", A);
        wf[A] = make_float2((float)weights[2 * A], (float)weights[2 * A + 1]);
    }
    // spin table
    std::vector<std::vector<meson::Term>> fam;
    meson::Perm g5p;
    double g4d[4];
    if (!meson::operator_terms(fam, g5p, g4d)) return fail(ctx, NUC_ERR_INTERNAL, "spin matrices are not permutations");
    SpinTable tab{};
    for (int f = 0; f < (int)fam.size(); ++f)
        for (const meson::Term& tm : fam[f])
            for (int al = 0; al < 4; ++al) {
                const int be = tm.G.col[al], ab = al * 4 + be;
                if (tab.nterm[ab] >= kMaxTerm) return fail(ctx, NUC_ERR_INTERNAL, "spin block has too many terms");
                const cd v = tm.G.val[al];
                tab.coef[ab][tab.nterm[ab]] = make_float2((float)v.real(), (float)v.imag());
                tab.fd[ab][tab.nterm[ab]] = f * 8 + tm.D;
                ++tab.nterm[ab];
            }
    for (int al = 0; al < 4; ++al) {
        tab.g4[al] = (float)g4d[al];
        tab.col5[al] = g5p.col[al];
        if (std::abs(g5p.val[al].imag()) > 1e-12) return fail(ctx, NUC_ERR_INTERNAL, "gamma_5 is not real");
        tab.v5[al] = (float)g5p.val[al].real();
    }
    // profiles at every t (FP32)
    const int N = g.nvec, T = g.T, n = 4 * N;
    std::vector<double> gall((size_t)nprof * T * N);
    eval_profiles(&g, evals, nprof, prof, gall.data());
    std::vector<float> gf(gall.size());
    for (size_t i = 0; i < gall.size(); ++i) gf[i] = (float)gall[i];
    const int ntile = (n + 63) / 64;
    const Plan P = plan_pairs(nmom, kbar, ntile);
    const int nitems = (int)P.items.size(), npair = (int)P.pairs.size();

    HostBlock hb;
    const size_t o_w = hb.add(wf.data(), wf.size() * sizeof(float2));
    const size_t o_g = hb.add(gf.data(), gf.size() * sizeof(float));
    const size_t o_items = hb.add(P.items.data(), P.items.size() * sizeof(int4));
    const size_t o_pairs = hb.add(P.pairs.data(), P.pairs.size() * sizeof(int4));
    const size_t o_pb = hb.add(P.pair_begin.data(), P.pair_begin.size() * sizeof(int));
    const size_t o_pm = hb.add(P.pair_mult.data(), P.pair_mult.size() * sizeof(int));
    const size_t mat = (size_t)n * n * sizeof(float2);
    const size_t per_t = align_up((size_t)3 * nmom * mat + mat + (size_t)nitems * 3 * sizeof(double2), 256);
    const size_t o_mbar = align_up(hb.bytes.size(), 256);
    const size_t fixed = o_mbar + align_up((size_t)nmom * mat, 256);
    const size_t cap = ctx->budget ? std::min(kTmCap, ctx->budget / 2) : kTmCap;
    // timeslices per round: within the workspace cap and the operator kernel's grid
    // (timeslices x momenta on grid y, at most 65535)
    const int tc = (int)std::max<size_t>(
        1, std::min<size_t>({(size_t)T, (cap > fixed ? cap - fixed : 0) / per_t, (size_t)(65535 / nmom)}));
    const size_t o_M = fixed;
    const size_t o_L = o_M + align_up((size_t)tc * nmom * mat, 256);
    const size_t o_R = o_L + align_up((size_t)tc * nmom * mat, 256);
    const size_t o_back = o_R + align_up((size_t)tc * nmom * mat, 256);
    const size_t o_part = o_back + align_up((size_t)tc * mat, 256);
    const size_t total = o_part + align_up((size_t)tc * nitems * 3 * sizeof(double2), 256);
    if ((size_t)tc * nitems > (size_t)INT32_MAX) return fail(ctx, NUC_ERR_INVALID, "too many pair tiles per launch");

    if ((st = begin_call(ctx, s)) != NUC_OK) return st;
    if ((st = ensure_workspace(ctx, total, s)) != NUC_OK) return st;
    char* base = (char*)ctx->ws;
    if ((st = upload_block(ctx, hb, base, s)) != NUC_OK) return st;
    float2* Mbar = (float2*)(base + o_mbar);
    float2* M = (float2*)(base + o_M);
    float2* Lm = (float2*)(base + o_L);
    float2* Rm = (float2*)(base + o_R);
    float2* back = (float2*)(base + o_back);

    OpArgs oa{};
    oa.phi = (const float2*)phi;
    oa.g = (const float*)(base + o_g);
    oa.w = (const float2*)(base + o_w);
    oa.N = N;
    oa.T = T;
    oa.nmom = nmom;
    oa.nprof = nprof;
    oa.t0 = g.t0;
    oa.tab = tab;
    const unsigned nblk_op = (unsigned)((N * N + 255) / 256);
    oa.out = Mbar;
    HIPCHK(ctx, timed_launch(ctx, NUC_K_TM_OPERATOR, s, [&] {
               hipLaunchKernelGGL(tm_operator_kernel<true>, dim3(nblk_op, nmom), dim3(256), 0, s, oa);
               return hipGetLastError();
           }));
    PairArgs pa{};
    pa.items = (const int4*)(base + o_items);
    pa.pairs = (const int4*)(base + o_pairs);
    pa.part = (double2*)(base + o_part);
    pa.L = Lm;
    pa.R = Rm;
    pa.n = n;
    pa.nmom = nmom;
    pa.nitems = nitems;
    SumArgs sa{};
    sa.part = pa.part;
    sa.pair_begin = (const int*)(base + o_pb);
    sa.pair_mult = (const int*)(base + o_pm);
    sa.corr = (double2*)corr;
    sa.nitems = nitems;
    sa.npair = npair;
    const long long nn = (long long)n * n;
    for (int t_off = 0; t_off < T; t_off += tc) {
        const int nt = std::min(tc, T - t_off);
        oa.t_off = t_off;
        oa.out = M;
        HIPCHK(ctx, timed_launch(ctx, NUC_K_TM_OPERATOR, s, [&] {
                   hipLaunchKernelGGL(tm_operator_kernel<false>, dim3(nblk_op, nt * nmom), dim3(256), 0, s, oa);
                   return hipGetLastError();
               }));
        BackArgs ba{(const float2*)peramb, back, N, t_off, tab};
        HIPCHK(ctx, timed_launch(ctx, NUC_K_TM_GEMM, s, [&] {
                   hipLaunchKernelGGL(tm_back_kernel, dim3((n + 31) / 32, (n + 31) / 32, nt), dim3(256), 0, s, ba);
                   return hipGetLastError();
               }));
        const float2* tau_t = (const float2*)peramb + (size_t)t_off * nn;
        HIPCHK(ctx, timed_launch(ctx, NUC_K_TM_GEMM, s, [&] {  // L[tl][k] = M[tl][k] tau(t)
                   return spin::gemm(M, tau_t, Lm, n, n, n, n, n, n, nn, nn, nn, nt * nmom, s, 1, 1 << 30, nmom,
                                     1 << 30);
               }));
        HIPCHK(ctx, timed_launch(ctx, NUC_K_TM_GEMM, s, [&] {  // R[tl][l] = Mbar[l] tau~(t)
                   return spin::gemm(Mbar, back, Rm, n, n, n, n, n, n, nn, nn, nn, nt * nmom, s, 1, nmom, nmom,
                                     1 << 30);
               }));
        HIPCHK(ctx, timed_launch(ctx, NUC_K_TM_PAIR, s, [&] {
                   hipLaunchKernelGGL(tm_pair_kernel, dim3((unsigned)(nt * nitems)), dim3(512), 0, s, pa);
                   return hipGetLastError();
               }));
        sa.t_off = t_off;
        HIPCHK(ctx, timed_launch(ctx, NUC_K_TM_SUM, s, [&] {
                   hipLaunchKernelGGL(tm_sum_kernel, dim3(nt), dim3(256), 0, s, sa);
                   return hipGetLastError();
               }));
    }
    return end_call(ctx, s);
}

}  // namespace twomeson
}  // namespace nuc

extern "C" nuc_status nuc_twomeson_correlator(nuc_ctx ctx, const nuc_geom* geom, const void* phi,
                                              const double* evals, int nprof, const nuc_profile* prof,
                                              const double* weights, int nmom, const int32_t* mom,
                                              const void* peramb, void* corr, void* stream) {
    if (!ctx) return nuc::rt::fail(nullptr, NUC_ERR_INVALID, "ctx is NULL");
    std::lock_guard<std::mutex> lock(ctx->mu);
    nuc::rt::DeviceGuard guard;
    return nuc::twomeson::tm_run(ctx, geom, phi, evals, nprof, prof, weights, nmom, mom, peramb, corr,
                                 (hipStream_t)stream);
}

extern "C" nuc_status nuc_twomeson_weights(const void* vec, int m, const void* basis, int n, void* w_out) {
    if (!vec || !w_out) return nuc::rt::fail(nullptr, NUC_ERR_INVALID, "vec or w_out is NULL");
    if (m < 1 || m > 64) return nuc::rt::fail(nullptr, NUC_ERR_INVALID, "m=%d out of range [1,64]", m);
    if (basis && (n < m || n > 64))
        return nuc::rt::fail(nullptr, NUC_ERR_INVALID, "n=%d out of range [m=%d,64]", n, m);
    typedef std::complex<double> cd;
    const cd* v = static_cast<const cd*>(vec);
    cd* w = static_cast<cd*>(w_out);
    if (!basis) {
        for (int a = 0; a < m; ++a) w[a] = std::conj(v[a]);
        return NUC_OK;
    }
    const cd* U = static_cast<const cd*>(basis);  // [n][m]
    for (int r = 0; r < n; ++r) {
        cd acc = 0.0;
        for (int a = 0; a < m; ++a) acc += U[(size_t)r * m + a] * v[a];
        w[r] = std::conj(acc);
    }
    return NUC_OK;
}

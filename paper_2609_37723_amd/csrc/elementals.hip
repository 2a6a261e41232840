// Baryon elementals on CDNA4 MFMA (paper Section 2.1: the nucleon elementals
// Phi[p,t]_ijk that the distillation profiles then reweight).
//
//   Phi[p,t]_ijk = sum_{x,a} A_p[i,(x,a)] W_jk^a(x),
//   A_p[i,(x,a)] = exp(-i p.x) v_i^a(x)       (phase-weighted eigenvectors)
//   W_jk^a(x)    = eps_abc v_j^b(x) v_k^c(x)   (colour cross products, j < k)
//
// is a complex GEMM with rows (p,i), columns the pairs j<k and the reduction
// over (site, colour). Neither operand is stored: each workgroup stages the
// eigenvectors of a block of sites in LDS and every wave builds its MFMA
// operands from there (the cross products in registers, one per lane and
// K-step, shared by all momenta). Only the canonical entries i<j<k are kept;
// the FP32 MFMA tile sums are folded into FP64 every few site blocks and the
// per-split FP64 partials are combined (in a fixed order) by the expand kernel,
// which also writes the five signed copies and the zeros of the dense output.
#include "nuc_internal.h"

namespace nuc {
namespace {

constexpr int CS = 16;              // sites per LDS block -> 48 (site, colour) values
constexpr int KSTEPS = CS * 3 / 4;  // 16x16x4 MFMA K-steps per site block
constexpr int MAXP = 4;             // momenta (row tiles) sharing one cross-product operand
constexpr int FLUSH = 2;            // site blocks summed in FP32 before the FP64 fold

__device__ __forceinline__ long long choose3(long long k) { return k * (k - 1) * (k - 2) / 6; }
__device__ __forceinline__ long long choose2(long long j) { return j * (j - 1) / 2; }

__global__ __launch_bounds__(256) void elem_kernel(ElemLaunch a, int sites_per_split, int npgroup) {
    extern __shared__ float2 smem[];
    float2* sv = smem;                  // [N][CS*3]
    float2* sph = smem + a.N * CS * 3;  // [MAXP][CS]

    unsigned bid = xcd_remap(blockIdx.x, gridDim.x);
    const int w = bid % a.nwork;
    bid /= a.nwork;
    const int pg = bid % npgroup;
    bid /= npgroup;
    const int split = bid % a.nsplit;
    bid /= a.nsplit;
    const int tl = bid;
    const int t = a.t_off + tl;

    const int2 wk = a.work[w];
    const int itile = wk.x, pblock = wk.y;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 15, g = lane >> 4;

    const int q = pblock * 64 + wv * 16 + col;
    const bool qok = q < a.npairs;
    const int2 pr = qok ? a.pairs[q] : make_int2(0, 0);
    const int i = itile * 16 + col;
    const bool iok = i < a.N;
    const int q0 = pblock * 64 + wv * 16;
    bool active = q0 < a.npairs;
    if (active) {
        const int qlast = min(q0 + 15, a.npairs - 1);
        active = itile * 16 < a.pairs[qlast].x;
    }
    const int p0 = pg * MAXP;
    const int np = min(MAXP, a.nmom - p0);

    floatx4 cr[MAXP], ci[MAXP];
    double dr[MAXP][4], di[MAXP][4];
#pragma unroll
    for (int r = 0; r < MAXP; ++r) {
        cr[r] = floatx4{0.f, 0.f, 0.f, 0.f};
        ci[r] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int v = 0; v < 4; ++v) dr[r][v] = di[r][v] = 0.0;
    }

    const int s_begin = split * sites_per_split;
    const int s_end = min(a.V3, s_begin + sites_per_split);
    const float2* vt = a.evecs + (size_t)t * a.N * a.V3 * 3;
    const int row3 = CS * 3;
    int nblk = 0;
    for (int c0 = s_begin; c0 < s_end; c0 += CS) {
        const int ns = min(CS, s_end - c0);
        __syncthreads();
        for (int idx = threadIdx.x; idx < a.N * row3; idx += 256) {
            const int n = idx / row3, e = idx - n * row3;
            float2 v = make_float2(0.f, 0.f);
            if (e < ns * 3) v = vt[((size_t)n * a.V3 + c0) * 3 + e];
            sv[idx] = v;
        }
        if (threadIdx.x < MAXP * CS) {
            const int r = threadIdx.x / CS, s = threadIdx.x % CS;
            float2 ph = make_float2(0.f, 0.f);
            if (r < np && s < ns) {
                const int x = c0 + s;
                const int x0 = x % a.L, x1 = (x / a.L) % a.L, x2 = x / (a.L * a.L);
                const int* n = a.mom + 3 * (p0 + r);
                long m = (long)n[0] * x0 + (long)n[1] * x1 + (long)n[2] * x2;
                m %= a.L;
                if (m < 0) m += a.L;
                double sn, cs;
                sincospi(2.0 * (double)m / (double)a.L, &sn, &cs);
                ph = make_float2((float)cs, (float)(-sn));
            }
            sph[threadIdx.x] = ph;
        }
        __syncthreads();
        if (active) {
#pragma unroll 4
            for (int ks = 0; ks < KSTEPS; ++ks) {
                const int kk = 4 * ks + g;
                const int s = kk / 3, ca = kk - 3 * s;
                const int cb = ca == 2 ? 0 : ca + 1;   // (a+1) mod 3
                const int cc = ca == 0 ? 2 : ca - 1;   // (a+2) mod 3
                const float2* svs = sv + s * 3;
                float2 wjk = make_float2(0.f, 0.f);
                if (qok) {
                    const float2 jb = svs[pr.x * row3 + cb], kc = svs[pr.y * row3 + cc];
                    const float2 jc = svs[pr.x * row3 + cc], kb = svs[pr.y * row3 + cb];
                    const float2 t1 = cmul(jb, kc), t2 = cmul(jc, kb);
                    wjk = make_float2(t1.x - t2.x, t1.y - t2.y);
                }
                const float2 vi = iok ? svs[i * row3 + ca] : make_float2(0.f, 0.f);
#pragma unroll
                for (int r = 0; r < MAXP; ++r) {
                    if (r < np) {
                        const float2 av = cmul(vi, sph[r * CS + s]);
                        cmfma16x4(av.x, av.y, wjk.x, wjk.y, cr[r], ci[r]);
                    }
                }
            }
            if (++nblk == FLUSH) {
                nblk = 0;
#pragma unroll
                for (int r = 0; r < MAXP; ++r) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        dr[r][v] += (double)cr[r][v];
                        di[r][v] += (double)ci[r][v];
                    }
                    cr[r] = floatx4{0.f, 0.f, 0.f, 0.f};
                    ci[r] = floatx4{0.f, 0.f, 0.f, 0.f};
                }
            }
        }
    }
    if (!active) return;
#pragma unroll
    for (int r = 0; r < MAXP; ++r) {
        if (r >= np) break;
        double2* out = a.part + ((size_t)(split * a.Tc + tl) * a.nmom + p0 + r) * a.C3;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = itile * 16 + 4 * g + v;
            if (qok && row < pr.x) {
                const long long idx = choose3(pr.y) + choose2(pr.x) + row;
                out[idx] = make_double2(dr[r][v] + (double)cr[r][v], di[r][v] + (double)ci[r][v]);
            }
        }
    }
}

__global__ __launch_bounds__(256) void elem_expand_kernel(ElemLaunch a) {
    const size_t n3 = (size_t)a.N * a.N * a.N;
    const size_t total = (size_t)a.Tc * a.nmom * n3;
    const size_t per_split = (size_t)a.Tc * a.nmom * a.C3;
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const size_t tp = idx / n3;
        const int r = (int)(idx - tp * n3);
        int x = r / (a.N * a.N), y = (r / a.N) % a.N, z = r % a.N;
        float2 out = make_float2(0.f, 0.f);
        if (x != y && y != z && x != z) {
            double sign = 1.0;
            int tmp;
            if (x > y) { tmp = x; x = y; y = tmp; sign = -sign; }
            if (y > z) { tmp = y; y = z; z = tmp; sign = -sign; }
            if (x > y) { tmp = x; x = y; y = tmp; sign = -sign; }
            const long long c = choose3(z) + choose2(y) + x;
            double sr = 0.0, si = 0.0;
            for (int s = 0; s < a.nsplit; ++s) {
                const double2 v = a.part[s * per_split + tp * a.C3 + c];
                sr += v.x;
                si += v.y;
            }
            out = make_float2((float)(sign * sr), (float)(sign * si));
        }
        a.phi[(size_t)a.t_off * a.nmom * n3 + idx] = out;
    }
}

}  // namespace

hipError_t launch_elementals(const ElemLaunch& a, hipStream_t s) {
    const int npgroup = (a.nmom + MAXP - 1) / MAXP;
    int sps = (a.V3 + a.nsplit - 1) / a.nsplit;
    sps = ((sps + CS - 1) / CS) * CS;
    const size_t lds = (size_t)(a.N * CS * 3 + MAXP * CS) * sizeof(float2);
    const unsigned grid = (unsigned)a.nwork * npgroup * a.nsplit * a.Tc;
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(elem_kernel, dim3(grid), dim3(256), lds, s, a, sps, npgroup);
    return hipGetLastError();
}

hipError_t launch_elem_expand(const ElemLaunch& a, hipStream_t s) {
    const size_t total = (size_t)a.Tc * a.nmom * a.N * a.N * a.N;
    const unsigned grid = (unsigned)((total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536);
    hipLaunchKernelGGL(elem_expand_kernel, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace nuc

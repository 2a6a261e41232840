// Baryon elementals on CDNA4 MFMA (paper Section 2.1: the nucleon elementals
// Phi[p,t]_ijk that the distillation profiles then reweight).
//
//   Phi[p,t]_ijk = sum_{x,a} A_p[i,(x,a)] W_jk^a(x),
//   A_p[i,(x,a)] = exp(-i p.x) v_i^a(x)       (phase-weighted eigenvectors)
//   W_jk^a(x)    = eps_abc v_j^b(x) v_k^c(x)   (colour cross products, j < k)
//
// is a complex GEMM with rows (p,i), columns the pairs j<k and the reduction
// over (site, colour). Neither operand is stored: each workgroup stages the
// eigenvectors of a block of sites in LDS (prefetching the next block into
// registers while the current one is consumed) and every wave builds its MFMA
// operands from there -- the cross products once per K-step, shared by up to
// eight momenta. The K order is (site group of 4, colour), so every LDS address
// is a per-lane base plus a compile-time offset.
//
// Each block of 16 sites is summed in FP32 MFMA accumulators and folded into
// per-lane FP64 sums; a workgroup stores the canonical entries (i<j<k) of its
// range of sites in FP64, the reduce kernel adds the ranges in FP64 (fixed
// order) and the expand kernel writes the dense, exactly antisymmetric output.
#include "nuc_internal.h"

namespace nuc {
namespace {

constexpr int CS = 16;              // sites per LDS block
constexpr int ROW3 = CS * 3;        // (site, colour) values per vector and block
constexpr int MAXP = 4;             // most momenta (row tiles) sharing one cross-product operand
constexpr int MAXPF = (kMaxNvec * ROW3 + 255) / 256;  // prefetch registers per thread

__device__ __forceinline__ long long choose3(long long k) { return k * (k - 1) * (k - 2) / 6; }
__device__ __forceinline__ long long choose2(long long j) { return j * (j - 1) / 2; }

template <int NPF, int MP>
__global__ __launch_bounds__(256) void elem_kernel(BatchRef bt) {
    extern __shared__ float2 smem[];
    const int item = xcd_remap(blockIdx.x, gridDim.x);
    const int inst = find_inst(bt.offs, bt.ninst, item);
    const ElemLaunch& a = reinterpret_cast<const ElemLaunch*>(bt.descs)[inst];
    const int sites_per_split = a.sites_per_split, npgroup = a.npgroup;
    float2* sv = smem;                  // [N][ROW3]
    float2* sph = sv + a.N * ROW3;      // [MP][CS]
    float2* tab = sph + MP * CS;        // [L]  exp(-2 pi i m / L)

    unsigned bid = item - bt.offs[inst];
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
    const int q0 = pblock * 64 + wv * 16;
    bool active = q0 < a.npairs;
    if (active) {
        const int qlast = min(q0 + 15, a.npairs - 1);
        active = itile * 16 < a.pairs[qlast].x;
    }
    const int p0 = pg * MP;
    const int np = min(MP, a.nmom - p0);

    for (int m = threadIdx.x; m < a.L; m += 256) {
        double sn, cs;
        sincospi(2.0 * (double)m / (double)a.L, &sn, &cs);
        tab[m] = make_float2((float)cs, (float)(-sn));
    }

    floatx4 cr[MP], ci[MP];
    double dr[MP][4], di[MP][4];
#pragma unroll
    for (int r = 0; r < MP; ++r) {
        cr[r] = floatx4{0.f, 0.f, 0.f, 0.f};
        ci[r] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int v = 0; v < 4; ++v) dr[r][v] = di[r][v] = 0.0;
    }

    const int s_begin = split * sites_per_split;
    const int s_end = min(a.V3, s_begin + sites_per_split);
    const float2* vt = a.evecs + (size_t)t * a.ev_tstride;
    const int nval = a.N * ROW3;

    // prefetch of one site block into registers: element idx = threadIdx.x + 256*r
    float2 pf[NPF];
    int pf_off[NPF];
#pragma unroll
    for (int r = 0; r < NPF; ++r) {
        const int idx = threadIdx.x + 256 * r;
        const int n = idx / ROW3, e = idx - n * ROW3;
        pf_off[r] = (idx < nval) ? n * a.V3 * 3 + e : -1;   // + 3*c0, valid while e < 3*ns
    }
#define NUC_PREFETCH(c0_)                                                   \
    {                                                                       \
        const int ns3_ = min(CS, s_end - (c0_)) * 3;                        \
        _Pragma("unroll") for (int r = 0; r < NPF; ++r) {                   \
            const int e_ = (threadIdx.x + 256 * r) % ROW3;                  \
            pf[r] = make_float2(0.f, 0.f);                                  \
            if (pf_off[r] >= 0 && e_ < ns3_) pf[r] = vt[pf_off[r] + 3 * (c0_)]; \
        }                                                                   \
    }
    if (s_begin < s_end) NUC_PREFETCH(s_begin);

    // per-lane LDS bases: site 4*sg + g, colour c  ->  offset 12*sg + 3*g + c
    const float2* bj = sv + pr.x * ROW3 + 3 * g;
    const float2* bk = sv + pr.y * ROW3 + 3 * g;
    const float2* bi = sv + (i < a.N ? i : 0) * ROW3 + 3 * g;
    const bool iok = i < a.N;

    for (int c0 = s_begin; c0 < s_end; c0 += CS) {
        const int ns = min(CS, s_end - c0);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NPF; ++r) {
            const int idx = threadIdx.x + 256 * r;
            if (idx < nval) sv[idx] = pf[r];
        }
        if (threadIdx.x < MP * CS) {
            const int r = threadIdx.x / CS, s = threadIdx.x % CS;
            float2 ph = make_float2(0.f, 0.f);
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
        if (!active) continue;
#pragma unroll 1
        for (int sg = 0; sg < CS / 4; ++sg) {
            float2 ph[MP];
#pragma unroll
            for (int r = 0; r < MP; ++r) ph[r] = sph[r * CS + 4 * sg + g];
#pragma unroll
            for (int ca = 0; ca < 3; ++ca) {
                const int cb = (ca + 1) % 3, cc = (ca + 2) % 3;
                const int o = 12 * sg;
                float2 wjk = make_float2(0.f, 0.f);
                {
                    const float2 jb = bj[o + cb], kc = bk[o + cc], jc = bj[o + cc], kb = bk[o + cb];
                    const float2 t1 = cmul(jb, kc), t2 = cmul(jc, kb);
                    if (qok) wjk = make_float2(t1.x - t2.x, t1.y - t2.y);
                }
                const float nwi = -wjk.y;
                float2 vi = bi[o + ca];
                if (!iok) vi = make_float2(0.f, 0.f);
#pragma unroll
                for (int r = 0; r < MP; ++r) {
                    const float2 av = cmul(vi, ph[r]);
                    cr[r] = mfma16x4(av.x, wjk.x, cr[r]);
                    cr[r] = mfma16x4(av.y, nwi, cr[r]);
                    ci[r] = mfma16x4(av.x, wjk.y, ci[r]);
                    ci[r] = mfma16x4(av.y, wjk.x, ci[r]);
                }
            }
        }
        // fold this block of sites into the FP64 sums
#pragma unroll
        for (int r = 0; r < MP; ++r) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                dr[r][v] += (double)cr[r][v];
                di[r][v] += (double)ci[r][v];
            }
            cr[r] = floatx4{0.f, 0.f, 0.f, 0.f};
            ci[r] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
    }
#undef NUC_PREFETCH
    if (!active) return;
#pragma unroll
    for (int r = 0; r < MP; ++r) {
        if (r >= np) break;
        double2* out = a.part + ((size_t)(split * a.Tc + tl) * a.nmom + p0 + r) * a.C3;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = itile * 16 + 4 * g + v;
            if (qok && row < pr.x) {
                const long long idx = choose3(pr.y) + choose2(pr.x) + row;
                out[idx] = make_double2(dr[r][v], di[r][v]);
            }
        }
    }
}

// FP64 sum of the per-split partials of every canonical entry (fixed split order).
// One item = 256 canonical entries.
__global__ __launch_bounds__(256) void elem_reduce_kernel(BatchRef bt) {
    const int item = blockIdx.x;
    const int inst = find_inst(bt.offs, bt.ninst, item);
    const ElemLaunch& a = reinterpret_cast<const ElemLaunch*>(bt.descs)[inst];
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
    const ElemLaunch& a = reinterpret_cast<const ElemLaunch*>(bt.descs)[inst];
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

template <int NPF, int MP>
hipError_t launch_elem_t(const BatchRef& b, size_t lds, hipStream_t s) {
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)elem_kernel<NPF, MP>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((elem_kernel<NPF, MP>), dim3(b.nitems), dim3(256), lds, s, b);
    return hipGetLastError();
}

// Shape class: prefetch depth (from N) and momenta per wave (from nmom).
int npf_bucket(int N) {
    const int npf = (N * ROW3 + 255) / 256;
    return npf <= 3 ? 3 : npf <= 6 ? 6 : npf <= 12 ? 12 : MAXPF;
}
int mp_of(int nmom) { return nmom <= 1 ? 1 : nmom <= 2 ? 2 : MAXP; }
int mp_sel(const ElemLaunch& a) { return a.mp == 1 || a.mp == 2 || a.mp == MAXP ? a.mp : mp_of(a.nmom); }

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
int elem_class(const ElemLaunch& a) { return npf_bucket(a.N) * 16 + mp_sel(a); }

// LDS of a class is sized for the largest N and L it may hold.
hipError_t launch_elementals(int cls, const BatchRef& b, hipStream_t s) {
    if (b.nitems == 0) return hipSuccess;
    const int npf = cls / 16, mp = cls % 16;
    const size_t lds = (size_t)(kMaxNvec * ROW3 + MAXP * CS + 256) * sizeof(float2);
#define NUC_ELEM_CASE(NPF_)                                            \
    if (npf == NPF_) {                                                 \
        if (mp == 1) return launch_elem_t<NPF_, 1>(b, lds, s);         \
        if (mp == 2) return launch_elem_t<NPF_, 2>(b, lds, s);         \
        return launch_elem_t<NPF_, MAXP>(b, lds, s);                   \
    }
    NUC_ELEM_CASE(3)
    NUC_ELEM_CASE(6)
    NUC_ELEM_CASE(12)
    NUC_ELEM_CASE(MAXPF)
#undef NUC_ELEM_CASE
    return hipErrorInvalidValue;
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

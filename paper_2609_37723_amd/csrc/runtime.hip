// Host runtime of the nucleon-correlator library: the C ABI of include/nucleon.h,
// argument checks, host-side FP64 profile evaluation, the context's HBM
// workspace and the kernel launch sequence.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/nucleon.h"
#include "nuc_internal.h"
#include "runtime_internal.h"

#define NUC_VERSION "nucleon-mi355x 0.1 (gfx950)"

using namespace nuc;



namespace nuc {
namespace rt {

thread_local std::string g_thread_err;

nuc_status fail(nuc_ctx ctx, nuc_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_thread_err = buf;
    if (ctx) ctx->err = buf;
    return s;
}

nuc_status hip_fail(nuc_ctx ctx, hipError_t e, const char* what) {
    return fail(ctx, NUC_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}




hipEvent_t pool_get(nuc_ctx ctx) {
    if (!ctx->ev_pool.empty()) {
        hipEvent_t e = ctx->ev_pool.back();
        ctx->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

long long choose3(long long n) { return n * (n - 1) * (n - 2) / 6; }

int pad16(int n) { return (n + 15) / 16 * 16; }

// ------------------------------------------------------------- argument checks

nuc_status check_geom(nuc_ctx ctx, const nuc_geom* g) {
    if (!g) return fail(ctx, NUC_ERR_INVALID, "geom is NULL");
    if (g->L < 1 || g->L > 256) return fail(ctx, NUC_ERR_INVALID, "L=%d out of range [1,256]", g->L);
    if (g->T < 1) return fail(ctx, NUC_ERR_INVALID, "T=%d must be >= 1", g->T);
    if (g->nvec < 3 || g->nvec > kMaxNvec)
        return fail(ctx, NUC_ERR_INVALID, "nvec=%d out of range [3,%d]", g->nvec, kMaxNvec);
    if (g->t0 < 0 || g->t0 >= g->T) return fail(ctx, NUC_ERR_INVALID, "t0=%d outside [0,T)", g->t0);
    return NUC_OK;
}

nuc_status check_moms(nuc_ctx ctx, const nuc_geom* g, int nmom, const int32_t* mom) {
    if (nmom < 1 || nmom > 64) return fail(ctx, NUC_ERR_INVALID, "nmom=%d out of range [1,64]", nmom);
    if (!mom) return fail(ctx, NUC_ERR_INVALID, "mom is NULL");
    for (int p = 0; p < nmom; ++p)
        for (int d = 0; d < 3; ++d)
            if (mom[3 * p + d] <= -g->L || mom[3 * p + d] >= g->L)
                return fail(ctx, NUC_ERR_INVALID, "momentum %d component %d = %d needs |n| < L=%d", p, d,
                            mom[3 * p + d], g->L);
    return NUC_OK;
}

nuc_status check_profiles(nuc_ctx ctx, const nuc_geom* g, const double* evals, int nprof,
                          const nuc_profile* prof) {
    if (nprof < 1 || nprof > kMaxProf)
        return fail(ctx, NUC_ERR_INVALID, "nprof=%d out of range [1,%d]", nprof, kMaxProf);
    if (!prof) return fail(ctx, NUC_ERR_INVALID, "prof is NULL");
    for (int a = 0; a < nprof; ++a) {
        switch (prof[a].kind) {
            case NUC_PROF_GAUSS:
                if (!(prof[a].sigma > 0.0) || !isfinite(prof[a].sigma))
                    return fail(ctx, NUC_ERR_INVALID, "profile %d: sigma=%g must be finite and > 0", a,
                                prof[a].sigma);
                if (!evals) return fail(ctx, NUC_ERR_INVALID, "profile %d is Gaussian but evals is NULL", a);
                break;
            case NUC_PROF_LINEAR:
            case NUC_PROF_ONE:
                break;
            case NUC_PROF_EXPLICIT:
                if (!prof[a].values) return fail(ctx, NUC_ERR_INVALID, "profile %d: values is NULL", a);
                break;
            default:
                return fail(ctx, NUC_ERR_INVALID, "profile %d: unknown kind %d", a, prof[a].kind);
        }
    }
    return NUC_OK;
}

nuc_status check_prec(nuc_ctx ctx, int p) {
    if (p == NUC_FP32 || p == NUC_BF16X3 || p == NUC_FP16X3 || p == NUC_FP64) return NUC_OK;
    return fail(ctx, NUC_ERR_INVALID, "unknown precision %d", p);
}

// The forms other than FP32 have perambulator chains for nvec <= 32 and for nvec a
// multiple of 16 (>= 48) with an even storage nvec.
nuc_status check_prec_shape(nuc_ctx ctx, nuc_precision p, const nuc_geom* g, int ld) {
    if (p != NUC_FP32 && !corr_bf16x3_supported(g->nvec, ld))
        return fail(ctx, NUC_ERR_UNSUPPORTED,
                    "the split and FP64 contraction forms are implemented for nvec <= 32 and for nvec a multiple "
                    "of 16 >= 48 with an even storage nvec (got nvec %d, stored %d)", g->nvec, ld);
    return NUC_OK;
}

// Section 2.1 profile functions, evaluated in FP64 on the host.
void eval_profiles(const nuc_geom* g, const double* evals, int nprof, const nuc_profile* prof,
                   double* out) {
    const int T = g->T, N = g->nvec;
    for (int a = 0; a < nprof; ++a)
        for (int t = 0; t < T; ++t)
            for (int i = 0; i < N; ++i) {
                double v = 1.0;
                const double sig = prof[a].sigma;
                switch (prof[a].kind) {
                    case NUC_PROF_GAUSS: {
                        const double lam = evals[(size_t)t * N + i];
                        v = exp(-(lam * lam) / (2.0 * sig * sig));
                        break;
                    }
                    case NUC_PROF_LINEAR: v = 1.0 - (double)i / (double)N; break;
                    case NUC_PROF_ONE: v = 1.0; break;
                    case NUC_PROF_EXPLICIT: v = prof[a].values[(size_t)t * N + i]; break;
                }
                out[((size_t)a * T + t) * N + i] = v;
            }
}

// ------------------------------------------------------------------ planning
//
// A call (single job or batch) becomes a Program: the constant block (small
// per-job arrays, launch descriptors, item offsets), internal buffers, and a
// list of stages. A stage is one kernel launch over several pieces (job,
// timeslice chunk) of one shape class. Pieces are packed into rounds whose
// scratch fits the workspace cap; rounds run in stream order and share the
// scratch region. Everything after the single upload of the constant block is
// asynchronous, so a Program can also be captured into a HIP graph.



void plan_elementals(Job& J, size_t cap) {
    const int N = J.g.nvec;
    J.pairs.clear();
    J.work.clear();
    const bool blk = elem_block_pairs(N);
    auto range = [&](int2 p) { return elem_row_range(N, p); };
    for (int j = 0; j < N; ++j)
        for (int k = j + 1; k < N; ++k)
            if (elem_pair_in_set(N, j, k)) J.pairs.push_back(make_int2(j, k));
    // by row range, so that the 16 pairs of a wave mostly share one
    if (blk)
        std::stable_sort(J.pairs.begin(), J.pairs.end(), [&](int2 a, int2 b) {
            const int2 ra = range(a), rb = range(b);
            return ra.x != rb.x ? ra.x < rb.x : ra.y < rb.y;
        });
    const int npairs = (int)J.pairs.size();
    J.C3 = (int)choose3(N);
    // one work item per (chunk of four row tiles, block of 16 pairs per wave); a wave's tiles
    // run from the smallest first tile of its 16 pairs to their largest end (the same
    // rule as in the kernel), and the block takes the chunks of its widest wave
    const int nwv = elem_waves(N), npw = 16 * nwv;
    const int npb = (npairs + npw - 1) / npw;
    for (int pb = npb - 1; pb >= 0; --pb) {
        int nchunk = 0;
        for (int w = 0; w < nwv; ++w) {
            const int q0 = pb * npw + w * 16;
            if (q0 >= npairs) break;
            int b = 1 << 30, e = 0;
            for (int i = 0; i < 16; ++i) {
                const int2 r = range(J.pairs[std::min(q0 + i, npairs - 1)]);
                b = std::min(b, r.x);
                e = std::max(e, r.y);
            }
            nchunk = std::max(nchunk, (e - b + 3) / 4);
        }
        for (int c = 0; c < nchunk; ++c) J.work.push_back(make_int2(c, pb));
    }
    // Each workgroup sums about 1024 sites up to 96 vectors and 512 beyond (256 below 8192
    // sites, where fewer splits would leave CUs idle), with at most kElemCap bytes of FP64
    // partials per timeslice. The split depends on the job's shape only, never on the other
    // jobs of a batch, so a job's result does not depend on its company.
    const int V3 = J.g.L * J.g.L * J.g.L;
    const size_t per_ts = (size_t)J.nmom * J.C3 * sizeof(double2);
    const int per_wg = V3 >= 8192 ? (J.g.nvec <= 96 ? 1024 : 512) : 256;
    int ns = std::max(1, (V3 + per_wg - 1) / per_wg);
    ns = std::min<int>(ns, (int)std::max<size_t>(1, kElemCap / per_ts));
    J.nsplit = ns;
    J.elem_tc = (int)std::max<size_t>(1, std::min<size_t>((size_t)J.g.T, cap / (per_ts * ns)));
}

size_t elem_piece_bytes(const Job& J, int Tc) {
    return align_up((size_t)J.nsplit * Tc * J.nmom * J.C3 * sizeof(double2), 256) +
           align_up((size_t)Tc * J.nmom * J.C3 * sizeof(float2), 256);
}

size_t corr_x_bytes(const Job& J, int Tc) {
    return (size_t)Tc * J.nmom * J.nprof * 2 * 4 * (size_t)J.Np * J.Np * J.Np * sizeof(float2);
}
size_t corr_part_bytes(const Job& J, int Tc) {
    const int ncs = corr_col_splits(J.g.nvec, J.Np, J.ld, J.prec);
    return (size_t)Tc * J.nmom * J.nprof * 2 * J.g.nvec * ncs * J.nprof * sizeof(double2);
}
size_t corr_scale_bytes(const Job& J, int Tc) {  // FP16x3 scales: per unit, then per timeslice
    return J.prec == NUC_FP16X3 ? (size_t)Tc * (J.nmom * J.nprof * 2 * J.g.nvec + 1) * sizeof(float) : 0;
}
size_t corr_tau16_bytes(const Job& J, int Tc) {  // BF16x3 pre-split: tau(t) as bf16 planes
    return corr_pre_split(J.g.nvec, J.Np, J.ld, J.prec) ? (size_t)Tc * 4 * kTauBlocks * J.Np * J.Np * sizeof(float2)
                                                        : 0;
}
size_t corr_piece_bytes(const Job& J, int Tc) {
    return align_up(corr_x_bytes(J, Tc), 256) + align_up(corr_part_bytes(J, Tc), 256) +
           align_up(corr_scale_bytes(J, Tc), 256) + align_up(corr_tau16_bytes(J, Tc), 256);
}

void plan_correlator(Job& J, size_t cap) {
    J.Np = pad16(J.g.nvec);
    const size_t per_t = corr_piece_bytes(J, 1);
    J.corr_tc = (int)std::max<size_t>(1, std::min<size_t>((size_t)J.g.T, cap / per_t));
}

// Greedy packing of pieces into rounds whose scratch fits cap; assigns each
// piece its offset in the scratch region. Returns the largest round.
template <class Bytes>
size_t pack_rounds(std::vector<Piece>& pieces, size_t cap, Bytes bytes, std::vector<std::vector<Piece>>& rounds) {
    size_t cur = 0, peak = 0;
    for (Piece& pc : pieces) {
        const size_t b = bytes(pc);
        if (rounds.empty() || (cur + b > cap && cur > 0)) {
            rounds.emplace_back();
            cur = 0;
        }
        pc.scratch_off = cur;
        rounds.back().push_back(pc);
        cur += align_up(b, 256);
        peak = std::max(peak, cur);
    }
    return peak;
}

nuc_status plan_program(nuc_ctx ctx, Program& P, size_t ws_cap) {
    HostBlock& hb = P.block;
    const size_t nj = std::max<size_t>(1, P.jobs.size());
    const size_t cap_e = std::max<size_t>((size_t)64 << 20, std::min(kElemCap, ws_cap / nj));
    const size_t cap_c = std::max<size_t>((size_t)64 << 20, std::min(kCorrCap, ws_cap / nj));
    std::vector<Piece> ep, cp;
    for (int j = 0; j < (int)P.jobs.size(); ++j) {
        Job& J = P.jobs[j];
        if (J.t_end <= J.t_begin) {
            J.t_begin = 0;
            J.t_end = J.g.T;
        }
        const int tb = J.t_begin, te = J.t_end;
        if (J.do_elem) {
            plan_elementals(J, cap_e);
            J.off_mom = hb.add(J.mom.data(), J.mom.size() * sizeof(int32_t));
            J.off_pairs = hb.add(J.pairs.data(), J.pairs.size() * sizeof(int2));
            J.off_work = hb.add(J.work.data(), J.work.size() * sizeof(int2));
            if (J.src_compute) ep.push_back({j, J.g.t0, 1, 0, true});
            for (int t = tb; t < te; t += J.elem_tc) ep.push_back({j, t, std::min(J.elem_tc, te - t), 0});
        }
        if (J.do_corr) {
            plan_correlator(J, cap_c);
            J.off_gsnk = hb.add(J.gsnk.data(), J.gsnk.size() * sizeof(double));
            J.off_gsrc = hb.add(J.gsrc.data(), J.gsrc.size() * sizeof(double));
            J.gsrc_f.assign(J.gsrc.begin(), J.gsrc.end());
            J.off_gsrc_f = hb.add(J.gsrc_f.data(), J.gsrc_f.size() * sizeof(float));
            for (int t = tb; t < te; t += J.corr_tc) cp.push_back({j, t, std::min(J.corr_tc, te - t), 0});
        }
    }
    std::vector<std::vector<Piece>> er, cr;
    const size_t se = pack_rounds(ep, ws_cap, [&](const Piece& pc) { return elem_piece_bytes(P.jobs[pc.job], pc.Tc); }, er);
    const size_t sc = pack_rounds(cp, ws_cap, [&](const Piece& pc) { return corr_piece_bytes(P.jobs[pc.job], pc.Tc); }, cr);
    for (auto& R : er) {
        std::map<int, std::vector<Piece>> bycls;
        for (auto& pc : R) {
            ElemLaunch e{};
            e.N = P.jobs[pc.job].g.nvec;
            e.nmom = P.jobs[pc.job].nmom;
            e.mp = P.jobs[pc.job].elem_mp;
            e.f64 = P.jobs[pc.job].prec == NUC_FP64;
            bycls[elem_class(e)].push_back(pc);
        }
        for (auto& kv : bycls) P.stages.push_back({NUC_K_ELEMENTALS, kv.first, 0, kv.second});
        P.stages.push_back({NUC_K_ELEM_EXPAND, -1, 0, R});
    }
    for (auto& R : cr) {
        std::map<int, std::vector<Piece>> bynp, bychain;
        std::vector<Piece> scaled, presplit;
        for (auto& pc : R) {
            const Job& J = P.jobs[pc.job];
            bynp[J.Np | (J.prec == NUC_FP64 ? kStep1F64 : 0) |
                 (corr_pre_split(J.g.nvec, J.Np, J.ld, J.prec) ? kStep1Pre : 0)].push_back(pc);
            bychain[corr_chain_class(J.g.nvec, J.Np, J.ld, J.prec) * 4 + J.prec].push_back(pc);
            if (J.prec == NUC_FP16X3) scaled.push_back(pc);
            if (corr_pre_split(J.g.nvec, J.Np, J.ld, J.prec)) presplit.push_back(pc);
        }
        for (auto& kv : bynp) P.stages.push_back({NUC_K_CORR_STEP1, kv.first, 0, kv.second});
        if (!scaled.empty()) P.stages.push_back({NUC_K_CORR_SCALE, -1, NUC_FP16X3, scaled});
        if (!presplit.empty()) P.stages.push_back({NUC_K_CORR_SCALE, -1, NUC_BF16X3, presplit});
        for (auto& kv : bychain) P.stages.push_back({NUC_K_CORR_CHAIN, kv.first / 4, kv.first % 4, kv.second});
        P.stages.push_back({NUC_K_CORR_REDUCE, -1, 0, R});
    }
    for (Stage& st : P.stages) {
        const bool elem = st.kid == NUC_K_ELEMENTALS || st.kid == NUC_K_ELEM_EXPAND;
        st.off_descs = hb.reserve(st.pcs.size() * (elem ? sizeof(ElemLaunch) : sizeof(CorrLaunch)));
        st.off_offs = hb.reserve((st.pcs.size() + 1) * sizeof(int));
        st.off_offs2 = hb.reserve((st.pcs.size() + 1) * sizeof(int));
    }
    size_t off = align_up(hb.bytes.size(), 256);
    for (Job& J : P.jobs) {
        J.phi_internal = J.do_elem && J.do_corr && !J.phi;
        if (J.phi_internal) {
            J.off_phi = off;
            off += align_up((size_t)(J.t_end - J.t_begin) * J.nmom * J.g.nvec * J.g.nvec * J.g.nvec * sizeof(float2),
                            256);
        }
    }
    for (const Job& J : P.jobs)
        if (J.do_corr && !J.src_phi && J.phi_internal && (J.g.t0 < J.t_begin || J.g.t0 >= J.t_end))
            return fail(ctx, NUC_ERR_INTERNAL, "source timeslice outside the planned range and no source block");
    P.scratch_off = off;
    P.scratch_bytes = std::max(se, sc);
    P.total_bytes = off + P.scratch_bytes;
    if (ctx && ctx->budget && P.total_bytes > ctx->budget)
        return fail(ctx, NUC_ERR_NOMEM, "workspace of %zu bytes exceeds the HBM budget of %zu bytes", P.total_bytes,
                    ctx->budget);
    return NUC_OK;
}

ElemLaunch make_elem(const Program& P, const Piece& pc, char* base) {
    const Job& J = P.jobs[pc.job];
    ElemLaunch e{};
    char* scr = base + P.scratch_off + pc.scratch_off;
    e.evecs = (const float2*)J.evecs;
    e.mom = (const int*)(base + J.off_mom);
    e.pairs = (const int2*)(base + J.off_pairs);
    e.work = (const int2*)(base + J.off_work);
    e.part = (double2*)scr;
    e.packed = (float2*)(scr + align_up((size_t)J.nsplit * pc.Tc * J.nmom * J.C3 * sizeof(double2), 256));
    if (pc.src) {
        e.phi = (float2*)J.src_phi;
        e.phi_t = J.g.t0;
    } else {
        e.phi = (float2*)(J.phi_internal ? (void*)(base + J.off_phi) : J.phi);
        e.phi_t = J.phi_internal ? J.t_begin : 0;
    }
    e.T = J.g.T;
    e.N = J.g.nvec;
    e.L = J.g.L;
    e.V3 = J.g.L * J.g.L * J.g.L;
    e.nmom = J.nmom;
    e.npairs = (int)J.pairs.size();
    e.nwork = (int)J.work.size();
    e.nsplit = J.nsplit;
    e.C3 = J.C3;
    e.t_off = pc.t_off;
    e.Tc = pc.Tc;
    e.ev_tstride = (size_t)J.ld * e.V3 * 3;
    e.mp = J.elem_mp;
    e.f64 = J.prec == NUC_FP64;
    elem_finalize(e);
    return e;
}

CorrLaunch make_corr(const Program& P, const Piece& pc, char* base) {
    const Job& J = P.jobs[pc.job];
    CorrLaunch c{};
    char* scr = base + P.scratch_off + pc.scratch_off;
    c.phi = (const float2*)(J.phi_internal ? (void*)(base + J.off_phi) : J.phi);
    c.phi_t = J.phi_internal ? J.t_begin : 0;
    const size_t n3 = (size_t)J.g.nvec * J.g.nvec * J.g.nvec;
    c.phi0 = J.src_phi ? (const float2*)J.src_phi : c.phi + (size_t)(J.g.t0 - c.phi_t) * J.nmom * n3;
    c.tau = (const float2*)J.peramb;
    c.gsnk = (const double*)(base + J.off_gsnk);
    c.gsrc = (const double*)(base + J.off_gsrc);
    c.gsrc_f = (const float*)(base + J.off_gsrc_f);
    c.X = (float2*)scr;
    c.part = (double2*)(scr + align_up(corr_x_bytes(J, pc.Tc), 256));
    if (J.prec == NUC_FP16X3) {
        c.xscale = (float*)(scr + align_up(corr_x_bytes(J, pc.Tc), 256) + align_up(corr_part_bytes(J, pc.Tc), 256));
        c.tscale = c.xscale + (size_t)pc.Tc * J.nmom * J.nprof * 2 * J.g.nvec;
    }
    c.corr = (double2*)J.corr;
    c.T = J.g.T;
    c.N = J.g.nvec;
    c.Np = J.Np;
    c.nmom = J.nmom;
    c.nprof = J.nprof;
    c.t0 = J.g.t0;
    c.t_off = pc.t_off;
    c.Tc = pc.Tc;
    c.Nt = J.ld;
    c.precision = J.prec;
    c.ncs = corr_col_splits(J.g.nvec, J.Np, J.ld, J.prec);
    c.pre = corr_pre_split(J.g.nvec, J.Np, J.ld, J.prec) ? 1 : 0;
    if (c.pre)
        c.tau16 = (uint16_t*)(scr + align_up(corr_x_bytes(J, pc.Tc), 256) + align_up(corr_part_bytes(J, pc.Tc), 256) +
                              align_up(corr_scale_bytes(J, pc.Tc), 256));
    corr_finalize(c, J.s1_target);
    return c;
}

// Fill descriptors and item offsets with device addresses (base = workspace).
void fill_program(Program& P, char* base) {
    char* hb = P.block.bytes.data();
    for (Stage& st : P.stages) {
        std::vector<int> o1(1, 0), o2(1, 0);
        if (st.kid == NUC_K_ELEMENTALS || st.kid == NUC_K_ELEM_EXPAND) {
            ElemLaunch* d = (ElemLaunch*)(hb + st.off_descs);
            for (size_t i = 0; i < st.pcs.size(); ++i) {
                d[i] = make_elem(P, st.pcs[i], base);
                if (st.kid == NUC_K_ELEMENTALS) {
                    o1.push_back(o1.back() + elem_items(d[i]));
                } else {
                    o1.push_back(o1.back() + elem_reduce_items(d[i]));
                    o2.push_back(o2.back() + elem_expand_items(d[i]));
                }
            }
        } else {
            CorrLaunch* d = (CorrLaunch*)(hb + st.off_descs);
            for (size_t i = 0; i < st.pcs.size(); ++i) {
                d[i] = make_corr(P, st.pcs[i], base);
                const int n = st.kid == NUC_K_CORR_STEP1   ? corr_step1_items(d[i])
                              : st.kid == NUC_K_CORR_CHAIN ? corr_chain_items(d[i])
                              : st.kid == NUC_K_CORR_SCALE ? (st.prec == NUC_BF16X3 ? corr_split_tau_items(d[i])
                                                                                    : corr_scale_items(d[i]))
                                                           : corr_reduce_items(d[i]);
                o1.push_back(o1.back() + n);
            }
        }
        memcpy(hb + st.off_offs, o1.data(), o1.size() * sizeof(int));
        st.nitems = o1.back();
        if (o2.size() > 1) {
            memcpy(hb + st.off_offs2, o2.data(), o2.size() * sizeof(int));
            st.nitems2 = o2.back();
        }
    }
}

nuc_status enqueue_program(nuc_ctx ctx, const Program& P, char* base, hipStream_t s) {
    for (const Stage& st : P.stages) {
        BatchRef b{base + st.off_descs, (const int*)(base + st.off_offs), (int)st.pcs.size(), st.nitems};
        switch (st.kid) {
            case NUC_K_ELEMENTALS:
                HIPCHK(ctx, timed_launch(ctx, NUC_K_ELEMENTALS, s, [&] { return launch_elementals(st.cls, b, s); }));
                break;
            case NUC_K_ELEM_EXPAND: {
                HIPCHK(ctx, timed_launch(ctx, NUC_K_ELEM_EXPAND, s, [&] { return launch_elem_reduce(b, s); }));
                BatchRef b2{base + st.off_descs, (const int*)(base + st.off_offs2), (int)st.pcs.size(), st.nitems2};
                HIPCHK(ctx, timed_launch(ctx, NUC_K_ELEM_EXPAND, s, [&] { return launch_elem_expand(b2, s); }));
                break;
            }
            case NUC_K_CORR_STEP1:
                HIPCHK(ctx, timed_launch(ctx, NUC_K_CORR_STEP1, s, [&] { return launch_corr_step1(st.cls, b, s); }));
                break;
            case NUC_K_CORR_CHAIN:
                HIPCHK(ctx, timed_launch(ctx, NUC_K_CORR_CHAIN, s,
                                         [&] { return launch_corr_chain(st.cls, st.prec, b, s); }));
                break;
            case NUC_K_CORR_REDUCE:
                HIPCHK(ctx, timed_launch(ctx, NUC_K_CORR_REDUCE, s, [&] { return launch_corr_reduce(b, s); }));
                break;
            case NUC_K_CORR_SCALE:
                HIPCHK(ctx, timed_launch(ctx, NUC_K_CORR_SCALE, s, [&] {
                           return st.prec == NUC_BF16X3 ? launch_corr_split_tau(b, s) : launch_corr_scale(b, s);
                       }));
                break;
        }
    }
    return NUC_OK;
}

nuc_status ensure_workspace(nuc_ctx ctx, size_t bytes, hipStream_t s) {
    if (ctx->budget && bytes > ctx->budget)
        return fail(ctx, NUC_ERR_NOMEM, "workspace of %zu bytes exceeds the HBM budget of %zu bytes", bytes,
                    ctx->budget);
    if (bytes <= ctx->ws_size) return NUC_OK;
    if (ctx->graphs_alive > 0)
        return fail(ctx, NUC_ERR_BUSY, "workspace must grow to %zu bytes but %d captured graph(s) use it", bytes,
                    ctx->graphs_alive);
    if (ctx->ws) {
        HIPCHK(ctx, hipStreamSynchronize(s));
        if (ctx->have_done) HIPCHK(ctx, hipEventSynchronize(ctx->done));
        HIPCHK(ctx, hipFree(ctx->ws));
        ctx->ws = nullptr;
        ctx->ws_size = 0;
    }
    const size_t want = align_up(bytes, (size_t)1 << 20);
    hipError_t e = hipMalloc(&ctx->ws, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        ctx->ws = nullptr;
        return fail(ctx, NUC_ERR_NOMEM, "hipMalloc(%zu) failed: %s", want, hipGetErrorString(e));
    }
    ctx->ws_size = want;
    return NUC_OK;
}

nuc_status upload_block(nuc_ctx ctx, const HostBlock& hb, void* dst, hipStream_t s, bool may_grow) {
    const size_t n = hb.bytes.size();
    if (n == 0) return NUC_OK;
    if (ctx->have_staged) HIPCHK(ctx, hipEventSynchronize(ctx->staged));
    if (n > ctx->staging_size && !may_grow)
        return fail(ctx, NUC_ERR_NOMEM, "launch constants of %zu bytes exceed the %zu-byte staging buffer", n,
                    ctx->staging_size);
    if (n > ctx->staging_size) {
        if (ctx->staging) HIPCHK(ctx, hipHostFree(ctx->staging));
        ctx->staging = nullptr;
        ctx->staging_size = 0;
        const size_t want = align_up(n, 65536);
        HIPCHK(ctx, hipHostMalloc(&ctx->staging, want, hipHostMallocDefault));
        ctx->staging_size = want;
    }
    memcpy(ctx->staging, hb.bytes.data(), n);
    HIPCHK(ctx, hipMemcpyAsync(dst, ctx->staging, n, hipMemcpyHostToDevice, s));
    HIPCHK(ctx, hipEventRecord(ctx->staged, s));
    ctx->have_staged = true;
    return NUC_OK;
}

// ------------------------------------------------- static scratch (no allocation)
//
// The scratch of nuc_correlator_noalloc: a file-scope device array that every GPU
// the library runs on holds until the process ends. In host code its name is only
// a stand-in; the device address of each GPU's copy comes from
// hipGetSymbolAddress, taken once per device in nuc_create with that device
// current, and only that address is ever passed to kernels or copies.
static __device__ __align__(256) char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // HIP device ordinal -> address of its copy of scratch

nuc_status static_scratch_setup(nuc_ctx ctx) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr.count(ctx->device)) return NUC_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return fail(ctx, NUC_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d failed: %s", ctx->device,
                    hipGetErrorString(e));
    }
    g_scratch_ptr[ctx->device] = ptr;
    return NUC_OK;
}

void* static_scratch(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    return it == g_scratch_ptr.end() ? nullptr : it->second;
}

// Order this call after the previous call of the context (which may have used
// another stream) so the shared workspace is never used by two calls at once.
nuc_status begin_call(nuc_ctx ctx, hipStream_t s) {
    HIPCHK(ctx, hipSetDevice(ctx->device));
    if (ctx->have_done) HIPCHK(ctx, hipStreamWaitEvent(s, ctx->done, 0));
    return NUC_OK;
}

nuc_status end_call(nuc_ctx ctx, hipStream_t s) {
    HIPCHK(ctx, hipEventRecord(ctx->done, s));
    ctx->have_done = true;
    return NUC_OK;
}


// Validate one job and copy its small host inputs. stage: 1 elementals,
// 2 correlator, 3 both.
nuc_status make_job(nuc_ctx ctx, const nuc_geom* g, const void* evecs, const double* evals, int nprof,
                    const nuc_profile* prof, int nmom, const int32_t* mom, const void* peramb, nuc_precision prec,
                    void* phi, void* corr, int stage, Job& J, int ld) {
    nuc_status st;
    if ((st = check_geom(ctx, g)) != NUC_OK) return st;
    if (ld != 0 && (ld < g->nvec || ld > 4096))
        return fail(ctx, NUC_ERR_INVALID, "ld_nvec=%d must be 0 or in [nvec=%d, 4096]", ld, g->nvec);
    J.ld = ld ? ld : g->nvec;
    if ((st = check_prec(ctx, raw_enum(prec))) != NUC_OK) return st;
    if (nmom < 1 || nmom > 64) return fail(ctx, NUC_ERR_INVALID, "nmom=%d out of range [1,64]", nmom);
    J.g = *g;
    J.nmom = nmom;
    J.prec = (int)prec;
    J.do_elem = stage & 1;
    J.do_corr = (stage & 2) != 0;
    J.evecs = evecs;
    J.peramb = peramb;
    J.phi = phi;
    J.corr = corr;
    if (J.do_elem) {
        if (!evecs) return fail(ctx, NUC_ERR_INVALID, "evecs is NULL");
        if ((st = check_moms(ctx, g, nmom, mom)) != NUC_OK) return st;
        if (!J.do_corr && !phi) return fail(ctx, NUC_ERR_INVALID, "phi is NULL");
        J.mom.assign(mom, mom + 3 * nmom);
    }
    if (J.do_corr) {
        if (!J.do_elem && !phi) return fail(ctx, NUC_ERR_INVALID, "phi is NULL");
        if ((st = check_prec_shape(ctx, prec, g, J.ld)) != NUC_OK) return st;
        if ((st = check_profiles(ctx, g, evals, nprof, prof)) != NUC_OK) return st;
        if (!peramb) return fail(ctx, NUC_ERR_INVALID, "peramb is NULL");
        if (!corr) return fail(ctx, NUC_ERR_INVALID, "corr is NULL");
        const int N = g->nvec;
        J.nprof = nprof;
        J.gsnk.resize((size_t)nprof * g->T * N);
        eval_profiles(g, evals, nprof, prof, J.gsnk.data());
        J.gsrc.resize((size_t)nprof * N);
        for (int a = 0; a < nprof; ++a)
            memcpy(&J.gsrc[(size_t)a * N], &J.gsnk[((size_t)a * g->T + g->t0) * N], N * sizeof(double));
    }
    return NUC_OK;
}

// Tuned launch shapes do not depend on the number of timeslices.
std::vector<int> shape_key(const Job& J) {
    return {J.g.L, J.g.nvec, J.ld, J.nmom, J.nprof, J.prec, J.do_elem, J.do_corr};
}

void apply_tuning(nuc_ctx ctx, Program& P) {
    for (Job& J : P.jobs) {
        auto it = ctx->tuned.find(shape_key(J));
        if (it != ctx->tuned.end()) {
            J.elem_mp = it->second.first;
            J.s1_target = it->second.second;
        }
    }
}

nuc_status run_program(nuc_ctx ctx, Program& P, hipStream_t s) {
    apply_tuning(ctx, P);
    nuc_status st;
    if ((st = plan_program(ctx, P, ctx->budget ? std::min(kBatchCap, ctx->budget / 2) : kBatchCap)) != NUC_OK)
        return st;
    if ((st = begin_call(ctx, s)) != NUC_OK) return st;
    if ((st = ensure_workspace(ctx, P.total_bytes, s)) != NUC_OK) return st;
    char* base = (char*)ctx->ws;
    fill_program(P, base);
    if ((st = upload_block(ctx, P.block, base, s)) != NUC_OK) return st;
    if ((st = enqueue_program(ctx, P, base, s)) != NUC_OK) return st;
    return end_call(ctx, s);
}

// A Program on the static scratch: no workspace growth, no staging growth.
nuc_status run_program_static(nuc_ctx ctx, Program& P, hipStream_t s) {
    apply_tuning(ctx, P);
    char* base = (char*)static_scratch(ctx->device);
    if (!base) return fail(ctx, NUC_ERR_INTERNAL, "no static scratch address for device %d", ctx->device);
    nuc_status st;
    // rounds sized so that the constants (at most the staging buffer) and the scratch fit
    if ((st = plan_program(ctx, P, kStaticScratchBytes - kStaticStagingBytes)) != NUC_OK) return st;
    if (P.total_bytes > kStaticScratchBytes)
        return fail(ctx, NUC_ERR_NOMEM,
                    "needs %zu bytes of scratch (one round holds at least one sink timeslice); the static "
                    "array holds %zu",
                    P.total_bytes, kStaticScratchBytes);
    if ((st = begin_call(ctx, s)) != NUC_OK) return st;
    fill_program(P, base);
    if ((st = upload_block(ctx, P.block, base, s, false)) != NUC_OK) return st;
    if ((st = enqueue_program(ctx, P, base, s)) != NUC_OK) return st;
    return end_call(ctx, s);
}

}  // namespace rt
}  // namespace nuc

using namespace nuc::rt;

// ======================================================================== ABI

extern "C" {

const char* nuc_version(void) { return NUC_VERSION; }

const char* nuc_status_string(nuc_status s) {
    switch (raw_enum(s)) {  // a caller may pass any int
        case NUC_OK: return "ok";
        case NUC_ERR_INVALID: return "invalid argument";
        case NUC_ERR_NOMEM: return "out of workspace memory";
        case NUC_ERR_DEVICE: return "device error";
        case NUC_ERR_UNSUPPORTED: return "unsupported";
        case NUC_ERR_BUSY: return "busy";
        case NUC_ERR_INTERNAL: return "internal error";
        case NUC_ERR_TIMEOUT: return "timed out";
        case NUC_ERR_CANCELLED: return "cancelled";
    }
    return "unknown status";
}

const char* nuc_last_error(nuc_ctx ctx) { return ctx ? ctx->err.c_str() : g_thread_err.c_str(); }

nuc_status nuc_create(nuc_ctx* out, int device, size_t hbm_budget_bytes) {
    if (!out) return fail(nullptr, NUC_ERR_INVALID, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        return fail(nullptr, NUC_ERR_DEVICE, "no HIP device available");
    }
    if (device < 0 || device >= ndev)
        return fail(nullptr, NUC_ERR_INVALID, "device %d outside [0,%d)", device, ndev);
    DeviceGuard guard;
    nuc_ctx c = new nuc_ctx_s();
    c->device = device;
    c->budget = hbm_budget_bytes;
    if ((e = hipSetDevice(device)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->done, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->staged, hipEventDisableTiming)) != hipSuccess ||
        (e = hipHostMalloc(&c->staging, kStaticStagingBytes, hipHostMallocDefault)) != hipSuccess) {
        nuc_status st = hip_fail(nullptr, e, "context setup");
        nuc_destroy(c);
        return st;
    }
    c->staging_size = kStaticStagingBytes;
    nuc_status st = static_scratch_setup(c);
    if (st != NUC_OK) {
        fail(nullptr, st, "%s", c->err.c_str());
        nuc_destroy(c);
        return st;
    }
    *out = c;
    return NUC_OK;
}

nuc_status nuc_destroy(nuc_ctx ctx) {
    if (!ctx) return NUC_OK;
    DeviceGuard guard;
    (void)hipSetDevice(ctx->device);
    if (ctx->have_done) (void)hipEventSynchronize(ctx->done);
    if (ctx->have_staged) (void)hipEventSynchronize(ctx->staged);
    for (auto& t : ctx->timed) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->staging) (void)hipHostFree(ctx->staging);
    if (ctx->done) (void)hipEventDestroy(ctx->done);
    if (ctx->staged) (void)hipEventDestroy(ctx->staged);
    delete ctx;
    return NUC_OK;
}

const char* nuc_kernel_name(int id) {
    static const char* names[NUC_K_COUNT] = {"elementals",   "elem_expand", "corr_step1",         "corr_chain",
                                             "corr_reduce",  "corr_scale",  "meson_deriv",        "meson_elem",
                                             "meson_reduce", "meson_gemm",  "meson_trace",        "meson_sum",
                                             "meson_weight", "meson_phase", "glue_stencil",      "glue_contract",
                                             "spin_source",  "spin_gemm",   "spin_sink",
                                             "tm_operator",  "tm_gemm",     "tm_pair",            "tm_sum"};
    return (id >= 0 && id < NUC_K_COUNT) ? names[id] : "?";
}

nuc_status nuc_timing_enable(nuc_ctx ctx, int on) {
    if (!ctx) return fail(nullptr, NUC_ERR_INVALID, "ctx is NULL");
    std::lock_guard<std::mutex> lock(ctx->mu);
    DeviceGuard guard;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    for (auto& t : ctx->timed) {
        HIPCHK(ctx, hipEventSynchronize(t.b));
        ctx->ev_pool.push_back(t.a);
        ctx->ev_pool.push_back(t.b);
    }
    ctx->timed.clear();
    ctx->timing = on != 0;
    return NUC_OK;
}

nuc_status nuc_timing_read(nuc_ctx ctx, double* ms, int* launches) {
    if (!ctx) return fail(nullptr, NUC_ERR_INVALID, "ctx is NULL");
    if (!ms || !launches) return fail(ctx, NUC_ERR_INVALID, "ms or launches is NULL");
    std::lock_guard<std::mutex> lock(ctx->mu);
    DeviceGuard guard;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    for (int k = 0; k < NUC_K_COUNT; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    for (auto& t : ctx->timed) {
        HIPCHK(ctx, hipEventSynchronize(t.b));
        float e = 0.f;
        HIPCHK(ctx, hipEventElapsedTime(&e, t.a, t.b));
        ms[t.id] += e;
        launches[t.id] += 1;
        ctx->ev_pool.push_back(t.a);
        ctx->ev_pool.push_back(t.b);
    }
    ctx->timed.clear();
    return NUC_OK;
}

nuc_status nuc_profiles_eval(const nuc_geom* geom, const double* evals, int nprof, const nuc_profile* prof,
                             double* g_out) {
    nuc_status st;
    if ((st = check_geom(nullptr, geom)) != NUC_OK) return st;
    if ((st = check_profiles(nullptr, geom, evals, nprof, prof)) != NUC_OK) return st;
    if (!g_out) return fail(nullptr, NUC_ERR_INVALID, "g_out is NULL");
    eval_profiles(geom, evals, nprof, prof, g_out);
    return NUC_OK;
}

nuc_status nuc_workspace_query(const nuc_geom* geom, int nmom, int nprof, nuc_precision prec, size_t* bytes) {
    nuc_status st;
    if ((st = check_geom(nullptr, geom)) != NUC_OK) return st;
    if (nmom < 1 || nmom > 64) return fail(nullptr, NUC_ERR_INVALID, "nmom=%d out of range [1,64]", nmom);
    if (nprof < 1 || nprof > kMaxProf) return fail(nullptr, NUC_ERR_INVALID, "nprof=%d out of range", nprof);
    if ((st = check_prec(nullptr, raw_enum(prec))) != NUC_OK) return st;
    if (!bytes) return fail(nullptr, NUC_ERR_INVALID, "bytes is NULL");
    Program P;
    P.jobs.resize(1);
    Job& J = P.jobs[0];
    J.g = *geom;
    J.nmom = nmom;
    J.nprof = nprof;
    J.prec = (int)prec;
    J.do_elem = J.do_corr = true;
    J.ld = geom->nvec;
    J.phi = (void*)1;  // caller supplies phi
    J.mom.assign((size_t)3 * nmom, 0);
    J.gsnk.assign((size_t)nprof * geom->T * geom->nvec, 1.0);
    J.gsrc.assign((size_t)nprof * geom->nvec, 1.0);
    if ((st = plan_program(nullptr, P, kBatchCap)) != NUC_OK) return st;
    *bytes = P.total_bytes;
    return NUC_OK;
}

static nuc_status run_single(nuc_ctx ctx, const nuc_geom* g, const void* evecs, const double* evals, int nprof,
                             const nuc_profile* prof, int nmom, const int32_t* mom, const void* peramb,
                             nuc_precision prec, void* phi, void* corr, void* stream, int stage) {
    if (!ctx) return fail(nullptr, NUC_ERR_INVALID, "ctx is NULL");
    std::lock_guard<std::mutex> lock(ctx->mu);
    Program P;
    P.jobs.resize(1);
    nuc_status st = make_job(ctx, g, evecs, evals, nprof, prof, nmom, mom, peramb, prec, phi, corr, stage, P.jobs[0]);
    if (st != NUC_OK) return st;
    DeviceGuard guard;
    return run_program(ctx, P, (hipStream_t)stream);
}

nuc_status nuc_elementals(nuc_ctx ctx, const nuc_geom* geom, const void* evecs, int nmom, const int32_t* mom,
                          nuc_precision prec, void* phi, void* stream) {
    if (check_prec(ctx, raw_enum(prec)) != NUC_OK) return NUC_ERR_INVALID;  // before any read of prec
    return run_single(ctx, geom, evecs, nullptr, 0, nullptr, nmom, mom, nullptr, prec, phi, nullptr, stream, 1);
}

nuc_status nuc_correlator(nuc_ctx ctx, const nuc_geom* geom, const void* phi, const double* evals, int nprof,
                          const nuc_profile* prof, int nmom, const void* peramb, nuc_precision prec, void* corr,
                          void* stream) {
    if (check_prec(ctx, raw_enum(prec)) != NUC_OK) return NUC_ERR_INVALID;  // before any read of prec
    return run_single(ctx, geom, nullptr, evals, nprof, prof, nmom, nullptr, peramb, prec, (void*)phi, corr, stream,
                      2);
}

nuc_status nuc_correlator_noalloc(nuc_ctx ctx, const nuc_geom* geom, const void* phi, const double* evals,
                                  int nprof, const nuc_profile* prof, int nmom, const void* peramb,
                                  nuc_precision prec, void* corr, void* stream) {
    if (!ctx) return fail(nullptr, NUC_ERR_INVALID, "ctx is NULL");
    if (check_prec(ctx, raw_enum(prec)) != NUC_OK) return NUC_ERR_INVALID;  // before any read of prec
    std::lock_guard<std::mutex> lock(ctx->mu);
    Program P;
    P.jobs.resize(1);
    nuc_status st =
        make_job(ctx, geom, nullptr, evals, nprof, prof, nmom, nullptr, peramb, prec, (void*)phi, corr, 2, P.jobs[0]);
    if (st != NUC_OK) return st;
    DeviceGuard guard;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    return run_program_static(ctx, P, (hipStream_t)stream);
}

nuc_status nuc_run(nuc_ctx ctx, const nuc_geom* geom, const void* evecs, const double* evals, int nprof,
                   const nuc_profile* prof, int nmom, const int32_t* mom, const void* peramb, nuc_precision prec,
                   void* phi, void* corr, void* stream) {
    if (check_prec(ctx, raw_enum(prec)) != NUC_OK) return NUC_ERR_INVALID;  // before any read of prec
    return run_single(ctx, geom, evecs, evals, nprof, prof, nmom, mom, peramb, prec, phi, corr, stream, 3);
}

static nuc_status build_batch(nuc_ctx ctx, int njobs, const nuc_job* jobs, nuc_precision prec, Program& P) {
    if (njobs < 1 || njobs > 4096) return fail(ctx, NUC_ERR_INVALID, "njobs=%d out of range [1,4096]", njobs);
    if (!jobs) return fail(ctx, NUC_ERR_INVALID, "jobs is NULL");
    P.jobs.resize(njobs);
    for (int i = 0; i < njobs; ++i) {
        const nuc_job& j = jobs[i];
        nuc_status st = make_job(ctx, &j.geom, j.evecs, j.evals, j.nprof, j.prof, j.nmom, j.mom, j.peramb, prec,
                                 j.phi, j.corr, 3, P.jobs[i], j.ld_nvec);
        if (st != NUC_OK) {
            fail(ctx, st, "job %d: %s", i, std::string(ctx->err).c_str());
            return st;
        }
    }
    return NUC_OK;
}

nuc_status nuc_batch_run(nuc_ctx ctx, int njobs, const nuc_job* jobs, nuc_precision prec, void* stream) {
    if (check_prec(ctx, raw_enum(prec)) != NUC_OK) return NUC_ERR_INVALID;  // before any read of prec
    if (!ctx) return fail(nullptr, NUC_ERR_INVALID, "ctx is NULL");
    std::lock_guard<std::mutex> lock(ctx->mu);
    Program P;
    nuc_status st = build_batch(ctx, njobs, jobs, prec, P);
    if (st != NUC_OK) return st;
    DeviceGuard guard;
    return run_program(ctx, P, (hipStream_t)stream);
}

nuc_status nuc_batch_graph(nuc_ctx ctx, int njobs, const nuc_job* jobs, nuc_precision prec, nuc_graph* out) {
    if (check_prec(ctx, raw_enum(prec)) != NUC_OK) return NUC_ERR_INVALID;  // before any read of prec
    if (!ctx) return fail(nullptr, NUC_ERR_INVALID, "ctx is NULL");
    if (!out) return fail(ctx, NUC_ERR_INVALID, "out is NULL");
    *out = nullptr;
    std::lock_guard<std::mutex> lock(ctx->mu);
    Program P;
    nuc_status st = build_batch(ctx, njobs, jobs, prec, P);
    if (st != NUC_OK) return st;
    DeviceGuard guard;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    apply_tuning(ctx, P);
    if ((st = plan_program(ctx, P, ctx->budget ? std::min(kBatchCap, ctx->budget / 2) : kBatchCap)) != NUC_OK)
        return st;
    hipStream_t cs = nullptr;
    HIPCHK(ctx, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    st = ensure_workspace(ctx, P.total_bytes, cs);
    if (st != NUC_OK) {
        (void)hipStreamDestroy(cs);
        return st;
    }
    char* base = (char*)ctx->ws;
    fill_program(P, base);
    nuc_graph g = new nuc_graph_s();
    g->ctx = ctx;
    hipError_t e = hipHostMalloc(&g->staging, std::max<size_t>(P.block.bytes.size(), 1), hipHostMallocDefault);
    if (e == hipSuccess) memcpy(g->staging, P.block.bytes.data(), P.block.bytes.size());
    const bool timing = ctx->timing;
    ctx->timing = false;
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        e = hipMemcpyAsync(base, g->staging, P.block.bytes.size(), hipMemcpyHostToDevice, cs);
        nuc_status est = (e == hipSuccess) ? enqueue_program(ctx, P, base, cs) : NUC_ERR_DEVICE;
        hipError_t e2 = hipStreamEndCapture(cs, &g->graph);
        if (e == hipSuccess && est != NUC_OK) e = hipErrorUnknown;
        if (e == hipSuccess) e = e2;
    }
    ctx->timing = timing;
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        if (g->staging) (void)hipHostFree(g->staging);
        delete g;
        return hip_fail(ctx, e, "graph capture");
    }
    ctx->graphs_alive += 1;
    *out = g;
    return NUC_OK;
}

nuc_status nuc_autotune(nuc_ctx ctx, const nuc_job* job, nuc_precision prec, void* stream, int* best) {
    if (check_prec(ctx, raw_enum(prec)) != NUC_OK) return NUC_ERR_INVALID;  // before any read of prec
    if (!ctx) return fail(nullptr, NUC_ERR_INVALID, "ctx is NULL");
    Program P0;
    nuc_status st;
    {
        std::lock_guard<std::mutex> lock(ctx->mu);
        if ((st = build_batch(ctx, 1, job, prec, P0)) != NUC_OK) return st;
    }
    const std::vector<int> key = shape_key(P0.jobs[0]);
    const int mps[3] = {1, 2, 4};
    const int s1s[3] = {768, 1536, 3072};
    const bool was_timing = ctx->timing;
    auto timed_run = [&](int mp, int s1, int kid, double& ms) -> nuc_status {
        std::lock_guard<std::mutex> lock(ctx->mu);
        Program P;
        P.jobs = P0.jobs;
        P.jobs[0].elem_mp = mp;
        P.jobs[0].s1_target = s1;
        for (auto& t : ctx->timed) {
            (void)hipEventSynchronize(t.b);
            ctx->ev_pool.push_back(t.a);
            ctx->ev_pool.push_back(t.b);
        }
        ctx->timed.clear();
        ctx->timing = true;
        DeviceGuard guard;
        nuc_status r = NUC_OK;
        double best_ms = 1e300;
        for (int rep = 0; rep < 3 && r == NUC_OK; ++rep) {  // first run warms up
            r = plan_program(ctx, P, ctx->budget ? std::min(kBatchCap, ctx->budget / 2) : kBatchCap);
            hipStream_t s = (hipStream_t)stream;
            if (r == NUC_OK) r = begin_call(ctx, s);
            if (r == NUC_OK) r = ensure_workspace(ctx, P.total_bytes, s);
            if (r == NUC_OK) {
                char* base = (char*)ctx->ws;
                fill_program(P, base);
                r = upload_block(ctx, P.block, base, s);
            }
            if (r == NUC_OK) r = enqueue_program(ctx, P, (char*)ctx->ws, s);
            if (r == NUC_OK) r = end_call(ctx, s);
            double sum = 0.0;
            for (auto& t : ctx->timed) {
                float e = 0.f;
                if (hipEventSynchronize(t.b) != hipSuccess || hipEventElapsedTime(&e, t.a, t.b) != hipSuccess)
                    r = NUC_ERR_DEVICE;
                if (t.id == kid) sum += e;
                ctx->ev_pool.push_back(t.a);
                ctx->ev_pool.push_back(t.b);
            }
            ctx->timed.clear();
            if (rep > 0) best_ms = std::min(best_ms, sum);
            P.stages.clear();
            P.block.bytes.clear();
        }
        ctx->timing = was_timing;
        ms = best_ms;
        return r;
    };
    int best_mp = 0, best_s1 = 0;
    double tmin = 1e300;
    if (P0.jobs[0].do_elem) {
        for (int mp : mps) {
            if (mp > 1 && P0.jobs[0].nmom < mp / 2 + 1) continue;
            double ms;
            if ((st = timed_run(mp, 0, NUC_K_ELEMENTALS, ms)) != NUC_OK) return st;
            if (ms < tmin) {
                tmin = ms;
                best_mp = mp;
            }
        }
    }
    tmin = 1e300;
    if (P0.jobs[0].do_corr) {
        for (int s1 : s1s) {
            double ms;
            if ((st = timed_run(best_mp, s1, NUC_K_CORR_STEP1, ms)) != NUC_OK) return st;
            if (ms < tmin) {
                tmin = ms;
                best_s1 = s1;
            }
        }
    }
    {
        std::lock_guard<std::mutex> lock(ctx->mu);
        ctx->tuned[key] = {best_mp, best_s1};
    }
    if (best) {
        best[0] = best_mp;
        best[1] = best_s1;
    }
    return NUC_OK;
}

nuc_status nuc_graph_launch(nuc_graph g, void* stream) {
    if (!g) return fail(nullptr, NUC_ERR_INVALID, "graph is NULL");
    nuc_ctx ctx = g->ctx;
    std::lock_guard<std::mutex> lock(ctx->mu);
    DeviceGuard guard;
    hipStream_t s = (hipStream_t)stream;
    nuc_status st = begin_call(ctx, s);
    if (st != NUC_OK) return st;
    HIPCHK(ctx, hipGraphLaunch(g->exec, s));
    return end_call(ctx, s);
}

nuc_status nuc_graph_destroy(nuc_graph g) {
    if (!g) return NUC_OK;
    nuc_ctx ctx = g->ctx;
    std::lock_guard<std::mutex> lock(ctx->mu);
    DeviceGuard guard;
    (void)hipSetDevice(ctx->device);
    if (ctx->have_done) (void)hipEventSynchronize(ctx->done);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->staging) (void)hipHostFree(g->staging);
    ctx->graphs_alive -= 1;
    delete g;
    return NUC_OK;
}

}  // extern "C"

// Host runtime of the profiled meson operators of the charmonium study (paper
// Section 3): argument checks, the spin algebra of the operator families, the plans of
// the elementals and correlator stages (timeslices per launch, K splits, GEMM item
// lists) and the C ABI entry points nuc_meson_elementals / nuc_meson_correlator /
// nuc_meson_run. The kernels are in meson_elem.hip and meson_corr.hip.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <complex>
#include <vector>

#include "../../include/nucleon.h"
#include "meson_internal.h"
#include "meson_spin.h"
#include "runtime_internal.h"

namespace nuc {
namespace meson {

constexpr size_t kMesonCap = (size_t)16 << 30;

// ================================================================ host side

using namespace nuc::rt;
float2 f2(cd z) { return make_float2((float)z.real(), (float)z.imag()); }

nuc_status check_meson_geom(nuc_ctx ctx, const nuc_geom* g) {
    if (!g) return fail(ctx, NUC_ERR_INVALID, "geom is NULL");
    if (g->L < 1 || g->L > 256) return fail(ctx, NUC_ERR_INVALID, "L=%d out of range [1,256]", g->L);
    if (g->T < 1) return fail(ctx, NUC_ERR_INVALID, "T=%d must be >= 1", g->T);
    if (g->nvec < 1 || g->nvec > kMaxNvecMeson)
        return fail(ctx, NUC_ERR_INVALID, "nvec=%d out of range [1,%d] for meson operators", g->nvec,
                    kMaxNvecMeson);
    if (g->t0 < 0 || g->t0 >= g->T) return fail(ctx, NUC_ERR_INVALID, "t0=%d outside [0,T)", g->t0);
    if ((long long)g->L * g->L * g->L * 3 > INT32_MAX / 2)
        return fail(ctx, NUC_ERR_INVALID, "L=%d too large", g->L);
    return NUC_OK;
}

// ------------------------------------------------------------ elementals plan

struct ElemPlan {
    int Tc = 1, nsplit = 1, cps = 1, nchunks = 1, mt = 1, nt = 1, Kp = 2;
    size_t off_ph = 0, off_A = 0, off_V = 0, off_F = 0, off_part = 0, bytes = 0;
};

ElemPlan plan_elem(const nuc_geom& g, int nmom, size_t cap) {
    ElemPlan P;
    const size_t N = g.nvec, V3 = (size_t)g.L * g.L * g.L, K = 3 * V3;
    P.Kp = (int)((K + 1) / 2 * 2);
    P.nchunks = (int)((K + EKC - 1) / EKC);
    P.mt = (int)((N + 63) / 64);
    P.nt = (int)((kND * N + ElemTile<kElemNB>::TN - 1) / ElemTile<kElemNB>::TN);
    // derivative fields, phase-weighted vectors and the vector copy, all with rows of Kp
    const size_t fields_t = (6 + nmom + 1) * N * P.Kp * sizeof(float2);
    const size_t part_t = (size_t)nmom * N * kND * N * sizeof(double2);
    const size_t ph = (size_t)nmom * V3 * sizeof(float2);
    // timeslices per launch Tc and K splits: a launch is tc nmom mt nt nsplit workgroups
    // of equal work (proportional to 1 / nsplit), run in rounds of `slots`. Pick the
    // pair whose workspace fits and whose summed rounds over all launches (the last one
    // may hold fewer timeslices) take the least time; a little extra for each split's
    // partials; ties go to the larger Tc.
    const long long slots = kElemNB <= 2 ? 512 : 256;
    const int max_split = std::max(1, std::min(16, P.nchunks / 16));
    const long long X = (long long)nmom * P.mt * P.nt;
    double best = 1e300;
    P.Tc = 1;
    P.nsplit = 1;
    for (int tc = g.T; tc >= 1; --tc)
        for (int ns = 1; ns <= max_split; ++ns) {
            if ((fields_t + part_t * ns) * tc > cap && !(tc == 1 && ns == 1)) continue;
            double rounds = 0.0;
            for (int t0c = 0; t0c < g.T; t0c += tc) {
                const long long items = (long long)std::min(tc, g.T - t0c) * X * ns;
                rounds += (double)((items + slots - 1) / slots);
            }
            const double cost = rounds / ns * (1.0 + 0.01 * ns);
            if (cost < best * (1.0 - 1e-9)) {
                best = cost;
                P.Tc = tc;
                P.nsplit = ns;
            }
        }
    P.cps = (P.nchunks + P.nsplit - 1) / P.nsplit;
    P.nsplit = (P.nchunks + P.cps - 1) / P.cps;
    P.off_ph = 0;
    P.off_A = align_up(ph, 256);
    P.off_V = P.off_A + align_up((size_t)nmom * N * P.Kp * sizeof(float2) * P.Tc, 256);
    P.off_F = P.off_V + align_up(N * P.Kp * sizeof(float2) * P.Tc, 256);
    P.off_part = P.off_F + align_up(6 * N * P.Kp * sizeof(float2) * P.Tc, 256);
    P.bytes = P.off_part + align_up(part_t * P.nsplit * P.Tc, 256);
    return P;
}

// --------------------------------------------------------- correlator plan

struct CorrPlan {
    int Tc = 1, nwg = 1, cpb = 1, nop = 3, tiles_per_tp = 0, nitems = 0;
    size_t off_items = 0, off_offs = 0, off_gsnk = 0, off_gsrc = 0, block_bytes = 0;
    size_t off_Pt = 0, off_Ps = 0, off_Y = 0, off_Z = 0, off_part = 0, bytes = 0;
    HostBlock block;
    int pi5[4];
    float2 s5[4];
};

nuc_status plan_corr(nuc_ctx ctx, const nuc_geom& g, int nmom, int nprof, const double* gall, size_t cap,
                     CorrPlan& P) {
    const int N = g.nvec, T = g.T;
    std::vector<std::vector<Term>> fam;
    Perm g5p;
    double g4d[4];
    if (!operator_terms(fam, g5p, g4d)) return fail(ctx, NUC_ERR_INTERNAL, "spin matrices are not permutations");
    P.nop = kNFam * nprof;
    const size_t N2 = (size_t)N * N, N16 = 16 * N2;
    const size_t wsz = (size_t)kND * nprof * N2;  // weighted elementals per (t, p)
    std::vector<GemmItem> items;
    auto tiles = [](int n) { return (n + 63) / 64; };
    // Y_(f,a) = M_(f,a) tau for all profiles a of family f at once, row block alpha:
    //   rows (a, i): sum_k Gamma_k[alpha][pi_k(alpha)] (g^a g^a Phi^{D_k})[i][.] tau[pi_k(alpha) block][.]
    for (int f = 0; f < kNFam; ++f)
        for (int al = 0; al < 4; ++al) {
            GemmItem I{};
            I.out_src = SRC_Y;
            I.out_off = (int)((size_t)f * nprof * N16 + (size_t)al * N * 4 * N);
            I.ldo = 4 * N;
            I.M = nprof * N;
            I.Nc = 4 * N;
            I.Kseg = N;
            I.nseg = (int)fam[f].size();
            I.rb = N;
            I.rbs = (int)N16;
            I.cb = I.Nc;
            I.cbs = 0;
            I.tiles_m = tiles(I.M);
            I.tiles_n = tiles(I.Nc);
            for (int k = 0; k < I.nseg; ++k) {
                const Term& tm = fam[f][k];
                GemmSeg& sg = I.seg[k];
                sg.a_src = SRC_PS;
                sg.a_off = (int)(tm.D * nprof * N2);
                sg.lda = N;
                sg.b_src = SRC_TAU;
                sg.b_off = (int)((size_t)tm.G.col[al] * N * 4 * N);
                sg.ldb = 4 * N;
                sg.coef = f2(tm.G.val[al]);
            }
            items.push_back(I);
        }
    // Z~_(f,b) for all profiles b of family f at once, column block beta: columns (b, j):
    //   sum_k s5'(alpha) g4(alpha) g4(beta) Gamma_k[alpha][beta] tau[:, rho5(alpha) block] (g^b g^b Phi^{D_k}(t0)),
    // alpha = the row of Gamma_k's nonzero in column beta. Z_B = (g5 tau g5)(g4 M_B(t0) g4) has
    // row block gamma equal to s5(gamma) times row block pi5(gamma) of Z~_B.
    for (int f = 0; f < kNFam; ++f)
        for (int be = 0; be < 4; ++be) {
            GemmItem I{};
            I.out_src = SRC_Z;
            I.out_off = (int)((size_t)f * nprof * N16 + (size_t)be * N);
            I.ldo = 4 * N;
            I.M = 4 * N;
            I.Nc = nprof * N;
            I.Kseg = N;
            I.nseg = (int)fam[f].size();
            I.rb = I.M;
            I.rbs = 0;
            I.cb = N;
            I.cbs = (int)N16;
            I.tiles_m = tiles(I.M);
            I.tiles_n = tiles(I.Nc);
            for (int k = 0; k < I.nseg; ++k) {
                const Term& tm = fam[f][k];
                const int al = tm.G.row_of_col[be];
                const int rho = g5p.row_of_col[al];
                const cd s5c = g5p.val[rho];  // g5[rho][al]
                GemmSeg& sg = I.seg[k];
                sg.a_src = SRC_TAU;
                sg.a_off = rho * N;
                sg.lda = 4 * N;
                sg.b_src = SRC_PT;
                sg.b_off = (int)(tm.D * nprof * N2);
                sg.ldb = nprof * N;
                sg.coef = f2(s5c * g4d[al] * g4d[be] * tm.G.val[al]);
            }
            items.push_back(I);
        }
    for (int gm = 0; gm < 4; ++gm) {
        P.pi5[gm] = g5p.col[gm];
        P.s5[gm] = f2(g5p.val[gm]);
    }
    // every operand and output element of every item inside its buffer
    auto src_size = [&](int src) -> size_t {
        switch (src) {
            case SRC_PS:
            case SRC_PT: return wsz;
            case SRC_TAU: return N16;
            case SRC_Y:
            case SRC_Z: return (size_t)P.nop * N16;
        }
        return 0;
    };
    for (const GemmItem& I : items) {
        bool ok = I.nseg >= 1 && I.nseg <= 3 && I.rb >= 1 && I.cb >= 1;
        size_t rmax = 0, cmax = 0;
        for (int r = 0; ok && r < I.M; ++r) rmax = std::max(rmax, (size_t)(r / I.rb) * I.rbs + (size_t)(r % I.rb) * I.ldo);
        for (int c = 0; ok && c < I.Nc; ++c) cmax = std::max(cmax, (size_t)(c / I.cb) * I.cbs + c % I.cb);
        ok = ok && (size_t)I.out_off + rmax + cmax < src_size(I.out_src);
        for (int k = 0; ok && k < I.nseg; ++k) {
            const GemmSeg& sg = I.seg[k];
            ok = ok && (size_t)sg.a_off + (size_t)(I.M - 1) * sg.lda + I.Kseg <= src_size(sg.a_src);
            ok = ok && (size_t)sg.b_off + (size_t)(I.Kseg - 1) * sg.ldb + I.Nc <= src_size(sg.b_src);
        }
        if (!ok) return fail(ctx, NUC_ERR_INTERNAL, "meson GEMM item out of bounds");
    }
    std::vector<int> offs(1, 0);
    for (const GemmItem& I : items) offs.push_back(offs.back() + I.tiles_m * I.tiles_n);
    P.nitems = (int)items.size();
    P.tiles_per_tp = offs.back();
    // FP32 profile values: sink [nprof][T][N], source (t0) [nprof][N]
    std::vector<float> gs((size_t)nprof * T * N), g0((size_t)nprof * N);
    for (size_t i = 0; i < gs.size(); ++i) gs[i] = (float)gall[i];
    for (int a = 0; a < nprof; ++a)
        for (int i = 0; i < N; ++i) g0[(size_t)a * N + i] = (float)gall[((size_t)a * T + g.t0) * N + i];
    P.off_items = P.block.add(items.data(), items.size() * sizeof(GemmItem));
    P.off_offs = P.block.add(offs.data(), offs.size() * sizeof(int));
    P.off_gsnk = P.block.add(gs.data(), gs.size() * sizeof(float));
    P.off_gsrc = P.block.add(g0.data(), g0.size() * sizeof(float));
    P.block_bytes = align_up(P.block.bytes.size(), 256);
    // timeslices per round
    P.cpb = (int)((4 * N2 + TCH - 1) / TCH);
    const size_t yz_tp = 2 * (size_t)P.nop * N16 * sizeof(float2) + wsz * sizeof(float2);
    auto part_tp = [&](int nwg) { return (size_t)nwg * P.nop * P.nop * sizeof(double2); };
    for (P.Tc = T; P.Tc > 1; --P.Tc)
        if ((yz_tp + part_tp(256)) * P.Tc * nmom <= cap) break;
    P.nwg = std::max(1, std::min({256, 4 * P.cpb, 2048 / std::max(1, P.Tc * nmom)}));
    P.off_Pt = P.block_bytes;
    P.off_Ps = P.off_Pt + align_up((size_t)nmom * wsz * sizeof(float2), 256);
    P.off_Y = P.off_Ps + align_up((size_t)P.Tc * nmom * wsz * sizeof(float2), 256);
    P.off_Z = P.off_Y + align_up((size_t)P.Tc * nmom * P.nop * N16 * sizeof(float2), 256);
    P.off_part = P.off_Z + align_up((size_t)P.Tc * nmom * P.nop * N16 * sizeof(float2), 256);
    P.bytes = P.off_part + align_up(part_tp(P.nwg) * P.Tc * nmom, 256);
    return NUC_OK;
}

// ------------------------------------------------------------------ calls

struct MesonCall {
    const nuc_geom* g;
    const void* evecs;
    const void* links;
    const double* evals;
    int nprof;
    const nuc_profile* prof;
    int nmom;
    const int32_t* mom;
    const void* peramb;
    void* phi;
    void* corr;
    int stage;  // 1 elementals, 2 correlator, 3 both
};

nuc_status meson_call(nuc_ctx ctx, const MesonCall& c, hipStream_t s) {
    nuc_status st;
    if ((st = check_meson_geom(ctx, c.g)) != NUC_OK) return st;
    const nuc_geom g = *c.g;
    const bool do_elem = c.stage & 1, do_corr = (c.stage & 2) != 0;
    if (c.nmom < 1 || c.nmom > 64) return fail(ctx, NUC_ERR_INVALID, "nmom=%d out of range [1,64]", c.nmom);
    if (do_elem) {
        if (!c.evecs) return fail(ctx, NUC_ERR_INVALID, "evecs is NULL");
        if (!c.links) return fail(ctx, NUC_ERR_INVALID, "links is NULL");
        if ((st = check_moms(ctx, &g, c.nmom, c.mom)) != NUC_OK) return st;
    }
    if (!c.phi && c.stage != 3) return fail(ctx, NUC_ERR_INVALID, "phi is NULL");
    std::vector<double> gall;
    if (do_corr) {
        if (!c.peramb) return fail(ctx, NUC_ERR_INVALID, "peramb is NULL");
        if (!c.corr) return fail(ctx, NUC_ERR_INVALID, "corr is NULL");
        if ((st = check_profiles(ctx, &g, c.evals, c.nprof, c.prof)) != NUC_OK) return st;
        gall.resize((size_t)c.nprof * g.T * g.nvec);
        eval_profiles(&g, c.evals, c.nprof, c.prof, gall.data());
    }
    const size_t cap = ctx->budget ? std::min(kMesonCap, ctx->budget / 2) : kMesonCap;
    const int N = g.nvec, V3 = g.L * g.L * g.L, K = 3 * V3;
    const size_t phi_bytes = (size_t)g.T * c.nmom * kND * N * N * sizeof(float2);
    const size_t off_phase = c.phi ? 0 : align_up(phi_bytes, 256);  // internal phi first
    ElemPlan EP;
    CorrPlan CP;
    if (do_elem) EP = plan_elem(g, c.nmom, cap);
    if (do_corr && (st = plan_corr(ctx, g, c.nmom, c.nprof, gall.data(), cap, CP)) != NUC_OK) return st;
    const size_t total = off_phase + std::max(do_elem ? EP.bytes : 0, do_corr ? CP.bytes : 0);

    if ((st = begin_call(ctx, s)) != NUC_OK) return st;
    if ((st = ensure_workspace(ctx, total, s)) != NUC_OK) return st;
    char* base = (char*)ctx->ws;
    float2* phi = c.phi ? (float2*)c.phi : (float2*)base;
    char* scr = base + off_phase;

    if (do_elem) {
        HostBlock hb;
        std::vector<float2> ph((size_t)c.nmom * V3);
        for (int p = 0; p < c.nmom; ++p)
            for (int x = 0; x < V3; ++x) {
                const int x0 = x % g.L, x1 = (x / g.L) % g.L, x2 = x / (g.L * g.L);
                long long nx = (long long)c.mom[3 * p] * x0 + (long long)c.mom[3 * p + 1] * x1 +
                               (long long)c.mom[3 * p + 2] * x2;
                nx = ((nx % g.L) + g.L) % g.L;
                const double ang = -2.0 * M_PI * (double)nx / g.L;
                ph[(size_t)p * V3 + x] = make_float2((float)cos(ang), (float)sin(ang));
            }
        hb.add(ph.data(), ph.size() * sizeof(float2));
        if ((st = upload_block(ctx, hb, scr + EP.off_ph, s)) != NUC_OK) return st;
        for (int t0c = 0; t0c < g.T; t0c += EP.Tc) {
            const int Tc = std::min(EP.Tc, g.T - t0c);
            DerivArgs da;
            da.v = (const float2*)c.evecs + (size_t)t0c * N * K;
            da.U = (const float2*)c.links + (size_t)t0c * V3 * 27;
            da.F = (float2*)(scr + EP.off_F);
            da.L = g.L;
            da.V3 = V3;
            da.N = N;
            da.Tc = Tc;
            da.jchunk = 8;
            da.Kp = EP.Kp;
            HIPCHK(ctx, timed_launch(ctx, NUC_K_MESON_DERIV, s, [&] {
                       return launch_deriv(0, da, s);
                   }));
            HIPCHK(ctx, timed_launch(ctx, NUC_K_MESON_DERIV, s, [&] {
                       return launch_deriv(1, da, s);
                   }));
            PhaseArgs pa;
            pa.v = da.v;
            pa.ph = (const float2*)(scr + EP.off_ph);
            pa.A = (float2*)(scr + EP.off_A);
            pa.V = (float2*)(scr + EP.off_V);
            pa.N = N;
            pa.K = K;
            pa.Kp = EP.Kp;
            pa.nmom = c.nmom;
            pa.Tc = Tc;
            HIPCHK(ctx, timed_launch(ctx, NUC_K_MESON_PHASE, s, [&] {
                       return launch_phase(pa, s);
                   }));
            ElemArgs ea;
            ea.A = pa.A;
            ea.V = pa.V;
            ea.F = da.F;
            ea.part = (double2*)(scr + EP.off_part);
            ea.N = N;
            ea.K = K;
            ea.Kp = EP.Kp;
            ea.nmom = c.nmom;
            ea.Tc = Tc;
            ea.nsplit = EP.nsplit;
            ea.cps = EP.cps;
            ea.nchunks = EP.nchunks;
            ea.mt = EP.mt;
            ea.nt = EP.nt;
            HIPCHK(ctx, timed_launch(ctx, NUC_K_MESON_ELEM, s, [&] {
                       return launch_elem(ea, s);
                   }));
            ElemReduceArgs ra;
            ra.part = ea.part;
            ra.phi = phi;
            ra.N = N;
            ra.nmom = c.nmom;
            ra.Tc = Tc;
            ra.nsplit = EP.nsplit;
            ra.t_off = t0c;
            HIPCHK(ctx, timed_launch(ctx, NUC_K_MESON_ELEM_REDUCE, s, [&] {
                       return launch_elem_reduce(ra, s);
                   }));
        }
    }
    if (do_corr) {
        if ((st = upload_block(ctx, CP.block, scr, s)) != NUC_OK) return st;
        const size_t wsz = (size_t)kND * c.nprof * N * N;
        WeightArgs wa;
        wa.phi = phi;
        wa.N = N;
        wa.T = g.T;
        wa.nmom = c.nmom;
        wa.nprof = c.nprof;
        wa.t0 = g.t0;
        {  // source elementals, once per call
            wa.out = (float2*)(scr + CP.off_Pt);
            wa.g = (const float*)(scr + CP.off_gsrc);
            wa.t_off = 0;
            wa.Tc = 1;
            wa.mode = 1;
            const size_t nel = (size_t)c.nmom * wsz;
            HIPCHK(ctx, timed_launch(ctx, NUC_K_MESON_WEIGHT, s, [&] {
                       return launch_weight(wa, nel, s);
                   }));
        }
        for (int t0c = 0; t0c < g.T; t0c += CP.Tc) {
            const int Tc = std::min(CP.Tc, g.T - t0c);
            wa.out = (float2*)(scr + CP.off_Ps);
            wa.g = (const float*)(scr + CP.off_gsnk);
            wa.t_off = t0c;
            wa.Tc = Tc;
            wa.mode = 0;
            const size_t nel = (size_t)Tc * c.nmom * wsz;
            HIPCHK(ctx, timed_launch(ctx, NUC_K_MESON_WEIGHT, s, [&] {
                       return launch_weight(wa, nel, s);
                   }));
            GemmArgs ga;
            ga.items = (const GemmItem*)(scr + CP.off_items);
            ga.offs = (const int*)(scr + CP.off_offs);
            ga.nitems = CP.nitems;
            ga.tiles_per_tp = CP.tiles_per_tp;
            ga.Ps = (const float2*)(scr + CP.off_Ps);
            ga.Pt = (const float2*)(scr + CP.off_Pt);
            ga.tau = (const float2*)c.peramb;
            ga.Y = (float2*)(scr + CP.off_Y);
            ga.Z = (float2*)(scr + CP.off_Z);
            ga.N = N;
            ga.nmom = c.nmom;
            ga.nprof = c.nprof;
            ga.nop = CP.nop;
            ga.t_off = t0c;
            const unsigned nblk = (unsigned)CP.tiles_per_tp * Tc * c.nmom;
            HIPCHK(ctx, timed_launch(ctx, NUC_K_MESON_GEMM, s, [&] {
                       return launch_gemm(ga, nblk, s);
                   }));
            TraceArgs ta;
            ta.Y = ga.Y;
            ta.Z = ga.Z;
            ta.part = (double2*)(scr + CP.off_part);
            ta.N = N;
            ta.nop = CP.nop;
            ta.nmom = c.nmom;
            ta.nwg = CP.nwg;
            ta.cpb = CP.cpb;
            for (int gm = 0; gm < 4; ++gm) {
                ta.pi5[gm] = CP.pi5[gm];
                ta.s5[gm] = CP.s5[gm];
            }
            HIPCHK(ctx, timed_launch(ctx, NUC_K_MESON_TRACE, s, [&] {
                       return launch_trace(ta, Tc * c.nmom, s);
                   }));
            SumArgs sa;
            sa.part = ta.part;
            sa.corr = (double2*)c.corr;
            sa.T = g.T;
            sa.nop = CP.nop;
            sa.nmom = c.nmom;
            sa.nwg = CP.nwg;
            sa.Tc = Tc;
            sa.t_off = t0c;
            const int nsum = Tc * c.nmom * CP.nop * CP.nop;
            HIPCHK(ctx, timed_launch(ctx, NUC_K_MESON_SUM, s, [&] {
                       return launch_sum(sa, nsum, s);
                   }));
        }
    }
    return end_call(ctx, s);
}

nuc_status meson_entry(nuc_ctx ctx, const MesonCall& c, void* stream) {
    if (!ctx) return fail(nullptr, NUC_ERR_INVALID, "ctx is NULL");
    std::lock_guard<std::mutex> lock(ctx->mu);
    DeviceGuard guard;
    return meson_call(ctx, c, (hipStream_t)stream);
}

}  // namespace meson
}  // namespace nuc

using nuc::meson::MesonCall;

extern "C" {

nuc_status nuc_meson_elementals(nuc_ctx ctx, const nuc_geom* geom, const void* evecs, const void* links, int nmom,
                                const int32_t* mom, void* phi, void* stream) {
    MesonCall c{geom, evecs, links, nullptr, 0, nullptr, nmom, mom, nullptr, phi, nullptr, 1};
    return nuc::meson::meson_entry(ctx, c, stream);
}

nuc_status nuc_meson_correlator(nuc_ctx ctx, const nuc_geom* geom, const void* phi, const double* evals, int nprof,
                                const nuc_profile* prof, int nmom, const void* peramb, void* corr, void* stream) {
    MesonCall c{geom, nullptr, nullptr, evals, nprof, prof, nmom, nullptr, peramb, (void*)phi, corr, 2};
    return nuc::meson::meson_entry(ctx, c, stream);
}

nuc_status nuc_meson_run(nuc_ctx ctx, const nuc_geom* geom, const void* evecs, const void* links,
                         const double* evals, int nprof, const nuc_profile* prof, int nmom, const int32_t* mom,
                         const void* peramb, void* phi, void* corr, void* stream) {
    MesonCall c{geom, evecs, links, evals, nprof, prof, nmom, mom, peramb, phi, corr, 3};
    return nuc::meson::meson_entry(ctx, c, stream);
}

}  // extern "C"

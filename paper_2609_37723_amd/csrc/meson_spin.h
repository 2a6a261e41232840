// Host-side spin algebra of the meson operator families (Section 3, charmonium
// operators): Euclidean Dirac-Pauli gamma matrices, their signed-permutation form and the
// (Gamma, D) terms of the three families g4 g5; g4 g5 g_k nabla_k; g_k B_k. Shared by the
// single-meson and two-meson host runtimes.
#pragma once

#include <complex>
#include <vector>

#include "../../include/nucleon.h"
#include "meson_internal.h"

namespace nuc {
namespace meson {

typedef std::complex<double> cd;

struct Mat4 {
    cd m[4][4];
};

inline Mat4 mul(const Mat4& x, const Mat4& y) {
    Mat4 r{};
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
            for (int k = 0; k < 4; ++k) r.m[i][j] += x.m[i][k] * y.m[k][j];
    return r;
}

// Euclidean Dirac-Pauli matrices: gamma_k = [[0, -i sigma_k], [i sigma_k, 0]],
// gamma_4 = diag(1, 1, -1, -1), gamma_5 = g1 g2 g3 g4.
struct Gammas {
    Mat4 g[3], g4, g5;
};

inline Gammas dirac_pauli() {
    const cd I(0.0, 1.0);
    const cd sig[3][2][2] = {{{0.0, 1.0}, {1.0, 0.0}}, {{0.0, -I}, {I, 0.0}}, {{1.0, 0.0}, {0.0, -1.0}}};
    Gammas G{};
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                G.g[k].m[a][2 + b] = -I * sig[k][a][b];
                G.g[k].m[2 + a][b] = I * sig[k][a][b];
            }
    for (int a = 0; a < 4; ++a) G.g4.m[a][a] = a < 2 ? 1.0 : -1.0;
    G.g5 = mul(mul(mul(G.g[0], G.g[1]), G.g[2]), G.g4);
    return G;
}

// A matrix with exactly one nonzero per row and per column: col[r] and val[r] of row r.
struct Perm {
    int col[4];
    cd val[4];
    int row_of_col[4];
};

inline bool as_perm(const Mat4& x, Perm& p) {
    int cnt_col[4] = {0, 0, 0, 0};
    for (int r = 0; r < 4; ++r) {
        int n = 0;
        for (int c = 0; c < 4; ++c)
            if (std::abs(x.m[r][c]) > 1e-12) {
                p.col[r] = c;
                p.val[r] = x.m[r][c];
                p.row_of_col[c] = r;
                ++n;
                ++cnt_col[c];
            }
        if (n != 1) return false;
    }
    for (int c = 0; c < 4; ++c)
        if (cnt_col[c] != 1) return false;
    return true;
}

struct Term {
    Perm G;
    int D;
};

// The three operator families: (Gamma, D) terms.
inline bool operator_terms(std::vector<std::vector<Term>>& fam, Perm& g5p, double g4d[4]) {
    const Gammas G = dirac_pauli();
    const Mat4 g45 = mul(G.g4, G.g5);
    fam.assign(kNFam, {});
    Term t;
    if (!as_perm(g45, t.G)) return false;
    t.D = 0;
    fam[0].push_back(t);
    for (int k = 0; k < 3; ++k) {
        if (!as_perm(mul(g45, G.g[k]), t.G)) return false;
        t.D = 1 + k;
        fam[1].push_back(t);
    }
    for (int k = 0; k < 3; ++k) {
        if (!as_perm(G.g[k], t.G)) return false;
        t.D = 4 + k;
        fam[2].push_back(t);
    }
    if (!as_perm(G.g5, g5p)) return false;
    for (int a = 0; a < 4; ++a) g4d[a] = G.g4.m[a][a].real();
    return true;
}

// Range checks of the geometry for meson operators (nvec <= 512); defined in meson.hip.
nuc_status check_meson_geom(nuc_ctx ctx, const nuc_geom* g);

}  // namespace meson
}  // namespace nuc

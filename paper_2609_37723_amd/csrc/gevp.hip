// Host FP64 analysis of the correlation matrix (paper Section 2.1): the
// generalised eigenvalue problem C(t) v = lambda C(t0) v, whose eigenvectors
// combine the profiled operators into optimised ones and whose eigenvalues give
// effective masses; and (Section 3) the pruning of a large correlation matrix to
// the leading singular vectors of C(t_p) before the GEVP. The matrices are at
// most 64 x 64: plain loops in FP64.
//
// Method: Hermitise H(t) = (C(t) + C(t)^H) / 2; Cholesky H(t0) = L L^H;
// A(t) = L^-1 H(t) L^-H is Hermitian with the same eigenvalues; diagonalise it by
// cyclic complex Jacobi rotations; v = L^-H u, so that v^H H(t0) v = 1.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <complex>
#include <vector>

#include "../../include/nucleon.h"

namespace {

typedef std::complex<double> cplx;

struct Mat {
    int n;
    std::vector<cplx> a;
    explicit Mat(int n_) : n(n_), a((size_t)n_ * n_) {}
    cplx& operator()(int i, int j) { return a[(size_t)i * n + j]; }
    cplx operator()(int i, int j) const { return a[(size_t)i * n + j]; }
};

// Lower Cholesky factor of a Hermitian matrix; false if not positive definite.
bool cholesky(const Mat& h, Mat& l) {
    const int n = h.n;
    for (int j = 0; j < n; ++j) {
        double d = h(j, j).real();
        for (int k = 0; k < j; ++k) d -= std::norm(l(j, k));
        if (!(d > 0.0)) return false;
        const double ljj = sqrt(d);
        l(j, j) = ljj;
        for (int i = j + 1; i < n; ++i) {
            cplx s = h(i, j);
            for (int k = 0; k < j; ++k) s -= l(i, k) * std::conj(l(j, k));
            l(i, j) = s / ljj;
        }
        for (int i = 0; i < j; ++i) l(i, j) = 0.0;
    }
    return true;
}

// X = L^-1 B (forward substitution, column by column)
Mat solve_lower(const Mat& l, const Mat& b) {
    const int n = l.n;
    Mat x(n);
    for (int c = 0; c < n; ++c)
        for (int i = 0; i < n; ++i) {
            cplx s = b(i, c);
            for (int k = 0; k < i; ++k) s -= l(i, k) * x(k, c);
            x(i, c) = s / l(i, i);
        }
    return x;
}

// X = L^-H B (back substitution with the conjugate transpose of L)
Mat solve_lower_h(const Mat& l, const Mat& b) {
    const int n = l.n;
    Mat x(n);
    for (int c = 0; c < n; ++c)
        for (int i = n - 1; i >= 0; --i) {
            cplx s = b(i, c);
            for (int k = i + 1; k < n; ++k) s -= std::conj(l(k, i)) * x(k, c);
            x(i, c) = s / l(i, i);
        }
    return x;
}

Mat adjoint(const Mat& m) {
    Mat r(m.n);
    for (int i = 0; i < m.n; ++i)
        for (int j = 0; j < m.n; ++j) r(i, j) = std::conj(m(j, i));
    return r;
}

// Cyclic Jacobi for a Hermitian matrix: a is overwritten (diagonal = eigenvalues),
// u accumulates the rotations (columns = eigenvectors).
void jacobi(Mat& a, Mat& u) {
    const int n = a.n;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) u(i, j) = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += std::norm(a(i, j));
                if (i != j) off += std::norm(a(i, j));
            }
        if (off <= 1e-32 * tot || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const cplx apq = a(p, q);
                const double mag = std::abs(apq);
                if (mag == 0.0) continue;
                // A_pq = |A_pq| e^{i phi}: rotate in the plane (p, q) with the real
                // Jacobi angle of [[a_pp, |a_pq|], [|a_pq|, a_qq]] and the phase e^{i phi}
                const cplx ph = apq / mag;
                const double app = a(p, p).real(), aqq = a(q, q).real();
                const double theta = 0.5 * atan2(2.0 * mag, aqq - app);
                const double c = cos(theta), s = sin(theta);
                // columns: p' = c p - s conj(ph) q... use G with G_pp = c, G_pq = s ph,
                // G_qp = -s conj(ph), G_qq = c;  A <- G^H A G, U <- U G
                for (int k = 0; k < n; ++k) {  // A G
                    const cplx akp = a(k, p), akq = a(k, q);
                    a(k, p) = c * akp - s * std::conj(ph) * akq;
                    a(k, q) = s * ph * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // G^H (A G)
                    const cplx apk = a(p, k), aqk = a(q, k);
                    a(p, k) = c * apk - s * ph * aqk;
                    a(q, k) = s * std::conj(ph) * apk + c * aqk;
                }
                a(p, q) = 0.0;
                a(q, p) = 0.0;
                for (int k = 0; k < n; ++k) {
                    const cplx ukp = u(k, p), ukq = u(k, q);
                    u(k, p) = c * ukp - s * std::conj(ph) * ukq;
                    u(k, q) = s * ph * ukp + c * ukq;
                }
            }
    }
}

}  // namespace

extern "C" {

nuc_status nuc_gevp(const void* corr, int T, int nb, int t0, double* lambda_out, void* vecs_out) {
    if (!corr || !lambda_out) return NUC_ERR_INVALID;
    if (T < 1 || nb < 1 || nb > 64 || t0 < 0 || t0 >= T) return NUC_ERR_INVALID;
    const cplx* c = (const cplx*)corr;
    auto herm = [&](int t) {
        Mat h(nb);
        for (int i = 0; i < nb; ++i)
            for (int j = 0; j < nb; ++j)
                h(i, j) = 0.5 * (c[((size_t)t * nb + i) * nb + j] + std::conj(c[((size_t)t * nb + j) * nb + i]));
        return h;
    };
    Mat l(nb);
    if (!cholesky(herm(t0), l)) return NUC_ERR_INVALID;
    for (int t = 0; t < T; ++t) {
        Mat a = solve_lower(l, adjoint(solve_lower(l, herm(t))));  // L^-1 (L^-1 H)^H = L^-1 H L^-H
        for (int i = 0; i < nb; ++i)  // exact Hermitian symmetry before the rotations
            for (int j = i; j < nb; ++j) {
                const cplx m = 0.5 * (a(i, j) + std::conj(a(j, i)));
                a(i, j) = m;
                a(j, i) = std::conj(m);
            }
        Mat u(nb);
        jacobi(a, u);
        std::vector<int> order(nb);
        for (int i = 0; i < nb; ++i) order[i] = i;
        std::sort(order.begin(), order.end(), [&](int x, int y) { return a(x, x).real() > a(y, y).real(); });
        for (int n = 0; n < nb; ++n) lambda_out[(size_t)t * nb + n] = a(order[n], order[n]).real();
        if (vecs_out) {
            Mat v = solve_lower_h(l, u);
            cplx* out = (cplx*)vecs_out + (size_t)t * nb * nb;
            for (int i = 0; i < nb; ++i)
                for (int n = 0; n < nb; ++n) out[(size_t)i * nb + n] = v(i, order[n]);
        }
    }
    return NUC_OK;
}

nuc_status nuc_svd_prune(const void* corr, int T, int n, int t_p, int m, void* out, void* basis) {
    if (!corr || !out) return NUC_ERR_INVALID;
    if (T < 1 || n < 1 || n > 64 || m < 1 || m > n || t_p < 0 || t_p >= T) return NUC_ERR_INVALID;
    const cplx* c = (const cplx*)corr;
    // left singular vectors of C(t_p) = eigenvectors of the Hermitian C C^H
    Mat h(n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            cplx s = 0.0;
            for (int k = 0; k < n; ++k) s += c[((size_t)t_p * n + i) * n + k] * std::conj(c[((size_t)t_p * n + j) * n + k]);
            h(i, j) = s;
        }
    for (int i = 0; i < n; ++i)
        for (int j = i; j < n; ++j) {
            const cplx v = 0.5 * (h(i, j) + std::conj(h(j, i)));
            h(i, j) = v;
            h(j, i) = std::conj(v);
        }
    Mat u(n);
    jacobi(h, u);
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return h(x, x).real() > h(y, y).real(); });
    std::vector<cplx> um((size_t)n * m);
    for (int q = 0; q < m; ++q) {
        const int col = order[q];
        int best = 0;
        for (int i = 1; i < n; ++i)
            if (std::abs(u(i, col)) > std::abs(u(best, col))) best = i;
        const cplx ph = std::abs(u(best, col)) > 0.0 ? std::conj(u(best, col)) / std::abs(u(best, col)) : 1.0;
        for (int i = 0; i < n; ++i) um[(size_t)i * m + q] = u(i, col) * ph;
    }
    cplx* o = (cplx*)out;
    for (int t = 0; t < T; ++t)
        for (int a = 0; a < m; ++a)
            for (int b = 0; b < m; ++b) {
                cplx s = 0.0;
                for (int i = 0; i < n; ++i) {
                    cplx r = 0.0;
                    for (int j = 0; j < n; ++j) r += c[((size_t)t * n + i) * n + j] * um[(size_t)j * m + b];
                    s += std::conj(um[(size_t)i * m + a]) * r;
                }
                o[((size_t)t * m + a) * m + b] = s;
            }
    if (basis) memcpy(basis, um.data(), um.size() * sizeof(cplx));
    return NUC_OK;
}

nuc_status nuc_effective_mass(const double* lambda, int T, int nb, double* meff_out) {
    if (!lambda || !meff_out || T < 2 || nb < 1) return NUC_ERR_INVALID;
    for (int t = 0; t + 1 < T; ++t)
        for (int n = 0; n < nb; ++n) {
            const double a = lambda[(size_t)t * nb + n], b = lambda[(size_t)(t + 1) * nb + n];
            meff_out[(size_t)t * nb + n] = (a > 0.0 && b > 0.0) ? log(a / b) : NAN;
        }
    return NUC_OK;
}

}  // extern "C"

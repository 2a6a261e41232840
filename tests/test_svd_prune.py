"""Host FP64 pruning of a correlation matrix to the leading left singular vectors of
C(t_p) (library nuc_svd_prune), against the oracle's numpy-SVD version and pinned
to what the singular value decomposition fixes: the basis solves
C(t_p) C(t_p)^H u_n = s_n^2 u_n with the m largest s_n, it is orthonormal, a
Hermitian positive C(t_p) becomes diagonal with its leading eigenvalues, and at
m = n the projection is a unitary similarity that keeps the GEVP spectrum."""
import numpy as np
import pytest

import oracle
import oracle.meson as om
import paper_2609_37723_amd as nuc


def _phase_fix(u):
    """Scale every column so its largest-modulus component is real positive."""
    idx = np.argmax(np.abs(u), axis=0)
    ph = np.conj(u[idx, np.arange(u.shape[1])])
    return u * (ph / np.abs(ph))[None, :]


def _random_corr(T, n, seed, hermitian=True):
    g = np.random.default_rng(seed)
    a = g.standard_normal((T, n, n)) + 1j * g.standard_normal((T, n, n))
    if hermitian:
        return a @ np.conj(np.swapaxes(a, 1, 2))
    return a


@pytest.mark.parametrize("hermitian", [True, False])
def test_library_matches_oracle(hermitian):
    T, n, m, tp = 5, 21, 8, 2
    c = _random_corr(T, n, 11, hermitian)
    cp, basis = nuc.svd_prune(c, tp, m)
    cp_o, u_o = om.svd_prune(c, tp, m)
    u_o = _phase_fix(u_o)
    np.testing.assert_allclose(basis, u_o, atol=1e-10)
    cp_o = np.einsum("in,tij,jm->tnm", u_o.conj(), c, u_o)
    np.testing.assert_allclose(cp, cp_o, atol=1e-10 * np.max(np.abs(c)))


def test_basis_solves_the_singular_vector_problem():
    T, n, m, tp = 3, 12, 5, 1
    c = _random_corr(T, n, 5, hermitian=False)
    _, u = nuc.svd_prune(c, tp, m)
    s = np.linalg.svd(c[tp], compute_uv=False)
    h = c[tp] @ c[tp].conj().T
    np.testing.assert_allclose(u.conj().T @ u, np.eye(m), atol=1e-12)
    np.testing.assert_allclose(h @ u, u * s[:m] ** 2, atol=1e-10 * s[0] ** 2)


def test_hermitian_psd_becomes_diagonal_at_tp():
    T, n, m, tp = 4, 9, 5, 2
    c = _random_corr(T, n, 4)
    cp, _ = nuc.svd_prune(c, tp, m)
    w = np.sort(np.linalg.eigvalsh(c[tp]))[::-1][:m]
    np.testing.assert_allclose(cp[tp], np.diag(w), atol=1e-10 * w[0])


def test_full_rank_keeps_gevp_spectrum():
    T, n = 6, 7
    c = _random_corr(T, n, 8)
    cp, _ = nuc.svd_prune(c, 3, n)
    np.testing.assert_allclose(nuc.gevp(cp, 0)[0], oracle.gevp(c, 0)[0], rtol=1e-9)


def test_rejects_bad_arguments():
    c = _random_corr(2, 4, 1)
    with pytest.raises(nuc.NucError):
        nuc.svd_prune(c, 2, 2)           # t_p out of range
    with pytest.raises(nuc.NucError):
        nuc.svd_prune(c, 0, 5)           # m > n
    lib = nuc.load()
    assert lib.nuc_svd_prune(None, 2, 4, 0, 2, None, None) == nuc.NUC_ERR_INVALID

"""Host FP64 GEVP of the correlation matrix and effective masses (library
nuc_gevp / nuc_effective_mass against the oracle's scipy-based version), both
pinned to the closed form of a matrix with a known spectrum:
C(t) = Z diag(exp(-E_n t)) Z^H has GEVP eigenvalues exp(-E_n (t - t0)) and
effective masses E_n."""
import numpy as np
import pytest

import oracle
import paper_2609_37723_amd as nuc

E = np.array([0.3, 0.5, 0.8, 1.1, 1.6])


def _spectral(T, seed=3, energies=E):
    g = np.random.default_rng(seed)
    nb = len(energies)
    z = g.standard_normal((nb, nb)) + 1j * g.standard_normal((nb, nb))
    c = np.stack([z @ np.diag(np.exp(-energies * t)) @ z.conj().T for t in range(T)])
    return c, z


def _closed_form(T, t0, energies=E):
    lam = np.exp(-np.outer(np.arange(T) - t0, energies))
    return -np.sort(-lam, axis=1)


@pytest.mark.parametrize("impl", ["library", "oracle"])
@pytest.mark.parametrize("t0", [0, 2])
def test_gevp_eigenvalues_closed_form(impl, t0):
    T = 9
    c, _ = _spectral(T)
    lam, vecs = (nuc.gevp(c, t0) if impl == "library" else oracle.gevp(c, t0))
    np.testing.assert_allclose(lam, _closed_form(T, t0), rtol=1e-10, atol=1e-13)


@pytest.mark.parametrize("impl", ["library", "oracle"])
def test_effective_mass_closed_form(impl):
    T, t0 = 10, 1
    c, _ = _spectral(T)
    lam, _ = (nuc.gevp(c, t0) if impl == "library" else oracle.gevp(c, t0))
    m = nuc.effective_mass(lam) if impl == "library" else oracle.effective_mass(lam)
    # from t0 on the order is by increasing energy and each mass is exact
    np.testing.assert_allclose(m[t0:], np.tile(E, (T - 1 - t0, 1)), rtol=1e-9)


def test_gevp_vectors_solve_the_problem():
    T, t0 = 7, 1
    g = np.random.default_rng(9)
    nb = 6
    a = g.standard_normal((T, nb, nb)) + 1j * g.standard_normal((T, nb, nb))
    c = a @ np.conj(np.swapaxes(a, 1, 2)) + 0.1 * (g.standard_normal((T, nb, nb)))  # not Hermitian
    lam, v = nuc.gevp(c, t0)
    h = 0.5 * (c + np.conj(np.swapaxes(c, 1, 2)))
    for t in range(T):
        res = h[t] @ v[t] - h[t0] @ v[t] @ np.diag(lam[t])
        assert np.max(np.abs(res)) <= 1e-10 * np.max(np.abs(h[t]))
        np.testing.assert_allclose(np.conj(v[t]).T @ h[t0] @ v[t], np.eye(nb), atol=1e-10)
    lam_o, _ = oracle.gevp(c, t0)
    np.testing.assert_allclose(lam, lam_o, rtol=1e-10, atol=1e-12)


def test_gevp_rejects_bad_input():
    c, _ = _spectral(4)
    bad = c.copy()
    bad[0] = -bad[0]                         # C(t0) negative definite
    with pytest.raises(nuc.NucError) as e:
        nuc.gevp(bad, 0)
    assert e.value.status == nuc.NUC_ERR_INVALID
    with pytest.raises(nuc.NucError):
        nuc.gevp(c, 7)                       # t0 out of range
    lib = nuc.load()
    assert lib.nuc_gevp(None, 4, 5, 0, None, None) == nuc.NUC_ERR_INVALID
    assert lib.nuc_effective_mass(None, 4, 5, None) == nuc.NUC_ERR_INVALID


def test_one_operator_reduces_to_the_correlator_ratio():
    # N_B = 1: lambda(t) = C(t) / C(t0) (real part of the Hermitised 1x1 matrix)
    c = np.array([[[2.0 + 0.5j]], [[1.0 - 0.2j]], [[0.4 + 0.1j]]])
    lam, v = nuc.gevp(c, 0)
    np.testing.assert_allclose(lam[:, 0], c.real[:, 0, 0] / c.real[0, 0, 0], rtol=1e-14)
    np.testing.assert_allclose(np.abs(v[:, 0, 0]), 1 / np.sqrt(2.0), rtol=1e-14)


@pytest.mark.gpu
def test_gevp_of_gpu_correlator_matches_oracle():
    """C_ab(t) from the GPU (tau = identity at t = t0 gives a positive definite C(t0)),
    analysed by the library's GEVP, against the oracle's GEVP of the oracle's C."""
    from tests.gpu_util import TOL_FP32, announce, to_dev, torch_cuda
    import synth
    torch = torch_cuda()
    cfg = synth.custom("gevp", 4, 4, 16, [(0, 0, 0)], [(0, 0.2), (0, 0.5), (0, 1.0), (1, 0.0)], "gauss_decay",
                       cfg_id=31)
    inp = synth.make_inputs(cfg)
    inp.tau[0] = np.eye(4 * cfg.nvec)
    corr = nuc.run(to_dev(torch, inp.evecs, np.complex64), inp.evals, cfg.profiles, inp.mom,
                   to_dev(torch, inp.tau, np.complex64), cfg.L)
    torch.cuda.synchronize()
    c_gpu = corr.cpu().numpy()[0]
    _, c_ref = oracle.run(cfg.L, inp.evecs, inp.evals, inp.tau, inp.mom, cfg.profiles)
    lam, _ = nuc.gevp(c_gpu, 0)
    lam_ref, _ = oracle.gevp(c_ref[0], 0)
    # first-order perturbation: |d lambda| <~ cond(C(t0)) |dC| / |C| max |lambda(t)|; C
    # carries at most the FP32 gate's relative error
    err = np.max(np.abs(lam - lam_ref) / np.max(np.abs(lam_ref), axis=1, keepdims=True))
    cond = np.linalg.cond(0.5 * (c_ref[0][0] + c_ref[0][0].conj().T))
    announce("gevp of the GPU correlator: max eigenvalue diff %.3e of max |lambda|, cond(C(t0)) %.3g" % (err, cond))
    assert err <= cond * TOL_FP32

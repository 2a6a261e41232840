"""Pins of the FP64 meson oracle (oracle/meson.py): closed forms and invariants of
the covariant derivatives, the meson elementals and the 21 x 21-type correlation
matrix, none of which re-types the oracle's formulas."""
import numpy as np
import pytest

import oracle.meson as om
import synth


def _cfg(L=3, T=2, N=6, mom=((0, 0, 0), (1, 0, 0)), prof=((0, 0.3), (0, 0.8)), kind="gauss", cid=50):
    return synth.custom("m", L, T, N, list(mom), list(prof), kind, cfg_id=cid)


def _fp64_inputs(cfg, seed=1):
    """FP64 (not c64-rounded) orthonormal vectors and SU(3) links, for exact invariances."""
    g = np.random.default_rng(seed)
    ev = np.empty((cfg.T, cfg.nvec, cfg.V3, 3), complex)
    for t in range(cfg.T):
        m = g.standard_normal((cfg.nvec, 3 * cfg.V3)) + 1j * g.standard_normal((cfg.nvec, 3 * cfg.V3))
        ev[t] = synth.orthonormalise(m).reshape(cfg.nvec, cfg.V3, 3)
    U = np.stack([synth.random_su3(g, cfg.V3 * 3).reshape(cfg.V3, 3, 3, 3) for _ in range(cfg.T)])
    return ev, U


def _gauge_transform(L, ev, U, seed=7):
    g = np.random.default_rng(seed)
    T, V3 = U.shape[0], U.shape[1]
    ev2, U2 = np.empty_like(ev), np.empty_like(U)
    for t in range(T):
        om_ = synth.random_su3(g, V3)  # Omega(x)
        ev2[t] = np.einsum("xab,nxb->nxa", om_, ev[t])
        for d in range(3):
            fwd = om.neighbours(L, d, +1)
            U2[t, :, d] = om_ @ U[t, :, d] @ np.conj(np.swapaxes(om_[fwd], 1, 2))
    return ev2, U2


def test_identity_elemental_at_zero_momentum_is_unit_matrix():
    cfg = _cfg()
    ev, U = _fp64_inputs(cfg)
    phi = om.elementals(cfg.L, ev, U, np.zeros((1, 3)))
    for t in range(cfg.T):
        np.testing.assert_allclose(phi[t, 0, 0], np.eye(cfg.nvec), atol=1e-13)


def test_elementals_are_gauge_invariant():
    cfg = _cfg()
    ev, U = _fp64_inputs(cfg)
    ev2, U2 = _gauge_transform(cfg.L, ev, U)
    mom = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 1]])
    a, b = om.elementals(cfg.L, ev, U, mom), om.elementals(cfg.L, ev2, U2, mom)
    assert np.max(np.abs(a[:, :, 1:])) > 0.05          # the derivative terms are not trivially zero
    np.testing.assert_allclose(a, b, atol=1e-12)


def test_derivative_elementals_antihermitian_at_zero_momentum():
    cfg = _cfg()
    ev, U = _fp64_inputs(cfg)
    phi = om.elementals(cfg.L, ev, U, np.zeros((1, 3)))
    for d in range(1, 7):                                  # nabla_k and B_k are anti-Hermitian
        m = phi[0, 0, d]
        np.testing.assert_allclose(m, -m.conj().T, atol=1e-12)


def test_trivial_links_plane_waves_closed_form():
    # U = 1 and v_j(x) = exp(2 pi i k_j.x / L) e_{c_j} / sqrt(V3): nabla_d v_j = i sin(2 pi k_{j,d} / L) v_j,
    # Phi^1_ij(p) = [c_i = c_j] [k_j - k_i = p mod L], and B v = 0 (derivatives commute)
    L, T = 4, 1
    cfg = _cfg(L=L, T=T, N=6)
    ks = [(0, 0, 0), (1, 0, 0), (0, 2, 1), (1, 0, 0), (3, 1, 0), (2, 2, 2)]
    cs = [0, 0, 1, 2, 1, 0]
    x = np.arange(L ** 3)
    xc = np.stack([x % L, (x // L) % L, x // (L * L)], axis=1)
    ev = np.zeros((T, 6, L ** 3, 3), complex)
    for j, (k, c) in enumerate(zip(ks, cs)):
        ev[0, j, :, c] = np.exp(2j * np.pi * (xc @ np.array(k)) / L) / np.sqrt(L ** 3)
    U = np.zeros((T, L ** 3, 3, 3, 3), complex)
    U[..., :, :] = np.eye(3)
    mom = np.array([[0, 0, 0], [1, 0, 0], [3, 2, 1]])
    phi = om.elementals(L, ev, U, mom)
    for p, pv in enumerate(mom):
        base = np.array([[float(cs[i] == cs[j] and np.all((np.array(ks[j]) - np.array(ks[i]) - pv) % L == 0))
                          for j in range(6)] for i in range(6)])
        np.testing.assert_allclose(phi[0, p, 0], base, atol=1e-13)
        for d in range(3):
            lam = 1j * np.sin(2 * np.pi * np.array([k[d] for k in ks]) / L)
            np.testing.assert_allclose(phi[0, p, 1 + d], base * lam[None, :], atol=1e-13)
        np.testing.assert_allclose(phi[0, p, 4:], 0, atol=1e-13)


def test_field_strength_elementals_vanish_for_trivial_links_any_vectors():
    cfg = _cfg()
    ev, _ = _fp64_inputs(cfg)
    U = np.zeros((cfg.T, cfg.V3, 3, 3, 3), complex)
    U[..., :, :] = np.eye(3)
    phi = om.elementals(cfg.L, ev, U, np.array([[0, 0, 0], [1, 1, 0]]))
    np.testing.assert_allclose(phi[:, :, 4:], 0, atol=1e-13)
    assert np.max(np.abs(phi[:, :, 1:4])) > 0.05


def _corr_inputs(cfg, tau_kind="gauss", seed=1):
    ev, U = _fp64_inputs(cfg, seed)
    g = np.random.default_rng(seed + 100)
    n4 = 4 * cfg.nvec
    if tau_kind == "identity":
        tau = np.stack([np.eye(n4, dtype=complex)] * cfg.T)
    else:
        tau = (g.standard_normal((cfg.T, n4, n4)) + 1j * g.standard_normal((cfg.T, n4, n4))) / np.sqrt(2)
    evals = np.sort(g.random((cfg.T, cfg.nvec)), axis=1)
    return ev, U, evals, tau


def test_correlator_closed_form_gamma4gamma5_identity_tau():
    # tau = 1, t = t0, p = 0, family 0 (Gamma = g4 g5, D = 1): Phi^1 = 1, so
    # C_ab = -Tr[g4g5 g4 (g4g5)^H g4] sum_i g_a,i^2 g_b,i^2 (the minus from the quark
    # loop), and g4 g5 g4 = -g5 makes the spin trace Tr[-1_4] = -4: C_ab = +4 sum g^2 g^2,
    # positive as the two-point function of an operator with itself
    cfg = _cfg(T=1, N=5, mom=((0, 0, 0),), prof=((0, 0.3), (0, 0.6), (1, 0.0)))
    ev, U, evals, tau = _corr_inputs(cfg, "identity")
    import oracle
    _, C = om.run(cfg.L, ev, U, evals, tau, np.zeros((1, 3)), cfg.profiles)
    g = oracle.profiles(evals, cfg.profiles)[:, 0, :]
    nb = len(cfg.profiles)
    expect = 4.0 * (g ** 2) @ (g ** 2).T
    np.testing.assert_allclose(C[0, 0, :nb, :nb], expect, atol=1e-12)


def test_correlator_hermitian_for_identity_tau_at_source_time():
    cfg = _cfg(T=1, N=5)
    ev, U, evals, tau = _corr_inputs(cfg, "identity")
    _, C = om.run(cfg.L, ev, U, evals, tau, np.array([[0, 0, 0], [1, 0, 0]]), cfg.profiles)
    for p in range(2):
        np.testing.assert_allclose(C[p, 0], C[p, 0].conj().T, atol=1e-12)
        assert np.max(np.abs(C[p, 0])) > 1e-3


def test_correlator_gauge_invariant_and_quadratic_in_tau():
    cfg = _cfg(T=2, N=5)
    ev, U, evals, tau = _corr_inputs(cfg)
    mom = np.array([[0, 0, 0], [0, 1, 0]])
    _, C = om.run(cfg.L, ev, U, evals, tau, mom, cfg.profiles)
    ev2, U2 = _gauge_transform(cfg.L, ev, U)
    _, C2 = om.run(cfg.L, ev2, U2, evals, tau, mom, cfg.profiles)
    np.testing.assert_allclose(C2, C, rtol=1e-10, atol=1e-12 * np.max(np.abs(C)))
    c = 0.7 - 0.4j
    _, C3 = om.run(cfg.L, ev, U, evals, c * tau, mom, cfg.profiles)
    np.testing.assert_allclose(C3, abs(c) ** 2 * C, rtol=1e-10, atol=1e-12 * np.max(np.abs(C)))


def test_field_strength_operators_decouple_for_trivial_links():
    cfg = _cfg(T=2, N=5)
    ev, _, evals, tau = _corr_inputs(cfg)
    U = np.zeros((cfg.T, cfg.V3, 3, 3, 3), complex)
    U[..., :, :] = np.eye(3)
    _, C = om.run(cfg.L, ev, U, evals, tau, np.zeros((1, 3)), cfg.profiles)
    nb = len(cfg.profiles)
    np.testing.assert_allclose(C[..., 2 * nb:, :], 0, atol=1e-13)
    np.testing.assert_allclose(C[..., :, 2 * nb:], 0, atol=1e-13)
    assert np.max(np.abs(C[..., :2 * nb, :2 * nb])) > 1e-3


def test_svd_pruning_diagonalises_hermitian_psd_matrix_at_tp():
    g = np.random.default_rng(4)
    n, T = 9, 4
    a = g.standard_normal((T, n, n)) + 1j * g.standard_normal((T, n, n))
    C = a @ np.conj(np.swapaxes(a, 1, 2))                    # Hermitian PSD per t
    Cp, um = om.svd_prune(C, 2, 5)
    w = np.sort(np.linalg.eigvalsh(C[2]))[::-1][:5]
    np.testing.assert_allclose(Cp[2], np.diag(w), atol=1e-10 * w[0])
    # m = n: a unitary similarity, so the GEVP spectrum is unchanged
    import oracle
    Cf, _ = om.svd_prune(C, 2, n)
    np.testing.assert_allclose(oracle.gevp(Cf, 0)[0], oracle.gevp(C, 0)[0], rtol=1e-9)

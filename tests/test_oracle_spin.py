"""Pins of the general-spin nucleon oracle (oracle/spin.py): it must reduce to the
plain-loop C oracle for the nucleon spin structure (C gamma5, P+), be linear in the sink
tensor and antilinear in the source tensor, be covariant under a change of spinor basis
at the sink and at the source, and turn the exchange term into the direct term when the
source's first and third quark slots are swapped."""
import numpy as np
import pytest

import oracle
import oracle.spin as osp


def _unitary(g, n):
    z = g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))[None, :]


def _inputs(N=4, nt=2, nmom=2, nprof=2, seed=1):
    g = np.random.default_rng(seed)
    c = lambda *s: g.standard_normal(s) + 1j * g.standard_normal(s)
    phi = c(nt, nmom, N, N, N)
    phi = phi - phi.transpose(0, 1, 2, 4, 3)                          # antisymmetric, as the nucleon's
    phi = phi + phi.transpose(0, 1, 3, 4, 2) + phi.transpose(0, 1, 4, 2, 3)
    phi0 = phi[0]
    tau = c(nt, 4 * N, 4 * N) / np.sqrt(2)
    gs = g.random((nprof, nt, N))
    g0 = gs[:, 0, :]
    return phi, phi0, tau, gs, g0, g


def test_reduces_to_the_nucleon_oracle():
    phi, phi0, tau, gs, g0, _ = _inputs()
    S = osp.nucleon_spin(+1)
    C, D, E = osp.correlator(phi, phi0, tau, gs, g0, S, S, terms=True)
    c_ref, d_ref, e_ref = oracle.correlator(phi, phi0, tau, gs, g0)
    sc = np.max(np.abs(d_ref))
    np.testing.assert_allclose(D, d_ref, atol=1e-11 * sc)
    np.testing.assert_allclose(E, e_ref, atol=1e-11 * sc)
    np.testing.assert_allclose(C, c_ref, atol=1e-11 * sc)


def test_linear_in_sink_antilinear_in_source():
    phi, phi0, tau, gs, g0, g = _inputs(N=3, seed=2)
    S = g.standard_normal((2, 4, 4, 4)) + 1j * g.standard_normal((2, 4, 4, 4))
    Sp = g.standard_normal((2, 4, 4, 4)) + 1j * g.standard_normal((2, 4, 4, 4))
    c = 0.6 - 0.8j
    C = osp.correlator(phi, phi0, tau, gs, g0, S, Sp)
    sc = np.max(np.abs(C))
    np.testing.assert_allclose(osp.correlator(phi, phi0, tau, gs, g0, c * S, Sp), c * C, atol=1e-12 * sc)
    np.testing.assert_allclose(osp.correlator(phi, phi0, tau, gs, g0, S, c * Sp), np.conj(c) * C, atol=1e-12 * sc)


def test_covariant_under_spinor_basis_changes():
    # tau -> (V (x) 1) tau (W (x) 1)^H with S -> S (V^H)^{(x)3} and S' -> conj(W)^{(x)3} S'
    phi, phi0, tau, gs, g0, g = _inputs(N=3, seed=3)
    S = g.standard_normal((2, 4, 4, 4)) + 1j * g.standard_normal((2, 4, 4, 4))
    Sp = g.standard_normal((2, 4, 4, 4)) + 1j * g.standard_normal((2, 4, 4, 4))
    V, W = _unitary(g, 4), _unitary(g, 4)
    N = phi.shape[2]
    VV, WW = np.kron(V, np.eye(N)), np.kron(W, np.eye(N))
    tau2 = np.einsum("ab,tbc,dc->tad", VV, tau, np.conj(WW))
    Vh = np.conj(V.T)
    S2 = np.einsum("rabc,ax,by,cz->rxyz", S, Vh, Vh, Vh)
    Sp2 = np.einsum("rabc,xa,yb,zc->rxyz", Sp, np.conj(W), np.conj(W), np.conj(W))
    C, D, E = osp.correlator(phi, phi0, tau, gs, g0, S, Sp, terms=True)
    C2, D2, E2 = osp.correlator(phi, phi0, tau2, gs, g0, S2, Sp2, terms=True)
    sc = np.max(np.abs(D))
    np.testing.assert_allclose(D2, D, atol=1e-11 * sc)
    np.testing.assert_allclose(E2, E, atol=1e-11 * sc)


def test_exchange_is_direct_with_source_slots_swapped():
    phi, phi0, tau, gs, g0, g = _inputs(N=3, seed=4)
    phi0 = g.standard_normal(phi0.shape) + 1j * g.standard_normal(phi0.shape)   # no symmetry assumed
    S = g.standard_normal((1, 4, 4, 4)) + 1j * g.standard_normal((1, 4, 4, 4))
    Sp = g.standard_normal((1, 4, 4, 4)) + 1j * g.standard_normal((1, 4, 4, 4))
    _, _, E = osp.correlator(phi, phi0, tau, gs, g0, S, Sp, terms=True)
    _, D13, _ = osp.correlator(phi, phi0.transpose(0, 3, 2, 1), tau, gs, g0, S, Sp.transpose(0, 3, 2, 1), terms=True)
    np.testing.assert_allclose(D13, E, atol=1e-11 * np.max(np.abs(E)))


def test_parity_projections_are_orthogonal_rows():
    # P+ and P- nucleon tensors project the third quark on complementary spinor rows
    Sp, Sm = osp.nucleon_spin(+1), osp.nucleon_spin(-1)
    assert np.all(Sp[:, :, :, 2:] == 0) and np.all(Sm[:, :, :, :2] == 0)
    cg5 = osp.charge_conjugation_g5()
    np.testing.assert_allclose(cg5, -cg5.T, atol=1e-15)                 # antisymmetric
    np.testing.assert_allclose(cg5 @ np.conj(cg5.T), np.eye(4), atol=1e-15)  # unitary

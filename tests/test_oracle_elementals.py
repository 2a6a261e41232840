"""Pins for the oracle's elementals, profiles and spin tables (CPU only).

Each test fixes the oracle against something other than itself: a closed form,
a literal brute-force sum, or an invariance the definition implies.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from tests import brute


def _rand_vecs(g, N, L, nt=1):
    z = (g.standard_normal((nt, N, L ** 3, 3)) + 1j * g.standard_normal((nt, N, L ** 3, 3)))
    return z / math.sqrt(2.0)


def test_identity_vectors_give_levi_civita():
    # one site, N = 3, v_i^a = delta_ia  =>  Phi_ijk = eps_ijk
    v = np.eye(3, dtype=complex).reshape(1, 3, 1, 3)
    phi = oracle.elementals(1, v, np.zeros((1, 3), np.int32))[0, 0]
    assert np.array_equal(phi.real, brute.levi_civita())
    assert np.all(phi.imag == 0)


@pytest.mark.parametrize("mom", [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, -1), (-2, 3, 1)])
def test_single_site_support_gives_phase_times_determinant(mom):
    # vectors supported on site x0 = (1, 2, 3) of a 4^3 lattice:
    # Phi_012 = exp(-2 pi i n.x0 / L) det(M) with M[i][a] = v_i^a(x0)
    L, x0 = 4, (1, 2, 3)
    g = np.random.default_rng(1)
    M = g.standard_normal((3, 3)) + 1j * g.standard_normal((3, 3))
    v = np.zeros((1, 3, L ** 3, 3), complex)
    xi = x0[0] + L * (x0[1] + L * x0[2])
    v[0, :, xi, :] = M
    phi = oracle.elementals(L, v, np.asarray([mom], np.int32))[0, 0]
    expect = np.exp(-2j * np.pi * np.dot(mom, x0) / L) * np.linalg.det(M)
    assert abs(phi[0, 1, 2] - expect) < 1e-12 * abs(expect)
    assert abs(phi[2, 1, 0] + expect) < 1e-12 * abs(expect)


def test_matches_literal_epsilon_sum():
    g = np.random.default_rng(2)
    L, N = 2, 5
    v = _rand_vecs(g, N, L, nt=2)
    mom = np.asarray([(0, 0, 0), (1, 0, 0), (1, -1, 1)], np.int32)
    got = oracle.elementals(L, v, mom)
    ref = brute.elementals(L, v, mom)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


def test_total_antisymmetry_and_zero_diagonals():
    g = np.random.default_rng(3)
    phi = oracle.elementals(2, _rand_vecs(g, 6, 2), np.asarray([(1, 0, 0)], np.int32))[0, 0]
    assert np.array_equal(phi, -phi.transpose(1, 0, 2))
    assert np.array_equal(phi, -phi.transpose(0, 2, 1))
    assert np.array_equal(phi, phi.transpose(1, 2, 0))
    for i in range(6):
        assert np.all(phi[i, i, :] == 0) and np.all(phi[i, :, i] == 0) and np.all(phi[:, i, i] == 0)


def test_su3_gauge_invariance_and_u3_determinant():
    g = np.random.default_rng(4)
    L, N = 2, 5
    v = _rand_vecs(g, N, L)
    mom = np.asarray([(0, 0, 0), (1, 1, 0)], np.int32)
    phi = oracle.elementals(L, v, mom)
    U = synth.random_su3(g, L ** 3)                      # one SU(3) matrix per site
    vr = np.einsum("xab,nixb->nixa", U, v)
    phir = oracle.elementals(L, vr, mom)
    assert np.max(np.abs(phir - phi)) < 1e-12 * np.max(np.abs(phi))
    # a constant U(3) rotation multiplies Phi by det U
    W = np.linalg.qr(g.standard_normal((3, 3)) + 1j * g.standard_normal((3, 3)))[0]
    vw = np.einsum("ab,nixb->nixa", W, v)
    phiw = oracle.elementals(L, vw, mom)
    assert np.max(np.abs(phiw - np.linalg.det(W) * phi)) < 1e-12 * np.max(np.abs(phi))


def test_rephasing_covariance():
    g = np.random.default_rng(5)
    L, N = 2, 6
    v = _rand_vecs(g, N, L)
    th = g.random(N) * 2 * np.pi
    mom = np.asarray([(1, 0, 1)], np.int32)
    phi = oracle.elementals(L, v, mom)[0, 0]
    phr = oracle.elementals(L, v * np.exp(1j * th)[None, :, None, None], mom)[0, 0]
    fac = np.exp(1j * (th[:, None, None] + th[None, :, None] + th[None, None, :]))
    assert np.max(np.abs(phr - fac * phi)) < 1e-12 * np.max(np.abs(phi))


def test_lattice_translation_multiplies_by_phase():
    # v'(x) = v(x - a)  =>  Phi'(p) = exp(-i p.a) Phi(p): pins the phase sign and site order
    g = np.random.default_rng(6)
    L, N, a = 3, 4, np.array([1, 2, 0])
    v = _rand_vecs(g, N, L)
    xs = brute.site_coords(L)
    src = (xs - a) % L
    perm = src[:, 0] + L * (src[:, 1] + L * src[:, 2])
    vs = v[:, :, perm, :]
    mom = np.asarray([(1, 0, 0), (0, 1, 0), (1, 2, -1)], np.int32)
    phi, phis = oracle.elementals(L, v, mom)[0], oracle.elementals(L, vs, mom)[0]
    for p, n in enumerate(mom):
        fac = np.exp(-2j * np.pi * np.dot(n, a) / L)
        assert np.max(np.abs(phis[p] - fac * phi[p])) < 1e-12 * np.max(np.abs(phi[p]))


def test_real_vectors_conjugate_under_momentum_reversal():
    g = np.random.default_rng(7)
    L, N = 3, 4
    v = g.standard_normal((1, N, L ** 3, 3)).astype(complex)
    phi = oracle.elementals(L, v, np.asarray([(1, -1, 2), (-1, 1, -2)], np.int32))[0]
    assert np.max(np.abs(phi[1] - np.conj(phi[0]))) < 1e-12 * np.max(np.abs(phi[0]))


def test_profiles_closed_forms():
    ev = np.array([[0.0, 0.3, 0.6, 1.2]])
    g = oracle.profiles(ev, [(0, 0.3), (0, 0.6), (1, 0.0)])
    assert g[0, 0, 0] == 1.0
    assert abs(g[0, 0, 1] - math.exp(-0.5)) < 1e-15
    assert abs(g[1, 0, 3] - math.exp(-2.0)) < 1e-15
    assert np.allclose(g[2, 0], [1.0, 0.75, 0.5, 0.25], rtol=0, atol=1e-15)


def test_profile_weighting_equals_rescaled_vectors():
    # Phi^(a)_ijk = g_i g_j g_k Phi_ijk  equals the elemental of the rescaled vectors g_i v_i
    g = np.random.default_rng(8)
    L, N = 2, 5
    v = _rand_vecs(g, N, L)
    gw = oracle.profiles(g.random((1, N)), [(0, 0.4)])[0, 0]
    mom = np.asarray([(1, 0, 0)], np.int32)
    phi = oracle.elementals(L, v, mom)[0, 0]
    phis = oracle.elementals(L, v * gw[None, :, None, None], mom)[0, 0]
    prof = gw[:, None, None] * gw[None, :, None] * gw[None, None, :] * phi
    assert np.max(np.abs(phis - prof)) < 1e-12 * np.max(np.abs(phi))


def test_spin_table_matches_gamma_algebra():
    cg5, pplus, C = brute.cg5_and_pplus()
    for gm in brute.gammas()[:4]:
        assert np.allclose(C @ gm @ np.linalg.inv(C), -gm.T)
    assert np.allclose(cg5.imag, 0)
    assert np.array_equal(oracle.cg5(), cg5.real)
    assert np.allclose(pplus, np.diag([1, 1, 0, 0]))


def test_selected_entries_agree_with_full_elementals():
    g = np.random.default_rng(9)
    L, N = 2, 6
    v = _rand_vecs(g, N, L)
    mom = np.asarray([(0, 0, 0), (1, 0, 1)], np.int32)
    full = oracle.elementals(L, v, mom)[0]
    idx = np.asarray([(0, 0, 1, 2), (1, 5, 3, 1), (1, 2, 2, 4), (0, 4, 0, 5)], np.int32)
    got = oracle.elemental_entries(L, v[0], mom, idx)
    ref = np.asarray([full[p, i, j, k] for p, i, j, k in idx])
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(full))
    assert got[2] == 0

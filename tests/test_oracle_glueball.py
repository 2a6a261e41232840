"""Pins of the FP64 glueball oracle (oracle/glueball.py) against what the symmetries fix:
gauge invariance of every trace, the quantum numbers of the five A1^{-+} operators
(invariant under the proper cubic rotations, odd under spatial inversion), zero fields
for trivial or constant abelian links, and the structure of the correlation matrix.
A wrong leaf orientation, epsilon sign, derivative direction or index order breaks at
least one of them."""
import itertools

import numpy as np
import pytest

import oracle.glueball as og
from oracle.meson import neighbours
import synth


def _links(L, T=1, seed=3):
    g = np.random.default_rng(seed)
    V3 = L ** 3
    return np.stack([synth.random_su3(g, V3 * 3).reshape(V3, 3, 3, 3) for _ in range(T)])


def _coords(L):
    x = np.arange(L ** 3)
    return np.stack([x % L, (x // L) % L, x // (L * L)], axis=1)


def _index(L, c):
    c = np.mod(c, L)
    return c[..., 0] + L * (c[..., 1] + L * c[..., 2])


def _transform(L, U, R):
    """Links of the configuration mapped by the signed permutation R (x -> R x)."""
    c = _coords(L)
    out = np.empty_like(U)
    for mu in range(3):
        img = R @ np.eye(3, dtype=int)[mu]          # R e_mu = s e_nu
        nu = int(np.flatnonzero(img)[0])
        s = int(img[nu])
        rx = _index(L, c @ R.T)
        if s > 0:
            out[:, rx, nu] = U[:, :, mu]
        else:                                        # the link from Rx to Rx - e_nu
            out[:, _index(L, c @ R.T - np.eye(3, dtype=int)[nu]), nu] = np.conj(np.swapaxes(U[:, :, mu], -1, -2))
    return out


def test_trivial_links_give_zero():
    L = 3
    U = np.zeros((1, L ** 3, 3, 3, 3), complex)
    U[..., :, :] = np.eye(3)
    assert np.max(np.abs(og.magnetic(L, U[0]))) == 0.0
    np.testing.assert_array_equal(og.operators(L, U), 0.0)


def test_constant_abelian_field_closed_form():
    # U_0(x) = exp(i b x1 lambda), lambda = diag(1,-1,0), b = 2 pi n / L (periodic):
    # every (0,1) leaf is exp(-i b lambda) [counter-clockwise in (0,1)], so
    # F_01 = -i sin(b lambda), B_2 = 2 F_01, B_0 = B_1 = 0; the field is constant and
    # commutes with the links, so every D B vanishes and every operator is 0.
    L = 4
    b = 2 * np.pi / L
    lam = np.array([1.0, -1.0, 0.0])
    c = _coords(L)
    U = np.zeros((L ** 3, 3, 3, 3), complex)
    U[..., :, :] = np.eye(3)
    U[:, 0] = np.einsum("xa,ab->xab", np.exp(1j * b * c[:, 1:2] * lam[None, :]), np.eye(3))
    B = og.magnetic(L, U)
    np.testing.assert_allclose(B[2], np.broadcast_to(np.diag(-2j * np.sin(b * lam)), B[2].shape), atol=1e-14)
    np.testing.assert_allclose(B[:2], 0.0, atol=1e-14)
    np.testing.assert_allclose(og.operators_timeslice(L, U), 0.0, atol=1e-12)


def test_field_strength_is_antihermitian_traceless():
    L = 3
    B = og.magnetic(L, _links(L)[0])
    np.testing.assert_allclose(B, -np.conj(np.swapaxes(B, -1, -2)), atol=1e-14)
    np.testing.assert_allclose(np.trace(B, axis1=-2, axis2=-1), 0.0, atol=1e-14)


def test_gauge_invariance():
    L = 3
    U = _links(L, T=2)
    g = np.random.default_rng(9)
    U2 = np.empty_like(U)
    for t in range(U.shape[0]):
        om = synth.random_su3(g, L ** 3)
        for d in range(3):
            U2[t, :, d] = om @ U[t, :, d] @ np.conj(np.swapaxes(om[neighbours(L, d, +1)], 1, 2))
    a, b = og.operators(L, U), og.operators(L, U2)
    assert np.min(np.abs(a)) > 1e-3                       # nothing is trivially zero
    np.testing.assert_allclose(b, a, rtol=1e-10, atol=1e-12 * np.max(np.abs(a)))


@pytest.mark.parametrize("name,R", [
    ("rot90_x2", np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]])),
    ("rot90_x0", np.array([[1, 0, 0], [0, 0, -1], [0, 1, 0]])),
    ("rot90_x1", np.array([[0, 0, 1], [0, 1, 0], [-1, 0, 0]])),
    ("cycle", np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]])),
])
def test_invariant_under_cubic_rotations(name, R):
    L = 3
    U = _links(L, seed=5)
    a = og.operators(L, U)
    b = og.operators(L, _transform(L, U, R))
    np.testing.assert_allclose(b, a, rtol=1e-10, atol=1e-12 * np.max(np.abs(a)))


def test_odd_under_spatial_inversion():
    L = 3
    U = _links(L, seed=6)
    a = og.operators(L, U)
    b = og.operators(L, _transform(L, U, -np.eye(3, dtype=int)))
    np.testing.assert_allclose(b, -a, rtol=1e-10, atol=1e-12 * np.max(np.abs(a)))
    # and a reflection (inversion times a rotation) as well
    b2 = og.operators(L, _transform(L, U, np.diag([1, 1, -1])))
    np.testing.assert_allclose(b2, -a, rtol=1e-10, atol=1e-12 * np.max(np.abs(a)))


def test_correlator_structure():
    g = np.random.default_rng(2)
    T = 6
    O = g.standard_normal((T, 5)) + 1j * g.standard_normal((T, 5))
    C = og.correlator(O)
    for dt in range(1, T):
        np.testing.assert_allclose(C[T - dt], np.conj(C[dt]).T, atol=1e-13)
    np.testing.assert_allclose(C[0], np.conj(C[0]).T, atol=1e-13)
    assert np.min(np.linalg.eigvalsh(C[0])) > -1e-12      # a covariance matrix
    np.testing.assert_allclose(og.correlator(np.tile(O[:1], (T, 1))), 0.0, atol=1e-13)


def test_double_epsilon_operator_matches_the_delta_identity():
    # eps_ijk eps_ilm = d_jl d_km - d_jm d_kl turns O2 into
    # sum_jk Tr(B_j B_k D_j B_k) - Tr(B_j B_k D_k B_j): a different contraction that
    # must give the same number
    L = 3
    U = _links(L, seed=8)[0]
    B = og.magnetic(L, U)
    DB = {(j, k): og.adjoint_diff(L, U, B[k], j) for j in range(3) for k in range(3)}
    tr = lambda a, b, c: np.trace(a @ b @ c, axis1=1, axis2=2).sum()
    alt = sum(tr(B[j], B[k], DB[(j, k)]) - tr(B[j], B[k], DB[(k, j)]) for j in range(3) for k in range(3))
    o = og.operators_timeslice(L, U)
    assert abs(alt) > 1e-3
    np.testing.assert_allclose(o[1], alt, rtol=1e-12)

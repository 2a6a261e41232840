"""Brute-force definitions used to pin the oracle on tiny inputs.

Everything here is written independently of ``oracle/oracle.c``: gamma
matrices are built from the Pauli matrices, the elemental is the literal
colour-epsilon sum over every (i, j, k), and the correlator is the literal
six-index sum over the full (spin x distillation) indices with dense spin
tensors, evaluated by ``numpy.einsum`` without contraction-path optimisation.
"""
from __future__ import annotations

import numpy as np

SIGMA = [np.array([[0, 1], [1, 0]], complex),
         np.array([[0, -1j], [1j, 0]], complex),
         np.array([[1, 0], [0, -1]], complex)]


def gammas():
    """Euclidean Dirac-Pauli gammas: g4 = diag(1,1,-1,-1), g_k = [[0,-i s_k],[i s_k,0]]."""
    z = np.zeros((2, 2), complex)
    g = []
    for s in SIGMA:
        g.append(np.block([[z, -1j * s], [1j * s, z]]))
    g4 = np.diag([1, 1, -1, -1]).astype(complex)
    g5 = g[0] @ g[1] @ g[2] @ g4
    return g[0], g[1], g[2], g4, g5


def cg5_and_pplus():
    g1, g2, g3, g4, g5 = gammas()
    C = g2 @ g4
    return C @ g5, (np.eye(4) + g4) / 2, C


def levi_civita():
    e = np.zeros((3, 3, 3))
    e[0, 1, 2] = e[1, 2, 0] = e[2, 0, 1] = 1.0
    e[0, 2, 1] = e[2, 1, 0] = e[1, 0, 2] = -1.0
    return e


def site_coords(L):
    x = np.arange(L ** 3)
    return np.stack([x % L, (x // L) % L, x // (L * L)], axis=1)


def phases(L, mom):
    xs = site_coords(L)
    return np.exp(-2j * np.pi * (xs @ np.asarray(mom, float).T) / L).T  # [nmom][V3]


def elementals(L, evecs, mom):
    """Literal Phi[t][p][i][j][k] = sum_x e^{-ipx} sum_abc eps_abc v_i^a v_j^b v_k^c."""
    eps = levi_civita()
    ph = phases(L, mom)
    out = []
    for v in evecs:
        per_p = []
        for p in range(ph.shape[0]):
            per_p.append(np.einsum("x,abc,ixa,jxb,kxc->ijk", ph[p], eps, v, v, v, optimize=False))
        out.append(per_p)
    return np.asarray(out)


def correlator(phi_t, phi_0, tau, g_t, g_0):
    """Literal D, E for one (t, p): dense spin tensors, six-index sums.

    phi_t, phi_0: [N][N][N]; tau: [4N][4N]; g_t, g_0: [nprof][N].
    Returns C, D, E as [nprof][nprof].
    """
    N = phi_t.shape[0]
    cg5, pplus, _ = cg5_and_pplus()
    S = np.einsum("ab,cs->abcs", cg5, np.eye(4))          # S_{abc sigma}
    nprof = g_t.shape[0]
    D = np.zeros((nprof, nprof), complex)
    E = np.zeros((nprof, nprof), complex)

    def big(spin, dist):  # (alpha,i),(beta,j),(gamma,k) -> flat index spin*N + i
        t = np.einsum("abc,ijk->aibjck", spin, dist)
        return t.reshape(4 * N, 4 * N, 4 * N)

    for a in range(nprof):
        A_dist = np.einsum("i,j,k,ijk->ijk", g_t[a], g_t[a], g_t[a], phi_t)
        for b in range(nprof):
            B_dist = np.conj(np.einsum("i,j,k,ijk->ijk", g_0[b], g_0[b], g_0[b], phi_0))
            for s in range(4):
                for sp in range(4):
                    w = pplus[sp, s]
                    if w == 0:
                        continue
                    A = big(S[:, :, :, s], A_dist)
                    B = big(np.conj(S[:, :, :, sp]), B_dist)
                    D[a, b] += w * np.einsum("IJK,IL,JM,KN,LMN->", A, tau, tau, tau, B, optimize=False)
                    E[a, b] += w * np.einsum("IJK,IN,JM,KL,LMN->", A, tau, tau, tau, B, optimize=False)
    return D - E, D, E

"""FP64 oracle of the nucleon correlation matrix with general spin tensors (moving-frame
irreps and other three-quark spin structures; the generalisation of the nucleon path of
Section 2.1 to the G1 operators of Section 2.1's moving-frame figure): test
infrastructure only (the library never imports it).

Definitions (the readings are listed in the design doc):

* sink operator row sigma of profile a at (t, p):
    A^(a)[sigma]_{(alpha i)(beta j)(gamma k)} = g_i g_j g_k Phi(t,p)_ijk S[sigma][alpha][beta][gamma];
* source operator row sigma of profile b:
    B^(b)[sigma]_{(alpha' i')(beta' j')(gamma' k')} = conj(g_i' g_j' g_k' Phi(t0,p)_i'j'k' S'[sigma][alpha'][beta'][gamma']);
* direct and u-quark exchange terms, tau = tau(t, t0) in every slot:
    D = sum_sigma sum A_{IJK} tau_{II'} tau_{JJ'} tau_{KK'} B_{I'J'K'},
    E = sum_sigma sum A_{IJK} tau_{IK'} tau_{JJ'} tau_{KI'} B_{I'J'K'},
    C_ab(t) = D - E.
With S = S' = (C gamma5)_{alpha beta} delta_{gamma sigma}, sigma in {0, 1} (parity
projector P+ = (1 + gamma4)/2) this is the nucleon correlator of oracle.correlator.

Plain numpy in FP64: the spin-expanded tensors are built densely ((4N)^3 entries) and
the three tau products are tensor contractions, one mode at a time.
"""
from __future__ import annotations

import numpy as np

from oracle.meson import dirac_pauli


def charge_conjugation_g5():
    """C gamma5 with C = gamma2 gamma4 (Dirac-Pauli)."""
    g, g4, g5 = dirac_pauli()
    return g[1] @ g4 @ g5


def nucleon_spin(parity: int = +1) -> np.ndarray:
    """S [2][4][4][4] of the nucleon with the third quark's parity projection
    (1 + parity gamma4)/2: rows sigma = 0, 1 (upper components) for +1, 2, 3 for -1."""
    cg5 = charge_conjugation_g5()
    rows = (0, 1) if parity > 0 else (2, 3)
    S = np.zeros((2, 4, 4, 4), complex)
    for r, s in enumerate(rows):
        S[r, :, :, s] = cg5
    return S


def _expand(phi: np.ndarray, S: np.ndarray) -> np.ndarray:
    """[(alpha i)(beta j)(gamma k)] = phi_ijk S_{alpha beta gamma}."""
    N = phi.shape[0]
    t = np.einsum("ijk,abc->aibjck", phi, S)
    return t.reshape(4 * N, 4 * N, 4 * N)


def _tau3(tau: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Y_{IJK} = sum tau_{II'} tau_{JJ'} tau_{KK'} B_{I'J'K'}."""
    y = np.tensordot(tau, B, axes=([1], [0]))                         # I J' K'
    y = np.tensordot(tau, y, axes=([1], [1])).transpose(1, 0, 2)      # I J K'
    return np.tensordot(y, tau, axes=([2], [1]))                      # I J K


def correlator(phi_snk, phi_src, tau, g_snk, g_src, S, Sp, terms: bool = False):
    """C [nmom][nt][nprof][nprof] (and D, E with terms=True).

    phi_snk [nt][nmom][N][N][N], phi_src [nmom][N][N][N], tau [nt][4N][4N],
    g_snk [nprof][nt][N], g_src [nprof][N], S and Sp [nrow][4][4][4]."""
    phi_snk = np.asarray(phi_snk, np.complex128)
    phi_src = np.asarray(phi_src, np.complex128)
    nt, nmom, N = phi_snk.shape[0], phi_snk.shape[1], phi_snk.shape[2]
    nprof, nrow = g_snk.shape[0], S.shape[0]
    D = np.zeros((nmom, nt, nprof, nprof), complex)
    E = np.zeros_like(D)
    for p in range(nmom):
        for b in range(nprof):
            gb = g_src[b]
            w0 = np.einsum("i,j,k->ijk", gb, gb, gb) * phi_src[p]
            Bs = [np.conj(_expand(w0, Sp[r])) for r in range(nrow)]
            for t in range(nt):
                Ys = [_tau3(tau[t], B) for B in Bs]
                YXs = [_tau3(tau[t], B.transpose(2, 1, 0)) for B in Bs]      # source slots 1 and 3 swapped
                for a in range(nprof):
                    ga = g_snk[a, t]
                    wt = np.einsum("i,j,k->ijk", ga, ga, ga) * phi_snk[t, p]
                    for r in range(nrow):
                        A = _expand(wt, S[r])
                        D[p, t, a, b] += np.sum(A * Ys[r])
                        E[p, t, a, b] += np.sum(A * YXs[r])
    C = D - E
    return (C, D, E) if terms else C

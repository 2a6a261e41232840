"""FP64 oracle of the I=2 A1++ two-meson correlator built from optimal one-meson
operators at zero total momentum and back-to-back momenta (the paper's Section 3,
"Improved charmonium operators"): test infrastructure only (the library never imports it).

Definitions (the readings are listed in the design doc):

* optimal one-meson operator with coefficients w_A over the 3 N_B profiled operators of
  oracle.meson (A = family * N_B + a), as a distillation matrix at (t, p):
    M_w(t, p) = sum_A w_A M_A(t, p);
  for a GEVP eigenvector v of C(t) v = lambda C(t0) v the operator sum_A conj(v_A) O_A
  has the correlator v^H C v, so w = conj(v) (w = conj(U_m v) after SVD pruning with
  basis U_m);
* pi+(p, t) = dbar M_w(t, p) u, its source Mbar = g4 M_w(t0, q)^H g4 (as in oracle.meson),
  quark lines tau = tau(t, t0) and the antiquark line g5 tau^H g5;
* P_kl(t) = M_w(t, p_k) tau Mbar_w(t0, p_l) g5 tau^H g5;
* two-meson operator O(t) = sum_k pi+(p_k, t) pi+(-p_k, t) over a list of momenta closed
  under negation (the star of a momentum gives the A1 projection at zero total momentum);
* Wick contractions of <O(t) O(t0)^H> for two identical mesons (two u lines, two d lines):
  the direct terms (two closed quark loops) and the crossed terms (one loop, sign -1):
    C(t) = sum_{k,l} c(k, kbar; l, lbar),
    c(1, 2; a, b) = Tr P_1a Tr P_2b + Tr P_1b Tr P_2a - Tr[P_1a P_2b] - Tr[P_1b P_2a],
  kbar the index of -p_k. Summed over k and l the two orders of each pairing coincide:
    C = 2 sum_{k,l} (Tr P_kl Tr P_kbar,lbar - Tr[P_kl P_kbar,lbar]).

Plain numpy in FP64; the four terms of c are written out one by one. correlator_by_pairs
evaluates the summed form (each P_kl formed once), for sizes where the term-by-term sum
is slow; the CPU tests pin the two against each other.
"""
from __future__ import annotations

import numpy as np

from oracle.meson import dirac_pauli, operator_matrices


def optimal_operator(phi_tp: np.ndarray, g: np.ndarray, w: np.ndarray) -> np.ndarray:
    """M_w [4N][4N] from one (t, p) of elementals [7][N][N], profiles g [nprof][N], w [3 nprof]."""
    mats = operator_matrices(phi_tp, g)
    return np.tensordot(np.asarray(w, complex), mats, axes=(0, 0))


def pair_term(m1, m2, mbar_a, mbar_b, tau, tau_back, terms: bool = False):
    """c(1, 2; a, b) for sink matrices m1, m2, source matrices mbar_a, mbar_b, the quark
    line tau and the antiquark line tau_back (with terms, the direct and crossed parts)."""
    P = lambda m, mb: m @ tau @ mb @ tau_back
    p1a, p2b, p1b, p2a = P(m1, mbar_a), P(m2, mbar_b), P(m1, mbar_b), P(m2, mbar_a)
    direct = np.trace(p1a) * np.trace(p2b) + np.trace(p1b) * np.trace(p2a)
    crossed = np.trace(p1a @ p2b) + np.trace(p1b @ p2a)
    return (direct - crossed, direct, crossed) if terms else direct - crossed


def negation_index(mom: np.ndarray) -> np.ndarray:
    """kbar [nmom]: mom[kbar[k]] = -mom[k] (the list must be closed under negation)."""
    mom = np.asarray(mom).reshape(-1, 3)
    out = np.empty(len(mom), int)
    for k, p in enumerate(mom):
        hit = np.nonzero(np.all(mom == -p, axis=1))[0]
        if len(hit) == 0:
            raise ValueError("momentum %s has no partner %s in the list" % (p, -p))
        out[k] = hit[0]
    return out


def correlator(phi_snk, phi_src, tau, g_snk, g_src, w, mom, terms: bool = False):
    """C [nt] (and the direct and crossed parts with terms) of the two-meson operator.

    phi_snk [nt][nmom][7][N][N], phi_src [nmom][7][N][N], tau [nt][4N][4N] (tau(t, t0),
    rows spin * N + i), g_snk [nprof][nt][N], g_src [nprof][N], w [3 nprof], mom [nmom][3]."""
    _, g4, g5 = dirac_pauli()
    N = phi_src.shape[-1]
    G4, G5 = np.kron(g4, np.eye(N)), np.kron(g5, np.eye(N))
    nt, nmom = phi_snk.shape[0], phi_snk.shape[1]
    kbar = negation_index(mom)
    msrc = [optimal_operator(phi_src[q], g_src, w) for q in range(nmom)]
    mbar = [G4 @ m.conj().T @ G4 for m in msrc]
    C = np.zeros(nt, complex)
    D = np.zeros(nt, complex)
    X = np.zeros(nt, complex)
    for t in range(nt):
        back = G5 @ tau[t].conj().T @ G5
        msnk = [optimal_operator(phi_snk[t, p], g_snk[:, t, :], w) for p in range(nmom)]
        for k in range(nmom):
            for l in range(nmom):
                c, d, x = pair_term(msnk[k], msnk[kbar[k]], mbar[l], mbar[kbar[l]], tau[t], back, terms=True)
                C[t] += c
                D[t] += d
                X[t] += x
    return (C, D, X) if terms else C


def correlator_by_pairs(phi_snk, phi_src, tau, g_snk, g_src, w, mom, terms: bool = False):
    """The same C [nt] from the summed form C = 2 sum_{k,l} (Tr P_kl Tr P_kbar,lbar -
    Tr[P_kl P_kbar,lbar]), every P_kl formed once (arguments as correlator)."""
    _, g4, g5 = dirac_pauli()
    N = phi_src.shape[-1]
    G4, G5 = np.kron(g4, np.eye(N)), np.kron(g5, np.eye(N))
    nt, nmom = phi_snk.shape[0], phi_snk.shape[1]
    kbar = negation_index(mom)
    mbar = [G4 @ optimal_operator(phi_src[q], g_src, w).conj().T @ G4 for q in range(nmom)]
    D = np.zeros(nt, complex)
    X = np.zeros(nt, complex)
    for t in range(nt):
        back = G5 @ tau[t].conj().T @ G5
        L = [optimal_operator(phi_snk[t, p], g_snk[:, t, :], w) @ tau[t] for p in range(nmom)]
        R = [mb @ back for mb in mbar]
        P = [[L[k] @ R[l] for l in range(nmom)] for k in range(nmom)]
        for k in range(nmom):
            for l in range(nmom):
                D[t] += 2 * np.trace(P[k][l]) * np.trace(P[kbar[k]][kbar[l]])
                X[t] += 2 * np.sum(P[k][l] * P[kbar[k]][kbar[l]].T)
    return (D - X, D, X) if terms else D - X

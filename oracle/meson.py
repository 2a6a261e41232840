"""FP64 oracle of the profiled meson operators of the paper's charmonium study
(Section 3): test infrastructure only (the library never imports it).

Definitions (the readings are listed in the design doc):

* covariant derivative, symmetric difference on periodic sites:
  (nabla_d f)(x) = 1/2 [U_d(x) f(x + d) - U_d(x - d)^H f(x - d)];
* B_i = eps_ijk nabla_j nabla_k, i.e. B_0 = nabla_1 nabla_2 - nabla_2 nabla_1 and cyclic;
* elementals, for D in (1, nabla_0, nabla_1, nabla_2, B_0, B_1, B_2):
  Phi^D[p,t]_ij = sum_x exp(-2 pi i n_p.x / L) v_i(x,t)^H (D v_j)(x,t);
* operator families (gamma_4 is the time direction, gamma_5 = g1 g2 g3 g4):
  f = 0: Gamma = g4 g5 with D = 1; f = 1: sum_k g4 g5 g_k (x) nabla_k; f = 2: sum_k g_k (x) B_k;
  each with the bilinear profile weighting g_i^(a) g_j^(a);
* operator matrix M_A(t)[(alpha,i),(beta,j)] = sum over the family's (Gamma, D) of
  Gamma[alpha][beta] g_i g_j Phi^D_ij, A = f N_B + a;
* correlation matrix C_AB(t) = -Tr[M_A(t) tau(t,t0) Mbar_B(t0) g5 tau(t,t0)^H g5],
  Mbar = g4 M^H g4 (the source operator; g5-hermiticity gives tau(t0,t); the minus
  sign is the closed quark loop's);
* SVD pruning: the m left singular vectors U_m of C(t_p) for the largest singular
  values project every C(t) to U_m^H C(t) U_m.

Everything is plain numpy in FP64: neighbour sites by index arrays, the site and
colour sum of the elementals by one matrix product per momentum, the operator
matrices by Kronecker products, the trace by matrix products, the SVD by numpy's
routine.
"""
from __future__ import annotations

import numpy as np

SIGMA = [np.array([[0, 1], [1, 0]], complex),
         np.array([[0, -1j], [1j, 0]], complex),
         np.array([[1, 0], [0, -1]], complex)]


def dirac_pauli():
    """Euclidean Dirac-Pauli gamma_1..3, gamma_4 = diag(1,1,-1,-1), gamma_5 = g1 g2 g3 g4."""
    z = np.zeros((2, 2), complex)
    g = [np.block([[z, -1j * s], [1j * s, z]]) for s in SIGMA]
    g4 = np.diag([1.0, 1.0, -1.0, -1.0]).astype(complex)
    g5 = g[0] @ g[1] @ g[2] @ g4
    return g, g4, g5


def neighbours(L: int, d: int, step: int) -> np.ndarray:
    """Site index of x + step * e_d for every x = x0 + L (x1 + L x2), periodic."""
    x = np.arange(L ** 3)
    c = [x % L, (x // L) % L, x // (L * L)]
    c[d] = (c[d] + step) % L
    return c[0] + L * (c[1] + L * c[2])


def nabla(L: int, f: np.ndarray, U: np.ndarray, d: int) -> np.ndarray:
    """Covariant symmetric difference of fields f [..][V3][3] with links U [V3][3][3][3]."""
    fwd, bwd = neighbours(L, d, +1), neighbours(L, d, -1)
    up = np.einsum("xab,...xb->...xa", U[:, d], f[..., fwd, :])
    dn = np.einsum("xba,...xb->...xa", np.conj(U[bwd, d]), f[..., bwd, :])
    return 0.5 * (up - dn)


def derivatives(L: int, v: np.ndarray, U: np.ndarray) -> np.ndarray:
    """(D v) for D in (1, nabla_0..2, B_0..2): [7][N][V3][3] from v [N][V3][3]."""
    w = [nabla(L, v, U, d) for d in range(3)]
    out = [v] + w
    for i in range(3):
        j, k = (i + 1) % 3, (i + 2) % 3
        out.append(nabla(L, w[k], U, j) - nabla(L, w[j], U, k))
    return np.stack(out)


def phases(L: int, mom: np.ndarray) -> np.ndarray:
    x = np.arange(L ** 3)
    c = np.stack([x % L, (x // L) % L, x // (L * L)], axis=1)
    return np.exp(-2j * np.pi * (c @ np.asarray(mom, float).reshape(-1, 3).T) / L).T  # [nmom][V3]


def elementals(L: int, evecs: np.ndarray, links: np.ndarray, mom: np.ndarray) -> np.ndarray:
    """Phi [T][nmom][7][N][N] from evecs [T][N][V3][3] and links [T][V3][3][3][3]."""
    ph = phases(L, mom)
    out = []
    for v, U in zip(np.asarray(evecs, np.complex128), np.asarray(links, np.complex128)):
        N, V3 = v.shape[0], v.shape[1]
        dv = derivatives(L, v, U).reshape(7 * N, 3 * V3)          # rows (D, j), columns (x, a)
        per_p = []
        for q in ph:                                              # the site and colour sum as one matrix product
            left = (np.conj(v) * q[None, :, None]).reshape(N, 3 * V3)
            per_p.append((left @ dv.T).reshape(N, 7, N).transpose(1, 0, 2))
        out.append(np.stack(per_p))
    return np.stack(out)


def operator_spins():
    """Per family, the (Gamma, D index) terms of the operator."""
    g, g4, g5 = dirac_pauli()
    return [[(g4 @ g5, 0)],
            [(g4 @ g5 @ g[k], 1 + k) for k in range(3)],
            [(g[k], 4 + k) for k in range(3)]]


def operator_matrices(phi_tp: np.ndarray, g: np.ndarray) -> np.ndarray:
    """M_A [3 nprof][4N][4N] from one (t,p) of elementals [7][N][N] and profile values g [nprof][N]."""
    mats = []
    for fam in operator_spins():
        for a in range(g.shape[0]):
            w = np.outer(g[a], g[a])
            mats.append(sum(np.kron(G, w * phi_tp[d]) for G, d in fam))
    return np.stack(mats)


def correlator(phi_snk: np.ndarray, phi_src: np.ndarray, tau: np.ndarray, g_snk: np.ndarray,
               g_src: np.ndarray) -> np.ndarray:
    """C [nmom][nt][3 nprof][3 nprof] from phi_snk [nt][nmom][7][N][N], phi_src [nmom][7][N][N],
    tau [nt][4N][4N] (tau(t, t0), rows spin * N + i), g_snk [nprof][nt][N], g_src [nprof][N]."""
    _, g4, g5 = dirac_pauli()
    N = phi_src.shape[-1]
    G4, G5 = np.kron(g4, np.eye(N)), np.kron(g5, np.eye(N))
    nt, nmom = phi_snk.shape[0], phi_snk.shape[1]
    nop = 3 * g_src.shape[0]
    out = np.empty((nmom, nt, nop, nop), np.complex128)
    for p in range(nmom):
        msrc = operator_matrices(phi_src[p], g_src)
        mbar = np.stack([G4 @ m.conj().T @ G4 for m in msrc])
        for t in range(nt):
            msnk = operator_matrices(phi_snk[t, p], g_snk[:, t, :])
            back = G5 @ tau[t].conj().T @ G5
            for A in range(nop):
                left = msnk[A] @ tau[t]
                for B in range(nop):
                    out[p, t, A, B] = -np.trace(left @ mbar[B] @ back)  # quark loop: -1
    return out


def svd_prune(corr: np.ndarray, t_p: int, m: int):
    """Project C(t) [T][n][n] onto the m left singular vectors of C(t_p) with the largest
    singular values: returns (C' [T][m][m], U_m [n][m])."""
    u, s, vh = np.linalg.svd(np.asarray(corr, np.complex128)[t_p])
    um = u[:, :m]
    return np.einsum("in,tij,jm->tnm", um.conj(), corr, um), um


def run(L, evecs, links, evals, tau, mom, prof, ts=None, t0=0):
    """Meson elementals at the sink times ts (default all) and C there."""
    import oracle as _o
    T = evecs.shape[0]
    ts = list(range(T)) if ts is None else list(ts)
    g = _o.profiles(evals, prof)
    phi_t = elementals(L, evecs[ts], links[ts], mom)
    phi_0 = elementals(L, evecs[[t0]], links[[t0]], mom)[0]
    return phi_t, correlator(phi_t, phi_0, tau[ts], g[:, ts, :], g[:, t0, :])

"""FP64 oracle of the glueball operators of the paper's Section 3 ("Improved glueball
operators"): test infrastructure only (the library never imports it).

Definitions (the readings are listed in the design doc):

* plaquette leaves of the clover in the plane (m, n) at x, each a closed path from x:
    x -> x+m -> x+m+n -> x+n -> x,   x -> x+n -> x-m+n -> x-m -> x,
    x -> x-m -> x-m-n -> x-n -> x,   x -> x-n -> x+m-n -> x+m -> x;
  Q_mn(x) their sum, F_mn(x) = (Q_mn - Q_mn^H) / 8 with the trace removed
  (anti-Hermitian and traceless);
* chromo-magnetic field B_i = eps_ijk F_jk (sum over j, k), i.e. B_0 = 2 F_12,
  B_1 = 2 F_20, B_2 = 2 F_01;
* adjoint gauge-covariant symmetric difference of a matrix field X:
    (D_j X)(x) = 1/2 [U_j(x) X(x+j) U_j(x)^H - U_j(x-j)^H X(x-j) U_j(x-j)];
  products of D act right to left (D_j D_k X = D_j (D_k X));
* the five A1^{-+} operators per timeslice, repeated indices summed over 0..2:
    O1 = sum_x Tr(eps_ijk B_i D_j B_k)
    O2 = sum_x Tr(eps_ijk eps_ilm B_j B_k D_l B_m)
    O3 = sum_x Tr(eps_ijk B_i D_j^3 B_k)
    O4 = sum_x Tr(eps_ijk B_i D_j^2 D_k B_j)
    O5 = sum_x Tr(eps_ijk B_i D_j D_i^2 B_k);
* correlation matrix of one configuration, time-averaged with the vacuum part removed:
    C_nm(dt) = 1/T sum_t O_n(t + dt) conj(O_m(t)) - Obar_n conj(Obar_m),
    Obar = 1/T sum_t O(t), periodic in t.

Plain numpy in FP64: neighbour sites by index arrays, 3 x 3 products by einsum/matmul
over all sites at once, each operator summed term by term as written.
"""
from __future__ import annotations

import itertools

import numpy as np

from oracle.meson import neighbours

EPS = np.zeros((3, 3, 3))
for _i, _j, _k in itertools.permutations(range(3)):
    EPS[_i, _j, _k] = np.linalg.det(np.eye(3)[[_i, _j, _k]])


def _h(u):
    return np.conj(np.swapaxes(u, -1, -2))


def clover(L: int, U: np.ndarray, m: int, n: int) -> np.ndarray:
    """F_mn [V3][3][3] (anti-Hermitian, traceless) from one timeslice's links U [V3][3][3][3]."""
    fm, fn = neighbours(L, m, +1), neighbours(L, n, +1)
    bm, bn = neighbours(L, m, -1), neighbours(L, n, -1)
    Um, Un = U[:, m], U[:, n]
    q = Um @ Un[fm] @ _h(Um[fn]) @ _h(Un)                                   # x, x+m, x+m+n, x+n
    q = q + Un @ _h(Um[bm[fn]]) @ _h(Un[bm]) @ Um[bm]                       # x, x+n, x-m+n, x-m
    q = q + _h(Um[bm]) @ _h(Un[bm[bn]]) @ Um[bm[bn]] @ Un[bn]               # x, x-m, x-m-n, x-n
    q = q + _h(Un[bn]) @ Um[bn] @ Un[fm[bn]] @ _h(Um)                       # x, x-n, x+m-n, x+m
    f = (q - _h(q)) / 8.0
    tr = np.trace(f, axis1=1, axis2=2)
    return f - tr[:, None, None] / 3.0 * np.eye(3)


def magnetic(L: int, U: np.ndarray) -> np.ndarray:
    """B_i [3][V3][3][3] = eps_ijk F_jk."""
    F = {(m, n): clover(L, U, m, n) for m in range(3) for n in range(3) if m != n}
    out = np.zeros((3,) + F[(0, 1)].shape, complex)
    for i, j, k in itertools.permutations(range(3)):
        out[i] += EPS[i, j, k] * F[(j, k)]
    return out


def adjoint_diff(L: int, U: np.ndarray, X: np.ndarray, j: int) -> np.ndarray:
    """(D_j X)(x) for a matrix field X [V3][3][3]."""
    f, b = neighbours(L, j, +1), neighbours(L, j, -1)
    Uj = U[:, j]
    return 0.5 * (Uj @ X[f] @ _h(Uj) - _h(Uj[b]) @ X[b] @ Uj[b])


def operators_timeslice(L: int, U: np.ndarray, with_scale: bool = False):
    """[O1..O5] of one timeslice (complex); with_scale, also the sum over terms and sites
    of |Tr(...)| per operator (the size of what is summed, which bounds |O_n| and the
    rounding error of any evaluation of it)."""
    B = magnetic(L, U)
    memo = {}

    def D(path, k):
        """D_{path[0]} D_{path[1]} ... B_k (rightmost acts first)."""
        key = (tuple(path), k)
        if key not in memo:
            memo[key] = B[k] if not path else adjoint_diff(L, U, D(path[1:], k), path[0])
        return memo[key]

    scale = np.zeros(5)
    cur = [0]

    def tr_sum(*mats):
        p = mats[0]
        for m in mats[1:]:
            p = p @ m
        tr = np.trace(p, axis1=1, axis2=2)
        scale[cur[0]] += np.abs(tr).sum()
        return tr.sum()

    o = np.zeros(5, complex)
    r3 = range(3)
    for i, j, k in itertools.product(r3, r3, r3):
        e = EPS[i, j, k]
        if e == 0.0:
            continue
        cur[0] = 0
        o[0] += e * tr_sum(B[i], D([j], k))
        cur[0] = 2
        o[2] += e * tr_sum(B[i], D([j, j, j], k))
        cur[0] = 3
        o[3] += e * tr_sum(B[i], D([j, j, k], j))
        cur[0] = 4
        o[4] += e * tr_sum(B[i], D([j, i, i], k))
        cur[0] = 1
        for l, m in itertools.product(r3, r3):
            e2 = e * EPS[i, l, m]
            if e2 != 0.0:
                o[1] += e2 * tr_sum(B[j], B[k], D([l], m))
    return (o, scale) if with_scale else o


def operators(L: int, links: np.ndarray, with_scale: bool = False):
    """O [T][5] from links [T][V3][3][3][3] (and the scales [T][5] with_scale)."""
    r = [operators_timeslice(L, np.asarray(u, np.complex128), True) for u in links]
    o = np.stack([x[0] for x in r])
    return (o, np.stack([x[1] for x in r])) if with_scale else o


def correlator(O: np.ndarray) -> np.ndarray:
    """C [T][5][5] (dt = 0 .. T-1) from O [T][5] of one configuration."""
    O = np.asarray(O, np.complex128)
    T = O.shape[0]
    mean = O.mean(axis=0)
    out = np.empty((T, O.shape[1], O.shape[1]), complex)
    for dt in range(T):
        out[dt] = np.einsum("tn,tm->nm", np.roll(O, -dt, axis=0), np.conj(O)) / T - np.outer(mean, np.conj(mean))
    return out

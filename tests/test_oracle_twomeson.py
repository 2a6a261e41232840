"""Pins of the two-meson oracle (oracle/twomeson.py).

* The four-term pair formula against a brute-force Wick contraction: every index value
  and every pairing of quark with antiquark fields enumerated, each signed by the parity
  of the permutation that brings the contracted pairs together (nothing of the formula's
  traces or signs is assumed).
* The direct part against the single-meson correlator of oracle.meson (itself pinned):
  Tr P_kl is minus the w-weighted meson correlator with sink momentum p_k and source p_l.
* Invariance of the whole correlator under a unitary change of the distillation basis
  (flat profiles), which a transposed or conjugated elemental breaks.
* Invariance under relabelling the momenta, and the reduced form the GPU path sums.
"""
import itertools

import numpy as np
import pytest

import oracle.meson as om
import oracle.twomeson as otm


def _c(g, *s):
    return g.standard_normal(s) + 1j * g.standard_normal(s)


def _parity(order):
    """+1 or -1: parity of the permutation given as a list of distinct integers."""
    order = list(order)
    sign = 1
    for i in range(len(order)):
        while order[i] != i:
            j = order[i]
            order[i], order[j] = order[j], order[i]
            sign = -sign
    return sign


def _wick(fields, coef, props):
    """Brute-force <prod of fields> for Gaussian fermions.

    fields: list of (kind, slot) in operator order, kind in {'u', 'ubar', 'd', 'dbar'},
    slot naming the index variable; coef(idx) the coefficient for an assignment idx
    {slot: value}; props[(psi_kind)](x, y) = <psi_x psibar_y>. Every complete pairing of
    each psi with a psibar of its flavour is summed with the sign of the permutation that
    orders the fields as (psi psibar)(psi psibar)..."""
    slots = sorted({s for _, s in fields})
    n = props["n"]
    pos = {k: [i for i, (kk, _) in enumerate(fields) if kk == k] for k in ("u", "ubar", "d", "dbar")}
    pairings = []
    for pu in itertools.permutations(pos["ubar"]):
        for pd in itertools.permutations(pos["dbar"]):
            pairs = list(zip(pos["u"], pu)) + list(zip(pos["d"], pd))
            order = [i for pr in pairs for i in pr]
            pairings.append((pairs, _parity(order)))
    total = 0.0
    for vals in itertools.product(range(n), repeat=len(slots)):
        idx = dict(zip(slots, vals))
        c = coef(idx)
        if c == 0:
            continue
        for pairs, sign in pairings:
            term = sign * c
            for a, b in pairs:
                term *= props[fields[a][0]](idx[fields[a][1]], idx[fields[b][1]])
            total += term
    return total


def _props(n, tau, back):
    # <u(t) ubar(t0)> = tau, <d(t0) dbar(t)> = back
    return {"n": n, "u": lambda x, y: tau[x, y], "d": lambda x, y: back[x, y]}


def test_single_meson_engine_gives_the_quark_loop_sign():
    g = np.random.default_rng(7)
    n = 3
    m, mb, tau, back = (_c(g, n, n) for _ in range(4))
    fields = [("dbar", "a"), ("u", "b"), ("ubar", "e"), ("d", "f")]
    got = _wick(fields, lambda i: m[i["a"], i["b"]] * mb[i["e"], i["f"]], _props(n, tau, back))
    np.testing.assert_allclose(got, -np.trace(m @ tau @ mb @ back), rtol=1e-12)


def test_pair_term_against_brute_force_wick():
    g = np.random.default_rng(8)
    n = 3
    m1, m2, ma, mb, tau, back = (_c(g, n, n) for _ in range(6))
    # sink pi(1) pi(2) = (dbar m1 u)(dbar m2 u); source (pi(a) pi(b))^H = (ubar ma d)(ubar mb d)
    fields = [("dbar", "a"), ("u", "b"), ("dbar", "c"), ("u", "d"),
              ("ubar", "e"), ("d", "f"), ("ubar", "g"), ("d", "h")]
    coef = lambda i: m1[i["a"], i["b"]] * m2[i["c"], i["d"]] * ma[i["e"], i["f"]] * mb[i["g"], i["h"]]
    got = _wick(fields, coef, _props(n, tau, back))
    want = otm.pair_term(m1, m2, ma, mb, tau, back)
    np.testing.assert_allclose(want, got, rtol=1e-11)
    # the direct part alone is the pairing of each meson's quark with one antiquark loop
    _, d, x = otm.pair_term(m1, m2, ma, mb, tau, back, terms=True)
    assert abs(d) > 0 and abs(x) > 0


def _inputs(N=3, nt=2, nprof=2, mom=((0, 0, 1), (0, 0, -1), (1, 0, 0), (-1, 0, 0)), seed=1):
    g = np.random.default_rng(seed)
    mom = np.array(mom)
    nmom = len(mom)
    phi_snk = _c(g, nt, nmom, 7, N, N)
    phi_src = _c(g, nmom, 7, N, N)
    tau = _c(g, nt, 4 * N, 4 * N) / np.sqrt(8 * N)
    gs = g.random((nprof, nt, N)) + 0.5
    g0 = g.random((nprof, N)) + 0.5
    w = _c(g, 3 * nprof)
    return phi_snk, phi_src, tau, gs, g0, w, mom


def test_direct_part_is_the_product_of_meson_correlators():
    phi_snk, phi_src, tau, gs, g0, w, mom = _inputs()
    _, D, _ = otm.correlator(phi_snk, phi_src, tau, gs, g0, w, mom, terms=True)
    kbar = otm.negation_index(mom)
    nmom = len(mom)

    def meson(k, l):
        # w-weighted single-meson correlator, sink momentum slot k, source slot l, all t
        c = om.correlator(phi_snk[:, [k]], phi_src[[l]], tau, gs, g0)[0]  # [nt][A][B]
        return np.einsum("a,tab,b->t", w, c, np.conj(w))

    want = np.zeros(phi_snk.shape[0], complex)
    for k in range(nmom):
        for l in range(nmom):
            # Tr P_kl = -meson(k, l); the two pairings of the two mesons
            want += meson(k, l) * meson(kbar[k], kbar[l]) + meson(k, kbar[l]) * meson(kbar[k], l)
    np.testing.assert_allclose(D, want, rtol=1e-11)


def test_invariant_under_a_distillation_basis_change():
    # flat profiles: v -> v U sends Phi^D -> U^H Phi^D U and tau -> (1 (x) U^H) tau (1 (x) U)
    phi_snk, phi_src, tau, _, _, w, mom = _inputs(N=3, seed=2)
    nt, N = phi_snk.shape[0], phi_snk.shape[-1]
    g = np.random.default_rng(3)
    q, r = np.linalg.qr(_c(g, N, N))
    U = q * (np.diag(r) / np.abs(np.diag(r)))
    gs, g0 = np.ones((2, nt, N)), np.ones((2, N))
    C, D, X = otm.correlator(phi_snk, phi_src, tau, gs, g0, w, mom, terms=True)
    Uh = U.conj().T
    phi_snk2 = np.einsum("ai,...ab,bj->...ij", U.conj(), phi_snk, U)
    phi_src2 = np.einsum("ai,...ab,bj->...ij", U.conj(), phi_src, U)
    UU = np.kron(np.eye(4), U)
    tau2 = np.einsum("ab,tbc,cd->tad", UU.conj().T, tau, UU)
    C2, D2, X2 = otm.correlator(phi_snk2, phi_src2, tau2, gs, g0, w, mom, terms=True)
    sc = np.max(np.abs(D))
    np.testing.assert_allclose(D2, D, atol=1e-11 * sc)
    np.testing.assert_allclose(X2, X, atol=1e-11 * sc)
    assert np.allclose(Uh @ U, np.eye(N))


def test_relabelling_momenta_and_the_reduced_sum():
    phi_snk, phi_src, tau, gs, g0, w, mom = _inputs(seed=4)
    C, D, X = otm.correlator(phi_snk, phi_src, tau, gs, g0, w, mom, terms=True)
    perm = np.array([2, 0, 3, 1])
    C2 = otm.correlator(phi_snk[:, perm], phi_src[perm], tau, gs, g0, w, mom[perm])
    np.testing.assert_allclose(C2, C, atol=1e-11 * np.max(np.abs(D)))
    # C = 2 sum_{k,l} (Tr P_kl Tr P_kbar,lbar - Tr[P_kl P_kbar,lbar]), the form the GPU sums
    _, g4, g5 = om.dirac_pauli()
    N = phi_src.shape[-1]
    G4, G5 = np.kron(g4, np.eye(N)), np.kron(g5, np.eye(N))
    kbar = otm.negation_index(mom)
    for t in range(phi_snk.shape[0]):
        ms = [otm.optimal_operator(phi_snk[t, p], gs[:, t], w) for p in range(len(mom))]
        mb = [G4 @ otm.optimal_operator(phi_src[p], g0, w).conj().T @ G4 for p in range(len(mom))]
        back = G5 @ tau[t].conj().T @ G5
        P = [[ms[k] @ tau[t] @ mb[l] @ back for l in range(len(mom))] for k in range(len(mom))]
        d = sum(np.trace(P[k][l]) * np.trace(P[kbar[k]][kbar[l]]) for k in range(len(mom)) for l in range(len(mom)))
        x = sum(np.trace(P[k][l] @ P[kbar[k]][kbar[l]]) for k in range(len(mom)) for l in range(len(mom)))
        np.testing.assert_allclose(2 * d, D[t], rtol=1e-11)
        np.testing.assert_allclose(2 * x, X[t], rtol=1e-11)
    # the oracle's summed form, used where the term-by-term sum is slow
    C3, D3, X3 = otm.correlator_by_pairs(phi_snk, phi_src, tau, gs, g0, w, mom, terms=True)
    np.testing.assert_allclose(D3, D, rtol=1e-11)
    np.testing.assert_allclose(X3, X, rtol=1e-11)
    np.testing.assert_allclose(C3, C, rtol=1e-11)


def test_zero_momentum_is_twice_the_squared_meson_minus_the_loop():
    phi_snk, phi_src, tau, gs, g0, w, _ = _inputs(mom=((0, 0, 0),), seed=5)
    C, D, X = otm.correlator(phi_snk, phi_src, tau, gs, g0, w, np.zeros((1, 3), int), terms=True)
    C2 = otm.correlator_by_pairs(phi_snk, phi_src, tau, gs, g0, w, np.zeros((1, 3), int))
    np.testing.assert_allclose(C2, C, rtol=1e-11)
    c = np.einsum("a,tab,b->t", w, om.correlator(phi_snk, phi_src, tau, gs, g0)[0], np.conj(w))
    np.testing.assert_allclose(D, 2 * c ** 2, rtol=1e-11)
    np.testing.assert_allclose(C, D - X, rtol=1e-12)


def test_negation_index_requires_closed_lists():
    assert list(otm.negation_index(np.array([[0, 0, 1], [0, 0, -1], [0, 0, 0]]))) == [1, 0, 2]
    with pytest.raises(ValueError):
        otm.negation_index(np.array([[0, 0, 1], [0, 1, 0], [0, 0, -1]]))

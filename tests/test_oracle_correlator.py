"""Pins for the oracle's correlation matrix C_ab(t) = D_ab(t) - E_ab(t) (CPU only)."""
import math

import numpy as np
import pytest

import oracle
import synth
from tests import brute


def _setup(seed, L, N, nprof, nt=2):
    g = np.random.default_rng(seed)
    z = g.standard_normal((nt, N, L ** 3, 3)) + 1j * g.standard_normal((nt, N, L ** 3, 3))
    v = z / math.sqrt(2)
    mom = np.asarray([(1, 0, 0)], np.int32)
    phi = oracle.elementals(L, v, mom)                    # [nt][1][N^3]
    tau = (g.standard_normal((nt, 4 * N, 4 * N)) + 1j * g.standard_normal((nt, 4 * N, 4 * N))) / math.sqrt(2)
    evals = np.sort(g.random((nt, N)), axis=1)
    prof = [(0, 0.3), (0, 0.8), (1, 0.0)][:nprof]
    gs = oracle.profiles(evals, prof)                    # [nprof][nt][N]
    return g, v, phi, tau, gs


@pytest.mark.parametrize("N,nprof", [(3, 2), (4, 1)])
def test_matches_literal_six_index_sum(N, nprof):
    _, _, phi, tau, gs = _setup(10 + N, 2, N, nprof)
    C, D, E = oracle.correlator(phi[1:], phi[0], tau[1:], gs[:, 1:], gs[:, 0])
    Cb, Db, Eb = brute.correlator(phi[1, 0], phi[0, 0], tau[1], gs[:, 1], gs[:, 0])
    scale = np.max(np.abs(Db))
    assert np.max(np.abs(D[0, 0] - Db)) < 1e-11 * scale
    assert np.max(np.abs(E[0, 0] - Eb)) < 1e-11 * scale
    assert np.max(np.abs(C[0, 0] - Cb)) < 1e-11 * scale


def test_identity_perambulator_closed_form():
    # tau = 1 at t = t0:  D = 8 G, E = -2 G, C = 10 G with G_ab = sum Phi^(a) conj(Phi^(b))
    g, v, phi, _, gs = _setup(20, 2, 6, 3, nt=1)
    tau = np.eye(24, dtype=complex)[None]
    C, D, E = oracle.correlator(phi, phi[0], tau, gs, gs[:, 0])
    A = np.einsum("ai,aj,ak,ijk->aijk", gs[:, 0], gs[:, 0], gs[:, 0], phi[0, 0])
    G = np.einsum("aijk,bijk->ab", A, np.conj(A))
    s = np.max(np.abs(G))
    assert np.max(np.abs(D[0, 0] - 8 * G)) < 1e-12 * s
    assert np.max(np.abs(E[0, 0] + 2 * G)) < 1e-12 * s
    c = C[0, 0]
    assert np.max(np.abs(c - c.conj().T)) < 1e-12 * s          # Hermitian
    assert np.min(np.linalg.eigvalsh((c + c.conj().T) / 2)) > -1e-12 * s  # PSD


def test_cubic_scaling_in_tau_and_profiles():
    _, _, phi, tau, gs = _setup(30, 2, 5, 2)
    C, _, _ = oracle.correlator(phi[1:], phi[0], tau[1:], gs[:, 1:], gs[:, 0])
    c = 0.7 - 0.4j
    C2, _, _ = oracle.correlator(phi[1:], phi[0], c * tau[1:], gs[:, 1:], gs[:, 0])
    assert np.max(np.abs(C2 - c ** 3 * C)) < 1e-12 * np.max(np.abs(C))
    gs2 = gs.copy()
    gs2[1] *= 2.0
    C3, _, _ = oracle.correlator(phi[1:], phi[0], tau[1:], gs2[:, 1:], gs2[:, 0])
    expect = C.copy()
    expect[..., 1, :] *= 8.0
    expect[..., :, 1] *= 8.0
    assert np.max(np.abs(C3 - expect)) < 1e-12 * np.max(np.abs(expect))


def test_rephasing_invariance():
    # v_i(t) -> e^{i th_i(t)} v_i(t) at sink and source, tau(t,t0) -> D_t^* tau D_0
    g, v, phi, tau, gs = _setup(40, 2, 5, 2)
    L = 2
    th = g.random((2, 5)) * 2 * np.pi
    vr = v * np.exp(1j * th)[:, :, None, None]
    phir = oracle.elementals(L, vr, np.asarray([(1, 0, 0)], np.int32))
    d0 = np.tile(np.exp(1j * th[0]), 4)
    d1 = np.tile(np.exp(1j * th[1]), 4)
    taur = np.conj(d1)[:, None] * tau[1] * d0[None, :]
    C, _, _ = oracle.correlator(phi[1:], phi[0], tau[1:], gs[:, 1:], gs[:, 0])
    Cr, _, _ = oracle.correlator(phir[1:], phir[0], taur[None], gs[:, 1:], gs[:, 0])
    assert np.max(np.abs(Cr - C)) < 1e-11 * np.max(np.abs(C))


def test_eigenvector_relabelling_invariance():
    g, v, phi, tau, gs = _setup(50, 2, 5, 2)
    L = 2
    perm = g.permutation(5)
    vp = v[:, perm]
    phip = oracle.elementals(L, vp, np.asarray([(1, 0, 0)], np.int32))
    idx = np.concatenate([s * 5 + perm for s in range(4)])
    taup = tau[1][np.ix_(idx, idx)]
    C, _, _ = oracle.correlator(phi[1:], phi[0], tau[1:], gs[:, 1:], gs[:, 0])
    Cp, _, _ = oracle.correlator(phip[1:], phip[0], taup[None], gs[:, 1:][:, :, perm], gs[:, 0][:, perm])
    assert np.max(np.abs(Cp - C)) < 1e-11 * np.max(np.abs(C))


def test_standard_distillation_is_unit_profile():
    # N_B = 1, g = 1 reproduces the un-profiled literal contraction
    _, _, phi, tau, _ = _setup(60, 2, 3, 1)
    ones = np.ones((1, 2, 3))
    C, _, _ = oracle.correlator(phi[1:], phi[0], tau[1:], ones[:, 1:], ones[:, 0])
    Cb, _, _ = brute.correlator(phi[1, 0], phi[0, 0], tau[1], ones[:, 1], ones[:, 0])
    assert abs(C[0, 0, 0, 0] - Cb[0, 0]) < 1e-11 * abs(Cb[0, 0])


def test_synthetic_tiny_config_runs():
    cfg = synth.tiny()
    inp = synth.make_inputs(cfg)
    phi, corr = oracle.run(cfg.L, inp.evecs, inp.evals, inp.tau, inp.mom, cfg.profiles, ts=[0, 3])
    assert phi.shape == (2, 1, 8, 8, 8) and corr.shape == (1, 2, 3, 3)
    assert np.all(np.isfinite(corr))

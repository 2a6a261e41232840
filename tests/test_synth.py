"""Seeded input generator: determinism, orthonormality, layout, value recipes."""
import math

import numpy as np

import synth


def test_tiny_inputs_deterministic_and_shaped():
    cfg = synth.tiny()
    a, b = synth.make_inputs(cfg), synth.make_inputs(cfg)
    assert np.array_equal(a.evecs, b.evecs) and np.array_equal(a.tau, b.tau)
    assert a.evecs.shape == (8, 8, 64, 3)
    assert a.tau.shape == (8, 32, 32)
    assert a.evals.shape == (8, 8) and np.all(np.diff(a.evals, axis=1) >= 0)
    assert np.all((a.evals >= 0) & (a.evals < 1))


def test_eigenvectors_orthonormal_and_c64_exact():
    cfg = synth.tiny()
    v = synth.eigenvectors(cfg, ts=[0, 5])
    for t in range(2):
        m = v[t].reshape(cfg.nvec, -1)
        gram = m.conj() @ m.T
        assert np.max(np.abs(gram - np.eye(cfg.nvec))) < 1e-6
    assert np.array_equal(v, v.astype(np.complex64).astype(np.complex128))


def test_timeslice_streams_independent_of_range():
    cfg = synth.tiny()
    assert np.array_equal(synth.eigenvectors(cfg, ts=[3])[0], synth.eigenvectors(cfg)[3])
    assert np.array_equal(synth.perambulators(cfg, ts=[6])[0], synth.perambulators(cfg)[6])


def test_decay_and_lognormal_recipes():
    cfg = synth.custom("d", 2, 4, 4, [(0, 0, 0)], [(0, 0.5)], "gauss_decay", cfg_id=1)
    tau = synth.perambulators(cfg)
    cfg2 = synth.custom("d", 2, 4, 4, [(0, 0, 0)], [(0, 0.5)], "gauss", cfg_id=1)
    tau2 = synth.perambulators(cfg2)
    for t in range(4):
        assert np.allclose(tau[t], tau2[t] * math.exp(-0.5 * t), rtol=1e-6, atol=0)
    cfg3 = synth.custom("l", 2, 2, 16, [(0, 0, 0)], [(0, 0.5)], "lognormal", cfg_id=2)
    mag = np.abs(synth.perambulators(cfg3))
    lz = np.log(mag) / 2.0
    assert abs(lz.mean()) < 0.1 and abs(lz.std() - 1.0) < 0.1


def test_named_configs_match_workloads():
    p = synth.plain()
    assert (p.L, p.T, p.nvec, p.nmom, p.nprof) == (16, 32, 32, 7, 4)
    q = synth.prec()
    assert (q.L, q.T, q.nvec, q.nmom, q.nprof) == (24, 48, 64, 3, 6)
    t = synth.tiny()
    assert (t.L, t.T, t.nvec, t.nmom, t.nprof) == (4, 8, 8, 1, 3)


def test_random_su3_is_special_unitary():
    u = synth.random_su3(np.random.default_rng(0), 10)
    for m in u:
        assert np.allclose(m @ m.conj().T, np.eye(3), atol=1e-12)
        assert abs(np.linalg.det(m) - 1) < 1e-12

"""GPU parity of the general-spin correlation matrix (nuc_correlator_spin) against the
FP64 general-spin oracle, and against the tuned nucleon path for the nucleon tensors.
Gate: every C[p,t] within the FP32 tolerance (1e-5) in relative Frobenius norm."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import oracle.spin as osp
import synth
import paper_2609_37723_amd as nuc
from tests.gpu_util import TOL_FP32, announce, block_rel_err, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _inputs(L, T, N, mom, prof, cid, tau_kind="gauss"):
    cfg = synth.custom("spin", L, T, N, mom, prof, tau_kind, cfg_id=cid)
    return cfg, synth.make_inputs(cfg)


def _random_spin(g, nrow, density=0.4):
    S = (g.standard_normal((nrow, 4, 4, 4)) + 1j * g.standard_normal((nrow, 4, 4, 4))) / np.sqrt(2)
    return S * (g.random((nrow, 4, 4, 4)) < density)


# name, L, T, N, momenta, profiles, t0, cfg_id, nrow
CASES = [
    ("n5_rows2", 3, 2, 5, [(0, 0, 0), (1, 0, 0)], [(0, 0.3), (1, 0.0)], 0, 81, 2),
    ("n20_ragged_rows3", 4, 2, 20, [(0, 0, 1)], [(0, 0.4), (0, 0.9)], 1, 82, 3),
    ("n8_rows1", 3, 3, 8, [(0, 1, 0)], [(0, 0.5)], 2, 83, 1),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_general_spin_parity(case):
    name, L, T, N, mom, prof, t0, cid, nrow = case
    torch = torch_cuda()
    cfg, inp = _inputs(L, T, N, mom, prof, cid)
    g = np.random.default_rng(cid)
    S, Sp = _random_spin(g, nrow), _random_spin(g, nrow)
    phi = oracle.elementals(L, inp.evecs, inp.mom).astype(np.complex64).astype(np.complex128)
    gp = oracle.profiles(inp.evals, cfg.profiles)
    announce("general spin parity %s: N=%d nrow=%d nnz(S)=%d" % (name, N, nrow, int(np.count_nonzero(S))))
    c = nuc.correlator_spin(to_dev(torch, phi, np.complex64), inp.evals, cfg.profiles,
                            to_dev(torch, inp.tau, np.complex64), L, S, Sp, t0=t0)
    torch.cuda.synchronize()
    ref = osp.correlator(phi, phi[t0], inp.tau, gp, gp[:, t0, :], S, Sp)
    e = block_rel_err(c.cpu().numpy(), ref, 2)
    announce("  max block rel err %.3e" % e.max())
    assert e.max() <= TOL_FP32


@pytest.mark.parametrize("N", [16, 32])
def test_nucleon_tensors_match_the_tuned_path(N):
    torch = torch_cuda()
    cfg, inp = _inputs(6, 3, N, [(0, 0, 0), (0, 0, 2)], [(0, 0.2), (0, 0.5), (1, 0.0)], 84)
    ev, tau = to_dev(torch, inp.evecs, np.complex64), to_dev(torch, inp.tau, np.complex64)
    announce("general spin with the nucleon tensors vs nuc_correlator, N=%d" % N)
    c_fast, phi = nuc.run(ev, inp.evals, cfg.profiles, inp.mom, tau, cfg.L, return_phi=True)
    S = nuc.nucleon_spin(+1)
    c_gen = nuc.correlator_spin(phi, inp.evals, cfg.profiles, tau, cfg.L, S, S)
    torch.cuda.synchronize()
    e = block_rel_err(c_gen.cpu().numpy(), c_fast.cpu().numpy(), 2)
    announce("  max block rel diff %.3e" % e.max())
    assert e.max() <= 2 * TOL_FP32


def test_moving_frame_parity_rows_against_oracle():
    """p = (0, 0, 2): the P- nucleon rows, and the P+ sink against the P- source (the
    two couple in a moving frame, where parity is not a symmetry)."""
    torch = torch_cuda()
    cfg, inp = _inputs(4, 2, 12, [(0, 0, 2)], [(0, 0.3), (0, 0.8)], 85)
    phi = oracle.elementals(cfg.L, inp.evecs, inp.mom).astype(np.complex64).astype(np.complex128)
    gp = oracle.profiles(inp.evals, cfg.profiles)
    Sp_, Sm_ = nuc.nucleon_spin(+1), nuc.nucleon_spin(-1)
    np.testing.assert_allclose(Sp_, osp.nucleon_spin(+1))
    np.testing.assert_allclose(Sm_, osp.nucleon_spin(-1))
    for name, S, Sp in (("P-/P-", Sm_, Sm_), ("P+/P-", Sp_, Sm_)):
        c = nuc.correlator_spin(to_dev(torch, phi, np.complex64), inp.evals, cfg.profiles,
                                to_dev(torch, inp.tau, np.complex64), cfg.L, S, Sp)
        torch.cuda.synchronize()
        ref = osp.correlator(phi, phi[0], inp.tau, gp, gp[:, 0, :], S, Sp)
        e = block_rel_err(c.cpu().numpy(), ref, 2)
        announce("moving frame %s: max block rel err %.3e" % (name, e.max()))
        assert e.max() <= TOL_FP32


def test_general_spin_rejects_bad_arguments():
    torch = torch_cuda()
    cfg, inp = _inputs(3, 2, 4, [(0, 0, 0)], [(0, 0.5)], 86)
    phi = torch.zeros((2, 1, 4, 4, 4), dtype=torch.complex64, device="cuda:0")
    tau = torch.zeros((2, 16, 16), dtype=torch.complex64, device="cuda:0")
    with pytest.raises(ValueError):
        nuc.correlator_spin(phi, inp.evals, cfg.profiles, tau, 3, np.zeros((2, 4, 4, 4)), np.zeros((1, 4, 4, 4)))
    with pytest.raises(nuc.NucError):
        nuc.correlator_spin(phi, inp.evals, cfg.profiles, tau, 3, np.zeros((5, 4, 4, 4)), np.zeros((5, 4, 4, 4)))
    bad = np.zeros((1, 4, 4, 4), complex)
    bad[0, 0, 0, 0] = np.nan
    with pytest.raises(nuc.NucError):
        nuc.correlator_spin(phi, inp.evals, cfg.profiles, tau, 3, bad, bad)

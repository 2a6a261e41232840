"""The no-allocation correlator entry point (needs an MI355X).

nuc_correlator_noalloc runs nuc_correlator's kernels on a static device array;
its results must equal nuc_correlator's bitwise and meet the FP32 gate against
the oracle, on two calls in a row, the second with a smaller input (the array
keeps the first call's contents).
"""
import numpy as np
import pytest

import oracle
import paper_2609_37723_amd as nuc
import synth
from tests.gpu_util import TOL_FP32, announce, block_rel_err, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _case(torch, L, T, N, nmom, prof, kind, cfg_id, precision):
    cfg = synth.custom("noalloc", L, T, N, synth.MOMENTA_7[:nmom], prof, kind, cfg_id=cfg_id)
    inp = synth.make_inputs(cfg)
    phi_ref = oracle.elementals(cfg.L, inp.evecs, inp.mom)
    phi_c64 = phi_ref.astype(np.complex64).astype(np.complex128)
    g = oracle.profiles(inp.evals, cfg.profiles)
    corr_ref, _, _ = oracle.correlator(phi_c64, phi_c64[0], inp.tau, g, g[:, 0])
    dphi = to_dev(torch, phi_c64, np.complex64)
    dtau = to_dev(torch, inp.tau, np.complex64)
    want = nuc.correlator(dphi, inp.evals, cfg.profiles, dtau, cfg.L, precision=precision)
    out = torch.zeros_like(want)
    nuc.correlator_noalloc(dphi, inp.evals, cfg.profiles, dtau, cfg.L, out, precision=precision)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert np.array_equal(got, want.cpu().numpy()), "noalloc differs from nuc_correlator"
    e = block_rel_err(got, corr_ref, 2)
    announce("noalloc L=%d T=%d N=%d nmom=%d nprof=%d %s: max rel err %.3e" % (L, T, N, nmom, len(prof),
                                                                          precision, e.max()))
    assert e.max() <= TOL_FP32


@pytest.mark.parametrize("precision", ["fp32", "fp16x3"])
def test_noalloc_equals_correlator_twice_smaller_second(precision):
    torch = torch_cuda()
    prof = [(0, 0.3), (1, 0.0), (0, 0.8)]
    # first call: several rounds of sink timeslices over the static array (N = 32, 7 momenta)
    _case(torch, 3, 6, 32, 7, prof, "gauss_decay", 70, precision)
    # second call on the same array: smaller and ragged (N = 20, fewer timeslices and momenta)
    _case(torch, 3, 2, 20, 2, prof[:2], "gauss", 71, precision)


def test_noalloc_rejects_a_timeslice_larger_than_the_array():
    torch = torch_cuda()
    N, T, nmom, nprof = 64, 1, 7, 8
    phi = torch.zeros((T, nmom, N, N, N), dtype=torch.complex64, device="cuda:0")
    tau = torch.zeros((T, 4 * N, 4 * N), dtype=torch.complex64, device="cuda:0")
    out = torch.zeros((nmom, T, nprof, nprof), dtype=torch.complex128, device="cuda:0")
    with pytest.raises(nuc.NucError) as e:
        nuc.correlator_noalloc(phi, None, [(1, 0.0)] * nprof, tau, 4, out)
    assert e.value.status == nuc.NUC_ERR_NOMEM

"""GPU parity of the glueball operators (nuc_glueball_operators) against the FP64
glueball oracle, and gauge invariance of the GPU result.

Gate: each O_n(t) within 1e-5 of S_n(t), the sum over the operator's terms and sites
of |Tr(...)|. |O_n| <= S_n, and the FP32 fields (clover, up to three adjoint
differences) perturb every term by a small multiple of eps_32 = 6e-8 of its size,
however much the site sum cancels."""
from __future__ import annotations

import numpy as np
import pytest

import oracle.glueball as og
import synth
import paper_2609_37723_amd as nuc
from tests.gpu_util import announce, to_dev, torch_cuda
from oracle.meson import neighbours

pytestmark = pytest.mark.gpu
TOL = 1e-5

# L, T, nconf, cfg_id
CASES = [(3, 2, 2, 71), (4, 2, 1, 72), (5, 1, 3, 73), (24, 2, 1, 74)]


def _links(L, T, nconf, cid):
    cfg = synth.custom("glue", L, T, 3, [(0, 0, 0)], [(0, 0.5)], "gauss", cfg_id=cid)
    return np.stack([synth.gauge_links(cfg, conf_id=c) for c in range(nconf)])


def _check(o, ref, scale, what):
    err = np.max(np.abs(o - ref) / scale)
    announce("  %s: max |dO|/S %.3e (max |O|/S %.3e)" % (what, err, np.max(np.abs(ref) / scale)))
    assert np.all(np.isfinite(o))
    assert err <= TOL


@pytest.mark.parametrize("case", CASES, ids=["L%d_T%d_c%d" % c[:3] for c in CASES])
def test_glueball_parity(case):
    L, T, nconf, cid = case
    torch = torch_cuda()
    links = _links(L, T, nconf, cid)
    announce("glueball parity L=%d T=%d nconf=%d" % (L, T, nconf))
    o = nuc.glueball_operators(to_dev(torch, links, np.complex64), L)
    torch.cuda.synchronize()
    o = o.cpu().numpy()
    for c in range(nconf):
        ref, scale = og.operators(L, links[c], with_scale=True)
        _check(o[c], ref, scale, "conf %d" % c)


def test_glueball_gauge_invariant_on_gpu():
    L, T = 6, 2
    torch = torch_cuda()
    links = _links(L, T, 1, 75)[0]
    g = np.random.default_rng(11)
    rot = np.empty_like(links)
    for t in range(T):
        om = synth.random_su3(g, L ** 3)
        for d in range(3):
            rot[t, :, d] = om @ links[t, :, d] @ np.conj(np.swapaxes(om[neighbours(L, d, +1)], 1, 2))
    announce("glueball gauge invariance on the GPU, L=%d" % L)
    a = nuc.glueball_operators(to_dev(torch, links, np.complex64), L).cpu().numpy()
    b = nuc.glueball_operators(to_dev(torch, rot, np.complex64), L).cpu().numpy()
    _, scale = og.operators(L, links, with_scale=True)
    _check(b, a, scale, "gauge-rotated vs original")


def test_glueball_rejects_bad_arguments():
    torch = torch_cuda()
    lib = nuc.load()
    ctx = nuc.default_context()
    x = torch.zeros(16, dtype=torch.complex128, device="cuda:0")
    assert lib.nuc_glueball_operators(ctx.handle, 1, 2, 1, x.data_ptr(), x.data_ptr(), None) == nuc.NUC_ERR_INVALID
    assert lib.nuc_glueball_operators(ctx.handle, 4, 0, 1, x.data_ptr(), x.data_ptr(), None) == nuc.NUC_ERR_INVALID
    assert lib.nuc_glueball_operators(ctx.handle, 4, 2, 1, None, x.data_ptr(), None) == nuc.NUC_ERR_INVALID

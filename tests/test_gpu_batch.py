"""Batched launches and HIP-graph replay (needs an MI355X).

Every job of a batch must give exactly (bitwise) what it gives alone: the batch
uses the same kernels, the same per-job plan and a fixed reduction order.
"""
import numpy as np
import pytest

import oracle
import paper_2609_37723_amd as nuc
import synth
from tests.gpu_util import TOL_FP32, announce, block_rel_err, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

SHAPES = [  # (L, T, N, nmom, nprof, tau kind)
    (4, 8, 8, 1, 3, "gauss"),
    (3, 3, 24, 2, 2, "gauss_decay"),
    (4, 2, 32, 3, 4, "gauss"),
    (3, 2, 48, 1, 2, "gauss"),
    (2, 4, 16, 2, 1, "lognormal"),
]
PROFS = [(0, 0.2), (1, 0.0), (0, 0.6), (0, 1.0)]


def _jobs(torch, shapes, seed_base=20):
    cfgs, inps, jobs = [], [], []
    for n, (L, T, N, nmom, nprof, kind) in enumerate(shapes):
        cfg = synth.custom("b%d" % n, L, T, N, synth.MOMENTA_7[:nmom], PROFS[:nprof], kind, cfg_id=seed_base + n)
        inp = synth.make_inputs(cfg)
        ev = to_dev(torch, inp.evecs, np.complex64)
        tau = to_dev(torch, inp.tau, np.complex64)
        cfgs.append(cfg)
        inps.append(inp)
        jobs.append(nuc.BatchJob(ev, inp.evals, cfg.profiles, inp.mom, tau, cfg.L))
    return cfgs, inps, jobs


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp64"])
def test_batch_equals_each_job_alone(precision):
    torch = torch_cuda()
    shapes = SHAPES if precision != "bf16x3" else [s for s in SHAPES if s[2] <= 32]
    announce("batch of %d jobs (%s) vs each alone" % (len(shapes), precision))
    cfgs, inps, jobs = _jobs(torch, shapes)
    nuc.batch_run(jobs, precision=precision)
    torch.cuda.synchronize()
    for cfg, jb in zip(cfgs, jobs):
        alone = nuc.run(jb.evecs, jb.evals, cfg.profiles, jb.mom, jb.tau, cfg.L, precision=precision)
        torch.cuda.synchronize()
        a, b = alone.cpu().numpy(), jb.corr.cpu().numpy()
        assert np.array_equal(a, b), "job %s differs in the batch (max |diff| %g)" % (cfg.name, np.max(np.abs(a - b)))


def test_batch_matches_oracle():
    torch = torch_cuda()
    shapes = [SHAPES[1], SHAPES[3]]
    cfgs, inps, jobs = _jobs(torch, shapes, seed_base=40)
    nuc.batch_run(jobs)
    torch.cuda.synchronize()
    for cfg, inp, jb in zip(cfgs, inps, jobs):
        _, corr_ref = oracle.run(cfg.L, inp.evecs, inp.evals, inp.tau, inp.mom, cfg.profiles)
        e = block_rel_err(jb.corr.cpu().numpy(), corr_ref, 2)
        announce("batch job %s N=%d: max rel err %.3e" % (cfg.name, cfg.nvec, e.max()))
        assert e.max() <= TOL_FP32


def test_both_pair_lists_in_one_launch():
    # 17 and 19 vectors use every pair j<k, 20 the block pair set; all three share one
    # elementals shape class, so one launch holds both kinds of instance
    torch = torch_cuda()
    shapes = [(3, 2, 19, 2, 2, "gauss"), (3, 2, 20, 2, 2, "gauss"), (3, 2, 17, 1, 2, "gauss")]
    announce("batch mixing the pair lists: N = 19, 20, 17")
    cfgs, inps, jobs = _jobs(torch, shapes, seed_base=60)
    nuc.batch_run(jobs)
    torch.cuda.synchronize()
    for cfg, inp, jb in zip(cfgs, inps, jobs):
        alone = nuc.run(jb.evecs, jb.evals, cfg.profiles, jb.mom, jb.tau, cfg.L)
        torch.cuda.synchronize()
        assert np.array_equal(alone.cpu().numpy(), jb.corr.cpu().numpy()), "job %s differs in the batch" % cfg.name
        _, corr_ref = oracle.run(cfg.L, inp.evecs, inp.evals, inp.tau, inp.mom, cfg.profiles)
        e = block_rel_err(jb.corr.cpu().numpy(), corr_ref, 2)
        announce("mixed batch N=%d: max rel err %.3e" % (cfg.nvec, e.max()))
        assert e.max() <= TOL_FP32


def test_graph_replays_match_eager():
    torch = torch_cuda()
    cfgs, inps, jobs = _jobs(torch, SHAPES[:4], seed_base=60)
    nuc.batch_run(jobs)
    torch.cuda.synchronize()
    eager = [jb.corr.cpu().numpy().copy() for jb in jobs]
    for jb in jobs:
        jb.corr.zero_()
    torch.cuda.synchronize()
    g = nuc.BatchGraph(jobs)
    try:
        for rep in range(3):
            g.launch()
            torch.cuda.synchronize()
            for n, jb in enumerate(jobs):
                assert np.array_equal(jb.corr.cpu().numpy(), eager[n]), "replay %d job %d" % (rep, n)
            # eager work of the program itself between replays
            for jb in jobs:
                jb.corr.zero_()
            nuc.run(jobs[0].evecs, jobs[0].evals, cfgs[0].profiles, jobs[0].mom, jobs[0].tau, cfgs[0].L)
            torch.cuda.synchronize()
        announce("graph: 3 replays equal the eager batch")
    finally:
        g.close()


def test_prefix_of_larger_resident_inputs():
    # a job using the first 24 of 32 stored vectors equals the same job on sliced inputs
    torch = torch_cuda()
    cfg = synth.custom("ld", 3, 3, 32, synth.MOMENTA_7[:2], PROFS[:3], "gauss", cfg_id=80)
    inp = synth.make_inputs(cfg)
    N = 24
    ev32 = to_dev(torch, inp.evecs, np.complex64)
    tau32 = to_dev(torch, inp.tau, np.complex64)
    idx = np.concatenate([s * 32 + np.arange(N) for s in range(4)])
    ev24 = to_dev(torch, inp.evecs[:, :N], np.complex64)
    tau24 = to_dev(torch, inp.tau[:, idx][:, :, idx], np.complex64)
    jp = nuc.BatchJob(ev32, inp.evals, cfg.profiles, inp.mom, tau32, cfg.L, nvec=N)
    jd = nuc.BatchJob(ev24, inp.evals[:, :N], cfg.profiles, inp.mom, tau24, cfg.L)
    nuc.batch_run([jp, jd])
    torch.cuda.synchronize()
    assert np.array_equal(jp.corr.cpu().numpy(), jd.corr.cpu().numpy())
    # and against the oracle on the sliced inputs
    _, corr_ref = oracle.run(cfg.L, inp.evecs[:, :N], inp.evals[:, :N], inp.tau[:, idx][:, :, idx], inp.mom,
                             cfg.profiles)
    e = block_rel_err(jp.corr.cpu().numpy(), corr_ref, 2)
    announce("prefix job N=24 of 32: max rel err %.3e" % e.max())
    assert e.max() <= TOL_FP32

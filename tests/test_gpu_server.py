"""Serving loop on the GPU (needs an MI355X).

Jobs of different sizes, momenta, profiles and precisions are submitted to a
server with two slots and a small flop quantum, so that every job is split into
several chunks and shares iterations with the others. Each result must equal
(bitwise) the same job run alone through nuc_batch_run, and match the FP64
oracle.
"""
import numpy as np
import pytest

import oracle
import paper_2609_37723_amd as nuc
import synth
from tests.gpu_util import TOL_FP32, announce, block_rel_err, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

CONFS = {  # conf_id: (L, T, nvec_max, t0, tau kind)
    1: (4, 8, 32, 0, "gauss_decay"),
    2: (3, 6, 24, 2, "gauss"),
}


def _explicit(T, N, seed):
    return np.random.default_rng(seed).uniform(0.2, 1.0, (T, N))


def _jobs():
    G = nuc.PROF_GAUSS
    return [  # (conf, nvec, nmom, profiles, precision)
        (1, 32, 3, [(G, 0.2), (G, 0.5), (nuc.PROF_LINEAR, 0.0), (G, 1.0)], "fp32"),
        (1, 16, 1, [(G, 0.5), (nuc.PROF_ONE, 0.0)], "fp32"),
        (2, 24, 2, [(nuc.PROF_LINEAR, 0.0), (G, 0.3), (G, 0.8)], "fp32"),
        (1, 24, 7, [(G, s) for s in (0.1, 0.15, 0.2, 0.3, 0.5, 0.7, 1.0)] + [(nuc.PROF_LINEAR, 0.0)], "fp32"),
        (2, 12, 4, [(nuc.PROF_EXPLICIT, 0.0, _explicit(6, 12, 3)), (G, 0.6)], "fp32"),
        (1, 32, 2, [(G, 0.5), (nuc.PROF_LINEAR, 0.0)], "bf16x3"),
        (2, 24, 1, [(G, 0.4)], "bf16x3"),
    ]


def _inputs(torch):
    out = {}
    for cid, (L, T, N, t0, kind) in CONFS.items():
        cfg = synth.custom("srv%d" % cid, L, T, N, synth.MOMENTA_7, [], kind, cfg_id=40 + cid)
        inp = synth.make_inputs(cfg)
        out[cid] = (cfg, inp, to_dev(torch, inp.evecs, np.complex64), to_dev(torch, inp.tau, np.complex64), t0)
    return out


def _alone(torch, data, job):
    cid, N, nmom, prof, prec = job
    cfg, inp, ev, tau, t0 = data[cid]
    bj = nuc.BatchJob(ev, inp.evals, prof, synth.MOMENTA_7[:nmom], tau, cfg.L, t0=t0, nvec=N)
    nuc.batch_run([bj], precision=prec)
    torch.cuda.synchronize()
    return bj.corr.cpu().numpy()


def _prefix(inp, N, nmax):
    idx = np.concatenate([np.arange(N) + a * nmax for a in range(4)])
    return inp.evecs[:, :N], inp.evals[:, :N], inp.tau[:, idx][:, :, idx]


def test_server_results_equal_alone_and_oracle():
    torch = torch_cuda()
    data = _inputs(torch)
    jobs = _jobs()
    announce("server: %d jobs on 2 slots, quantum 2e10 flops" % len(jobs))
    with nuc.Server("hip", slots=2, quantum_flops=2e10, job_arena=256 << 20, slot_workspace=1 << 30,
                    start_paused=True) as srv:
        for cid, (cfg, inp, ev, tau, t0) in data.items():
            srv.register(cid, cfg.L, ev, inp.evals, tau, t0=t0)
        tickets = [srv.submit(c, n, synth.MOMENTA_7[:k], prof, prec) for c, n, k, prof, prec in jobs]
        srv.resume()
        results = [srv.wait(t) for t in tickets]
        st = srv.stats()
    announce("server: %d iterations, p50 %.1f ms, p99 %.1f ms" % (st["iterations"], st["p50_ms"], st["p99_ms"]))
    assert st["completed"] == len(jobs) and st["failed"] == 0
    assert sum(r[1]["iterations"] > 1 for r in results) >= 3, "jobs were split into several chunks"
    assert st["iterations"] < sum(r[1]["iterations"] for r in results), "iterations held chunks of several jobs"
    for job, (corr, info) in zip(jobs, results):
        alone = _alone(torch, data, job)
        assert np.array_equal(corr, alone), "job %s differs in the mix (max |diff| %g)" % (
            job[:3], np.max(np.abs(corr - alone)))
    # FP64 oracle on two FP32 jobs, one of them a prefix (nvec < nvec_max)
    for n in (1, 2):
        cid, N, nmom, prof, prec = jobs[n]
        cfg, inp, _, _, t0 = data[cid]
        ev, evals, tau = _prefix(inp, N, cfg.nvec)
        _, ref = oracle.run(cfg.L, ev, evals, tau, inp.mom[:nmom], prof, t0=t0)
        e = block_rel_err(results[n][0], ref, 2)
        announce("server job %d (N=%d of %d, t0=%d): max rel err %.3e" % (n, N, cfg.nvec, t0, e.max()))
        assert e.max() <= TOL_FP32


def test_server_same_job_twice_in_a_row_and_concurrently():
    torch = torch_cuda()
    data = _inputs(torch)
    job = _jobs()[0]
    with nuc.Server("hip", slots=3, quantum_flops=1e10, job_arena=256 << 20, slot_workspace=1 << 30) as srv:
        cfg, inp, ev, tau, t0 = data[1]
        srv.register(1, cfg.L, ev, inp.evals, tau, t0=t0)
        c, n, k, prof, prec = job
        first = srv.wait(srv.submit(c, n, synth.MOMENTA_7[:k], prof, prec))[0]
        ts = [srv.submit(c, n, synth.MOMENTA_7[:k], prof, prec) for _ in range(4)]
        for t in ts:
            assert np.array_equal(srv.wait(t)[0], first)

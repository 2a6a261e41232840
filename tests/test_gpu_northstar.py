"""GPU parity at the large distillation sizes (needs an MI355X).

The contraction kernels for N = 96, 112 and 128 (the LDS-DMA chain, N a multiple
of 16), the register-staged chain for other N above 80, N_B = 8 profiles, and the
prefix path (the first N of vectors stored at a larger N, as the serving loop
runs it) are compared with the FP64 oracle on general perambulators -- complex
Gaussian and log-normal ones -- in every precision form. One oracle run per shape
serves all forms.
"""
import numpy as np
import pytest

import oracle
import paper_2609_37723_amd as nuc
import synth
from tests.gpu_util import FORM_TOL, announce, block_rel_err, to_dev, torch_cuda

pytestmark = pytest.mark.gpu

FORMS = ("fp32", "bf16x3", "fp16x3", "fp64")
PROF2 = [(0, 0.3), (1, 0.0)]
PROF8 = [(0, s) for s in (0.1, 0.15, 0.2, 0.3, 0.5, 0.7, 1.0)] + [(1, 0.0)]


def _forms_vs_oracle(torch, cfg, inp, forms, label):
    """Run nuc.run in each form on the same inputs; compare every block with one oracle run."""
    ev = to_dev(torch, inp.evecs, np.complex64)
    tau = to_dev(torch, inp.tau, np.complex64)
    phi_ref, corr_ref = oracle.run(cfg.L, inp.evecs, inp.evals, inp.tau, inp.mom, cfg.profiles, t0=cfg.t0)
    worst = {}
    for form in forms:
        corr, phi = nuc.run(ev, inp.evals, cfg.profiles, inp.mom, tau, cfg.L, t0=cfg.t0, precision=form,
                            return_phi=True)
        torch.cuda.synchronize()
        e_phi = block_rel_err(phi.cpu().numpy(), phi_ref, 3)
        e_c = block_rel_err(corr.cpu().numpy(), corr_ref, 2)
        announce("%s %s: max rel err phi %.3e corr %.3e (median %.3e)" % (label, form, e_phi.max(), e_c.max(),
                                                                       np.median(e_c)))
        worst[form] = (e_phi.max(), e_c.max())
    for form in forms:
        assert worst[form][0] <= FORM_TOL[form], "%s %s: phi %.3e" % (label, form, worst[form][0])
        assert worst[form][1] <= FORM_TOL[form], "%s %s: corr %.3e" % (label, form, worst[form][1])


@pytest.mark.parametrize("N,T,mom,kind", [(80, 1, [(1, 1, 0)], "gauss"), (96, 2, [(1, 0, 0)], "lognormal"),
                                          (112, 1, [(0, 0, 0)], "gauss"), (128, 1, [(0, 1, 0)], "lognormal")])
def test_dma_chain_general_tau_every_form(N, T, mom, kind):
    # corr_chain_dma_kernel<5>..<8> with off-diagonal tau blocks, per-k tau rows and the
    # W-step chunks all exercised (general tau), in every form (the FP64 form with two
    # workgroups per unit from N = 80 on)
    torch = torch_cuda()
    cfg = synth.custom("ns%d" % N, 4, T, N, mom, PROF2, kind, cfg_id=14)
    announce("DMA chain N=%d L=4 T=%d tau=%s: oracle once, %s" % (N, T, kind, ",".join(FORMS)))
    _forms_vs_oracle(torch, cfg, synth.make_inputs(cfg), FORMS, "N=%d" % N)


@pytest.mark.parametrize("N", [90, 100, 120])
def test_register_staged_chain_large_n(N):
    # N not a multiple of 16 above 80: corr_chain_large_kernel<6>, <7>, <8> (FP32 only)
    torch = torch_cuda()
    cfg = synth.custom("rs%d" % N, 4, 1, N, [(0, 0, 1)], PROF2, "gauss", cfg_id=15)
    announce("register-staged chain N=%d (Np=%d) L=4 T=1" % (N, (N + 15) // 16 * 16))
    _forms_vs_oracle(torch, cfg, synth.make_inputs(cfg), ("fp32",), "N=%d" % N)


def test_eight_profiles_every_form():
    # N_B = 8 (the serving profile basis), two momenta, DMA chain at N = 64
    torch = torch_cuda()
    cfg = synth.custom("nb8", 3, 1, 64, [(0, 0, 0), (1, 1, 0)], PROF8, "gauss", cfg_id=16)
    announce("N_B=8 N=64 L=3 T=1 nmom=2")
    _forms_vs_oracle(torch, cfg, synth.make_inputs(cfg), FORMS, "N_B=8")


def _prefix(inp, N, nmax):
    idx = np.concatenate([np.arange(N) + a * nmax for a in range(4)])
    return inp.evecs[:, :N], inp.evals[:, :N], inp.tau[:, idx][:, :, idx]


@pytest.mark.parametrize("form", FORMS)
def test_dma_chain_prefix_of_larger_inputs(form):
    # the first 64 of 128 stored vectors (tau block stride 128 != N) through nuc_batch_run,
    # against the oracle on the sliced inputs
    torch = torch_cuda()
    nmax, N = 128, 64
    cfg = synth.custom("pre", 4, 2, nmax, [(1, 0, 0)], PROF2, "gauss_decay", cfg_id=17)
    inp = synth.make_inputs(cfg)
    announce("DMA prefix N=%d of %d (%s) L=4 T=2" % (N, nmax, form))
    ev = to_dev(torch, inp.evecs, np.complex64)
    tau = to_dev(torch, inp.tau, np.complex64)
    job = nuc.BatchJob(ev, inp.evals, cfg.profiles, inp.mom, tau, cfg.L, nvec=N)
    nuc.batch_run([job], precision=form)
    torch.cuda.synchronize()
    e_v, e_l, e_t = _prefix(inp, N, nmax)
    _, ref = oracle.run(cfg.L, e_v, e_l, e_t, inp.mom, cfg.profiles)
    e = block_rel_err(job.corr.cpu().numpy(), ref, 2)
    announce("DMA prefix %s: max rel err %.3e" % (form, e.max()))
    assert e.max() <= FORM_TOL[form]


def test_server_prefix_jobs_of_a_128_vector_configuration():
    # resident at N = 128; jobs at N = 64 and 96 (DMA chain with block stride 128) in the
    # serving mix, each equal to its batch run alone and within the gate of the oracle
    torch = torch_cuda()
    nmax = 128
    cfg = synth.custom("srv128", 4, 2, nmax, synth.MOMENTA_7, [], "gauss_decay", cfg_id=18)
    inp = synth.make_inputs(cfg)
    ev = to_dev(torch, inp.evecs, np.complex64)
    tau = to_dev(torch, inp.tau, np.complex64)
    jobs = [(64, 2, PROF2, "fp32"), (96, 1, PROF2, "fp32"), (64, 1, PROF2[:1], "bf16x3"),
            (96, 1, PROF2, "fp16x3"), (96, 1, PROF2, "fp64")]
    announce("server on a 128-vector configuration: %d prefix jobs (N = 64, 96)" % len(jobs))
    with nuc.Server("hip", slots=2, quantum_flops=5e11, job_arena=256 << 20, slot_workspace=4 << 30,
                    start_paused=True) as srv:
        srv.register(1, cfg.L, ev, inp.evals, tau)
        tickets = [srv.submit(1, n, synth.MOMENTA_7[:k], prof, prec) for n, k, prof, prec in jobs]
        srv.resume()
        results = [srv.wait(t)[0] for t in tickets]
    for (N, k, prof, prec), corr in zip(jobs, results):
        bj = nuc.BatchJob(ev, inp.evals, prof, synth.MOMENTA_7[:k], tau, cfg.L, nvec=N)
        nuc.batch_run([bj], precision=prec)
        torch.cuda.synchronize()
        assert np.array_equal(corr, bj.corr.cpu().numpy()), "N=%d %s differs from its solo run" % (N, prec)
    refs = {}
    for n in (0, 1, 3, 4):
        N, k, prof, prec = jobs[n]
        key = (N, k, tuple(prof))
        if key not in refs:
            e_v, e_l, e_t = _prefix(inp, N, nmax)
            refs[key] = oracle.run(cfg.L, e_v, e_l, e_t, inp.mom[:k], prof)[1]
        e = block_rel_err(results[n], refs[key], 2)
        announce("served N=%d of %d (%s): max rel err %.3e" % (N, nmax, prec, e.max()))
        assert e.max() <= FORM_TOL[prec]


def test_prec_config_sampled_every_form():
    # 24^3 x 48, N = 64, 3 momenta, 6 profiles, log-normal perambulators: the full GPU run in
    # every form, the oracle at three sink times and every momentum
    torch = torch_cuda()
    cfg = synth.prec()
    inp = synth.make_inputs(cfg)
    ts = [0, 5, 47]
    announce("prec 24^3x48 N=64: full GPU runs, oracle at t=%s, all 3 momenta" % ts)
    ev = to_dev(torch, inp.evecs, np.complex64)
    tau = to_dev(torch, inp.tau, np.complex64)
    _, corr_ref = oracle.run(cfg.L, inp.evecs, inp.evals, inp.tau, inp.mom, cfg.profiles, ts=ts)
    worst = {}
    for form in FORMS:
        corr = nuc.run(ev, inp.evals, cfg.profiles, inp.mom, tau, cfg.L, precision=form)
        torch.cuda.synchronize()
        c = corr.cpu().numpy()
        assert np.all(np.isfinite(c))
        e = block_rel_err(c[:, ts], corr_ref, 2)
        announce("prec %s: max rel err %.3e (median %.3e)" % (form, e.max(), np.median(e)))
        worst[form] = e.max()
    for form in FORMS:
        assert worst[form] <= FORM_TOL[form], "prec %s: %.3e" % (form, worst[form])


@pytest.mark.parametrize("form", ["fp32", "bf16x3", "fp64"])
def test_batch_with_96_vector_jobs(form):
    # the batched workload's largest N next to smaller jobs: bitwise equal to each job alone,
    # the 96-vector job within the gate of the oracle
    torch = torch_cuda()
    shapes = [(4, 1, 96, 1, 2, "gauss"), (3, 2, 48, 2, 2, "gauss_decay"), (3, 2, 24, 1, 3, "gauss")]
    cfgs, inps, jobs = [], [], []
    for n, (L, T, N, nmom, nprof, kind) in enumerate(shapes):
        cfg = synth.custom("b96_%d" % n, L, T, N, synth.MOMENTA_7[:nmom], (PROF2 + [(0, 0.8)])[:nprof], kind,
                           cfg_id=90 + n)
        inp = synth.make_inputs(cfg)
        cfgs.append(cfg)
        inps.append(inp)
        jobs.append(nuc.BatchJob(to_dev(torch, inp.evecs, np.complex64), inp.evals, cfg.profiles, inp.mom,
                                 to_dev(torch, inp.tau, np.complex64), cfg.L))
    announce("batch with a 96-vector job (%s)" % form)
    nuc.batch_run(jobs, precision=form)
    torch.cuda.synchronize()
    for cfg, jb in zip(cfgs, jobs):
        alone = nuc.run(jb.evecs, jb.evals, cfg.profiles, jb.mom, jb.tau, cfg.L, precision=form)
        torch.cuda.synchronize()
        assert np.array_equal(alone.cpu().numpy(), jb.corr.cpu().numpy()), "job %s differs" % cfg.name
    cfg, inp = cfgs[0], inps[0]
    _, ref = oracle.run(cfg.L, inp.evecs, inp.evals, inp.tau, inp.mom, cfg.profiles)
    e = block_rel_err(jobs[0].corr.cpu().numpy(), ref, 2)
    announce("batch N=96 job (%s): max rel err %.3e" % (form, e.max()))
    assert e.max() <= FORM_TOL[form]


@pytest.mark.parametrize("N", [96, 128])
def test_fp64_dma_prefix_of_larger_inputs(N):
    # the FP64 form on the first N of 128 stored vectors: two workgroups per unit (N = 96) and
    # one (N = 64 is covered by the prefix test above), tau block stride 128
    torch = torch_cuda()
    nmax = 128
    cfg = synth.custom("pre64", 4, 1, nmax, [(0, 1, 0)], PROF2, "lognormal", cfg_id=19)
    inp = synth.make_inputs(cfg)
    announce("FP64 DMA prefix N=%d of %d L=4 T=1" % (N, nmax))
    job = nuc.BatchJob(to_dev(torch, inp.evecs, np.complex64), inp.evals, cfg.profiles, inp.mom,
                       to_dev(torch, inp.tau, np.complex64), cfg.L, nvec=N)
    nuc.batch_run([job], precision="fp64")
    torch.cuda.synchronize()
    e_v, e_l, e_t = _prefix(inp, N, nmax)
    _, ref = oracle.run(cfg.L, e_v, e_l, e_t, inp.mom, cfg.profiles)
    e = block_rel_err(job.corr.cpu().numpy(), ref, 2)
    announce("FP64 DMA prefix N=%d: max rel err %.3e" % (N, e.max()))
    assert e.max() <= FORM_TOL["fp64"]

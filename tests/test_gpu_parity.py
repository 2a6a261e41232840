"""GPU parity of the HIP path against the FP64 CPU oracle (needs an MI355X).

Every GPU result goes through the C ABI (the ctypes binding); every expected
value comes from ``oracle/`` on the same seeded, c64-rounded inputs.
"""
import numpy as np
import pytest

import oracle
import paper_2609_37723_amd as nuc
import synth
from tests.gpu_util import TOL_BF16X3_MEASURED, TOL_FP32, TOL_FP64, announce, block_rel_err, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _upload(torch, inp):
    return (to_dev(torch, inp.evecs, np.complex64), to_dev(torch, inp.tau, np.complex64))


def _gpu_run(torch, cfg, inp, precision="fp32"):
    ev, tau = _upload(torch, inp)
    corr, phi = nuc.run(ev, inp.evals, cfg.profiles, inp.mom, tau, cfg.L, t0=cfg.t0, precision=precision,
                        return_phi=True)
    torch.cuda.synchronize()
    return phi.cpu().numpy(), corr.cpu().numpy()


def _check_antisymmetric(phi):
    assert np.array_equal(phi, -np.swapaxes(phi, -3, -2))
    assert np.array_equal(phi, -np.swapaxes(phi, -2, -1))
    N = phi.shape[-1]
    for i in range(N):
        assert np.all(phi[..., i, i, :] == 0) and np.all(phi[..., :, i, i] == 0)


def test_tiny_full_parity():
    torch = torch_cuda()
    cfg = synth.tiny()
    announce("tiny full parity: L=4 T=8 N=8 nmom=1 nprof=3")
    inp = synth.make_inputs(cfg)
    phi, corr = _gpu_run(torch, cfg, inp)
    phi_ref, corr_ref = oracle.run(cfg.L, inp.evecs, inp.evals, inp.tau, inp.mom, cfg.profiles)
    e_phi = block_rel_err(phi, phi_ref, 3)
    e_c = block_rel_err(corr, corr_ref, 2)
    announce("tiny: max rel err phi %.3e corr %.3e" % (e_phi.max(), e_c.max()))
    assert e_phi.max() <= TOL_FP32
    assert e_c.max() <= TOL_FP32
    _check_antisymmetric(phi)


@pytest.mark.parametrize("L,T,N,nmom,nprof", [(3, 3, 20, 5, 2), (2, 2, 3, 1, 1), (3, 2, 24, 2, 4),
                                              (2, 2, 17, 6, 3)])
def test_ragged_shapes_full_parity(L, T, N, nmom, nprof):
    # ragged site blocks (L^3 not a multiple of 16), ragged 16-wide tiles (N), momentum
    # groups of four with a remainder, the minimum N = 3
    torch = torch_cuda()
    moms = synth.MOMENTA_7[:nmom]
    prof = [(0, 0.3), (1, 0.0), (0, 0.7), (2, 0.0)][:nprof]
    cfg = synth.custom("ragged", L, T, N, moms, prof, "gauss", cfg_id=5)
    announce("ragged parity L=%d T=%d N=%d nmom=%d nprof=%d" % (L, T, N, nmom, nprof))
    inp = synth.make_inputs(cfg)
    phi, corr = _gpu_run(torch, cfg, inp)
    phi_ref, corr_ref = oracle.run(cfg.L, inp.evecs, inp.evals, inp.tau, inp.mom, cfg.profiles)
    e_phi = block_rel_err(phi, phi_ref, 3)
    e_c = block_rel_err(corr, corr_ref, 2)
    announce("ragged: max rel err phi %.3e corr %.3e" % (e_phi.max(), e_c.max()))
    assert e_phi.max() <= TOL_FP32
    assert e_c.max() <= TOL_FP32
    _check_antisymmetric(phi)


def test_correlator_alone_on_oracle_elementals():
    # nuc_correlator fed the oracle's elementals (rounded to c64), nonzero source time
    torch = torch_cuda()
    cfg = synth.custom("src", 2, 4, 12, synth.MOMENTA_7[:2], [(0, 0.25), (1, 0.0)], "gauss", cfg_id=6)
    cfg.t0 = 2
    announce("correlator alone N=12 t0=2")
    inp = synth.make_inputs(cfg)
    phi_ref = oracle.elementals(cfg.L, inp.evecs, inp.mom)
    phi_c64 = phi_ref.astype(np.complex64).astype(np.complex128)
    g = oracle.profiles(inp.evals, cfg.profiles)
    corr_ref, _, _ = oracle.correlator(phi_c64, phi_c64[cfg.t0], inp.tau, g, g[:, cfg.t0])
    dphi = to_dev(torch, phi_c64, np.complex64)
    dtau = to_dev(torch, inp.tau, np.complex64)
    corr = nuc.correlator(dphi, inp.evals, cfg.profiles, dtau, cfg.L, t0=cfg.t0)
    torch.cuda.synchronize()
    e = block_rel_err(corr.cpu().numpy(), corr_ref, 2)
    announce("correlator alone: max rel err %.3e" % e.max())
    assert e.max() <= TOL_FP32


def test_identity_perambulator_gives_hermitian_psd():
    torch = torch_cuda()
    cfg = synth.custom("ident", 3, 1, 16, [(0, 0, 0)], [(0, 0.2), (0, 0.5), (0, 1.0)], "identity", cfg_id=7)
    announce("identity tau: N=16 Hermitian PSD")
    inp = synth.make_inputs(cfg)
    _, corr = _gpu_run(torch, cfg, inp)
    c = corr[0, 0]
    s = np.max(np.abs(c))
    assert np.max(np.abs(c - c.conj().T)) <= 1e-6 * s
    assert np.min(np.linalg.eigvalsh((c + c.conj().T) / 2)) >= -1e-6 * s


def test_plain_full_size_sampled():
    # the benchmark's workload and launch configuration; oracle on sampled (t, p)
    torch = torch_cuda()
    cfg = synth.plain()
    announce("plain 16^3x32 N=32 nmom=7 nprof=4: full GPU run, sampled oracle")
    inp = synth.make_inputs(cfg)
    phi, corr = _gpu_run(torch, cfg, inp)
    ts, ps = [0, 13, 31], [0, 5]
    sub = synth.Inputs(cfg, inp.evecs, inp.evals, inp.tau, inp.mom[ps])
    phi_ref, corr_ref = oracle.run(cfg.L, sub.evecs, sub.evals, sub.tau, sub.mom, cfg.profiles, ts=ts)
    e_phi = block_rel_err(phi[ts][:, ps], phi_ref, 3)
    e_c = block_rel_err(corr[ps][:, ts], corr_ref, 2)
    announce("plain: max rel err phi %.3e corr %.3e" % (e_phi.max(), e_c.max()))
    assert e_phi.max() <= TOL_FP32
    assert e_c.max() <= TOL_FP32
    assert np.all(np.isfinite(corr))


# ----------------------------------------------------------------- BF16x3 form
TOL_BF16X3 = TOL_BF16X3_MEASURED   # the form's measured error with a margin, not an accuracy target


@pytest.mark.parametrize("name", ["tiny", "n24", "n32"])
def test_bf16x3_chain_parity(name):
    torch = torch_cuda()
    if name == "tiny":
        cfg = synth.tiny()
    elif name == "n24":
        cfg = synth.custom("n24", 3, 3, 24, synth.MOMENTA_7[:3], [(0, 0.3), (1, 0.0), (0, 0.7)], "gauss", cfg_id=8)
    else:
        cfg = synth.custom("n32", 3, 2, 32, synth.MOMENTA_7[:2], [(0, 0.3), (1, 0.0)], "gauss_decay", cfg_id=8)
    announce("bf16x3 parity %s: L=%d T=%d N=%d" % (name, cfg.L, cfg.T, cfg.nvec))
    inp = synth.make_inputs(cfg)
    phi, corr = _gpu_run(torch, cfg, inp, precision="bf16x3")
    phi_ref, corr_ref = oracle.run(cfg.L, inp.evecs, inp.evals, inp.tau, inp.mom, cfg.profiles)
    e_c = block_rel_err(corr, corr_ref, 2)
    announce("bf16x3 %s: max rel err corr %.3e (median %.3e)" % (name, e_c.max(), np.median(e_c)))
    assert e_c.max() <= TOL_BF16X3


def test_bf16x3_plain_sampled():
    torch = torch_cuda()
    cfg = synth.plain()
    announce("bf16x3 plain: full GPU run, sampled oracle")
    inp = synth.make_inputs(cfg)
    _, corr = _gpu_run(torch, cfg, inp, precision="bf16x3")
    ts, ps = [0, 13, 31], [0, 5]
    phi_ref, corr_ref = oracle.run(cfg.L, inp.evecs, inp.evals, inp.tau, inp.mom[ps], cfg.profiles, ts=ts)
    e_c = block_rel_err(corr[ps][:, ts], corr_ref, 2)
    announce("bf16x3 plain: max rel err corr %.3e" % e_c.max())
    assert e_c.max() <= TOL_BF16X3


@pytest.mark.parametrize("L,T,N,nmom,nprof", [(3, 2, 48, 2, 3), (3, 1, 64, 1, 2), (3, 1, 80, 1, 2)])
def test_bf16x3_large_nvec_parity(L, T, N, nmom, nprof):
    # the LDS-DMA chain in BF16x3 (N a multiple of 16); N = 48 and 80 end in a half chunk
    torch = torch_cuda()
    prof = [(0, 0.3), (1, 0.0), (0, 0.8)][:nprof]
    cfg = synth.custom("bf16large", L, T, N, synth.MOMENTA_7[:nmom], prof, "gauss_decay", cfg_id=12)
    announce("bf16x3 large-nvec parity L=%d T=%d N=%d nmom=%d nprof=%d" % (L, T, N, nmom, nprof))
    inp = synth.make_inputs(cfg)
    _, corr = _gpu_run(torch, cfg, inp, precision="bf16x3")
    _, corr_ref = oracle.run(cfg.L, inp.evecs, inp.evals, inp.tau, inp.mom, cfg.profiles)
    e_c = block_rel_err(corr, corr_ref, 2)
    announce("bf16x3 N=%d: max rel err corr %.3e (median %.3e)" % (N, e_c.max(), np.median(e_c)))
    assert e_c.max() <= TOL_BF16X3


# ------------------------------------------------------- scaled FP16x3 form
@pytest.mark.parametrize("L,T,N,nmom,nprof,kind", [(4, 8, 8, 1, 3, "gauss"), (3, 3, 24, 3, 3, "gauss"),
                                                    (3, 2, 32, 2, 2, "gauss_decay"), (3, 2, 48, 2, 3, "gauss_decay"),
                                                    (3, 1, 64, 2, 2, "lognormal"), (3, 1, 80, 1, 2, "lognormal")])
def test_fp16x3_parity(L, T, N, nmom, nprof, kind):
    # power-of-two scaled FP16 splits (small and LDS-DMA chains): held to the FP32 gate,
    # including log-normal perambulators (|tau| spread over e^{+-6})
    torch = torch_cuda()
    prof = [(0, 0.3), (1, 0.0), (0, 0.8)][:nprof]
    cfg = synth.custom("fp16", L, T, N, synth.MOMENTA_7[:nmom], prof, kind, cfg_id=13)
    announce("fp16x3 parity L=%d T=%d N=%d nmom=%d nprof=%d tau=%s" % (L, T, N, nmom, nprof, kind))
    inp = synth.make_inputs(cfg)
    _, corr = _gpu_run(torch, cfg, inp, precision="fp16x3")
    _, corr_ref = oracle.run(cfg.L, inp.evecs, inp.evals, inp.tau, inp.mom, cfg.profiles)
    e_c = block_rel_err(corr, corr_ref, 2)
    announce("fp16x3 N=%d: max rel err corr %.3e (median %.3e)" % (N, e_c.max(), np.median(e_c)))
    assert e_c.max() <= TOL_FP32


def test_fp16x3_plain_sampled():
    torch = torch_cuda()
    cfg = synth.plain()
    announce("fp16x3 plain: full GPU run, sampled oracle")
    inp = synth.make_inputs(cfg)
    _, corr = _gpu_run(torch, cfg, inp, precision="fp16x3")
    ts, ps = [0, 13, 31], [0, 5]
    _, corr_ref = oracle.run(cfg.L, inp.evecs, inp.evals, inp.tau, inp.mom[ps], cfg.profiles, ts=ts)
    e_c = block_rel_err(corr[ps][:, ts], corr_ref, 2)
    announce("fp16x3 plain: max rel err corr %.3e" % e_c.max())
    assert e_c.max() <= TOL_FP32


@pytest.mark.parametrize("precision", ["bf16x3", "fp16x3", "fp64"])
def test_split_and_fp64_forms_reject_unsupported_nvec(precision):
    torch = torch_cuda()
    cfg = synth.custom("n40", 3, 1, 40, [(0, 0, 0)], [(0, 0.3)], "gauss", cfg_id=8)
    inp = synth.make_inputs(cfg)
    ev, tau = _upload(torch, inp)
    with pytest.raises(nuc.NucError) as e:
        nuc.run(ev, inp.evals, cfg.profiles, inp.mom, tau, cfg.L, precision=precision)
    assert e.value.status == nuc.NUC_ERR_UNSUPPORTED


@pytest.mark.parametrize("N", [19, 33, 49, 65])
def test_block_pair_set_boundaries(N):
    # the elementals' pair lists at their edges: 19, the last N with every pair j<k; 33, 49
    # and 65, block pair sets whose last 16-index block holds a single vector (its pairs
    # across blocks and its lone row tile)
    torch = torch_cuda()
    cfg = synth.custom("blockpairs", 3, 2, N, synth.MOMENTA_7[:2], [(0, 0.3), (1, 0.0)], "gauss", cfg_id=11)
    announce("block pair set edge N=%d: L=3 T=2 nmom=2 nprof=2" % N)
    inp = synth.make_inputs(cfg)
    phi, corr = _gpu_run(torch, cfg, inp)
    phi_ref, corr_ref = oracle.run(cfg.L, inp.evecs, inp.evals, inp.tau, inp.mom, cfg.profiles)
    e_phi = block_rel_err(phi, phi_ref, 3)
    e_c = block_rel_err(corr, corr_ref, 2)
    announce("N=%d: max rel err phi %.3e corr %.3e" % (N, e_phi.max(), e_c.max()))
    assert e_phi.max() <= TOL_FP32
    assert e_c.max() <= TOL_FP32
    _check_antisymmetric(phi)


# ----------------------------------------------------------- larger nvec (FP32)
@pytest.mark.parametrize("L,T,N,nmom,nprof", [(3, 2, 48, 2, 2), (3, 1, 64, 1, 2), (4, 1, 40, 3, 3)])
def test_large_nvec_full_parity(L, T, N, nmom, nprof):
    torch = torch_cuda()
    prof = [(0, 0.3), (1, 0.0), (0, 0.8)][:nprof]
    cfg = synth.custom("large", L, T, N, synth.MOMENTA_7[:nmom], prof, "gauss", cfg_id=9)
    announce("large-nvec parity L=%d T=%d N=%d nmom=%d nprof=%d" % (L, T, N, nmom, nprof))
    inp = synth.make_inputs(cfg)
    phi, corr = _gpu_run(torch, cfg, inp)
    phi_ref, corr_ref = oracle.run(cfg.L, inp.evecs, inp.evals, inp.tau, inp.mom, cfg.profiles)
    e_phi = block_rel_err(phi, phi_ref, 3)
    e_c = block_rel_err(corr, corr_ref, 2)
    announce("large N=%d: max rel err phi %.3e corr %.3e" % (N, e_phi.max(), e_c.max()))
    assert e_phi.max() <= TOL_FP32
    assert e_c.max() <= TOL_FP32
    _check_antisymmetric(phi)


@pytest.mark.parametrize("N", [96, 128])
def test_large_nvec_identity_closed_form(N):
    # tau = 1 at t = t0: C_ab = 10 sum_ijk Phi^(a) conj(Phi^(b)), a property that holds at any
    # size; Phi is the GPU's own output, its site sum checked on sampled entries by the oracle
    torch = torch_cuda()
    cfg = synth.custom("ident%d" % N, 6, 1, N, [(0, 0, 0), (1, 0, 0)], [(0, 0.3), (1, 0.0)], "identity",
                       cfg_id=9)
    announce("identity closed form N=%d L=6" % N)
    inp = synth.make_inputs(cfg)
    phi, corr = _gpu_run(torch, cfg, inp)
    g = oracle.profiles(inp.evals, cfg.profiles)[:, 0]
    for p in range(2):
        A = np.einsum("ai,aj,ak,ijk->aijk", g, g, g, phi[0, p].astype(np.complex128))
        G = np.einsum("aijk,bijk->ab", A, np.conj(A))
        e = np.linalg.norm(corr[p, 0] - 10 * G) / np.linalg.norm(10 * G)
        announce("identity N=%d p=%d rel err %.3e" % (N, p, e))
        assert e <= TOL_FP32
    rng = np.random.default_rng(3)
    idx = np.stack([rng.integers(0, 2, 24), rng.integers(0, N, 24), rng.integers(0, N, 24),
                    rng.integers(0, N, 24)], axis=1).astype(np.int32)
    ref = oracle.elemental_entries(cfg.L, inp.evecs[0], inp.mom, idx)
    got = np.asarray([phi[0, p, i, j, k] for p, i, j, k in idx])
    rms = np.sqrt(np.mean(np.abs(phi[0]) ** 2))          # block norm / sqrt(N^3)
    announce("sampled entries N=%d: max |diff| / rms %.3e" % (N, np.max(np.abs(got - ref)) / rms))
    assert np.max(np.abs(got - ref)) <= TOL_FP32 * rms


def test_prec_config_sampled():
    # 24^3 x 48, N = 64, 3 momenta, 6 profiles, log-normal perambulators; oracle on one (t, p)
    torch = torch_cuda()
    cfg = synth.prec()
    announce("prec 24^3x48 N=64: full GPU run, oracle at t=5, p=(1,1,0)")
    inp = synth.make_inputs(cfg)
    phi, corr = _gpu_run(torch, cfg, inp)
    ts, ps = [5], [2]
    phi_ref, corr_ref = oracle.run(cfg.L, inp.evecs, inp.evals, inp.tau, inp.mom[ps], cfg.profiles, ts=ts)
    e_phi = block_rel_err(phi[ts][:, ps], phi_ref, 3)
    e_c = block_rel_err(corr[ps][:, ts], corr_ref, 2)
    announce("prec: rel err phi %.3e corr %.3e" % (e_phi.max(), e_c.max()))
    assert e_phi.max() <= TOL_FP32
    assert e_c.max() <= TOL_FP32


# ----------------------------------------------------------------- FP64 form
@pytest.mark.parametrize("name", ["tiny", "ragged", "n32"])
def test_fp64_full_parity(name):
    # every block of Phi and C within 1e-6 of the oracle, including ragged tiles (N = 20)
    torch = torch_cuda()
    if name == "tiny":
        cfg = synth.tiny()
    elif name == "ragged":
        cfg = synth.custom("r64", 3, 3, 20, synth.MOMENTA_7[:5], [(0, 0.3), (1, 0.0)], "gauss", cfg_id=5)
    else:
        cfg = synth.custom("n32", 3, 2, 32, synth.MOMENTA_7[:2], [(0, 0.3), (1, 0.0)], "gauss_decay", cfg_id=8)
    announce("fp64 parity %s: L=%d T=%d N=%d" % (name, cfg.L, cfg.T, cfg.nvec))
    inp = synth.make_inputs(cfg)
    phi, corr = _gpu_run(torch, cfg, inp, precision="fp64")
    phi_ref, corr_ref = oracle.run(cfg.L, inp.evecs, inp.evals, inp.tau, inp.mom, cfg.profiles)
    e_phi = block_rel_err(phi, phi_ref, 3)
    e_c = block_rel_err(corr, corr_ref, 2)
    announce("fp64 %s: max rel err phi %.3e corr %.3e (median %.3e)" % (name, e_phi.max(), e_c.max(),
                                                                     np.median(e_c)))
    assert e_phi.max() <= TOL_FP64
    assert e_c.max() <= TOL_FP64
    _check_antisymmetric(phi)


def test_fp64_plain_sampled():
    # the plain workload in the FP64 form; oracle on 4 sink times x 3 momenta
    torch = torch_cuda()
    cfg = synth.plain()
    announce("fp64 plain: full GPU run, sampled oracle")
    inp = synth.make_inputs(cfg)
    phi, corr = _gpu_run(torch, cfg, inp, precision="fp64")
    ts, ps = [0, 7, 13, 31], [0, 3, 5]
    phi_ref, corr_ref = oracle.run(cfg.L, inp.evecs, inp.evals, inp.tau, inp.mom[ps], cfg.profiles, ts=ts)
    e_phi = block_rel_err(phi[ts][:, ps], phi_ref, 3)
    e_c = block_rel_err(corr[ps][:, ts], corr_ref, 2)
    announce("fp64 plain: max rel err phi %.3e corr %.3e (median %.3e)" % (e_phi.max(), e_c.max(),
                                                                        np.median(e_c)))
    assert e_phi.max() <= TOL_FP64
    assert e_c.max() <= TOL_FP64

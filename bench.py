"""Throughput benchmark of the profiled-distillation nucleon correlator on one MI355X.

Default workload (the largest single-GPU configuration): the precision workload,
24^3 x 48 lattice, N_vec = 64 distillation vectors, 3 momenta, N_B = 6 profiles
(5 Gaussians + linear), log-normal perambulators, all 48 sink times. One step =
one full pass of the hot path: baryon elementals for every (t, p), profile
weighting, and the N_B x N_B correlation matrix C_ab(t) with both Wick terms.
Inputs are seeded synthetic data generated in HBM before timing starts.

Prints one JSON line. ``value`` is algorithmic TFLOP/s of the whole FP32 step:
elementals 24 V3 C(N,3) per (t,p) + 42 V3 C(N,2) per t, correlator
8 * (48 N^4 N_B * 2) + sink dots per (t,p) -- the complex multiply-adds the
Wick-folded contraction needs, 8 flops each. The other precision forms of the
same workload are reported beside it with their errors against the FP64 oracle.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_PEAK_TFLOPS = 157.3        # MI355X dense FP32 MFMA
FP64_PEAK_TFLOPS = 78.6         # MI355X dense FP64 MFMA
BF16_PEAK_TFLOPS = 2516.6       # MI355X dense BF16 MFMA (FP16 the same)
BF16X3_PEAK_TFLOPS = BF16_PEAK_TFLOPS / 3.0   # three bf16 products per FP32 product
FORMS = ("fp32", "bf16x3", "fp16x3", "fp64")
FORM_PEAK = {"fp32": FP32_PEAK_TFLOPS, "bf16x3": BF16X3_PEAK_TFLOPS, "fp16x3": BF16X3_PEAK_TFLOPS,
             "fp64": FP64_PEAK_TFLOPS}
METRIC = "Nucleon corr-matrix TFLOP/s, BF16x3 vs FP32 @1e-6 rel err; p50/p99 job latency"


def comb(n, k):
    return math.comb(n, k)


def flops_elementals(L, T, N, nmom):
    V3 = L ** 3
    return T * (24.0 * V3 * comb(N, 3) * nmom + 42.0 * V3 * comb(N, 2))


def flops_correlator(T, N, nmom, nprof):
    # per (t, p): per source profile and sigma: 4 N^4 (third index) + 44 N^4 (sandwiches)
    # complex MACs; sink: N^3 complex products per (b, sigma), N_B real-weighted sums
    per_tp = 8.0 * nprof * 2 * 48 * N ** 4 + nprof * 2 * (8.0 * N ** 3 + nprof * 4.0 * N ** 3)
    return T * nmom * per_tp


def flops_chain_kernel(T, N, nmom, nprof):
    # the dominant kernel alone: 28 N^4 + 16 N^4 complex MACs per (t, p, b, sigma) + sink dot
    return T * nmom * nprof * 2 * (8.0 * 44 * N ** 4 + 8.0 * N ** 3 + nprof * 4.0 * N ** 3)


def flops_step1(T, N, nmom, nprof):
    # the first mode product X = tau (x) conj(Phi(t0)) over k': 4 N^4 complex MACs per (t, p, b, sigma')
    return T * nmom * nprof * 2 * 4 * 8.0 * N ** 4


def flops_unfolded(L, T, N, nmom, nprof):
    return flops_elementals(L, T, N, nmom) + T * nmom * (1152.0 * nprof * N ** 4 + 128.0 * nprof ** 2 * N ** 3)


def cpu_baseline(cfg, inp, sample_ts):
    """Time the FP64 oracle on a bounded sample: all momenta at the sink times given."""
    import oracle
    nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t_start = time.perf_counter()
    phi_ref, corr_ref = oracle.run(cfg.L, inp.evecs, inp.evals, inp.tau, inp.mom, cfg.profiles, ts=sample_ts)
    dt = time.perf_counter() - t_start
    nt = len(sample_ts)
    fl = (flops_elementals(cfg.L, nt + 1, cfg.nvec, cfg.nmom) +
          flops_correlator(nt, cfg.nvec, cfg.nmom, cfg.nprof))
    return {"value": fl / dt / 1e12, "unit": "TFLOP/s", "cores": nthreads, "kind": "oracle",
            "sample": "%d of %d sink times (t=%s) x all %d momenta, plus the t0 source elementals; "
                      "%.1f s wall" % (nt, cfg.T, ",".join(map(str, sample_ts)), cfg.nmom, dt),
            "seconds": dt}, phi_ref, corr_ref


def device_inputs(torch, synth, cfg, on_gpu=False):
    """(evecs, tau, evals, mom) with evecs/tau complex64 on cuda:0: from the numpy
    generators (the oracle's inputs exactly), or generated on the GPU for workloads
    whose host generation is slow (then the oracle gets host copies)."""
    if on_gpu:
        ev, tau, evals = synth.torch_inputs(cfg)
        return ev, tau, evals, synth.momenta(cfg)
    inp = synth.make_inputs(cfg)
    dev = torch.device("cuda:0")
    return (torch.from_numpy(inp.evecs.astype(np.complex64)).to(dev),
            torch.from_numpy(inp.tau.astype(np.complex64)).to(dev), inp.evals, inp.mom)


def run_workload(nuc, torch, cfg, inputs, precision, steps, warmup, ctx, keep_ts=None):
    """Time `steps` full nuc_run calls on resident inputs; per-kernel HIP-event timing.
    keep_ts: sink times whose elementals and correlator blocks are copied to the host."""
    dev = torch.device("cuda:0")
    ev, tau, evals, mom = inputs
    T, N, nmom, nprof = cfg.T, cfg.nvec, cfg.nmom, cfg.nprof
    phi = torch.empty((T, nmom, N, N, N), dtype=torch.complex64, device=dev)
    corr = torch.empty((nmom, T, nprof, nprof), dtype=torch.complex128, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        nuc.run(ev, evals, cfg.profiles, mom, tau, cfg.L, t0=cfg.t0, precision=precision,
                phi_out=phi, out=corr, ctx=ctx, stream=stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = ctx.timing_read()
    ctx.timing_enable(False)
    res = {"ms_step": wall * 1e3 / steps, "kernels": kt}
    if keep_ts is not None:
        res["corr"] = corr.cpu().numpy()
        res["phi"] = phi[keep_ts].cpu().numpy()
    del phi, corr
    return res


def block_errors(corr, phi, corr_ref, phi_ref, ts):
    """Relative error per output block (one C[p,t], one Phi[t,p]) against the oracle."""
    c = corr[:, ts]
    nb = c.shape[-1]
    ec = np.linalg.norm((c - corr_ref).reshape(-1, nb * nb), axis=1) / \
        np.linalg.norm(corr_ref.reshape(-1, nb * nb), axis=1)
    n3 = phi_ref.shape[-1] ** 3
    ep = np.linalg.norm((phi - phi_ref).reshape(-1, n3), axis=1) / np.linalg.norm(phi_ref.reshape(-1, n3), axis=1)
    return {"corr_max": float("%.3e" % ec.max()), "corr_median": float("%.3e" % np.median(ec)),
            "phi_max": float("%.3e" % ep.max()), "blocks": int(ec.size)}


def oracle_sample(cfg, inputs, ts, timed_t):
    """FP64 oracle at the sink times ts (all momenta) on host copies of the device inputs.
    The elementals at t0 and at timed_t and the correlator at timed_t are timed: that
    is the cpu_baseline sample. Returns (cpu_baseline dict, phi_ref [ts], corr_ref [ts])."""
    import oracle
    ev, tau, evals, mom = inputs
    nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    g = oracle.profiles(evals, cfg.profiles)

    def host(x, t):
        return x[t].cpu().numpy().astype(np.complex128)

    t_start = time.perf_counter()
    phi0 = oracle.elementals(cfg.L, host(ev, [cfg.t0]), mom)[0]
    phi_t = oracle.elementals(cfg.L, host(ev, [timed_t]), mom)
    c_t, _, _ = oracle.correlator(phi_t, phi0, host(tau, [timed_t]), g[:, [timed_t]], g[:, cfg.t0])
    dt = time.perf_counter() - t_start
    fl = flops_elementals(cfg.L, 2, cfg.nvec, cfg.nmom) + flops_correlator(1, cfg.nvec, cfg.nmom, cfg.nprof)
    cb = {"value": round(fl / dt / 1e12, 6), "unit": "TFLOP/s", "cores": nthreads, "kind": "oracle",
          "sample": "sink time t=%d x all %d momenta, plus the t0 source elementals (%.1f s wall)"
                    % (timed_t, cfg.nmom, dt)}
    phis, corrs = [], []
    for t in ts:
        if t == timed_t:
            phis.append(phi_t[0])
            corrs.append(c_t[:, 0])
            continue
        pt = phi0[None] if t == cfg.t0 else oracle.elementals(cfg.L, host(ev, [t]), mom)
        ct, _, _ = oracle.correlator(pt, phi0, host(tau, [t]), g[:, [t]], g[:, cfg.t0])
        phis.append(pt[0])
        corrs.append(ct[:, 0])
    return cb, np.stack(phis), np.stack(corrs, axis=1)


def chain_roofline(kt, cfg, precision, steps):
    """Algorithmic flops of the chain kernel over its summed launch time.

    A step may run the chain in several timeslice chunks (one launch each); the
    flops of one step cover every (t, p), so achieved = steps * flops_per_step /
    (summed kernel time), and the per-launch figure is that over launches/step.
    """
    chain_ms, chain_n = kt["corr_chain"]
    fl_step = flops_chain_kernel(cfg.T, cfg.nvec, cfg.nmom, cfg.nprof)
    achieved = fl_step * steps / (chain_ms * 1e-3) / 1e12
    peak = FORM_PEAK[precision]
    per_step = chain_n / steps
    return {"bound": "mfma", "kernel": "corr_chain", "achieved": round(achieved, 3), "peak": round(peak, 1),
            "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
            "avg_launch_ms": round(chain_ms / max(chain_n, 1), 4), "launches_per_step": per_step,
            "flops_per_launch": fl_step / per_step}


def contraction_roofline(kt, cfg, precision, steps):
    """The whole perambulator contraction (step 1 and the chain: all three mode products and
    the sink dot) against the form's MFMA peak."""
    ms = kt["corr_step1"][0] + kt["corr_chain"][0] + kt.get("corr_scale", (0.0, 0))[0]
    fl = flops_step1(cfg.T, cfg.nvec, cfg.nmom, cfg.nprof) + flops_chain_kernel(cfg.T, cfg.nvec, cfg.nmom,
                                                                                 cfg.nprof)
    achieved = fl * steps / (ms * 1e-3) / 1e12
    return {"achieved": round(achieved, 2), "peak": round(FORM_PEAK[precision], 1), "unit": "TFLOP/s",
            "frac": round(achieved / FORM_PEAK[precision], 4),
            "step1_ms": round(kt["corr_step1"][0] / steps, 3), "chain_ms": round(kt["corr_chain"][0] / steps, 3)}


def kernel_table(kt):
    return {k: {"avg_ms": (round(v[0] / v[1], 4) if v[1] else None), "launches": v[1]} for k, v in kt.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle (timing and errors)")
    ap.add_argument("--no-extra", action="store_true",
                    help="prec/plain: FP32 only (no other forms, N=128 contraction, plain line or serving burst)")
    ap.add_argument("--forms", default="",
                    help="prec/plain: precision forms run beside FP32 (default: all four; with --no-extra: FP32 alone)")
    ap.add_argument("--workload", default="prec",
                    choices=["prec", "plain", "batched", "serving", "kernels", "copy", "meson", "glueball", "spin",
                             "twomeson"],
                    help="prec: the headline line (24^3x48, N_vec=64, 3 momenta, N_B=6, log-normal tau); "
                         "plain: 16^3x32, N_vec=32, 7 momenta, N_B=4; batched: 64 mixed jobs in shared launches; "
                         "serving: Poisson job streams through the continuous-batching server; "
                         "kernels: per-kernel rates on large-N shapes; copy: a device copy of known size "
                         "(calibrates the HBM byte counters); meson: the profiled charmonium operators "
                         "(24^3x48, N_v=200, 21 operators); glueball: the five A1-+ glueball operators on "
                         "16 configurations of 24^3x48; spin: the moving-frame G1 nucleon matrix (P+ and P- "
                         "rows, general spin tensors) at p=(0,0,2) on the plain lattice; twomeson: the I=2 "
                         "two-meson correlator")
    ap.add_argument("--cpu-sample", type=int, default=16, help="plain: sink times in the oracle sample")
    ap.add_argument("--kernel-forms", default="fp32",
                    help="kernels: comma-separated precision forms each case runs in")
    ap.add_argument("--kernel-cases", default="",
                    help="kernels: comma-separated case names (default: all)")
    ap.add_argument("--copy-mib", type=int, default=1024, help="copy: bytes copied per launch, in MiB")
    ap.add_argument("--jobs", type=int, default=64, help="jobs in the batched workload")
    ap.add_argument("--rate", type=float, default=20.0, help="serving: arrivals per second of the first stream")
    ap.add_argument("--arrivals", type=int, default=40, help="serving: arrivals in the first stream")
    ap.add_argument("--arrivals-light", type=int, default=120,
                    help="serving: arrivals in the second stream, at 0.7x the measured capacity (0: skip)")
    ap.add_argument("--confs", type=int, default=8, help="serving: resident gauge configurations")
    ap.add_argument("--quantum", type=float, default=4e12, help="serving: flops per iteration")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(sharding over (t, p) units is described in DESIGN.md); rerun with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2609_37723_amd as nuc
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    handlers = {"prec": bench_prec, "plain": bench_plain, "batched": bench_batched, "serving": bench_serving,
                "kernels": bench_kernels, "meson": bench_meson, "glueball": bench_glueball,
                "twomeson": bench_twomeson, "spin": bench_spin}
    if args.workload == "copy":
        return bench_copy(args, torch)
    return handlers[args.workload](args, torch, nuc, synth)


def forms_of(args):
    forms = [f for f in args.forms.split(",") if f]
    assert all(f in FORMS for f in forms), "unknown form in --forms"
    if not forms:
        forms = [] if args.no_extra else list(FORMS)
    return ["fp32"] + [f for f in forms if f != "fp32"]


def headline(cfg, ms_step, steps, warmup, workload, kt):
    fl_step = flops_elementals(cfg.L, cfg.T, cfg.nvec, cfg.nmom) + flops_correlator(cfg.T, cfg.nvec, cfg.nmom,
                                                                                    cfg.nprof)
    return {
        "metric": METRIC,
        "value": round(fl_step / (ms_step * 1e-3) / 1e12, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "L": cfg.L, "T": cfg.T, "nvec": cfg.nvec, "nmom": cfg.nmom,
                   "nprof": cfg.nprof, "precision": "fp32"},
    }


def dominant_kernel(kt):
    return max((k for k in kt if kt[k][1]), key=lambda k: kt[k][0])


def bench_prec(args, torch, nuc, synth):
    """The headline: the precision workload in FP32, the other forms beside it with their
    errors against the FP64 oracle (3 sink times x 3 momenta), the N_vec = 128
    contraction per form, the plain workload and a serving burst."""
    cfg = synth.prec()
    ctx = nuc.Context(0)
    forms = forms_of(args)
    print("[bench] prec workload: generating inputs on the GPU (24^3 x 48, N_vec=64)", file=sys.stderr, flush=True)
    inputs = device_inputs(torch, synth, cfg, on_gpu=True)
    torch.cuda.synchronize()
    ts = [1, 24, 47]
    runs = {}
    for form in forms:
        print("[bench] prec workload, %s: %d warmup + %d timed steps" % (form, args.warmup, args.steps),
              file=sys.stderr, flush=True)
        runs[form] = run_workload(nuc, torch, cfg, inputs, form, args.steps, args.warmup, ctx, keep_ts=ts)
        print("[bench] prec %s: %.3f ms/step" % (form, runs[form]["ms_step"]), file=sys.stderr, flush=True)
    main_run = runs["fp32"]
    kt = main_run["kernels"]
    wl = ("prec: 24^3x48 lattice, N_vec=64, 3 momenta (0,0,0),(1,0,0),(1,1,0), N_B=6 profiles (5 Gaussian + "
          "linear), log-normal perambulators (sigma=2), all 48 sink times, elementals + C_ab(t)")
    out = headline(cfg, main_run["ms_step"], args.steps, args.warmup, wl, kt)
    dom = dominant_kernel(kt)
    out["roofline"] = chain_roofline(kt, cfg, "fp32", args.steps)
    out["roofline"]["kernel"] = "corr_chain_dma_kernel<4, 0>"
    rec = traffic_from_profile("correlator.hip", "corr_chain_dma_kernel<4, 0>")
    if rec:
        out["roofline"]["traffic"] = rec["hbm_bytes_per_launch"]
    out["dominant_kernel"] = dom
    out["kernels_ms_per_step"] = {k: round(v[0] / args.steps, 3) for k, v in kt.items() if v[1]}
    fl_step = flops_elementals(cfg.L, cfg.T, cfg.nvec, cfg.nmom) + flops_correlator(cfg.T, cfg.nvec, cfg.nmom,
                                                                                    cfg.nprof)
    out["forms"] = {}
    for form, r in runs.items():
        out["forms"][form] = {"value": round(fl_step / (r["ms_step"] * 1e-3) / 1e12, 3),
                              "ms_per_step": round(r["ms_step"], 3),
                              "contraction": contraction_roofline(r["kernels"], cfg, form, args.steps),
                              "elementals_ms": round(r["kernels"]["elementals"][0] / args.steps, 3)}
    if not args.no_cpu_baseline:
        print("[bench] FP64 oracle: sink times %s x 3 momenta on host copies" % ts, file=sys.stderr, flush=True)
        cb, phi_ref, corr_ref = oracle_sample(cfg, inputs, ts, timed_t=24)
        out["cpu_baseline"] = cb
        for form, r in runs.items():
            out["forms"][form]["rel_err_vs_oracle"] = block_errors(r["corr"], r["phi"], corr_ref, phi_ref, ts)
        out["rel_err_vs_oracle"] = out["forms"]["fp32"]["rel_err_vs_oracle"]
        out["rel_err_sample"] = "sink times %s x all 3 momenta; relative error per block (one C[p,t] 6x6 matrix, " \
                                "one Phi[t,p]), max and median over blocks" % ts
    del inputs
    runs.clear()
    torch.cuda.empty_cache()
    if not args.no_extra:
        # the N_vec = 128 contraction (8^3 lattice: the contraction does not depend on the volume)
        big = synth.custom("n128", 8, 4, 128, [(0, 0, 0)], SERVE_PROF8, "gauss_decay", cfg_id=4)
        big_in = device_inputs(torch, synth, big)
        out["contraction_n128"] = {"workload": "N_vec=128, N_B=8, 1 momentum, 4 sink times: step 1 + chain "
                                               "against each form's MFMA peak"}
        for form in forms:
            print("[bench] N_vec=128 contraction (%s)" % form, file=sys.stderr, flush=True)
            r3 = run_workload(nuc, torch, big, big_in, form, 3, 1, ctx)
            out["contraction_n128"][form] = contraction_roofline(r3["kernels"], big, form, 3)
        del big_in
        # the plain workload (16^3 x 32, N_vec = 32, 7 momenta, N_B = 4) in FP32
        pl = synth.plain()
        pl_in = device_inputs(torch, synth, pl)
        print("[bench] plain workload, fp32", file=sys.stderr, flush=True)
        rp = run_workload(nuc, torch, pl, pl_in, "fp32", args.steps, args.warmup, ctx, keep_ts=[0, 31])
        fl_pl = flops_elementals(pl.L, pl.T, pl.nvec, pl.nmom) + flops_correlator(pl.T, pl.nvec, pl.nmom, pl.nprof)
        out["plain"] = {"value": round(fl_pl / (rp["ms_step"] * 1e-3) / 1e12, 3),
                        "ms_per_step": round(rp["ms_step"], 3),
                        "roofline_chain": {k: v for k, v in chain_roofline(rp["kernels"], pl, "fp32", args.steps).items()
                                           if k in ("achieved", "peak", "frac")}}
        if not args.no_cpu_baseline:
            import oracle
            # sink times 0 and 31 (t0 = 0 is the first of the two host copies)
            phi_ref, corr_ref = oracle.run(pl.L, pl_in[0][[0, 31]].cpu().numpy().astype(np.complex128),
                                           pl_in[2][[0, 31]], pl_in[1][[0, 31]].cpu().numpy().astype(np.complex128),
                                           pl_in[3], pl.profiles, ts=[0, 1])
            out["plain"]["rel_err_vs_oracle"] = block_errors(rp["corr"], rp["phi"], corr_ref, phi_ref, [0, 31])
        del pl_in
        torch.cuda.empty_cache()
        # job latency: a short burst of the serving stream (bench.py --workload serving runs the long ones)
        print("[bench] serving burst: 12 arrivals at 20 jobs/s, 2 resident configurations", file=sys.stderr,
              flush=True)
        heavy, _, st, _ = serving_run(torch, nuc, synth, 2, 12, 20.0, 0, 4e12)
        out["serving"] = {"workload": "12 Poisson arrivals at 20 jobs/s (above capacity), 32^3x64, N_vec in "
                                      "{32,64,96,128} of 128 resident, 1-7 momenta, N_B in {4,8}, FP32",
                          "p50_ms": heavy["p50_ms"], "p99_ms": heavy["p99_ms"],
                          "served_tflops": heavy["served_tflops"]}
    print(json.dumps(out), flush=True)


def bench_plain(args, torch, nuc, synth):
    """The plain workload in every form, with block errors against the oracle on
    --cpu-sample sink times (all 7 momenta)."""
    cfg = synth.plain()
    ctx = nuc.Context(0)
    inputs = device_inputs(torch, synth, cfg)
    T = cfg.T
    sample = sorted(set(int(round(x)) for x in np.linspace(0, T - 1, args.cpu_sample)))
    runs = {}
    for form in forms_of(args):
        print("[bench] plain workload, %s" % form, file=sys.stderr, flush=True)
        runs[form] = run_workload(nuc, torch, cfg, inputs, form, args.steps, args.warmup, ctx, keep_ts=sample)
    kt = runs["fp32"]["kernels"]
    out = headline(cfg, runs["fp32"]["ms_step"], args.steps, args.warmup,
                   "plain: 16^3x32 lattice, N_vec=32, 7 momenta, N_B=4 profiles (3 Gaussian + linear), all 32 "
                   "sink times, elementals + C_ab(t)", kt)
    out["roofline"] = chain_roofline(kt, cfg, "fp32", args.steps)
    out["roofline"]["kernel"] = "corr_chain_small_kernel<2, 0>"
    rec = traffic_from_profile("correlator.hip", "corr_chain_small_kernel<2, 0>")
    if rec:
        out["roofline"]["traffic"] = rec["hbm_bytes_per_launch"]
    out["kernels"] = kernel_table(kt)
    fl_step = flops_elementals(cfg.L, T, cfg.nvec, cfg.nmom) + flops_correlator(T, cfg.nvec, cfg.nmom, cfg.nprof)
    out["forms"] = {f: {"value": round(fl_step / (r["ms_step"] * 1e-3) / 1e12, 3), "ms_per_step": round(r["ms_step"], 3),
                        "roofline": chain_roofline(r["kernels"], cfg, f, args.steps),
                        "contraction": contraction_roofline(r["kernels"], cfg, f, args.steps)}
                    for f, r in runs.items()}
    if not args.no_cpu_baseline:
        import oracle
        evh = inputs[0].cpu().numpy().astype(np.complex128)
        tauh = inputs[1].cpu().numpy().astype(np.complex128)
        t_start = time.perf_counter()
        phi_ref, corr_ref = oracle.run(cfg.L, evh, inputs[2], tauh, inputs[3], cfg.profiles, ts=sample)
        dt = time.perf_counter() - t_start
        nt = len(sample)
        fl = flops_elementals(cfg.L, nt + 1, cfg.nvec, cfg.nmom) + flops_correlator(nt, cfg.nvec, cfg.nmom,
                                                                                    cfg.nprof)
        out["cpu_baseline"] = {"value": round(fl / dt / 1e12, 6), "unit": "TFLOP/s",
                               "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
                               "kind": "oracle", "sample": "%d of %d sink times x all %d momenta, plus the t0 "
                                                           "source elementals (%.1f s wall)" % (nt, T, cfg.nmom, dt)}
        for f, r in runs.items():
            out["forms"][f]["rel_err_vs_oracle"] = block_errors(r["corr"], r["phi"], corr_ref, phi_ref, sample)
        out["rel_err_vs_oracle"] = out["forms"]["fp32"]["rel_err_vs_oracle"]
    print(json.dumps(out), flush=True)


BATCH_MOMENTA = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0)]
BATCH_LATTICES = [(16, 32), (24, 48), (32, 64)]
BATCH_NVEC = [24, 32, 48, 64, 96]


def batched_jobs(njobs):
    """The batched workload: njobs configurations with N_vec uniform in {24,...,96},
    lattices uniform in {16^3x32, 24^3x48, 32^3x64}, 1-4 momenta, N_B = 4."""
    import synth
    g = synth.rng(3, 0, synth.FIELD_JOBS, 0)
    cfgs = []
    for n in range(njobs):
        L, T = BATCH_LATTICES[g.integers(0, 3)]
        N = BATCH_NVEC[g.integers(0, 5)]
        nm = int(g.integers(1, 5))
        cfgs.append(synth.custom("batch%d" % n, L, T, N, BATCH_MOMENTA[:nm], synth.plain().profiles,
                                 "gauss_decay", cfg_id=3))
    return cfgs


def bench_batched(args, torch, nuc, synth):
    cfgs = batched_jobs(args.jobs)
    ctx = nuc.Context(0)
    print("[bench] batched: generating %d jobs on the GPU" % len(cfgs), file=sys.stderr, flush=True)
    jobs, fl = [], 0.0
    for n, cfg in enumerate(cfgs):
        ev, tau, evals = synth.torch_inputs(cfg, conf_id=n)
        jobs.append(nuc.BatchJob(ev, evals, cfg.profiles, synth.momenta(cfg), tau, cfg.L))
        fl += flops_elementals(cfg.L, cfg.T, cfg.nvec, cfg.nmom) + flops_correlator(cfg.T, cfg.nvec, cfg.nmom,
                                                                                      cfg.nprof)
    torch.cuda.synchronize()
    # autotune every distinct shape on a two-timeslice slice of one of its jobs
    tuned = {}
    for cfg, jb in zip(cfgs, jobs):
        key = (cfg.L, cfg.nvec, cfg.nmom)
        if key in tuned:
            continue
        small = nuc.BatchJob(jb.evecs[:2].contiguous(), jb.evals[:2], cfg.profiles, jb.mom,
                             jb.tau[:2].contiguous(), cfg.L)
        tuned[key] = nuc.autotune(small, ctx=ctx)
    print("[bench] batched: tuned %d shapes; capturing the batch" % len(tuned), file=sys.stderr, flush=True)
    graph = nuc.BatchGraph(jobs, ctx=ctx)
    graph.launch()
    torch.cuda.synchronize()
    ctx.timing_enable(False)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.launch()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    print("[bench] batched: %.1f ms per batch" % ms, file=sys.stderr, flush=True)
    # kernel breakdown of one eager batch
    ctx.timing_enable(True)
    nuc.batch_run(jobs, ctx=ctx)
    torch.cuda.synchronize()
    kt = ctx.timing_read()
    ctx.timing_enable(False)
    graph.close()
    # parity: the smallest jobs against the oracle on two sink times
    import oracle
    errs = []
    order = sorted(range(len(cfgs)), key=lambda n: cfgs[n].V3 * cfgs[n].nvec ** 2)[:2]
    for n in order:
        cfg, jb = cfgs[n], jobs[n]
        ts = [0, cfg.T // 2]
        evh = jb.evecs.cpu().numpy().astype(np.complex128)
        tauh = jb.tau.cpu().numpy().astype(np.complex128)
        _, cref = oracle.run(cfg.L, evh, jb.evals, tauh, jb.mom, cfg.profiles, ts=ts)
        c = jb.corr.cpu().numpy()[:, ts]
        e = np.linalg.norm((c - cref).reshape(-1, cfg.nprof ** 2), axis=1) / \
            np.linalg.norm(cref.reshape(-1, cfg.nprof ** 2), axis=1)
        errs.append(float(e.max()))
    out = {
        "metric": "Nucleon corr-matrix TFLOP/s, BF16x3 vs FP32 @1e-6 rel err; p50/p99 job latency",
        "value": round(fl / (ms * 1e-3) / 1e12, 3), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
        "config": {"workload": "batched: %d jobs, N_vec in {24,32,48,64,96}, lattices 16^3x32/24^3x48/32^3x64, "
                               "1-4 momenta, N_B=4, one HIP graph of shared launches" % len(cfgs),
                   "jobs": [[c.L, c.T, c.nvec, c.nmom] for c in cfgs]},
        "tuned_shapes": {"%d,%d,%d" % k: v for k, v in tuned.items()},
        "kernels": kernel_table(kt),
        "rel_err_vs_oracle_smallest_jobs": errs,
    }
    print(json.dumps(out), flush=True)


KERNEL_CASES = [  # (name, L, T, N, momenta, profiles, tau kind, cfg id)
    ("n128_nb8", 8, 4, 128, 1, "p8", "gauss_decay", 4),
    ("n128_L24", 24, 2, 128, 2, "p4", "gauss_decay", 7),
    ("n96_L32", 32, 2, 96, 4, "p4", "gauss_decay", 5),
    ("n64_L24", 24, 4, 64, 3, "p6", "lognormal", 6),
]


def bench_kernels(args, torch, nuc, synth):
    """Per-kernel time and algorithmic rate on large-N shapes (one JSON line per case)."""
    profs = {"p4": synth.plain().profiles, "p6": synth.prec().profiles,
             "p8": [(0, s) for s in (0.1, 0.15, 0.2, 0.3, 0.5, 0.7, 1.0)] + [(1, 0.0)]}
    moms = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0)]
    ctx = nuc.Context(0)
    forms = [f for f in args.kernel_forms.split(",") if f]
    names = [c for c in args.kernel_cases.split(",") if c]
    for f in forms:
        if f not in FORM_PEAK:
            raise SystemExit("unknown form %r (one of %s)" % (f, ", ".join(FORM_PEAK)))
    for name, L, T, N, nm, pk, kind, cid in KERNEL_CASES:
        if names and name not in names:
            continue
        cfg = synth.custom(name, L, T, N, moms[:nm], profs[pk], kind, cfg_id=cid)
        inputs = device_inputs(torch, synth, cfg)
        for form in forms:
            r = run_workload(nuc, torch, cfg, inputs, form, args.steps, args.warmup, ctx)
            kt = r["kernels"]
            fl = {"elementals": flops_elementals(L, T, N, nm),
                  "corr_step1": T * nm * len(profs[pk]) * 2 * 4 * 8.0 * N ** 4,
                  "corr_chain": flops_chain_kernel(T, N, nm, len(profs[pk]))}
            out = {"case": name, "form": form, "L": L, "T": T, "nvec": N, "nmom": nm, "nprof": len(profs[pk]),
                   "ms_per_step": round(r["ms_step"], 3), "kernels": kernel_table(kt),
                   "tflops": {k: round(v * args.steps / (kt[k][0] * 1e-3) / 1e12, 1) for k, v in fl.items()}}
            print(json.dumps(out), flush=True)
        del inputs


def bench_copy(args, torch):
    """A plain device-to-device copy of --copy-mib MiB, repeated: reads and writes
    exactly that many bytes per launch, to scale the FETCH_SIZE / WRITE_SIZE counters."""
    n = args.copy_mib << 20
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(args.warmup + args.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"workload": "copy", "bytes_per_launch": n, "launches": args.warmup + args.steps}), flush=True)


def traffic_from_profile(kernel_file, kernel):
    """HBM bytes per launch of `kernel` measured by rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE
    (scaled by a copy of known size) and recorded in profiles/, if the kernel's source
    file still has the hash recorded there; else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.md")
    src = os.path.join(ROOT, "paper_2609_37723_amd", "csrc", kernel_file)
    if not os.path.exists(path) or not os.path.exists(src):
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for line in open(path):
        line = line.strip()
        if line.startswith("{") and '"kernel": "%s"' % kernel in line:
            rec = json.loads(line)
            if rec.get("source_sha256") == sha:
                return rec
    return None


SERVE_NVEC = (32, 64, 96, 128)
SERVE_PROF8 = [(0, s) for s in (0.1, 0.15, 0.2, 0.3, 0.5, 0.7, 1.0)] + [(1, 0.0)]


def serving_stream(n, rate, stream_id, nconf):
    """Seeded Poisson job stream: (arrival s, conf, N, nmom, profiles). N uniform in
    {32,64,96,128}, 1-7 momenta (the first k of the 7-momentum set), N_B 4 (three
    Gaussians + linear) or 8 (seven Gaussians + linear), configuration uniform."""
    import synth
    g = synth.rng(4, stream_id, synth.FIELD_JOBS, 0)
    t, out = 0.0, []
    for _ in range(n):
        t += float(g.exponential(1.0 / rate))
        conf = int(g.integers(0, nconf))
        N = int(SERVE_NVEC[g.integers(0, 4)])
        nm = int(g.integers(1, 8))
        prof = synth.plain().profiles if g.integers(0, 2) == 0 else SERVE_PROF8
        out.append((t, conf, N, nm, prof))
    return out


def expected_job_flops(L, T):
    """Mean algorithmic flops of a job of serving_stream (N, momenta and N_B uniform)."""
    tot = 0.0
    for N in SERVE_NVEC:
        for nm in range(1, 8):
            for nprof in (4, 8):
                tot += flops_elementals(L, T, N, nm) + flops_correlator(T, N, nm, nprof)
    return tot / (len(SERVE_NVEC) * 7 * 2)


def run_stream(srv, synth, stream, label, keep=()):
    """Submit each job at its arrival time, collect every result; per-job latencies
    come from the server's clock (submission to result in host memory). Results of the
    jobs whose stream index is in keep are returned (for oracle checks)."""
    t0 = time.perf_counter()
    pending, infos, fl, kept = {}, [], 0.0, {}
    nxt = 0
    while nxt < len(stream) or pending:
        now = time.perf_counter() - t0
        while nxt < len(stream) and stream[nxt][0] <= now:
            _, conf, N, nm, prof = stream[nxt]
            tk = srv.submit(conf, N, synth.MOMENTA_7[:nm], prof)
            pending[tk] = (nxt, stream[nxt])
            nxt += 1
        for tk in list(pending):
            try:
                corr, info = srv.wait(tk, timeout_ms=0)
            except Exception as e:  # still running
                if getattr(e, "status", None) == -7:
                    continue
                raise
            idx, job = pending.pop(tk)
            info["index"] = idx
            infos.append(info)
            fl += info["flops"]
            if idx in keep:
                kept[idx] = (job, corr)
            print("[bench] %s: job %d/%d done (N=%d, %d mom, N_B=%d) latency %.2f s" % (
                label, len(infos), len(stream), job[2], job[3], len(job[4]),
                info["done_s"] - info["submit_s"]), file=sys.stderr, flush=True)
        time.sleep(0.01)

    def pct(sel):
        lat = np.sort([1e3 * (i["done_s"] - i["submit_s"]) for i in sel])
        rank = lambda q: float(lat[max(1, int(math.ceil(q * len(lat)))) - 1])
        return round(rank(0.5), 1), round(rank(0.99), 1), lat

    p50, p99, lat = pct(infos)
    first = min(i["submit_s"] for i in infos)
    last = max(i["done_s"] for i in infos)
    win = last - first
    half = len(stream) // 2
    h1 = pct([i for i in infos if i["index"] < half])
    h2 = pct([i for i in infos if i["index"] >= half])
    return {"arrivals": len(stream), "offered_jobs_per_s": round(len(stream) / stream[-1][0], 3),
            "completed": len(infos), "p50_ms": p50, "p99_ms": p99,
            "halves_p50_p99_ms": [[h1[0], h1[1]], [h2[0], h2[1]]],
            "mean_ms": round(float(lat.mean()), 1), "max_ms": round(float(lat[-1]), 1),
            "window_s": round(win, 3), "served_jobs_per_s": round(len(infos) / win, 4),
            "served_tflops": round(fl / win / 1e12, 3), "mean_job_tflop": round(fl / len(infos) / 1e12, 3)}, kept


SERVE_L, SERVE_T, SERVE_NMAX = 32, 64, 128


def serving_run(torch, nuc, synth, confs, arrivals, rate, arrivals_light, quantum):
    """Make `confs` configurations resident, warm up, then run the Poisson stream at
    `rate` and (if arrivals_light) a second one at 0.7x the measured capacity."""
    L, T, NMAX = SERVE_L, SERVE_T, SERVE_NMAX
    srv = nuc.Server("hip", slots=2, job_arena=8 << 30, slot_workspace=16 << 30, quantum_flops=quantum)
    for c in range(confs):
        cfg = synth.custom("serve", L, T, NMAX, synth.MOMENTA_7, [], "gauss_decay", cfg_id=4)
        ev, tau, evals = synth.torch_inputs(cfg, conf_id=c)
        srv.register(c, L, ev, evals, tau)
        del ev, tau
        torch.cuda.empty_cache()
        print("[bench] serving: configuration %d/%d resident" % (c + 1, confs), file=sys.stderr, flush=True)
    # warm-up: load every kernel shape class once
    for N in SERVE_NVEC:
        srv.wait(srv.submit(0, N, synth.MOMENTA_7[:1], synth.plain().profiles))
    print("[bench] serving: warm", file=sys.stderr, flush=True)
    heavy, _ = run_stream(srv, synth, serving_stream(arrivals, rate, 1, confs), "stream@%g/s" % rate)
    light, kept = None, {}
    if arrivals_light > 0:
        # 0.7 x capacity in work: served flop rate over the expected flops of a job of the stream
        rate_b = 0.7 * heavy["served_tflops"] * 1e12 / expected_job_flops(L, T)
        stream_b = serving_stream(arrivals_light, rate_b, 2, confs)
        keep = {}
        # the first job of N = 64 and of N = 96, for the oracle (its elementals at N = 128 on
        # 32^3 sites take the host cores several minutes per timeslice)
        for n, job in enumerate(stream_b):
            if job[2] in (64, 96) and job[2] not in keep:
                keep[job[2]] = n
        light, kept = run_stream(srv, synth, stream_b, "stream@%.3g/s" % rate_b, keep=set(keep.values()))
        print("[bench] serving: stated-rate stream %s" % json.dumps(heavy), file=sys.stderr, flush=True)
        print("[bench] serving: 0.7x-capacity stream %s" % json.dumps(light), file=sys.stderr, flush=True)
    st = srv.stats()
    srv.close()
    torch.cuda.empty_cache()
    return heavy, light, st, kept


def served_oracle_check(torch, synth, kept):
    """FP64 oracle on served jobs: sink time 1, the job's first momentum, host copies of
    the resident configuration's first N vectors (regenerated from the same seeds)."""
    import oracle
    L, T, NMAX = SERVE_L, SERVE_T, SERVE_NMAX
    out = []
    for idx, (job, corr) in sorted(kept.items()):
        _, conf, N, nm, prof = job
        cfg = synth.custom("serve", L, T, NMAX, synth.MOMENTA_7, [], "gauss_decay", cfg_id=4)
        ev, tau, evals = synth.torch_inputs(cfg, conf_id=conf)
        sel = torch.cat([torch.arange(N) + a * NMAX for a in range(4)]).to(tau.device)
        evh = ev[:2, :N].cpu().numpy().astype(np.complex128)
        tauh = tau[:2][:, sel][:, :, sel].cpu().numpy().astype(np.complex128)
        del ev, tau
        torch.cuda.empty_cache()
        print("[bench] serving: oracle on served job %d (N=%d), t=1, first momentum" % (idx, N), file=sys.stderr,
              flush=True)
        tc = time.perf_counter()
        _, ref = oracle.run(L, evh, evals[:2, :N], tauh, np.asarray(synth.MOMENTA_7[:1], np.int32), prof, ts=[1])
        got = corr[0, 1]
        out.append({"job": idx, "nvec": N, "nprof": len(prof),
                    "rel_err": float("%.3e" % (np.linalg.norm(got - ref[0, 0]) / np.linalg.norm(ref[0, 0])))})
        print("[bench] serving: oracle on job %d done in %.0f s, rel err %.3e" % (
            idx, time.perf_counter() - tc, out[-1]["rel_err"]), file=sys.stderr, flush=True)
    return out


def bench_serving(args, torch, nuc, synth):
    L, T = SERVE_L, SERVE_T
    heavy, light, st, kept = serving_run(torch, nuc, synth, args.confs, args.arrivals, args.rate,
                                         args.arrivals_light, args.quantum)
    out = {
        "metric": "Nucleon corr-matrix TFLOP/s, BF16x3 vs FP32 @1e-6 rel err; p50/p99 job latency",
        "value": heavy["served_tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": heavy["completed"],
        "warmup": len(SERVE_NVEC), "ms_per_step": round(1e3 / heavy["served_jobs_per_s"], 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
        "config": {"workload": "serving: Poisson job stream, 32^3x64 lattices, %d resident configurations at "
                               "N_vec=128 (prefixes used), N_vec uniform in {32,64,96,128}, 1-7 momenta, N_B in "
                               "{4,8}; continuous batching on 2 slots, quantum %.3g flops" % (args.confs, args.quantum)},
        "p50_ms": heavy["p50_ms"], "p99_ms": heavy["p99_ms"],
        "expected_job_tflop": round(expected_job_flops(L, T) / 1e12, 3),
        "stream_stated_rate": heavy, "stream_0p7_capacity": light,
        "served_vs_oracle": served_oracle_check(torch, synth, kept) if not args.no_cpu_baseline else None,
        "server": {k: st[k] for k in ("submitted", "completed", "failed", "iterations", "max_outstanding",
                                      "bytes_resident", "bytes_arena_peak", "bytes_total")},
    }
    print(json.dumps(out), flush=True)



# ------------------------------------------------------------------ meson operators
MESON_SIGMAS = (0.05, 0.1, 0.15, 0.2, 0.3, 0.5, 1.0)
HBM_PEAK_GBS = 8000.0


def meson_config(synth):
    """The charmonium study's shape: 24^3 x 48 lattice, N_v = 200, zero momentum, 7
    Gaussian profiles in each of the 3 operator families (21 operators)."""
    return synth.custom("charmonium", 24, 48, 200, [(0, 0, 0)],
                        [(synth.PROF_GAUSS, sg) for sg in MESON_SIGMAS], "gauss", cfg_id=5)


def meson_flops(L, T, N, nmom, nprof):
    """Algorithmic flops per kernel of one meson step (8 per complex multiply-add)."""
    V3 = L ** 3
    nterms = nprof * (1 + 3 + 3)          # (Gamma, D) terms over the 3 nprof operators
    nop = 3 * nprof
    return {"meson_elem": 8.0 * N * 7 * N * 3 * V3 * nmom * T,
            # Y_A = M_A tau and Z_B = tau' M'_B: 4 spin row (column) blocks x N x 4N x N per term
            "meson_gemm": 2 * 8.0 * 4 * N * 4 * N * N * nterms * nmom * T,
            "meson_trace": 8.0 * nop * nop * 16 * N * N * nmom * T}


def meson_bytes(L, T, N):
    """Algorithmic HBM bytes of the derivative stencils (both passes) per step: read v
    and the links once, write the three nabla fields; read them, write the three B fields."""
    V3 = L ** 3
    field = N * V3 * 3 * 8
    return T * (field + V3 * 27 * 8 + 3 * field + 3 * field + 3 * field)


def meson_measure(torch, nuc, synth, steps, warmup, oracle_check=True):
    import oracle as _oracle
    import oracle.meson as om
    cfg = meson_config(synth)
    L, T, N, nmom, nprof = cfg.L, cfg.T, cfg.nvec, cfg.nmom, cfg.nprof
    dev = torch.device("cuda:0")
    print("[bench] meson workload: generating inputs (24^3 x 48, N_v=200)", file=sys.stderr, flush=True)
    ev, tau, evals = synth.torch_inputs(cfg, device="cuda:0")
    links_h = synth.gauge_links(cfg)
    links = torch.from_numpy(links_h.astype(np.complex64)).to(dev)
    mom = synth.momenta(cfg)
    nop = 3 * nprof
    phi = torch.empty((T, nmom, 7, N, N), dtype=torch.complex64, device=dev)
    corr = torch.empty((nmom, T, nop, nop), dtype=torch.complex128, device=dev)
    ctx = nuc.Context(0)
    stream = torch.cuda.current_stream()

    def step():
        nuc.meson_run(ev, links, evals, cfg.profiles, mom, tau, L, t0=cfg.t0, phi_out=phi, out=corr, ctx=ctx,
                      stream=stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.timing_enable(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    kt = ctx.timing_read()
    ctx.timing_enable(False)
    ms = wall * 1e3 / steps
    print("[bench] meson: %.3f ms/step" % ms, file=sys.stderr, flush=True)
    fl = meson_flops(L, T, N, nmom, nprof)
    total = sum(fl.values())
    roof = {}
    for k, f in fl.items():
        kms, kn = kt[k]
        ach = f * steps / (kms * 1e-3) / 1e12
        roof[k] = {"bound": "mfma" if k != "meson_trace" else "alu", "achieved": round(ach, 3),
                   "peak": FP32_PEAK_TFLOPS if k != "meson_trace" else 78.6, "unit": "TFLOP/s",
                   "frac": round(ach / (FP32_PEAK_TFLOPS if k != "meson_trace" else 78.6), 4), "traffic": None,
                   "avg_launch_ms": round(kms / max(kn, 1), 4), "launches_per_step": kn / steps,
                   "flops_per_launch": f / (kn / steps)}
    dms, dn = kt["meson_deriv"]
    by = meson_bytes(L, T, N)
    gbs = by * steps / (dms * 1e-3) / 1e9
    roof["meson_deriv"] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                           "avg_launch_ms": round(dms / max(dn, 1), 4), "launches_per_step": dn / steps,
                           "bytes_per_launch": by / (dn / steps)}
    dominant = max(("meson_elem", "meson_gemm"), key=lambda k: kt[k][0])
    for k, kern, src in (("meson_elem", "meson_elem_kernel", "meson_elem.hip"),
                         ("meson_gemm", "meson_gemm_kernel", "meson_corr.hip")):
        rec = traffic_from_profile(src, kern)
        if rec:
            per_launch = rec["hbm_bytes_per_launch"]
            # the record's launches cover the same work as this run's (same plan)
            roof[k]["traffic"] = per_launch
            roof[k]["traffic_note"] = rec["note"]
    res = {"workload": "charmonium operators: 24^3x48 lattice, N_v=200, p=0, 7 Gaussian profiles x 3 operator "
                       "families (g4g5; g4g5 g_k nabla_k; g_k B_k) = 21 operators, all 48 sink times: "
                       "covariant derivatives, 7 meson elementals, 21x21 C_AB(t)",
           "value": round(total / (ms * 1e-3) / 1e12, 3), "unit": "TFLOP/s", "ms_per_step": round(ms, 4),
           "roofline": dict(roof[dominant], kernel=dominant), "kernels": {"rooflines": roof, **kernel_table(kt)},
           "flops_per_step": total}
    if oracle_check:
        print("[bench] meson oracle sample: elementals at t=0,1 and the 3 operators of profile 0 at t=1",
              file=sys.stderr, flush=True)
        ts = [0, 1]
        ev_h = ev[:2].cpu().numpy().astype(np.complex128)
        tau_h = tau[:2].cpu().numpy().astype(np.complex128)
        t_start = time.perf_counter()
        phi_ref = om.elementals(L, ev_h, links_h[:2], mom)
        g = _oracle.profiles(evals, cfg.profiles)
        c_ref = om.correlator(phi_ref[1:2], phi_ref[0], tau_h[1:2], g[0:1, 1:2, :], g[0:1, 0, :])
        dt = time.perf_counter() - t_start
        fl_s = (meson_flops(L, 2, N, nmom, 1)["meson_elem"] + meson_flops(L, 1, N, nmom, 1)["meson_gemm"] +
                meson_flops(L, 1, N, nmom, 1)["meson_trace"])
        nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        res["cpu_baseline"] = {"value": fl_s / dt / 1e12, "unit": "TFLOP/s", "cores": nthreads, "kind": "oracle",
                               "sample": "elementals at t=0 (source) and t=1, C_AB at t=1 for the 3 operators of "
                                         "the first profile; %.1f s wall" % dt}
        p = phi[:2].cpu().numpy()
        e_phi = np.linalg.norm((p - phi_ref).reshape(-1, N * N), axis=1) / \
            np.linalg.norm(phi_ref.reshape(-1, N * N), axis=1)
        sel = [f * nprof for f in range(3)]
        c = corr.cpu().numpy()[:, 1:2][:, :, sel][:, :, :, sel]
        e_c = np.linalg.norm(c - c_ref) / np.linalg.norm(c_ref)
        res["rel_err_vs_oracle"] = {"phi_max": float(e_phi.max()), "corr_profile0_t1": float(e_c)}
        # the correlator sample is checked entrywise in tests/test_gpu_meson.py as well
    return res


def bench_meson(args, torch, nuc, synth):
    res = meson_measure(torch, nuc, synth, args.steps, args.warmup, oracle_check=not args.no_cpu_baseline)
    cfg = meson_config(synth)
    out = {"metric": "Meson (charmonium) corr-matrix TFLOP/s", "value": res["value"], "unit": "TFLOP/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
           "config": {"workload": res["workload"], "L": cfg.L, "T": cfg.T, "nvec": cfg.nvec, "nmom": cfg.nmom,
                      "nprof": cfg.nprof, "operators": 3 * cfg.nprof},
           "roofline": res["roofline"], "kernels": res["kernels"], "flops_per_step": res["flops_per_step"]}
    for k in ("cpu_baseline", "rel_err_vs_oracle"):
        if k in res:
            out[k] = res[k]
    print(json.dumps(out), flush=True)



# ------------------------------------------------------------------ glueball operators
GLUE_L, GLUE_T, GLUE_NCONF = 24, 48, 16


def glueball_bytes_per_site():
    """Algorithmic HBM bytes per site and timeslice of one configuration, with the fields
    stored as the 8 reals of a traceless anti-Hermitian matrix (32 B) and the links as
    their first two rows (6 complex, 48 B per direction): link relayout (read the caller's
    27 complex, write 18), clover (read the links, write 3 fields), 18 stored adjoint
    differences (read the input field and the link direction, write the output), the
    contraction (read B, the 6 first and 12 second differences, and the links for the
    third difference taken on the fly)."""
    field, link = 8 * 4, 6 * 8
    return (27 * 8 + 3 * link) + (3 * link + 3 * field) + 18 * (field + link + field) + (21 * field + 3 * link)


def glueball_flops_per_site():
    """Algorithmic flops per site and timeslice (8 per complex multiply-add), counting the
    products the su(3) structure leaves: clover, 3 planes x 4 leaves x 3 products of 3 x 3
    matrices (27 MACs each); 36 adjoint differences of two terms u X u^H, each a full
    product (27) and the product's algebra part (the upper entries and the imaginary
    diagonal, 13.5); O2, 6 products B_j B_k (27) and 12 traces against a field (9);
    the 24 traces of su(3) pairs of O1, O3, O4, O5, 20 real flops each."""
    return 8 * (3 * 4 * 3 * 27 + 36 * 2 * (27 + 13.5) + 6 * 27 + 12 * 9) + 24 * 20


VEC_FP32_PEAK_TFLOPS = 78.6  # FP32 vector without packed math: 256 CUs x 4 SIMDs x 16 lanes x 2 x 2.4 GHz


def glueball_measure(torch, nuc, synth, steps, warmup, oracle_check=True):
    import oracle.glueball as og
    L, T, nconf = GLUE_L, GLUE_T, GLUE_NCONF
    print("[bench] glueball workload: %d configurations of %d^3 x %d" % (nconf, L, T), file=sys.stderr, flush=True)
    cfg = synth.custom("glueball", L, T, 3, [(0, 0, 0)], [(0, 0.5)], "gauss", cfg_id=6)
    dev = torch.device("cuda:0")
    links = synth.torch_links(cfg, nconf, device="cuda:0")
    ops = torch.empty((nconf, T, 5), dtype=torch.complex128, device=dev)
    ctx = nuc.Context(0)
    stream = torch.cuda.current_stream()

    def step():
        nuc.glueball_operators(links, L, out=ops, ctx=ctx, stream=stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.timing_enable(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    kt = ctx.timing_read()
    ctx.timing_enable(False)
    ms = wall * 1e3 / steps
    sites = nconf * T * L ** 3
    by = glueball_bytes_per_site() * sites
    kms = kt["glue_stencil"][0] + kt["glue_contract"][0]
    gbs = by * steps / (kms * 1e-3) / 1e9
    fl = glueball_flops_per_site() * sites
    tfs = fl * steps / (kms * 1e-3) / 1e12
    # the stencils read about their compulsory bytes (profiles/traffic.md) at well under the
    # HBM rate: FP32 vector arithmetic (3 x 3 complex products) bounds them
    res = {"workload": "glueball operators O1-O5 (A1-+): %d configurations of %d^3 x %d, clover B_i, adjoint "
                       "symmetric differences up to third order, FP64 site sums per timeslice" % (nconf, L, T),
           "value": round(nconf / (ms * 1e-3), 2), "unit": "configurations/s", "ms_per_step": round(ms, 4),
           "roofline": {"bound": "alu", "kernel": "glue_stencil + glue_contract", "achieved": round(tfs, 2),
                        "peak": VEC_FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(tfs / VEC_FP32_PEAK_TFLOPS, 4),
                        "traffic": None, "flops_per_step": fl, "bytes_per_step": by,
                        "hbm_achieved_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)},
           "kernels": kernel_table(kt)}
    rec = traffic_from_profile("glueball.hip", "glue_stencil + glue_contract")
    if rec:
        res["roofline"]["traffic"] = rec["hbm_bytes_per_step"]
        res["roofline"]["traffic_note"] = rec["note"] + " (per step, like bytes_per_step)"
    if oracle_check:
        print("[bench] glueball oracle sample: configuration 0, timeslices 0 and 1", file=sys.stderr, flush=True)
        t_start = time.perf_counter()
        ref, scale = og.operators(L, links[0, :2].cpu().numpy().astype(np.complex128), with_scale=True)
        dt = time.perf_counter() - t_start
        o = ops[0, :2].cpu().numpy()
        res["rel_err_vs_oracle"] = {"max_abs_err_over_scale": float(np.max(np.abs(o - ref) / scale))}
        nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        res["cpu_baseline"] = {"value": 2.0 / T / dt, "unit": "configurations/s", "cores": nthreads, "kind": "oracle",
                               "sample": "2 of %d timeslices of one %d^3 configuration; %.1f s wall" % (T, L, dt)}
    return res


def bench_glueball(args, torch, nuc, synth):
    res = glueball_measure(torch, nuc, synth, args.steps, args.warmup, oracle_check=not args.no_cpu_baseline)
    out = {"metric": "Glueball operators, configurations/s", "value": res["value"], "unit": res["unit"],
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
           "config": {"workload": res["workload"], "L": GLUE_L, "T": GLUE_T, "nconf": GLUE_NCONF},
           "roofline": res["roofline"], "kernels": res["kernels"]}
    for k in ("cpu_baseline", "rel_err_vs_oracle"):
        if k in res:
            out[k] = res[k]
    print(json.dumps(out), flush=True)



# ------------------------------------------------------------ general spin tensors
def spin_flops(T, N, nmom, nprof, nrow, nnz):
    """Algorithmic flops of one nuc_correlator_spin call: per (t, p, b, row) the three dense
    tau products (4N)^4 complex MACs each, and the sink dot (nnz triples x N^3 x nprof)."""
    return T * nmom * nprof * nrow * (3 * 8.0 * (4 * N) ** 4 + nnz * N ** 3 * nprof * 8.0)


def spin_measure(torch, nuc, synth, steps, warmup, oracle_check=True):
    """The moving-frame G1 nucleon correlation matrix over {P+, P-} x profiles at
    p = (0, 0, 2) on the plain lattice (16^3 x 32, N = 32, N_B = 4): four calls (sink,
    source) in {+, -}^2 with two irrep rows each."""
    import oracle
    import oracle.spin as osp
    cfg = synth.custom("g1_moving", 16, 32, 32, [(0, 0, 2)],
                       [(0, 0.2), (0, 0.5), (0, 1.0), (1, 0.0)], "gauss_decay", cfg_id=7)
    T, N, nprof = cfg.T, cfg.nvec, cfg.nprof
    print("[bench] spin workload: moving-frame G1, p=(0,0,2), 16^3 x 32, N=32, P+/P- rows", file=sys.stderr,
          flush=True)
    dev = torch.device("cuda:0")
    inp = synth.make_inputs(cfg)
    ev = torch.from_numpy(inp.evecs.astype(np.complex64)).to(dev)
    tau = torch.from_numpy(inp.tau.astype(np.complex64)).to(dev)
    ctx = nuc.Context(0)
    phi = nuc.elementals(ev, cfg.L, inp.mom, ctx=ctx)
    tens = {"+": nuc.nucleon_spin(+1), "-": nuc.nucleon_spin(-1)}
    pairs = [("+", "+"), ("+", "-"), ("-", "+"), ("-", "-")]
    outs = {pq: torch.empty((1, T, nprof, nprof), dtype=torch.complex128, device=dev) for pq in pairs}
    stream = torch.cuda.current_stream()

    def step():
        for a_, b_ in pairs:
            nuc.correlator_spin(phi, inp.evals, cfg.profiles, tau, cfg.L, tens[a_], tens[b_], out=outs[(a_, b_)],
                                ctx=ctx, stream=stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.timing_enable(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    kt = ctx.timing_read()
    ctx.timing_enable(False)
    ms = wall * 1e3 / steps
    nnz = int(np.count_nonzero(tens["+"][0]))
    fl = 4 * spin_flops(T, N, 1, nprof, 2, nnz)
    gemm_fl = 4 * T * nprof * 2 * 3 * 8.0 * (4 * N) ** 4
    gms, gn = kt["spin_gemm"]
    ach = gemm_fl * steps / (gms * 1e-3) / 1e12
    res = {"workload": "moving-frame G1 nucleon correlation matrix at p=(0,0,2): {P+, P-} x 4 profiles (an 8 x 8 "
                       "matrix in four 4 x 4 blocks, two irrep rows each), 16^3 x 32, N=32, all 32 sink times, "
                       "general spin tensors (dense tau products)",
           "value": round(fl / (ms * 1e-3) / 1e12, 3), "unit": "TFLOP/s", "ms_per_step": round(ms, 4),
           "roofline": {"bound": "mfma", "kernel": "spin_cgemm (three tau products)", "achieved": round(ach, 3),
                        "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(ach / FP32_PEAK_TFLOPS, 4),
                        "traffic": None, "launches_per_step": gn / steps},
           "kernels": kernel_table(kt)}
    if oracle_check:
        print("[bench] spin oracle sample: P+ sink / P- source at t = 1", file=sys.stderr, flush=True)
        t_start = time.perf_counter()
        gp = oracle.profiles(inp.evals, cfg.profiles)
        ph = oracle.elementals(cfg.L, inp.evecs[[0, 1]], inp.mom)
        ref = osp.correlator(ph[1:2], ph[0], inp.tau[1:2], gp[:, 1:2, :], gp[:, 0, :], tens["+"], tens["-"])
        dt = time.perf_counter() - t_start
        c = outs[("+", "-")].cpu().numpy()[:, 1:2]
        res["rel_err_vs_oracle"] = {"corr_P+P-_t1": float(np.linalg.norm(c - ref) / np.linalg.norm(ref))}
        nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        res["cpu_baseline"] = {"value": spin_flops(1, N, 1, nprof, 2, nnz) / dt / 1e12, "unit": "TFLOP/s",
                               "cores": nthreads, "kind": "oracle",
                               "sample": "one (sink, source) block at one sink time, with its elementals; %.1f s wall"
                                         % dt}
    return res


def bench_spin(args, torch, nuc, synth):
    res = spin_measure(torch, nuc, synth, args.steps, args.warmup, oracle_check=not args.no_cpu_baseline)
    out = {"metric": "Moving-frame G1 nucleon corr-matrix TFLOP/s (general spin tensors)", "value": res["value"],
           "unit": res["unit"], "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": res["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "fp32", "data": "synthetic",
           "config": {"workload": res["workload"], "L": 16, "T": 32, "nvec": 32, "nmom": 1, "nprof": 4},
           "roofline": res["roofline"], "kernels": res["kernels"]}
    for k in ("cpu_baseline", "rel_err_vs_oracle"):
        if k in res:
            out[k] = res[k]
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------------ two-meson operators
TM_STAR = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]


def twomeson_config(synth):
    """The charmonium study's two-meson shape: 24^3 x 48, N_v = 200, 7 Gaussian profiles
    in each of the 3 families (21 operators), back-to-back momenta over the star of (0,0,1)."""
    return synth.custom("charmonium_two_meson", 24, 48, 200, TM_STAR,
                        [(synth.PROF_GAUSS, sg) for sg in MESON_SIGMAS], "gauss", cfg_id=5)


def twomeson_flops(T, N, nmom):
    """Algorithmic flops of one two-meson correlator (8 per complex multiply-add): per
    sink time the products L_k = M_k tau and R_l = Mbar_l g5 tau^H g5 (2 nmom) and every
    P_kl = L_k R_l (nmom^2), each an n^3 complex product with n = 4N."""
    n = 4 * N
    return {"tm_gemm": T * 2 * nmom * 8.0 * n ** 3, "tm_pair": T * nmom * nmom * 8.0 * n ** 3}


def twomeson_measure(torch, nuc, synth, steps, warmup, oracle_check=True):
    import oracle as _oracle
    import oracle.meson as om
    import oracle.twomeson as otm
    cfg = twomeson_config(synth)
    L, T, N, nmom, nprof, t0 = cfg.L, cfg.T, cfg.nvec, cfg.nmom, cfg.nprof, cfg.t0
    dev = torch.device("cuda:0")
    print("[bench] two-meson workload: inputs and elementals at the star of (0,0,1) (24^3 x 48, N_v=200)",
          file=sys.stderr, flush=True)
    ev, tau, evals = synth.torch_inputs(cfg, device="cuda:0")
    links_h = synth.gauge_links(cfg)
    links = torch.from_numpy(links_h.astype(np.complex64)).to(dev)
    mom = synth.momenta(cfg)
    ctx = nuc.Context(0)
    phi = nuc.meson_elementals(ev, links, mom, L, ctx=ctx)
    gw = np.random.default_rng(np.random.SeedSequence([0x37723, cfg.cfg_id, 0, 6, 0]))
    w = gw.standard_normal(3 * nprof) + 1j * gw.standard_normal(3 * nprof)
    w /= np.linalg.norm(w)
    out = torch.empty((T, 3), dtype=torch.complex128, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        nuc.twomeson_correlator(phi, evals, cfg.profiles, w, mom, tau, L, t0=t0, out=out, ctx=ctx, stream=stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.timing_enable(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    kt = ctx.timing_read()
    ctx.timing_enable(False)
    ms = wall * 1e3 / steps
    print("[bench] two-meson: %.3f ms/step" % ms, file=sys.stderr, flush=True)
    fl = twomeson_flops(T, N, nmom)
    total = sum(fl.values())
    roof = {}
    for k, f in fl.items():
        kms, kn = kt[k]
        ach = f * steps / (kms * 1e-3) / 1e12
        roof[k] = {"bound": "mfma", "achieved": round(ach, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                   "frac": round(ach / FP32_PEAK_TFLOPS, 4), "traffic": None,
                   "avg_launch_ms": round(kms / max(kn, 1), 4), "launches_per_step": kn / steps,
                   "flops_per_launch": f / max(kn / steps, 1)}
    rec = traffic_from_profile("twomeson.hip", "tm_pair_kernel")
    if rec:
        roof["tm_pair"]["traffic"] = rec["hbm_bytes_per_launch"]
        roof["tm_pair"]["traffic_note"] = rec["note"]
    res = {"workload": "I=2 A1++ two-meson correlator of the optimal one-meson operator (21 profiled operators: "
                       "7 Gaussian profiles x {g4g5; g4g5 g_k nabla_k; g_k B_k}), back-to-back momenta over the "
                       "star of (0,0,1), 24^3x48 lattice, N_v=200, all 48 sink times: direct and crossed Wick terms",
           "value": round(total / (ms * 1e-3) / 1e12, 3), "unit": "TFLOP/s", "ms_per_step": round(ms, 4),
           "roofline": dict(roof["tm_pair"], kernel="tm_pair"), "kernels": {"rooflines": roof, **kernel_table(kt)},
           "flops_per_step": total}
    if oracle_check:
        print("[bench] two-meson oracle sample: elementals at t=0 (source) and t=1, C at t=1",
              file=sys.stderr, flush=True)
        ev_h = ev[:2].cpu().numpy().astype(np.complex128)
        tau_h = tau[:2].cpu().numpy().astype(np.complex128)
        t_start = time.perf_counter()
        phi_ref = om.elementals(L, ev_h, links_h[:2], mom)
        g = _oracle.profiles(evals, cfg.profiles)
        C, D, X = otm.correlator_by_pairs(phi_ref[1:2], phi_ref[0], tau_h[1:2], g[:, 1:2, :], g[:, 0, :], w, mom,
                                          terms=True)
        dt = time.perf_counter() - t_start
        fl_s = meson_flops(L, 2, N, nmom, 1)["meson_elem"] + sum(twomeson_flops(1, N, nmom).values())
        nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        res["cpu_baseline"] = {"value": fl_s / dt / 1e12, "unit": "TFLOP/s", "cores": nthreads, "kind": "oracle",
                               "sample": "elementals at t=0 (source) and t=1 for the 6 momenta, then C at t=1; "
                                         "%.1f s wall" % dt}
        o = out.cpu().numpy()[1]
        res["rel_err_vs_oracle"] = {"C_t1": float(abs(o[0] - C[0]) / abs(C[0])),
                                    "D_t1": float(abs(o[1] - D[0]) / abs(D[0])),
                                    "X_t1": float(abs(o[2] - X[0]) / abs(X[0]))}
    return res


def bench_twomeson(args, torch, nuc, synth):
    res = twomeson_measure(torch, nuc, synth, args.steps, args.warmup, oracle_check=not args.no_cpu_baseline)
    cfg = twomeson_config(synth)
    out = {"metric": "Two-meson (I=2) correlator TFLOP/s", "value": res["value"], "unit": "TFLOP/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
           "config": {"workload": res["workload"], "L": cfg.L, "T": cfg.T, "nvec": cfg.nvec, "nmom": cfg.nmom,
                      "nprof": cfg.nprof, "operators": 3 * cfg.nprof},
           "roofline": res["roofline"], "kernels": res["kernels"], "flops_per_step": res["flops_per_step"]}
    for k in ("cpu_baseline", "rel_err_vs_oracle"):
        if k in res:
            out[k] = res[k]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

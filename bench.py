"""Throughput benchmark of the profiled-distillation nucleon correlator on one MI355X.

One step = one full pass of the hot path over the plain workload (16^3 x 32
lattice, N_vec = 32 distillation vectors, 7 momenta, N_B = 4 profiles, all 32
sink times): baryon elementals for every (t, p), profile weighting, and the
N_B x N_B correlation matrix C_ab(t) with both Wick terms. Inputs are seeded
synthetic data resident in HBM before timing starts.

Prints one JSON line (rank 0). ``value`` is algorithmic TFLOP/s of the whole
step: elementals 24 V3 C(N,3) per (t,p) + 42 V3 C(N,2) per t, correlator
8 * (48 N^4 N_B * 2) + sink dots per (t,p) -- the complex multiply-adds the
Wick-folded contraction needs, 8 flops each. ``value_survey_convention``
restates the same time with the unfolded count 1152 N_B N^4 + 128 N_B^2 N^3.
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
BF16_PEAK_TFLOPS = 2516.6       # MI355X dense BF16 MFMA
BF16X3_PEAK_TFLOPS = BF16_PEAK_TFLOPS / 3.0   # three bf16 products per FP32 product


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


def flops_survey(L, T, N, nmom, nprof):
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=8, help="sink times in the oracle sample")
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
    dev = torch.device("cuda:0")
    cfg = synth.plain()
    print("[bench] generating plain inputs ...", file=sys.stderr, flush=True)
    inp = synth.make_inputs(cfg)
    ev = torch.from_numpy(inp.evecs.astype(np.complex64)).to(dev)
    tau = torch.from_numpy(inp.tau.astype(np.complex64)).to(dev)
    T, N, nmom, nprof = cfg.T, cfg.nvec, cfg.nmom, cfg.nprof
    phi = torch.empty((T, nmom, N, N, N), dtype=torch.complex64, device=dev)
    corr = torch.empty((nmom, T, nprof, nprof), dtype=torch.complex128, device=dev)
    ctx = nuc.Context(0)
    stream = torch.cuda.current_stream()

    def step():
        nuc.run(ev, inp.evals, cfg.profiles, inp.mom, tau, cfg.L, t0=cfg.t0, precision=args.precision,
                phi_out=phi, out=corr, ctx=ctx, stream=stream)

    print("[bench] warmup %d steps" % args.warmup, file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = ctx.timing_read()
    ctx.timing_enable(False)
    ms_step = wall * 1e3 / args.steps
    print("[bench] %d steps, %.3f ms/step" % (args.steps, ms_step), file=sys.stderr, flush=True)

    fl_step = flops_elementals(cfg.L, T, N, nmom) + flops_correlator(T, N, nmom, nprof)
    value = fl_step / (ms_step * 1e-3) / 1e12
    survey_value = flops_survey(cfg.L, T, N, nmom, nprof) / (ms_step * 1e-3) / 1e12

    chain_ms, chain_n = kt["corr_chain"]
    chain_avg = chain_ms / max(chain_n, 1)
    chain_fl_launch = flops_chain_kernel(T, N, nmom, nprof)  # one launch covers all (t, p) of the step
    achieved = chain_fl_launch / (chain_avg * 1e-3) / 1e12
    peak = FP32_PEAK_TFLOPS if args.precision == "fp32" else BF16X3_PEAK_TFLOPS
    kernels = {k: {"avg_ms": (v[0] / v[1] if v[1] else None), "launches": v[1]} for k, v in kt.items()}

    out = {
        "metric": "Nucleon corr-matrix TFLOP/s, BF16x3 vs FP32 @1e-6 rel err; p50/p99 job latency",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": "plain: 16^3x32 lattice, N_vec=32, 7 momenta, N_B=4 profiles "
                               "(3 Gaussian + linear), all 32 sink times, elementals + C_ab(t)",
                   "L": cfg.L, "T": T, "nvec": N, "nmom": nmom, "nprof": nprof, "precision": args.precision},
        "value_survey_convention": round(survey_value, 3),
        "roofline": {"bound": "mfma", "kernel": "corr_chain", "achieved": round(achieved, 3), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                     "avg_launch_ms": round(chain_avg, 4),
                     "flops_per_launch": chain_fl_launch},
        "kernels": kernels,
    }
    if not args.no_cpu_baseline:
        print("[bench] oracle cpu baseline ...", file=sys.stderr, flush=True)
        sample = sorted(set(int(round(x)) for x in np.linspace(0, T - 1, args.cpu_sample)))
        cb, phi_ref, corr_ref = cpu_baseline(cfg, inp, sample)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        # parity of the timed run on the same sample (block-wise relative error)
        c = corr.cpu().numpy()[:, sample]
        p = phi.cpu().numpy()[sample]
        ec = np.linalg.norm((c - corr_ref).reshape(-1, nprof * nprof), axis=1) / \
            np.linalg.norm(corr_ref.reshape(-1, nprof * nprof), axis=1)
        ep = np.linalg.norm((p - phi_ref).reshape(-1, N ** 3), axis=1) / \
            np.linalg.norm(phi_ref.reshape(-1, N ** 3), axis=1)
        out["rel_err_vs_oracle"] = {"corr_max": float(ec.max()), "corr_median": float(np.median(ec)),
                                    "phi_max": float(ep.max())}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

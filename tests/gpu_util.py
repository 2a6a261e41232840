"""Helpers shared by the GPU tests: device upload and block-wise relative errors.

Relative error of an output block (one elemental Phi[t,p], or one N_B x N_B
matrix C[p,t]) is ||X - X_ref||_F / ||X_ref||_F; tests gate on the maximum
over blocks.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

TOL_FP32 = 1e-5     # FP32 path against the FP64 oracle
# BF16x3 cannot reach FP32's level by construction (each product keeps about 17
# bits: the lo*lo term and lo's own rounding are dropped); this gate is its
# measured error with a margin, not an accuracy target.
TOL_BF16X3_MEASURED = 5e-5
# The FP64 form is held to the relative tolerance the precision forms aim at.
TOL_FP64 = 1e-6
FORM_TOL = {"fp32": TOL_FP32, "bf16x3": TOL_BF16X3_MEASURED, "fp16x3": TOL_FP32, "fp64": TOL_FP64}


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    return torch


def announce(msg: str):
    print("[gpu] " + msg, file=sys.stderr, flush=True)


def to_dev(torch, a: np.ndarray, dtype):
    return torch.from_numpy(np.ascontiguousarray(a.astype(dtype))).to("cuda:0")


def block_rel_err(x: np.ndarray, ref: np.ndarray, block_ndim: int) -> np.ndarray:
    lead = x.shape[: x.ndim - block_ndim]
    xf = x.reshape(int(np.prod(lead)), -1)
    rf = ref.reshape(int(np.prod(lead)), -1)
    num = np.linalg.norm(xf - rf, axis=1)
    den = np.linalg.norm(rf, axis=1)
    return num / np.where(den == 0, 1.0, den)

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

"""Helpers shared by the GPU tests: device fixtures and oracle-side references."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2305_11645_amd import inputs as I

U24 = 2.0 ** -24   # FP32 unit roundoff
U_SPLIT = 2.0 ** -16  # bound on the relative error of one split-bf16 3-term product


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test selected but no HIP device is visible")
    return torch


def to_dev(a, torch):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def oracle_tables(wl, r):
    """FP64 distinct values of every coordinate (oracle), list indexed by j."""
    from oracle import oracle as O
    return [O.point_values(wl, r, j) for j in range(wl.s)]


def oracle_rows(wl, r, ks, tabs=None):
    """y_k = x_k^T A in FP64 for the sampled points ks, from the oracle's tables
    (x_kj = X_j[k mod n_j]), plus the magnitude sum |x_k|^T |A| for error bounds."""
    tabs = oracle_tables(wl, r) if tabs is None else tabs
    A = wl.A.astype(np.float64)
    X = np.array([[tabs[j][k % len(tabs[j])] for j in range(wl.s)] for k in ks])
    return X @ A, np.abs(X) @ np.abs(A)


def elementwise_bound(wl, prec):
    """Worst-case relative-to-|X||A| error of an FP32 evaluation of x^T A with
    FP32-rounded point values: table rounding u plus a summation depth <= s + 2;
    split-bf16 adds one product error of the 3-term split."""
    b = (wl.s + 3) * U24
    if prec == I.SPLIT_BF16X3:
        b += 2 * U_SPLIT
    return b

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


# ------------------------------------------------------------------ gradient bounds

# v_sin / v_cos absolute error allowance (values of magnitude <= 1), generous
EPS_SIN = 2.0 ** -19


def adjoint_chain(wl, pts) -> int:
    """Longest chain of FP32 roundings a term of dA passes through on the GPU
    before its FP64 combination.
    Tree path (base 2, periodic): inside a subtree at most 2^{L'} <= 64 leaf
    terms per level product and L' folds, the per-wave accumulator over at
    most 33 subtrees, the waves of a workgroup; above L' the fold pyramid
    (<= m levels) and the adjoint level products over K-chunks of <= 256 rows
    (the bound allows 1024).
    Gathered tiles: the matrix cores sum at most 4096 points before each FP64
    flush; in base b > 2 the upper coordinates first fold b^{L'} points."""
    if wl.b == 2 and pts.grad_split_level >= 0:
        return 1024 + wl.m + 64 + 33 + 8
    L = max(pts.grad_split_level, 0)
    return 4096 + wl.b ** L + 16


def sensitivity_terms(wl, Y, magY, prec):
    """Per point and column, from the exact FP64 products Y and |x_k|^T|A|:
      Gabs   |G_ki| = |h'(u_k)| |g'(y_ki)| / (N t)   (the oracle's sensitivities)
      Gerr   what the GPU's G_ki may be off by: the FP32 error of y_ki (the
             forward bound) carried through g'', the transcendental's own
             error, and, for h = max(0, u - K), the whole of g'/(N t) at
             points whose u_k lies within its own error of K (h' may flip)."""
    N, t = Y.shape
    u = U24
    dy = ((wl.s + 8) * u + (2 * U_SPLIT if prec == I.SPLIT_BF16X3 else 0.0)) * magY
    if wl.g == I.G_COS:
        g, g1, g2 = np.cos(Y), -np.sin(Y), -np.cos(Y)
        eps1 = EPS_SIN + u * np.abs(Y)
        eps0 = eps1
    elif wl.g == I.G_EXP:
        g = np.exp(wl.c * Y)
        g1, g2 = wl.c * g, wl.c * wl.c * g
        rel = 4 * u + u * abs(wl.c) * np.abs(Y)
        eps1, eps0 = np.abs(g1) * rel, np.abs(g) * rel
    else:
        g, g1, g2 = Y, np.ones_like(Y), np.zeros_like(Y)
        eps1 = eps0 = np.zeros_like(Y)
    scale = 1.0 / (N * t)
    if wl.h == I.H_ID:
        hp = np.ones(N)
        flip = np.zeros(N, dtype=bool)
    else:
        ug = g.mean(axis=1)
        du = (np.abs(g1) * dy + eps0).mean(axis=1) + 2 * (64 + t) * u * np.abs(g).mean(axis=1)
        hp = (ug > wl.K).astype(np.float64)
        flip = np.abs(ug - wl.K) <= du
    hmag = np.maximum(hp, flip.astype(np.float64))[:, None]
    Gabs = scale * hp[:, None] * np.abs(g1)
    Gerr = scale * (hmag * (np.abs(g2) * dy + eps1) + flip[:, None] * np.abs(g1))
    return Gabs, Gerr


def grad_bound_dense(wl, r, prec, D):
    """Element-wise bound E[j, i] on |dA_gpu - dA_oracle| for randomisation r,
    from the dense point matrix (small cases):
        E = (D u + 2u [+ 2 u_split]) (|X|^T |G|) + |X|^T Gerr."""
    from oracle import oracle as O
    X = O.point_matrix_unreduced(wl, r)
    A = wl.A.astype(np.float64)
    Y = X @ A
    magY = np.abs(X) @ np.abs(A)
    Gabs, Gerr = sensitivity_terms(wl, Y, magY, prec)
    c = (D + 2) * U24 + (2 * U_SPLIT if prec == I.SPLIT_BF16X3 else 0.0)
    aX = np.abs(X)
    return c * (aX.T @ Gabs) + aX.T @ Gerr


def check_grad_elementwise(dA, dAo, E, what=""):
    """|dA - dAo| <= E element by element; returns the worst ratio."""
    err = np.abs(dA.astype(np.float64) - dAo)
    ratio = err / (E + 1e-300)
    worst = float(ratio.max())
    j, i = np.unravel_index(int(np.argmax(ratio)), ratio.shape)
    assert worst <= 1.0, (f"{what} dA[{j},{i}] error {err[j, i]:.3e} exceeds its bound {E[j, i]:.3e} "
                          f"({worst:.3g} x)")
    return worst


def grad_bound_lattice(wl, r, prec, D):
    """The bound of grad_bound_dense for a point set with x_kj = X_j[k mod n_j]
    and nonnegative values (a base-2 lattice without map, shifted or not), at
    any size: |X|^T M is formed from the distinct values and the sums of M over
    the residue classes k mod n_j, and |x_k|^T|A| = x_k^T|A| by the oracle's
    reduced product with |A|."""
    from oracle import oracle as O
    A = wl.A.astype(np.float64)
    Y = O.reduced_matvec(wl, r, A=A)
    magY = O.reduced_matvec(wl, r, A=np.abs(A))
    Gabs, Gerr = sensitivity_terms(wl, Y, magY, prec)
    del Y, magY
    c = (D + 2) * U24 + (2 * U_SPLIT if prec == I.SPLIT_BF16X3 else 0.0)
    M = c * Gabs + Gerr
    del Gabs, Gerr
    N, t = M.shape
    E = np.zeros((wl.s, t))
    folded = {}
    for j in range(wl.s):
        tab = O.point_values(wl, r, j)
        assert np.all(tab >= 0.0), "grad_bound_lattice needs nonnegative point values"
        n = len(tab)
        if n not in folded:
            folded[n] = M.reshape(N // n, n, t).sum(axis=0)
        E[j] = tab @ folded[n]
    return E

"""Brute-force point sets from the paper's unreduced definitions (tiny m only).

Independent of the C oracle: exact rational arithmetic with Python integers
and Fractions, explicit digit vectors, explicit F_2 matrices and polynomials.
Used to pin the oracle's point tables.

  lattice      Sec. 1.1 / 1.3: x_k = {k z / N}, z_j = b^{w_j} z'_j, N = b^m (any prime b)
  polynomial   Sec. 1.1: x_k = nu(k(x) g_j(x) / x^m), g_j = x^{w_j} g'_j
  digital net  eq. def:digital with the reduced matrices of eq.
               reduced_genmat_net2: last min(w_j, m) rows of C^{(j)} set to 0
               (polynomials and matrices over F_b, any prime b)
  reduced MC   Sec. 4, eq. randpts: the mixed-radix digits of n select the
               sample of each coordinate (greedy from the top digit down)
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np
from scipy.special import ndtri

from paper_2305_11645_amd.inputs import (DIGITAL_NET, DIGITAL_SHIFT, IID, LATTICE, MAP_CENTER,
                                         MAP_INVNORM, MAP_TENT, POLY_LATTICE, RANDOM_SHIFT)


def digits(n: int, m: int, b: int = 2) -> list[int]:
    """b-adic digits of n, least significant first."""
    return [(n // b ** q) % b for q in range(m)]


def net_matrix(wl, j: int) -> list[list[int]]:
    """C^{(j)} as an m x m matrix over F_b: row p-1 = output digit p, column
    q-1 = input digit q; entry (p, q) is base-b digit p-1 of column word q-1."""
    m = wl.m
    C = [[0] * m for _ in range(m)]
    for q in range(m):
        col = digits(int(wl.gen[j * m + q]), m, wl.b)
        for p in range(m):
            C[p][q] = col[p]
    return C


def reduced_net_matrix(wl, j: int) -> list[list[int]]:
    m = wl.m
    C = net_matrix(wl, j)
    keep = m - min(int(wl.w[j]), m)
    for p in range(keep, m):
        C[p] = [0] * m
    return C


def poly_mul_mod2(a: list[int], b: list[int]) -> list[int]:
    out = [0] * (len(a) + len(b))
    for i, ai in enumerate(a):
        if ai:
            for k, bk in enumerate(b):
                out[i + k] ^= bk
    return out


def poly_mul_modb(a: list[int], g: list[int], b: int) -> list[int]:
    """Product in F_b[x] of two coefficient lists (lowest degree first)."""
    out = [0] * (len(a) + len(g))
    for i, ai in enumerate(a):
        for k, gk in enumerate(g):
            out[i + k] = (out[i + k] + ai * gk) % b
    return out


def unshifted_value(wl, k: int, j: int) -> Fraction:
    """The unreduced point definition, as an exact fraction in [0, 1)."""
    m, N = wl.m, wl.b ** wl.m
    w = int(wl.w[j])
    if wl.kind == LATTICE:
        z = (wl.b ** w) * int(wl.gen[j])
        return Fraction((k * z) % N, N)
    b = wl.b
    if wl.kind == POLY_LATTICE:
        gp = digits(int(wl.gen[j]), 64 if b == 2 else m, b)
        g = [0] * w + gp                           # x^{w_j} g'_j(x)
        if b == 2:
            f = poly_mul_mod2(digits(k, m), g)[:m]     # k(x) g_j(x) mod x^m
        else:
            f = poly_mul_modb(digits(k, m, b), g, b)[:m]
        return sum((Fraction(f[i], b ** (m - i)) for i in range(m)), Fraction(0))
    C = reduced_net_matrix(wl, j)
    n = digits(k, m, b)
    y = [sum(C[p][q] * n[q] for q in range(m)) % b for p in range(m)]
    return sum((Fraction(y[p], b ** (p + 1)) for p in range(m)), Fraction(0))


def shift_digits(b: int) -> int:
    """K: the largest number of base-b digits with b^K <= 2^52 (52 for b = 2)."""
    K = 0
    while b ** (K + 1) <= 2 ** 52:
        K += 1
    return K


def digital_shift(x: Fraction, delta: int, b: int = 2) -> float:
    """Digit-wise addition mod b of the first K base-b digits of x and of delta
    (delta's digits most significant first; XOR for b = 2); the tail is
    replaced by its midpoint b^-K / 2."""
    K = shift_digits(b)
    assert (x * b ** K).denominator == 1
    xd = [int(x * b ** (p + 1)) % b for p in range(K)]             # digit p+1 of x
    sd = [(delta // b ** (K - 1 - p)) % b for p in range(K)]       # digit p+1 of delta / b^K
    val = sum((Fraction((xd[p] + sd[p]) % b, b ** (p + 1)) for p in range(K)), Fraction(0))
    return float(val + Fraction(1, 2 * b ** K))


def randpts_index(wl, n: int, j: int) -> int:
    """eq. randpts: with N_i = b^{m - min(w_i, m)}, N_{s+1} = 1, write
    n = m_1 N_2 + m_2 N_3 + ... + m_s N_{s+1} (0 <= m_i < N_i / N_{i+1}, top
    digit first); coordinate j takes sample m_j N_{j+1} + ... + m_s N_{s+1}."""
    m, s = wl.m, wl.s
    Nn = [wl.b ** (m - min(int(wl.w[i]), m)) for i in range(s)] + [1]
    rest, dig = n, []
    for i in range(s):
        dig.append(rest // Nn[i + 1])
        rest -= dig[-1] * Nn[i + 1]
    assert rest == 0 and all(0 <= dig[i] < Nn[i] // Nn[i + 1] for i in range(s))
    return sum(dig[i] * Nn[i + 1] for i in range(j, s))


def value(wl, r: int, k: int, j: int) -> float:
    """Point k, coordinate j, shift r, after the map (FP64)."""
    if wl.kind == IID:
        nb = [wl.m - min(int(wl.w[i]), wl.m) for i in range(wl.s)]
        off = sum(wl.b ** nb[i] for i in range(j))
        v = float(wl.samples[r, off + randpts_index(wl, k, j)])
    elif wl.rand == DIGITAL_SHIFT:
        v = digital_shift(unshifted_value(wl, k, j), int(wl.dshift[r, j]), wl.b)
    else:
        v = float(unshifted_value(wl, k, j))
        if wl.rand == RANDOM_SHIFT:
            v = v + float(wl.shift[r, j])
            if v >= 1.0:
                v = v - 1.0
    if wl.map == MAP_CENTER:
        return v - 0.5
    if wl.map == MAP_TENT:
        return 1.0 - abs(1.0 - 2.0 * v)
    if wl.map == MAP_INVNORM:
        return float(ndtri(v))
    return v


def point_matrix(wl, r: int = 0) -> np.ndarray:
    N = wl.b ** wl.m
    return np.array([[value(wl, r, k, j) for j in range(wl.s)] for k in range(N)])

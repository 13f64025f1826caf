"""Seeded synthetic inputs for the reduced QMC matrix-vector product.

This module only draws and assembles inputs: generating vectors or generating
matrices, reduction indices, the matrix A, and the random shifts.  It holds
none of the method's arithmetic (no point values, no products, no integrands),
so the FP64 oracle and the HIP library can both be fed from it without sharing
any computation.

The five workloads mirror the shapes of the paper's experiments (Section 5:
b = 2, reduction indices of the form floor(log2 j^c)) and of its motivating
applications (Section 1: Gaussian expectations through a factor of the
covariance, and PDE coefficients written as x^T A).  Indices are 0-based here,
so the paper's w_j = floor(log2 j) for j = 1..s becomes floor(log2(j+1)).

Draw order per workload: generators, then A, then shifts (or, for reduced
Monte Carlo, the i.i.d. samples), all from ``numpy.random.default_rng(seed)``
with ``seed = 1000 + c`` by default.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# enum values shared by convention with include/qmcred.h (plain integers)
LATTICE, POLY_LATTICE, DIGITAL_NET, IID = 0, 1, 2, 3
NO_SHIFT, RANDOM_SHIFT, DIGITAL_SHIFT = 0, 1, 2
MAP_ID, MAP_CENTER, MAP_INVNORM, MAP_TENT = 0, 1, 2, 3
G_ID, G_COS, G_EXP = 0, 1, 2
H_ID, H_CALL = 0, 1
FP32, SPLIT_BF16X3 = 0, 1


@dataclass
class Workload:
    """One synthetic problem instance: point set, A and integrand."""

    name: str
    kind: int
    b: int
    m: int
    s: int
    t: int
    w: np.ndarray            # int32 [s], non-decreasing, w[0] == 0
    gen: np.ndarray          # uint64: lattice z'_j [s]; poly g'_j [s]; net column words [s*m]
    rand: int
    R: int
    shift: np.ndarray | None   # float64 [R, s] in [0, 1)        (RANDOM_SHIFT)
    dshift: np.ndarray | None  # uint64  [R, s] in [0, 2^52)     (DIGITAL_SHIFT)
    map: int
    A64: np.ndarray          # float64 [s, t], as drawn
    g: int
    c: float
    h: int
    K: float
    prec: int = FP32
    samples: np.ndarray | None = None  # float64 [R, sum_j n_j] in (0, 1)    (kind IID)
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.b ** self.m

    @property
    def A(self) -> np.ndarray:
        """A rounded to FP32: the matrix both the oracle and the GPU consume."""
        return np.ascontiguousarray(self.A64.astype(np.float32))

    def nbits(self) -> np.ndarray:
        """m - min(w_j, m): coordinate j takes b**nbits[j] distinct values."""
        return (self.m - np.minimum(self.w, self.m)).astype(np.int64)


# ---------------------------------------------------------------- w rules

def w_log2(s: int, cap: int) -> np.ndarray:
    """w_j = min(cap, floor(log2(j+1))), j = 0..s-1 (exact integer arithmetic)."""
    return np.array([min(cap, (j + 1).bit_length() - 1) for j in range(s)], dtype=np.int32)


def w_logb(s: int, cap: int, b: int) -> np.ndarray:
    """w_j = min(cap, floor(log_b(j+1))), j = 0..s-1: the largest q with b^q <= j+1."""
    out = []
    for j in range(s):
        q = 0
        while b ** (q + 1) <= j + 1:
            q += 1
        out.append(min(cap, q))
    return np.array(out, dtype=np.int32)


def w_logb_pow(s: int, cap: int, num: int, den: int, b: int) -> np.ndarray:
    """w_j = min(cap, floor((num/den) * log_b(j+1))), exact: largest q with b^(q*den) <= (j+1)^num."""
    out = []
    for j in range(s):
        n = (j + 1) ** num
        q = 0
        while b ** ((q + 1) * den) <= n:
            q += 1
        out.append(min(cap, q))
    return np.array(out, dtype=np.int32)


def w_log2_pow(s: int, cap: int, num: int, den: int) -> np.ndarray:
    """w_j = min(cap, floor((num/den) * log2(j+1))), exact: largest q with 2^(q*den) <= (j+1)^num."""
    out = []
    for j in range(s):
        n = (j + 1) ** num
        q = 0
        while (1 << ((q + 1) * den)) <= n:
            q += 1
        out.append(min(cap, q))
    return np.array(out, dtype=np.int32)


# ---------------------------------------------------------------- generators

def draw_lattice(rng: np.random.Generator, nb: np.ndarray, b: int = 2) -> np.ndarray:
    """z'_j uniform over the units modulo b^nb_j (the integers in [1, b^nb_j)
    not divisible by b; for b = 2 the odd ones); z'_j = 1 when nb_j = 0."""
    z = np.ones(len(nb), dtype=np.uint64)
    for j, n in enumerate(nb):
        if n >= 1:
            if b == 2:
                z[j] = np.uint64(2 * int(rng.integers(0, 1 << (int(n) - 1))) + 1)
            else:
                q = int(rng.integers(0, b ** (int(n) - 1)))
                z[j] = np.uint64(b * q + int(rng.integers(1, b)))
    return z


def draw_poly(rng: np.random.Generator, nb: np.ndarray, b: int = 2) -> np.ndarray:
    """g'_j in F_b[x] with degree < nb_j and a nonzero constant term, given as
    the integer g'_j(b) (coefficient i = base-b digit i; for b = 2 the bit mask
    with constant term 1)."""
    if b == 2:
        return draw_lattice(rng, nb)  # same distribution over bit masks
    g = np.ones(len(nb), dtype=np.uint64)
    for j, n in enumerate(nb):
        if n >= 1:
            coef = [int(rng.integers(1, b))] + [int(rng.integers(0, b)) for _ in range(int(n) - 1)]
            g[j] = np.uint64(sum(c * b ** i for i, c in enumerate(coef)))
    return g


def shift_digits(b: int) -> int:
    """K: the base-b digits of a digital shift, the largest with b^K <= 2^52."""
    K = 0
    while b ** (K + 1) <= 1 << 52:
        K += 1
    return K


def draw_dshift(rng: np.random.Generator, R: int, s: int, b: int = 2) -> np.ndarray:
    """Digital shifts: integers uniform below b^K, whose K base-b digits (most
    significant first) are added to the point's digits mod b."""
    if b == 2:
        return rng.integers(0, 1 << 52, size=(R, s), dtype=np.uint64)
    return rng.integers(0, b ** shift_digits(b), size=(R, s), dtype=np.uint64)


def draw_net_lower(rng: np.random.Generator, s: int, m: int, b: int = 2) -> np.ndarray:
    """Random lower-triangular generating matrices over F_b with a nonzero
    diagonal (F_2: unit diagonal).

    Entry C_{p,q} (output digit p, input digit q, both 1-based) is zero for
    q > p, nonzero on the diagonal, and independent uniform below it.  Returned
    as column words: word (j, q-1) holds C^{(j)}_{p,q} as its base-b digit p-1
    (for b = 2, bit p-1).  The full (unreduced) matrices are returned; the
    reduction by w is applied by the consumer.
    """
    if b != 2:
        words = np.zeros(s * m, dtype=np.uint64)
        for j in range(s):
            for q in range(m):
                col = [0] * q + [int(rng.integers(1, b))] + [int(rng.integers(0, b)) for _ in range(m - q - 1)]
                words[j * m + q] = np.uint64(sum(c * b ** p for p, c in enumerate(col)))
        return words
    words = np.zeros(s * m, dtype=np.uint64)
    for j in range(s):
        bits = rng.integers(0, 2, size=(m, m))
        for q in range(m):
            word = 1 << q  # diagonal C_{q+1,q+1}
            for p in range(q + 1, m):
                if bits[p, q]:
                    word |= 1 << p
            words[j * m + q] = np.uint64(word)
    return words


def draw_iid_samples(rng: np.random.Generator, R: int, nb: np.ndarray, b: int = 2) -> np.ndarray:
    """Reduced Monte Carlo inputs: for each of R replicates and each coordinate j,
    b^nb_j independent uniforms, coordinate blocks contiguous: [R, sum_j b^nb_j].
    Each value is (k + 1/2) 2^-53 with k uniform below 2^53: exact in FP64 and
    strictly inside (0, 1), so the inverse-normal map is always finite."""
    total = int(sum(b ** int(n) for n in nb))
    k = rng.integers(0, 1 << 53, size=(R, total), dtype=np.uint64)
    return (k.astype(np.float64) + 0.5) * 2.0 ** -53


def tridiag_cholesky_T(s: int, diag: float = 0.4, off: float = 0.2) -> np.ndarray:
    """A = L^T with L L^T = Sigma, Sigma tridiagonal Toeplitz (diag on the
    diagonal, off next to it): the basket-option covariance of Section 5."""
    Sig = np.diag(np.full(s, diag)) + np.diag(np.full(s - 1, off), 1) + np.diag(np.full(s - 1, off), -1)
    return np.ascontiguousarray(np.linalg.cholesky(Sig).T)


def draw_net_upper(rng: np.random.Generator, s: int, m: int, b: int = 2) -> np.ndarray:
    """Random upper-triangular generating matrices over F_b with a nonzero
    diagonal (the shape of Sobol' matrices; F_2: unit diagonal): C_{p,q} = 0
    for p > q, uniform digits above the diagonal.  Column words as in
    draw_net_lower.  After the row reduction the points still depend on every
    digit of k (not periodic), so products over them need Algorithm 4."""
    if b != 2:
        words = np.zeros(s * m, dtype=np.uint64)
        for j in range(s):
            for q in range(m):
                col = [int(rng.integers(0, b)) for _ in range(q)] + [int(rng.integers(1, b))] + [0] * (m - q - 1)
                words[j * m + q] = np.uint64(sum(c * b ** p for p, c in enumerate(col)))
        return words
    words = np.zeros(s * m, dtype=np.uint64)
    for j in range(s):
        bits = rng.integers(0, 2, size=(m, m))
        for q in range(m):
            word = 1 << q
            for p in range(q):
                if bits[p, q]:
                    word |= 1 << p
            words[j * m + q] = np.uint64(word)
    return words


# ---------------------------------------------------------------- A matrices

def exp_kernel_cholesky_T(n: int, ell: float = 0.1) -> np.ndarray:
    """A = L^T with L L^T = K, K_uv = exp(-|u_u - u_v|/ell) on u_i = (i+1/2)/n."""
    u = (np.arange(n) + 0.5) / n
    Kmat = np.exp(-np.abs(u[:, None] - u[None, :]) / ell)
    L = np.linalg.cholesky(Kmat)
    return np.ascontiguousarray(L.T)


def kl_matrix(s: int, t: int) -> np.ndarray:
    """A_ji = (j+1)^-2 sin((j+1) pi xi_i), xi_i = (i+1/2)/t."""
    j = np.arange(1, s + 1, dtype=np.float64)[:, None]
    xi = (np.arange(t, dtype=np.float64)[None, :] + 0.5) / t
    return j ** -2.0 * np.sin(j * math.pi * xi)


# ---------------------------------------------------------------- workloads

CONFIG_NAMES = {
    1: "C1 reduced lattice m=10 s=t=64 cos-mean",
    2: "C2 shifted reduced lattice m=16 s=t=256 R=8 cos-mean",
    3: "C3 digitally shifted reduced net m=20 s=t=1024 Gaussian call",
    4: "C4 KL coefficients reduced lattice m=18 s=2048 t=4096 R=32 exp-mean",
    5: "C5 shifted reduced lattice m=20 s=t=1024 cos-mean gradient",
    6: "C6 reduced Monte Carlo basket call m=20 s=t=512 R=4",
    7: "C7 digitally shifted reduced Sobol'-type net (Algorithm 4) m=16 s=t=512 R=2 Gaussian cos-mean",
    8: "C8 shifted reduced lattice in base 3 m=10 (N=59049) s=t=256 R=8 cos-mean",
}

# Basket option of Section 5 (Black-Scholes, zero rate): S_j(0) = 100, T = 1,
# strike 110, Sigma_jj = 0.4.  S_j(T) = 100 exp(-0.2 + y_j), so the payoff is
# BASKET_SCALE * max(0, mean_j exp(y_j) - BASKET_K): the library's estimate
# times BASKET_SCALE is the option price.
BASKET_SCALE = 100.0 * math.exp(-0.2)
BASKET_K = 110.0 / BASKET_SCALE


def make_config(c: int, seed: int | None = None, *, m: int | None = None, s: int | None = None,
                t: int | None = None, R: int | None = None, kind: int | None = None) -> Workload:
    """Build workload C<c> (1..8).  Size overrides give the same recipe at other shapes."""
    if seed is None:
        seed = 1000 + c
    rng = np.random.default_rng(seed)
    if c == 1:
        m_, s_, t_, R_ = 10, 64, 64, 1
        m_, s_, t_, R_ = m or m_, s or s_, t or t_, R or R_
        w = w_log2(s_, max(m_ - 2, 0))
        kind_ = LATTICE if kind is None else kind
        rand, mp = NO_SHIFT, MAP_ID
        g, cc, h, K = G_COS, 1.0, H_ID, 0.0
        A_fn = lambda: rng.standard_normal((s_, t_))
        prec = FP32
    elif c == 2:
        m_, s_, t_, R_ = 16, 256, 256, 8
        m_, s_, t_, R_ = m or m_, s or s_, t or t_, R or R_
        w = w_log2_pow(s_, max(m_ - 4, 0), 3, 2)
        kind_ = LATTICE if kind is None else kind
        rand, mp = RANDOM_SHIFT, MAP_ID
        g, cc, h, K = G_COS, 1.0, H_ID, 0.0
        A_fn = lambda: rng.standard_normal((s_, t_)) / math.sqrt(s_)
        prec = FP32
    elif c == 3:
        m_, s_, t_, R_ = 20, 1024, 1024, 1
        m_, s_, t_, R_ = m or m_, s or s_, t or t_, R or R_
        w = w_log2(s_, max(m_ - 4, 0))
        kind_ = DIGITAL_NET if kind is None else kind
        rand, mp = DIGITAL_SHIFT, MAP_INVNORM
        g, cc, h, K = G_EXP, 0.2, H_CALL, 1.0
        if s_ != t_:
            raise ValueError("C3 uses a square Cholesky factor: s must equal t")
        A_fn = lambda: exp_kernel_cholesky_T(s_)
        prec = SPLIT_BF16X3
    elif c == 4:
        m_, s_, t_, R_ = 18, 2048, 4096, 32
        m_, s_, t_, R_ = m or m_, s or s_, t or t_, R or R_
        w = w_log2(s_, max(m_ - 4, 0))
        kind_ = LATTICE if kind is None else kind
        rand, mp = RANDOM_SHIFT, MAP_CENTER
        g, cc, h, K = G_EXP, -1.0, H_ID, 0.0
        A_fn = lambda: kl_matrix(s_, t_)
        prec = FP32
    elif c == 5:
        m_, s_, t_, R_ = 20, 1024, 1024, 1
        m_, s_, t_, R_ = m or m_, s or s_, t or t_, R or R_
        w = w_log2(s_, max(m_ - 4, 0))
        kind_ = LATTICE if kind is None else kind
        rand, mp = RANDOM_SHIFT, MAP_ID
        g, cc, h, K = G_COS, 1.0, H_ID, 0.0
        A_fn = lambda: rng.standard_normal((s_, t_)) / math.sqrt(s_)
        prec = FP32
    elif c == 6:
        m_, s_, t_, R_ = 20, 512, 512, 4
        m_, s_, t_, R_ = m or m_, s or s_, t or t_, R or R_
        w = w_log2(s_, max(m_ - 4, 0))
        kind_ = IID
        rand, mp = NO_SHIFT, MAP_INVNORM
        g, cc, h, K = G_EXP, 1.0, H_CALL, BASKET_K
        if s_ != t_:
            raise ValueError("C6 uses a square Cholesky factor: s must equal t")
        A_fn = lambda: tridiag_cholesky_T(s_)
        prec = FP32
    elif c == 7:
        m_, s_, t_, R_ = 16, 512, 512, 2
        m_, s_, t_, R_ = m or m_, s or s_, t or t_, R or R_
        w = w_log2(s_, max(m_ - 4, 0))
        kind_ = DIGITAL_NET if kind is None else kind
        rand, mp = DIGITAL_SHIFT, MAP_INVNORM
        g, cc, h, K = G_COS, 1.0, H_ID, 0.0
        A_fn = lambda: rng.standard_normal((s_, t_)) / math.sqrt(s_)
        prec = FP32
    elif c == 8:
        # C2's shape, integrand and w rule in base 3: w_j = floor(1.5 log_3(j+1)),
        # capped at m - 2
        b_ = 3
        m_, s_, t_, R_ = 10, 256, 256, 8
        m_, s_, t_, R_ = m or m_, s or s_, t or t_, R or R_
        w = w_logb_pow(s_, max(m_ - 2, 0), 3, 2, b_)
        kind_ = LATTICE if kind is None else kind
        rand, mp = RANDOM_SHIFT, MAP_ID
        g, cc, h, K = G_COS, 1.0, H_ID, 0.0
        A_fn = lambda: rng.standard_normal((s_, t_)) / math.sqrt(s_)
        prec = FP32
    else:
        raise ValueError(f"unknown workload C{c}")
    b_ = b_ if c == 8 else 2

    nb = (m_ - np.minimum(w, m_)).astype(np.int64)
    if kind_ == LATTICE:
        gen = draw_lattice(rng, nb, b_)
    elif kind_ == POLY_LATTICE:
        gen = draw_poly(rng, nb)
    elif kind_ == DIGITAL_NET:
        gen = draw_net_upper(rng, s_, m_) if c == 7 else draw_net_lower(rng, s_, m_)
    elif kind_ == IID:
        gen = np.ones(s_, dtype=np.uint64)  # unused
    else:
        raise ValueError("kind")
    A64 = np.ascontiguousarray(A_fn(), dtype=np.float64)
    shift = dshift = samples = None
    if kind_ == IID:
        samples = draw_iid_samples(rng, R_, nb, b_)
    elif rand == RANDOM_SHIFT:
        shift = rng.random((R_, s_))
    elif rand == DIGITAL_SHIFT:
        dshift = rng.integers(0, 1 << 52, size=(R_, s_), dtype=np.uint64)
    else:
        R_ = 1
    return Workload(name=CONFIG_NAMES[c], kind=kind_, b=b_, m=m_, s=s_, t=t_, w=w,
                    gen=gen, rand=rand, R=R_, shift=shift, dshift=dshift, map=mp,
                    A64=A64, g=g, c=cc, h=h, K=K, prec=prec, samples=samples)


def make_custom(*, kind: int, m: int, s: int, t: int, w: np.ndarray, rand: int = NO_SHIFT,
                R: int = 1, map: int = MAP_ID, g: int = G_COS, c: float = 1.0, h: int = H_ID,
                K: float = 0.0, A_scale: float = 1.0, seed: int = 7, net: str = "lower",
                b: int = 2) -> Workload:
    """A small random workload of any shape (tests): N(0,1)*A_scale matrix, random
    generators; a prime base b > 2 is for lattices and reduced Monte Carlo."""
    rng = np.random.default_rng(seed)
    w = np.asarray(w, dtype=np.int32)
    nb = (m - np.minimum(w, m)).astype(np.int64)
    if kind == LATTICE:
        gen = draw_lattice(rng, nb, b)
    elif kind == POLY_LATTICE:
        gen = draw_poly(rng, nb, b)
    elif kind == IID:
        gen = np.ones(s, dtype=np.uint64)  # unused
    elif net == "upper":
        gen = draw_net_upper(rng, s, m, b)
    else:
        gen = draw_net_lower(rng, s, m, b)
    A64 = rng.standard_normal((s, t)) * A_scale
    shift = dshift = samples = None
    if kind == IID:
        if rand != NO_SHIFT:
            raise ValueError("reduced Monte Carlo takes no shift: R counts independent replicates")
        samples = draw_iid_samples(rng, R, nb, b)
    elif rand == RANDOM_SHIFT:
        shift = rng.random((R, s))
    elif rand == DIGITAL_SHIFT:
        dshift = draw_dshift(rng, R, s, b)
    else:
        R = 1
    return Workload(name="custom", kind=kind, b=b, m=m, s=s, t=t, w=w, gen=gen, rand=rand,
                    R=R, shift=shift, dshift=dshift, map=map, A64=np.ascontiguousarray(A64),
                    g=g, c=c, h=h, K=K, samples=samples)

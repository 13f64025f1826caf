"""Python face of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It loads ``liboracle.so`` built from ``qmc_oracle.c``
(plain C, FP64, no FMA contraction) and marshals numpy arrays into it.  The
arithmetic lives in the C file; each C function cites the passage of the paper
it follows.  Nothing here is shared with the HIP library.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "qmc_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-std=c11", "-Wall", "-shared", "-fPIC", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Spec(ct.Structure):
    _fields_ = [("b", ct.c_int32), ("kind", ct.c_int32), ("m", ct.c_int32), ("s", ct.c_int32),
                ("w", ct.POINTER(ct.c_int32)), ("gen", ct.POINTER(ct.c_uint64)),
                ("rand", ct.c_int32), ("R", ct.c_int32),
                ("shift", ct.POINTER(ct.c_double)), ("dshift", ct.POINTER(ct.c_uint64)),
                ("map", ct.c_int32), ("samples", ct.POINTER(ct.c_double))]


class _Integrand(ct.Structure):
    _fields_ = [("g", ct.c_int32), ("c", ct.c_double), ("h", ct.c_int32), ("K", ct.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = ct.CDLL(LIB)
        P, I64P, DP = ct.POINTER(_Spec), ct.POINTER(ct.c_int64), ct.POINTER(ct.c_double)
        L.qo_point_values.argtypes = [P, ct.c_int, ct.c_int, DP]
        L.qo_point_matrix_unreduced.argtypes = [P, ct.c_int, DP]
        L.qo_dense_matvec.argtypes = [DP, ct.c_int64, ct.c_int, DP, ct.c_int, DP]
        L.qo_alg1.argtypes = [P, ct.c_int, DP, ct.c_int, ct.c_int, ct.c_int, DP, I64P]
        L.qo_estimate.argtypes = [P, DP, ct.c_int, ct.POINTER(_Integrand), DP, I64P]
        L.qo_estimate_grad.argtypes = [P, DP, ct.c_int, ct.POINTER(_Integrand), DP, DP]
        L.qo_reduced_matvec.argtypes = [P, ct.c_int, DP, ct.c_int, DP, I64P]
        L.qo_alg4.argtypes = [P, ct.c_int, DP, ct.c_int, ct.c_int, ct.c_int, DP, I64P]
        L.qo_output_values.argtypes = [P, ct.c_int, ct.c_int, DP]
        L.qo_net_is_periodic.argtypes = [P]
        L.qo_invnorm.argtypes = [ct.c_double]
        L.qo_invnorm.restype = ct.c_double
        L.qo_neumaier.argtypes = [DP, ct.c_int64]
        L.qo_neumaier.restype = ct.c_double
        L.qo_num_threads.restype = ct.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


class Spec:
    """Keeps the numpy arrays alive while the C struct points into them."""

    def __init__(self, wl):
        self.w = np.ascontiguousarray(wl.w, dtype=np.int32)
        self.gen = np.ascontiguousarray(wl.gen, dtype=np.uint64)
        self.shift = None if wl.shift is None else np.ascontiguousarray(wl.shift, dtype=np.float64)
        self.dshift = None if wl.dshift is None else np.ascontiguousarray(wl.dshift, dtype=np.uint64)
        samples = getattr(wl, "samples", None)
        self.samples = None if samples is None else np.ascontiguousarray(samples, dtype=np.float64)
        self.R = wl.R
        self.m, self.s = wl.m, wl.s
        self.c = _Spec(b=wl.b, kind=wl.kind, m=wl.m, s=wl.s,
                       w=self.w.ctypes.data_as(ct.POINTER(ct.c_int32)),
                       gen=self.gen.ctypes.data_as(ct.POINTER(ct.c_uint64)),
                       rand=wl.rand, R=wl.R,
                       shift=None if self.shift is None else _dp(self.shift),
                       dshift=None if self.dshift is None else
                       self.dshift.ctypes.data_as(ct.POINTER(ct.c_uint64)),
                       map=wl.map,
                       samples=None if self.samples is None else _dp(self.samples))


def _A64(wl):
    """The FP32-rounded A, promoted to FP64 (what the GPU consumes)."""
    return np.ascontiguousarray(wl.A.astype(np.float64))


def point_values(wl, r: int, j: int) -> np.ndarray:
    sp = Spec(wl)
    nb = int(wl.m - min(int(wl.w[j]), wl.m))
    out = np.empty(wl.b ** nb, dtype=np.float64)
    assert lib().qo_point_values(ct.byref(sp.c), r, j, _dp(out)) == 0
    return out


def point_matrix_unreduced(wl, r: int = 0) -> np.ndarray:
    sp = Spec(wl)
    X = np.empty((wl.N, wl.s), dtype=np.float64)
    assert lib().qo_point_matrix_unreduced(ct.byref(sp.c), r, _dp(X)) == 0
    return X


def dense_matvec(X: np.ndarray, A: np.ndarray) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float64)
    A = np.ascontiguousarray(A, dtype=np.float64)
    N, s = X.shape
    t = A.shape[1]
    Y = np.empty((N, t), dtype=np.float64)
    lib().qo_dense_matvec(_dp(X), N, s, _dp(A), t, _dp(Y))
    return Y


def alg1(wl, r: int, A: np.ndarray | None = None, i0: int = 0, i1: int | None = None):
    """Algorithm 1 on columns [i0, i1): returns (P, multiply-add count)."""
    sp = Spec(wl)
    A = _A64(wl) if A is None else np.ascontiguousarray(A, dtype=np.float64)
    t = A.shape[1]
    i1 = t if i1 is None else i1
    P = np.empty((wl.N, i1 - i0), dtype=np.float64)
    cnt = ct.c_int64(0)
    rc = lib().qo_alg1(ct.byref(sp.c), r, _dp(A), t, i0, i1, _dp(P), ct.byref(cnt))
    assert rc == 0
    return P, int(cnt.value)


def alg4(wl, r: int, A: np.ndarray | None = None, i0: int = 0, i1: int | None = None):
    """Algorithm 4 on columns [i0, i1) for shift r: (P, multiplication count)."""
    sp = Spec(wl)
    A = _A64(wl) if A is None else np.ascontiguousarray(A, dtype=np.float64)
    t = A.shape[1]
    i1 = t if i1 is None else i1
    P = np.empty((wl.N, i1 - i0), dtype=np.float64)
    cnt = ct.c_int64(0)
    rc = lib().qo_alg4(ct.byref(sp.c), r, _dp(A), t, i0, i1, _dp(P), ct.byref(cnt))
    assert rc == 0
    return P, int(cnt.value)


def output_values(wl, r: int, j: int) -> np.ndarray:
    """Values of coordinate j indexed by the integer of its reduced output digits."""
    sp = Spec(wl)
    n = wl.b ** int(wl.nbits()[j])
    out = np.empty(n, dtype=np.float64)
    assert lib().qo_output_values(ct.byref(sp.c), r, j, _dp(out)) == 0
    return out


def net_is_periodic(wl) -> bool:
    return bool(lib().qo_net_is_periodic(ct.byref(Spec(wl).c)))


def reduced_matvec(wl, r: int = 0, A: np.ndarray | None = None) -> np.ndarray:
    sp = Spec(wl)
    A = _A64(wl) if A is None else np.ascontiguousarray(A, dtype=np.float64)
    t = A.shape[1]
    Y = np.empty((wl.N, t), dtype=np.float64)
    rc = lib().qo_reduced_matvec(ct.byref(sp.c), r, _dp(A), t, _dp(Y), None)
    assert rc == 0
    return Y


def _integrand(wl):
    return _Integrand(g=wl.g, c=wl.c, h=wl.h, K=wl.K)


def estimate(wl, A: np.ndarray | None = None, shifts: int | None = None):
    """Q[r] for r < R (or the first `shifts` shifts) and the multiply-add count."""
    sp = Spec(wl)
    if shifts is not None:
        sp.c.R = min(shifts, wl.R)
    A = _A64(wl) if A is None else np.ascontiguousarray(A, dtype=np.float64)
    Q = np.empty(sp.c.R, dtype=np.float64)
    cnt = ct.c_int64(0)
    f = _integrand(wl)
    rc = lib().qo_estimate(ct.byref(sp.c), _dp(A), A.shape[1], ct.byref(f), _dp(Q), ct.byref(cnt))
    assert rc == 0
    return Q, int(cnt.value)


def estimate_grad(wl, A: np.ndarray | None = None, shifts: int | None = None):
    """(Q [R], dA [R, s, t]) in FP64."""
    sp = Spec(wl)
    if shifts is not None:
        sp.c.R = min(shifts, wl.R)
    A = _A64(wl) if A is None else np.ascontiguousarray(A, dtype=np.float64)
    t = A.shape[1]
    Q = np.empty(sp.c.R, dtype=np.float64)
    dA = np.empty((sp.c.R, wl.s, t), dtype=np.float64)
    f = _integrand(wl)
    rc = lib().qo_estimate_grad(ct.byref(sp.c), _dp(A), t, ct.byref(f), _dp(Q), _dp(dA))
    assert rc == 0
    return Q, dA


def invnorm(p: float) -> float:
    return lib().qo_invnorm(p)


def neumaier(x: np.ndarray) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib().qo_neumaier(_dp(x), len(x))


def num_threads() -> int:
    return lib().qo_num_threads()


def timed_estimate(wl, shifts: int | None = None):
    """Wall-clock the oracle estimate (table generation included)."""
    t0 = time.perf_counter()
    Q, _ = estimate(wl, shifts=shifts)
    return Q, time.perf_counter() - t0

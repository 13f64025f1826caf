"""Reduced QMC matrix-vector products on MI355X (gfx950).

Python face of libqmcred (include/qmcred.h).  This module only marshals
arguments: every step of the computation runs in the library's HIP kernels.
PyTorch provides device memory, the current stream and autograd plumbing.

    pts = Points.from_workload(wl)           # or Points(kind=..., m=..., ...)
    Q = estimate(pts, A, g=COS)              # float64 [R] on the GPU
    Y = reduced_matvec(pts, A, r=0)          # float32 [N, t]
    Q = QMCEstimate.apply(A, pts, f, prec)   # differentiable in A
"""
from __future__ import annotations

import ctypes as ct
from dataclasses import dataclass

import numpy as np

from ._lib import (EXPORTS, Integrand, PointSpec, QMCDeviceError, QMCError, QMCInvalid,
                   QMCNoMemory, QMCUnsupported, check, load)
from .inputs import (DIGITAL_NET, DIGITAL_SHIFT, FP32, IID, G_COS, G_EXP, G_ID, H_CALL, H_ID, LATTICE,
                     MAP_CENTER, MAP_ID, MAP_INVNORM, MAP_TENT, NO_SHIFT, POLY_LATTICE,
                     RANDOM_SHIFT, SPLIT_BF16X3)

__all__ = ["Points", "Integrand_", "estimate", "estimate_grad", "reduced_matvec", "point_values",
           "point_matrix", "QMCEstimate", "QMCError", "QMCInvalid", "QMCUnsupported",
           "QMCNoMemory", "QMCDeviceError", "EXPORTS", "timing", "probe_valu", "probe_mfma"]


def _torch():
    import torch
    return torch


def _stream():
    return ct.c_void_p(_torch().cuda.current_stream().cuda_stream)


@dataclass(frozen=True)
class Integrand_:
    """f(y) = h(t^-1 sum_i g(y_i)); g = exp(c y) for G_EXP, h = max(0, u - K) for H_CALL."""
    g: int = G_COS
    c: float = 1.0
    h: int = H_ID
    K: float = 0.0

    def c_struct(self) -> Integrand:
        return Integrand(g=self.g, c=self.c, h=self.h, K=self.K)

    @staticmethod
    def of(wl) -> "Integrand_":
        return Integrand_(g=wl.g, c=wl.c, h=wl.h, K=wl.K)


class Points:
    """A reduced point set living on the current GPU (wraps qmc_points_init)."""

    def __init__(self, *, kind: int, m: int, s: int, w, gen=None, rand: int = NO_SHIFT, R: int = 1,
                 shift=None, dshift=None, map: int = MAP_ID, b: int = 2, samples=None):
        L = load()
        self._w = np.ascontiguousarray(w, dtype=np.int32)
        self._gen = np.ascontiguousarray(np.ones(s) if gen is None else gen, dtype=np.uint64)
        self._samples = None if samples is None else np.ascontiguousarray(samples, dtype=np.float64)
        self._shift = None if shift is None else np.ascontiguousarray(shift, dtype=np.float64)
        self._dshift = None if dshift is None else np.ascontiguousarray(dshift, dtype=np.uint64)
        spec = PointSpec(
            b=b, m=m, s=s, kind=kind,
            w=self._w.ctypes.data_as(ct.POINTER(ct.c_int32)),
            gen=self._gen.ctypes.data_as(ct.POINTER(ct.c_uint64)),
            rand=rand, R=R,
            shift=None if self._shift is None else self._shift.ctypes.data_as(ct.POINTER(ct.c_double)),
            dshift=None if self._dshift is None else self._dshift.ctypes.data_as(ct.POINTER(ct.c_uint64)),
            map=map,
            samples=None if self._samples is None else self._samples.ctypes.data_as(ct.POINTER(ct.c_double)))
        h = ct.c_void_p()
        check(L.qmc_points_init(ct.byref(h), ct.byref(spec)))
        self._h = h
        self.b, self.m, self.s, self.R, self.kind, self.map, self.rand = b, m, s, R, kind, map, rand
        self.N = b ** m
        N, s_, R_, sp, dv = ct.c_int64(), ct.c_int32(), ct.c_int32(), ct.c_int32(), ct.c_int64()
        check(L.qmc_points_info(h, ct.byref(N), ct.byref(s_), ct.byref(R_), ct.byref(sp), ct.byref(dv)))
        self.split_level = sp.value
        gs = ct.c_int32()
        check(L.qmc_points_grad_split(h, ct.byref(gs)))
        self.grad_split_level = gs.value  # the gradient's (capped at 5)
        self.distinct_values = dv.value
        self.device = _torch().cuda.current_device()

    @classmethod
    def from_workload(cls, wl) -> "Points":
        return cls(kind=wl.kind, m=wl.m, s=wl.s, w=wl.w, gen=wl.gen, rand=wl.rand, R=wl.R,
                   shift=wl.shift, dshift=wl.dshift, map=wl.map, samples=getattr(wl, "samples", None),
                   b=wl.b)

    @property
    def handle(self) -> ct.c_void_p:
        return self._h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            load().qmc_points_free(self._h)
            self._h = ct.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, op: int, t: int, f: Integrand_ | None = None, prec: int = FP32) -> int:
        n = ct.c_size_t()
        fs = None if f is None else ct.byref(f.c_struct())
        check(load().qmc_workspace_size(self._h, op, t, fs, prec, ct.byref(n)))
        return n.value

    def workspace(self, op: int, t: int, f: Integrand_ | None = None, prec: int = FP32):
        torch = _torch()
        n = self.workspace_bytes(op, t, f, prec)
        return torch.empty(max(n, 256), dtype=torch.uint8, device=f"cuda:{self.device}")


def _check_A(A, s):
    torch = _torch()
    if not (isinstance(A, torch.Tensor) and A.is_cuda and A.dtype == torch.float32):
        raise TypeError("A must be a float32 CUDA (HIP) tensor")
    if A.dim() != 2 or A.shape[0] != s:
        raise ValueError(f"A must be s x t with s = {s}, got {tuple(A.shape)}")
    if A.stride(1) != 1:
        raise ValueError("A must have unit column stride (row-major)")


def point_values(pts: Points, r: int, j: int):
    """FP64 distinct values of coordinate j for randomisation r (device tensor)."""
    torch = _torch()
    nb = pts.m - min(int(pts._w[j]), pts.m)
    out = torch.empty(pts.b ** nb, dtype=torch.float64, device=f"cuda:{pts.device}")
    check(load().qmc_point_values(pts.handle, r, j, ct.c_void_p(out.data_ptr()), _stream()))
    return out


def point_matrix(pts: Points, r: int = 0):
    """The N x s FP32 point matrix of randomisation r (device tensor)."""
    torch = _torch()
    X = torch.empty((pts.N, pts.s), dtype=torch.float32, device=f"cuda:{pts.device}")
    check(load().qmc_point_matrix(pts.handle, r, ct.c_void_p(X.data_ptr()), pts.s, _stream()))
    return X


def reduced_matvec(pts: Points, A, r: int = 0, prec: int = FP32, Y=None, workspace=None):
    """Y = X A for randomisation r: float32 [N, t] device tensor."""
    torch = _torch()
    _check_A(A, pts.s)
    t = A.shape[1]
    if Y is None:
        Y = torch.empty((pts.N, t), dtype=torch.float32, device=A.device)
    ws = pts.workspace(0, t, None, prec) if workspace is None else workspace
    check(load().qmc_reduced_matvec(pts.handle, r, ct.c_void_p(A.data_ptr()), t, A.stride(0), prec,
                                    ct.c_void_p(Y.data_ptr()), Y.stride(0),
                                    ct.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return Y


def estimate(pts: Points, A, f: Integrand_ = Integrand_(), prec: int = FP32, Q=None, workspace=None):
    """Q[r] = N^-1 sum_k f(x_k^T A) for every randomisation: float64 [R] device tensor."""
    torch = _torch()
    _check_A(A, pts.s)
    t = A.shape[1]
    if Q is None:
        Q = torch.empty(pts.R, dtype=torch.float64, device=A.device)
    ws = pts.workspace(1, t, f, prec) if workspace is None else workspace
    check(load().qmc_estimate(pts.handle, ct.c_void_p(A.data_ptr()), t, A.stride(0),
                              ct.byref(f.c_struct()), prec, ct.c_void_p(Q.data_ptr()),
                              ct.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return Q


def estimate_grad(pts: Points, A, f: Integrand_ = Integrand_(), prec: int = FP32, workspace=None):
    """(Q [R] float64, dA [R, s, t] float32): dQ_r/dA for every randomisation."""
    torch = _torch()
    _check_A(A, pts.s)
    t = A.shape[1]
    Q = torch.empty(pts.R, dtype=torch.float64, device=A.device)
    dA = torch.empty((pts.R, pts.s, t), dtype=torch.float32, device=A.device)
    ws = pts.workspace(2, t, f, prec) if workspace is None else workspace
    check(load().qmc_estimate_grad(pts.handle, ct.c_void_p(A.data_ptr()), t, A.stride(0),
                                   ct.byref(f.c_struct()), prec, ct.c_void_p(Q.data_ptr()),
                                   ct.c_void_p(dA.data_ptr()), ct.c_void_p(ws.data_ptr()),
                                   ws.numel(), _stream()))
    return Q, dA


def _make_autograd():
    torch = _torch()

    class QMCEstimate(torch.autograd.Function):
        """Q = estimate(pts, A, f) with dQ/dA from the reduced adjoint (Y recomputed)."""

        @staticmethod
        def forward(ctx, A, pts, f=Integrand_(), prec=FP32):
            ctx.pts, ctx.f, ctx.prec = pts, f, prec
            ctx.save_for_backward(A)
            return estimate(pts, A, f, prec)

        @staticmethod
        def backward(ctx, gQ):
            (A,) = ctx.saved_tensors
            _, dA = estimate_grad(ctx.pts, A.contiguous(), ctx.f, ctx.prec)
            gA = (gQ.to(torch.float64).view(-1, 1, 1) * dA.to(torch.float64)).sum(dim=0)
            return gA.to(A.dtype), None, None, None

    return QMCEstimate


class _Lazy:
    _cls = None

    def __getattr__(self, name):
        if _Lazy._cls is None:
            _Lazy._cls = _make_autograd()
        return getattr(_Lazy._cls, name)


QMCEstimate = _Lazy()


def probe_valu():
    """Measured VALU issue rates of the current GPU (lane operations per second):
    {"fma": v_fma_f32, "exp": v_exp_f32 (+ one multiply), "sin": v_sin_f32}."""
    f, e, s = ct.c_double(), ct.c_double(), ct.c_double()
    check(load().qmc_probe_valu(ct.byref(f), ct.byref(e), ct.byref(s), _stream()))
    return {"fma": f.value, "exp": e.value, "sin": s.value}


def probe_mfma():
    """Measured matrix-core rates of the current GPU (flop/s): {"f32_32x32x2",
    "f32_16x16x4", "bf16_32x32x16"}."""
    a, b, c = ct.c_double(), ct.c_double(), ct.c_double()
    check(load().qmc_probe_mfma(ct.byref(a), ct.byref(b), ct.byref(c), _stream()))
    return {"f32_32x32x2": a.value, "f32_16x16x4": b.value, "bf16_32x32x16": c.value}


class timing:
    """Per-kernel event timing of the library (measurement only)."""

    @staticmethod
    def enable(on: bool = True) -> None:
        check(load().qmc_timing_enable(1 if on else 0))

    @staticmethod
    def reset() -> None:
        check(load().qmc_timing_reset())

    @staticmethod
    def read(name: str):
        ms, n = ct.c_double(), ct.c_int64()
        check(load().qmc_timing_read(name.encode(), ct.byref(ms), ct.byref(n)))
        return ms.value, n.value

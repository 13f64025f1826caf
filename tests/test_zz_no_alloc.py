"""qmc_estimate_static (the entry point that allocates nothing) against
qmc_estimate with a caller-owned workspace, through the C ABI.

Both run the same kernels in the same order, so the estimates must agree bit
for bit.  Two calls in a row share the library's static scratch array; the
second is smaller, so it runs over what the first left behind.
"""
from __future__ import annotations

import ctypes as ct

import numpy as np
import pytest

import paper_2305_11645_amd as q
from gpu_common import to_dev, torch_cuda
from paper_2305_11645_amd import inputs as I

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 64 << 20


def _static(pts, A, f, prec, Q, torch):
    L = q.load()
    st = ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    return L.qmc_estimate_static(pts.handle, ct.c_void_p(A.data_ptr()), A.shape[1], A.stride(0),
                                 ct.byref(f.c_struct()), prec, ct.c_void_p(Q.data_ptr()), st)


def _case(wl, prec, torch):
    """(static-scratch estimate, workspace estimate) of one workload."""
    pts = q.Points.from_workload(wl)
    A = to_dev(wl.A, torch)
    f = q.Integrand_.of(wl)
    assert pts.workspace_bytes(1, wl.t, f, prec) <= SCRATCH_BYTES
    Qs = torch.full((wl.R,), float("nan"), dtype=torch.float64, device="cuda")
    print(f"static scratch: {wl.name} m={wl.m} s={wl.s} t={wl.t} R={wl.R} prec={prec}", flush=True)
    assert _static(pts, A, f, prec, Qs, torch) == 0, q.load().qmc_last_error()
    Qw = q.estimate(pts, A, f, prec, workspace=pts.workspace(1, wl.t, f, prec))
    torch.cuda.synchronize()
    return Qs.cpu().numpy(), Qw.cpu().numpy()


def test_static_scratch_matches_workspace_two_calls():
    """Tree path (lattice with random shifts, cos-mean), then a smaller digital
    net with the non-separable call payoff, then a net that is not periodic
    (gathered tiles): each equal bit for bit to qmc_estimate."""
    torch = torch_cuda()
    cases = [
        (I.make_custom(kind=I.LATTICE, m=12, s=128, t=200, w=I.w_log2(128, 13), rand=I.RANDOM_SHIFT, R=4,
                       g=I.G_COS, A_scale=0.2, seed=21), I.FP32),
        (I.make_custom(kind=I.DIGITAL_NET, m=9, s=40, t=70, w=I.w_log2(40, 10), rand=I.DIGITAL_SHIFT, R=2,
                       map=I.MAP_INVNORM, g=I.G_EXP, c=0.2, h=I.H_CALL, K=1.0, A_scale=0.2, seed=22),
         I.SPLIT_BF16X3),
        (I.make_custom(kind=I.DIGITAL_NET, m=8, s=30, t=65, w=I.w_log2(30, 9), rand=I.DIGITAL_SHIFT, R=2,
                       map=I.MAP_CENTER, g=I.G_COS, A_scale=0.3, seed=23, net="upper"), I.FP32),
    ]
    for wl, prec in cases:
        Qs, Qw = _case(wl, prec, torch)
        assert np.array_equal(Qs, Qw), (wl.name, Qs, Qw)


def test_static_scratch_rejects_a_workload_beyond_its_size():
    """A workload whose workspace exceeds the 64 MiB array is refused with
    QMC_ENOMEM before anything is launched; Q stays untouched and the next
    call succeeds."""
    torch = torch_cuda()
    big = I.make_custom(kind=I.LATTICE, m=16, s=256, t=1024, w=I.w_log2(256, 12), rand=I.RANDOM_SHIFT,
                        R=16, g=I.G_COS, A_scale=0.05, seed=24)
    pts = q.Points.from_workload(big)
    f = q.Integrand_.of(big)
    assert pts.workspace_bytes(1, big.t, f, I.FP32) > SCRATCH_BYTES
    A = to_dev(big.A, torch)
    Q = torch.full((big.R,), 7.0, dtype=torch.float64, device="cuda")
    assert _static(pts, A, f, I.FP32, Q, torch) == 3
    assert b"static scratch" in q.load().qmc_last_error()
    torch.cuda.synchronize()
    assert torch.all(Q == 7.0)
    small = I.make_custom(kind=I.LATTICE, m=10, s=50, t=64, w=I.w_log2(50, 11), rand=I.RANDOM_SHIFT, R=2,
                          g=I.G_COS, A_scale=0.3, seed=25)
    Qs, Qw = _case(small, I.FP32, torch)
    assert np.array_equal(Qs, Qw)

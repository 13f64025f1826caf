"""GPU parity: the HIP library against the FP64 oracle, through the C ABI.

Small cases compare every output element with the oracle (several tiles and a
ragged column tail); the full-size workloads compare sampled outputs that
the oracle computes one by one, and the estimates against oracle values stored
by tests/golden/make_expected.py (a script that calls only the oracle).
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

import paper_2305_11645_amd as q
from gpu_common import (adjoint_chain, check_grad_elementwise, elementwise_bound, grad_bound_dense,
                        grad_bound_lattice, oracle_rows, oracle_tables, to_dev, torch_cuda)
from paper_2305_11645_amd import inputs as I

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
KINDS = [I.LATTICE, I.POLY_LATTICE, I.DIGITAL_NET]
RANDS = [I.NO_SHIFT, I.RANDOM_SHIFT, I.DIGITAL_SHIFT]
Q_TOL = 1e-6      # relative error target on every estimate


def small(kind, rand, mp=I.MAP_ID, m=9, s=40, t=100, R=2, seed=3, w=None, g=I.G_COS, h=I.H_ID,
          K=0.0, c=1.0, A_scale=0.3):
    if w is None:
        w = I.w_log2(s, m + 1)
    return I.make_custom(kind=kind, m=m, s=s, t=t, w=w, rand=rand, R=R, map=mp, g=g, h=h, K=K, c=c,
                         seed=seed, A_scale=A_scale)


# ------------------------------------------------------------------ tables

@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("rand", RANDS)
@pytest.mark.parametrize("mp", [I.MAP_ID, I.MAP_CENTER, I.MAP_TENT, I.MAP_INVNORM])
def test_tables_bit_exact(kind, rand, mp):
    """Distinct values (FP64) equal the oracle's bit for bit; the inverse-normal
    map (device normcdfinv vs AS241) agrees to a few ulp."""
    if mp == I.MAP_INVNORM and rand == I.NO_SHIFT:
        pytest.skip("the inverse-normal map requires a shift")
    torch = torch_cuda()
    wl = small(kind, rand, mp, m=10, s=24)
    pts = q.Points.from_workload(wl)
    for r in range(wl.R):
        ref = oracle_tables(wl, r)
        for j in range(wl.s):
            got = q.point_values(pts, r, j).cpu().numpy()
            if mp == I.MAP_INVNORM:
                np.testing.assert_allclose(got, ref[j], rtol=1e-14, atol=0)
            else:
                np.testing.assert_array_equal(got, ref[j])
    torch.cuda.synchronize()


@pytest.mark.parametrize("kind", KINDS)
def test_point_matrix_matches_unreduced(kind):
    """The FP32 point matrix equals the FP32 rounding of the oracle's unreduced X."""
    from oracle import oracle as O
    torch_cuda()
    wl = small(kind, I.RANDOM_SHIFT, m=9, s=30)
    pts = q.Points.from_workload(wl)
    for r in range(wl.R):
        X = q.point_matrix(pts, r).cpu().numpy()
        np.testing.assert_array_equal(X, O.point_matrix_unreduced(wl, r).astype(np.float32))


# ------------------------------------------------------------------ matvec

def _check_Y(wl, Y, r, prec):
    from oracle import oracle as O
    Yo = O.reduced_matvec(wl, r)
    X = O.point_matrix_unreduced(wl, r)
    mag = np.abs(X) @ np.abs(wl.A.astype(np.float64))
    err = np.abs(Y.astype(np.float64) - Yo)
    bound = elementwise_bound(wl, prec) * mag + 1e-30
    worst = float(np.max(err / bound))
    assert worst <= 1.0, f"element error {worst:.3g} x bound"
    return float(np.linalg.norm(Y - Yo) / np.linalg.norm(Yo))


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("rand", RANDS)
@pytest.mark.parametrize("prec", [I.FP32, I.SPLIT_BF16X3])
@pytest.mark.parametrize("form", ["direct", "packed"])
def test_matvec_elementwise(kind, rand, prec, form, monkeypatch):
    """Y = X A for every element within the FP32 (or split-bf16) error bound.
    t = 100 spans two 64-column tiles with a ragged tail; m = 9 gives several
    subtrees and several upper levels.  Both forms of the upper-level products:
    straight from the tables on 64 x 64 tiles, and from the packed K-step slabs
    on 128 x 256 tiles (a small grid takes the first unless forced)."""
    monkeypatch.setenv("QMC_LEVELS_FORM", form)
    torch = torch_cuda()
    mp = I.MAP_INVNORM if rand == I.DIGITAL_SHIFT else I.MAP_ID
    wl = small(kind, rand, mp)
    pts = q.Points.from_workload(wl)
    A = to_dev(wl.A, torch)
    for r in range(wl.R):
        Y = q.reduced_matvec(pts, A, r=r, prec=prec).cpu().numpy()
        rel = _check_Y(wl, Y, r, prec)
        assert rel < (1e-6 if prec == I.FP32 else 2e-4)


@pytest.mark.parametrize("split_case", ["deep", "flat", "tiny", "wide"])
def test_matvec_shapes(split_case):
    """Level structures that exercise the planner: many lower levels, w = 0
    everywhere (all coordinates in level 0), m below the split cap, and
    coordinates with w_j >= m (constant columns)."""
    torch = torch_cuda()
    if split_case == "deep":
        wl = small(I.LATTICE, I.RANDOM_SHIFT, m=12, s=70, t=64, w=I.w_log2(70, 12))
    elif split_case == "flat":
        wl = small(I.LATTICE, I.RANDOM_SHIFT, m=8, s=20, t=65, w=[0] * 20)
    elif split_case == "tiny":
        wl = small(I.DIGITAL_NET, I.DIGITAL_SHIFT, m=3, s=5, t=3, w=[0, 1, 1, 2, 5])
    else:
        wl = small(I.POLY_LATTICE, I.NO_SHIFT, m=7, s=150, t=130, w=I.w_log2(150, 9))
    pts = q.Points.from_workload(wl)
    A = to_dev(wl.A, torch)
    Y = q.reduced_matvec(pts, A, r=0).cpu().numpy()
    _check_Y(wl, Y, 0, I.FP32)


def test_split_level_zero():
    """More than 64 coordinates in level 0 leave no lower levels (split level
    0: every level, level 0 included, is an upper-level product and a subtree
    is one point): Y element by element, Q, and dQ/dA element by element."""
    torch = torch_cuda()
    wl = small(I.LATTICE, I.RANDOM_SHIFT, m=6, s=70, t=65, w=[0] * 66 + [1, 2, 3, 7], R=2)
    pts = q.Points.from_workload(wl)
    assert pts.split_level == 0 and pts.grad_split_level == 0
    A = to_dev(wl.A, torch)
    for r in range(wl.R):
        Y = q.reduced_matvec(pts, A, r=r).cpu().numpy()
        _check_Y(wl, Y, r, I.FP32)
    _check_grad(wl, pts)


def test_matvec_identity_is_point_matrix():
    """A = I_s gives Y = X exactly (FP32 path)."""
    torch = torch_cuda()
    wl = small(I.LATTICE, I.RANDOM_SHIFT, m=10, s=64, t=64)
    pts = q.Points.from_workload(wl)
    A = torch.eye(64, dtype=torch.float32, device="cuda")
    Y = q.reduced_matvec(pts, A, r=1)
    X = q.point_matrix(pts, 1)
    assert torch.equal(Y, X)


def test_matvec_strided_A_and_Y():
    """Leading dimensions larger than t on both A and Y."""
    torch = torch_cuda()
    wl = small(I.LATTICE, I.RANDOM_SHIFT, m=9, s=40, t=70)
    pts = q.Points.from_workload(wl)
    Abig = torch.zeros((40, 96), dtype=torch.float32, device="cuda")
    Abig[:, :70] = to_dev(wl.A, torch)
    Ybig = torch.full((wl.N, 128), 7.0, dtype=torch.float32, device="cuda")
    q.reduced_matvec(pts, Abig[:, :70], r=0, Y=Ybig[:, :70])
    Y = Ybig.cpu().numpy()
    assert np.all(Y[:, 70:] == 7.0)
    _check_Y(wl, Y[:, :70], 0, I.FP32)


# ------------------------------------------------------------------ estimate

@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("g,h,c", [(I.G_COS, I.H_ID, 1.0), (I.G_EXP, I.H_ID, -0.7),
                                   (I.G_EXP, I.H_CALL, 0.2), (I.G_ID, I.H_ID, 1.0)])
@pytest.mark.parametrize("form", ["direct", "packed"])
def test_estimate_small(kind, g, h, c, form, monkeypatch):
    """Q[r] against the oracle to 1e-6 relative for every integrand family,
    with either form of the upper-level products."""
    from oracle import oracle as O
    monkeypatch.setenv("QMC_LEVELS_FORM", form)
    torch = torch_cuda()
    rand = I.DIGITAL_SHIFT if kind == I.DIGITAL_NET else I.RANDOM_SHIFT
    K = 1.0 if h == I.H_CALL else 0.0
    wl = small(kind, rand, g=g, h=h, c=c, K=K, R=3)
    pts = q.Points.from_workload(wl)
    A = to_dev(wl.A, torch)
    Q = q.estimate(pts, A, q.Integrand_.of(wl)).cpu().numpy()
    Qo, _ = O.estimate(wl)
    scale = np.maximum(np.abs(Qo), 1e-3)
    assert np.all(np.abs(Q - Qo) <= Q_TOL * scale), (Q, Qo)


def test_estimate_linear_closed_form():
    """g(y) = y, h = id: the exact closed form t^-1 sum_i sum_j a_ji mu_j holds
    at any N; the GPU estimate matches it within FP32 accumulation error."""
    torch = torch_cuda()
    wl = small(I.LATTICE, I.RANDOM_SHIFT, m=14, s=200, t=192, g=I.G_ID, R=4)
    pts = q.Points.from_workload(wl)
    Q = q.estimate(pts, to_dev(wl.A, torch), q.Integrand_.of(wl)).cpu().numpy()
    A = wl.A.astype(np.float64)
    for r in range(wl.R):
        mu = []
        for j in range(wl.s):
            n = 2 ** (wl.m - min(int(wl.w[j]), wl.m))
            mu.append((n - 1 + 2 * ((n * float(wl.shift[r, j])) % 1.0)) / (2 * n))
        ref = float(np.mean(np.array(mu) @ A))
        assert abs(Q[r] - ref) <= 1e-6 * max(abs(ref), float(np.mean(np.abs(A).sum(0))))


def test_estimate_deterministic():
    """Two runs are bitwise equal (fixed-order reductions, no float atomics)."""
    torch = torch_cuda()
    wl = I.make_config(2, m=13, R=4)
    pts = q.Points.from_workload(wl)
    A = to_dev(wl.A, torch)
    f = q.Integrand_.of(wl)
    Q1 = q.estimate(pts, A, f)
    Q2 = q.estimate(pts, A, f)
    assert torch.equal(Q1, Q2)


def test_estimate_library_workspace():
    """workspace = NULL: the library allocates a stream-ordered workspace itself."""
    import ctypes as ct
    torch = torch_cuda()
    wl = small(I.LATTICE, I.RANDOM_SHIFT, R=2)
    pts = q.Points.from_workload(wl)
    A = to_dev(wl.A, torch)
    f = q.Integrand_.of(wl)
    Q = torch.empty(2, dtype=torch.float64, device="cuda")
    L = q.load()
    st = ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    q._lib.check(L.qmc_estimate(pts.handle, ct.c_void_p(A.data_ptr()), wl.t, wl.t, ct.byref(f.c_struct()),
                                0, ct.c_void_p(Q.data_ptr()), None, 0, st))
    assert torch.equal(Q, q.estimate(pts, A, f))


def test_workspace_allocation_failure_leaves_the_point_set_usable(monkeypatch):
    """QMC_FAULT_INJECT=alloc makes the library's own workspace allocation fail:
    the call returns QMC_ENOMEM before launching anything (Q untouched), and
    the next call on the same point set succeeds with the usual result."""
    import ctypes as ct
    torch = torch_cuda()
    wl = small(I.LATTICE, I.RANDOM_SHIFT, R=2)
    pts = q.Points.from_workload(wl)
    A = to_dev(wl.A, torch)
    f = q.Integrand_.of(wl)
    L = q.load()
    st = ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    Q = torch.full((2,), 5.0, dtype=torch.float64, device="cuda")
    monkeypatch.setenv("QMC_FAULT_INJECT", "alloc")
    rc = L.qmc_estimate(pts.handle, ct.c_void_p(A.data_ptr()), wl.t, wl.t, ct.byref(f.c_struct()), 0,
                        ct.c_void_p(Q.data_ptr()), None, 0, st)
    assert rc == 3 and b"fault injection" in L.qmc_last_error()
    torch.cuda.synchronize()
    assert torch.all(Q == 5.0)
    monkeypatch.delenv("QMC_FAULT_INJECT")
    q._lib.check(L.qmc_estimate(pts.handle, ct.c_void_p(A.data_ptr()), wl.t, wl.t, ct.byref(f.c_struct()), 0,
                                ct.c_void_p(Q.data_ptr()), None, 0, st))
    assert torch.equal(Q, q.estimate(pts, A, f))


# ------------------------------------------------------------------ gradient

@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("g,h,c", [(I.G_COS, I.H_ID, 1.0), (I.G_EXP, I.H_CALL, 0.2)])
@pytest.mark.parametrize("form", ["direct", "packed"])
def test_gradient_small(kind, g, h, c, form, monkeypatch):
    """dQ/dA against the oracle gradient: every element within its FP32 error
    bound (c u |X|^T|G| plus the propagated error of y, see gpu_common), and
    relative Frobenius <= 1e-6 per shift.  Both forms of the level products
    (the 64 x 64 ones, and the packed forward and tiled adjoint ones that large
    problems take)."""
    monkeypatch.setenv("QMC_LEVELS_FORM", form)
    wl = small(kind, I.DIGITAL_SHIFT if kind == I.DIGITAL_NET else I.RANDOM_SHIFT, m=10, s=50, t=80, g=g, h=h,
               c=c, K=1.0 if h == I.H_CALL else 0.0, R=2)
    pts = q.Points.from_workload(wl)
    assert pts.split_level >= 0
    _check_grad(wl, pts)


@pytest.mark.parametrize("form", ["direct", "packed"])
def test_gradient_all_adjoint_tile_shapes(form, monkeypatch):
    """Upper levels with 32, 64, 128 and 45 coordinates (w_j = floor(log2(j+1)),
    s = 300) take all three tile shapes of the tiled adjoint products; every
    element of dA within its FP32 bound, in both forms."""
    monkeypatch.setenv("QMC_LEVELS_FORM", form)
    wl = small(I.LATTICE, I.RANDOM_SHIFT, m=12, s=300, t=100, g=I.G_COS, h=I.H_ID, c=1.0, R=1, A_scale=0.1,
               w=I.w_log2(300, 12))
    pts = q.Points.from_workload(wl)
    assert pts.grad_split_level == 5
    _check_grad(wl, pts)


@pytest.mark.parametrize("g,h,c", [(I.G_COS, I.H_ID, 1.0), (I.G_EXP, I.H_CALL, 0.2)])
def test_gradient_split_bf16_tree(g, h, c):
    """The tree-path adjoint in split BF16 (forward and adjoint upper-level
    products as three BF16 products): every element within the split bound,
    Frobenius within 1e-5.  w_j = floor(1.5 log2(j+1)) puts the nonempty
    levels 5 to 9 above the gradient's split (5)."""
    wl = small(I.LATTICE, I.RANDOM_SHIFT, m=12, s=90, t=100, g=g, h=h, c=c, K=1.0 if h == I.H_CALL else 0.0,
               R=2, A_scale=0.15, w=I.w_log2_pow(90, 12, 3, 2))
    pts = q.Points.from_workload(wl)
    assert pts.split_level == 6 and pts.grad_split_level == 5
    _check_grad(wl, pts, prec=I.SPLIT_BF16X3, tol=1e-5)


def test_autograd_matches_grad():
    """QMCEstimate.backward returns sum_r gQ_r dQ_r/dA."""
    torch = torch_cuda()
    wl = small(I.LATTICE, I.RANDOM_SHIFT, R=3)
    pts = q.Points.from_workload(wl)
    A = to_dev(wl.A, torch).requires_grad_(True)
    f = q.Integrand_.of(wl)
    Q = q.QMCEstimate.apply(A, pts, f, I.FP32)
    wts = torch.tensor([0.5, -1.0, 2.0], dtype=torch.float64, device="cuda")
    (Q * wts).sum().backward()
    _, dA = q.estimate_grad(pts, A.detach(), f)
    ref = (wts.view(-1, 1, 1) * dA.double()).sum(0).float()
    assert torch.allclose(A.grad, ref, rtol=1e-6, atol=1e-12)


# ------------------------------------------------------------------ reduced Monte Carlo (Section 4)

def iid_small(mp=I.MAP_ID, m=9, s=40, t=100, R=3, seed=4, w=None, g=I.G_COS, h=I.H_ID, K=0.0, c=1.0,
              A_scale=0.3):
    if w is None:
        w = I.w_log2(s, m + 1)
    return I.make_custom(kind=I.IID, m=m, s=s, t=t, w=w, rand=I.NO_SHIFT, R=R, map=mp, g=g, h=h, K=K,
                         c=c, seed=seed, A_scale=A_scale)


@pytest.mark.parametrize("mp", [I.MAP_ID, I.MAP_CENTER, I.MAP_TENT, I.MAP_INVNORM])
def test_iid_tables_bit_exact(mp):
    """eq. randpts: the device tables are the caller's samples after the map,
    bit for bit (the inverse-normal map to 1e-14)."""
    torch = torch_cuda()
    wl = iid_small(mp, m=10, s=24)
    pts = q.Points.from_workload(wl)
    for r in range(wl.R):
        ref = oracle_tables(wl, r)
        for j in range(wl.s):
            got = q.point_values(pts, r, j).cpu().numpy()
            if mp == I.MAP_INVNORM:
                np.testing.assert_allclose(got, ref[j], rtol=1e-14, atol=0)
            else:
                np.testing.assert_array_equal(got, ref[j])
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec", [I.FP32, I.SPLIT_BF16X3])
@pytest.mark.parametrize("m,mp", [(9, I.MAP_INVNORM), (12, I.MAP_INVNORM), (12, I.MAP_CENTER)])
def test_iid_matvec_elementwise(prec, m, mp):
    """Reduced Monte Carlo products Y = X A, every element within the bound.
    m = 12 puts all 40 coordinates below the split (no upper level) over 64
    subtree roots."""
    torch = torch_cuda()
    wl = iid_small(mp, m=m, A_scale=0.1, w=I.w_log2(40, m + 1))
    pts = q.Points.from_workload(wl)
    A = to_dev(wl.A, torch)
    for r in range(wl.R):
        Y = q.reduced_matvec(pts, A, r=r, prec=prec).cpu().numpy()
        rel = _check_Y(wl, Y, r, prec)
        assert rel < (1e-6 if prec == I.FP32 else 2e-4)


@pytest.mark.parametrize("g,h,c,mp", [(I.G_COS, I.H_ID, 1.0, I.MAP_ID), (I.G_EXP, I.H_ID, -0.7, I.MAP_CENTER),
                                      (I.G_EXP, I.H_CALL, 0.2, I.MAP_INVNORM)])
def test_iid_estimate_and_gradient(g, h, c, mp):
    """Estimates of every replicate within 1e-6 and their gradients element by
    element within the FP32 bound and within 1e-6 (Frobenius) of the oracle."""
    from oracle import oracle as O
    torch = torch_cuda()
    K = 1.0 if h == I.H_CALL else 0.0
    wl = iid_small(mp, m=10, s=50, t=80, g=g, h=h, c=c, K=K)
    pts = q.Points.from_workload(wl)
    A = to_dev(wl.A, torch)
    f = q.Integrand_.of(wl)
    Q = q.estimate(pts, A, f).cpu().numpy()
    Qo, _ = O.estimate(wl)
    assert np.all(np.abs(Q - Qo) <= Q_TOL * np.maximum(np.abs(Qo), 1e-3)), (Q, Qo)
    _check_grad(wl, pts)


# ------------------------------------------------------------------ Algorithm 4 (nets not periodic after reduction)

def upper_small(rand=I.DIGITAL_SHIFT, mp=I.MAP_CENTER, m=9, s=40, t=100, R=2, seed=6, w=None, g=I.G_COS,
                h=I.H_ID, K=0.0, c=1.0, A_scale=0.3):
    if w is None:
        w = I.w_log2(s, m + 1)
    return I.make_custom(kind=I.DIGITAL_NET, m=m, s=s, t=t, w=w, rand=rand, R=R, map=mp, g=g, h=h, K=K,
                         c=c, seed=seed, A_scale=A_scale, net="upper")


def test_alg4_is_planned_for_upper_triangular_nets():
    torch_cuda()
    assert q.Points.from_workload(upper_small()).split_level == -1
    assert q.Points.from_workload(small(I.DIGITAL_NET, I.DIGITAL_SHIFT)).split_level >= 0


@pytest.mark.parametrize("rand", RANDS)
@pytest.mark.parametrize("mp", [I.MAP_ID, I.MAP_CENTER, I.MAP_TENT, I.MAP_INVNORM])
def test_alg4_tables_bit_exact(rand, mp):
    """Section 3: the n_j values c / n_j of each coordinate (indexed by the
    reduced output digits), shifted and mapped, equal the oracle's bit for bit
    (the inverse-normal map to 1e-14)."""
    from oracle import oracle as O
    if mp == I.MAP_INVNORM and rand == I.NO_SHIFT:
        pytest.skip("the inverse-normal map requires a shift")
    torch_cuda()
    wl = upper_small(rand, mp, m=10, s=24, R=2 if rand != I.NO_SHIFT else 1)
    pts = q.Points.from_workload(wl)
    for r in range(wl.R):
        for j in range(wl.s):
            got = q.point_values(pts, r, j).cpu().numpy()
            ref = O.output_values(wl, r, j)
            if mp == I.MAP_INVNORM:
                np.testing.assert_allclose(got, ref, rtol=1e-14, atol=0)
            else:
                np.testing.assert_array_equal(got, ref)


def test_alg4_point_matrix_matches_unreduced():
    """Every point from all its digits: the FP32 point matrix equals the FP32
    rounding of the oracle's unreduced net."""
    from oracle import oracle as O
    torch_cuda()
    wl = upper_small(m=9, s=30)
    pts = q.Points.from_workload(wl)
    for r in range(wl.R):
        np.testing.assert_array_equal(q.point_matrix(pts, r).cpu().numpy(),
                                      O.point_matrix_unreduced(wl, r).astype(np.float32))


@pytest.mark.parametrize("rand", RANDS)
@pytest.mark.parametrize("prec", [I.FP32, I.SPLIT_BF16X3])
def test_alg4_matvec_elementwise(rand, prec):
    """Algorithm 4 products Y = X A, every element within the FP32 (split-bf16)
    bound: several 64-point tiles, two column tiles with a ragged tail, and a
    coordinate count that is not a multiple of the 32-coordinate step."""
    torch = torch_cuda()
    mp = I.MAP_INVNORM if rand == I.DIGITAL_SHIFT else I.MAP_ID
    wl = upper_small(rand, mp, s=45, R=2 if rand != I.NO_SHIFT else 1)
    pts = q.Points.from_workload(wl)
    A = to_dev(wl.A, torch)
    for r in range(wl.R):
        Y = q.reduced_matvec(pts, A, r=r, prec=prec).cpu().numpy()
        rel = _check_Y(wl, Y, r, prec)
        assert rel < (1e-6 if prec == I.FP32 else 2e-4)


@pytest.mark.parametrize("m,s,t", [(4, 7, 3), (6, 33, 64), (11, 70, 130)])
def test_alg4_matvec_shapes(m, s, t):
    """Fewer points than one tile (m = 4), exactly one tile (m = 6), many tiles."""
    torch = torch_cuda()
    wl = upper_small(I.DIGITAL_SHIFT, I.MAP_CENTER, m=m, s=s, t=t, R=1)
    pts = q.Points.from_workload(wl)
    Y = q.reduced_matvec(pts, to_dev(wl.A, torch), r=0).cpu().numpy()
    _check_Y(wl, Y, 0, I.FP32)


@pytest.mark.parametrize("g,h,c,mp", [(I.G_COS, I.H_ID, 1.0, I.MAP_ID), (I.G_EXP, I.H_ID, -0.7, I.MAP_CENTER),
                                      (I.G_EXP, I.H_CALL, 0.2, I.MAP_INVNORM), (I.G_ID, I.H_ID, 1.0, I.MAP_TENT)])
def test_alg4_estimate(g, h, c, mp):
    """Estimates over Algorithm 4 for every integrand family within 1e-6."""
    from oracle import oracle as O
    torch = torch_cuda()
    K = 1.0 if h == I.H_CALL else 0.0
    wl = upper_small(I.DIGITAL_SHIFT, mp, m=10, s=50, t=80, g=g, h=h, c=c, K=K)
    pts = q.Points.from_workload(wl)
    Q = q.estimate(pts, to_dev(wl.A, torch), q.Integrand_.of(wl)).cpu().numpy()
    Qo, _ = O.estimate(wl)
    assert np.all(np.abs(Q - Qo) <= Q_TOL * np.maximum(np.abs(Qo), 1e-3)), (Q, Qo)


def _check_grad(wl, pts, prec=I.FP32, tol=1e-6):
    """Q within the estimate tolerance; dA per randomisation element by element
    within its error bound (grad_bound_dense with the path's FP32 chain
    length) and within tol (relative Frobenius) of the oracle's gradient."""
    from oracle import oracle as O
    torch = torch_cuda()
    A = to_dev(wl.A, torch)
    Q, dA = q.estimate_grad(pts, A, q.Integrand_.of(wl), prec=prec)
    Qo, dAo = O.estimate_grad(wl)
    Q, dA = Q.cpu().numpy(), dA.cpu().numpy().astype(np.float64)
    # split BF16: the estimate carries the split products' error (about 1e-7 of
    # the integrand's scale), so small estimates get 1e-5 relative
    qtol = Q_TOL if prec == I.FP32 else 1e-5
    assert np.all(np.abs(Q - Qo) <= qtol * np.maximum(np.abs(Qo), 1e-3)), (Q, Qo)
    D = adjoint_chain(wl, pts)
    for r in range(wl.R):
        rel = np.linalg.norm(dA[r] - dAo[r]) / np.linalg.norm(dAo[r])
        assert rel <= tol, (r, rel)
        check_grad_elementwise(dA[r], dAo[r], grad_bound_dense(wl, r, prec, D), f"r={r}")
    return dA


@pytest.mark.parametrize("g,h,c,mp", [(I.G_COS, I.H_ID, 1.0, I.MAP_CENTER), (I.G_EXP, I.H_CALL, 0.2, I.MAP_INVNORM),
                                      (I.G_ID, I.H_ID, 1.0, I.MAP_TENT)])
def test_alg4_gradient(g, h, c, mp):
    """dQ/dA of a net that is not periodic (Algorithm 4 transposed, X^T G on
    the matrix cores) against the oracle: several point tiles and chunks,
    coordinates past one 64-coordinate tile, two column tiles with a ragged
    tail."""
    K = 1.0 if h == I.H_CALL else 0.0
    wl = upper_small(I.DIGITAL_SHIFT, mp, m=11, s=70, t=300, g=g, h=h, c=c, K=K)
    _check_grad(wl, q.Points.from_workload(wl))


@pytest.mark.parametrize("m,s,t", [(4, 7, 3), (6, 33, 64), (9, 64, 257)])
def test_alg4_gradient_shapes(m, s, t):
    """Fewer points than one tile, exactly one tile, and whole coordinate and
    column tiles plus one column."""
    wl = upper_small(I.DIGITAL_SHIFT, I.MAP_CENTER, m=m, s=s, t=t, g=I.G_COS)
    _check_grad(wl, q.Points.from_workload(wl))


def test_alg4_gradient_split_bf16():
    """The adjoint products in split BF16 (three products) stay within 1e-5."""
    wl = upper_small(I.DIGITAL_SHIFT, I.MAP_CENTER, m=10, s=50, t=100, g=I.G_COS)
    _check_grad(wl, q.Points.from_workload(wl), prec=I.SPLIT_BF16X3, tol=1e-5)


def test_alg4_gradient_is_deterministic():
    """The chunk partials are added in fixed order: two calls agree bit for bit."""
    torch = torch_cuda()
    wl = upper_small(m=10, s=50, t=100)
    pts = q.Points.from_workload(wl)
    A = to_dev(wl.A, torch)
    f = q.Integrand_.of(wl)
    Q1, d1 = q.estimate_grad(pts, A, f)
    Q2, d2 = q.estimate_grad(pts, A, f)
    assert torch.equal(Q1, Q2) and torch.equal(d1, d2)


# ------------------------------------------------------------------ prime base b > 2 (Section 1.3, Section 4)

BASE_B = [(3, 6), (5, 4), (7, 3)]   # N = 729, 625, 343


def lat_b(b, m, rand=I.RANDOM_SHIFT, mp=I.MAP_ID, s=40, t=100, R=2, seed=8, kind=I.LATTICE, g=I.G_COS,
          h=I.H_ID, K=0.0, c=1.0, A_scale=0.3):
    R = R if rand != I.NO_SHIFT or kind == I.IID else 1
    return I.make_custom(kind=kind, m=m, s=s, t=t, w=I.w_logb(s, m + 1, b), rand=rand, R=R, map=mp, g=g,
                         h=h, K=K, c=c, seed=seed, A_scale=A_scale, b=b)


def test_base_b_is_planned_for_gathered_tiles():
    """A base b > 2 has N = b^m points and takes the gathered-tile path.  With
    b = 3, m = 6, s = 40 (w_j = floor(log_3(j+1))) the split level L' = 2 is
    the cheapest: in whole 32-coordinate steps plus 16 per point for the root
    rows, 729 * 32 + 81 * 32 + 16 * 729 = 37584 against 729 * 32 + 243 * 64 +
    16 * 729 = 50544 at L' = 1 and 729 * 64 = 46656 in one pass (L' = 3 would
    leave 27 < 64 residues).  N = 27 has no split."""
    torch_cuda()
    wl = lat_b(3, 6)
    pts = q.Points.from_workload(wl)
    nb = wl.m - np.minimum(wl.w, wl.m)
    assert pts.N == 3 ** 6 and pts.split_level == 2
    assert pts.distinct_values == int(np.sum(3 ** nb))
    assert q.Points.from_workload(lat_b(3, 3, s=7)).split_level == -1


@pytest.mark.parametrize("b,m", BASE_B)
@pytest.mark.parametrize("rand,mp", [(I.NO_SHIFT, I.MAP_ID), (I.RANDOM_SHIFT, I.MAP_CENTER),
                                     (I.RANDOM_SHIFT, I.MAP_TENT), (I.RANDOM_SHIFT, I.MAP_INVNORM)])
def test_base_b_tables_bit_exact(b, m, rand, mp):
    """Section 1.3 in base b: the n_j = b^e values c / n_j of each coordinate
    (one correctly rounded FP64 division), shifted and mapped, equal the
    oracle's bit for bit (the inverse-normal map to 1e-14)."""
    from oracle import oracle as O
    torch_cuda()
    wl = lat_b(b, m, rand, mp, s=24)
    pts = q.Points.from_workload(wl)
    for r in range(wl.R):
        for j in range(wl.s):
            got = q.point_values(pts, r, j).cpu().numpy()
            ref = O.point_values(wl, r, j)
            if mp == I.MAP_INVNORM:
                np.testing.assert_allclose(got, ref, rtol=1e-14, atol=0)
            else:
                np.testing.assert_array_equal(got, ref)


def test_base_b_point_matrix_matches_unreduced():
    """The FP32 point matrix of a base-5 lattice equals the FP32 rounding of
    the oracle's unreduced lattice {k b^{w_j} z'_j / b^m}."""
    from oracle import oracle as O
    torch_cuda()
    wl = lat_b(5, 4, s=30)
    pts = q.Points.from_workload(wl)
    for r in range(wl.R):
        np.testing.assert_array_equal(q.point_matrix(pts, r).cpu().numpy(),
                                      O.point_matrix_unreduced(wl, r).astype(np.float32))


@pytest.mark.parametrize("b,m", BASE_B)
@pytest.mark.parametrize("prec", [I.FP32, I.SPLIT_BF16X3])
def test_base_b_matvec_elementwise(b, m, prec):
    """Base-b products Y = X A, every element within the FP32 (split-bf16)
    bound: N not a multiple of the 64-point tile, a ragged column tail and a
    coordinate count that is not a multiple of the 32-coordinate step."""
    torch = torch_cuda()
    wl = lat_b(b, m, s=45)
    pts = q.Points.from_workload(wl)
    A = to_dev(wl.A, torch)
    for r in range(wl.R):
        Y = q.reduced_matvec(pts, A, r=r, prec=prec).cpu().numpy()
        rel = _check_Y(wl, Y, r, prec)
        assert rel < (1e-6 if prec == I.FP32 else 2e-4)


@pytest.mark.parametrize("b,m,s,t", [(3, 3, 7, 3), (3, 8, 70, 300), (11, 2, 20, 17)])
def test_base_b_matvec_shapes(b, m, s, t):
    """27 points (under one tile), 6561 points (102 tiles and a ragged one) with
    two column tiles, and 121 points in base 11."""
    torch = torch_cuda()
    wl = lat_b(b, m, I.RANDOM_SHIFT, I.MAP_CENTER, s=s, t=t, R=1)
    pts = q.Points.from_workload(wl)
    Y = q.reduced_matvec(pts, to_dev(wl.A, torch), r=0).cpu().numpy()
    _check_Y(wl, Y, 0, I.FP32)


@pytest.mark.parametrize("g,h,c,mp", [(I.G_COS, I.H_ID, 1.0, I.MAP_ID), (I.G_EXP, I.H_ID, -0.7, I.MAP_CENTER),
                                      (I.G_EXP, I.H_CALL, 0.2, I.MAP_INVNORM), (I.G_ID, I.H_ID, 1.0, I.MAP_TENT)])
def test_base_b_estimate(g, h, c, mp):
    """Estimates over a shifted base-3 lattice for every integrand family within 1e-6."""
    from oracle import oracle as O
    torch = torch_cuda()
    K = 1.0 if h == I.H_CALL else 0.0
    wl = lat_b(3, 7, I.RANDOM_SHIFT, mp, s=50, t=80, g=g, h=h, c=c, K=K)
    pts = q.Points.from_workload(wl)
    Q = q.estimate(pts, to_dev(wl.A, torch), q.Integrand_.of(wl)).cpu().numpy()
    Qo, _ = O.estimate(wl)
    assert np.all(np.abs(Q - Qo) <= Q_TOL * np.maximum(np.abs(Qo), 1e-3)), (Q, Qo)


@pytest.mark.parametrize("mp", [I.MAP_ID, I.MAP_INVNORM])
def test_base_b_reduced_monte_carlo(mp):
    """Section 4 in base 3: the samples of coordinate j are read at n mod N_j;
    tables bit for bit (the inverse-normal map to 1e-14), products element-wise
    and the estimate within 1e-6."""
    from oracle import oracle as O
    torch = torch_cuda()
    wl = lat_b(3, 6, I.NO_SHIFT, mp, s=40, t=100, R=3, kind=I.IID, g=I.G_EXP, c=0.3)
    pts = q.Points.from_workload(wl)
    for j in range(wl.s):
        got, ref = q.point_values(pts, 1, j).cpu().numpy(), O.point_values(wl, 1, j)
        if mp == I.MAP_INVNORM:
            np.testing.assert_allclose(got, ref, rtol=1e-14, atol=0)
        else:
            np.testing.assert_array_equal(got, ref)
    A = to_dev(wl.A, torch)
    _check_Y(wl, q.reduced_matvec(pts, A, r=2).cpu().numpy(), 2, I.FP32)
    Q = q.estimate(pts, A, q.Integrand_.of(wl)).cpu().numpy()
    Qo, _ = O.estimate(wl)
    assert np.all(np.abs(Q - Qo) <= Q_TOL * np.abs(Qo)), (Q, Qo)


@pytest.mark.parametrize("b,m", [(3, 6), (5, 4)])
@pytest.mark.parametrize("kind", [I.POLY_LATTICE, I.DIGITAL_NET])
@pytest.mark.parametrize("rand,mp", [(I.NO_SHIFT, I.MAP_ID), (I.RANDOM_SHIFT, I.MAP_TENT),
                                     (I.DIGITAL_SHIFT, I.MAP_ID), (I.DIGITAL_SHIFT, I.MAP_INVNORM)])
def test_base_b_nets_and_polys_tables_bit_exact(b, m, kind, rand, mp):
    """Polynomial lattices and nets over F_b (Sections 1.1, 3), unshifted,
    randomly shifted or digitally shifted mod b: the n_j values equal the
    oracle's bit for bit (the inverse-normal map to 1e-14)."""
    from oracle import oracle as O
    torch_cuda()
    wl = lat_b(b, m, rand, mp, s=20, kind=kind)
    pts = q.Points.from_workload(wl)
    for r in range(wl.R):
        for j in range(wl.s):
            got, ref = q.point_values(pts, r, j).cpu().numpy(), O.point_values(wl, r, j)
            if mp == I.MAP_INVNORM:
                np.testing.assert_allclose(got, ref, rtol=1e-14, atol=0)
            else:
                np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("kind", [I.POLY_LATTICE, I.DIGITAL_NET])
@pytest.mark.parametrize("prec", [I.FP32, I.SPLIT_BF16X3])
def test_base_b_nets_and_polys_matvec_and_estimate(kind, prec):
    """Digitally shifted base-3 polynomial lattice and net through Phi^-1: every
    product element within the bound (point matrix equal to the FP32 rounding
    of the unreduced points), and a call-type estimate within 1e-6."""
    from oracle import oracle as O
    torch = torch_cuda()
    wl = lat_b(3, 7, I.DIGITAL_SHIFT, I.MAP_INVNORM, s=45, t=100, kind=kind, g=I.G_EXP, h=I.H_CALL, c=0.2,
               K=1.0)
    pts = q.Points.from_workload(wl)
    np.testing.assert_array_equal(q.point_matrix(pts, 1).cpu().numpy(),
                                  O.point_matrix_unreduced(wl, 1).astype(np.float32))
    A = to_dev(wl.A, torch)
    for r in range(wl.R):
        Y = q.reduced_matvec(pts, A, r=r, prec=prec).cpu().numpy()
        _check_Y(wl, Y, r, prec)
    if prec == I.FP32:
        Q = q.estimate(pts, A, q.Integrand_.of(wl)).cpu().numpy()
        Qo, _ = O.estimate(wl)
        assert np.all(np.abs(Q - Qo) <= Q_TOL * np.maximum(np.abs(Qo), 1e-3)), (Q, Qo)


@pytest.mark.parametrize("b,m", BASE_B)
@pytest.mark.parametrize("g,h,c", [(I.G_COS, I.H_ID, 1.0), (I.G_EXP, I.H_CALL, 0.2)])
def test_base_b_gradient(b, m, g, h, c):
    """dQ/dA of base-b lattices against the oracle's residue-class fold: with
    the planner's split (b = 3: level 2, the upper coordinates contracted over
    G summed into the b^{m-2} residues) and in one pass; t = 301 folds one
    column per thread, t = 300 four."""
    K = 1.0 if h == I.H_CALL else 0.0
    t = 301 if g == I.G_COS else 300
    wl = lat_b(b, m, I.RANDOM_SHIFT, I.MAP_CENTER, s=70, t=t, g=g, h=h, c=c, K=K)
    pts = q.Points.from_workload(wl)
    if b == 3:
        assert pts.split_level == 2
    _check_grad(wl, pts)


@pytest.mark.parametrize("which", ["net", "base3"])
def test_gather_path_autograd(which):
    """QMCEstimate.backward on the gathered-tile paths (a net that is not
    periodic, a base-3 lattice with the split) returns sum_r gQ_r dQ_r/dA."""
    torch = torch_cuda()
    wl = upper_small(m=10, s=50, t=100) if which == "net" else lat_b(3, 6, s=70, t=100)
    pts = q.Points.from_workload(wl)
    A = to_dev(wl.A, torch).requires_grad_(True)
    f = q.Integrand_.of(wl)
    Q = q.QMCEstimate.apply(A, pts, f, I.FP32)
    wts = torch.tensor([0.75, -1.25], dtype=torch.float64, device="cuda")
    (Q * wts).sum().backward()
    _, dA = q.estimate_grad(pts, A.detach(), f)
    ref = (wts.view(-1, 1, 1) * dA.double()).sum(0).float()
    assert torch.allclose(A.grad, ref, rtol=1e-6, atol=1e-12)


@pytest.mark.parametrize("kind", [I.POLY_LATTICE, I.DIGITAL_NET, I.IID])
def test_base_b_gradient_kinds(kind):
    """Polynomial lattices and nets over F_b (digital shift) and reduced Monte
    Carlo in base 3: the gradient against the oracle."""
    rand = I.NO_SHIFT if kind == I.IID else I.DIGITAL_SHIFT
    wl = lat_b(3, 7, rand, I.MAP_ID if kind == I.IID else I.MAP_INVNORM, s=45, t=100, kind=kind, g=I.G_EXP,
               h=I.H_ID, c=0.2)
    _check_grad(wl, q.Points.from_workload(wl))


# ------------------------------------------------------------------ Algorithm 4 over F_b (b > 2)

UPPER_B = [(3, 6), (5, 4), (7, 3)]   # N = 729, 625, 343


def upper_b(b, m, rand=I.DIGITAL_SHIFT, mp=I.MAP_CENTER, s=45, t=100, R=2, seed=13, g=I.G_COS, h=I.H_ID, K=0.0,
            c=1.0, A_scale=0.3):
    R = R if rand != I.NO_SHIFT else 1
    return I.make_custom(kind=I.DIGITAL_NET, m=m, s=s, t=t, w=I.w_logb(s, m + 1, b), rand=rand, R=R, map=mp, g=g,
                         h=h, K=K, c=c, seed=seed, A_scale=A_scale, net="upper", b=b)


def test_base_b_alg4_is_planned_for_upper_triangular_nets():
    from oracle import oracle as O
    torch_cuda()
    for b, m in UPPER_B:
        wl = upper_b(b, m)
        assert not O.net_is_periodic(wl)
        assert q.Points.from_workload(wl).split_level == -1


@pytest.mark.parametrize("b,m", UPPER_B)
@pytest.mark.parametrize("rand", RANDS)
@pytest.mark.parametrize("mp", [I.MAP_ID, I.MAP_CENTER, I.MAP_INVNORM])
def test_base_b_alg4_tables_bit_exact(b, m, rand, mp):
    """Values indexed by the integer of the reduced output digits over F_b
    (FP64) equal the oracle's bit for bit (the inverse-normal map to 1e-14)."""
    from oracle import oracle as O
    if mp == I.MAP_INVNORM and rand == I.NO_SHIFT:
        pytest.skip("the inverse-normal map requires a shift")
    torch_cuda()
    wl = upper_b(b, m, rand, mp, s=20)
    pts = q.Points.from_workload(wl)
    for r in range(wl.R):
        for j in range(wl.s):
            got = q.point_values(pts, r, j).cpu().numpy()
            ref = O.output_values(wl, r, j)
            if mp == I.MAP_INVNORM:
                np.testing.assert_allclose(got, ref, rtol=1e-14, atol=0)
            else:
                np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("b,m", UPPER_B)
def test_base_b_alg4_point_matrix_matches_unreduced(b, m):
    from oracle import oracle as O
    torch_cuda()
    wl = upper_b(b, m, s=30)
    pts = q.Points.from_workload(wl)
    for r in range(wl.R):
        X = q.point_matrix(pts, r).cpu().numpy()
        np.testing.assert_array_equal(X, O.point_matrix_unreduced(wl, r).astype(np.float32))


@pytest.mark.parametrize("b,m", UPPER_B)
@pytest.mark.parametrize("prec", [I.FP32, I.SPLIT_BF16X3])
def test_base_b_alg4_matvec_elementwise(b, m, prec):
    """Y = X A over every element within the FP32 (or split-BF16) bound: more
    than one 64-point tile (N not a multiple of 64), coordinates past one
    32-coordinate step, two column tiles with a ragged tail (t = 300)."""
    torch = torch_cuda()
    wl = upper_b(b, m, t=300)
    pts = q.Points.from_workload(wl)
    A = to_dev(wl.A, torch)
    for r in range(wl.R):
        Y = q.reduced_matvec(pts, A, r=r, prec=prec).cpu().numpy()
        _check_Y(wl, Y, r, prec)


@pytest.mark.parametrize("b,m", UPPER_B)
@pytest.mark.parametrize("g,h,c,mp", [(I.G_COS, I.H_ID, 1.0, I.MAP_CENTER), (I.G_EXP, I.H_CALL, 0.2, I.MAP_INVNORM)])
def test_base_b_alg4_estimate_and_gradient(b, m, g, h, c, mp):
    """Estimates within 1e-6 of the oracle; dQ/dA element by element within
    its bound and within 1e-6 (Frobenius), Algorithm 4 transposed over F_b."""
    from oracle import oracle as O
    torch = torch_cuda()
    K = 1.0 if h == I.H_CALL else 0.0
    wl = upper_b(b, m, I.DIGITAL_SHIFT, mp, g=g, h=h, c=c, K=K)
    pts = q.Points.from_workload(wl)
    Q = q.estimate(pts, to_dev(wl.A, torch), q.Integrand_.of(wl)).cpu().numpy()
    Qo, _ = O.estimate(wl)
    assert np.all(np.abs(Q - Qo) <= Q_TOL * np.maximum(np.abs(Qo), 1e-3)), (Q, Qo)
    _check_grad(wl, pts)


def test_base_b_alg4_static_scratch_and_autograd():
    """The allocation-free estimate and the autograd hook on a base-5 net that
    is not periodic."""
    import ctypes as ct
    torch = torch_cuda()
    wl = upper_b(5, 4, R=2)
    pts = q.Points.from_workload(wl)
    A = to_dev(wl.A, torch)
    f = q.Integrand_.of(wl)
    Qs = torch.empty(2, dtype=torch.float64, device="cuda")
    L = q.load()
    st = ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    q._lib.check(L.qmc_estimate_static(pts.handle, ct.c_void_p(A.data_ptr()), wl.t, wl.t, ct.byref(f.c_struct()), 0,
                                       ct.c_void_p(Qs.data_ptr()), st))
    assert torch.equal(Qs, q.estimate(pts, A, f))
    Ag = A.clone().requires_grad_(True)
    Qa = q.QMCEstimate.apply(Ag, pts, f, I.FP32)
    Qa.sum().backward()
    _, dA = q.estimate_grad(pts, A, f)
    assert torch.allclose(Ag.grad, dA.double().sum(0).float(), rtol=1e-6, atol=1e-12)


# ------------------------------------------------------------------ full-size workloads

def _expected():
    path = os.path.join(GOLDEN, "expected_full.json")
    with open(path) as fh:
        return json.load(fh)


@pytest.mark.parametrize("c", [1, 2, 3, 4, 5, 6, 7, 8])
def test_full_config_estimate(c):
    """Each workload at its full size, in the launch configuration the
    benchmark times: Q[r] within 1e-6 relative of the stored oracle values."""
    torch = torch_cuda()
    exp = _expected()[f"C{c}"]
    wl = I.make_config(c)
    pts = q.Points.from_workload(wl)
    A = to_dev(wl.A, torch)
    for prec in exp["precisions"]:
        Q = q.estimate(pts, A, q.Integrand_.of(wl), prec=prec).cpu().numpy()
        Qo = np.array(exp["Q"])
        n = len(Qo)
        rel = np.abs(Q[:n] - Qo) / np.abs(Qo)
        print(f"C{c} prec={prec} max rel err {rel.max():.3e}", flush=True)
        assert rel.max() <= Q_TOL, (c, prec, rel)


@pytest.mark.parametrize("c", [2, 3, 4, 5, 6, 8])
def test_full_config_sampled_rows(c):
    """qmc_reduced_matvec at full size: 48 sampled rows of Y = X A against the
    oracle's FP64 rows (tables indexed by k mod n_j), element-wise bound."""
    torch = torch_cuda()
    wl = I.make_config(c)
    pts = q.Points.from_workload(wl)
    A = to_dev(wl.A, torch)
    r = wl.R - 1
    Y = q.reduced_matvec(pts, A, r=r, prec=I.FP32)
    rng = np.random.default_rng(c)
    ks = np.concatenate([[0, 1, wl.N - 1], rng.integers(0, wl.N, 45)])
    Ys = Y[torch.from_numpy(ks).cuda()].cpu().numpy().astype(np.float64)
    del Y
    Yo, mag = oracle_rows(wl, r, ks)
    err = np.abs(Ys - Yo) / (elementwise_bound(wl, I.FP32) * mag + 1e-30)
    assert err.max() <= 1.0


def test_full_config_alg4_sampled_rows():
    """C7 (Algorithm 4) at full size: 48 sampled rows of Y = X A against the
    FP64 rows of the oracle's unreduced net, element-wise bound."""
    from oracle import oracle as O
    torch = torch_cuda()
    wl = I.make_config(7)
    pts = q.Points.from_workload(wl)
    A = to_dev(wl.A, torch)
    r = wl.R - 1
    Y = q.reduced_matvec(pts, A, r=r, prec=I.FP32)
    rng = np.random.default_rng(7)
    ks = np.concatenate([[0, 1, wl.N - 1], rng.integers(0, wl.N, 45)])
    Ys = Y[torch.from_numpy(ks).cuda()].cpu().numpy().astype(np.float64)
    del Y
    X = O.point_matrix_unreduced(wl, r)[ks]
    A64 = wl.A.astype(np.float64)
    err = np.abs(Ys - X @ A64) / (elementwise_bound(wl, I.FP32) * (np.abs(X) @ np.abs(A64)) + 1e-30)
    assert err.max() <= 1.0


@pytest.mark.parametrize("c", [5, 7, 8])
def test_full_config_gradient_columns(c):
    """Full-size gradients (C5 tree path; C7 Algorithm 4 transposed; C8 base 3
    with the split): for separable f each column of dA depends only on the same
    column of A, so the oracle computes a 64-column sample of the first
    randomisation exactly (rescaled by 64/t).  Relative Frobenius error <= 1e-6
    on the sample, and every sampled element within its error bound."""
    from oracle import oracle as O
    torch = torch_cuda()
    wl = I.make_config(c)
    pts = q.Points.from_workload(wl)
    A = to_dev(wl.A, torch)
    Q, dA = q.estimate_grad(pts, A, q.Integrand_.of(wl))
    cols = np.arange(3, wl.t, 16)[:64]
    sub = I.make_config(c)
    sub.A64 = np.ascontiguousarray(wl.A64[:, cols])
    sub.t = len(cols)
    _, dAo = O.estimate_grad(sub, shifts=1)
    dAo = dAo[0] * (len(cols) / wl.t)
    got = dA[0][:, torch.from_numpy(cols).cuda()].cpu().numpy().astype(np.float64)
    rel = np.linalg.norm(got - dAo) / np.linalg.norm(dAo)
    print(f"C{c} gradient sample rel err {rel:.3e}", flush=True)
    assert rel <= 1e-6
    # element by element: the bound of the 64-column workload, rescaled like dA
    D = adjoint_chain(wl, pts)
    E = grad_bound_lattice(sub, 0, I.FP32, D) if c == 5 else grad_bound_dense(sub, 0, I.FP32, D)
    worst = check_grad_elementwise(got, dAo, E * (len(cols) / wl.t), f"C{c}")
    print(f"C{c} gradient sample: worst element {worst:.3g} x its bound", flush=True)
    exp = _expected()[f"C{c}"]
    assert np.all(np.abs(Q.cpu().numpy() - exp["Q"]) <= Q_TOL * np.abs(exp["Q"]))

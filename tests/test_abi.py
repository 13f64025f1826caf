"""Host-side tests of the C ABI (no GPU needed): symbols, status codes, validation.

Every argument check of qmc_points_init runs on the host before any device
call, so each error path is exercised here without a GPU.
"""
import ctypes as ct
import os
import re

import numpy as np
import pytest

import paper_2305_11645_amd as q
from paper_2305_11645_amd import _lib
from paper_2305_11645_amd import inputs as I

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "qmcred.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qmc_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    L = _lib.load()
    names = declared_functions()
    assert len(names) >= 14
    assert sorted(names) == sorted(_lib.EXPORTS)
    for n in names:
        assert hasattr(L, n), n


def test_status_strings():
    L = _lib.load()
    for code, text in [(0, b"success"), (1, b"invalid argument"), (2, b"unsupported"),
                       (3, b"out of memory"), (4, b"device error")]:
        assert L.qmc_status_string(code) == text


def _spec(wl, **over):
    arrs = {}
    w = np.ascontiguousarray(over.pop("w", wl.w), dtype=np.int32)
    gen = np.ascontiguousarray(over.pop("gen", wl.gen), dtype=np.uint64)
    shift = over.pop("shift", wl.shift)
    dshift = over.pop("dshift", wl.dshift)
    samples = over.pop("samples", wl.samples)
    arrs["w"], arrs["gen"] = w, gen
    sp = _lib.PointSpec(b=over.pop("b", wl.b), m=over.pop("m", wl.m), s=over.pop("s", wl.s),
                        kind=over.pop("kind", wl.kind),
                        w=w.ctypes.data_as(ct.POINTER(ct.c_int32)),
                        gen=gen.ctypes.data_as(ct.POINTER(ct.c_uint64)),
                        rand=over.pop("rand", wl.rand), R=over.pop("R", wl.R), map=over.pop("map", wl.map))
    if shift is not None:
        arrs["shift"] = np.ascontiguousarray(shift, dtype=np.float64)
        sp.shift = arrs["shift"].ctypes.data_as(ct.POINTER(ct.c_double))
    if dshift is not None:
        arrs["dshift"] = np.ascontiguousarray(dshift, dtype=np.uint64)
        sp.dshift = arrs["dshift"].ctypes.data_as(ct.POINTER(ct.c_uint64))
    if samples is not None:
        arrs["samples"] = np.ascontiguousarray(samples, dtype=np.float64)
        sp.samples = arrs["samples"].ctypes.data_as(ct.POINTER(ct.c_double))
    assert not over, over
    return sp, arrs


def _init_status(sp):
    L = _lib.load()
    h = ct.c_void_p()
    st = L.qmc_points_init(ct.byref(h), ct.byref(sp))
    if st == 0:
        L.qmc_points_free(h)
    return st, L.qmc_last_error().decode()


def lat(**kw):
    return I.make_custom(kind=I.LATTICE, m=8, s=10, t=4, w=I.w_log2(10, 9), rand=I.RANDOM_SHIFT, R=2, **kw)


CASES = [
    ("b not prime", lambda wl: _spec(wl, b=4), 1),
    ("m too large", lambda wl: _spec(wl, m=25), 2),
    ("m zero", lambda wl: _spec(wl, m=0), 2),
    ("w0 nonzero", lambda wl: _spec(wl, w=np.r_[1, wl.w[1:]]), 1),
    ("w decreasing", lambda wl: _spec(wl, w=np.r_[wl.w[:5], [0] * 5]), 1),
    ("even generator", lambda wl: _spec(wl, gen=np.r_[[2], wl.gen[1:]]), 1),
    ("generator too big", lambda wl: _spec(wl, gen=np.r_[[2 ** 9 + 1], wl.gen[1:]]), 1),
    ("shift out of range", lambda wl: _spec(wl, shift=np.full((2, 10), 1.0)), 1),
    ("negative R", lambda wl: _spec(wl, R=0), 1),
    ("unknown kind", lambda wl: _spec(wl, kind=7), 1),
    ("unknown map", lambda wl: _spec(wl, map=9), 1),
    ("invnorm without shift", lambda wl: _spec(wl, rand=I.NO_SHIFT, R=1, shift=None, map=I.MAP_INVNORM), 1),
    ("R > 1 without shift", lambda wl: _spec(wl, rand=I.NO_SHIFT, R=2), 1),
]


@pytest.mark.parametrize("name,make,code", CASES, ids=[c[0] for c in CASES])
def test_points_init_validation(name, make, code):
    sp, keep = make(lat())
    st, msg = _init_status(sp)
    assert st == code, (name, st, msg)
    assert msg


def lat3(**kw):
    return I.make_custom(kind=I.LATTICE, m=5, s=10, t=4, w=I.w_logb(10, 6, 3), rand=I.RANDOM_SHIFT, R=2,
                         b=3, **kw)


BASE_CASES = [
    ("b = 3 net not periodic (Algorithm 4; stops at the device check)",
     lambda wl: _spec(wl, kind=I.DIGITAL_NET, gen=np.ones(10 * 5, dtype=np.uint64)), 4),
    ("b = 3 polynomial lattice", lambda wl: _spec(wl, kind=I.POLY_LATTICE), 4),
    ("b = 3 polynomial without constant term", lambda wl: _spec(wl, kind=I.POLY_LATTICE,
                                                                gen=np.r_[[3], wl.gen[1:]]), 1),
    ("b = 3 digital shift", lambda wl: _spec(wl, rand=I.DIGITAL_SHIFT, shift=None,
                                             dshift=np.zeros((2, 10), dtype=np.uint64)), 4),
    ("b = 3 digital shift >= b^K", lambda wl: _spec(wl, rand=I.DIGITAL_SHIFT, shift=None,
                                                    dshift=np.full((2, 10), 3 ** I.shift_digits(3),
                                                                   dtype=np.uint64)), 1),
    ("b^m above 2^24", lambda wl: _spec(wl, m=16), 2),
    ("generator divisible by b", lambda wl: _spec(wl, gen=np.r_[[3], wl.gen[1:]]), 1),
    ("generator not below b^e", lambda wl: _spec(wl, gen=np.r_[[3 ** 5 + 1], wl.gen[1:]]), 1),
    ("generator 2 is a unit mod 3^e", lambda wl: _spec(wl, gen=np.r_[[2], wl.gen[1:]]), 4),
]


@pytest.mark.parametrize("name,make,code", BASE_CASES, ids=[c[0] for c in BASE_CASES])
def test_base_b_points_init_validation(name, make, code):
    """A prime base b > 2 (Sections 1.1, 1.3, 3): N = b^m up to 2^24, lattice
    generators units modulo b^{m-w_j}, polynomials with a nonzero constant
    term, nets periodic after reduction or not, digital shifts below b^K (code 4: the
    spec is valid and the call reaches the device check, no GPU here)."""
    import torch
    if code == 4 and torch.cuda.is_available():
        pytest.skip("a valid spec creates the point set on a GPU")
    sp, keep = make(lat3())
    st, msg = _init_status(sp)
    assert st == code, (name, st, msg)
    assert msg


def iid(**kw):
    return I.make_custom(kind=I.IID, m=7, s=9, t=4, w=I.w_log2(9, 8), R=3, **kw)


def _bad_sample(wl, value):
    x = wl.samples.copy()
    x[2, 5] = value
    return x


IID_CASES = [
    ("with a random shift", lambda wl: _spec(wl, rand=I.RANDOM_SHIFT, shift=np.full((3, 9), 0.5)), 1),
    ("samples missing", lambda wl: _spec(wl, samples=None), 1),
    ("sample equal to one", lambda wl: _spec(wl, samples=_bad_sample(wl, 1.0)), 1),
    ("negative sample", lambda wl: _spec(wl, samples=_bad_sample(wl, -0.25)), 1),
    ("NaN sample", lambda wl: _spec(wl, samples=_bad_sample(wl, float("nan"))), 1),
    ("zero sample under Phi^-1", lambda wl: _spec(wl, map=I.MAP_INVNORM, samples=_bad_sample(wl, 0.0)), 1),
]


@pytest.mark.parametrize("name,make,code", IID_CASES, ids=[c[0] for c in IID_CASES])
def test_iid_points_init_validation(name, make, code):
    """Reduced Monte Carlo (Section 4): no shift, R independent replicates, and
    caller samples in [0,1) ((0,1) under the inverse-normal map)."""
    sp, keep = make(iid())
    st, msg = _init_status(sp)
    assert st == code, (name, st, msg)
    assert msg


def test_iid_valid_spec_reaches_the_device_check():
    """A valid reduced Monte Carlo spec with R > 1, no shift, Phi^-1 and a zero
    sample allowed only without that map passes validation (no GPU here)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible: the no-device path is not reachable")
    for mp in (I.MAP_ID, I.MAP_INVNORM):
        wl = iid(map=mp)
        sp, keep = _spec(wl, samples=_bad_sample(wl, 0.0) if mp == I.MAP_ID else wl.samples)
        st, msg = _init_status(sp)
        assert st == 4 and "device" in msg, msg


def test_digital_shift_range():
    wl = I.make_custom(kind=I.DIGITAL_NET, m=6, s=5, t=3, w=[0, 1, 2, 3, 3], rand=I.DIGITAL_SHIFT, R=1)
    sp, keep = _spec(wl, dshift=np.full((1, 5), 1 << 52, dtype=np.uint64))
    assert _init_status(sp)[0] == 1


def test_net_not_periodic_is_accepted():
    """An upper-triangular (Sobol'-type) matrix keeps columns beyond n_j after the
    row reduction, so the points are not periodic in k: valid, handled by
    Algorithm 4 (no GPU here, so the call stops at the device check)."""
    m, s = 6, 3
    words = []
    for j in range(s):
        for qq in range(m):
            words.append(sum(1 << p for p in range(qq + 1)))  # C_{p,q} = 1 for p <= q
    wl = I.make_custom(kind=I.DIGITAL_NET, m=m, s=s, t=2, w=[0, 2, 3], rand=I.NO_SHIFT)
    sp, keep = _spec(wl, gen=np.array(words, dtype=np.uint64))
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible: the no-device path is not reachable")
    assert _init_status(sp)[0] == 4


def test_net_word_beyond_m():
    wl = I.make_custom(kind=I.DIGITAL_NET, m=5, s=2, t=2, w=[0, 1], rand=I.NO_SHIFT)
    g = wl.gen.copy()
    g[0] |= np.uint64(1 << 7)
    sp, keep = _spec(wl, gen=g)
    assert _init_status(sp)[0] == 1


def test_valid_spec_without_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible: the no-device path is not reachable")
    sp, keep = _spec(lat())
    st, msg = _init_status(sp)
    assert st == 4 and "device" in msg


def test_null_handle_calls():
    L = _lib.load()
    f = _lib.Integrand(g=1, c=1.0, h=0, K=0.0)
    n = ct.c_size_t()
    assert L.qmc_workspace_size(None, 1, 8, ct.byref(f), 0, ct.byref(n)) == 1
    assert L.qmc_estimate(None, None, 8, 8, ct.byref(f), 0, None, None, 0, None) == 1
    assert L.qmc_reduced_matvec(None, 0, None, 8, 8, 0, None, 8, None, 0, None) == 1
    assert L.qmc_estimate_grad(None, None, 8, 8, ct.byref(f), 0, None, None, None, 0, None) == 1
    assert L.qmc_point_values(None, 0, 0, None, None) == 1
    assert L.qmc_points_free(None) == 0


def test_python_errors_are_typed():
    sp, keep = _spec(lat(), b=4)
    with pytest.raises(q.QMCInvalid):
        _lib.check(_lib.load().qmc_points_init(ct.byref(ct.c_void_p()), ct.byref(sp)))


def test_timing_api_on_host():
    q.timing.enable(True)
    q.timing.reset()
    assert q.timing.read("leaf") == (0.0, 0)
    q.timing.enable(False)


def test_one_hip_runtime_when_the_library_loads_first():
    """PyTorch's wheel carries its own HIP runtime under the system soname.
    Loading libqmcred before touching torch must still leave one HIP runtime in
    the process (torch's), or torch would find no GPU after the library took it."""
    import subprocess
    import sys
    code = ("import paper_2305_11645_amd as q; q.load()\n"
            "libs = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
            "print(len(libs)); print(sorted(libs))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.splitlines()[0] == "1", out.stdout

#!/usr/bin/env python3
"""Benchmark: reduced QMC estimate on one MI355X.

One step = qmc_estimate over every randomisation of the workload (point tables,
grouped upper-level products on the matrix cores, fused leaf pass with g and
the FP64 mean).  Inputs are resident in HBM before timing starts.

Prints ONE JSON line:
  metric/value   effective GFLOP/s = 2 N s t R / time (dense-equivalent count)
  roofline       the dominant kernel (the fused leaf pass) against the VALU peak
  cpu_baseline   the FP64 oracle on the host cores
  dense          the plain form on the same GPU: point matrix + FP32 GEMM + f + mean
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# ALU roofline.  MI355X's FP32 vector peak of 157.3 TFLOP/s counts the packed
# form v_pk_fma_f32 (two FP32 operations per lane and instruction).  This
# library is built without packed FP32 instructions (-packed-fp32-ops), so the
# unit count that bounds it is 256 CUs x 4 SIMDs x 16 lanes = 64 FP32 lanes
# per CU and clock: 256 x 64 x 2.4 GHz = 3.93e13 FMA lane-slots/s, 78.6 TFLOP/s
# (the same as the FP64 vector peak).  A transcendental (v_exp_f32, v_sin_f32,
# v_cos_f32) issues at half the FMA rate (qmc_probe_valu measures both on the
# box; the line carries the measured rates), so it costs 2 slots.  Achieved =
# 2 x algorithmic slots / duration, in FMA-equivalent TFLOP/s, against 78.6;
# the fraction against the packed 157.3 is reported beside it.
VALU_SLOTS_PER_S = 256 * 64 * 2.4e9
VALU_PEAK_TFLOPS = 2 * VALU_SLOTS_PER_S / 1e12
VALU_PACKED_PEAK_TFLOPS = 157.3
G_SLOTS = {0: 0, 1: 2, 2: 2}  # per evaluation of g: id; cos; exp (one transcendental)
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
MFMA_PEAK_TFLOPS = {0: 157.3, 1: 2500.0}  # dense FP32 and BF16 matrix-core peaks


def leaf_traffic(config: int, op: str = "estimate", kernel: str = "leaf_kernel"):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary of this workload, or None when there is none or the kernel's sources
    (listed in the summary) changed since the counters were taken."""
    import hashlib
    name = f"{kernel}_C{config}_counters.md" if op == "estimate" else f"{kernel}_{op}_C{config}_counters.md"
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    fields = {}
    for ln in open(path):
        if ":" in ln and ln.startswith("    "):
            k, v = ln.strip().split(":", 1)
            fields[k.strip()] = v.strip()
    csrc = os.path.join(ROOT, "paper_2305_11645_amd", "csrc")
    sources = fields.get("kernel_sources", "leaf.hip leaf_common.h qmc_internal.h").split()
    sha = hashlib.sha256(b"".join(open(os.path.join(csrc, f), "rb").read() for f in sources)).hexdigest()[:16]
    if fields.get("kernel_source_sha256_16") != sha or "hbm_bytes_per_dispatch" not in fields:
        return None
    return int(fields["hbm_bytes_per_dispatch"])


def leaf_algorithmic_slots(wl, split: int) -> float:
    """VALU lane slots the fused leaf pass must spend per launch (all shifts):
    the lower-level multiply-adds t R sum_{j: min(w_j,m) < L'} n_j (Theorem 2's
    count on those coordinates), one add per subtree root and upper level, and
    per point and column one g (a transcendental: 2 slots) and one accumulation."""
    m, t, R, N = wl.m, wl.t, wl.R, wl.N
    lev = np.minimum(wl.w, m)
    nlow = sum(2 ** (m - int(I)) for I in lev if I < split)
    nup = len({int(I) for I in lev if I >= split})
    nsub = 2 ** (m - split)
    return float(t * R * nlow + t * R * nsub * nup + N * t * R * (1 + G_SLOTS[wl.g]))


def grad_leaf_algorithmic_slots(wl, split: int) -> float:
    """VALU lane slots of the gradient-mode leaf pass per launch (all shifts):
    the lower-level multiply-adds forward and transposed, 2 t R sum_low n_j; one
    add per subtree root and upper level; per point and column g' (one
    transcendental, 2 slots, none for g = y) and, for separable h, g (shared
    with g' for exp) and its accumulation, else the factor h'; the folds of the
    transposed recursion (2^{L'} - 1 adds per subtree and column); and one
    accumulation per lower coordinate, subtree and column."""
    m, t, R, N = wl.m, wl.t, wl.R, wl.N
    lev = np.minimum(wl.w, m)
    nlow = sum(2 ** (m - int(I)) for I in lev if I < split)
    jlow = int(sum(1 for I in lev if I < split))
    nup = len({int(I) for I in lev if I >= split})
    nsub = 2 ** (m - split)
    per_point = G_SLOTS[wl.g]
    if wl.h == 0:
        per_point += (G_SLOTS[wl.g] if wl.g == 1 else 0) + 1
    else:
        per_point += 1
    return float(2 * t * R * nlow + t * R * nsub * nup + N * t * R * per_point
                 + t * R * nsub * (2 ** split - 1) + t * R * nsub * jlow)


_VALU_RATES = None


def measured_valu():
    """The VALU issue rates measured on this GPU (qmc_probe_valu), in T lane-ops/s."""
    global _VALU_RATES
    if _VALU_RATES is None:
        import paper_2305_11645_amd as q
        r = q.probe_valu()
        _VALU_RATES = {k: round(v / 1e12, 2) for k, v in r.items()}
    return _VALU_RATES


_MFMA_RATES = None


def measured_mfma():
    """The matrix-core rates measured on this GPU (qmc_probe_mfma), in TFLOP/s."""
    global _MFMA_RATES
    if _MFMA_RATES is None:
        import paper_2305_11645_amd as q
        q.probe_mfma()  # the first pass runs while the clocks ramp up
        r = q.probe_mfma()
        _MFMA_RATES = {k: round(v / 1e12, 1) for k, v in r.items()}
    return _MFMA_RATES


def alu_roofline(kernel: str, achieved: float, slots: float, avg_ms: float, traffic):
    """The roofline object of an ALU-bound kernel: achieved FMA-equivalent
    TFLOP/s against the unpacked FP32 peak, with the packed-peak fraction and the
    rates measured on this GPU beside it."""
    return {"bound": "alu", "kernel": kernel, "achieved": round(achieved, 3),
            "peak": round(VALU_PEAK_TFLOPS, 1), "unit": "TFLOP/s",
            "frac": round(achieved / VALU_PEAK_TFLOPS, 4), "traffic": traffic,
            "avg_ms": round(avg_ms, 5), "algorithmic_lane_ops": slots,
            "peak_note": "unpacked FP32: 256 CUs x 64 lanes x 2 flops x 2.4 GHz; transcendentals 2 slots",
            "frac_vs_packed_peak_157.3": round(achieved / VALU_PACKED_PEAK_TFLOPS, 4),
            "measured_rates_T_per_s": measured_valu()}


def calibrate_copy(mib: int) -> None:
    """One plain copy kernel over `mib` MiB after the timed work (an
    elementwise negation: reads mib MiB and writes mib MiB): the reference
    dispatch for scaling the HBM traffic counters.  (A plain tensor copy may
    run on the copy engines, which the counters do not see.)"""
    if not mib:
        return
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    del src, dst


def matvec_leaf_bytes(wl, pts) -> float:
    """Algorithmic HBM bytes of the matvec leaf pass for one randomisation: Y
    written once (N t 4 B), the subtree records, the upper-level rows U and the
    lower rows of A read once each."""
    m, t, N = wl.m, wl.t, wl.N
    split = pts.split_level
    lev = np.minimum(wl.w, m)
    nsub = 2 ** (m - split)
    rec = sum(2 ** (split - int(I)) for I in lev if I < split)
    urows = sum(2 ** (m - int(I)) for I in sorted({int(I) for I in lev if I >= split}))
    jlow = int(sum(1 for I in lev if I < split))
    ldu = -(-t // 64) * 64
    return float(4 * (N * t + nsub * rec + urows * ldu + jlow * t))


def bench_matvec(args, wl) -> int:
    """Y = X A for one randomisation per step, stored in HBM (the stored-Y form of
    the method): the leaf pass streams N x t FP32 values out."""
    import torch

    import paper_2305_11645_amd as q
    from paper_2305_11645_amd import inputs as I

    prec = wl.prec if args.prec is None else args.prec
    pts = q.Points.from_workload(wl)
    A = torch.from_numpy(wl.A).cuda()
    Y = torch.empty((wl.N, wl.t), dtype=torch.float32, device="cuda")
    ws = pts.workspace(0, wl.t, None, prec)
    stream = torch.cuda.current_stream()
    state = {"i": 0}

    def step():
        q.reduced_matvec(pts, A, r=state["i"] % wl.R, prec=prec, Y=Y, workspace=ws)
        state["i"] += 1

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps

    q.timing.reset()
    q.timing.enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    q.timing.enable(False)
    kern = {}
    for name in ("tables", "levels", "leaf"):
        tot, n = q.timing.read(name)
        if n:
            kern[name] = {"avg_ms": tot / n, "launches": n}
    q.timing.reset()

    ybytes = 4.0 * wl.N * wl.t
    value = ybytes / (ms * 1e-3) / 1e9
    leaf_ms = kern.get("leaf", {}).get("avg_ms", float("nan"))
    lbytes = matvec_leaf_bytes(wl, pts)
    achieved = lbytes / (leaf_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": "leaf_kernel (matvec mode)", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": leaf_traffic(args.config, "matvec"), "avg_ms": round(leaf_ms, 5),
                "algorithmic_bytes": lbytes}

    # accuracy gate and CPU baseline on a column sample: the FP64 oracle
    rel_err = None
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        r = (state["i"] - 1) % wl.R  # the shift of the last step
        Yg = Y.cpu().numpy()
        k = min(wl.t, 8)
        t0 = time.perf_counter()
        Yo = O.reduced_matvec(wl, r, A=wl.A[:, :k])
        one = time.perf_counter() - t0
        budget = 20.0
        k2 = int(max(k, min(wl.t, k * budget / max(one, 1e-9))))
        if k2 > k:
            t0 = time.perf_counter()
            Yo = O.reduced_matvec(wl, r, A=wl.A[:, :k2])
            one = time.perf_counter() - t0
            k = k2
        rel_err = float(np.max(np.abs(Yg[:, :k] - Yo)) / max(np.max(np.abs(Yo)), 1e-300))
        full = one * wl.t / k
        cpu = {"value": round(ybytes / full / 1e9, 4), "unit": "GB/s", "cores": O.num_threads(),
               "kind": "oracle", "seconds": round(one, 3),
               "sample": f"{k} of {wl.t} columns of Y for one randomisation, FP64 Algorithm 1 with "
                         f"point tables, scaled to all columns"}

    out = {
        "metric": "effective Y bandwidth GB/s (N*t*4 bytes of Y = X A per randomisation / time), reduced matvec",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == I.FP32 else "bf16x3",
        "data": "synthetic (seeded generators and shifts, random A)",
        "config": {"workload": wl.name + " (matvec)", "N": wl.N, "s": wl.s, "t": wl.t,
                   "split_level": pts.split_level,
                   "effective_gflops": round(2.0 * wl.N * wl.s * wl.t / (ms * 1e-3) / 1e9, 1)},
        "rel_err_vs_oracle": rel_err,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kern,
    }
    calibrate_copy(args.calibrate_copy_mib)
    print(json.dumps(out), flush=True)
    return 0


def bench_grad(args, wl) -> int:
    """Q and dQ/dA for every randomisation per step (qmc_estimate_grad): the
    forward pass, the sensitivities and the adjoint products.  value counts the
    dense-equivalent flops of the forward and adjoint products, 4 N s t R."""
    import torch

    import paper_2305_11645_amd as q

    prec = wl.prec if args.prec is None else args.prec
    f = q.Integrand_.of(wl)
    pts = q.Points.from_workload(wl)
    A = torch.from_numpy(wl.A).cuda()
    ws = pts.workspace(2, wl.t, f, prec)
    stream = torch.cuda.current_stream()

    def step():
        return q.estimate_grad(pts, A, f, prec, workspace=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        Q, dA = step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps

    q.timing.reset()
    q.timing.enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    q.timing.enable(False)
    kern = {}
    for name in ("tables", "levels", "leaf", "leaf_grad", "reduce", "levels_adj", "adjoint", "fold", "combine"):
        tot, n = q.timing.read(name)
        if n:
            kern[name] = {"ms_per_step": tot / args.steps, "launches": n}
    q.timing.reset()
    roofline = None
    if "adjoint" in kern:
        # the adjoint products: 2 N jlow t R flops over all points, plus
        # 2 n_split (s - jlow) t R over the folded upper coordinates (base b > 2)
        L = pts.grad_split_level
        jlow = wl.s if L < 0 else int(np.sum(np.minimum(wl.w, wl.m) < L))
        nsplit = wl.b ** (wl.m - L) if L >= 0 else 0
        mf = 2.0 * wl.t * wl.R * (wl.N * jlow + nsplit * (wl.s - jlow)) * (3 if prec == 1 else 1)
        peak = MFMA_PEAK_TFLOPS[prec]
        achieved = mf / (kern["adjoint"]["ms_per_step"] * 1e-3) / 1e12
        roofline = {"bound": "mfma", "kernel": "alg4_adj_kernel", "achieved": round(achieved, 3), "peak": peak,
                    "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                    "traffic": leaf_traffic(args.config, "grad", kernel="alg4_adj_kernel"),
                    "algorithmic_flops": mf, "measured_rates_TFLOP_per_s": measured_mfma()}
    elif "leaf_grad" in kern:
        # the tree path: the gradient-mode leaf pass is the dominant kernel
        lms = kern["leaf_grad"]["ms_per_step"] * args.steps / kern["leaf_grad"]["launches"]
        slots = grad_leaf_algorithmic_slots(wl, pts.grad_split_level)
        roofline = alu_roofline("grad_kernel (leaf, gradient mode)", 2 * slots / (lms * 1e-3) / 1e12, slots, lms,
                                leaf_traffic(args.config, "grad", kernel="grad_kernel"))
    flops = 4.0 * wl.N * wl.s * wl.t * wl.R
    out = {"metric": "estimate_grad_dense_equivalent_GFLOPs", "value": round(flops / (ms * 1e-3) / 1e9, 3),
           "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5),
           "higher_is_better": True, "dtype": "f32" if prec == 0 else "bf16x3", "data": "synthetic",
           "config": {"workload": f"C{args.config}", "N": wl.N, "s": wl.s, "t": wl.t, "R": wl.R, "b": wl.b,
                      "split_level": pts.grad_split_level},
           "roofline": roofline, "kernels": kern}
    calibrate_copy(args.calibrate_copy_mib)
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", type=int, default=4,
                    help="workload C1..C8 (default C4, the largest single-GPU workload)")
    ap.add_argument("--prec", type=int, default=None, help="0 = FP32, 1 = split-BF16x3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--dense-steps", type=int, default=3, help="timed steps of the dense plain form")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="after timing, run one plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--op", choices=("estimate", "matvec", "grad"), default="estimate",
                    help="estimate: Q for every randomisation (default); matvec: Y = X A stored in HBM; "
                         "grad: Q and dQ/dA")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (it would shard "
              "by randomisation, subtree root or column tile, with one all-reduce per call)",
              file=sys.stderr)
        return 2

    import torch

    import paper_2305_11645_amd as q
    from paper_2305_11645_amd import inputs as I

    torch.cuda.set_device(0)
    wl = I.make_config(args.config)
    if args.op == "matvec":
        return bench_matvec(args, wl)
    if args.op == "grad":
        return bench_grad(args, wl)
    return bench_estimate(args, wl)


def dense_estimate(pts, wl, A, rows: int):
    """The plain form on the same GPU, one randomisation at a time so that it
    fits in HBM at any workload: the FP32 point matrix X (N x s), then per
    chunk of `rows` points Y = X A on the matrix cores (hipBLASLt), g and the
    point means in place, and the FP64 sum of h over the points."""
    import torch

    from paper_2305_11645_amd import inputs as I
    import paper_2305_11645_amd as q
    Q = torch.empty(wl.R, dtype=torch.float64, device="cuda")
    for r in range(wl.R):
        X = q.point_matrix(pts, r)
        acc = torch.zeros((), dtype=torch.float64, device="cuda")
        for k0 in range(0, wl.N, rows):
            Y = X[k0:k0 + rows] @ A
            if wl.g == I.G_COS:
                Y.cos_()
            elif wl.g == I.G_EXP:
                Y.mul_(wl.c).exp_()
            u = Y.sum(dim=1, dtype=torch.float64) / wl.t
            if wl.h == I.H_CALL:
                u = torch.clamp(u - wl.K, min=0.0)
            acc += u.sum()
            del Y, u
        Q[r] = acc / wl.N
        del X
    return Q


def stored_oracle(wl, config: int, prec: int):
    """The FP64 oracle's estimates of this workload written by
    tests/golden/make_expected.py (a script that calls only the oracle), or
    None when the file has no entry for this workload and precision."""
    path = os.path.join(ROOT, "tests", "golden", "expected_full.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        exp = json.load(fh).get(f"C{config}")
    if not exp or exp.get("name") != wl.name or prec not in exp.get("precisions", []):
        return None
    return np.array(exp["Q"], dtype=np.float64)


def bench_estimate(args, wl) -> int:
    """Q for every randomisation per step (qmc_estimate): point tables, grouped
    upper-level products, fused leaf pass with g, FP64 mean.  Exits non-zero
    when an estimate differs from the FP64 oracle by more than 1e-6 relative."""
    import torch

    import paper_2305_11645_amd as q
    from paper_2305_11645_amd import inputs as I

    prec = wl.prec if args.prec is None else args.prec
    f = q.Integrand_.of(wl)
    pts = q.Points.from_workload(wl)
    A = torch.from_numpy(wl.A).cuda()
    ws = pts.workspace(1, wl.t, f, prec)
    Q = torch.empty(wl.R, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def step():
        q.estimate(pts, A, f, prec, Q=Q, workspace=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    Qg = Q.cpu().numpy()
    print(f"timed {args.steps} steps of {wl.name}: {ms:.4f} ms per step", file=sys.stderr, flush=True)

    # per-kernel durations: the same steps again with the library's event hooks
    q.timing.reset()
    q.timing.enable(True)
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    q.timing.enable(False)
    kern = {}
    for name in ("tables", "levels", "leaf", "reduce"):
        tot, n = q.timing.read(name)
        if n:
            kern[name] = {"avg_ms": tot / n, "launches": n}
    q.timing.reset()

    flops = 2.0 * wl.N * wl.s * wl.t * wl.R
    value = flops / (ms * 1e-3) / 1e9
    leaf_ms = kern.get("leaf", {}).get("avg_ms", float("nan"))
    if pts.split_level < 0 or wl.b != 2:
        # gathered value tiles (a net that is not periodic, Algorithm 4; or a
        # base b > 2): the tile products run on the matrix cores.  The timed
        # kernel is the pass over all N points and the jlow lower coordinates
        # (jlow = s in one pass; a base b > 2 with split level L' sums the
        # coordinates with w_j >= L' over the b^{m-L'} residues first):
        # 2 N jlow t R flops per launch (three BF16 products each with the
        # split precision)
        L = pts.split_level
        jlow = wl.s if L < 0 else int(np.sum(np.minimum(wl.w, wl.m) < L))
        mf = 2.0 * wl.N * jlow * wl.t * wl.R * (3 if prec == I.SPLIT_BF16X3 else 1)
        peak = MFMA_PEAK_TFLOPS[prec]
        achieved = mf / (leaf_ms * 1e-3) / 1e12
        # the method's own count (Section 3, the remark after Algorithm 4):
        # N jlow t R additions and t R sum_j n_j multiplications, one flop each
        nsum = float(np.sum(wl.b ** (wl.m - np.minimum(wl.w, wl.m))[: jlow]))
        method = float(wl.N * jlow * wl.t * wl.R + wl.t * wl.R * nsum)
        roofline = {"bound": "mfma", "kernel": "alg4_kernel", "achieved": round(achieved, 3),
                    "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                    "traffic": leaf_traffic(args.config, kernel="alg4_kernel"), "avg_ms": round(leaf_ms, 5),
                    "algorithmic_flops": mf,
                    "note": "algorithmic_flops are the matrix-core multiply-adds the kernel issues "
                            "(each of the method's additions becomes one multiply-add on a point value)",
                    "method_flops": method,
                    "frac_method_count": round(method / (leaf_ms * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS[0], 4),
                    "measured_rates_TFLOP_per_s": measured_mfma()}
    else:
        slots = leaf_algorithmic_slots(wl, pts.split_level)
        achieved = 2 * slots / (leaf_ms * 1e-3) / 1e12
        roofline = alu_roofline("leaf_kernel", achieved, slots, leaf_ms, leaf_traffic(args.config))

    dense = None
    if not args.no_dense:
        rows = min(wl.N, 1 << 16)
        Qd = dense_estimate(pts, wl, A, rows)
        torch.cuda.synchronize()
        d0, d1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        nd = args.dense_steps
        d0.record(stream)
        for _ in range(nd):
            Qd = dense_estimate(pts, wl, A, rows)
        d1.record(stream)
        torch.cuda.synchronize()
        dms = d0.elapsed_time(d1) / nd
        dense = {"ms_per_step": round(dms, 4), "value": round(flops / (dms * 1e-3) / 1e9, 1),
                 "speedup_reduced_vs_dense": round(dms / ms, 2), "steps": nd,
                 "rows_per_gemm": rows,
                 "rel_diff_vs_reduced": float(np.max(np.abs(Qd.cpu().numpy() - Qg) / np.abs(Qg)))}
        print(f"dense plain form: {dms:.2f} ms per step", file=sys.stderr, flush=True)

    calibrate_copy(args.calibrate_copy_mib)
    del ws

    # accuracy gate and CPU baseline: the FP64 oracle, live on a sample of the
    # randomisations (timed on the host cores) and, for every randomisation,
    # the oracle's stored estimates of this workload
    rel_err = None
    rel_all = None
    cpu = None
    Qs = stored_oracle(wl, args.config, prec)
    if Qs is not None:
        rel_all = float(np.max(np.abs(Qg - Qs) / np.abs(Qs)))
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        sample_R = wl.R
        budget = 25.0
        t0 = time.perf_counter()
        Qo, _ = O.estimate(wl, shifts=1)
        one = time.perf_counter() - t0
        if one * wl.R > budget:
            sample_R = max(1, int(budget // max(one, 1e-9)))
        if sample_R > 1:
            t0 = time.perf_counter()
            Qo, _ = O.estimate(wl, shifts=sample_R)
            dt = time.perf_counter() - t0
        else:
            dt = one
        rel_err = float(np.max(np.abs(Qg[:sample_R] - Qo) / np.abs(Qo)))
        cpu_flops = 2.0 * wl.N * wl.s * wl.t * sample_R
        cpu = {"value": round(cpu_flops / dt / 1e9, 3), "unit": "GFLOP/s", "cores": O.num_threads(),
               "kind": "oracle", "seconds": round(dt, 3),
               "sample": f"{sample_R} of {wl.R} randomisations of the full workload, FP64 Algorithm 1 "
                         f"with point tables, f and compensated mean"}

    out = {
        "metric": "effective GFLOP/s (2*N*s*t*R/time), reduced QMC estimate vs dense X*A, rel err <= 1e-6",
        "value": round(value, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == I.FP32 else "bf16x3",
        "data": "synthetic (seeded generators, shifts and A of the workload recipe)",
        "config": {"workload": wl.name, "N": wl.N, "s": wl.s, "t": wl.t, "R": wl.R,
                   "split_level": pts.split_level, "distinct_values_per_shift": pts.distinct_values},
        "rel_err_vs_oracle": rel_err,
        "rel_err_vs_stored_oracle_all_shifts": rel_all,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "dense": dense,
        "kernels": kern,
    }
    print(json.dumps(out), flush=True)
    errs = [e for e in (rel_err, rel_all) if e is not None]
    if any(not (e <= 1e-6) for e in errs):
        print(f"estimate differs from the FP64 oracle by {max(errs):.3e} > 1e-6", file=sys.stderr)
        return 1
    return 0


if __name__ == "__main__":
    sys.exit(main())

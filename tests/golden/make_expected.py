"""Write expected_full.json: FP64 oracle estimates of the full-size workloads.

Calls only the oracle (oracle/) and the seeded input generators.  Run from the
repository root:  python tests/golden/make_expected.py [c ...]
(with workload numbers, only those are recomputed and merged into the file).
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2305_11645_amd import inputs as I  # noqa: E402

PRECISIONS = {1: [I.FP32], 2: [I.FP32, I.SPLIT_BF16X3], 3: [I.SPLIT_BF16X3, I.FP32],
              4: [I.FP32, I.SPLIT_BF16X3], 5: [I.FP32], 6: [I.FP32], 7: [I.FP32, I.SPLIT_BF16X3],
              8: [I.FP32, I.SPLIT_BF16X3]}


def main():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "expected_full.json")
    which = [int(a) for a in sys.argv[1:]] or sorted(PRECISIONS)
    out = {}
    if sys.argv[1:] and os.path.exists(path):
        with open(path) as fh:
            out = json.load(fh)
    for c in which:
        wl = I.make_config(c)
        t0 = time.perf_counter()
        Q, nmadd = O.estimate(wl)
        dt = time.perf_counter() - t0
        out[f"C{c}"] = {"name": wl.name, "Q": [float(v) for v in Q], "precisions": PRECISIONS[c],
                        "oracle_seconds": round(dt, 2), "oracle_threads": O.num_threads(),
                        "multiply_adds": nmadd}
        print(f"C{c}: R={len(Q)} Q[0]={Q[0]:.15g} {dt:.1f}s", flush=True)
    out = {k: out[k] for k in sorted(out, key=lambda k: int(k[1:]))}
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(path)


if __name__ == "__main__":
    main()

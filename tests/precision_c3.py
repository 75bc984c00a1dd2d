"""Precision report for the 1024 x 1024 workload (c3_1024) against the FP64 oracle.

Test infrastructure (runs the oracle on the CPU; too slow for the test suite):

  python tests/precision_c3.py mu
      Generates c3_1024 in FP64, computes u_max by the oracle's power
      iteration and writes tests/golden/c3_1024_mu.json with the step
      mu = 0.9 / (2 u_max) rounded to FP32.  Both sides use this mu.

  python bench.py --config c3_1024 --vt f32 --mu-file tests/golden/c3_1024_mu.json \
      --dump-every 50 --dump c3_f32.npz   (on the GPU; likewise --vt f16)

  python tests/precision_c3.py compare c3_f32.npz c3_f16.npz
      Runs 300 oracle epochs (FP64 values, the FP32-rounded y and mu) and
      prints the relative L2 error ||x_dev - x_orc|| / ||x_orc|| of each
      device run every 50 epochs.  With --dequantised, the oracle uses the
      FP16-rounded matrix instead (isolates the accumulation error of the
      FP16-value form).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

MU_FILE = os.path.join(ROOT, "tests", "golden", "c3_1024_mu.json")


def _problem():
    t = time.time()
    p = synth.make_problem("c3_1024", with_transpose=False)
    print(f"generated c3_1024: nnz={p.nnz} in {time.time() - t:.0f} s", flush=True)
    return p


def _matrix(p, values=None):
    # int32 row pointers keep scipy from copying the 1.9e9 indices to int64
    rp = p.row_ptr.astype(np.int32) if p.nnz < 2**31 - 1 else p.row_ptr
    return oracle.as_matrix(rp, p.col, p.val if values is None else values, p.ncols)


def cmd_mu(_args):
    p = _problem()
    A = _matrix(p)
    t = time.time()
    u = oracle.power_umax(A, tol=1e-10)
    mu32 = float(np.float32(oracle.step_size(u)))
    out = {"workload": "c3_1024", "u_max": u, "mu_f32": mu32, "lam": p.lam,
           "epochs": p.epochs, "prox_iters": p.prox_iters,
           "source": "oracle.power_umax(tol=1e-10) on the FP64 matrix; mu = 0.9/(2 u_max) "
                     "rounded to FP32 (Theorem 1 bound 1/(2 u_max))"}
    with open(MU_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(f"u_max = {u!r} ({time.time() - t:.0f} s), mu = {mu32!r} -> {MU_FILE}")


def cmd_compare(args):
    ref = json.load(open(MU_FILE))
    runs = {os.path.basename(f): np.load(f) for f in args.npz}
    p = _problem()
    vals = None
    if args.dequantised:
        vals = p.val.astype(np.float32).astype(np.float16).astype(np.float64)
    A = _matrix(p, vals)
    y32 = p.y.astype(np.float32).astype(np.float64)
    mu, lam, K = ref["mu_f32"], ref["lam"], ref["prox_iters"]
    x, r = oracle.initial_state(A, y32)
    every = args.every
    rows = []
    t = time.time()
    for k in range(1, ref["epochs"] + 1):
        x, r = oracle.bsgd_epoch(A, y32, x, r, mu, lam, K, (p.H, p.W))
        if k % every == 0:
            line = {"epoch": k}
            for name, d in runs.items():
                key = f"x{k}"
                if key in d:
                    xd = d[key].astype(np.float64)
                    line[name] = float(np.linalg.norm(xd - x) / np.linalg.norm(x))
            rel_true = float(np.linalg.norm(x - p.x_true.ravel()) / np.linalg.norm(p.x_true))
            line["oracle_vs_phantom"] = rel_true
            rows.append(line)
            print(json.dumps(line), f"({time.time() - t:.0f} s)", flush=True)
    print("| epoch | " + " | ".join(runs) + " | oracle vs phantom |")
    print("|---" * (len(runs) + 2) + "|")
    for line in rows:
        print(f"| {line['epoch']} | " + " | ".join(f"{line.get(n, float('nan')):.2e}" for n in runs)
              + f" | {line['oracle_vs_phantom']:.4f} |")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    sub.add_parser("mu")
    c = sub.add_parser("compare")
    c.add_argument("npz", nargs="+")
    c.add_argument("--every", type=int, default=50)
    c.add_argument("--dequantised", action="store_true")
    args = ap.parse_args()
    {"mu": cmd_mu, "compare": cmd_compare}[args.cmd](args)


if __name__ == "__main__":
    main()

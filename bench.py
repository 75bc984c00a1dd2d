#!/usr/bin/env python3
"""Benchmark of the BSGD-TV hot path on one MI355X.

One step = one whole reconstruction job of the 512 x 512 workload
(720 angles x 729 bins, M = N = 8 blocks, lambda = 0.01, 200 epochs, 20 FGP
iterations), starting from A, A^T (FP32 CSR) and y already resident in HBM:
    S0   the plan                         (bsgd_plan_create: no block store with
                                           --path fused, block stores of A and A^T
                                           with --path rows)
         and the tile-sliced store         (bsgd_fused_create, from A's CSR; --path fused)
    S0'  u_max by Lanczos bidiagonalisation (or --umax power), mu = 0.9 / (2 u_max)
    S1-S5 x 200 epochs                     (bsgd_run_epochs)
With --path fused (default) every epoch reads the matrix once (both
products in one pass); --path rows runs one pass over A and one over A^T.
The reported value is epochs per second over whole jobs (setup included).

Prints one JSON line.  --gpus above 1 is refused: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HBM_PEAK_GBS = 8000.0

# Ray chunks of the volume workload's tile-sliced store (0 = the library's
# one-RHS choice, 16 at 512^2).
VOLUME_CHUNKS = 4

# Kernel durations inside the timed jobs are sampled on one epoch in 20 (10 of
# a 200-epoch job; the events cost about 1% of a job at one epoch in 8).
TIMING_STRIDE = 20

# HBM bytes per launch of the dominant kernel, from rocprofv3 FETCH_SIZE /
# WRITE_SIZE runs (scaled by what the counters read for a plain copy), keyed
# by (path, workload, value type[, staged, direction]).  Valid only while the
# kernel and layout sources hash to the value recorded with the counters;
# otherwise the figure is reported as null.
PMC_TRAFFIC = {
    # profiles/k_fused_c2_512_hbm_counters.md
    ("fused", "c2_512", "f32"): {
        "sha256": "b1031d260261612f55747aebdfd13da5c405b84b08459f6671cb4adb02f44269",
        "bytes": 1328371187},
    # profiles/k_fused_f16_c2_512_counters.md
    ("fused", "c2_512", "f16"): {
        "sha256": "b1031d260261612f55747aebdfd13da5c405b84b08459f6671cb4adb02f44269",
        "bytes": 826097760},
    # profiles/k_fused_c3_1024_counters_and_trace.md
    ("fused", "c3_1024", "f32"): {
        "sha256": "b1031d260261612f55747aebdfd13da5c405b84b08459f6671cb4adb02f44269",
        "bytes": 10604834425},
    ("fused", "c3_1024", "f16"): {
        "sha256": "b1031d260261612f55747aebdfd13da5c405b84b08459f6671cb4adb02f44269",
        "bytes": 6820311354},
    # profiles/k_fused_ista_c2_512_hbm_counters.md (the A x-only pass)
    ("fused", "c2_512", "f32", "ista"): {
        "sha256": "b1031d260261612f55747aebdfd13da5c405b84b08459f6671cb4adb02f44269",
        "bytes": 1310861175},
    ("fused", "c2_512", "f32", "gd"): {
        "sha256": "b1031d260261612f55747aebdfd13da5c405b84b08459f6671cb4adb02f44269",
        "bytes": 1310861175},
    # profiles/k_vol_c4_hbm_counters.md (256 slices, 4 ray chunks)
    ("fused_mr", "c4_vol", "f32", 256, 4, "fwd"): {
        "sha256": "b1031d260261612f55747aebdfd13da5c405b84b08459f6671cb4adb02f44269",
        "bytes": 24547917882},
    # profiles/k_sel_c2_512_hbm_counters.md (mean over the 1600 draws of the profiled run)
    ("selected", "c2_512", "f32", 0.5, 0.5, 7, "fwd"): {
        "sha256": "6770bf9e9f1b1b8762c95e142841c0b5db6cb88ca2f49af4baa5a0a4d5c921b6",
        "bytes": 613991197},
}


# Sources that determine each path's dominant kernel and the layout it reads
# (the kernel's file and the block-store build it starts from).
_KERNEL_SOURCES = {
    "fused": ("fused.hip", "plan.hip"),
    "rows": ("spmv.hip", "plan.hip", "staged.hip"),
    "selected": ("spmv.hip", "plan.hip", "state.hip"),
}


def _code_text(src):
    """The source with its comments and blank lines taken out: what the compiler
    sees, so that a change of wording in a comment keeps the recorded counters.
    (The kernel sources hold no string literal with a comment marker in it.)"""
    import re
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return "\n".join(l.rstrip() for l in src.splitlines() if l.strip()) + "\n"


def _kernel_source_hash(path):
    import hashlib
    h = hashlib.sha256()
    base = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1812_01307_amd", "csrc")
    for f in _KERNEL_SOURCES[path]:
        with open(os.path.join(base, f), encoding="utf-8") as fh:
            h.update(_code_text(fh.read()).encode())
    return h.hexdigest()


def _block_stores(flags):
    """Which block stores a plan with these flags builds."""
    import paper_1812_01307_amd as bsgd
    if flags & bsgd.BSGD_PLAN_SINGLE_PASS_ONLY:
        return "none (tile-sliced store from A's CSR)"
    return "A" if flags & bsgd.BSGD_PLAN_FWD_ONLY else "A and A^T"


def _alg_bytes(nnz, r, c, val_bytes):
    """Algorithmic HBM bytes per launch of the two fused row kernels."""
    fwd = (val_bytes + 4) * nnz + 8 * (r + 1) + 4 * c + 4 * r + 4 * r  # A, ptr, x, y, r'
    bwd = (val_bytes + 4) * nnz + 8 * (c + 1) + 4 * r + 4 * c + 4 * c  # A^T, ptr, r, x, x^
    return fwd, bwd


def cpu_baseline_bsgd(args):
    """The FP64 oracle of Algorithm 1 timed on the host: one thread, then one
    independent reconstruction per core (worker processes forked after the
    matrix is built, so they share it).  Returns the cpu_baseline record."""
    import multiprocessing as mp

    import numpy as np

    import oracle  # CPU baseline leg only
    import synth

    t = time.perf_counter()
    prob = synth.make_problem(args.config, with_transpose=False)
    rp = prob.row_ptr.astype(np.int32) if prob.nnz < 2**31 - 1 else prob.row_ptr
    A64 = oracle.as_matrix(rp, prob.col, prob.val, prob.ncols)
    # any stable step serves for timing: a few power iterations
    mu = 0.9 / (2.0 * oracle.power_umax(A64, tol=1e-6, max_iter=5))
    shape, K, y = (prob.H, prob.W), prob.prox_iters, prob.y
    # about 10 s of one core at 512^2 (0.5 s per epoch); fewer epochs at 1024^2
    e1 = args.cpu_epochs if args.config == "c2_512" else max(2, args.cpu_epochs // 8)
    print(f"[bench] cpu baseline: oracle set-up {time.perf_counter() - t:.1f} s, "
          f"{e1} epochs on one thread", file=sys.stderr, flush=True)
    xc, rc = oracle.initial_state(A64, y)
    t0 = time.perf_counter()
    oracle.bsgd_tv(A64, y, mu, prob.lam, e1, K, shape, state=(xc, rc))
    t1 = time.perf_counter() - t0
    try:
        ncores = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        ncores = os.cpu_count() or 1
    nproc = max(1, min(ncores, 16))
    ea = max(2, e1 // 2)
    ctx = mp.get_context("fork")
    gate = ctx.Barrier(nproc + 1)

    def work():
        x0, r0 = oracle.initial_state(A64, y)
        gate.wait()
        oracle.bsgd_tv(A64, y, mu, prob.lam, ea, K, shape, state=(x0, r0))

    print(f"[bench] cpu baseline: {nproc} processes x {ea} epochs", file=sys.stderr, flush=True)
    procs = [ctx.Process(target=work) for _ in range(nproc)]
    for pr in procs:
        pr.start()
    gate.wait()
    t0 = time.perf_counter()
    for pr in procs:
        pr.join()
    ta = time.perf_counter() - t0
    ok = all(pr.exitcode == 0 for pr in procs)
    one = {"value": round(e1 / t1, 4), "unit": "epochs/s", "cores": 1,
           "sample": f"{e1} epochs in {t1:.1f} s"}
    if not ok:
        return dict(one, kind="oracle", sample=one["sample"] + " (all-cores leg failed)")
    return {"value": round(nproc * ea / ta, 4), "unit": "epochs/s", "cores": nproc,
            "kind": "oracle",
            "sample": f"{nproc} independent reconstructions of {args.config} on {nproc} of "
                      f"{ncores} host cores, {ea} epochs each (FP64 numpy/scipy, one thread "
                      f"per process, set-up excluded) in {ta:.1f} s",
            "single_thread": one}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2_512")
    ap.add_argument("--vt", choices=["f32", "f16"], default="f32")
    ap.add_argument("--epochs", type=int, default=None, help="override the workload's epoch count")
    ap.add_argument("--umax", default="lanczos", choices=["lanczos", "power"],
                    help="u_max for the step size: Lanczos bidiagonalisation or power iteration")
    ap.add_argument("--umax-steps", type=int, default=4,
                    help="Lanczos steps (each one product with A and one with A^T)")
    ap.add_argument("--power-iters", type=int, default=30)
    ap.add_argument("--cpu-epochs", type=int, default=20,
                    help="oracle epochs timed for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true")
    ap.add_argument("--autotune", action="store_true", help="time lane counts during plan creation")
    ap.add_argument("--path", default="fused", choices=["fused", "rows"],
                    help="epoch products: one pass over the tile-sliced store (fused) or one "
                         "pass over A and one over A^T (rows)")
    ap.add_argument("--method", default="bsgd", choices=["bsgd", "ista", "gd", "selected"],
                    help="update rule: Algorithm 1 (bsgd), the Simulations section's comparison "
                         "methods (ista; gd = ista without the TV term), or Algorithm 1 on drawn "
                         "block subsets (selected: fractions --alpha of the column blocks and "
                         "--gamma of the row blocks per iteration; epochs normalised)")
    ap.add_argument("--alpha", type=float, default=0.5)
    ap.add_argument("--gamma", type=float, default=0.5)
    ap.add_argument("--select-seed", type=int, default=7)
    ap.add_argument("--fused-chunks", type=int, default=0,
                    help="ray chunks of the tile-sliced store (0: automatic; volumes: %d)"
                    % VOLUME_CHUNKS)
    ap.add_argument("--fused-waves", type=int, default=8, choices=[2, 4, 8],
                    help="wavefronts per (tile, chunk) workgroup of the single pass")
    ap.add_argument("--mr-waves", type=int, default=0, choices=[0, 8, 16],
                    help="volume workload: wavefronts per workgroup of the several-RHS pass "
                         "(0: the library's default, 16)")
    ap.add_argument("--staged", default=None, choices=["none", "fwd", "bwd", "both"],
                    help="directions built in the staged form (LDS-served gathers) and used by "
                         "the epochs of --path rows (default bwd; none with --path fused)")
    ap.add_argument("--overlap", type=int, default=1, choices=[0, 1, 2],
                    help="epoch schedule: forward pass concurrent with backprojection (0), after it "
                         "and concurrent with the prox (1), or after the prox on one stream (2)")
    ap.add_argument("--prox-schedule", type=int, default=None, choices=[0, 1],
                    help="2-D prox kernels: 0 fused chunks, 1 one launch per iteration "
                         "(default: the library's)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--mu-file", default=None,
                    help="JSON with a fixed step mu_f32 (precision runs against the oracle); "
                         "the jobs then skip the power iteration")
    ap.add_argument("--dump", default=None, help="save the iterate every --dump-every epochs (npz)")
    ap.add_argument("--dump-every", type=int, default=50)
    ap.add_argument("--slices", type=int, default=256,
                    help="volume workload (--config c4_vol): number of slices")
    ap.add_argument("--no-graph", action="store_true",
                    help="volume workload: run the epochs eagerly instead of graph replays")
    ap.add_argument("--requests", type=int, default=160,
                    help="serving workload (--config c5_serve): number of requests")
    ap.add_argument("--rate", type=float, default=40.0, help="serving: mean arrivals per second")
    ap.add_argument("--slots", type=int, default=8, help="serving: slots per batch state")
    ap.add_argument("--chunk", type=int, default=10, help="serving: epochs between stop checks")
    ap.add_argument("--no-unbatched", action="store_true",
                    help="serving: skip the one-request-at-a-time comparison run")
    args = ap.parse_args(argv)

    if args.method == "selected":
        args.path = "rows"   # the subset iterations run on the block store
    if args.staged is None:
        args.staged = "none" if args.path == "fused" or args.method == "selected" else "bwd"
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; the library runs on exactly one GPU "
              "(see the design notes for how the path would shard)", file=sys.stderr)
        return 2

    # the oracle's all-cores leg forks worker processes: it runs before this
    # process touches the GPU
    pre_cpu = None
    if (not args.no_cpu_baseline and args.cpu_epochs > 0 and args.method == "bsgd"
            and args.config in ("c2_512", "c3_1024") and not args.copy_calibration):
        pre_cpu = cpu_baseline_bsgd(args)

    import numpy as np
    import torch

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_dispatch": src.numel() * 4, "dispatches": 3}))
        return 0

    import synth
    import paper_1812_01307_amd as bsgd

    if args.config == "c4_vol":
        return run_volume(args, np, torch, synth, bsgd)
    if args.config == "c5_serve":
        return run_serve(args, np, torch, synth, bsgd)

    print(f"[bench] generating {args.config}", file=sys.stderr, flush=True)
    t_gen = time.perf_counter()
    # FP32 matrix values for the device (the projections y are FP64-computed)
    prob = synth.make_problem(args.config, dtype=np.float32)
    tp, tc, tv = prob.ensure_transpose()
    t_gen = time.perf_counter() - t_gen
    epochs = args.epochs or prob.epochs
    K = prob.prox_iters
    vt = bsgd.BSGD_VAL_F16 if args.vt == "f16" else bsgd.BSGD_VAL_F32
    flags = bsgd.BSGD_PLAN_F16 if vt == bsgd.BSGD_VAL_F16 else 0
    flags |= {"none": 0, "fwd": bsgd.BSGD_PLAN_STAGED_FWD, "bwd": bsgd.BSGD_PLAN_STAGED_BWD,
              "both": bsgd.BSGD_PLAN_STAGED}[args.staged]
    r, c, nnz = prob.nrows, prob.ncols, prob.nnz

    # inputs resident in HBM before the timed region
    A = (r, c, bsgd.to_device(prob.row_ptr, torch.int64), bsgd.to_device(prob.col, torch.int32),
         bsgd.to_device(prob.val, torch.float32))
    At = (c, r, bsgd.to_device(tp, torch.int64), bsgd.to_device(tc, torch.int32),
          bsgd.to_device(tv, torch.float32))
    y = bsgd.to_device(prob.y, torch.float32)
    torch.cuda.synchronize()
    print(f"[bench] nnz={nnz} rows={r} cols={c} gen={t_gen:.1f}s", file=sys.stderr, flush=True)

    timing = not args.no_kernel_timing
    acc = {"fwd": 0.0, "bwd": 0.0, "prox": 0.0, "n": 0}
    fused = args.path == "fused"

    tuned = None
    launch = {}
    if args.autotune and not fused:
        # one autotuned plan outside the timed region; its launch choice is
        # reused by every timed job (the tuner's cache)
        p0 = bsgd.bsgd_plan_create(A, At, prob.M, prob.N, prob.row_off, prob.col_off, prob.H,
                                   prob.W, 1, prob.bins, flags | bsgd.BSGD_PLAN_AUTOTUNE)
        tuned = (bsgd.bsgd_plan_lanes(p0), bsgd.bsgd_plan_staged(p0))
        del p0
        print(f"[bench] autotuned launch {tuned}", file=sys.stderr, flush=True)

    selected = args.method == "selected"
    if fused and args.umax == "lanczos" and not selected and args.staged in ("none", "fwd"):
        # the tile-sliced store serves both products (and the Lanczos ones):
        # the plan keeps no block store of A^T, and none of A unless its
        # staged form is asked for (the tile-sliced store is then built
        # straight from A's CSR)
        flags |= bsgd.BSGD_PLAN_FWD_ONLY
        if args.staged == "none":
            flags |= bsgd.BSGD_PLAN_SINGLE_PASS_ONLY
    lam_run = 0.0 if args.method == "gd" else prob.lam
    n_updates = epochs
    if selected:
        # enough iterations that the normalised epoch count reaches `epochs`
        frac = (max(1, round(args.gamma * prob.M)) * max(1, round(args.alpha * prob.N))
                / (prob.M * prob.N))
        n_updates = int(math.ceil(epochs / frac - 1e-9))
        rows_sel, cols_sel = synth.block_subsets(n_updates, prob.M, prob.N, args.alpha,
                                                 args.gamma, args.select_seed)
        epochs_norm = n_updates * frac
    else:
        epochs_norm = epochs

    def make_state(plan, F):
        st = bsgd.bsgd_state_create(plan, 1, vt,
                                    flags=bsgd.BSGD_STATE_BLOCK_SELECT if selected else 0)
        if F is not None:
            bsgd.bsgd_state_attach_fused(st, F)
        if args.method in ("ista", "gd"):
            bsgd.bsgd_state_set_method(st, bsgd.BSGD_METHOD_ISTA)
        bsgd.bsgd_state_set_overlap(st, args.overlap)
        if args.prox_schedule is not None:
            bsgd.bsgd_state_set_prox_schedule(st, args.prox_schedule)
        return st

    def run(st, mu):
        if selected:
            bsgd.bsgd_run_selected(st, mu, lam_run, rows_sel, cols_sel, K)
        else:
            bsgd.bsgd_run_epochs(st, mu, lam_run, epochs, K)

    fixed_mu = None
    if args.mu_file:
        with open(args.mu_file) as f:
            fixed_mu = float(json.load(f)["mu_f32"])

    def job(record):
        plan = bsgd.bsgd_plan_create(A, At, prob.M, prob.N, prob.row_off, prob.col_off, prob.H,
                                     prob.W, 1, prob.bins, flags)
        if tuned is not None:
            bsgd.bsgd_plan_set_lanes(plan, *tuned[0])
            bsgd.bsgd_plan_set_staged(plan, *[max(v, 0) for v in tuned[1]])
        F = None
        if fused:
            F = bsgd.bsgd_fused_create(plan, args.fused_chunks)
            bsgd.bsgd_fused_set_waves(F, args.fused_waves)
        if fixed_mu is None:
            if args.umax == "lanczos":
                # on the single-pass path the Lanczos products run on its store
                u = (bsgd.bsgd_lanczos_umax_fused(F, args.umax_steps, vt=vt) if F is not None
                     else bsgd.bsgd_lanczos_umax(plan, args.umax_steps, vt=vt))
            else:
                u = bsgd.bsgd_power_umax(plan, args.power_iters, vt=vt)
            mu = 0.9 / (2.0 * u)
        else:
            mu = fixed_mu
        st = make_state(plan, F)
        if args.autotune and fused:
            # the state's launch shapes (pass wavefronts, prox iterations per
            # launch) timed once, on the first job's state, and reused
            if "shape" not in launch:
                launch["shape"] = bsgd.bsgd_state_autotune(st, mu, lam_run, K, reps=5)
                print(f"[bench] autotuned launch (pass waves, prox split) {launch['shape']}",
                      file=sys.stderr, flush=True)
            bsgd.bsgd_state_set_launch(st, *launch["shape"])
        if record and timing:
            # one epoch in TIMING_STRIDE carries the events (each leaves the GPU
            # idle for microseconds between kernels)
            bsgd.bsgd_state_enable_timing(st, -(-n_updates // TIMING_STRIDE), TIMING_STRIDE)
        bsgd.bsgd_state_init(st, y)
        run(st, mu)
        x = bsgd.bsgd_get_x(st)
        if record and timing:
            f, b, p, n = bsgd.bsgd_state_timing(st)  # waits for this job's events
            acc["fwd"] += f
            acc["bwd"] += b
            acc["prox"] += p
            acc["n"] += n
        return st, x, mu, plan, F

    for w in range(args.warmup):
        # timed like the steps, so that the library's pool holds the timing
        # events before the timed region; these durations are discarded
        job(True)
        torch.cuda.synchronize()
        print(f"[bench] warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    acc.update(fwd=0.0, bwd=0.0, prox=0.0, n=0)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = None
    for k in range(args.steps):
        res = None  # the previous job's state goes first (its timing events return to the pool)
        res = job(True)
        print(f"[bench] step {k + 1}/{args.steps}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st, x, mu, plan, F = res
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = epochs_norm * args.steps / (t1 - t0)

    rn2, ep, _ = bsgd.bsgd_get_stats(st)
    xh = x.cpu().numpy().astype(np.float64)
    xt = prob.x_true.ravel()
    rel_err_true = float(np.linalg.norm(xh - xt) / np.linalg.norm(xt))

    # epoch-only rate (no setup), for context
    st2 = make_state(plan, F)
    bsgd.bsgd_state_init(st2, y)
    torch.cuda.synchronize()
    te = time.perf_counter()
    run(st2, mu)
    torch.cuda.synchronize()
    epoch_ms = (time.perf_counter() - te) * 1e3 / epochs_norm

    if args.dump and not selected:
        # untimed: the iterate every --dump-every epochs of one more job
        st3 = make_state(plan, F)
        bsgd.bsgd_state_init(st3, y)
        snaps = {}
        done = 0
        while done < epochs:
            n = min(args.dump_every, epochs - done)
            bsgd.bsgd_run_epochs(st3, mu, lam_run, n, K)
            done += n
            snaps[f"x{done}"] = bsgd.bsgd_get_x(st3).cpu().numpy()
        np.savez(args.dump, mu=np.float32(mu), **snaps)
        print(f"[bench] saved {sorted(snaps)} to {args.dump}", file=sys.stderr, flush=True)

    val_bytes = 2 if vt == bsgd.BSGD_VAL_F16 else 4
    b_fwd, b_bwd = _alg_bytes(nnz, r, c, val_bytes)
    staged_info = None
    if args.staged != "none":
        lanes = bsgd.bsgd_plan_staged(plan)
        staged_info = {"lanes": list(lanes)}
        for d, name in ((0, "fwd"), (1, "bwd")):
            if lanes[d] <= 0:
                continue
            P, SW, ent = bsgd.bsgd_plan_staged_shape(plan, d)
            nr, ncv = (r, c) if d == 0 else (c, r)
            # stored entries (2-byte columns), segment table, per-stage partials
            # written and read, the gathered vector once, the epilogue vectors
            b = (val_bytes + 2) * ent + 4 * ((nr + 2047) // 2048) * P * 2049 + 8 * P * nr \
                + 4 * ncv + 8 * nr
            staged_info[name] = {"stages": P, "stage_width": SW, "entries": ent, "alg_bytes": b}
            if d == 0:
                b_fwd = b
            else:
                b_bwd = b
    fused_info = None
    if F is not None:
        tiles, chunks, segs, slices, entries, cbytes = bsgd.bsgd_fused_shape(F)
        # matrix read once (columns, values; padding excluded), per-slot ray,
        # rank (and start address with 1-byte columns), per-slice count and
        # offset, x tile and r gathers once, per-segment partials and per-chunk
        # partials of A^T r written
        slot = 6 + (2 if cbytes == 1 else 0)
        b_pass = (val_bytes + cbytes) * nnz + slot * 64 * slices + 12 * slices + 4 * c + 4 * r \
            + 4 * segs + 4 * chunks * c
        # reduce: partials read, segment offsets, y, r' written, x read, x^ written;
        # with overlap modes 0/1 the timed reduce is the pixel half only (the ray
        # half runs concurrently with it and the prox on the state's second stream)
        if args.overlap == 2:
            b_red = 4 * segs + 4 * (r + 1) + 8 * r + 4 * chunks * c + 8 * c
        else:
            b_red = 4 * chunks * c + 8 * c
        b_fwd, b_bwd = b_pass, b_red
        if args.method in ("ista", "gd"):
            # two passes per epoch: A x only (timed as "fwd": matrix, slots, x tile,
            # segment partials) and A^T r only with the pixel half of the reduce
            # (timed as "bwd": matrix, slots, r gathers, chunk partials, then the
            # partials, x and x^)
            b_fwd = (val_bytes + cbytes) * nnz + slot * 64 * slices + 12 * slices + 4 * c \
                + 4 * segs
            b_bwd = (val_bytes + cbytes) * nnz + slot * 64 * slices + 12 * slices + 4 * r \
                + 4 * chunks * c + 4 * chunks * c + 8 * c
            b_pass, b_red = b_fwd, b_bwd
        fused_info = {"tiles": tiles, "chunks": chunks, "segments": segs, "slices": slices,
                      "stored_entries": entries, "padding": round(entries / nnz - 1, 4),
                      "column_bytes": cbytes,
                      "waves": args.fused_waves, "alg_bytes_pass": b_pass,
                      "alg_bytes_reduce": b_red}
    sel_info = None
    if selected:
        M, N = prob.M, prob.N
        tnnz = np.array([[bsgd.bsgd_tile_nnz(plan, i, j) for j in range(N)] for i in range(M)],
                        np.int64)
        rsz, csz = np.diff(prob.row_off), np.diff(prob.col_off)
        bf = bb = 0
        for rm_, cm_ in zip(rows_sel, cols_sel):
            I = [i for i in range(M) if (int(rm_) >> i) & 1]
            J = [j for j in range(N) if (int(cm_) >> j) & 1]
            ent = int(tnnz[np.ix_(I, J)].sum())
            nr_sel, nc_sel = int(rsz[I].sum()), int(csz[J].sum())
            # forward: drawn entries (value + column); per drawn ray its pointer, segment
            # bounds, block id, the N kept products (drawn ones written, others read), y and
            # r'; other rays: block id, r read and written; x of the drawn column blocks once
            bf += (val_bytes + 4) * ent + nr_sel * (8 + 4 * (N + 1) + 1 + 4 * N + 8) \
                + (r - nr_sel) * 9 + 4 * nc_sel
            # backward: drawn entries; per drawn pixel pointer, bounds, block id, x read, x^
            # written; other pixels: block id, x read, x^ written; r of the drawn rows once
            bb += (val_bytes + 4) * ent + nc_sel * (8 + 4 * (M + 1) + 1 + 8) \
                + (c - nc_sel) * 9 + 4 * nr_sel
        b_fwd, b_bwd = bf / n_updates, bb / n_updates
        sel_info = {"alpha": args.alpha, "gamma": args.gamma, "iterations": n_updates,
                    "normalised_epochs": round(epochs_norm, 3), "seed": args.select_seed,
                    "alg_bytes_fwd_avg": round(b_fwd), "alg_bytes_bwd_avg": round(b_bwd)}
    roofline = None
    kernel = {}
    if timing and acc["n"] and selected:
        f_ms = acc["fwd"] / acc["n"]
        b_ms = acc["bwd"] / acc["n"]
        p_ms = acc["prox"] / acc["n"]
        kernel = {"fwd_ms": f_ms, "bwd_ms": b_ms, "prox_ms": p_ms,
                  "fwd_gbs": b_fwd / f_ms / 1e6, "bwd_gbs": b_bwd / b_ms / 1e6}
        dom_bytes, dom_ms, dom = (b_fwd, f_ms, "fwd") if f_ms >= b_ms else (b_bwd, b_ms, "bwd")
        achieved = dom_bytes / dom_ms / 1e6
        traffic = None
        key = ("selected", args.config, args.vt, args.alpha, args.gamma, args.select_seed, dom)
        if key in PMC_TRAFFIC and _kernel_source_hash("selected") == PMC_TRAFFIC[key]["sha256"]:
            traffic = PMC_TRAFFIC[key]["bytes"]
        roofline = {"bound": "hbm",
                    "kernel": ("k_sel_forward (drawn pairs, forward projection, residual)" if dom == "fwd"
                               else "k_sel_backward (drawn pairs, backprojection, gradient sum and step)"),
                    "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "alg_bytes_per_launch": round(dom_bytes)}
    elif timing and acc["n"] and F is not None:
        f_ms = acc["fwd"] / acc["n"]
        b_ms = acc["bwd"] / acc["n"]
        p_ms = acc["prox"] / acc["n"]
        if args.method in ("ista", "gd"):
            kernel = {"pass_ax_ms": f_ms, "pass_atr_and_reduce_ms": b_ms, "prox_ms": p_ms,
                      "pass_ax_gbs": b_fwd / f_ms / 1e6, "pass_atr_gbs": b_bwd / b_ms / 1e6}
        else:
            kernel = {"pass_ms": f_ms, "reduce_ms": b_ms, "prox_ms": p_ms,
                      "pass_gbs": b_fwd / f_ms / 1e6, "reduce_gbs": b_bwd / b_ms / 1e6}
        achieved = b_fwd / f_ms / 1e6
        traffic = None
        key = ("fused", args.config, args.vt) if args.method == "bsgd" else \
            ("fused", args.config, args.vt, args.method)
        if key in PMC_TRAFFIC and _kernel_source_hash("fused") == PMC_TRAFFIC[key]["sha256"]:
            traffic = PMC_TRAFFIC[key]["bytes"]
        kdesc = ("k_fused (A x only: ISTA's forward pass)" if args.method in ("ista", "gd")
                 else "k_fused (A x and A^T r in one pass: both block products)")
        roofline = {"bound": "hbm", "kernel": kdesc,
                    "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "alg_bytes_per_launch": b_fwd}
    elif timing and acc["n"]:
        f_ms = acc["fwd"] / acc["n"]
        b_ms = acc["bwd"] / acc["n"]
        p_ms = acc["prox"] / acc["n"]
        kernel = {"fwd_ms": f_ms, "bwd_ms": b_ms, "prox_ms": p_ms,
                  "fwd_gbs": b_fwd / f_ms / 1e6, "bwd_gbs": b_bwd / b_ms / 1e6}
        dom_bytes, dom_ms, dom = (b_fwd, f_ms, "fwd") if f_ms >= b_ms else (b_bwd, b_ms, "bwd")
        achieved = dom_bytes / dom_ms / 1e6
        traffic = None
        key = ("rows", args.config, args.vt, args.staged, dom)
        if key in PMC_TRAFFIC and _kernel_source_hash("rows") == PMC_TRAFFIC[key]["sha256"]:
            traffic = PMC_TRAFFIC[key]["bytes"]
        kname = "k_staged" if staged_info and staged_info["lanes"][0 if dom == "fwd" else 1] > 0 \
            else "k_rows"
        roofline = {"bound": "hbm", "kernel": "%s (%s)" % (kname, "A x: forward projection, residual" if dom == "fwd"
                                                          else "A^T r: backprojection, gradient sum and step"),
                    "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "alg_bytes_per_launch": dom_bytes}

    cpu = pre_cpu
    if cpu is None and not args.no_cpu_baseline and args.cpu_epochs > 0:
        import oracle  # CPU baseline leg only
        rp64, col64, val64 = synth.projection_matrix(prob.H, prob.W, prob.n_ang, prob.bins)
        A64 = oracle.as_matrix(rp64, col64, val64, c)
        mu_cpu = 0.9 / (2.0 * oracle.power_umax(A64, tol=1e-6, max_iter=20))
        print(f"[bench] cpu baseline: {args.cpu_epochs} oracle epochs", file=sys.stderr, flush=True)
        shape = (prob.H, prob.W)
        cpu_epochs = float(args.cpu_epochs)
        if selected:
            blocks = oracle.tiles(rp64, col64, val64, prob.row_off, prob.col_off)
            n_cpu = max(1, int(math.ceil(args.cpu_epochs / frac - 1e-9)))
            st_c = oracle.selected_initial_state(blocks, prob.row_off, prob.col_off, prob.y)
            tc0 = time.perf_counter()
            oracle.bsgd_selected(blocks, prob.row_off, prob.col_off, prob.y, mu_cpu, lam_run, K,
                                 shape, rows_sel[:n_cpu], cols_sel[:n_cpu], state=st_c)
            cpu_epochs = n_cpu * frac
        elif args.method in ("ista", "gd"):
            tc0 = time.perf_counter()
            oracle.ista_tv(A64, prob.y, mu_cpu, lam_run, args.cpu_epochs, K, shape)
        else:
            xc, rc = oracle.initial_state(A64, prob.y)
            tc0 = time.perf_counter()
            xc, rc = oracle.bsgd_tv(A64, prob.y, mu_cpu, prob.lam, args.cpu_epochs, K, shape,
                                    state=(xc, rc))
        tcs = time.perf_counter() - tc0
        cpu = {"value": round(cpu_epochs / tcs, 4), "unit": "epochs/s", "cores": 1,
               "kind": "oracle",
               "sample": f"{cpu_epochs:g} epochs of {args.config} ({args.method}; FP64 "
                         f"numpy/scipy, single thread, setup excluded) in {tcs:.1f} s"}

    out = {
        "metric": "BSGD-TV epochs/s + HBM GB/s vs peak; served recon p50/p99 latency",
        "value": round(value, 2),
        "unit": "epochs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if vt == bsgd.BSGD_VAL_F32 else "f16-values/f32-accumulate",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: one reconstruction job per step ({prob.H}x{prob.W} "
                               f"image, {prob.n_ang} angles x {prob.bins} bins, M=N={prob.M}, "
                               f"lambda={lam_run}, {epochs} epochs, {K} FGP iterations, "
                               f"setup S0+S0' included)",
                   "method": args.method,
                   "nnz": nnz, "epochs_per_step": epochs,
                   "path": args.path,
                   "block_stores": _block_stores(flags),
                   "lanes_per_row": (None if flags & bsgd.BSGD_PLAN_SINGLE_PASS_ONLY
                                     else list(bsgd.bsgd_plan_lanes(plan))),
                   "overlap": args.overlap,
                   "staged": args.staged,
                   "launch": list(bsgd.bsgd_state_launch(st)),
                   "mu": "fixed from " + args.mu_file if fixed_mu is not None
                   else (f"Lanczos bidiagonalisation ({args.umax_steps} steps"
                         + (", products on the tile-sliced store)" if fused else ")")
                         if args.umax == "lanczos"
                         else f"power iteration ({args.power_iters} steps)")},
        "epoch_only_ms": round(epoch_ms, 4),
        "epoch_only_epochs_per_s": round(1e3 / epoch_ms, 2),
        "alg_bytes_per_epoch": b_fwd + b_bwd,
        "alg_gbs_epoch_only": round((b_fwd + b_bwd) / epoch_ms / 1e6, 1),
        "kernels": {k: round(v, 4) for k, v in kernel.items()},
        "staged": staged_info,
        "fused": fused_info,
        "selected": sel_info,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "quality": {"res_norm2": rn2, "rel_err_vs_phantom": round(rel_err_true, 5)},
    }
    print(json.dumps(out), flush=True)
    return 0


def run_volume(args, np, torch, synth, bsgd):
    """Batched volume: S slices of the 512 x 512 geometry share one A.

    One step = one whole job: plan (S0), power iteration (S0'), a state with
    S right-hand sides and the 3-D TV prox, then 200 epochs replayed as a HIP
    graph of two epochs.  The value is slice-epochs per second.
    """
    S = args.slices
    print(f"[bench] generating c4_vol with {S} slices", file=sys.stderr, flush=True)
    t_gen = time.perf_counter()
    prob = synth.make_volume_problem(S=S, dtype=np.float32)
    tp, tc, tv = prob.ensure_transpose()
    t_gen = time.perf_counter() - t_gen
    epochs = args.epochs or prob.epochs
    if epochs % 2 and not args.no_graph:
        epochs += 1  # the graph holds two epochs
    K = prob.prox_iters
    vt = bsgd.BSGD_VAL_F16 if args.vt == "f16" else bsgd.BSGD_VAL_F32
    flags = bsgd.BSGD_PLAN_F16 if vt == bsgd.BSGD_VAL_F16 else 0
    r, c, nnz = prob.nrows, prob.ncols, prob.nnz
    A = (r, c, bsgd.to_device(prob.row_ptr, torch.int64), bsgd.to_device(prob.col, torch.int32),
         bsgd.to_device(prob.val, torch.float32))
    At = (c, r, bsgd.to_device(tp, torch.int64), bsgd.to_device(tc, torch.int32),
          bsgd.to_device(tv, torch.float32))
    # [r][S]: slice index fastest
    Y = bsgd.to_device(np.ascontiguousarray(prob.y.T.astype(np.float32)), torch.float32)
    torch.cuda.synchronize()
    print(f"[bench] nnz={nnz} rows={r} cols={c} slices={S} gen={t_gen:.1f}s", file=sys.stderr,
          flush=True)
    timing = not args.no_kernel_timing
    acc = {"fwd": 0.0, "bwd": 0.0, "prox": 0.0, "n": 0}
    stream = torch.cuda.Stream()  # graph capture needs a non-default stream

    fused = args.path == "fused"
    shape = {}

    if fused:
        # the tile-sliced store serves both products and is built from A's CSR
        flags |= bsgd.BSGD_PLAN_FWD_ONLY | bsgd.BSGD_PLAN_SINGLE_PASS_ONLY

    def job(graph, n_epochs=epochs, timed=False):
        plan = bsgd.bsgd_plan_create(A, At, prob.M, prob.N, prob.row_off, prob.col_off, prob.H,
                                     prob.W, 1, prob.bins, flags)
        F = None
        if fused:
            # the single pass for several RHS reads the tile-sliced store; the
            # Lanczos products run on it too.  4 ray chunks: with 64 RHS columns
            # per unit there are workgroups enough, and fewer chunks mean fewer
            # A^T R partials to write and reduce (measured at 256 slices: 8.3 k
            # slice-epochs/s at 2 or 4 chunks, 7.7 k at 6 and 8, 6.5 k at 16)
            F = bsgd.bsgd_fused_create(plan, args.fused_chunks or VOLUME_CHUNKS)
            u = bsgd.bsgd_lanczos_umax_fused(F, args.umax_steps, vt=vt)
            shape["fused"] = bsgd.bsgd_fused_shape(F)
        else:
            u = bsgd.bsgd_power_umax(plan, args.power_iters, vt=vt)
        mu = 0.9 / (2.0 * u)
        st = bsgd.bsgd_state_create(plan, S, vt, flags=bsgd.BSGD_STATE_VOLUME)
        if F is not None:
            bsgd.bsgd_state_attach_fused(st, F)
        if args.autotune and "tuned" not in shape:
            # launch shapes timed once, outside the timed jobs, and reused
            shape["tuned"] = bsgd.bsgd_state_autotune(st, mu, prob.lam, K, reps=2)
            print(f"[bench] autotuned launch (pass waves, prox split) {shape['tuned']}",
                  file=sys.stderr, flush=True)
        if "tuned" in shape:
            bsgd.bsgd_state_set_launch(st, *shape["tuned"])
        elif args.mr_waves:
            bsgd.bsgd_state_set_launch(st, args.mr_waves, 0)
        if timed:
            bsgd.bsgd_state_enable_timing(st, n_epochs)
        bsgd.bsgd_state_init(st, Y)
        if graph:
            g = bsgd.bsgd_graph_create(st, mu, prob.lam, 2, K)
            for _ in range(n_epochs // 2):
                bsgd.bsgd_graph_launch(g)
        else:
            bsgd.bsgd_run_epochs(st, mu, prob.lam, n_epochs, K)
        x = bsgd.bsgd_get_x(st)
        if timed:
            f, b, p, n = bsgd.bsgd_state_timing(st)
            acc["fwd"] += f
            acc["bwd"] += b
            acc["prox"] += p
            acc["n"] += n
        return st, x, mu, plan

    graph = not args.no_graph
    with torch.cuda.stream(stream):
        for w in range(args.warmup):
            job(graph)
            torch.cuda.synchronize()
            print(f"[bench] warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            st, x, mu, plan = job(graph)
            torch.cuda.synchronize()
            print(f"[bench] step {k + 1}/{args.steps}", file=sys.stderr, flush=True)
        t1 = time.perf_counter()
        Xh = x.cpu().numpy().astype(np.float64).reshape(c, S).T
        if timing:
            # kernel timers are not captured into graphs: one eager job with events
            job(False, n_epochs=min(epochs, 20), timed=True)
            torch.cuda.synchronize()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = S * epochs * args.steps / (t1 - t0)
    rel = float(np.linalg.norm(Xh - prob.x_true.reshape(S, -1)) / np.linalg.norm(prob.x_true))

    val_bytes = 2 if vt == bsgd.BSGD_VAL_F16 else 4
    nvox = c * S
    # 3-D FGP in launches of up to 3 iterations (temporally blocked): per
    # launch b and two dual triples in, two triples out; the output kernel
    # reads b and one triple, writes x
    nlaunch = -(-K // 3)
    b_prox = (28 + 24) * nvox * nlaunch - 24 * nvox + 20 * nvox
    if fused:
        tiles, chunks, segs, slices, entries, cbytes = shape["fused"]
        # the pass: the stored entries once (value + column byte, padding not
        # counted), 8 B per segment slot and 12 B per slice of metadata; per
        # RHS, x once per chunk (each unit loads its tile), r once per segment,
        # the A x partial per segment and the A^T r partial per (chunk, pixel)
        b_fwd = ((val_bytes + cbytes) * nnz + 8 * slices * 64 + 12 * slices
                 + 4 * S * (chunks * c + segs + segs + chunks * c))
        # the reduce: partials in, y and x in, r' and x^ out
        b_bwd = 4 * S * (segs + chunks * c) + 4 * S * 2 * (r + c)
        names = {"fwd": "k_fused_mr (A X and A^T R in one pass)",
                 "bwd": "k_fz_reduce_mr (block sums and gradient step)", "prox": "k_fgp_tb3 (3-D FGP, K iterations)"}
    else:
        b_fwd = (val_bytes + 4) * nnz + 8 * (r + 1) + 4 * S * (c + 2 * r)
        b_bwd = (val_bytes + 4) * nnz + 8 * (c + 1) + 4 * S * (r + 2 * c)
        names = {"fwd": "k_spmm (A X)", "bwd": "k_spmm (A^T R)",
                 "prox": "k_fgp_tb3 (3-D FGP, K iterations)"}
    kernel, roofline = {}, None
    if timing and acc["n"]:
        f_ms, b_ms, p_ms = (acc[k] / acc["n"] for k in ("fwd", "bwd", "prox"))
        kernel = {"fwd_ms": f_ms, "bwd_ms": b_ms, "prox_ms": p_ms,
                  "fwd_gbs": b_fwd / f_ms / 1e6, "bwd_gbs": b_bwd / b_ms / 1e6,
                  "prox_gbs": b_prox / p_ms / 1e6}
        dom = max((("fwd", b_fwd, f_ms), ("bwd", b_bwd, b_ms), ("prox", b_prox, p_ms)),
                  key=lambda t: t[2])
        achieved = dom[1] / dom[2] / 1e6
        traffic = None
        key = ("fused_mr", args.config, args.vt, S, shape["fused"][1] if fused else 0, dom[0])
        if key in PMC_TRAFFIC and _kernel_source_hash("fused") == PMC_TRAFFIC[key]["sha256"]:
            traffic = PMC_TRAFFIC[key]["bytes"]
        roofline = {"bound": "hbm", "kernel": names[dom[0]],
                    "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "alg_bytes_per_launch": dom[1]}
    out = {
        "metric": "BSGD-TV epochs/s + HBM GB/s vs peak; served recon p50/p99 latency",
        "value": round(value, 1),
        "unit": "slice-epochs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if vt == bsgd.BSGD_VAL_F32 else "f16-values/f32-accumulate",
        "data": "synthetic",
        "config": {"workload": f"c4_vol: {S} slices of {prob.H}x{prob.W} sharing one A "
                               f"({prob.n_ang} angles x {prob.bins} bins, M=N={prob.M}), 3-D TV, "
                               f"lambda={prob.lam}, {epochs} epochs, {K} FGP iterations, "
                               f"setup S0+S0' included",
                   "nnz": nnz, "slices": S, "epochs_per_step": epochs,
                   "graph": graph, "path": args.path,
                   "block_stores": _block_stores(flags),
                   "launch": (list(shape["tuned"]) if "tuned" in shape
                              else [args.mr_waves, 0]),
                   "kernel_timing": "events on one eager 20-epoch job after the timed region"},
        "alg_bytes_per_epoch": b_fwd + b_bwd + b_prox,
        "kernels": {k: round(v, 4) for k, v in kernel.items()},
        "roofline": roofline,
        "cpu_baseline": None,
        "quality": {"rel_err_vs_phantoms": round(rel, 5)},
    }
    print(json.dumps(out), flush=True)
    return 0


C5_SIZES = (128, 256, 512, 768, 1024)
C5_ANGLES = (180, 360, 720, 1440)


def _c5_bins(n):
    """Smallest odd detector count covering the image diagonal (n sqrt 2)."""
    import math
    b = math.ceil(n * math.sqrt(2.0))
    return b if b % 2 else b + 1


def run_serve(args, np, torch, synth, bsgd):
    """Serving: a seeded Poisson stream of independent reconstructions over 20
    resident geometries, served with continuous batching and, for comparison,
    one request at a time on the one-RHS path.  Latency = completion - arrival.
    """
    from paper_1812_01307_amd.serve import DeviceBackend, Request, Server, percentile

    rng = np.random.default_rng(2024)
    nreq = args.requests
    gaps = rng.exponential(1.0 / args.rate, nreq)
    arrivals = np.cumsum(gaps) - gaps[0]
    geoms = [(n, a) for n in C5_SIZES for a in C5_ANGLES]
    pick = rng.integers(0, len(geoms), nreq)
    lams = rng.uniform(0.002, 0.02, nreq).astype(np.float32)
    be = DeviceBackend()
    resident = {}
    ys = {}
    total_nnz = 0
    t_gen = time.perf_counter()
    for gi, (n, ang) in enumerate(geoms):
        ks = [k for k in range(nreq) if pick[k] == gi]
        bins = _c5_bins(n)
        X = (np.stack([synth.ellipse_phantom(n, n, 10, 10**6 + k) for k in ks]) if ks
             else np.zeros((1, n * n)))
        rp, col, val, AX = synth.projection_matrix(n, n, ang, bins, dtype=np.float32, x=X)
        AX = AX.reshape(len(X), -1)
        tp, tc, tv = synth.transpose_csr(ang * bins, n * n, rp, col, val)
        row_off, col_off = synth.block_offsets(ang, bins, n * n, 8, 8)
        A = (ang * bins, n * n, bsgd.to_device(rp, torch.int64), bsgd.to_device(col, torch.int32),
             bsgd.to_device(val, torch.float32))
        At = (n * n, ang * bins, bsgd.to_device(tp, torch.int64),
              bsgd.to_device(tc, torch.int32), bsgd.to_device(tv, torch.float32))
        plan = bsgd.bsgd_plan_create(A, At, 8, 8, row_off, col_off, n, n, 1, bins, 0)
        geo = be.geometry(plan, power_iters=args.power_iters, prox_iters=20)
        torch.cuda.synchronize()
        del A, At
        total_nnz += len(col)
        for i, k in enumerate(ks):
            y = AX[i] + 0.01 * float(np.max(AX[i])) * \
                np.random.default_rng(2 * 10**6 + k).standard_normal(AX.shape[1])
            ys[k] = bsgd.to_device(y.astype(np.float32), torch.float32)
        resident[(n, ang)] = geo
        del rp, col, val, tp, tc, tv, AX, X
        print(f"[bench] geometry {gi + 1}/20: {n}^2, {ang} angles x {bins} bins, "
              f"{len(ks)} requests", file=sys.stderr, flush=True)
    t_gen = time.perf_counter() - t_gen
    plan_bytes = sum(g.plan.workspace.numel() for g in resident.values())
    print(f"[bench] geometries resident: {total_nnz} nnz, {plan_bytes / 1e9:.1f} GB, "
          f"setup {t_gen:.0f} s", file=sys.stderr, flush=True)

    def serve(slots, max_states, label):
        srv = Server(be, slots=slots, chunk=args.chunk, tol=1e-4, max_epochs=300,
                     max_states=max_states)
        for key, g in resident.items():
            srv.add_geometry(key, g)
        reqs = [Request(rid=k, geometry=geoms[pick[k]], y=ys[k], lam=float(lams[k]),
                        arrival=float(arrivals[k])) for k in range(nreq)]
        torch.cuda.synchronize()
        srv.t0 = srv.clock()
        last = [0]

        def progress():
            if len(srv.done) >= last[0] + max(1, nreq // 8):
                last[0] = len(srv.done)
                print(f"[bench] {label}: {len(srv.done)}/{nreq} done at {srv.now():.1f} s",
                      file=sys.stderr, flush=True)

        orig = srv.step

        def step():
            out = orig()
            progress()
            return out

        srv.step = step
        done = srv.run(reqs)
        torch.cuda.synchronize()
        span = max(r.finished for r in done) - min(r.arrival for r in done)
        lat = [r.latency for r in done]
        epochs = [r.epochs for r in done]
        return {"recon_per_s": round(len(done) / span, 3), "makespan_s": round(span, 3),
                "p50_s": round(percentile(lat, 50), 4), "p99_s": round(percentile(lat, 99), 4),
                "mean_epochs": round(float(np.mean(epochs)), 1),
                "converged": sum(r.stop == "converged" for r in done),
                "epochs_per_s": round(sum(epochs) / span, 1), "slots": slots,
                "rounds": srv.rounds}, {r.rid: r for r in done}

    batched, res_b = serve(args.slots, None, "batched")
    print(f"[bench] batched: {batched}", file=sys.stderr, flush=True)
    unbatched = None
    if not args.no_unbatched:
        unbatched, res_u = serve(1, 1, "unbatched")
        print(f"[bench] unbatched: {unbatched}", file=sys.stderr, flush=True)
        same_epochs = sum(res_b[k].epochs == res_u[k].epochs for k in res_b)
        diffs = [float(torch.linalg.norm(res_b[k].x - res_u[k].x) / torch.linalg.norm(res_u[k].x))
                 for k in res_b if res_b[k].epochs == res_u[k].epochs]
        unbatched["same_stop_epoch"] = same_epochs
        unbatched["max_rel_diff_vs_batched"] = max(diffs) if diffs else None
    out = {
        "metric": "BSGD-TV epochs/s + HBM GB/s vs peak; served recon p50/p99 latency",
        "value": batched["recon_per_s"],
        "unit": "reconstructions/s",
        "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(batched["makespan_s"] * 1e3, 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"c5_serve: {nreq} requests, Poisson {args.rate}/s, 20 geometries "
                               f"(n in {list(C5_SIZES)}, angles in {list(C5_ANGLES)}, M=N=8), "
                               f"lambda U[0.002, 0.02], stop |d||r|||/||r|| < 1e-4 or 300 "
                               f"epochs, checked every {args.chunk}, 20 FGP iterations",
                   "total_nnz": total_nnz, "resident_plan_bytes": plan_bytes},
        "p50_s": batched["p50_s"], "p99_s": batched["p99_s"],
        "batched": batched, "unbatched": unbatched,
        "speedup_vs_unbatched": (round(batched["recon_per_s"] / unbatched["recon_per_s"], 3)
                                 if unbatched else None),
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

#!/usr/bin/env python3
"""Throughput of the fused batched solve on one MI355X.

Workload (default): the chemistry-Jacobian stand-in batch -- 2^17 systems of
n = 54 sharing one random pattern (full diagonal + 35% off-diagonal fill, 1042
stored entries at seed 0), A = I - 1e-6 J with J = +-10^U(-3,3), b ~ U(-1,1),
x0 = 0 -- solved by FP64 BiCGSTAB with scalar Jacobi in BatchCsr to relative
residual 1e-10.  One step = one launch of the fused kernel over the whole batch,
inputs resident in HBM.  The line also reports the BatchEll and mixed-precision
forms of the same batch, the uneven batch (100k banded systems with n in
[16, 1024] in one persistent launch, eager and graph-replayed), the HBM
roofline of the solver kernel, and the CPU oracle's throughput on the host
cores.
"""
from __future__ import annotations

import argparse
import hashlib
import glob
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2308_08417_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(name: str):
    """HBM bytes per launch from committed rocprofv3 FETCH_SIZE/WRITE_SIZE runs,
    valid only for the kernel sources they were taken on."""
    path = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha") != kernel_source_sha():
        return None
    return t


def uneven_leg(args, bs, W, torch, np, dev, tol, max_iter):
    """Uneven batch in one persistent launch: ``args.uneven_batch`` banded
    nonsymmetric systems, n ~ U{16..1024}, band width ~ U{5..9}, BiCGSTAB +
    Jacobi to 1e-10, queue policy picked by the library's tuner, then timed as
    eager launches and as replays of the captured graph (FP64 and mixed)."""
    t0 = time.time()
    vb = W.uneven_banded(args.uneven_batch, 16, 1024, seed=0)
    gen_s = time.time() - t0
    h = bs.VarBatch(vb.pat_rows, vb.pat_rowptr_off, vb.rowptr_all, vb.pat_col_off, vb.col_all,
                    vb.pat_id)
    B = vb.n_batch
    vals = torch.from_numpy(vb.values).to(dev)
    b = torch.from_numpy(vb.b).to(dev)
    x = torch.empty_like(b)
    iters = torch.empty(B, dtype=torch.int32, device=dev)
    resid = torch.empty(B, dtype=torch.float64, device=dev)
    status = torch.empty(B, dtype=torch.int32, device=dev)
    out = {"workload": f"uneven_banded_b{B}_n16-1024_w5-9_bicgstab_jacobi",
           "n_batch": B, "total_rows": int(vb.b.size), "total_values": int(vb.values.size),
           "gen_seconds": gen_s}
    steps = max(3, args.steps // 4)
    for name, prec in (("fp64", bs.FP64), ("mixed", bs.MIXED)):
        opts = bs.make_options(flags=bs.FLAG_X0_ZERO, precision=prec)
        args_ = (h.handle, vals, b, x, bs.BICGSTAB, bs.PREC_JACOBI, tol, max_iter, iters, resid,
                 status, opts)
        report = bs.bs_varbatch_tune(*args_, reps=2)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            bs.bs_varbatch_solve(*args_)
        e1.record()
        torch.cuda.synchronize()
        eager_ms = e0.elapsed_time(e1) / steps
        bs.bs_varbatch_capture(*args_)
        bs.bs_varbatch_replay(h.handle)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            bs.bs_varbatch_replay(h.handle)
        e1.record()
        torch.cuda.synchronize()
        graph_ms = e0.elapsed_time(e1) / steps
        st, rs, it = status.cpu().numpy(), resid.cpu().numpy(), iters.cpu().numpy()
        # algorithmic bytes: every system's values, b and x once, the outputs,
        # and each distinct pattern once
        alg = (8 * vb.values.size + 16 * vb.b.size + 16 * B + 4 * vb.rowptr_all.size
               + 8 * vb.col_all.size)
        ms = min(eager_ms, graph_ms)
        out[name] = {"tune": report, "eager_ms": eager_ms, "graph_ms": graph_ms,
                     "systems_per_s": B / (ms * 1e-3),
                     "hbm_frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "algorithmic_bytes_per_launch": int(alg),
                     "all_converged": bool(np.all(st == bs.CONVERGED) and np.all(rs <= tol)),
                     "iters_mean": float(it.mean()), "iters_max": int(it.max()),
                     "max_resid": float(rs.max())}
    del vals, b, x
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=1 << 17)
    ap.add_argument("--fmt", choices=["csr", "ell"], default="csr")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="wall-clock budget of the CPU-oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="time only the headline form (for profiler runs)")
    ap.add_argument("--no-uneven", action="store_true",
                    help="skip the uneven-batch leg (100k systems, n in [16, 1024])")
    ap.add_argument("--uneven-batch", type=int, default=100_000)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run one device copy of this size (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the batched solve has no cross-GPU step; "
              "run it with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2308_08417_amd import batchsolve as bs
    from paper_2308_08417_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    bs.lib()

    t0 = time.time()
    bt = W.chem_jacobian(n_batch=args.batch, n=54, fill=0.35, gamma=1e-6, seed=0)
    gen_s = time.time() - t0
    B, n, nnz = bt.n_batch, bt.n, bt.nnz
    P = bs.Pattern.from_csr(bt.row_ptr, bt.col_idx)
    W_ell = P.ell_width
    vals_csr = torch.from_numpy(bt.values).to(dev)
    vals_ell = torch.empty((B, W_ell * n), dtype=torch.float64, device=dev)
    bs.bs_values_csr_to_ell(P.handle, vals_csr, vals_ell)
    b = torch.from_numpy(bt.b).to(dev)
    x = torch.empty_like(b)
    iters = torch.empty(B, dtype=torch.int32, device=dev)
    resid = torch.empty(B, dtype=torch.float64, device=dev)
    status = torch.empty(B, dtype=torch.int32, device=dev)
    tol, max_iter = 1e-10, 500
    torch.cuda.synchronize()

    def run(fmt, precision):
        v = vals_csr if fmt == bs.CSR else vals_ell
        opts = bs.make_options(flags=bs.FLAG_X0_ZERO, precision=precision)
        bs.bs_batch_solve(fmt, P.handle, v, b, x, bs.BICGSTAB, bs.PREC_JACOBI, tol, max_iter,
                          iters, resid, status, opts)

    def timed(fmt, precision, steps, warmup):
        for _ in range(warmup):
            run(fmt, precision)
        torch.cuda.synchronize()
        # the K launches run back to back on this stream between two events;
        # one launch is one step, so the average launch duration is region / K
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t_wall = time.perf_counter()
        e0.record()
        for _ in range(steps):
            run(fmt, precision)
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_wall
        total_ms = e0.elapsed_time(e1)
        st = status.cpu().numpy()
        rs = resid.cpu().numpy()
        it = iters.cpu().numpy()
        ok = bool(np.all(st == bs.CONVERGED) and np.all(rs <= tol))
        return {"kernel_ms": total_ms / steps, "ms_per_step": total_ms / steps,
                "wall_ms_per_step": 1e3 * wall / steps, "all_converged": ok,
                "iters_mean": float(it.mean()), "iters_max": int(it.max()),
                "max_resid": float(rs.max())}

    headline_fmt = bs.CSR if args.fmt == "csr" else bs.ELL
    head = timed(headline_fmt, bs.FP64, args.steps, args.warmup)

    variants = {}
    if not args.no_variants:
        for name, fmt, prec in (("ell_fp64", bs.ELL, bs.FP64), ("csr_fp64", bs.CSR, bs.FP64),
                                ("csr_mixed", bs.CSR, bs.MIXED), ("ell_mixed", bs.ELL, bs.MIXED)):
            if fmt == headline_fmt and prec == bs.FP64:
                continue
            r = timed(fmt, prec, max(5, args.steps // 2), 2)
            r["systems_per_s"] = B / (r["ms_per_step"] * 1e-3)
            variants[name] = r

    uneven = None
    if not args.no_uneven:
        uneven = uneven_leg(args, bs, W, torch, np, dev, tol, max_iter)

    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # algorithmic HBM bytes of one launch: each system's values, b and x once,
    # the three per-system outputs, and the shared pattern once
    stored = nnz if headline_fmt == bs.CSR else W_ell * n
    per_sys = 8 * stored + 8 * n + 8 * n + 4 + 8 + 4
    pattern_bytes = 4 * (n + 1) + 4 * W_ell * n + 4 * n + 4 * n
    alg_bytes = B * per_sys + pattern_bytes
    kernel_s = head["kernel_ms"] * 1e-3
    achieved = alg_bytes / kernel_s / 1e9
    wl = f"chem_jacobian_b{B}_n{n}_{args.fmt}_bicgstab_jacobi_fp64"
    tr = load_traffic(wl)
    traffic = None
    if tr is not None:
        traffic = tr["fetch_bytes_per_launch"] + tr["write_bytes_per_launch"]

    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O  # CPU baseline leg only: the oracle, timed as it stands
        OP = O.Pattern(n, bt.row_ptr, bt.col_idx)
        nt = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        ev = O.csr_values_to_ell(OP, bt.values) if headline_fmt == bs.ELL else bt.values
        ofmt = O.ELL if headline_fmt == bs.ELL else O.CSR
        done, t_cpu, reps = 0, 0.0, 0
        while reps == 0 or t_cpu < args.cpu_seconds:
            t1 = time.perf_counter()
            O.batch_solve(OP, ev, bt.b, fmt=ofmt, solver=O.BICGSTAB, precond=O.PREC_JACOBI,
                          tol=tol, max_iter=max_iter, nthreads=nt)
            t_cpu += time.perf_counter() - t1
            done += B
            reps += 1
        cpu = {"value": done / t_cpu, "unit": "systems/s", "cores": nt, "kind": "oracle",
               "sample": f"the full {B}-system batch solved {reps}x by the FP64 C oracle "
                         f"({t_cpu:.1f} s, OpenMP over systems)"}

    value = B / (head["ms_per_step"] * 1e-3)
    line = {
        "metric": "systems solved/sec at rel. residual 1e-10 (plain vs mixed+warm-start); % HBM",
        "value": value,
        "unit": "systems/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl, "n_batch": B, "n_rows": n, "nnz": nnz, "ell_width": W_ell,
                   "format": args.fmt, "solver": "bicgstab", "precond": "scalar_jacobi",
                   "tol": tol, "max_iter": max_iter, "x0": "zero", "seed": 0},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "kernel_ms": head["kernel_ms"]},
        "cpu_baseline": cpu,
        "check": {"all_converged": head["all_converged"], "iters_mean": head["iters_mean"],
                  "iters_max": head["iters_max"], "max_resid": head["max_resid"]},
        "variants": variants,
        "uneven": uneven,
        "gen_seconds": gen_s,
        "kernel_source_sha": kernel_source_sha(),
    }
    if traffic is not None:
        line["roofline"]["traffic_frac_of_alg"] = traffic / alg_bytes
    print(json.dumps(line))
    return 0 if head["all_converged"] else 3


if __name__ == "__main__":
    sys.exit(main())

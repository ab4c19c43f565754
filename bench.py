#!/usr/bin/env python3
"""Throughput benchmark of the MI355X sparse LU path (one JSON line on stdout).

A step is one pass of the hot path over one synthetic matrix already resident in
HBM: value scatter into the permuted block storage, numeric factorization of every
diagonal block (BTF blocks and nested-dissection nodes, one launch per ND level) and
a one-right-hand-side block back-substitution.  Workloads (see --workload):

  c2  batched BTF (default): 50,000 power-law MNA blocks (sizes 1..2,000) plus one
      100,000-node MNA block ordered by ND with 16 leaves, upper block-triangular
      coupling with 3 entries per row (n = 346,411)
  c0  one MNA circuit, n = 2,000
  c1  447 x 447 power-grid mesh with 2% long-range branches, ND with 16 leaves
  c3  MNA circuit n = 500,000; a step is a refactorization with new values + solve

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def make_workload(name):
    import synth
    if name == "c0":
        a = synth.gen_mna(2000)
        return a, dict(workload="mna_circuit_n2000", n=a.n, nnz=a.nnz), {}
    if name == "c1":
        a = synth.gen_power_grid(447)
        return a, dict(workload="power_grid_447x447_nd16", n=a.n, nnz=a.nnz), dict(nd_leaves=16)
    if name == "c2":
        inp = synth.gen_batched_btf()
        a = inp.a
        return a, dict(workload="batched_btf_50000_blocks_plus_100k_nd16", n=a.n, nnz=a.nnz,
                       small_blocks=int(len(inp.block_sizes) - 1), big_block=100000), dict(nd_leaves=16)
    if name == "c3":
        a = synth.gen_mna(500000)
        return a, dict(workload="mna_refactor_sequence_n500000", n=a.n, nnz=a.nnz), dict(nd_leaves=16)
    raise SystemExit("unknown workload %s" % name)


def cpu_baseline(a, order, budget_s, refactor_piv=None):
    """The oracle (serial C, one core) on the same matrix and ordering: factor + solve
    repeated until about budget_s seconds are spent."""
    import oracle
    import synth
    b = synth.rhs(a.n, 1)
    reps = 0
    t0 = time.perf_counter()
    while True:
        if refactor_piv is not None:
            f = oracle.refactor(a, order, refactor_piv)
        else:
            f = oracle.factor(a, order)
        oracle.solve(a, order, f, b)
        reps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or reps >= 1000:
            break
    return reps / el, reps, el


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=os.environ.get("BASKER_WORKLOAD", "c2"))
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle time for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the factorization of one matrix is not split across GPUs "
              "in this build (multi-GPU sharding is a design note); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1601_05725_amd as bk
    import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    bk.load()

    t = time.perf_counter()
    a, cfg, opts = make_workload(args.workload)
    log("workload %s n=%d nnz=%d generated in %.1fs" % (cfg["workload"], a.n, a.nnz, time.perf_counter() - t))
    t = time.perf_counter()
    h = bk.Handle.symbolic(a, bk.default_options(**opts))
    info = h.info()
    log("symbolic %.1fs: blocks=%d groups=%d nd_blocks=%d levels=%d crit_cols=%d" % (
        time.perf_counter() - t, info["nblocks"], info["ngroups"], info["nd_blocks"], info["nlevels"],
        info["crit_cols"]))

    refactor = args.workload == "c3"
    vals0 = torch.from_numpy(a.values.copy()).cuda()
    seq = []
    if refactor:
        for v in synth.value_sequence(a, max(1, args.steps + args.warmup)):
            seq.append(torch.from_numpy(v).cuda())
    b_host = synth.rhs(a.n, 1)[:, 0].copy()
    B = torch.from_numpy(b_host).cuda()
    Bwork = torch.empty_like(B)

    h.factor(vals0)          # first factorization (pattern, pivots, pool sizes)
    info = h.info()
    log("first factor: lnz=%d unz=%d kernel %.2f ms regrows=%d" % (info["lnz"], info["unz"],
                                                                     info["factor_kernel_ms"], info["pool_regrows"]))

    def step(i):
        if refactor:
            h.refactor(seq[i % len(seq)])
        else:
            h.factor(vals0)
        Bwork.copy_(B)
        h.solve(Bwork)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    lat = []
    fk, sk, sc = [], [], []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        step(args.warmup + i)
        lat.append(time.perf_counter() - ts)
        inf = h.info()
        fk.append(inf["factor_kernel_ms"])
        sk.append(inf["solve_kernel_ms"])
        sc.append(inf["scatter_kernel_ms"])
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    info = h.info()

    # correctness of the last step (not timed)
    x = Bwork.cpu().numpy()
    import scipy.sparse as sp
    if refactor:
        av = seq[(args.warmup + args.steps - 1) % len(seq)].cpu().numpy()
        A = sp.csc_matrix((av, a.rowind, a.colptr), shape=(a.n, a.n))
    else:
        A = a.to_scipy()
    r = A @ x - b_host
    resid = float(np.abs(r).max() / (abs(A).sum(axis=1).max() * np.abs(x).max() + np.abs(b_host).max()))

    nnzd, nnzo = info["nnz_diag"], info["nnz_offdiag"]
    lu = info["lnz"] + info["unz"]
    n = a.n
    # algorithmic bytes of one factorization (values + permuted pattern in, factors
    # with their row indices, column offsets and pivots out)
    bytes_factor = 12 * nnzd + 12 * lu + 12 * n
    fk_ms = float(np.mean(fk))
    achieved = bytes_factor / (fk_ms * 1e-3) / 1e9
    lat_ms = np.array(lat) * 1e3

    out = {
        "metric": "factorizations/s",
        "value": args.steps / total,
        "unit": "factorizations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": dict(cfg, tau=1e-3, step="refactor+solve" if refactor else "factor+solve", nrhs=1, nblocks=info["nblocks"], nd_blocks=info["nd_blocks"],
                       levels=info["nlevels"], crit_cols=info["crit_cols"], lnz=info["lnz"], unz=info["unz"]),
        "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)),
        "factor_kernel_ms": fk_ms,
        "solve_kernel_ms": float(np.mean(sk)),
        "scatter_kernel_ms": float(np.mean(sc)),
        "hbm_gbs_factor": achieved,
        "residual": resid,
        "roofline": {
            "kernel": "factor_kernel (sum of the per-level launches of one factorization)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "algorithmic_bytes": bytes_factor,
        },
    }
    if not args.no_cpu_baseline:
        import oracle
        prow, qcol, bp, gp = h.ordering()
        order = oracle.Ordering(prow, qcol, bp, gp)
        piv = h.extract().piv if refactor else None
        rate, reps, el = cpu_baseline(a, order, args.cpu_budget, refactor_piv=piv)
        out["cpu_baseline"] = {"value": rate, "unit": "factorizations/s", "cores": 1, "kind": "oracle",
                               "sample": "%d x (%s + solve) of the full workload, %.1f s, serial C oracle" % (
                                   reps, "refactor" if refactor else "factor", el)}
    h.free()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

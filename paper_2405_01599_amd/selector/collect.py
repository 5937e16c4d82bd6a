"""Measure the selector's training data on the GPU.

For every matrix of the selector set (four families: stencils, banded,
power-law rows, block-diagonal; n log-uniform in [1e4, 4e6]; half of the
stencils and banded matrices stored as symmetric lower triangles) record the
12 features and, for every valid class, the mean device time of 10 SpMVs
after 2 warm-ups (FP64, x = 1), the plan set-up time, and what the
exhaustive TIME policy itself picks and how long its selection takes.

  python -m paper_2405_01599_amd.selector.collect --set train --start 0 --stop 500 --out part0.npz
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SEEDS = {"train": 5, "heldout": 50005}


def measure(ctx, A, reps=10, warmup=2):
    import torch
    import paper_2405_01599_amd as xab
    K = xab.NCLASSES
    M = ctx.matrix_from_csr(A)
    feat, stats = ctx.features(M)
    x = torch.ones(A.ncols, dtype=torch.float64, device="cuda")
    y = torch.empty(A.n, dtype=torch.float64, device="cuda")
    cost = np.full(K, np.inf, dtype=np.float32)
    build = np.full(K, np.nan, dtype=np.float32)
    valid = np.zeros(K, dtype=np.uint8)
    for k in range(K):
        if k not in (xab.SYM_CLASSES if A.sym_lower else xab.GENERAL_CLASSES):
            continue
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            P = ctx.plan_class(M, k)
        except xab.XabError as e:
            if e.status == -6:
                continue
            raise
        build[k] = (time.perf_counter() - t0) * 1e3
        cost[k] = ctx.time_spmv(P, x, y, warmup=warmup, reps=reps)
        valid[k] = 1
        P.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P, info = ctx.select(M, xab.TIME)
    sel_wall = (time.perf_counter() - t0) * 1e3
    choice = int(info.chosen)
    P.close()
    M.close()
    return dict(feat=feat, stats=stats, cost=cost, build=build, valid=valid, time_choice=choice,
                time_select_ms=np.float32(info.select_ms), time_select_wall_ms=np.float32(sel_wall))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--set", choices=sorted(SEEDS), default="train")
    ap.add_argument("--start", type=int, default=0)
    ap.add_argument("--stop", type=int, default=2000)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    import torch
    import gen
    import paper_2405_01599_amd as xab
    ctx = xab.Context(0)
    seed = SEEDS[args.set]
    recs = []
    t_all = time.perf_counter()
    for idx in range(args.start, args.stop):
        A = gen.selector_matrix(idx, seed)
        r = measure(ctx, A)
        r.update(idx=idx, n=A.n, nnz=A.nnz, family=A.meta["family"], sym=int(A.sym_lower))
        recs.append(r)
        del A
        if idx % 10 == 0:
            torch.cuda.empty_cache()
        best = int(np.argmin(r["cost"]))
        print(f"[{args.set} {idx}] {r['family']:9s} n={r['n']} nnz={r['nnz']} best={best} "
              f"t={r['cost'][best] * 1e3:.1f}us time_choice={r['time_choice']} "
              f"elapsed={time.perf_counter() - t_all:.0f}s", flush=True)
    out = {k: np.stack([r[k] for r in recs]) for k in ("feat", "stats", "cost", "build", "valid", "time_choice",
                                                      "time_select_ms", "time_select_wall_ms", "idx", "n", "nnz",
                                                      "sym")}
    out["family"] = np.array([r["family"] for r in recs])
    out["seed"] = np.int64(seed)
    np.savez(args.out, **out)
    print("wrote", args.out, len(recs), flush=True)


if __name__ == "__main__":
    main()

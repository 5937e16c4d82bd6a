"""Train the learned SpMV selector on the GPU and score it.

Reads the timings collect.py measured (data/train.npz, data/heldout.npz),
trains the 12-64-64-K cost model with the library's own kernels
(xab_selector_train: masked MSE on log2(t_k / t_best), Adam, batch 128,
300 epochs, He-uniform start from the seeded fixture generator, one
seeded shuffle per epoch), writes model.bin, and scores the held-out set:

  regret(policy) = mean over matrices of t(chosen) / t(best) - 1

against the measured per-class times, for LEARNED, for the exhaustive TIME
policy's own pick and for STABLE (no tuning).

  python -m paper_2405_01599_amd.selector.train [--epochs 300] [--report out.json]
"""
import argparse
import json
import math
import os
import sys

import numpy as np

from . import DATA_DIR, MODEL_PATH

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

STABLE_GENERAL, STABLE_SYM = 3, 11


def load(name):
    d = np.load(os.path.join(DATA_DIR, f"{name}.npz"), allow_pickle=False)
    return {k: d[k] for k in d.files}


def he_init(K, seed=5, F=12, H=64):
    import gen
    shapes = [(H, F), (H,), (H, H), (H,), (K, H), (K,)]
    out = []
    for idx, s in enumerate(shapes):
        size = int(np.prod(s))
        if len(s) == 2:
            bound = math.sqrt(6.0 / s[1])
            out.append(gen.uniform_vec(size, seed * 16 + idx, -bound, bound))
        else:
            out.append(np.zeros(size))
    return np.concatenate(out).astype(np.float32)


def regret_of(choice, cost):
    best = np.min(np.where(np.isfinite(cost), cost, np.inf), axis=1)
    t = cost[np.arange(cost.shape[0]), choice]
    return t / best - 1.0


def evaluate(ctx, data):
    """Predicted choice per held-out matrix (argmin of the model over valid classes)."""
    import torch
    pred = ctx.selector_forward(torch.from_numpy(data["feat"].astype(np.float32)).cuda(), raw=True).cpu().numpy()
    pred = np.where(data["valid"] > 0, pred, np.inf)
    return np.argmin(pred, axis=1)


def summarize(r):
    return {"mean": float(np.mean(r)), "geomean_ratio_minus_1": float(np.exp(np.mean(np.log1p(r))) - 1),
            "max": float(np.max(r)), "p90": float(np.percentile(r, 90)), "exact_best_frac": float(np.mean(r == 0))}


def train_model(ctx, tr, epochs=300, batch=128, lr=1e-3):
    """Train the cost model on `ctx` from the He start; returns (losses, info)."""
    import torch
    import paper_2405_01599_amd as xab
    m = tr["feat"].shape[0]
    cost = np.where(tr["valid"] > 0, tr["cost"], 1.0).astype(np.float32)
    order = np.concatenate([np.random.default_rng(1000 + e).permutation(m) for e in range(epochs)])
    ctx.selector_set(he_init(xab.NCLASSES), np.zeros(12), np.ones(12))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return ctx.selector_train(dev(tr["feat"].astype(np.float32)), dev(cost), dev(tr["valid"].astype(np.uint8)),
                              order.astype(np.int32), epochs=epochs, batch=batch, lr=lr)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--batch", type=int, default=128)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--report", default=None)
    ap.add_argument("--no-save", action="store_true")
    args = ap.parse_args()
    import paper_2405_01599_amd as xab
    K = xab.NCLASSES
    tr, ho = load("train"), load("heldout")
    m = tr["feat"].shape[0]
    ctx = xab.Context(0)
    loss, info = train_model(ctx, tr, args.epochs, args.batch, args.lr)
    if not args.no_save:
        ctx.selector_save(MODEL_PATH)
    choice = evaluate(ctx, ho)
    hcost = np.where(ho["valid"] > 0, ho["cost"], np.inf)
    stable = np.where(ho["sym"] > 0, STABLE_SYM, STABLE_GENERAL)
    rep = {
        "train_matrices": int(m), "heldout_matrices": int(ho["feat"].shape[0]), "epochs": args.epochs,
        "final_loss": float(loss[-1]), "first_loss": float(loss[0]), "train_seconds": float(info.seconds),
        "regret_learned": summarize(regret_of(choice, hcost)),
        "regret_time_policy": summarize(regret_of(ho["time_choice"].astype(np.int64), hcost)),
        "regret_stable": summarize(regret_of(stable, hcost)),
        "time_policy_select_ms_mean": float(np.mean(ho["time_select_ms"])),
        "best_class_histogram": np.bincount(np.argmin(hcost, axis=1), minlength=K).tolist(),
        "learned_class_histogram": np.bincount(choice, minlength=K).tolist(),
    }
    print(json.dumps(rep, indent=1))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)


if __name__ == "__main__":
    main()

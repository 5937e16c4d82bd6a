"""The learned run-time selector shipped with the package (section 3.1's
before-execution judge with a learned cost model in place of exhaustive
timing): the model retrains bit for bit from the stored timings with the
library's own kernels, its held-out regret is within 10 % of the measured
best, and on fresh matrices it keeps the tuned speed while selecting far
faster than the exhaustive TIME policy and beating the untuned default once
the selection is amortised over repeated SpMVs.

The stored timings (selector/data) and the regret figures are GPU
measurements, so this file has no CPU counterpart; the MLP arithmetic itself
is checked against the oracle in test_gpu_selector.py.
"""
import time

import numpy as np
import pytest

import gen
import paper_2405_01599_amd as xab
from paper_2405_01599_amd.selector import MODEL_PATH
from paper_2405_01599_amd.selector import train as tr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    return xab.Context(0)


def test_shipped_model_retrains_bit_exact(ctx, tmp_path):
    c = xab.Context(0)
    loss, _ = tr.train_model(c, tr.load("train"))
    assert np.all(np.isfinite(loss)) and loss[-1] < 0.05 * loss[0]
    out = tmp_path / "m.bin"
    c.selector_save(out)
    assert out.read_bytes() == open(MODEL_PATH, "rb").read()


def test_heldout_regret_within_ten_percent(ctx):
    c = xab.Context(0)
    c.selector_load(MODEL_PATH)
    ho = tr.load("heldout")
    choice = tr.evaluate(c, ho)
    cost = np.where(ho["valid"] > 0, ho["cost"], np.inf)
    assert np.all(ho["valid"][np.arange(len(choice)), choice] == 1)
    r = tr.regret_of(choice, cost)
    stable = np.where(ho["sym"] > 0, tr.STABLE_SYM, tr.STABLE_GENERAL)
    r_stable = tr.regret_of(stable, cost)
    print(f"held-out regret: learned {r.mean():.4f} (max {r.max():.3f}), stable {r_stable.mean():.4f}")
    assert r.mean() <= 0.10
    assert r.mean() < r_stable.mean()


def _class_time(ctx, M, A, k, x, y):
    P = ctx.plan_class(M, k)
    t = ctx.time_spmv(P, x, y, warmup=3, reps=20)
    P.close()
    return t


def _select_wall(ctx, M, policy):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P, info = ctx.select(M, policy)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    k = int(info.chosen)
    P.close()
    return k, ms


def test_learned_gain_on_fresh_matrices(ctx):
    # one matrix of each family (seed outside the training and held-out sets)
    seed, reps = 777, 100
    tot = {"learned": 0.0, "time": 0.0, "stable": 0.0}
    spmv = {"learned": 0.0, "time": 0.0, "stable": 0.0}
    sel = {"learned": 0.0, "time": 0.0, "stable": 0.0}
    c = xab.Context(0)
    c.selector_load(MODEL_PATH)
    for idx in range(8):
        A = gen.selector_matrix(idx, seed)
        M = c.matrix_from_csr(A)
        x = torch.ones(A.ncols, dtype=torch.float64, device="cuda")
        y = torch.empty(A.n, dtype=torch.float64, device="cuda")
        _select_wall(c, M, xab.LEARNED)  # warm the code paths once
        kl, ms_l = _select_wall(c, M, xab.LEARNED)
        kt, ms_t = _select_wall(c, M, xab.TIME)
        ks, ms_s = _select_wall(c, M, xab.STABLE)
        assert ks == (tr.STABLE_SYM if A.sym_lower else tr.STABLE_GENERAL)
        t = {name: _class_time(c, M, A, k, x, y) for name, k in (("learned", kl), ("time", kt), ("stable", ks))}
        for name in spmv:
            spmv[name] += t[name]
        sel["learned"] += ms_l
        sel["time"] += ms_t
        sel["stable"] += ms_s
        tot["learned"] += ms_l + reps * t["learned"]
        tot["time"] += ms_t + reps * t["time"]
        tot["stable"] += ms_s + reps * t["stable"]
        print(f"{A.meta['family']:9s} n={A.n:8d} nnz={A.nnz:9d} learned {kl:2d} ({ms_l:6.2f} ms) "
              f"time {kt:2d} ({ms_t:6.2f} ms) stable {ks:2d}; us/SpMV {t['learned']*1e3:.1f} "
              f"{t['time']*1e3:.1f} {t['stable']*1e3:.1f}")
        M.close()
    print("selection (ms):", {k: round(v, 2) for k, v in sel.items()})
    print("selection + 100 SpMVs over 8 matrices (ms):", {k: round(v, 2) for k, v in tot.items()})
    # the learned choice runs within 10 % of the exhaustive pick
    assert spmv["learned"] <= 1.10 * spmv["time"]
    # selecting by the model is cheaper than building and timing every class
    assert sel["learned"] < sel["time"]
    # tuned beats untuned once selection is paid for over 100 SpMVs
    assert tot["learned"] < tot["stable"]

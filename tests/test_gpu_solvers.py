"""GPU checks of the Krylov drivers against the oracle and closed forms.

There is no bitwise parity for solvers (the GPU orthogonalises with CGS +
DGKS re-orthogonalisation, the oracle with MGS): the bar is the true
relative residual, the forward error against the oracle's solution, and
iteration counts close to the oracle's.
"""
import math

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
xab = pytest.importorskip("paper_2405_01599_amd")


@pytest.fixture(scope="module")
def ctx():
    return xab.Context(0)


def dev(a, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda().to(dt)


def _diag(d):
    n = d.size
    return gen.CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d.astype(np.float64))


def _setup(ctx, A, k=3, f32=True):
    M = ctx.matrix_from_csr(A, with_f32=f32)
    return M, ctx.plan_class(M, k)


def test_gmres_identity(ctx):
    A = _diag(np.ones(1000))
    M, P = _setup(ctx, A)
    b = gen.uniform_vec(1000, 3)
    x, info, st = ctx.gmres(P, dev(b), precond=xab.PRECOND_NONE, tol=1e-12)
    assert st == 0 and info["iters"] == 1
    assert np.allclose(x.cpu().numpy(), b, atol=1e-15, rtol=0)


@pytest.mark.parametrize("q", [1, 3, 7])
def test_gmres_diagonal_minimal_polynomial(ctx, q):
    n = 3000
    A = _diag(np.arange(1, q + 1, dtype=np.float64)[np.arange(n) % q])
    M, P = _setup(ctx, A)
    x, info, st = ctx.gmres(P, dev(np.ones(n)), precond=xab.PRECOND_NONE, tol=1e-12)
    assert st == 0 and info["iters"] <= q


def test_gmres_eigenvector_rhs(ctx):
    g = 64
    A = gen.laplacian2d(g)
    p = np.arange(g * g) % g
    q = np.arange(g * g) // g
    v = np.sin(3 * math.pi * (p + 1) / (g + 1)) * np.sin(5 * math.pi * (q + 1) / (g + 1))
    M, P = _setup(ctx, A)
    x, info, st = ctx.gmres(P, dev(v), precond=xab.PRECOND_NONE, tol=1e-10)
    lam = 4 - 2 * math.cos(3 * math.pi / (g + 1)) - 2 * math.cos(5 * math.pi / (g + 1))
    assert st == 0 and info["iters"] == 1
    assert np.allclose(x.cpu().numpy(), v / lam, atol=1e-12, rtol=0)


@pytest.mark.parametrize("k", [0, 3, 6])
@pytest.mark.parametrize("mode", [xab.MODE_FP64, xab.MODE_IR])
def test_gmres_powerlaw_vs_oracle(ctx, k, mode):
    A = gen.powerlaw(50_000, seed=2)
    b = np.ones(A.n)
    ref = oracle.gmres(A, b, m=30, tol=1e-10, precond=1)
    assert ref["status"] == 0
    M, P = _setup(ctx, A, k)
    x, info, st = ctx.gmres(P, dev(b), m=30, tol=1e-10, mode=mode, precond=xab.PRECOND_JACOBI)
    assert st == 0
    xs = x.cpu().numpy()
    # the true residual, recomputed by the oracle's own product
    r = b - oracle.spmv(A, xs)[0]
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10
    assert info["true_relres"] <= 1e-10
    # forward error: both residuals <= 1e-10 and the Jacobi-scaled matrix
    # is well conditioned (diagonal dominance 1.1)
    assert np.linalg.norm(xs - ref["x"]) / np.linalg.norm(ref["x"]) <= 1e-8
    if mode == xab.MODE_FP64:
        assert abs(info["iters"] - ref["iters"]) <= max(2, 0.2 * ref["iters"])
    else:
        assert info["refinements"] >= 1


@pytest.mark.parametrize("k", [9, 10, 11])
@pytest.mark.parametrize("mode", [xab.MODE_FP64, xab.MODE_IR])
def test_gmres_sym_stencil(ctx, k, mode):
    A = gen.stencil27(24, lower=True)
    b = np.ones(A.n)
    if k == 9 and mode == xab.MODE_IR:
        # the atomic baseline accumulates in its output type: it has no
        # FP32-out / FP64-accumulation form, and the library says so
        M, P = _setup(ctx, A, k)
        with pytest.raises(xab.XabError) as ei:
            ctx.gmres(P, dev(b), m=30, tol=1e-10, mode=mode, precond=xab.PRECOND_JACOBI)
        assert ei.value.status == -3
        return
    rp, ci, v = oracle.sym_expand(A)
    F = gen.CSR(A.n, A.n, rp, ci, v)
    ref = oracle.gmres(F, b, m=30, tol=1e-10, precond=1)
    M, P = _setup(ctx, A, k)
    x, info, st = ctx.gmres(P, dev(b), m=30, tol=1e-10, mode=mode, precond=xab.PRECOND_JACOBI)
    assert st == 0
    xs = x.cpu().numpy()
    r = b - oracle.spmv(F, xs)[0]
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10
    assert np.linalg.norm(xs - ref["x"]) / np.linalg.norm(ref["x"]) <= 1e-8


def test_gmres_status_codes(ctx):
    A = gen.stencil27(12, lower=False)
    M, P = _setup(ctx, A)
    b = dev(np.ones(A.n))
    _, info, st = ctx.gmres(P, b, maxiter=1, tol=1e-12)
    assert st == 1 and info["iters"] == 1 and info["status"] == 1
    _, info, st = ctx.gmres(P, b, tol=1e-14, max_time_s=1e-9, maxiter=10 ** 6)
    assert st in (0, 3)
    with pytest.raises(xab.XabError) as e:
        ctx.gmres(P, b, x=b)
    assert e.value.status == -5
    M64 = ctx.matrix_from_csr(A, with_f32=False)
    P64 = ctx.plan_class(M64, 3)
    with pytest.raises(xab.XabError) as e:
        ctx.gmres(P64, b, mode=xab.MODE_IR)
    assert e.value.status == -3


def test_gmres_resume_from_x(ctx):
    """x doubles as the initial guess: a converged x needs no further step."""
    A = gen.powerlaw(20_000, seed=2)
    M, P = _setup(ctx, A)
    b = dev(np.ones(A.n))
    x, info, st = ctx.gmres(P, b, tol=1e-10)
    assert st == 0
    x2, info2, st2 = ctx.gmres(P, b, x=x.clone(), tol=1e-10)
    assert st2 == 0 and info2["iters"] == 0


@pytest.mark.parametrize("mode", [xab.MODE_FP64, xab.MODE_IR])
def test_gmres_step_wait_drain_fallback(ctx, mode, monkeypatch):
    """The host waits for a step through the counter the step kernel writes
    to pinned memory and drains the stream when it has not arrived within
    XAB_STEP_WAIT_MS; at 0 every wait drains.  The queued kernels and their
    order are the same either way (steps queued past the stop touch neither
    the rotated system nor the basis vectors the update uses), so the solve
    is the same bit for bit."""
    A = gen.powerlaw(50_000, seed=2)
    M, P = _setup(ctx, A, 12)
    b = dev(np.ones(A.n))
    x0, i0, s0 = ctx.gmres(P, b, m=30, tol=1e-10, mode=mode, precond=xab.PRECOND_JACOBI)
    monkeypatch.setenv("XAB_STEP_WAIT_MS", "0")
    x1, i1, s1 = ctx.gmres(P, b, m=30, tol=1e-10, mode=mode, precond=xab.PRECOND_JACOBI)
    assert s0 == s1 == 0
    assert (i0["iters"], i0["restarts"], i0["refinements"]) == (i1["iters"], i1["restarts"], i1["refinements"])
    assert i0["true_relres"] == i1["true_relres"] <= 1e-10
    assert torch.equal(x0, x1)


# ----------------------------------------------------------------- batch
def _batch(nsys=12, nmin=300, nmax=3000):
    return gen.batch(nsys, seed=4, nmin=nmin, nmax=nmax)


@pytest.mark.parametrize("tiles", [False, True])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_spmv_integer_exact(ctx, tiles, dtype):
    """Both layouts (the sliced ELLPACK copy and the segmented-scan tiles),
    both precisions: small integers make every sum exact."""
    B = _batch()
    rng = np.random.default_rng(1)
    B.val = rng.integers(-8, 9, B.nnz).astype(np.float64)
    x = gen.int_vec(B.n, 3)
    bt = ctx.batch(B, dtype=dtype, tiles=tiles)
    assert bt.layout == ("tiles" if tiles else "sell")
    tdt = torch.float64 if dtype == "f64" else torch.float32
    y = bt.spmv(dev(x, tdt)).double().cpu().numpy()
    _batch_check_exact(B, x, y)


def _batch_check_exact(B, x, y):
    for k in range(B.nsys):
        S = B.system(k)
        r0, r1 = int(B.row_off[k]), int(B.row_off[k + 1])
        yo, _ = oracle.spmv(S, x[r0:r1])
        assert np.array_equal(y[r0:r1], yo)


def _long_row_batch():
    """Three systems: the first has a 5000-entry row (beyond the sliced copy's
    4096 limit) and an empty row, the second is empty, the third diagonal."""
    n0 = 6000
    rows = [list(range(5000))] + [[]] + [[i] for i in range(2, n0)] + [[n0 + i] for i in range(40)]
    rp = np.zeros(len(rows) + 1, dtype=np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.array([c for r in rows for c in r], dtype=np.int32)
    v = np.random.default_rng(5).integers(-8, 9, ci.size).astype(np.float64)
    row_off = np.array([0, n0, n0, n0 + 40])
    nnz_off = np.array([0, int(rp[n0]), int(rp[n0]), int(rp[-1])])
    return gen.Batch(3, row_off, nnz_off, rp, ci, v, np.zeros(3), np.zeros(3))


@pytest.mark.parametrize("tiles", [False, True])
def test_batch_single_system_matches_single_solve(ctx, tiles):
    """A batch of one system: SpMV exact, BiCGStab to 1e-10 like the oracle."""
    B = gen.batch(1, seed=4, nmin=2000, nmax=2001)
    x = gen.int_vec(B.n, 4)
    Bi = gen.Batch(B.nsys, B.row_off, B.nnz_off, B.rowptr, B.colind,
                   np.random.default_rng(2).integers(-8, 9, B.nnz).astype(np.float64), B.kinds, B.params)
    bt = ctx.batch(Bi, tiles=tiles)
    _batch_check_exact(Bi, x, bt.spmv(dev(x)).cpu().numpy())
    bt = ctx.batch(B, tiles=tiles)
    b = np.ones(B.n)
    xs, per, agg, st = ctx.bicgstab(bt, dev(b), tol=1e-10)
    assert st == 0 and per[0]["true_relres"] <= 1e-10 * 1.01
    ref = oracle.bicgstab(B.system(0), b, tol=1e-10, precond=1)
    assert np.linalg.norm(xs.cpu().numpy() - ref["x"]) / np.linalg.norm(ref["x"]) <= 1e-8


def test_batch_long_row_uses_tiles(ctx):
    B = _long_row_batch()
    x = gen.int_vec(B.n, 7)
    bt = ctx.batch(B)
    assert bt.layout == "tiles"
    _batch_check_exact(B, x, bt.spmv(dev(x)).cpu().numpy())


def test_batch_sell_empty_system_and_rows(ctx):
    """Empty systems and empty rows through the sliced copy."""
    rows = [[0, 2], [], [0, 1, 2]] + [[3 + i % 5] for i in range(5)]
    rp = np.zeros(len(rows) + 1, dtype=np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.array([c for r in rows for c in r], dtype=np.int32)
    v = np.arange(1, ci.size + 1, dtype=np.float64)
    B = gen.Batch(3, np.array([0, 3, 3, 8]), np.array([0, 5, 5, int(rp[-1])]), rp, ci, v, np.zeros(3), np.zeros(3))
    x = gen.int_vec(B.n, 2)
    bt = ctx.batch(B)
    assert bt.layout == "sell"
    _batch_check_exact(B, x, bt.spmv(dev(x)).cpu().numpy())


@pytest.mark.parametrize("tiles", [False, True])
@pytest.mark.parametrize("graph", [True, False])
def test_bicgstab_batch_fp64(ctx, graph, tiles):
    B = _batch()
    bt = ctx.batch(B, tiles=tiles)
    b = np.ones(B.n)
    x, per, agg, st = ctx.bicgstab(bt, dev(b), tol=1e-10, graph=graph, check_every=4)
    assert st == 0
    xs = x.cpu().numpy()
    for k in range(B.nsys):
        S = B.system(k)
        r0, r1 = int(B.row_off[k]), int(B.row_off[k + 1])
        ref = oracle.bicgstab(S, b[r0:r1], tol=1e-10, precond=1)
        assert ref["status"] == 0
        rr = b[r0:r1] - oracle.spmv(S, xs[r0:r1])[0]
        assert np.linalg.norm(rr) / np.linalg.norm(b[r0:r1]) <= 1e-10 * 1.01
        assert per[k]["status"] == 0 and per[k]["true_relres"] <= 1e-10 * 1.01
        assert np.linalg.norm(xs[r0:r1] - ref["x"]) / np.linalg.norm(ref["x"]) <= 1e-8
        assert abs(per[k]["iters"] - ref["iters"]) <= max(2, 0.25 * ref["iters"])


@pytest.mark.parametrize("tiles", [False, True])
def test_bicgstab_graph_equals_eager(ctx, tiles):
    B = _batch(8)
    bt = ctx.batch(B, tiles=tiles)
    b = dev(np.ones(B.n))
    x1, _, _, _ = ctx.bicgstab(bt, b, tol=1e-10, graph=True, check_every=4)
    x2, _, _, _ = ctx.bicgstab(bt, b, tol=1e-10, graph=False, check_every=4)
    assert torch.equal(x1, x2)


@pytest.mark.parametrize("tiles", [False, True])
def test_bicgstab_batch_fp32(ctx, tiles):
    B = _batch(10)
    bt = ctx.batch(B, dtype="f32", tiles=tiles)
    b = np.ones(B.n)
    x, per, agg, st = ctx.bicgstab(bt, dev(b, torch.float32), tol=1e-5, graph=True)
    assert st == 0
    xs = x.double().cpu().numpy()
    for k in range(B.nsys):
        S = B.system(k)
        r0, r1 = int(B.row_off[k]), int(B.row_off[k + 1])
        rr = b[r0:r1] - oracle.spmv(S, xs[r0:r1])[0]
        assert np.linalg.norm(rr) / np.linalg.norm(b[r0:r1]) <= 2e-5


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_bicgstab_large_systems_span_segments(ctx, dtype):
    """Systems of 6000-40000 rows (6-40 row segments each, ragged last
    segments) with an empty system between them: every per-system solution
    matches the oracle's, the empty system reports convergence at zero
    iterations and its (empty) slice leaves the others untouched."""
    B0 = gen.batch(5, seed=9, nmin=6000, nmax=40000)
    k0 = 2  # insert an empty system before system 2
    row_off = np.insert(B0.row_off, k0 + 1, B0.row_off[k0])
    nnz_off = np.insert(B0.nnz_off, k0 + 1, B0.nnz_off[k0])
    B = gen.Batch(B0.nsys + 1, row_off, nnz_off, B0.rowptr, B0.colind, B0.val, np.insert(B0.kinds, k0, 0),
                  np.insert(B0.params, k0, 0))
    tol = 1e-10 if dtype == "f64" else 1e-5
    tdt = torch.float64 if dtype == "f64" else torch.float32
    bt = ctx.batch(B, dtype=dtype)
    b = np.ones(B.n)
    x, per, agg, st = ctx.bicgstab(bt, dev(b, tdt), tol=tol, check_every=4)
    assert st == 0
    assert per[k0]["status"] == 0 and per[k0]["iters"] == 0
    xs = x.double().cpu().numpy()
    for k in range(B.nsys):
        r0, r1 = int(B.row_off[k]), int(B.row_off[k + 1])
        if r1 == r0:
            continue
        S = B.system(k)
        rr = b[r0:r1] - oracle.spmv(S, xs[r0:r1])[0]
        assert np.linalg.norm(rr) / np.linalg.norm(b[r0:r1]) <= (tol * 1.01 if dtype == "f64" else 2e-5)
        if dtype == "f64":
            ref = oracle.bicgstab(S, b[r0:r1], tol=tol, precond=1)
            assert ref["status"] == 0
            assert np.linalg.norm(xs[r0:r1] - ref["x"]) / np.linalg.norm(ref["x"]) <= 1e-8
            assert abs(per[k]["iters"] - ref["iters"]) <= max(2, 0.25 * ref["iters"])


def test_bicgstab_breakdown(ctx):
    """Rotation [[0,-1],[1,0]] as one system: <rhat, A p> = 0 at step one."""
    rp = np.array([0, 1, 2, 3, 4], dtype=np.int32)
    ci = np.array([1, 0, 2, 3], dtype=np.int32)
    v = np.array([-1.0, 1.0, 2.0, 2.0])
    B = gen.Batch(2, np.array([0, 2, 4]), np.array([0, 2, 4]), rp, ci, v, np.zeros(2), np.zeros(2))
    bt = ctx.batch(B)
    x, per, agg, st = ctx.bicgstab(bt, dev(np.array([0.3, -1.7, 1.0, 1.0])), tol=1e-12, precond=xab.PRECOND_NONE,
                                   graph=False, check_every=1)
    assert per[0]["status"] == 2 and per[1]["status"] == 0
    assert st == 2


def test_batch_rejects_cross_system_columns(ctx):
    rp = np.array([0, 1, 2], dtype=np.int32)
    ci = np.array([1, 1], dtype=np.int32)     # row 0 of system 0 points into system 1
    B = gen.Batch(2, np.array([0, 1, 2]), np.array([0, 1, 2]), rp, ci, np.ones(2), np.zeros(2), np.zeros(2))
    with pytest.raises(xab.XabError) as e:
        ctx.batch(B)
    assert e.value.status == -4


# ------------------------------------------------- restart-length tuning
def test_gmres_restart_tuning_vs_oracle(ctx):
    """GMRES(4) on the 64x64 Laplacian with the MM-ratio rule (threshold 10,
    step 4, m_max 40): the final restart length equals the oracle's, the
    iteration count is within 20 % of it and the true residual meets 1e-10."""
    A = gen.laplacian2d(64)
    b = np.ones(A.n)
    ref = oracle.gmres_at(A, b, 4, 40, 4, 10.0, tol=1e-10, maxiter=3000)
    assert ref["status"] == 0
    M = ctx.matrix_from_csr(A)
    P = ctx.plan_class(M, 5)
    x, inf, st = ctx.gmres(P, dev(b), m=4, tol=1e-10, maxiter=3000, precond=xab.PRECOND_NONE, restart_step=4,
                           m_max=40, mm_ratio=10.0)
    assert st == 0
    assert inf["m_final"] == ref["m_hist"][-1]
    assert abs(inf["iters"] - ref["iters"]) <= 0.2 * ref["iters"]
    xs = x.cpu().numpy()
    assert np.linalg.norm(b - oracle.spmv(A, xs)[0]) / np.linalg.norm(b) <= 1e-10


@pytest.mark.parametrize("mode", [0, 1])
def test_gmres_restart_tuning_extremes(ctx, mode):
    """Threshold infinity grows m by the step after every cycle (capped);
    threshold 0 never does."""
    A = gen.laplacian2d(20)
    b = np.ones(A.n)
    M = ctx.matrix_from_csr(A, with_f32=True)
    P = ctx.plan_class(M, 5)
    for thr in (math.inf, 0.0):
        x, inf, st = ctx.gmres(P, dev(b), m=3, tol=1e-10, maxiter=3000, mode=mode, precond=xab.PRECOND_NONE,
                               restart_step=5, m_max=17, mm_ratio=thr)
        assert st == 0
        want = min(3 + 5 * (inf["restarts"] - 1), 17) if thr == math.inf else 3
        assert inf["m_final"] == want


# ------------------------------------------------- orthogonalisation menu + accuracy policy
@pytest.mark.parametrize("ortho", [0, 1, 2, 3])
@pytest.mark.parametrize("mode", [0, 1])
def test_gmres_ortho_menu_vs_oracle(ctx, ortho, mode):
    """Every orthogonalisation converges to the true-residual target with an
    iteration count within 20 % of the oracle's run of the same method."""
    A = gen.laplacian2d(32)
    b = np.ones(A.n)
    ref = oracle.gmres_at(A, b, 30, 30, 0, 0.0, tol=1e-10, maxiter=1500, ortho=ortho)
    M = ctx.matrix_from_csr(A, with_f32=True)
    P = ctx.plan_class(M, 5)
    x, inf, st = ctx.gmres(P, dev(b), m=30, tol=1e-10, maxiter=1500, mode=mode, precond=xab.PRECOND_NONE,
                           ortho=ortho)
    assert st == 0 and inf["ortho"] == ortho
    xs = x.cpu().numpy()
    assert np.linalg.norm(b - oracle.spmv(A, xs)[0]) / np.linalg.norm(b) <= 1e-10
    if mode == 0:
        assert abs(inf["iters"] - ref["iters"]) <= 0.2 * ref["iters"]
        assert np.linalg.norm(xs - ref["x"]) <= 1e-8 * np.linalg.norm(ref["x"])


def test_gmres_accuracy_policy(ctx):
    """The policy picks MGS at 1e-10 and BCGS at 1e-8; at 1e-15 (below the
    attainable true residual) the recurrence keeps meeting narrowed
    thresholds the true residual misses: faults are counted and DGKS takes
    over, as in the oracle."""
    A = gen.laplacian2d(32)
    b = np.ones(A.n)
    M = ctx.matrix_from_csr(A)
    P = ctx.plan_class(M, 5)
    for tol, want in ((1e-10, xab.ORTHO_MGS), (1e-8, xab.ORTHO_BCGS)):
        x, inf, st = ctx.gmres(P, dev(b), m=30, tol=tol, maxiter=1500, precond=xab.PRECOND_NONE,
                               ortho=xab.ORTHO_POLICY)
        assert st == 0 and inf["faults"] == 0 and inf["ortho"] == want
    # mixed precision: the rule reads the inner solve's requirement (1e-6)
    M32 = ctx.matrix_from_csr(A, with_f32=True)
    x, inf, st = ctx.gmres(ctx.plan_class(M32, 5), dev(b), m=30, tol=1e-10, maxiter=1500, mode=xab.MODE_IR,
                           precond=xab.PRECOND_NONE, ortho=xab.ORTHO_POLICY)
    assert st == 0 and inf["ortho"] == xab.ORTHO_BCGS
    ref = oracle.gmres_at(A, b, 30, 30, 0, 0.0, tol=1e-15, maxiter=600, ortho=oracle.ORTHO_POLICY)
    x, inf, st = ctx.gmres(P, dev(b), m=30, tol=1e-15, maxiter=600, precond=xab.PRECOND_NONE,
                           ortho=xab.ORTHO_POLICY)
    assert st == 1 and ref["status"] == 1
    assert inf["faults"] >= 1 and ref["faults"] >= 1 and inf["ortho"] == xab.ORTHO_DGKS


def test_memory_policy_keeps_restart_length():
    """On a context whose policy is MEMORY the MM-ratio rule does not grow
    the basis: GMRES(4) on the 32x32 Laplacian with the rule of the tuning
    test above (which grows m to 28 and needs 240 steps) stays at m = 4 and
    takes about the oracle's fixed GMRES(4) count (1,256 steps)."""
    cm = xab.Context(0, policy=xab.MEMORY)
    A = gen.laplacian2d(32)
    b = np.ones(A.n)
    ref = oracle.gmres(A, b, m=4, tol=1e-10, maxiter=5000)
    assert ref["status"] == 0
    M = cm.matrix_from_csr(A)
    P = cm.plan_class(M, 5)
    x, inf, st = cm.gmres(P, dev(b), m=4, tol=1e-10, maxiter=5000, precond=xab.PRECOND_NONE, restart_step=4,
                          m_max=40, mm_ratio=10.0)
    assert st == 0 and inf["m_final"] == 4
    assert abs(inf["iters"] - ref["iters"]) <= 0.2 * ref["iters"]
    xs = x.cpu().numpy()
    assert np.linalg.norm(b - oracle.spmv(A, xs)[0]) / np.linalg.norm(b) <= 1e-10


def test_accuracy_policy_context(ctx):
    """On a context whose policy is ACCURACY, GMRES follows the accuracy
    policy whatever ortho asks: the same solution bit for bit, the same
    steps and the same method as an explicit ORTHO_POLICY solve on a TIME
    context (MGS at 1e-10; at 1e-15 faults and the switch to DGKS); the
    selector then chooses as TIME does."""
    ca = xab.Context(0, policy=xab.ACCURACY)
    A = gen.laplacian2d(32)
    b = np.ones(A.n)
    Pt = ctx.plan_class(ctx.matrix_from_csr(A), 5)
    Ma = ca.matrix_from_csr(A)
    Pa = ca.plan_class(Ma, 5)
    for tol, maxiter in ((1e-10, 1500), (1e-15, 600)):
        xt, it, st_t = ctx.gmres(Pt, dev(b), m=30, tol=tol, maxiter=maxiter, precond=xab.PRECOND_NONE,
                                 ortho=xab.ORTHO_POLICY)
        xa, ia, st_a = ca.gmres(Pa, dev(b), m=30, tol=tol, maxiter=maxiter, precond=xab.PRECOND_NONE,
                                ortho=xab.ORTHO_CGS)
        assert st_a == st_t and ia["iters"] == it["iters"] and ia["ortho"] == it["ortho"]
        assert ia["faults"] == it["faults"]
        assert torch.equal(xa, xt)
    P, info = ca.select(Ma, xab.ACCURACY)
    valid = [k for k in range(xab.NCLASSES) if info.valid[k]]
    assert all(info.time_ms[k] >= 0 for k in valid)
    assert info.chosen == min(valid, key=lambda k: (info.time_ms[k], k))


def test_bicgstab_accuracy_policy(ctx):
    """FP32 batched BiCGStab at 1e-7 on 64 systems: under TIME some systems
    stop on their recurrence residual while the true residual misses tol
    (the fault convergence of the accuracy policy's section).  On an
    ACCURACY context each such system runs again from its x with a tenfold
    narrower threshold, so a system that reports convergence meets tol with
    its true residual; the others report non-convergence.  Where TIME has no
    fault (FP64 at 1e-10) both contexts give the same solution bit for bit."""
    B = gen.batch(64, seed=4, nmin=1000, nmax=20000)
    b = np.ones(B.n)
    x, per, agg, st = ctx.bicgstab(ctx.batch(B, dtype="f32"), dev(b, torch.float32), tol=1e-7, maxiter=2000)
    faults = [k for k, p in enumerate(per) if p["status"] == 0 and p["true_relres"] > 1e-7]
    assert faults
    ca = xab.Context(0, policy=xab.ACCURACY)
    xa, pa, agga, sta = ca.bicgstab(ca.batch(B, dtype="f32"), dev(b, torch.float32), tol=1e-7, maxiter=2000)
    for k, p in enumerate(pa):
        assert p["status"] in (0, 1)
        if p["status"] == 0:
            assert p["true_relres"] <= 1e-7
    assert all(pa[k]["faults"] >= 1 for k in faults)
    xs = xa.double().cpu().numpy()
    for k, p in enumerate(pa):
        if p["status"] == 0:
            r0, r1 = int(B.row_off[k]), int(B.row_off[k + 1])
            rr = b[r0:r1] - oracle.spmv(B.system(k), xs[r0:r1])[0]
            assert np.linalg.norm(rr) / np.linalg.norm(b[r0:r1]) <= 5e-7
    Bs = _batch()
    bs = dev(np.ones(Bs.n))
    x1, p1, _, s1 = ctx.bicgstab(ctx.batch(Bs), bs, tol=1e-10)
    x2, p2, _, s2 = ca.bicgstab(ca.batch(Bs), bs, tol=1e-10)
    assert s1 == s2 == 0 and all(p["true_relres"] <= 1e-10 for p in p1)
    assert torch.equal(x1, x2) and all(p["faults"] == 0 for p in p2)


@pytest.mark.parametrize("maxiter", [40, 4000])
def test_bicgstab_accuracy_policy_unconfirmed(ctx, maxiter):
    """ACCURACY context, FP32 values and a tolerance FP32 cannot reach with
    its true residual (1e-10): the narrowed reruns run out (after 8
    narrowings, or at the iteration limit), and every system whose true
    residual misses tol reports non-convergence, as does the aggregate."""
    B = gen.batch(16, seed=4, nmin=1000, nmax=5000)
    b = np.ones(B.n)
    ca = xab.Context(0, policy=xab.ACCURACY)
    xa, pa, agg, st = ca.bicgstab(ca.batch(B, dtype="f32"), dev(b, torch.float32), tol=1e-10, maxiter=maxiter)
    missed = [k for k, p in enumerate(pa) if p["true_relres"] > 1e-10]
    assert missed
    for k, p in enumerate(pa):
        assert p["status"] in (0, 1, 2)
        if p["true_relres"] > 1e-10:
            assert p["status"] != 0
    assert st != 0 and agg["status"] == st
    if maxiter == 4000:
        assert any(pa[k]["faults"] == 8 for k in missed)

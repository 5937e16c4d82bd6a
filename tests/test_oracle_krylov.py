"""Pins for the oracle's GMRES(m) and BiCGStab (CPU only)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import gen
import oracle


def _diag(d):
    n = d.size
    return gen.CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d.astype(np.float64))


def _scipy(A):
    return sp.csr_matrix((A.val, A.colind, A.rowptr), shape=(A.n, A.ncols))


def test_gmres_identity_one_step():
    A = _diag(np.ones(100))
    b = gen.uniform_vec(100, 3)
    r = oracle.gmres(A, b, tol=1e-12)
    assert r["status"] == 0 and r["iters"] == 1
    assert np.allclose(r["x"], b, rtol=0, atol=1e-15)


@pytest.mark.parametrize("q", [1, 3, 7, 12])
def test_gmres_diagonal_minimal_polynomial(q):
    n = 120
    vals = np.arange(1, q + 1, dtype=np.float64)
    A = _diag(vals[np.arange(n) % q])
    b = np.ones(n)
    r = oracle.gmres(A, b, m=30, tol=1e-12)
    assert r["status"] == 0 and r["iters"] <= q


def test_gmres_eigenvector_rhs_one_step():
    g = 64
    A = gen.laplacian2d(g)
    p = np.arange(g * g) % g
    q = np.arange(g * g) // g
    v = np.sin(3 * math.pi * (p + 1) / (g + 1)) * np.sin(5 * math.pi * (q + 1) / (g + 1))
    r = oracle.gmres(A, v, m=30, tol=1e-10)
    assert r["status"] == 0 and r["iters"] == 1
    lam = 4 - 2 * math.cos(3 * math.pi / (g + 1)) - 2 * math.cos(5 * math.pi / (g + 1))
    assert np.allclose(r["x"], v / lam, rtol=0, atol=1e-12)


def test_gmres_arnoldi_relation_and_monotone():
    A = gen.powerlaw(3000, seed=2, mu=1.5)
    b = np.ones(A.n)
    r = oracle.gmres(A, b, m=30, tol=1e-10, history=True)
    assert r["status"] == 0
    assert r["arnoldi_err"] <= 1e-12
    h = r["hist"]
    # within the first cycle the recurrence residual never increases
    first = h[1:min(31, h.size)]
    assert np.all(np.diff(first) <= 1e-15)
    assert r["relres"] <= 1e-10


@pytest.mark.parametrize("precond", [0, 1])
def test_gmres_vs_direct_solve(precond):
    # unpreconditioned GMRES(30) stagnates on the badly scaled power-law rows,
    # so that case uses rows of uniform length
    A = gen.powerlaw(4000, seed=2) if precond else gen.random_uniform_rows(3000, 77, 5, 50)
    b = np.ones(A.n)
    r = oracle.gmres(A, b, m=30, tol=1e-12, precond=precond)
    assert r["status"] == 0 and r["relres"] <= 1e-12
    xs = spla.spsolve(_scipy(A).tocsc(), b)
    assert np.linalg.norm(r["x"] - xs) / np.linalg.norm(xs) <= 1e-10


def test_gmres_true_residual_restart_and_maxiter():
    A = gen.stencil27(8, lower=False)
    b = np.ones(A.n)
    r = oracle.gmres(A, b, m=5, tol=1e-10)
    assert r["status"] == 0 and r["cycles"] > 1
    res = b - _scipy(A) @ r["x"]
    assert np.linalg.norm(res) / np.linalg.norm(b) <= 1e-10
    r1 = oracle.gmres(A, b, m=30, tol=1e-10, maxiter=1)
    assert r1["status"] == 1 and r1["iters"] == 1


def test_bicgstab_identity_one_step():
    A = _diag(np.ones(50))
    b = gen.uniform_vec(50, 9)
    r = oracle.bicgstab(A, b, tol=1e-12)
    assert r["status"] == 0 and r["iters"] == 1
    assert np.allclose(r["x"], b, atol=1e-15, rtol=0)


@pytest.mark.parametrize("precond", [0, 1])
def test_bicgstab_vs_direct_solve(precond):
    A = gen.random_uniform_rows(3000, 77, 5, 50)
    b = np.ones(A.n)
    r = oracle.bicgstab(A, b, tol=1e-12, precond=precond)
    assert r["status"] == 0 and r["relres"] <= 1e-11
    xs = spla.spsolve(_scipy(A).tocsc(), b)
    assert np.linalg.norm(r["x"] - xs) / np.linalg.norm(xs) <= 1e-10


def test_bicgstab_rotation_breakdown():
    """A = [[0,-1],[1,0]]: <rhat, A p> = 0 at the first step for any b."""
    A = gen.CSR(2, 2, np.array([0, 1, 2], dtype=np.int32), np.array([1, 0], dtype=np.int32), np.array([-1.0, 1.0]))
    r = oracle.bicgstab(A, np.array([0.3, -1.7]), tol=1e-12)
    assert r["status"] == 2


def test_gmres_banded_batch_system():
    n, kind, h = gen.batch_params(4, seed=4, nmin=1000, nmax=4000)
    for k in range(4):
        A = gen.batch_system(k, int(n[k]), int(kind[k]), int(h[k]))
        r = oracle.gmres(A, np.ones(A.n), tol=1e-10, precond=1)
        assert r["status"] == 0 and r["relres"] <= 1e-10


# ------------------------------------------------- restart-length tuning (eq. (1))
def test_mm_ratio_closed_forms():
    """R(s, t) of eq. (1): geometric decay q^z gives q^-(t-1); a constant
    sequence gives 1; the window is z = s-t+1 .. s."""
    q = 0.5
    r = q ** np.arange(1, 21)
    for s, t in [(20, 20), (10, 4), (5, 1), (7, 7)]:
        assert math.isclose(oracle.mm_ratio(r, s, t), q ** -(t - 1), rel_tol=1e-15)
    assert oracle.mm_ratio(np.full(9, 3.7), 9, 9) == 1.0
    r = np.array([5.0, 1.0, 4.0, 2.0, 8.0])
    assert oracle.mm_ratio(r, 4, 3) == 4.0      # [1, 4, 2]
    assert oracle.mm_ratio(r, 5, 2) == 4.0      # [2, 8]
    assert oracle.mm_ratio(r, 5, 5) == 8.0      # [5, 1, 4, 2, 8]
    rng = np.random.default_rng(3)
    for _ in range(50):
        v = rng.uniform(0.1, 10.0, 30)
        s = int(rng.integers(1, 31))
        t = int(rng.integers(1, s + 1))
        w = v[s - t:s]
        assert oracle.mm_ratio(v, s, t) == w.max() / w.min()


def test_gmres_at_without_tuning_is_plain_gmres():
    A = gen.random_uniform_rows(3000, 7, 5, 30)
    b = np.ones(A.n)
    a = oracle.gmres(A, b, m=8, tol=1e-10, maxiter=2000)
    t = oracle.gmres_at(A, b, 8, 8, 0, 10.0, tol=1e-10, maxiter=2000)
    assert np.array_equal(a["x"], t["x"]) and a["iters"] == t["iters"]
    assert t["m_hist"] == [8] * t["cycles"]


@pytest.mark.parametrize("m0,step,mmax", [(4, 4, 40), (3, 5, 17), (10, 10, 63)])
def test_gmres_at_rule_extremes(m0, step, mmax):
    """Threshold 0: never stagnant, m stays; threshold infinity: every cycle
    is stagnant, so m grows by `step` per cycle up to m_max."""
    A = gen.laplacian2d(40)
    b = np.ones(A.n)
    never = oracle.gmres_at(A, b, m0, mmax, step, 0.0, tol=1e-10, maxiter=400)
    assert never["m_hist"] == [m0] * never["cycles"]
    always = oracle.gmres_at(A, b, m0, mmax, step, math.inf, tol=1e-10, maxiter=400)
    want = [min(m0 + step * c, mmax) for c in range(always["cycles"])]
    assert always["m_hist"] == want


def test_gmres_at_cures_stagnation():
    """GMRES(4) on the 64x64 Laplacian stalls within 3000 steps; growing m
    when a cycle's MM ratio is below 10 converges, and reaches the true
    residual target."""
    A = gen.laplacian2d(64)
    b = np.ones(A.n)
    fixed = oracle.gmres(A, b, m=4, tol=1e-10, maxiter=3000)
    tuned = oracle.gmres_at(A, b, 4, 40, 4, 10.0, tol=1e-10, maxiter=3000)
    assert fixed["status"] == 1 and tuned["status"] == 0
    assert np.linalg.norm(b - oracle.spmv(A, tuned["x"])[0]) / np.linalg.norm(b) <= 1e-10
    mh = tuned["m_hist"]
    assert mh[0] == 4 and all(y - x in (0, 4) for x, y in zip(mh, mh[1:])) and max(mh) <= 40


# ------------------------------------------------- orthogonalisation menu + accuracy policy
ORTHOS = [oracle.ORTHO_DGKS, oracle.ORTHO_CGS, oracle.ORTHO_MGS, oracle.ORTHO_BCGS]


def test_ortho_variants_agree_when_well_conditioned():
    """DGKS, CGS, MGS and BCGS build the same Arnoldi decomposition in exact
    arithmetic: on a well-conditioned problem they take the same steps, reach
    the same solution and satisfy the Arnoldi relation to rounding."""
    A = gen.laplacian2d(32)
    b = np.ones(A.n)
    outs = [oracle.gmres_at(A, b, 30, 30, 0, 0.0, tol=1e-10, maxiter=1500, ortho=o, history=True) for o in ORTHOS]
    ref = outs[2]  # MGS
    for o, r in zip(ORTHOS, outs):
        assert r["status"] == 0 and r["iters"] == ref["iters"], o
        assert np.linalg.norm(r["x"] - ref["x"]) <= 1e-9 * np.linalg.norm(ref["x"]), o
        assert r["arnoldi_err"] <= 1e-14, o


def test_bcgs_within_one_block_is_cgs():
    """With m <= 4 every BCGS step is a single block: bit for bit CGS."""
    A = gen.random_uniform_rows(2000, 9, 5, 30)
    b = np.ones(A.n)
    c = oracle.gmres_at(A, b, 4, 4, 0, 0.0, tol=1e-10, maxiter=800, ortho=oracle.ORTHO_CGS)
    k = oracle.gmres_at(A, b, 4, 4, 0, 0.0, tol=1e-10, maxiter=800, ortho=oracle.ORTHO_BCGS)
    assert np.array_equal(c["x"], k["x"]) and c["iters"] == k["iters"]


def test_accuracy_policy_rule():
    """MGS for requirements of 1e-10 or tighter, BCGS otherwise; a fault
    convergence (recurrence met, true residual missed) switches to DGKS and
    narrows the recurrence threshold.  On the 32x32 Laplacian the true
    residual cannot go much below 1e-14, so 1e-14 converges after a fault
    and 1e-15 keeps faulting until the step limit."""
    A = gen.laplacian2d(32)
    b = np.ones(A.n)
    P = oracle.ORTHO_POLICY
    r = oracle.gmres_at(A, b, 30, 30, 0, 0.0, tol=1e-10, maxiter=1500, ortho=P)
    assert (r["status"], r["faults"], r["ortho"]) == (0, 0, oracle.ORTHO_MGS)
    r = oracle.gmres_at(A, b, 30, 30, 0, 0.0, tol=1e-8, maxiter=1500, ortho=P)
    assert (r["status"], r["faults"], r["ortho"]) == (0, 0, oracle.ORTHO_BCGS)
    r = oracle.gmres_at(A, b, 30, 30, 0, 0.0, tol=1e-14, maxiter=1500, ortho=P)
    assert r["status"] == 0 and r["faults"] >= 1 and r["ortho"] == oracle.ORTHO_DGKS
    r = oracle.gmres_at(A, b, 30, 30, 0, 0.0, tol=1e-15, maxiter=1500, ortho=P)
    assert r["status"] == 1 and r["faults"] >= 2 and r["ortho"] == oracle.ORTHO_DGKS

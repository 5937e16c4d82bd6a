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

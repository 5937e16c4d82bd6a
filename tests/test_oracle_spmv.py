"""Pins for the oracle's SpMV and symmetric SpMV (CPU only).

Each pin fixes the oracle to something other than itself: a dense matvec
(library routine) on tiny matrices, exact integer arithmetic, closed forms of
the stencil matrices (A*1 and eigenpairs), and the full-storage generator.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import gen
import oracle


def _dense(A):
    D = np.zeros((A.n, A.ncols))
    for i in range(A.n):
        for k in range(A.rowptr[i], A.rowptr[i + 1]):
            D[i, A.colind[k]] += A.val[k]
    return D


def _tiny(n, ncols, rng, lens, intvals=False):
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum(lens)
    ci, v = [], []
    for i in range(n):
        cols = np.sort(rng.choice(ncols, size=lens[i], replace=False)) if lens[i] else np.array([], int)
        ci.extend(cols.tolist())
        if intvals:
            v.extend(rng.integers(-8, 9, size=lens[i]).astype(float).tolist())
        else:
            v.extend(rng.standard_normal(lens[i]).tolist())
    return gen.CSR(n, ncols, rp, np.array(ci, dtype=np.int32), np.array(v, dtype=np.float64))


TINY_CASES = {
    "random": lambda rng: _tiny(40, 40, rng, rng.integers(0, 12, 40)),
    "empty_rows": lambda rng: _tiny(30, 30, rng, np.array([0, 3, 0, 0, 5] * 6)),
    "n1": lambda rng: _tiny(1, 1, rng, np.array([1])),
    "n1_empty": lambda rng: _tiny(1, 1, rng, np.array([0])),
    "dense_row": lambda rng: _tiny(20, 64, rng, np.array([64] + [2] * 19)),
    "all_zero": lambda rng: _tiny(16, 16, rng, np.zeros(16, dtype=int)),
    "rect": lambda rng: _tiny(10, 50, rng, rng.integers(0, 30, 10)),
}


@pytest.mark.parametrize("case", sorted(TINY_CASES))
def test_spmv_vs_dense(case):
    rng = np.random.default_rng(7)
    A = TINY_CASES[case](rng)
    x = rng.uniform(-1, 1, A.ncols)
    y, s = oracle.spmv(A, x)
    D = _dense(A)
    ref = D @ x
    # numpy's own rounding (<= ncols * u * s) dominates the tolerance
    assert np.all(np.abs(y - ref) <= 64 * 2.3e-16 * s + 0.0)
    assert np.allclose(s, np.abs(D) @ np.abs(x), rtol=1e-14, atol=0)
    empty = np.diff(A.rowptr) == 0
    assert np.all(y[empty] == 0.0)


def test_spmv_detects_transpose():
    """A plausible bug (A^T x instead of A x) would be caught by the dense pin."""
    rng = np.random.default_rng(3)
    A = _tiny(20, 20, rng, rng.integers(1, 8, 20))
    x = rng.uniform(-1, 1, 20)
    y, _ = oracle.spmv(A, x)
    D = _dense(A)
    assert not np.allclose(y, D.T @ x)


def test_integer_exact_powerlaw():
    """Integer values in [-8, 8]: every partial sum is exact, so any summation
    order gives the same bits; scipy's int64 product is the reference."""
    A = gen.powerlaw(20_000, seed=2)
    rng = np.random.default_rng(1)
    A.val = rng.integers(-8, 9, A.nnz).astype(np.float64)
    x = gen.int_vec(A.n, 11)
    y, _ = oracle.spmv(A, x)
    M = sp.csr_matrix((A.val.astype(np.int64), A.colind, A.rowptr), shape=(A.n, A.n))
    ref = M @ x.astype(np.int64)
    assert np.array_equal(y, ref.astype(np.float64))


def test_dot2_beats_naive():
    """Compensated row sums: a cancelling row is exact where naive summation is not."""
    rp = np.array([0, 4], dtype=np.int32)
    ci = np.array([0, 1, 2, 3], dtype=np.int32)
    v = np.array([1e16, 1.0, -1e16, 1.0])
    A = gen.CSR(1, 4, rp, ci, v)
    y, s = oracle.spmv(A, np.ones(4))
    assert y[0] == 2.0
    assert s[0] == 2e16 + 2.0


def _ones_stencil_closed_form_2d(g):
    i = np.arange(g * g)
    x, y = i % g, i // g
    nb = (x > 0).astype(int) + (x < g - 1) + (y > 0) + (y < g - 1)
    return 4.0 - nb


def _ones_stencil_closed_form_27(g):
    i = np.arange(g ** 3)
    x, y, z = i % g, (i // g) % g, i // (g * g)
    cnt = lambda c: 3 - (c == 0).astype(int) - (c == g - 1)
    return 27.0 - (cnt(x) * cnt(y) * cnt(z) - 1)


@pytest.mark.parametrize("lower", [False, True])
def test_laplacian_times_ones(lower):
    A = gen.laplacian2d(64, lower=lower)
    y, _ = oracle.spmv(A, np.ones(A.n))
    ref = _ones_stencil_closed_form_2d(64)
    assert np.array_equal(y, ref)
    # interior 0, edges 1, corners 2
    assert sorted(set(y.tolist())) == [0.0, 1.0, 2.0]


@pytest.mark.parametrize("g,lower", [(9, True), (9, False), (20, True)])
def test_stencil27_times_ones(g, lower):
    A = gen.stencil27(g, lower=lower)
    y, _ = oracle.spmv(A, np.ones(A.n))
    assert np.array_equal(y, _ones_stencil_closed_form_27(g))
    assert sorted(set(y.tolist())) == [1.0, 10.0, 16.0, 20.0]


@pytest.mark.parametrize("j,k", [(1, 1), (3, 7), (64, 2), (31, 33)])
def test_laplacian_eigenpairs(j, k):
    g = 64
    A = gen.laplacian2d(g)
    p = np.arange(g * g) % g
    q = np.arange(g * g) // g
    v = np.sin(j * math.pi * (p + 1) / (g + 1)) * np.sin(k * math.pi * (q + 1) / (g + 1))
    lam = 4 - 2 * math.cos(j * math.pi / (g + 1)) - 2 * math.cos(k * math.pi / (g + 1))
    y, _ = oracle.spmv(A, v)
    assert np.max(np.abs(y - lam * v)) <= 1e-13


@pytest.mark.parametrize("ks", [(1, 1, 1), (2, 5, 7), (8, 1, 3)])
def test_stencil27_eigenpairs_lower(ks):
    g = 12
    A = gen.stencil27(g, lower=True)
    i = np.arange(g ** 3)
    c = [i % g, (i // g) % g, i // (g * g)]
    v = np.ones(g ** 3)
    lam_prod = 1.0
    for d in range(3):
        v *= np.sin(math.pi * ks[d] * (c[d] + 1) / (g + 1))
        lam_prod *= 1 + 2 * math.cos(ks[d] * math.pi / (g + 1))
    lam = 28 - lam_prod
    y, _ = oracle.spmv(A, v)
    assert np.max(np.abs(y - lam * v)) <= 1e-12


@pytest.mark.parametrize("g", [5, 16])
def test_sym_expand_equals_full_generator(g):
    L = gen.stencil27(g, lower=True)
    F = gen.stencil27(g, lower=False)
    rp, ci, v = oracle.sym_expand(L)
    assert np.array_equal(rp, F.rowptr)
    assert np.array_equal(ci, F.colind)
    assert np.array_equal(v, F.val)
    ndiag = L.n
    assert F.nnz == 2 * L.nnz - ndiag


def test_sym_lower_equals_full_spmv():
    L = gen.laplacian2d(64, lower=True)
    F = gen.laplacian2d(64, lower=False)
    x = gen.uniform_vec(L.n, 1)
    yl, sl = oracle.spmv(L, x)
    yf, sf = oracle.spmv(F, x)
    assert np.array_equal(yl, yf) and np.array_equal(sl, sf)


def test_sym_banded_vs_dense():
    L = gen.banded(300, 7, seed=9, lower=True)
    D = _dense(L)
    Dfull = D + np.tril(D, -1).T
    x = gen.uniform_vec(L.n, 5)
    y, s = oracle.spmv(L, x)
    assert np.all(np.abs(y - Dfull @ x) <= 32 * 2.3e-16 * s)


def test_spmv_rows_matches_full():
    A = gen.powerlaw(5000, seed=2)
    x = gen.uniform_vec(A.n, 12)
    y, s = oracle.spmv(A, x)
    rows = np.array([0, 17, 4999, 2500, 17])
    yr, sr = oracle.spmv_rows(A, x, rows)
    assert np.array_equal(yr, y[rows]) and np.array_equal(sr, s[rows])

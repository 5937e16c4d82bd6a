"""Generator checks (CPU only): counts fixed by geometry, the random streams
against SplitMix64's published definition, and structural invariants."""
import numpy as np
import pytest

import gen

MASK = (1 << 64) - 1


def _splitmix(state):
    """SplitMix64 written out from its definition (Steele, Lea & Flood)."""
    state = (state + 0x9E3779B97F4A7C15) & MASK
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return state, z ^ (z >> 31)


def _mix(z):
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


@pytest.mark.parametrize("seed,sid", [(0, 0), (2, 12345), (4 << 32, 7)])
def test_stream_is_splitmix64(seed, sid):
    s = _mix(seed ^ 0x5851F42D4C957F2D) ^ _mix((sid + 0x14057B7EF767814F) & MASK)
    for k in range(5):
        s, v = _splitmix(s)
        assert gen.stream_u64(seed, sid, k) == v


def test_counts():
    assert gen.laplacian2d(64).nnz == 5 * 4096 - 4 * 64 == 20224
    assert gen.laplacian2d(64, lower=True).nnz == 12160
    L = gen.stencil27(40, lower=True)
    F = gen.stencil27(40, lower=False)
    assert F.nnz == (3 * 40 - 2) ** 3
    assert F.nnz == 2 * L.nnz - L.n


@pytest.mark.slow
def test_counts_full_size():
    assert gen.stencil27(128, lower=True).nnz == 28_920_060
    assert gen.stencil27(128, lower=False).nnz == 55_742_968 == 382 ** 3


def _valid_csr(A, sym=False):
    rp, ci = A.rowptr.astype(np.int64), A.colind.astype(np.int64)
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == ci.size
    assert np.all(ci >= 0) and np.all(ci < A.ncols)
    for i in range(A.n):
        c = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0)
        if sym:
            assert np.all(c <= i)


def test_powerlaw_structure():
    A = gen.powerlaw(20000, seed=2)
    _valid_csr(A)
    ln = np.diff(A.rowptr)
    assert ln.min() >= 1 and ln.max() <= 5000
    # diagonal present, dominant: a_ii = 1.1 * sum |offdiag|
    for i in [0, 5, 19999]:
        c = A.colind[A.rowptr[i]:A.rowptr[i + 1]]
        v = A.val[A.rowptr[i]:A.rowptr[i + 1]]
        d = v[c == i]
        assert d.size == 1
        off = np.abs(v[c != i]).sum()
        assert abs(d[0] - (1.1 * off if off > 0 else 1.0)) <= 1e-14 * d[0]
    assert abs(ln.mean() - np.exp(3.0)) < 0.5   # E[lognormal(2.5,1)] = e^3


def test_trans4_shape():
    A = gen.trans4_like()
    ln = np.diff(A.rowptr)
    assert A.n == 116_835 and A.nnz == 749_800
    assert ln.max() == 114_910 and ln.min() == 1
    assert np.sort(ln)[-2] <= 7


def test_banded_and_blockdiag():
    B = gen.banded(500, 9, seed=3, lower=True)
    _valid_csr(B, sym=True)
    D = gen.blockdiag(700, 5)
    _valid_csr(D)
    G = gen.banded(500, 9, seed=3, lower=False)
    _valid_csr(G)


def test_batch_assembly():
    b = gen.batch(6, seed=4, nmin=100, nmax=400)
    assert b.row_off[-1] == b.rowptr.size - 1
    for k in range(6):
        S = b.system(k)
        _valid_csr(S)
        n, kind, h = gen.batch_params(6, seed=4, nmin=100, nmax=400)
        assert S.n == n[k]
        R = gen.batch_system(k, int(n[k]), int(kind[k]), int(h[k]))
        assert np.array_equal(R.colind, S.colind) and np.array_equal(R.val, S.val)


def test_vectors_deterministic():
    a = gen.uniform_vec(1000, 12)
    b = gen.uniform_vec(1000, 12)
    assert np.array_equal(a, b) and a.min() >= -1 and a.max() < 1
    c = gen.int_vec(1000, 3)
    assert np.all(c == np.round(c)) and c.min() >= -8 and c.max() <= 8

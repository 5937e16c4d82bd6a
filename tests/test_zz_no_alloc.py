"""The allocation-free SpMV (xab_spmv_csr_noalloc) against the planned
branchless segmented scan (xab_spmv_csr with a BSS plan of the same entries
per lane), through the C ABI.

Both run the same split, tile and fix-up kernels in the same order, so the
bar is bit equality; the FP64 result also meets the oracle's per-row gate
(abs error <= 1e-12 * sum abs(a x)) and integer-valued inputs give the
oracle's result exactly.  Each case makes two calls in a row, the second on a
smaller matrix, so the second call runs over descriptors and carries the
first one left in the shared buffer.
"""
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


def _dev(a, dt=None):
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return t.to(dt) if dt is not None else t


def _arrays(A, dt):
    return _dev(A.rowptr.astype(np.int32)), _dev(A.colind.astype(np.int32)), _dev(A.val, dt)


def _planned(ctx, A, x, j, dt, acc=None, ydtype=None):
    M = ctx.matrix_from_csr(A, with_f32=dt == torch.float32, with_f64=dt == torch.float64)
    P = ctx.plan(M, xab.BSS, j_per_lane=j)
    y = ctx.spmv(P, x, acc=acc, ydtype=ydtype)
    torch.cuda.synchronize()
    return y


def _ragged():
    """Power-law rows with empty rows and a ragged last tile."""
    A = gen.powerlaw(n=30_000, seed=7, mu=2.0, sigma=1.2, lmax=3000)
    ln = np.diff(A.rowptr)
    keep = np.ones(A.n, dtype=bool)
    keep[::97] = False  # empty every 97th row
    rp = np.zeros(A.n + 1, dtype=np.int64)
    rp[1:] = np.cumsum(np.where(keep, ln, 0))
    sel = np.repeat(keep, ln)
    return gen.CSR(A.n, A.n, rp.astype(np.int32), A.colind[sel], A.val[sel])


CASES = [
    ("powerlaw-60k then laplacian-40", lambda: gen.powerlaw(n=60_000, seed=2), lambda: gen.laplacian2d(40)),
    ("ragged then trans4-shaped", _ragged, lambda: gen.trans4_like(n=12_000, nnz=60_000, long_len=9000, seed=22)),
]


@pytest.mark.parametrize("j", [1, 4, 16, 32])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_noalloc_equals_planned_bss_fp64(ctx, case, j):
    _, big, small = case
    for A, seed in ((big(), 12), (small(), 1)):
        print(f"noalloc fp64 j={j} n={A.n} nnz={A.nnz}", flush=True)
        rp, ci, v = _arrays(A, torch.float64)
        xh = gen.uniform_vec(A.ncols, seed)
        x = _dev(xh)
        y = torch.full((A.n,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.spmv_noalloc(rp, ci, v, x, y, j=j)
        torch.cuda.synchronize()
        ref = _planned(ctx, A, x, j, torch.float64)
        assert torch.equal(y, ref)
        yo, s = oracle.spmv(A, xh)
        yh = y.cpu().numpy()
        assert np.all(np.abs(yh - yo) <= 1e-12 * s)
        assert np.all(yh[s == 0] == 0)


@pytest.mark.parametrize("j", [4, 8])
def test_noalloc_integer_exact_two_calls(ctx, j):
    for A, seed in ((gen.powerlaw(n=40_000, seed=5), 3), (gen.banded(5000, 9, seed=4), 4)):
        print(f"noalloc integer j={j} n={A.n} nnz={A.nnz}", flush=True)
        A.val = np.round(A.val * 4.0).clip(-8, 8)
        rp, ci, v = _arrays(A, torch.float64)
        xh = gen.int_vec(A.ncols, seed)
        y = torch.full((A.n,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.spmv_noalloc(rp, ci, v, _dev(xh), y, j=j)
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy(), oracle.spmv(A, xh)[0])


@pytest.mark.parametrize("yt,acc", [(torch.float32, xab.F32), (torch.float32, xab.F64), (torch.float64, xab.F64)])
def test_noalloc_equals_planned_bss_fp32_values(ctx, yt, acc):
    for A, seed in ((gen.powerlaw(n=50_000, seed=3), 13), (gen.laplacian2d(30), 2)):
        print(f"noalloc fp32 values y={yt} acc={acc} n={A.n}", flush=True)
        rp, ci, v = _arrays(A, torch.float32)
        x = _dev(gen.uniform_vec(A.ncols, seed), torch.float32)
        y = torch.full((A.n,), float("nan"), dtype=yt, device="cuda")
        ctx.spmv_noalloc(rp, ci, v, x, y, j=8, acc=acc)
        torch.cuda.synchronize()
        ref = _planned(ctx, A, x, 8, torch.float32, acc=acc, ydtype=yt)
        assert torch.equal(y, ref)


def test_noalloc_empty_and_limits(ctx):
    # no entries at all: every row is 0
    n = 300
    rp = _dev(np.zeros(n + 1, dtype=np.int32))
    ci = _dev(np.zeros(4, dtype=np.int32))
    v = _dev(np.zeros(4))
    x = _dev(np.ones(n))
    y = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    ctx.spmv_noalloc(rp, ci[:0], v[:0], x, y, j=4)
    torch.cuda.synchronize()
    assert torch.all(y == 0)
    # host-side refusals, before any launch
    h = xab.lib()
    too_many = (xab.NOALLOC_MAX_TILES + 1) * 256  # tiles of 256 entries at j = 1
    assert h.xab_spmv_csr_noalloc(ctx.h, n, n, too_many, xab._ptr(rp), xab._ptr(ci), xab._ptr(v), 1, xab._ptr(x),
                                  xab.F64, xab._ptr(y), xab.F64, xab.F64) == -2
    assert h.xab_spmv_csr_noalloc(ctx.h, n, n, 0, xab._ptr(rp), xab._ptr(ci), xab._ptr(v), 3, xab._ptr(x),
                                  xab.F64, xab._ptr(y), xab.F64, xab.F64) == -6
    assert h.xab_spmv_csr_noalloc(ctx.h, n, n, 0, xab._ptr(rp), xab._ptr(ci), xab._ptr(v), 4, xab._ptr(x),
                                  xab.F64, xab._ptr(x), xab.F64, xab.F64) == -5
    assert h.xab_spmv_csr_noalloc(ctx.h, n, n, 0, xab._ptr(rp), xab._ptr(ci), xab._ptr(v), 4, xab._ptr(x),
                                  xab.F64, xab._ptr(y), xab.F32, xab.F64) == -3

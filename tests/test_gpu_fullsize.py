"""Parity at the full sizes the benchmark runs, in the implementations it
times: the power-law matrix (n = 2,000,000, about 40 M entries; x seed 12,
as the benchmark) through the column-blocked XCB class in FP64 and with
FP32 values, the 27-point stencil 128^3 in lower storage through S3, and
the 512-system batch through its sliced ELLPACK copy.  The serial oracle
computes every row of these products in about a second, so the products are
compared element by element; the solvers at these sizes are checked
through properties the oracle can verify: the true residual of the
returned solution (one oracle product) meets the tolerance."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
xab = pytest.importorskip("paper_2405_01599_amd")

U32 = 2.0 ** -24


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0").to(dtype)


@pytest.fixture(scope="module")
def ctx():
    return xab.Context(0)


@pytest.fixture(scope="module")
def c2():
    print("generating the power-law matrix n=2,000,000", flush=True)
    return gen.powerlaw(2_000_000, seed=2)


def test_c2_spmv_fp64_and_fp32_values(ctx, c2):
    A = c2
    x = gen.uniform_vec(A.n, 12)
    yo, s = oracle.spmv(A, x)
    M = ctx.matrix_from_csr(A, with_f32=True)
    P = ctx.plan_class(M, 12)  # XCB J=4, the class the selector picks here
    y = ctx.spmv(P, dev(x)).cpu().numpy()
    assert np.all(np.abs(y - yo) <= 1e-12 * s)
    # FP32 values and x, FP64 accumulation and y: against the rounded inputs
    # only the final rounding of the FP64 sums, against the FP64 inputs the
    # rounding of val and x (2.01 u)
    x32 = x.astype(np.float32)
    A32 = gen.CSR(A.n, A.ncols, A.rowptr, A.colind, A.val.astype(np.float32).astype(np.float64))
    yr, sr = oracle.spmv(A32, x32.astype(np.float64))
    y32 = ctx.spmv(P, dev(x32, torch.float32), ydtype=torch.float64, acc=xab.F64).cpu().numpy()
    assert np.all(np.abs(y32 - yr) <= 1e-12 * sr)
    assert np.all(np.abs(y32 - yo) <= (1e-12 + 2.01 * U32) * s)


@pytest.mark.parametrize("mode", [0, 1])
def test_c2_gmres_true_residual(ctx, c2, mode):
    """GMRES(30) + Jacobi to 1e-10 on the full power-law matrix, FP64 and
    IR: the oracle's product with the returned x meets the tolerance."""
    A = c2
    b = np.ones(A.n)
    M = ctx.matrix_from_csr(A, with_f32=True)
    P = ctx.plan_class(M, 12)
    x, inf, st = ctx.gmres(P, dev(b), m=30, tol=1e-10, mode=mode)
    assert st == 0
    r = b - oracle.spmv(A, x.cpu().numpy())[0]
    res = np.linalg.norm(r) / np.linalg.norm(b)
    assert res <= 1e-10 and abs(res - inf["true_relres"]) <= 1e-12


def test_c3_symmetric_spmv(ctx):
    print("generating the 27-point stencil 128^3 (lower storage)", flush=True)
    L = gen.stencil27(128, lower=True)
    x = gen.uniform_vec(L.n, 13)
    yo, s = oracle.spmv(L, x)
    M = ctx.matrix_from_csr(L)
    for k in (10, 11):  # S3 with 64- and 256-column blocks
        P = ctx.plan_class(M, k)
        y = ctx.spmv(P, dev(x)).cpu().numpy()
        assert np.all(np.abs(y - yo) <= 1e-12 * s), k


def test_c4_batch_spmv_and_bicgstab(ctx):
    """The 512-system batch (n = 7.87 M, 371 M entries): the batched SpMV
    element by element, then BiCGStab + Jacobi to 1e-10: every system's
    true residual, from one oracle product over the concatenation, meets
    the tolerance."""
    print("generating the 512-system batch", flush=True)
    B = gen.batch()
    A = gen.CSR(B.n, B.n, B.rowptr, B.colind, B.val)
    bt = ctx.batch(B)
    assert bt.layout == "sell"
    x = gen.uniform_vec(B.n, 3)
    yo, s = oracle.spmv(A, x)
    y = bt.spmv(dev(x)).cpu().numpy()
    assert np.all(np.abs(y - yo) <= 1e-12 * s)
    del y, yo, s
    b = np.ones(B.n)
    xs, per, agg, st = ctx.bicgstab(bt, dev(b), tol=1e-10)
    assert st == 0
    r = b - oracle.spmv(A, xs.cpu().numpy())[0]
    for k in range(B.nsys):
        r0, r1 = int(B.row_off[k]), int(B.row_off[k + 1])
        assert np.linalg.norm(r[r0:r1]) / np.linalg.norm(b[r0:r1]) <= 1e-10 * 1.01, k
        assert per[k]["status"] == 0


def test_c3_lanczos_smallest_closed_form(ctx):
    """Lanczos (m = 30) for the 10 smallest eigenpairs of the 27-point
    stencil 128^3 through S3, as the benchmark runs it: every value is an
    eigenvalue of the stencil's closed-form spectrum (within 1e-9 of ||A||),
    the first is the smallest, the true residuals are within 1.5 tol."""
    g = 128
    L = gen.stencil27(g, lower=True)
    M = ctx.matrix_from_csr(L)
    P = ctx.plan_class(M, 10)
    t = 1.0 + 2.0 * np.cos(np.arange(1, g + 1) * np.pi / (g + 1))
    lam = np.sort((28.0 - np.einsum("i,j,k->ijk", t, t, t)).ravel())
    ev, X, info, st = ctx.lanczos(P, dev(gen.uniform_vec(L.n, 5)), nev=10, m=30, tol=1e-8,
                                  which=xab.EIG_SMALLEST, max_time_s=60.0)
    assert st == 0
    assert abs(ev[0] - lam[0]) <= 1e-9 * info["anrm"]
    for v in ev:
        assert np.min(np.abs(lam - v)) <= 1e-9 * info["anrm"]
    assert info["max_resid"] <= 1.5e-8


def test_convdiff_arnoldi_largest_closed_form(ctx):
    """Arnoldi (m = 30) for the 10 largest-real-part eigenvalues of the
    7-point convection-diffusion operator 128^3 (beta = 0.02) through the
    sliced ELLPACK class, as the benchmark runs it: real values of the
    closed-form spectrum (within 1e-9 of ||A||), the first the largest,
    true residuals within 1.5 tol."""
    g, beta = 128, 0.02
    A = gen.convdiff3d(g, beta)
    M = ctx.matrix_from_csr(A)
    P = ctx.plan_class(M, 13)
    k = np.arange(1, g + 1)
    lx = 2.0 + 2.0 * np.sqrt(1.0 - beta * beta) * np.cos(k * np.pi / (g + 1))
    ly = 2.0 - 2.0 * np.cos(k * np.pi / (g + 1))
    lam = np.sort((lx[:, None, None] + ly[None, :, None] + ly[None, None, :]).ravel())
    ev, X, info, st = ctx.arnoldi(P, dev(gen.uniform_vec(A.n, 5)), nev=10, m=30, tol=1e-8,
                                  which=xab.EIG_LARGEST, max_time_s=60.0)
    assert st == 0
    assert abs(ev[0].real - lam[-1]) <= 1e-9 * info["anrm"]
    for v in ev:
        assert abs(v.imag) <= 1e-9 * info["anrm"] and np.min(np.abs(lam - v.real)) <= 1e-9 * info["anrm"]
    assert info["max_resid"] <= 1.5e-8

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


@pytest.fixture(scope="module")
def c3():
    print("generating the 27-point stencil 128^3 (lower storage)", flush=True)
    return gen.stencil27(128, lower=True)


def test_c2_spmv_fp64_and_fp32_values(ctx, c2):
    A = c2
    x = gen.uniform_vec(A.n, 12)
    yo, s = oracle.spmv(A, x)
    M = ctx.matrix_from_csr(A, with_f32=True)
    P = ctx.plan_class(M, 12)  # XCB, the class the selector picks here
    assert P.describe()["j_per_lane"] == 32  # 40.2M entries: 4908 tiles of 8192
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


def test_c2_xcb_walks_integer_exact(ctx, c2):
    """At this size the XCB plan walks FP64 values with 32 entries per lane
    and FP32 values with 16 (their own interleaved columns and tiles): with
    integer values and x (every partial sum exact) both products equal the
    oracle's, before and after the values are changed in place and the
    plan refreshed."""
    rng = np.random.default_rng(31)
    A1 = gen.CSR(c2.n, c2.ncols, c2.rowptr, c2.colind, rng.integers(-8, 9, c2.nnz).astype(np.float64))
    A2 = gen.CSR(c2.n, c2.ncols, c2.rowptr, c2.colind, rng.integers(-8, 9, c2.nnz).astype(np.float64))
    x = gen.int_vec(c2.n, 7)
    M = ctx.matrix_from_csr(A1, with_f32=True)
    P = ctx.plan_class(M, 12)
    assert P.describe()["j_per_lane"] == 32
    for A in (A1, A2):
        if A is A2:
            M.val.copy_(dev(A2.val))
            M.val32.copy_(dev(A2.val, torch.float32))
            P.refresh()
        yo, _ = oracle.spmv(A, x)
        assert np.array_equal(ctx.spmv(P, dev(x)).cpu().numpy(), yo)
        y32 = ctx.spmv(P, dev(x, torch.float32), ydtype=torch.float64, acc=xab.F64).cpu().numpy()
        assert np.array_equal(y32, yo)


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


def test_c3_symmetric_spmv(ctx, c3):
    L = c3
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


@pytest.mark.parametrize("k", [10, 11])
def test_c3_symmetric_spmv_fp32_values(ctx, c3, k):
    """FP32 values and x on the full 27-point stencil through both S3
    classes, stated per row as abs(dy)/s against the FP64 oracle on the
    FP64 inputs: FP32 accumulation and y within (row length + 4) u32 (the
    recursive-sum bound plus the input roundings), FP64 accumulation with
    FP32 y within 4.01 u32 (input roundings, the tile's write of y and the
    block reduce's), FP64 accumulation and y within 2.01 u32 + 1e-12; every
    product repeats bit for bit."""
    L = c3
    x64 = gen.uniform_vec(L.n, 13)
    x32 = x64.astype(np.float32)
    yo, s = oracle.spmv(L, x64)
    lens = np.diff(oracle.sym_expand(L)[0]).astype(np.float64)
    M = ctx.matrix_from_csr(L, with_f32=True)
    P = ctx.plan_class(M, k)
    xd = dev(x32, torch.float32)
    for ydt, acc, bound in ((torch.float32, xab.F32, (lens + 4) * U32), (torch.float32, xab.F64, 4.01 * U32),
                            (torch.float64, xab.F64, 2.01 * U32 + 1e-12)):
        yd = ctx.spmv(P, xd, ydtype=ydt, acc=acc)
        y = yd.double().cpu().numpy()
        err = np.abs(y - yo) / np.where(s > 0, s, 1.0)
        print(f"class {k} y={ydt} acc={acc}: max |dy|/s = {err.max():.3e}", flush=True)
        assert np.all(np.abs(y - yo) <= bound * s)
        assert torch.equal(ctx.spmv(P, xd, ydtype=ydt, acc=acc), yd)


@pytest.mark.parametrize("mode", [0, 1])
def test_c3_gmres_true_residual(ctx, c3, mode):
    """GMRES(30) + Jacobi to 1e-10 on the full 27-point stencil through the
    symmetric S3 plan, FP64 and IR (FP32 values inside): the oracle's product
    with the returned x meets the tolerance, and the FP64 iteration count is
    within 20 % of the oracle's own GMRES (MGS) on the expanded matrix."""
    L = c3
    b = np.ones(L.n)
    M = ctx.matrix_from_csr(L, with_f32=True)
    P = ctx.plan_class(M, 10)
    x, inf, st = ctx.gmres(P, dev(b), m=30, tol=1e-10, mode=mode, precond=xab.PRECOND_JACOBI)
    assert st == 0
    r = b - oracle.spmv(L, x.cpu().numpy())[0]
    res = np.linalg.norm(r) / np.linalg.norm(b)
    print(f"mode {mode}: {inf['iters']} steps, {inf['refinements']} refinements, true relres {res:.3e}", flush=True)
    assert res <= 1e-10 and abs(res - inf["true_relres"]) <= 1e-12
    if mode == 0:
        rp, ci, v = oracle.sym_expand(L)
        ref = oracle.gmres(gen.CSR(L.n, L.n, rp, ci, v), b, m=30, tol=1e-10, precond=1)
        assert abs(inf["iters"] - ref["iters"]) <= max(2, 0.2 * ref["iters"])


def test_c3_lanczos_largest_closed_form(ctx, c3):
    """Lanczos (m = 30) for the 10 largest eigenpairs of the full 27-point
    stencil through S3: every value is an eigenvalue of the closed-form
    spectrum (within 1e-9 of ||A||), the first is the largest, and the
    oracle's product confirms every returned pair's residual."""
    g = 128
    L = c3
    M = ctx.matrix_from_csr(L)
    P = ctx.plan_class(M, 10)
    t = 1.0 + 2.0 * np.cos(np.arange(1, g + 1) * np.pi / (g + 1))
    lam = np.sort((28.0 - np.einsum("i,j,k->ijk", t, t, t)).ravel())
    ev, X, info, st = ctx.lanczos(P, dev(gen.uniform_vec(L.n, 5)), nev=10, m=30, tol=1e-8,
                                  which=xab.EIG_LARGEST, max_time_s=60.0)
    assert st == 0
    assert abs(ev[0] - lam[-1]) <= 1e-9 * info["anrm"]
    for v in ev:
        assert np.min(np.abs(lam - v)) <= 1e-9 * info["anrm"]
    Xh = X.cpu().numpy()
    for i, v in enumerate(ev):
        r = oracle.spmv(L, Xh[:, i])[0] - v * Xh[:, i]
        assert np.linalg.norm(r) <= 1.5e-8 * info["anrm"]


def test_c2_arnoldi_largest_magnitude(ctx, c2):
    """Arnoldi (m = 30) for the 10 largest-magnitude eigenvalues of the full
    power-law matrix through XCB, as the benchmark runs it: the oracle's
    product confirms every returned eigenpair (a complex pair through its
    real and imaginary parts), the values come in order of magnitude, and
    every eigenvector has unit norm."""
    A = c2
    M = ctx.matrix_from_csr(A)
    P = ctx.plan_class(M, 12)
    ev, X, info, st = ctx.arnoldi(P, dev(gen.uniform_vec(A.n, 5)), nev=10, m=30, tol=1e-8,
                                  which=xab.EIG_MAGNITUDE, max_time_s=60.0)
    assert st == 0
    mags = np.abs(ev)
    assert np.all(np.diff(mags) <= 1e-9 * info["anrm"])
    Xh = X.cpu().numpy()
    i = 0
    while i < len(ev):
        lr, li = ev[i].real, ev[i].imag
        if abs(li) <= 1e-12 * info["anrm"]:
            x = Xh[:, i]
            r = oracle.spmv(A, x)[0] - lr * x
            nrm = np.linalg.norm(x)
            i += 1
        else:
            xr, xi = Xh[:, i], Xh[:, i + 1]
            ar, ai = oracle.spmv(A, xr)[0], oracle.spmv(A, xi)[0]
            r = np.concatenate([ar - lr * xr + li * xi, ai - li * xr - lr * xi])
            nrm = np.sqrt(np.linalg.norm(xr) ** 2 + np.linalg.norm(xi) ** 2)
            i += 2
        assert abs(nrm - 1.0) <= 1e-10
        assert np.linalg.norm(r) <= 1.5e-8 * info["anrm"]


def test_c4_batch_fp32(ctx):
    """The 512-system batch with FP32 values, as the benchmark runs it: the
    batched SpMV (FP64 accumulation, FP32 y) element by element within one
    rounding of the oracle on the FP32-rounded inputs (1.01 u32 of s), and
    BiCGStab + Jacobi to 1e-5: every system reports convergence and its
    true residual, from the oracle's product on the FP32 matrix with the
    returned x, meets the tolerance."""
    print("generating the 512-system batch", flush=True)
    B = gen.batch()
    v32 = B.val.astype(np.float32).astype(np.float64)
    A = gen.CSR(B.n, B.n, B.rowptr, B.colind, v32)
    bt = ctx.batch(B, dtype="f32")
    assert bt.layout == "sell"
    x = gen.uniform_vec(B.n, 3).astype(np.float32)
    yo, s = oracle.spmv(A, x.astype(np.float64))
    y = bt.spmv(dev(x, torch.float32)).double().cpu().numpy()
    err = np.abs(y - yo) / np.where(s > 0, s, 1.0)
    print(f"batched FP32 SpMV: max |dy|/s = {err.max():.3e}", flush=True)
    assert np.all(np.abs(y - yo) <= 1.01 * U32 * s)
    del y, yo, s
    b = np.ones(B.n)
    xs, per, agg, st = ctx.bicgstab(bt, dev(b, torch.float32), tol=1e-5)
    assert st == 0
    r = b - oracle.spmv(A, xs.double().cpu().numpy())[0]
    worst = 0.0
    for k in range(B.nsys):
        r0, r1 = int(B.row_off[k]), int(B.row_off[k + 1])
        rel = np.linalg.norm(r[r0:r1]) / np.linalg.norm(b[r0:r1])
        worst = max(worst, rel)
        assert per[k]["status"] == 0
        assert rel <= 1e-5 * 1.01, k
    print(f"batched FP32 BiCGStab: worst true relres {worst:.3e}", flush=True)

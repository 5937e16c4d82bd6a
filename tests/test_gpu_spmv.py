"""GPU parity of every SpMV implementation against the CPU oracle.

Through the C ABI (Python binding).  Bars:
  * plan arrays (work splits, segmented-scan descriptors, touch map) equal
    the oracle's bit for bit;
  * integer-valued A and x (every partial sum exact): y equals the oracle
    bit for bit for every variant;
  * random FP64 values: |y - y_oracle| <= 1e-12 * sum_k |a_ik x_k| per row,
    and y_i is exactly 0 where that sum is 0;
  * FP32 values: the per-row error relative to the same sum, against the
    oracle run on the FP32-rounded inputs (accumulation error) and on the
    original FP64 inputs (total error), under the bounds stated per test;
  * two runs give identical bits (all variants but the atomic baseline).
"""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
xab = pytest.importorskip("paper_2405_01599_amd")

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def ctx():
    return xab.Context(0)


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0").to(dtype)


def _tiny(lens, ncols=None, seed=0, intvals=True):
    rng = np.random.default_rng(seed)
    n = len(lens)
    ncols = ncols or max(n, max(lens) if lens else 1)
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum(lens)
    ci = np.concatenate([np.sort(rng.choice(ncols, size=l, replace=False)) for l in lens] + [np.zeros(0)])
    v = rng.integers(-8, 9, int(rp[-1])).astype(np.float64) if intvals else rng.standard_normal(int(rp[-1]))
    return gen.CSR(n, ncols, rp, ci.astype(np.int32), v, name="tiny")


def general_suite():
    out = {
        "tiny_mixed": _tiny([0, 3, 17, 0, 1, 1, 0, 40, 2, 0, 0, 16, 16, 1] * 7, ncols=120),
        "empty_edges": _tiny([16, 0, 0, 16, 0, 16, 0] * 40, ncols=300),
        "trailing_empty": _tiny([5, 7] * 50 + [0] * 37, ncols=200),
        "all_empty": _tiny([0] * 33, ncols=33),
        "one_long_row": _tiny([1, 3000, 1, 2], ncols=4000),
        "n1": _tiny([77], ncols=100),
        "lap2d": gen.laplacian2d(64),
        "powerlaw": gen.powerlaw(60_000, seed=2),
        "trans4": gen.trans4_like(),
        "blockdiag": gen.blockdiag(20_000, 3),
        "blockdiag_ragged": gen.blockdiag(10_001, 4),   # n not a multiple of 4
        "kron4": _kron_blocks(gen.laplacian2d(24), 4, seed=6),
    }
    return out


def _kron_blocks(A, b, seed):
    """A with every entry replaced by a dense b x b block of N(0, 1) values
    (b unknowns per grid node, as in FEM systems): aligned b x b blocks."""
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for i in range(A.n):
        for k in range(A.rowptr[i], A.rowptr[i + 1]):
            j = int(A.colind[k])
            blk = rng.standard_normal((b, b))
            for p in range(b):
                for q in range(b):
                    rows.append(i * b + p)
                    cols.append(j * b + q)
                    vals.append(blk[p, q])
    rows, cols, vals = np.array(rows), np.array(cols), np.array(vals)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    n = A.n * b
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum(np.bincount(rows, minlength=n))
    return gen.CSR(n, n, rp, cols.astype(np.int32), vals, name=f"kron{b}")


GENERAL = general_suite()
GENERAL_CLASSES = list(xab.GENERAL_CLASSES)


def _sell_supported(A, sigma=1024):
    """The SELL plan's own limits, from the oracle's layout of A."""
    p = oracle.plan_sell(A, 64, sigma)
    longest = int(np.max(np.diff(A.rowptr))) if A.n else 0
    return longest <= 4096 and int(p["cptr"][-1]) <= 2 * A.nnz + 64 * longest


def _bcsr_supported(A):
    """The BCSR plan's own limits, from the oracle's layout of A: block rows
    of at most 4096 entries, blocks holding at most twice the entries."""
    p = oracle.plan_bcsr(A, 4)
    rows = np.diff(A.rowptr[np.minimum(np.arange(0, A.n + 4, 4), A.n)]) if A.n else np.zeros(1)
    return int(np.max(rows, initial=0)) <= 4096 and 16 * len(p["bci"]) <= 2 * A.nnz


def _plan_class(ctx, M, A, k):
    """Plan of class k; for SELL or BCSR on a matrix outside its limits,
    check the library refuses it (XAB_E_UNSUPPORTED) and return None."""
    v = xab.class_params(k)[0]
    if (v == xab.SELL and not _sell_supported(A, xab.class_params(k)[1].tile_rows)) or \
            (v == xab.BCSR and not _bcsr_supported(A)):
        with pytest.raises(xab.XabError) as e:
            ctx.plan_class(M, k)
        assert e.value.status == -6
        return None
    return ctx.plan_class(M, k)


def _int_version(A, seed=5):
    rng = np.random.default_rng(seed)
    B = gen.CSR(A.n, A.ncols, A.rowptr, A.colind, rng.integers(-8, 9, A.nnz).astype(np.float64),
                sym_lower=A.sym_lower, name=A.name)
    return B


@pytest.mark.parametrize("name", sorted(GENERAL))
@pytest.mark.parametrize("k", GENERAL_CLASSES)
def test_general_integer_bitexact(ctx, name, k):
    A = _int_version(GENERAL[name])
    x = gen.int_vec(A.ncols, 9)
    yo, _ = oracle.spmv(A, x)
    M = ctx.matrix_from_csr(A)
    P = _plan_class(ctx, M, A, k)
    if P is None:
        return
    y = ctx.spmv(P, dev(x))
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy(), yo), f"class {k} on {name}"


@pytest.mark.parametrize("name", sorted(GENERAL))
@pytest.mark.parametrize("k", GENERAL_CLASSES)
def test_general_fp64_gate_and_determinism(ctx, name, k):
    A = GENERAL[name]
    x = gen.uniform_vec(A.ncols, 12)
    yo, s = oracle.spmv(A, x)
    M = ctx.matrix_from_csr(A)
    P = _plan_class(ctx, M, A, k)
    if P is None:
        return
    xd = dev(x)
    y1 = ctx.spmv(P, xd).cpu().numpy()
    y2 = ctx.spmv(P, xd).cpu().numpy()
    err = np.abs(y1 - yo)
    assert np.all(err <= 1e-12 * s), f"max rel {np.max(err / np.maximum(s, 1e-300))}"
    assert np.all(y1[s == 0] == 0.0)
    assert np.array_equal(y1, y2)


@pytest.mark.parametrize("sigma", [64, 192, 1024])
def test_sell_plan_bitexact(ctx, sigma):
    for name, A in GENERAL.items():
        if not _sell_supported(A, sigma):
            continue
        M = ctx.matrix_from_csr(A)
        P = ctx.plan(M, xab.SELL, tile_rows=sigma)
        ref = oracle.plan_sell(A, 64, sigma)
        assert np.array_equal(P.array(11), ref["perm"]), (name, sigma)
        assert np.array_equal(P.array(12), ref["rlen"]), (name, sigma)
        assert np.array_equal(P.array(13), ref["clen"]), (name, sigma)
        assert np.array_equal(P.array(14), ref["cols"]), (name, sigma)


def test_bcsr_plan_bitexact(ctx):
    """Block row pointers, block columns and position masks equal the
    oracle's; the blocked values are checked through the exact SpMVs.  The
    suite has matrices on both sides of the limits."""
    seen = [0, 0]
    for name, A in GENERAL.items():
        M = ctx.matrix_from_csr(A)
        if not _bcsr_supported(A):
            with pytest.raises(xab.XabError) as e:
                ctx.plan(M, xab.BCSR)
            assert e.value.status == -6
            seen[1] += 1
            continue
        P = ctx.plan(M, xab.BCSR)
        ref = oracle.plan_bcsr(A, 4)
        assert np.array_equal(P.array(15), ref["brp"]), name
        assert np.array_equal(P.array(16), ref["bci"]), name
        assert np.array_equal(P.array(17).astype(np.uint32), ref["bmask"]), name
        seen[0] += 1
    assert seen[0] >= 3 and seen[1] >= 1


def test_bcsr_duplicates_and_nonfinite_x(ctx):
    """Duplicate entries are summed in the block; a non-finite x entry at a
    column that shares a block with every row but is stored nowhere does not
    reach them."""
    cols = [0, 1, 2, 2, 3, 4, 5, 7]                 # column 2 twice, column 6 never
    rp = np.arange(0, 4 * len(cols) + 1, len(cols), dtype=np.int32)
    ci = np.array(cols * 4, dtype=np.int32)
    v = np.arange(1.0, 4 * len(cols) + 1)
    A = gen.CSR(4, 8, rp, ci, v)
    M = ctx.matrix_from_csr(A)
    P = ctx.plan(M, xab.BCSR)
    x = np.arange(1.0, 9.0)
    assert np.array_equal(ctx.spmv(P, dev(x)).cpu().numpy(), oracle.spmv(A, x)[0])
    x[6] = np.inf
    y = ctx.spmv(P, dev(x)).cpu().numpy()
    assert np.all(np.isfinite(y)) and np.array_equal(y, oracle.spmv(A, x)[0])


def test_nnz_plan_bitexact(ctx):
    for name, A in GENERAL.items():
        M = ctx.matrix_from_csr(A)
        for T in (64, 2048, 8192):
            P = ctx.plan(M, xab.NNZ, tile_nnz=T)
            assert np.array_equal(P.array(0), oracle.plan_nnz(A.rowptr, T)), (name, T)


def test_bss_plan_bitexact(ctx):
    for name, A in GENERAL.items():
        M = ctx.matrix_from_csr(A)
        for J in (1, 4, 8, 16, 32):
            P = ctx.plan(M, xab.BSS, j_per_lane=J)
            row_lo, tile_row, carry = oracle.plan_bss(A.rowptr, 256 * J)
            assert np.array_equal(P.array(1), row_lo), (name, J)
            assert np.array_equal(P.array(2), tile_row), (name, J)
            assert np.array_equal(P.array(3), carry), (name, J)


def test_xcb_plan_bitexact(ctx):
    # J = 16 and 32 store full tiles interleaved in groups; the read-back is
    # in block order whatever the device layout
    for name, A in GENERAL.items():
        M = ctx.matrix_from_csr(A)
        rp, ci = oracle.plan_xcb(A, 8, flagged=True)
        for J in (4, 16, 32):
            P = ctx.plan(M, xab.XCB, j_per_lane=J)
            assert np.array_equal(P.array(9), rp.reshape(-1)), (name, J)
            assert np.array_equal(P.array(10), ci), (name, J)


@pytest.mark.parametrize("name", ["powerlaw50k", "trans4", "one_long_row"])
@pytest.mark.parametrize("J", [1, 2, 4, 8, 16, 32])
def test_xcb_all_lane_widths(ctx, J, name):
    # power-law: about 125k entries per column block, many full tiles and a
    # ragged last tile in each block at every J; trans4: one row of 114,910
    # entries whose part in each block spans many tiles (carries through
    # interleaved full tiles); a 3000-entry row in a tiny matrix
    A = _int_version(gen.powerlaw(50_000, seed=2) if name == "powerlaw50k" else GENERAL[name])
    x = gen.int_vec(A.ncols, 2)
    yo, _ = oracle.spmv(A, x)
    M = ctx.matrix_from_csr(A, with_f32=True)
    P = ctx.plan(M, xab.XCB, j_per_lane=J)
    assert np.array_equal(ctx.spmv(P, dev(x)).cpu().numpy(), yo)
    # FP32 values and x (integers, sums below 2^24: exact in either accumulation)
    for acc in (xab.F32, xab.F64):
        y32 = ctx.spmv(P, dev(x, torch.float32), ydtype=torch.float32, acc=acc).double().cpu().numpy()
        assert np.array_equal(y32, yo), acc


@pytest.mark.parametrize("J", [16, 32])
def test_xcb_tiles_with_more_rows_than_staged(ctx, J):
    # one or two entries per row at random columns: a block's compressed rows
    # hold about one entry each, so a tile of 256 J entries starts up to
    # 256 J rows, more than the 4096 the kernel stages in LDS at J = 32
    rng = np.random.default_rng(21)
    n = 300_000
    lens = rng.integers(1, 3, n)
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum(lens)
    first = rng.integers(0, n - 1, n)
    second = first + 1 + rng.integers(0, 1 << 30, n) % (n - 1 - first)  # in (first, n)
    ci = np.empty(int(rp[-1]), dtype=np.int32)
    ci[rp[:-1]] = first
    two = lens == 2
    ci[rp[:-1][two] + 1] = second[two]
    A = gen.CSR(n, n, rp, ci, rng.integers(-8, 9, ci.size).astype(np.float64))
    x = gen.int_vec(n, 4)
    yo, _ = oracle.spmv(A, x)
    M = ctx.matrix_from_csr(A)
    P = ctx.plan(M, xab.XCB, j_per_lane=J)
    assert np.array_equal(ctx.spmv(P, dev(x)).cpu().numpy(), yo)


def test_xcb_size_chosen_lane_width(ctx):
    # class 12 leaves the entries per lane to the plan: the largest of 4, 8,
    # 16, 32 that keeps at least 4096 tiles of 256 J entries
    A = gen.powerlaw(50_000, seed=2)
    M = ctx.matrix_from_csr(A)
    P = ctx.plan_class(M, 12)
    assert P.variant == xab.XCB and P.describe()["j_per_lane"] == 4
    x = gen.uniform_vec(A.ncols, 3)
    yo, s = oracle.spmv(A, x)
    assert np.all(np.abs(ctx.spmv(P, dev(x)).cpu().numpy() - yo) <= 1e-12 * s)


@pytest.mark.parametrize("J", [1, 2, 4, 8, 16, 32])
def test_bss_all_lane_widths(ctx, J):
    A = _int_version(gen.trans4_like())
    x = gen.int_vec(A.ncols, 2)
    yo, _ = oracle.spmv(A, x)
    M = ctx.matrix_from_csr(A)
    P = ctx.plan(M, xab.BSS, j_per_lane=J)
    assert np.array_equal(ctx.spmv(P, dev(x)).cpu().numpy(), yo)


@pytest.mark.parametrize("S", [1, 2, 4, 8, 16, 32, 64])
def test_row_all_lane_counts(ctx, S):
    A = _int_version(gen.powerlaw(20_000, seed=2))
    x = gen.int_vec(A.ncols, 2)
    yo, _ = oracle.spmv(A, x)
    M = ctx.matrix_from_csr(A)
    P = ctx.plan(M, xab.ROW, lanes_per_row=S)
    assert np.array_equal(ctx.spmv(P, dev(x)).cpu().numpy(), yo)


# ----------------------------------------------------------------- FP32
FP32_COMBOS = [  # (y dtype, acc) with x and values FP32
    (torch.float32, xab.F32),
    (torch.float32, xab.F64),
    (torch.float64, xab.F64),
]


@pytest.mark.parametrize("name", ["powerlaw", "trans4", "lap2d", "one_long_row", "blockdiag"])
@pytest.mark.parametrize("k", [0, 1, 3, 6, 8, 12, 13, 14])
@pytest.mark.parametrize("combo", range(3))
def test_general_fp32(ctx, name, k, combo):
    ydt, acc = FP32_COMBOS[combo]
    A = GENERAL[name]
    x64 = gen.uniform_vec(A.ncols, 12)
    x32 = x64.astype(np.float32)
    A32 = gen.CSR(A.n, A.ncols, A.rowptr, A.colind, A.val.astype(np.float32).astype(np.float64))
    y_rounded, s_r = oracle.spmv(A32, x32.astype(np.float64))
    y_exact, s = oracle.spmv(A, x64)
    M = ctx.matrix_from_csr(A, with_f32=True)
    P = _plan_class(ctx, M, A, k)
    if P is None:
        return
    y = ctx.spmv(P, dev(x32, torch.float32), ydtype=ydt, acc=acc).double().cpu().numpy()
    lens = np.diff(A.rowptr).astype(np.float64)
    # accumulation error alone (rounded inputs): recursive-summation bound
    # (len + 2) u for FP32 accumulation; FP64 accumulation only rounds the
    # result (and BSS/row partials) once more when y is FP32
    if acc == xab.F32:
        bound_acc = (lens + 2) * U32
    elif ydt == torch.float32:
        bound_acc = np.full(A.n, 1.01 * U32)
    else:
        bound_acc = np.full(A.n, 1e-12)
    ea = np.abs(y - y_rounded)
    assert np.all(ea <= bound_acc * s_r + 0.0)
    # total error against the FP64 inputs: value and x rounding add 2u
    et = np.abs(y - y_exact)
    assert np.all(et <= (bound_acc + 2.01 * U32) * s)


# ----------------------------------------------------------------- symmetric
def _drop_rows(L, rows):
    """L with every entry of `rows` removed (empty rows inside some tiles)."""
    keep = np.ones(L.n, dtype=bool)
    keep[rows] = False
    lens = np.diff(L.rowptr) * keep
    rp = np.zeros(L.n + 1, dtype=np.int32)
    rp[1:] = np.cumsum(lens)
    m = np.repeat(keep, np.diff(L.rowptr))
    return gen.CSR(L.n, L.ncols, rp, L.colind[m].copy(), L.val[m].copy(), sym_lower=True, name="holes")


def _arrow(n, band, seed):
    """Lower triangle of an arrowhead matrix: row i holds column 0 and the
    band i - band .. i.  Rows of 8 entries start at multiples of 8, so one
    slot of every chunk holds column 0 in every lane: the walk adds those
    entries one lane at a time."""
    rng = np.random.default_rng(seed)
    rows = [np.unique(np.r_[0, np.arange(max(0, i - band), i + 1)]) for i in range(n)]
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum([r.size for r in rows])
    ci = np.concatenate(rows).astype(np.int32)
    v = rng.standard_normal(ci.size)
    return gen.CSR(n, n, rp, ci, v, sym_lower=True, name="arrow")


def _sym_powerlaw(n, seed):
    """Lower triangle with lognormal row lengths (the diagonal plus distinct
    random columns in the 600 below it): rows of very different lengths, so
    the symmetric product walks the CSR entry stream, not the sliced copy."""
    rng = np.random.default_rng(seed)
    lens = np.clip(np.round(np.exp(rng.normal(1.5, 1.2, n))), 1, 400).astype(np.int64)
    rows = []
    for i in range(n):
        lo = max(0, i - 600)
        k = int(min(lens[i] - 1, i - lo))
        below = lo + rng.choice(i - lo, size=k, replace=False) if k > 0 else np.zeros(0, dtype=np.int64)
        rows.append(np.sort(np.r_[below, i]).astype(np.int32))
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum([r.size for r in rows])
    ci = np.concatenate(rows)
    return gen.CSR(n, n, rp, ci, rng.standard_normal(ci.size), sym_lower=True, name="sym_powerlaw")


def sym_suite():
    B = gen.banded(20_000, 30, 9, lower=True)
    return {
        "arrow": _arrow(3000, 6, 5),
        "sym_powerlaw": _sym_powerlaw(12_000, 4),
        "sym_powerlaw_holes": _drop_rows(_sym_powerlaw(9_000, 6), np.r_[0:3, 2000:2040, 5001:9000:211, 8999]),
        "banded_holes": _drop_rows(B, np.r_[0:5, 7000:7100, 13001:20000:997, 19999]),
        "lap2d_lower": gen.laplacian2d(64, lower=True),
        "st27_16": gen.stencil27(16, lower=True),
        "st27_24": gen.stencil27(24, lower=True),
        "banded_lower": gen.banded(30_000, 40, 7, lower=True),
        "tiny_sym": gen.banded(37, 3, 2, lower=True),
    }


SYM = sym_suite()
SYM_CLASSES = [9, 10, 11]


@pytest.mark.parametrize("name", sorted(SYM))
@pytest.mark.parametrize("k", SYM_CLASSES)
def test_sym_integer_bitexact(ctx, name, k):
    A = _int_version(SYM[name])
    x = gen.int_vec(A.n, 4)
    yo, _ = oracle.spmv(A, x)
    M = ctx.matrix_from_csr(A)
    P = ctx.plan_class(M, k)
    y = ctx.spmv(P, dev(x)).cpu().numpy()
    assert np.array_equal(y, yo)


@pytest.mark.parametrize("name", sorted(SYM))
@pytest.mark.parametrize("k", SYM_CLASSES)
def test_sym_fp64_gate(ctx, name, k):
    A = SYM[name]
    x = gen.uniform_vec(A.n, 13)
    yo, s = oracle.spmv(A, x)
    M = ctx.matrix_from_csr(A)
    P = ctx.plan_class(M, k)
    y = ctx.spmv(P, dev(x)).cpu().numpy()
    assert np.all(np.abs(y - yo) <= 1e-12 * s)


@pytest.mark.parametrize("name", sorted(SYM))
def test_sym_lower_equals_full(ctx, name):
    """Invariant: symmetric lower storage gives the full-storage product."""
    L = SYM[name]
    rp, ci, v = oracle.sym_expand(L)
    F = gen.CSR(L.n, L.n, rp, ci, v)
    x = gen.uniform_vec(L.n, 3)
    ML, MF = ctx.matrix_from_csr(L), ctx.matrix_from_csr(F)
    yl = ctx.spmv(ctx.plan_class(ML, 11), dev(x)).cpu().numpy()
    yf = ctx.spmv(ctx.plan_class(MF, 3), dev(x)).cpu().numpy()
    _, s = oracle.spmv(F, x)
    assert np.all(np.abs(yl - yf) <= 2e-12 * s)


@pytest.mark.parametrize("name", sorted(SYM))
@pytest.mark.parametrize("C,T,R", [(64, 16384, 2048), (256, 16384, 2048), (16, 512, 64), (1024, 4096, 300)])
def test_sym_plan_bitexact(ctx, name, C, T, R):
    A = SYM[name]
    M = ctx.matrix_from_csr(A)
    try:
        P = ctx.plan(M, xab.SYM_S3, col_block=C, tile_nnz=T, tile_rows=R)
    except xab.XabError as e:
        assert e.status == -6  # transpose part does not fit this block size
        return
    want = oracle.plan_sym(A, T, R, C)
    assert np.array_equal(P.array(0), want["b"])
    assert np.array_equal(P.array(4), want["tm_ptr"])
    assert np.array_equal(P.array(5), want["tm_tile"])
    assert np.array_equal(P.array(6), want["tile_ptr"])
    assert np.array_equal(P.array(7), want["tile_blk"])
    assert np.array_equal(P.array(8), want["tile_slot"])
    lay = oracle.plan_sym_slices(A, want["b"])
    if lay["sliced"]:
        assert P.array(18).size == 0
        assert np.array_equal(P.array(19), lay["ch0"])
        assert np.array_equal(P.array(20), lay["cw"])
        assert np.array_equal(P.array(21), lay["cols"])
    else:
        assert P.array(19).size == 0 and P.array(21).size == 0
        assert np.array_equal(P.array(18), oracle.plan_sym_colflags(A, want["b"], 64, 8))
    x = gen.int_vec(A.n, 1)
    Ai = _int_version(A)
    Mi = ctx.matrix_from_csr(Ai)
    Pi = ctx.plan(Mi, xab.SYM_S3, col_block=C, tile_nnz=T, tile_rows=R)
    assert np.array_equal(ctx.spmv(Pi, dev(x)).cpu().numpy(), oracle.spmv(Ai, x)[0])


@pytest.mark.parametrize("k", [10, 11])
@pytest.mark.parametrize("combo", range(3))
def test_sym_fp32(ctx, k, combo):
    ydt, acc = FP32_COMBOS[combo]
    A = SYM["st27_24"]
    x64 = gen.uniform_vec(A.n, 13)
    x32 = x64.astype(np.float32)
    y_exact, s = oracle.spmv(A, x64)
    M = ctx.matrix_from_csr(A, with_f32=True)
    y = ctx.spmv(ctx.plan_class(M, k), dev(x32, torch.float32), ydtype=ydt, acc=acc).double().cpu().numpy()
    L = np.diff(oracle.sym_expand(A)[0]).astype(np.float64)
    bound = (L + 4) * U32 if acc == xab.F32 else np.full(A.n, 4.01 * U32)
    assert np.all(np.abs(y - y_exact) <= bound * s)


@pytest.mark.parametrize("name", ["st27_24", "arrow", "sym_powerlaw", "sym_powerlaw_holes"])
@pytest.mark.parametrize("k", [10, 11])
def test_sym_s3_fp32_accumulation_is_fp64(ctx, name, k):
    """S3 keeps its tile sums in FP64 for either accumulation type (the FP32
    LDS atomic add is the slow one on this chip), so asking for FP32
    accumulation gives the FP64-accumulation bits, on both walks."""
    A = SYM[name]
    x32 = dev(gen.uniform_vec(A.n, 17).astype(np.float32), torch.float32)
    M = ctx.matrix_from_csr(A, with_f32=True)
    P = ctx.plan_class(M, k)
    y32 = ctx.spmv(P, x32, ydtype=torch.float32, acc=xab.F32)
    y64 = ctx.spmv(P, x32, ydtype=torch.float32, acc=xab.F64)
    assert torch.equal(y32, y64)


@pytest.mark.parametrize("name", ["st27_24", "banded_holes", "arrow", "sym_powerlaw", "sym_powerlaw_holes"])
@pytest.mark.parametrize("k", [10, 11])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_sym_determinism(ctx, name, k, prec):
    """The symmetric product is the same bit for bit on every run, in both
    walks (sliced: the stencils, bands and the arrow; entry stream: the
    power-law rows): every addition to a tile's accumulators happens in one
    fixed order."""
    A = SYM[name]
    M = ctx.matrix_from_csr(A, with_f32=True)
    P = ctx.plan_class(M, k)
    xh = gen.uniform_vec(A.n, 1)
    if prec == "f64":
        x, kw = dev(xh), {}
    else:
        x, kw = dev(xh, torch.float32), {"ydtype": torch.float32, "acc": xab.F64}
    ref = ctx.spmv(P, x, **kw)
    for _ in range(20):
        assert torch.equal(ctx.spmv(P, x, **kw), ref)


# ----------------------------------------------------------------- value refresh
REFRESH_CASES = [("powerlaw", k) for k in GENERAL_CLASSES] + [("blockdiag_ragged", 14), ("kron4", 14)] + \
    [("st27_24", k) for k in SYM_CLASSES] + [("banded_holes", 10), ("arrow", 10)]


@pytest.mark.parametrize("name,k", REFRESH_CASES)
def test_plan_refresh_after_value_change(ctx, name, k):
    # the plan built on one set of values, then the matrix's values changed
    # in place and the plan refreshed: the product is the oracle's for the
    # new values (integers: exact, FP64 and FP32 values), and bit-equal to a
    # plan built afresh on the new values
    A = GENERAL[name] if name in GENERAL else SYM[name]
    A1, A2 = _int_version(A, seed=5), _int_version(A, seed=9)
    x = gen.int_vec(A.ncols, 3)
    M = ctx.matrix_from_csr(A1, with_f32=True)
    P = _plan_class(ctx, M, A1, k) if name in GENERAL else ctx.plan_class(M, k)
    if P is None:
        return
    assert np.array_equal(ctx.spmv(P, dev(x)).cpu().numpy(), oracle.spmv(A1, x)[0])
    M.val.copy_(dev(A2.val))
    M.val32.copy_(dev(A2.val, torch.float32))
    P.refresh()
    yo, _ = oracle.spmv(A2, x)
    y = ctx.spmv(P, dev(x)).cpu().numpy()
    assert np.array_equal(y, yo)
    y32 = ctx.spmv(P, dev(x, torch.float32), ydtype=torch.float64, acc=xab.F64).cpu().numpy()
    assert np.array_equal(y32, yo)
    Q = ctx.plan_class(M, k)
    assert torch.equal(ctx.spmv(Q, dev(x)), ctx.spmv(P, dev(x)))


def test_plan_refresh_drops_the_jacobi_diagonal(ctx):
    # GMRES with Jacobi after a value change and refresh solves the new
    # system (the cached diagonal of the old values is not reused)
    A = gen.laplacian2d(32)
    M = ctx.matrix_from_csr(A)
    P = ctx.plan_class(M, 12)
    b = torch.ones(A.n, dtype=torch.float64, device="cuda")
    ctx.gmres(P, b, tol=1e-10, precond=xab.PRECOND_JACOBI)
    A2 = gen.CSR(A.n, A.ncols, A.rowptr, A.colind, A.val * np.where(A.colind == np.repeat(np.arange(A.n), np.diff(A.rowptr)), 2.0, 1.0))
    M.val.copy_(dev(A2.val))
    P.refresh()
    x, inf, st = ctx.gmres(P, b, tol=1e-10, precond=xab.PRECOND_JACOBI)
    assert st == 0
    r = oracle.spmv(A2, x.cpu().numpy())[0] - 1.0
    assert np.linalg.norm(r) <= 1e-9 * np.sqrt(A.n)


def test_plan_refresh_errors():
    import ctypes
    assert xab.lib().xab_plan_refresh(None) == -1


# ----------------------------------------------------------------- XCB column slices
@pytest.mark.parametrize("S", [2, 4])
@pytest.mark.parametrize("J", [0, 4, 32])
def test_xcb_sliced_integer_exact(ctx, S, J):
    # S column slices walked one after another (8 blocks each), summed in
    # slice order: integer products exact in every precision combination,
    # before and after a value refresh; J = 0 chooses each slice's entries
    # per lane from its own size
    A1 = _int_version(gen.powerlaw(50_000, seed=2), seed=5)
    A2 = _int_version(gen.powerlaw(50_000, seed=2), seed=9)
    x = gen.int_vec(A1.ncols, 2)
    M = ctx.matrix_from_csr(A1, with_f32=True)
    P = ctx.plan(M, xab.XCB, j_per_lane=J, xcb_slices=S)
    assert P.describe()["xcb_slices"] == S
    assert P.array(10).size == 0  # the slices hold the copies
    for A in (A1, A2):
        if A is A2:
            M.val.copy_(dev(A2.val))
            M.val32.copy_(dev(A2.val, torch.float32))
            P.refresh()
        yo, _ = oracle.spmv(A, x)
        assert np.array_equal(ctx.spmv(P, dev(x)).cpu().numpy(), yo)
        for ydt, acc in ((torch.float64, xab.F64), (torch.float32, xab.F64), (torch.float32, xab.F32)):
            y = ctx.spmv(P, dev(x, torch.float32), ydtype=ydt, acc=acc).double().cpu().numpy()
            assert np.array_equal(y, yo), (ydt, acc)


@pytest.mark.parametrize("name", sorted(GENERAL))
def test_xcb_sliced_general_suite(ctx, name):
    # empty rows and matrices, a single row, 3000- and 114,910-entry rows,
    # fewer columns than blocks per slice
    A = _int_version(GENERAL[name])
    x = gen.int_vec(A.ncols, 4)
    yo, _ = oracle.spmv(A, x)
    M = ctx.matrix_from_csr(A)
    for S in (2, 8):
        P = ctx.plan(M, xab.XCB, j_per_lane=8, xcb_slices=S)
        assert np.array_equal(ctx.spmv(P, dev(x)).cpu().numpy(), yo), S


def test_xcb_sliced_fp64_gate_and_reruns(ctx):
    A = gen.powerlaw(60_000, seed=3)
    x = gen.uniform_vec(A.ncols, 5)
    yo, s = oracle.spmv(A, x)
    M = ctx.matrix_from_csr(A)
    P = ctx.plan(M, xab.XCB, j_per_lane=16, xcb_slices=4)
    y0 = ctx.spmv(P, dev(x))
    assert np.all(np.abs(y0.cpu().numpy() - yo) <= 1e-12 * s)
    for _ in range(5):
        assert torch.equal(ctx.spmv(P, dev(x)), y0)


def test_xcb_slice_count_from_the_size(ctx):
    # up to 262,144 columns per block: one slice below 2,097,153 columns
    A = gen.powerlaw(50_000, seed=2)
    M = ctx.matrix_from_csr(A)
    assert ctx.plan_class(M, 12).describe()["xcb_slices"] == 1
    with pytest.raises(xab.XabError):
        ctx.plan(M, xab.XCB, j_per_lane=8, xcb_slices=3)

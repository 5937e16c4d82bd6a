"""Pins for the oracle's integer plans (CPU only).

Each plan array is checked against a linear-scan brute force of its
definition on tiny adversarial inputs, and each plan is shown to define a
correct decomposition by evaluating A*x through it (integer values, so any
order is exact) in a plain Python walk.
"""
import numpy as np
import pytest

import gen
import oracle


def _rp(lens):
    rp = np.zeros(len(lens) + 1, dtype=np.int32)
    rp[1:] = np.cumsum(lens)
    return rp


def _mat(lens, seed=0, ncols=None):
    rng = np.random.default_rng(seed)
    rp = _rp(lens)
    n = len(lens)
    ncols = ncols or max(n, max(lens) if lens else 1)
    ci = np.concatenate([np.sort(rng.choice(ncols, size=l, replace=False)) for l in lens] + [np.zeros(0)])
    v = rng.integers(-8, 9, int(rp[-1])).astype(np.float64)
    return gen.CSR(n, ncols, rp, ci.astype(np.int32), v)


ADVERSARIAL = {
    "nnz_lt_T": [1, 2, 0, 3],
    "nnz_multiple_T": [4] * 16,                       # 64 entries, T = 16
    "one_row_3_tiles": [1, 50, 1],                    # row spans >= 3 tiles of 16
    "empty_at_edges": [16, 0, 0, 16, 0, 16, 0],       # empty rows at tile edges
    "trailing_empty": [5, 7, 0, 0, 0],
    "leading_empty": [0, 0, 9, 9],
    "all_empty": [0, 0, 0],
    "n1": [33],
    "mixed": [0, 3, 17, 0, 1, 1, 0, 40, 2, 0, 0, 16, 16, 1],
}


def brute_nnz(rp, P):
    n = rp.size - 1
    nnz = int(rp[-1])
    b = [0]
    for p in range(1, P):
        t = (p * nnz) // P
        r = 0
        while r <= n and rp[r] < t:
            r += 1
        b.append(r)
    b.append(n)
    return np.array(b)


@pytest.mark.parametrize("case", sorted(ADVERSARIAL))
@pytest.mark.parametrize("T", [1, 3, 16, 1000])
def test_plan_nnz_brute(case, T):
    rp = _rp(ADVERSARIAL[case])
    b = oracle.plan_nnz(rp, T)
    P = b.size - 1
    assert P == max(1, -(-int(rp[-1]) // T))
    assert np.array_equal(b, brute_nnz(rp, P))
    assert b[0] == 0 and b[-1] == rp.size - 1 and np.all(np.diff(b) >= 0)


def brute_bss(rp, T):
    n = rp.size - 1
    nnz = int(rp[-1])
    P = max(1, -(-nnz // T))
    row_lo, tile_row, carry = [], [], []
    for t in range(P):
        e = t * T
        row_lo.append(next((r for r in range(n + 1) if rp[r] >= e), n))
        cand = [r for r in range(n + 1) if rp[r] <= e]
        tr = max(cand) if cand else 0
        tr = min(max(tr, 0), max(n - 1, 0))
        tile_row.append(tr)
        carry.append(tr if (n > 0 and rp[tr] < e) else -1)
    row_lo.append(n)
    tile_row.append(n)
    return np.array(row_lo), np.array(tile_row), np.array(carry)


@pytest.mark.parametrize("case", sorted(ADVERSARIAL))
@pytest.mark.parametrize("T", [1, 4, 16, 1000])
def test_plan_bss_brute(case, T):
    rp = _rp(ADVERSARIAL[case])
    got = oracle.plan_bss(rp, T)
    want = brute_bss(rp, T)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)


def _eval_bss(A, x, T):
    """Walk the BSS decomposition exactly as the plan defines it: each tile
    sums its entries per row; a row's first tile writes y, later tiles send
    their leading partial as a carry; carries are added in ascending tile
    order; empty rows are written 0 by the tile holding their start."""
    row_lo, tile_row, carry = oracle.plan_bss(A.rowptr, T)
    P = carry.size
    nnz = A.nnz
    y = np.full(A.n, np.nan)
    cval = np.zeros(P)
    for t in range(P):
        e0, e1 = t * T, min((t + 1) * T, nnz)
        # rows starting in this tile
        for r in range(row_lo[t], row_lo[t + 1]):
            k0, k1 = A.rowptr[r], min(A.rowptr[r + 1], e1)
            y[r] = sum(A.val[k] * x[A.colind[k]] for k in range(k0, k1))
        if carry[t] >= 0:
            r = carry[t]
            k1 = min(A.rowptr[r + 1], e1)
            cval[t] = sum(A.val[k] * x[A.colind[k]] for k in range(e0, k1))
    for t in range(P):
        if carry[t] >= 0:
            y[carry[t]] += cval[t]
    return y


@pytest.mark.parametrize("case", sorted(ADVERSARIAL))
@pytest.mark.parametrize("T", [1, 5, 16])
def test_bss_decomposition_is_exact(case, T):
    A = _mat(ADVERSARIAL[case], seed=3)
    x = gen.int_vec(A.ncols, 4)
    y, _ = oracle.spmv(A, x)
    assert np.array_equal(_eval_bss(A, x, T), y)


def _mat_sym(n, seed, band, p_empty=0.0):
    rng = np.random.default_rng(seed)
    rows, vals = [], []
    for i in range(n):
        lo = max(0, i - band)
        cand = np.arange(lo, i)
        keep = cand[rng.random(cand.size) < 0.5] if cand.size else cand
        if rng.random() < p_empty:
            keep = keep[:0]
        cols = np.concatenate([keep, [i]]).astype(np.int32)
        rows.append(cols)
    lens = [c.size for c in rows]
    rp = _rp(lens)
    ci = np.concatenate(rows).astype(np.int32)
    v = rng.integers(-8, 9, ci.size).astype(np.float64)
    return gen.CSR(n, n, rp, ci, v, sym_lower=True)


def brute_tiles(A, T, Rmax):
    """Tile starts: the nnz split; with Rmax >= 256 its inner boundaries
    rounded to the nearest multiple of 256 rows (capped at n), empty parts
    dropped, parts cut into pieces of whole 256-row groups as even as the
    groups allow; with Rmax < 256 parts cut into ceil(R / Rmax) even pieces."""
    rp = A.rowptr
    P0 = max(1, -(-A.nnz // T))
    b0 = list(brute_nnz(rp, P0))
    g = Rmax // 256
    if g:
        b0 = [b0[0]] + [min(A.n, 256 * ((v + 128) // 256)) for v in b0[1:-1]] + [b0[-1]]
    parts = [(b0[p], b0[p + 1]) for p in range(P0)]
    if P0 > 1:
        parts = [(lo, hi) for lo, hi in parts if hi > lo]
    b = []
    for lo, hi in parts:
        R = hi - lo
        if g:
            u = -(-R // 256)
            k = max(1, -(-u // g))
            b.extend(lo + 256 * ((i * u) // k) for i in range(k))
        else:
            k = max(1, -(-R // Rmax))
            b.extend(lo + (i * R) // k for i in range(k))
    b.append(A.n)
    return [int(v) for v in b]


def brute_sym(A, T, Rmax, C):
    rp, ci = A.rowptr, A.colind
    b = brute_tiles(A, T, Rmax)
    P = len(b) - 1
    pairs = set()
    for p in range(P):
        for i in range(b[p], b[p + 1]):
            for k in range(rp[i], rp[i + 1]):
                if ci[k] < b[p]:
                    pairs.add((int(ci[k]) // C, p))
    order = sorted(pairs)
    nblk = -(-A.n // C)
    tm_ptr = np.zeros(nblk + 1, dtype=np.int64)
    for c, _ in order:
        tm_ptr[c + 1] += 1
    tm_ptr = np.cumsum(tm_ptr)
    tm_tile = np.array([p for _, p in order])
    slot = {pc: s for s, pc in enumerate(order)}
    per_tile = sorted((p, c) for c, p in order)
    tile_ptr = np.zeros(P + 1, dtype=np.int64)
    for p, _ in per_tile:
        tile_ptr[p + 1] += 1
    tile_ptr = np.cumsum(tile_ptr)
    tile_blk = np.array([c for _, c in per_tile])
    tile_slot = np.array([slot[(c, p)] for p, c in per_tile])
    return dict(b=np.array(b), tm_ptr=tm_ptr, tm_tile=tm_tile, tile_ptr=tile_ptr, tile_blk=tile_blk,
                tile_slot=tile_slot)


SYM_CASES = [(60, 1, 5, 0.0), (80, 2, 20, 0.2), (200, 3, 70, 0.1), (1, 4, 1, 0.0), (33, 5, 0, 0.0)]


@pytest.mark.parametrize("n,seed,band,pe", SYM_CASES)
@pytest.mark.parametrize("T,Rmax,C", [(16, 8, 4), (40, 1000, 16), (7, 3, 1), (1000, 5, 64)])
def test_plan_sym_brute(n, seed, band, pe, T, Rmax, C):
    A = _mat_sym(n, seed, band, pe)
    got = oracle.plan_sym(A, T, Rmax, C)
    want = brute_sym(A, T, Rmax, C)
    for key in want:
        assert np.array_equal(got[key].astype(np.int64), want[key].astype(np.int64)), key


@pytest.mark.parametrize("n,band,pe", [(3000, 20, 0.0), (5000, 3, 0.3), (700, 60, 0.1), (256, 5, 0.0), (2, 1, 0.0)])
@pytest.mark.parametrize("T,Rmax", [(512, 256), (2000, 1024), (4096, 300), (100, 2048), (64, 700)])
def test_plan_sym_whole_groups(n, band, pe, T, Rmax):
    """With Rmax >= 256 every tile but the last holds a multiple of 256 rows
    (the sliced walk's rounds of four 64-row chunks are full), no tile holds
    more than Rmax rows, none is empty, and the tiles cover the rows in
    order; the tile starts are the brute-force ones."""
    A = _mat_sym(n, 11, band, pe)
    b = oracle.plan_sym(A, T, Rmax, 16)["b"].astype(np.int64)
    assert b[0] == 0 and b[-1] == A.n
    sizes = np.diff(b)
    assert np.all(sizes > 0) and np.all(sizes <= Rmax)
    assert np.all(sizes[:-1] % 256 == 0)
    assert list(b) == brute_tiles(A, T, Rmax)


def test_plan_sym_tiles_hand_case():
    """A hand-worked split: 1000 rows of 3 entries (3000 entries), T = 700
    gives 5 parts with boundaries at rows 233, 466, 700, 933 (entry counts
    699/700, 1398/1400, 2100, 2799/2800); rounded to 256 multiples: 256,
    512, 768, 1000 (933 rounds to 1024, capped at n); Rmax = 512 (two
    groups per piece) keeps them; Rmax = 256 cuts nothing further either."""
    lens = [1] + [2] + [3] * 998
    rows = []
    for i, L in enumerate(lens):
        rows.append(np.arange(i - L + 1, i + 1, dtype=np.int32))
    rp = _rp([r.size for r in rows])
    A = gen.CSR(1000, 1000, rp, np.concatenate(rows), np.ones(int(rp[-1])), sym_lower=True)
    assert A.nnz == 2997
    b = oracle.plan_sym(A, 700, 512, 16)["b"]
    assert list(b) == [0, 256, 512, 768, 1000]
    b = oracle.plan_sym(A, 700, 256, 16)["b"]
    assert list(b) == [0, 256, 512, 768, 1000]
    # one part of 1000 rows cut into pieces of at most 3 groups: u = 4, k = 2
    b = oracle.plan_sym(A, 1 << 20, 768, 16)["b"]
    assert list(b) == [0, 512, 1000]


def _eval_sym(A, x, plan, C):
    """Walk the symmetric decomposition: each tile forms its rows' own sums
    plus the transposed entries landing inside the tile; entries landing
    below the tile go to the (tile, block) partial named by the touch map;
    the reduction adds, block by block, the partials in the map's order."""
    b = plan["b"]
    P = b.size - 1
    y = np.zeros(A.n)
    nt = plan["tm_tile"].size
    part = np.zeros((nt, C))
    for p in range(P):
        slots = {int(c): int(s) for c, s in zip(plan["tile_blk"][plan["tile_ptr"][p]:plan["tile_ptr"][p + 1]],
                                                plan["tile_slot"][plan["tile_ptr"][p]:plan["tile_ptr"][p + 1]])}
        for i in range(b[p], b[p + 1]):
            for k in range(A.rowptr[i], A.rowptr[i + 1]):
                j = int(A.colind[k])
                y[i] += A.val[k] * x[j]
                if j != i:
                    if j >= b[p]:
                        y[j] += A.val[k] * x[i]
                    else:
                        part[slots[j // C], j % C] += A.val[k] * x[i]
    for c in range(plan["tm_ptr"].size - 1):
        for s in range(plan["tm_ptr"][c], plan["tm_ptr"][c + 1]):
            for jj in range(C):
                j = c * C + jj
                if j < A.n:
                    y[j] += part[s, jj]
    return y


@pytest.mark.parametrize("n,seed,band,pe", SYM_CASES)
def test_sym_decomposition_is_exact(n, seed, band, pe):
    A = _mat_sym(n, seed, band, pe)
    x = gen.int_vec(A.n, 8)
    y, _ = oracle.spmv(A, x)
    for T, Rmax, C in [(16, 8, 4), (9, 4, 2)]:
        plan = oracle.plan_sym(A, T, Rmax, C)
        assert np.array_equal(_eval_sym(A, x, plan, C), y)


def test_plan_sym_stencil_touch_is_sparse():
    """On a 3D stencil only a few column blocks per tile are touched: the
    zero-element omission skips almost the whole reduction vector."""
    A = gen.stencil27(16, lower=True)
    C = 64
    plan = oracle.plan_sym(A, 2048, 512, C)
    P = plan["b"].size - 1
    nblk = -(-A.n // C)
    per_tile = np.diff(plan["tile_ptr"])
    assert per_tile.max() <= 12
    assert plan["tm_tile"].size < 0.2 * P * nblk


@pytest.mark.parametrize("case", sorted(ADVERSARIAL))
@pytest.mark.parametrize("nb", [1, 3, 8])
def test_plan_xcb_brute(case, nb):
    """Column blocks k = [floor(k ncols/nb), floor((k+1) ncols/nb)): per-block
    row pointers and the concatenated, order-preserving column lists."""
    A = _mat(ADVERSARIAL[case], seed=2, ncols=50)
    rp, ci = oracle.plan_xcb(A, nb)
    bounds = [(k * A.ncols) // nb for k in range(nb + 1)]
    want_ci = []
    for k in range(nb):
        cnt = [0]
        for i in range(A.n):
            row = [int(c) for c in A.colind[A.rowptr[i]:A.rowptr[i + 1]] if bounds[k] <= c < bounds[k + 1]]
            want_ci.extend(row)
            cnt.append(cnt[-1] + len(row))
        assert np.array_equal(rp[k], np.array(cnt))
    assert np.array_equal(ci, np.array(want_ci, dtype=np.int32))


def test_xcb_decomposition_is_exact():
    """Summing the per-block products reproduces A x exactly (integers)."""
    A = _mat([3, 0, 7, 1, 12, 0, 5] * 5, seed=4, ncols=40)
    x = gen.int_vec(A.ncols, 2)
    rp, ci = oracle.plan_xcb(A, 8)
    # values follow their column in the same stable order
    vals = []
    bounds = [(k * A.ncols) // 8 for k in range(9)]
    for k in range(8):
        for i in range(A.n):
            for e in range(A.rowptr[i], A.rowptr[i + 1]):
                if bounds[k] <= A.colind[e] < bounds[k + 1]:
                    vals.append(A.val[e])
    y = np.zeros(A.n)
    base = 0
    for k in range(8):
        for i in range(A.n):
            for q in range(base + rp[k][i], base + rp[k][i + 1]):
                y[i] += vals[q] * x[ci[q]]
        base += rp[k][A.n]
    assert np.array_equal(y, oracle.spmv(A, x)[0])


@pytest.mark.parametrize("case", sorted(ADVERSARIAL))
@pytest.mark.parametrize("nb", [1, 3, 8])
def test_xcb_flags_brute(case, nb):
    """Bit 31 is set exactly on the first entry of every row of every block;
    clearing it gives back the unflagged columns."""
    A = _mat(ADVERSARIAL[case], seed=3, ncols=50)
    rp, ci = oracle.plan_xcb(A, nb)
    _, cf = oracle.plan_xcb(A, nb, flagged=True)
    want = ci.copy()
    base = 0
    for k in range(nb):
        for i in range(A.n):
            if rp[k][i + 1] > rp[k][i]:
                want[base + rp[k][i]] = np.int32(int(want[base + rp[k][i]]) - 2**31)
        base += rp[k][A.n]
    assert np.array_equal(cf, want)
    assert np.array_equal(cf & 0x7FFFFFFF, ci)


def test_xcb_flag_walk_is_exact():
    """Walking each block's flagged entries in order, counting heads to find
    compressed rows (no row pointers), and adding the block partials in
    block order reproduces A x exactly (integers): the decoding the
    column-blocked kernel performs."""
    A = _mat([3, 0, 7, 1, 12, 0, 5, 0, 0, 1] * 4, seed=6, ncols=40)
    x = gen.int_vec(A.ncols, 2)
    rp, cf = oracle.plan_xcb(A, 8, flagged=True)
    bounds = [(k * A.ncols) // 8 for k in range(9)]
    vals = [A.val[e] for k in range(8) for i in range(A.n) for e in range(A.rowptr[i], A.rowptr[i + 1])
            if bounds[k] <= A.colind[e] < bounds[k + 1]]
    y = np.zeros(A.n)
    base = 0
    for k in range(8):
        rows = [i for i in range(A.n) if rp[k][i + 1] > rp[k][i]]  # the block's compressed rows
        nk = int(rp[k][A.n])
        part = np.zeros(len(rows))
        r = -1
        for q in range(base, base + nk):
            if cf[q] < 0:
                r += 1
            part[r] += vals[q] * x[cf[q] & 0x7FFFFFFF]
        assert r == len(rows) - 1
        for j, i in enumerate(rows):
            y[i] += part[j]
        base += nk
    assert np.array_equal(y, oracle.spmv(A, x)[0])


# ------------------------------------------------------------------ SELL-C-sigma
def _sell_brute(A, C, sigma):
    lens = np.diff(A.rowptr)
    perm = []
    for w0 in range(0, A.n, sigma):
        perm += sorted(range(w0, min(w0 + sigma, A.n)), key=lambda r: (-lens[r], r))
    rlen = [int(lens[r]) for r in perm]
    clen = [max(rlen[c:c + C]) for c in range(0, A.n, C)]
    cptr = [0]
    for w in clen:
        cptr.append(cptr[-1] + w * C)
    cols = np.zeros(cptr[-1], dtype=np.int32)
    vals = np.zeros(cptr[-1])
    for r, row in enumerate(perm):
        c, l = divmod(r, C)
        for k in range(rlen[r]):
            cols[cptr[c] + k * C + l] = A.colind[A.rowptr[row] + k]
            vals[cptr[c] + k * C + l] = A.val[A.rowptr[row] + k]
    return perm, rlen, clen, cptr, cols, vals


@pytest.mark.parametrize("case", sorted(ADVERSARIAL))
@pytest.mark.parametrize("C,sigma", [(4, 4), (4, 16), (64, 64), (2, 8)])
def test_plan_sell_brute(case, C, sigma):
    """Rows ordered longest first inside each sigma-window (ties by row),
    chunks of C padded column-major to their longest row."""
    A = _mat(ADVERSARIAL[case] * 3, seed=5, ncols=60)
    p = oracle.plan_sell(A, C, sigma)
    perm, rlen, clen, cptr, cols, vals = _sell_brute(A, C, sigma)
    assert p["perm"].tolist() == perm and p["rlen"].tolist() == rlen
    assert p["clen"].tolist() == clen and p["cptr"].tolist() == cptr
    assert np.array_equal(p["cols"], cols) and np.array_equal(p["vals"], vals)


def test_sell_walk_is_exact():
    """Row sums over the padded chunks, written back through perm, give A x
    exactly (integer values)."""
    A = _mat([3, 0, 7, 1, 12, 0, 5, 9, 9, 2] * 13, seed=7, ncols=90)
    x = gen.int_vec(A.ncols, 2)
    C = 8
    p = oracle.plan_sell(A, C, 32)
    y = np.full(A.n, np.nan)
    for r in range(A.n):
        c, l = divmod(r, C)
        s = 0.0
        for k in range(p["rlen"][r]):
            q = p["cptr"][c] + k * C + l
            s += p["vals"][q] * x[p["cols"][q]]
        y[p["perm"][r]] = s
    assert np.array_equal(y, oracle.spmv(A, x)[0])


# ------------------------------------------------------------------ BCSR
def _bcsr_brute(A, b):
    """Block CSR from its definition, by dictionaries."""
    nbr = (A.n + b - 1) // b
    brp, bci, bmask, bval = [0], [], [], []
    for R in range(nbr):
        blocks = {}
        for r in range(R * b, min(R * b + b, A.n)):
            for k in range(A.rowptr[r], A.rowptr[r + 1]):
                c = int(A.colind[k])
                blk = blocks.setdefault(c // b, [0, np.zeros(b * b)])
                e = (r - R * b) * b + c % b
                blk[0] |= 1 << e
                blk[1][e] += A.val[k]
        for cb in sorted(blocks):
            bci.append(cb)
            bmask.append(blocks[cb][0])
            bval.append(blocks[cb][1])
        brp.append(len(bci))
    return np.array(brp), np.array(bci), np.array(bmask), np.array(bval).reshape(-1, b * b)


@pytest.mark.parametrize("lengths,ncols,b", [
    ([3, 0, 7, 1, 12, 0, 5, 9, 9, 2] * 7, 90, 4),
    ([0] * 9, 9, 4),                       # all empty
    ([1] * 13, 13, 4),                     # ragged last block row
    ([30, 0, 0, 30, 5], 31, 4),            # columns near the end, empty rows inside a block row
    ([3, 3, 3], 7, 2),
])
def test_bcsr_brute(lengths, ncols, b):
    A = _mat(lengths, seed=11, ncols=ncols)
    p = oracle.plan_bcsr(A, b)
    brp, bci, bmask, bval = _bcsr_brute(A, b)
    assert np.array_equal(p["brp"], brp)
    assert np.array_equal(p["bci"], bci.astype(np.int32).reshape(-1))
    assert np.array_equal(p["bmask"], bmask.astype(np.uint32).reshape(-1))
    assert np.array_equal(p["bval"], bval.reshape(-1, b * b) if bval.size else p["bval"])


def test_bcsr_duplicates_summed_and_dense_reconstruction():
    rp = np.array([0, 3, 3, 5], dtype=np.int32)
    ci = np.array([2, 2, 5, 0, 5], dtype=np.int32)   # (0, 2) twice
    v = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    A = gen.CSR(3, 6, rp, ci, v)
    p = oracle.plan_bcsr(A, 4)
    D = np.zeros((4, 8))
    for q, cb in enumerate(p["bci"]):
        D[:, cb * 4:cb * 4 + 4] += p["bval"][q].reshape(4, 4)
    want = np.zeros((4, 8))
    want[0, 2], want[0, 5], want[2, 0], want[2, 5] = 3.0, 3.0, 4.0, 5.0
    assert np.array_equal(D, want)
    assert list(p["bmask"]) == [(1 << 2) | (1 << 8), 1 << 1 | 1 << 9]


def test_bcsr_walk_is_exact():
    """Block-row sums over the masked block entries reproduce A x exactly
    (integer values)."""
    A = _mat([3, 0, 7, 1, 12, 0, 5, 9, 9, 2] * 13, seed=7, ncols=90)
    x = gen.int_vec(A.ncols, 2)
    b = 4
    p = oracle.plan_bcsr(A, b)
    y = np.zeros(A.n)
    for R in range(len(p["brp"]) - 1):
        for q in range(p["brp"][R], p["brp"][R + 1]):
            for e in range(b * b):
                if p["bmask"][q] >> e & 1:
                    r, c = R * b + e // b, p["bci"][q] * b + e % b
                    y[r] += p["bval"][q][e] * x[c]
    assert np.array_equal(y, oracle.spmv(A, x)[0])


# ------------------------------------------------- symmetric walk: deferred adds
def _colflags_brute(A, b, lanes, J):
    """Per tile, a dictionary of (chunk, slot, column) seen so far in stream
    order: an entry whose key was seen gets bit 30; each non-empty row's
    first entry gets bit 31."""
    CH = lanes * J
    rp = A.rowptr.astype(np.int64)
    out = A.colind.astype(np.int64) & 0xFFFFFFFF
    for p in range(len(b) - 1):
        seen = set()
        for q in range(rp[b[p]], rp[b[p + 1]]):
            key = (q // CH, q % J, int(A.colind[q]))
            if key in seen:
                out[q] |= 1 << 30
            seen.add(key)
    for i in range(A.n):
        if rp[i + 1] > rp[i]:
            out[rp[i]] |= 1 << 31
    return out.astype(np.uint32).view(np.int32)


@pytest.mark.parametrize("n,seed,band,pe", SYM_CASES)
@pytest.mark.parametrize("lanes,J", [(4, 2), (2, 3), (64, 8), (1, 1)])
def test_sym_colflags_brute(n, seed, band, pe, lanes, J):
    A = _mat_sym(n, seed, band, pe)
    for T, Rmax in ((16, 8), (40, 1000), (7, 3)):
        b = oracle.plan_sym(A, T, Rmax, 4)["b"]
        got = oracle.plan_sym_colflags(A, b, lanes, J)
        assert np.array_equal(got, _colflags_brute(A, b, lanes, J))


def test_sym_colflags_hand_case():
    """Chunks of 4 lanes x 2 entries (8 entries, slot = position % 2).
    Rows (columns): 0: 0 | 1: 0 1 | 2: 0 2 | 3: 0 1 3 | 4: 0 4, so the
    stream's columns are 0 0 1 0 2 0 1 3 | 0 4 (chunk 0 | chunk 1).
    One tile: slot 1 holds column 0 at positions 1, 3, 5 (3 and 5 flagged),
    slot 0 holds column 1 at positions 2 and 6 (6 flagged); column 0 at
    position 8 is in chunk 1 and at 0, 4 in the other slot (not flagged).
    Tiles [0, 2) and [2, 5): position 2 belongs to the first tile, so 6 is
    no longer flagged, and neither is 3 (position 1 is in the first tile)."""
    rows = [[0], [0, 1], [0, 2], [0, 1, 3], [0, 4]]
    rp = _rp([len(r) for r in rows])
    ci = np.concatenate(rows).astype(np.int32)
    A = gen.CSR(5, 5, rp, ci, np.ones(ci.size), sym_lower=True)
    got = oracle.plan_sym_colflags(A, np.array([0, 5]), 4, 2)
    assert [(int(v) >> 30) & 1 for v in got] == [0, 0, 0, 1, 0, 1, 1, 0, 0, 0]
    assert [(int(v) >> 31) & 1 for v in got] == [1, 1, 0, 1, 0, 1, 0, 0, 1, 0]
    assert [int(v) & 0x3FFFFFFF for v in got] == list(ci)
    got2 = oracle.plan_sym_colflags(A, np.array([0, 2, 5]), 4, 2)
    assert [(int(v) >> 30) & 1 for v in got2] == [0, 0, 0, 0, 0, 1, 0, 0, 0, 0]


@pytest.mark.parametrize("n,seed,band,pe", SYM_CASES)
def test_sym_colflags_make_slots_distinct(n, seed, band, pe):
    """What the kernel relies on: inside a tile, the entries of one chunk
    and slot that are not flagged have distinct columns."""
    A = _mat_sym(n, seed, band, pe)
    lanes, J = 4, 2
    b = oracle.plan_sym(A, 16, 8, 4)["b"]
    f = oracle.plan_sym_colflags(A, b, lanes, J).view(np.uint32)
    rp = A.rowptr
    for p in range(len(b) - 1):
        groups = {}
        for q in range(rp[b[p]], rp[b[p + 1]]):
            if not (f[q] >> 30) & 1:
                key = (q // (lanes * J), q % J)
                groups.setdefault(key, []).append(int(f[q] & 0x3FFFFFFF))
        for cols in groups.values():
            assert len(cols) == len(set(cols))


# ------------------------------------------------- symmetric walk: sliced layout
def _slices_brute(A, b, lanes):
    """Per tile, per chunk of `lanes` rows: a dense (width x rows) table of
    columns (-1 past a row's end) read out slot-major; a column already seen
    at the same slot of the chunk gets bit 30."""
    rp = A.rowptr.astype(np.int64)
    ch0, cw, coff, cols = [], [], [0], []
    for p in range(len(b) - 1):
        ch0.append(len(cw))
        for rc in range(b[p], b[p + 1], lanes):
            rows = list(range(rc, min(rc + lanes, b[p + 1])))
            lens = [rp[i + 1] - rp[i] for i in rows]
            w = max(lens)
            cw.append(w)
            for k in range(w):
                seen = set()
                for i, ln in zip(rows, lens):
                    c = int(A.colind[rp[i] + k]) if k < ln else -1
                    v = c
                    if c >= 0:
                        if c in seen:
                            v = c | (1 << 30)
                        seen.add(c)
                    cols.append(v)
            coff.append(coff[-1] + w * len(rows))
    ch0.append(len(cw))
    return dict(ch0=np.array(ch0), cw=np.array(cw, dtype=np.int64), coff=np.array(coff),
                cols=np.array(cols, dtype=np.int64).astype(np.uint32).view(np.int32))


@pytest.mark.parametrize("n,seed,band,pe", SYM_CASES)
@pytest.mark.parametrize("lanes", [1, 3, 4, 64])
def test_sym_slices_brute(n, seed, band, pe, lanes):
    A = _mat_sym(n, seed, band, pe)
    for T, Rmax in ((16, 8), (40, 1000), (7, 3)):
        b = oracle.plan_sym(A, T, Rmax, 4)["b"]
        got = oracle.plan_sym_slices(A, b, lanes)
        want = _slices_brute(A, b, lanes)
        for key in ("ch0", "cw", "coff", "cols"):
            assert np.array_equal(got[key].astype(np.int64), want[key].astype(np.int64)), key


def _eval_slices(A, x, b, lay, lanes):
    """Walk the sliced layout the way the product does: per chunk, slot by
    slot, each row adds its entry to its own sum and, below the diagonal,
    the transposed product to row j; integer values make every order exact."""
    y = np.zeros(A.n)
    val = {}
    rp = A.rowptr
    for i in range(A.n):
        for q in range(rp[i], rp[i + 1]):
            val[(i, int(A.colind[q]))] = val.get((i, int(A.colind[q])), 0.0) + A.val[q]
    g = 0
    for p in range(len(b) - 1):
        for rc in range(b[p], b[p + 1], lanes):
            nr = min(lanes, b[p + 1] - rc)
            w, o = lay["cw"][g], lay["coff"][g]
            cnt = {}
            for k in range(w):
                for l in range(nr):
                    c = int(lay["cols"][o + k * nr + l])
                    if c == -1:
                        continue
                    j, i = c & 0x3FFFFFFF, rc + l
                    kk = cnt.get((i, j), 0)  # the k-th stored (i, j) entry (duplicates are summed)
                    cnt[(i, j)] = kk + 1
                    ks = [q for q in range(rp[i], rp[i + 1]) if A.colind[q] == j]
                    a = A.val[ks[kk]]
                    y[i] += a * x[j]
                    if j < i:
                        y[j] += a * x[i]
            g += 1
    return y


@pytest.mark.parametrize("n,seed,band,pe", SYM_CASES[:3])
def test_sym_slices_walk_is_exact(n, seed, band, pe):
    A = _mat_sym(n, seed, band, pe)
    x = gen.int_vec(A.n, 8)
    y, _ = oracle.spmv(A, x)
    for T, Rmax, lanes in ((16, 8, 4), (40, 1000, 64), (7, 3, 3)):
        b = oracle.plan_sym(A, T, Rmax, 4)["b"]
        lay = oracle.plan_sym_slices(A, b, lanes)
        assert np.array_equal(_eval_slices(A, x, b, lay, lanes), y)


def test_sym_slices_slots_distinct_and_walk_rule():
    """Unflagged entries of one chunk and slot have distinct columns; the
    27-point stencil takes the sliced walk (little padding), a lower
    triangle with rows of very different lengths does not."""
    A = gen.stencil27(12, lower=True)
    b = oracle.plan_sym(A, 2048, 512, 64)["b"]
    lay = oracle.plan_sym_slices(A, b)
    assert lay["sliced"]
    cols = lay["cols"].view(np.uint32)
    for g in range(len(lay["cw"])):
        o, w = lay["coff"][g], lay["cw"][g]
        nr = (lay["coff"][g + 1] - o) // max(w, 1) if w else 0
        for k in range(w):
            s = cols[o + k * nr:o + (k + 1) * nr]
            live = s[(s != 0xFFFFFFFF) & ((s >> 30) & 1 == 0)] & 0x3FFFFFFF
            assert len(live) == len(set(live.tolist()))
    rng = np.random.default_rng(3)
    rows = [np.unique(np.r_[rng.integers(0, i + 1, int(rng.integers(1, 60)) if i % 9 == 0 else 1), i])
            for i in range(400)]
    rp = _rp([r.size for r in rows])
    ci = np.concatenate(rows).astype(np.int32)
    B = gen.CSR(400, 400, rp, ci, np.ones(ci.size), sym_lower=True)
    bb = oracle.plan_sym(B, 2048, 512, 64)["b"]
    assert not oracle.plan_sym_slices(B, bb)["sliced"]

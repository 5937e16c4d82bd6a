"""CPU oracle (ctypes wrapper over liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the benchmark's CPU-baseline leg, never by the product path.  Serial,
plain FP64; see oracle.h for what each routine follows.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None
F_FEATURES = 12
HIDDEN = 64


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            raise RuntimeError(f"oracle library missing: {_build.LIB} (run __graft_entry__.build())")
        L = ctypes.CDLL(_build.LIB)
        P = ctypes.c_void_p
        i64, i32, d, ci = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_int
        sig = {
            "orc_spmv_csr": (None, [i64, P, P, P, P, P, P]),
            "orc_spmv_rows": (None, [i64, P, P, P, P, P, P, P]),
            "orc_sym_expand": (i64, [i64, P, P, P, P, P, P]),
            "orc_spmv_sym": (ci, [i64, P, P, P, P, P, P]),
            "orc_nparts": (i64, [i64, i64]),
            "orc_plan_nnz": (None, [i64, P, i64, P]),
            "orc_plan_bss": (None, [i64, P, i64, i64, P, P, P]),
            "orc_plan_sym_ntiles": (i64, [i64, P, i64, i64]),
            "orc_plan_sym_tiles": (None, [i64, P, i64, i64, P]),
            "orc_plan_sym_touch": (i64, [i64, P, P, i64, P, i64, P, P, P, P, P]),
            "orc_plan_xcb": (None, [i64, i64, P, P, ci, P, P]),
            "orc_xcb_flag_heads": (None, [i64, ci, P, P]),
            "orc_plan_sym_colflags": (None, [i64, P, P, i64, P, i64, i64, P]),
            "orc_plan_sym_slices": (i64, [i64, P, P, i64, P, i64, P, P, P, P, P, P]),
            "orc_sym_walk_sliced": (ci, [i64, i64, i64]),
            "orc_plan_sell": (i64, [i64, P, P, P, ci, ci, P, P, P, P, P, P]),
            "orc_plan_bcsr": (i64, [i64, P, P, P, ci, P, P, P, P]),
            "orc_features": (None, [i64, P, P, ci, P, P]),
            "orc_mlp_nparams": (i64, [ci, ci, ci]),
            "orc_mlp_forward": (None, [ci, ci, ci, P, i64, P, P]),
            "orc_mlp_loss_grad": (d, [ci, ci, ci, P, i64, P, P, P, P]),
            "orc_adam_step": (None, [i64, P, P, P, P, i64, d, d, d, d]),
            "orc_mlp_train": (None, [ci, ci, ci, P, i64, P, P, P, P, ci, ci, d, P]),
            "orc_gmres": (ci, [i64, P, P, P, P, P, ci, d, i64, ci, P, P, P, P]),
            "orc_mm_ratio": (d, [P, i64, i64]),
            "orc_gmres_at": (ci, [i64, P, P, P, P, P, ci, ci, ci, d, d, i64, ci, P, P, P, P, P, ci, P]),
            "orc_bicgstab": (ci, [i64, P, P, P, P, P, d, i64, ci, P, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _csr(A):
    rp = np.ascontiguousarray(A.rowptr, dtype=np.int32)
    ci = np.ascontiguousarray(A.colind, dtype=np.int32)
    v = np.ascontiguousarray(A.val, dtype=np.float64)
    return rp, ci, v


# ------------------------------------------------------------------ SpMV
def spmv(A, x):
    """(y, s): y = A x with compensated row sums, s_i = sum |a_ij x_j|.
    Symmetric lower-stored matrices are expanded first."""
    rp, ci, v = _csr(A)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(A.n, dtype=np.float64)
    s = np.empty(A.n, dtype=np.float64)
    if A.sym_lower:
        if lib().orc_spmv_sym(A.n, _p(rp), _p(ci), _p(v), _p(x), _p(y), _p(s)) != 0:
            raise MemoryError("oracle expansion failed")
    else:
        lib().orc_spmv_csr(A.n, _p(rp), _p(ci), _p(v), _p(x), _p(y), _p(s))
    return y, s


def spmv_rows(A, x, rows):
    """Rows `rows` of A x (general storage only), with their s_i."""
    rp, ci, v = _csr(A)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(rows.size, dtype=np.float64)
    s = np.empty(rows.size, dtype=np.float64)
    lib().orc_spmv_rows(rows.size, _p(rows), _p(rp), _p(ci), _p(v), _p(x), _p(y), _p(s))
    return y, s


def sym_expand(A):
    """Full storage of a lower-stored symmetric matrix: (rowptr, colind, val)."""
    rp, ci, v = _csr(A)
    nnz = lib().orc_sym_expand(A.n, _p(rp), _p(ci), _p(v), None, None, None)
    rpf = np.empty(A.n + 1, dtype=np.int32)
    cif = np.empty(nnz, dtype=np.int32)
    vf = np.empty(nnz, dtype=np.float64)
    lib().orc_sym_expand(A.n, _p(rp), _p(ci), _p(v), _p(rpf), _p(cif), _p(vf))
    return rpf, cif, vf


# ------------------------------------------------------------------ plans
def nparts(nnz, T):
    return int(lib().orc_nparts(nnz, T))


def plan_nnz(rowptr, T):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    n = rowptr.size - 1
    P = nparts(int(rowptr[-1]), T)
    b = np.empty(P + 1, dtype=np.int32)
    lib().orc_plan_nnz(n, _p(rowptr), P, _p(b))
    return b


def plan_bss(rowptr, T):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    n = rowptr.size - 1
    P = nparts(int(rowptr[-1]), T)
    row_lo = np.empty(P + 1, dtype=np.int32)
    tile_row = np.empty(P + 1, dtype=np.int32)
    carry = np.empty(P, dtype=np.int32)
    lib().orc_plan_bss(n, _p(rowptr), T, P, _p(row_lo), _p(tile_row), _p(carry))
    return row_lo, tile_row, carry


def plan_sym(A, T, Rmax, C):
    """dict with b (tiles), tm_ptr, tm_tile, tile_ptr, tile_blk, tile_slot."""
    rp, ci, _ = _csr(A)
    n = A.n
    P = int(lib().orc_plan_sym_ntiles(n, _p(rp), T, Rmax))
    b = np.empty(P + 1, dtype=np.int32)
    lib().orc_plan_sym_tiles(n, _p(rp), T, Rmax, _p(b))
    nt = int(lib().orc_plan_sym_touch(n, _p(rp), _p(ci), P, _p(b), C, None, None, None, None, None))
    nblk = (n + C - 1) // C
    tm_ptr = np.empty(nblk + 1, dtype=np.int32)
    tm_tile = np.empty(max(nt, 1), dtype=np.int32)
    tile_ptr = np.empty(P + 1, dtype=np.int32)
    tile_blk = np.empty(max(nt, 1), dtype=np.int32)
    tile_slot = np.empty(max(nt, 1), dtype=np.int32)
    lib().orc_plan_sym_touch(n, _p(rp), _p(ci), P, _p(b), C, _p(tm_ptr), _p(tm_tile), _p(tile_ptr),
                             _p(tile_blk), _p(tile_slot))
    return dict(b=b, tm_ptr=tm_ptr, tm_tile=tm_tile[:nt], tile_ptr=tile_ptr, tile_blk=tile_blk[:nt],
                tile_slot=tile_slot[:nt])


def plan_sym_colflags(A, b, lanes=64, J=8):
    """The symmetric walk's column copy for tiles b: bit 31 on each non-empty
    row's first entry, bit 30 on an entry added after its chunk's slots."""
    rp, ci, _ = _csr(A)
    out = np.empty(max(A.nnz, 1), dtype=np.int32)
    bb = np.ascontiguousarray(b, dtype=np.int32)
    lib().orc_plan_sym_colflags(A.n, _p(rp), _p(ci), len(bb) - 1, _p(bb), lanes, J, _p(out))
    return out[:A.nnz]


def plan_sym_slices(A, b, lanes=64):
    """The symmetric product's sliced layout for tiles b: dict with ch0,
    cw, coff, cols (bit 30 on an entry a lower lane of its slot meets) and
    `sliced`, whether the product takes this walk."""
    rp, ci, _ = _csr(A)
    bb = np.ascontiguousarray(b, dtype=np.int32)
    P = len(bb) - 1
    nch, widest = ctypes.c_int64(), ctypes.c_int64()
    tot = int(lib().orc_plan_sym_slices(A.n, _p(rp), _p(ci), P, _p(bb), lanes, None, None, None, None,
                                        ctypes.byref(nch), ctypes.byref(widest)))
    ch0 = np.empty(P + 1, dtype=np.int32)
    cw = np.empty(max(nch.value, 1), dtype=np.int32)
    coff = np.empty(nch.value + 1, dtype=np.int64)
    cols = np.empty(max(tot, 1), dtype=np.int32)
    lib().orc_plan_sym_slices(A.n, _p(rp), _p(ci), P, _p(bb), lanes, _p(ch0), _p(cw), _p(coff), _p(cols),
                              ctypes.byref(nch), ctypes.byref(widest))
    return dict(ch0=ch0, cw=cw[:nch.value], coff=coff, cols=cols[:tot], widest=widest.value,
                sliced=bool(lib().orc_sym_walk_sliced(A.nnz, tot, widest.value)))


def plan_xcb(A, nb=8, flagged=False):
    """Column-blocked split: (rp[nb, n+1] relative row pointers, concatenated
    colind); with flagged=True the first entry of each row of each block
    carries bit 31 in its column index."""
    rp, ci, _ = _csr(A)
    out_rp = np.empty((nb, A.n + 1), dtype=np.int32)
    out_ci = np.empty(max(A.nnz, 1), dtype=np.int32)
    lib().orc_plan_xcb(A.n, A.ncols, _p(rp), _p(ci), nb, _p(out_rp), _p(out_ci))
    if flagged:
        lib().orc_xcb_flag_heads(A.n, nb, _p(out_rp), _p(out_ci))
    return out_rp, out_ci[:A.nnz]


def plan_sell(A, C=64, sigma=1024):
    """SELL-C-sigma layout: dict(perm, cptr, clen, rlen, cols, vals)."""
    rp, ci, v = _csr(A)
    n = A.n
    nch = (n + C - 1) // C
    perm = np.empty(max(n, 1), dtype=np.int32)
    rlen = np.empty(max(n, 1), dtype=np.int32)
    cptr = np.empty(nch + 1, dtype=np.int64)
    clen = np.empty(max(nch, 1), dtype=np.int32)
    tot = lib().orc_plan_sell(n, _p(rp), _p(ci), _p(v), C, sigma, _p(perm), _p(cptr), _p(clen), _p(rlen), None, None)
    cols = np.empty(max(tot, 1), dtype=np.int32)
    vals = np.empty(max(tot, 1), dtype=np.float64)
    lib().orc_plan_sell(n, _p(rp), _p(ci), _p(v), C, sigma, _p(perm), _p(cptr), _p(clen), _p(rlen), _p(cols), _p(vals))
    return dict(perm=perm[:n], cptr=cptr, clen=clen[:nch], rlen=rlen[:n], cols=cols[:tot], vals=vals[:tot])


def plan_bcsr(A, b=4):
    """Block CSR layout: dict(brp int64[nbr+1], bci int32[nb], bmask uint32[nb],
    bval float64[nb, b*b])."""
    rp, ci, v = _csr(A)
    n = A.n
    nbr = (n + b - 1) // b
    brp = np.empty(nbr + 1, dtype=np.int64)
    nb = lib().orc_plan_bcsr(n, _p(rp), _p(ci), _p(v), b, _p(brp), None, None, None)
    bci = np.empty(max(nb, 1), dtype=np.int32)
    bmask = np.empty(max(nb, 1), dtype=np.uint32)
    bval = np.empty((max(nb, 1), b * b), dtype=np.float64)
    lib().orc_plan_bcsr(n, _p(rp), _p(ci), _p(v), b, _p(brp), _p(bci), _p(bmask), _p(bval))
    return dict(brp=brp, bci=bci[:nb], bmask=bmask[:nb], bval=bval[:nb])


# ------------------------------------------------------------------ features
def features(A):
    """(stats int64[9], features float64[12]); see oracle.h."""
    rp, ci, _ = _csr(A)
    st = np.empty(9, dtype=np.int64)
    f = np.empty(F_FEATURES, dtype=np.float64)
    lib().orc_features(A.n, _p(rp), _p(ci), int(A.sym_lower), _p(st), _p(f))
    return st, f


# ------------------------------------------------------------------ MLP
def mlp_nparams(K, F=F_FEATURES, H=HIDDEN):
    return int(lib().orc_mlp_nparams(F, H, K))


def mlp_forward(params, feat, K, F=F_FEATURES, H=HIDDEN):
    p = np.ascontiguousarray(params, dtype=np.float64)
    f = np.ascontiguousarray(feat, dtype=np.float64).reshape(-1, F)
    out = np.empty((f.shape[0], K), dtype=np.float64)
    lib().orc_mlp_forward(F, H, K, _p(p), f.shape[0], _p(f), _p(out))
    return out


def mlp_loss_grad(params, feat, y, mask, K, F=F_FEATURES, H=HIDDEN):
    p = np.ascontiguousarray(params, dtype=np.float64)
    f = np.ascontiguousarray(feat, dtype=np.float64).reshape(-1, F)
    y = np.ascontiguousarray(y, dtype=np.float64).reshape(-1, K)
    m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1, K)
    g = np.empty(p.size, dtype=np.float64)
    loss = lib().orc_mlp_loss_grad(F, H, K, _p(p), f.shape[0], _p(f), _p(y), _p(m), _p(g))
    return float(loss), g


def adam_step(params, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In place on params, m, v (all float64)."""
    lib().orc_adam_step(params.size, _p(params), _p(np.ascontiguousarray(grad, dtype=np.float64)), _p(m),
                        _p(v), t, lr, b1, b2, eps)


def mlp_train(params, feat, y, mask, order, epochs, batch, lr, K, F=F_FEATURES, H=HIDDEN):
    p = np.array(params, dtype=np.float64)
    f = np.ascontiguousarray(feat, dtype=np.float64).reshape(-1, F)
    y = np.ascontiguousarray(y, dtype=np.float64).reshape(-1, K)
    m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1, K)
    order = np.ascontiguousarray(order, dtype=np.int32)
    losses = np.empty(epochs, dtype=np.float64)
    lib().orc_mlp_train(F, H, K, _p(p), f.shape[0], _p(f), _p(y), _p(m), _p(order), epochs, batch, lr,
                        _p(losses))
    return p, losses


# ------------------------------------------------------------------ Krylov
def gmres(A, b, x0=None, m=30, tol=1e-10, maxiter=10000, precond=0, history=False):
    rp, ci, v = _csr(A)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64)
    info = np.zeros(3, dtype=np.int64)
    dinfo = np.zeros(1, dtype=np.float64)
    hist = np.full(maxiter + 1, np.nan) if history else None
    aerr = np.zeros(1, dtype=np.float64) if history else None
    lib().orc_gmres(A.n, _p(rp), _p(ci), _p(v), _p(b), _p(x), m, tol, maxiter, precond, _p(info), _p(dinfo),
                    _p(hist), _p(aerr))
    out = dict(x=x, iters=int(info[0]), cycles=int(info[1]), status=int(info[2]), relres=float(dinfo[0]))
    if history:
        out["hist"] = hist[: out["iters"] + 1]
        out["arnoldi_err"] = float(aerr[0])
    return out


def mm_ratio(r, s, t):
    """Eq. (1): max / min of r(z), z = s-t+1 .. s (1-based samples)."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    return float(lib().orc_mm_ratio(_p(r), s, t))


ORTHO_DGKS, ORTHO_CGS, ORTHO_MGS, ORTHO_BCGS, ORTHO_POLICY = 0, 1, 2, 3, 4


def gmres_at(A, b, m0, m_max, step, ratio, x0=None, tol=1e-10, maxiter=10000, precond=0, ortho=ORTHO_MGS,
             history=False):
    """GMRES with the restart length tuned by the MM ratio after every cycle
    (step > 0) and a choice of orthogonalisation; returns the solve summary,
    the m of every cycle and [faults, final ortho]."""
    rp, ci, v = _csr(A)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64)
    info = np.zeros(3, dtype=np.int64)
    dinfo = np.zeros(1, dtype=np.float64)
    mh = np.zeros(maxiter + 1, dtype=np.int32)
    pol = np.zeros(2, dtype=np.int32)
    hist = np.full(maxiter + 1, np.nan) if history else None
    aerr = np.zeros(1, dtype=np.float64) if history else None
    lib().orc_gmres_at(A.n, _p(rp), _p(ci), _p(v), _p(b), _p(x), m0, m_max, step, ratio, tol, maxiter, precond,
                       _p(info), _p(dinfo), _p(hist), _p(aerr), _p(mh), ortho, _p(pol))
    out = dict(x=x, iters=int(info[0]), cycles=int(info[1]), status=int(info[2]), relres=float(dinfo[0]))
    out["m_hist"] = mh[: out["cycles"]].tolist()
    out["faults"], out["ortho"] = int(pol[0]), int(pol[1])
    if history:
        out["hist"] = hist[: out["iters"] + 1]
        out["arnoldi_err"] = float(aerr[0])
    return out


def bicgstab(A, b, x0=None, tol=1e-10, maxiter=10000, precond=0, history=False):
    rp, ci, v = _csr(A)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64)
    info = np.zeros(3, dtype=np.int64)
    dinfo = np.zeros(1, dtype=np.float64)
    hist = np.full(maxiter + 1, np.nan) if history else None
    lib().orc_bicgstab(A.n, _p(rp), _p(ci), _p(v), _p(b), _p(x), tol, maxiter, precond, _p(info), _p(dinfo),
                       _p(hist))
    out = dict(x=x, iters=int(info[0]), status=int(info[2]), relres=float(dinfo[0]))
    if history:
        out["hist"] = hist[: out["iters"] + 1]
    return out

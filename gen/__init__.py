"""Seeded synthetic matrices and vectors shaped like the paper's workloads.

Fixture module shared by the CPU oracle tests and the GPU path.  It holds no
SpMV arithmetic: the C library only writes CSR arrays and vectors.

Configurations (sizes follow the workloads the paper evaluates in its
section 4; the paper's own University of Florida matrices are not used, these
synthetic shapes stand in for them):

* ``laplacian2d(64)``          2D 5-point Laplacian, 4 / -1, n = 4096
* ``powerlaw(2_000_000)``      lognormal(2.5, 1) row lengths clipped to
                               [1, 5000], uniform distinct columns plus the
                               diagonal, N(0,1) values, dominant diagonal
* ``trans4_like()``            one row of 114,910 entries among 116,835 rows
                               of 1..7 entries, 749,800 in total (the very
                               unbalanced matrix of section 4.4.1.3)
* ``stencil27(128, lower)``    3D 27-point, 27 / -1, symmetric lower storage
* ``batch(512)``               uneven banded / random systems
* ``selector_family(...)``     the learned-selector training families
"""
import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            raise RuntimeError(f"generator library missing: {_build.LIB} (run __graft_entry__.build())")
        L = ctypes.CDLL(_build.LIB)
        P = ctypes.c_void_p
        i64, i32, u64, d = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
        sig = {
            "xg_stream_u64": (u64, [u64, u64, i64]),
            "xg_uniform_vec": (None, [i64, u64, d, d, P]),
            "xg_int_vec": (None, [i64, u64, i32, i32, P]),
            "xg_stencil_lengths": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, i32, ctypes.c_int, P]),
            "xg_stencil_fill": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, i32, ctypes.c_int, d, d,
                                               ctypes.c_int, P, P, P]),
            "xg_lognormal_lengths": (None, [i64, u64, d, d, i32, i32, P]),
            "xg_uniform_lengths": (None, [i64, u64, i32, i32, P]),
            "xg_trans4_lengths": (ctypes.c_int, [i64, u64, i64, i32, i64, P]),
            "xg_random_rows_fill": (ctypes.c_int, [i64, i64, u64, ctypes.c_int, ctypes.c_int, P, P, P]),
            "xg_banded_lengths": (None, [i64, i32, ctypes.c_int, P]),
            "xg_banded_fill": (None, [i64, i32, ctypes.c_int, u64, P, P, P]),
            "xg_blockdiag_blocks": (i64, [i64, u64, i32, i32, P]),
            "xg_blockdiag_lengths": (None, [i64, P, P]),
            "xg_blockdiag_fill": (None, [i64, P, u64, P, P, P]),
            "xg_batch_params": (None, [i32, u64, d, d, i32, P, P, P]),
            "xg_batch_sid": (u64, [u64, i32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class CSR:
    """Host CSR matrix: int32 rowptr[n+1], int32 colind[nnz], float64 val[nnz].

    ``sym_lower`` marks symmetric matrices stored as their lower triangle
    (diagonal included)."""
    n: int
    ncols: int
    rowptr: np.ndarray
    colind: np.ndarray
    val: np.ndarray
    sym_lower: bool = False
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self):
        return int(self.rowptr[-1]) if self.n > 0 else 0


def _rowptr_from_lengths(len32):
    rp = np.zeros(len32.size + 1, dtype=np.int64)
    np.cumsum(len32, out=rp[1:])
    if rp[-1] >= 2**31:
        raise ValueError(f"nnz {rp[-1]} does not fit int32 indices")
    return rp.astype(np.int32)


# ----------------------------------------------------------------- vectors
def uniform_vec(n, seed, lo=-1.0, hi=1.0):
    out = np.empty(n, dtype=np.float64)
    lib().xg_uniform_vec(n, seed, lo, hi, _p(out))
    return out


def int_vec(n, seed, lo=-8, hi=8):
    out = np.empty(n, dtype=np.float64)
    lib().xg_int_vec(n, seed, lo, hi, _p(out))
    return out


def stream_u64(seed, sid, k):
    return int(lib().xg_stream_u64(seed, sid, k))


# ----------------------------------------------------------------- stencils
def stencil(dim, npts, g, lower=False, diag=None, off=-1.0, dominant=False, name=""):
    n = g ** dim
    ln = np.empty(n, dtype=np.int32)
    if lib().xg_stencil_lengths(dim, npts, g, int(lower), _p(ln)) != 0:
        raise ValueError("bad stencil")
    rp = _rowptr_from_lengths(ln)
    nnz = int(rp[-1])
    ci = np.empty(nnz, dtype=np.int32)
    v = np.empty(nnz, dtype=np.float64)
    d = float(npts - 1) if diag is None else float(diag)
    lib().xg_stencil_fill(dim, npts, g, int(lower), d, off, int(dominant), _p(rp), _p(ci), _p(v))
    return CSR(n, n, rp, ci, v, sym_lower=lower, name=name or f"stencil{dim}d{npts}_{g}")


def laplacian2d(g=64, lower=False):
    """2D 5-point Laplacian, 4 on the diagonal, -1 off it (Dirichlet)."""
    return stencil(2, 5, g, lower=lower, diag=4.0, off=-1.0, name=f"lap2d_{g}")


def convdiff3d(g, beta):
    """3D 7-point convection-diffusion on a g^3 grid (Dirichlet), central
    differences with convection along x: 6 on the diagonal, -1 - beta / -1 +
    beta to the x neighbours below / above, -1 to the others.  Unsymmetric
    for beta != 0; its eigenvalues are real for abs(beta) < 1:
    2 + 2 sqrt(1 - beta^2) cos(i pi / (g + 1)) + sum over y, z of
    2 - 2 cos(j pi / (g + 1))."""
    A = stencil(3, 7, g, diag=6.0, off=-1.0, name=f"convdiff3d_{g}_{beta}")
    rows = np.repeat(np.arange(A.n, dtype=np.int64), np.diff(A.rowptr))
    c = A.colind.astype(np.int64)
    A.val[c == rows - 1] = -1.0 - beta
    A.val[c == rows + 1] = -1.0 + beta
    return A


def stencil27(g=128, lower=True):
    """3D 27-point stencil, 27 on the diagonal, -1 off it (Dirichlet)."""
    return stencil(3, 27, g, lower=lower, diag=27.0, off=-1.0, name=f"st27_{g}")


# ----------------------------------------------------------------- random rows
def _random_rows(n, ncols, seed, lengths, skip, with_diag=True, name=""):
    rp = _rowptr_from_lengths(lengths)
    nnz = int(rp[-1])
    ci = np.empty(nnz, dtype=np.int32)
    v = np.empty(nnz, dtype=np.float64)
    if lib().xg_random_rows_fill(n, ncols, seed, skip, int(with_diag), _p(rp), _p(ci), _p(v)) != 0:
        raise ValueError("row longer than the column range")
    return CSR(n, ncols, rp, ci, v, name=name)


def powerlaw(n=2_000_000, seed=2, mu=2.5, sigma=1.0, lmin=1, lmax=5000):
    """Unsymmetric power-law rows: len = clip(round(exp(N(mu, sigma))), lmin, lmax),
    diagonal included, distinct uniform columns, N(0,1) values, dominant diagonal."""
    ln = np.empty(n, dtype=np.int32)
    lib().xg_lognormal_lengths(n, seed, mu, sigma, lmin, min(lmax, n), _p(ln))
    return _random_rows(n, n, seed, ln, 2, name=f"powerlaw_{n}")


def random_uniform_rows(n, seed, lmin, lmax):
    ln = np.empty(n, dtype=np.int32)
    lib().xg_uniform_lengths(n, seed, lmin, min(lmax, n), _p(ln))
    return _random_rows(n, n, seed, ln, 1, name=f"randrows_{n}")


def trans4_like(n=116_835, nnz=749_800, long_len=114_910, seed=22):
    """The very unbalanced shape of the paper's trans4 experiment (sec. 4.4.1.3):
    one row of `long_len` entries, the others 1..7 entries, `nnz` in total."""
    ln = np.empty(n, dtype=np.int32)
    if lib().xg_trans4_lengths(n, seed, n // 2, long_len, nnz, _p(ln)) != 0:
        raise ValueError("infeasible trans4 lengths")
    return _random_rows(n, n, seed, ln, 1, name="trans4_like")


def banded(n, h, seed, lower=False):
    ln = np.empty(n, dtype=np.int32)
    lib().xg_banded_lengths(n, h, int(lower), _p(ln))
    rp = _rowptr_from_lengths(ln)
    nnz = int(rp[-1])
    ci = np.empty(nnz, dtype=np.int32)
    v = np.empty(nnz, dtype=np.float64)
    lib().xg_banded_fill(n, h, int(lower), seed, _p(rp), _p(ci), _p(v))
    return CSR(n, n, rp, ci, v, sym_lower=lower, name=f"banded_{n}_{h}")


def blockdiag(n, seed, bmin=8, bmax=64):
    bs = np.empty(n + 1, dtype=np.int64)
    nb = int(lib().xg_blockdiag_blocks(n, seed, bmin, bmax, _p(bs)))
    ln = np.empty(n, dtype=np.int32)
    lib().xg_blockdiag_lengths(nb, _p(bs), _p(ln))
    rp = _rowptr_from_lengths(ln)
    nnz = int(rp[-1])
    ci = np.empty(nnz, dtype=np.int32)
    v = np.empty(nnz, dtype=np.float64)
    lib().xg_blockdiag_fill(nb, _p(bs), seed, _p(rp), _p(ci), _p(v))
    return CSR(n, n, rp, ci, v, name=f"blockdiag_{n}")


# ----------------------------------------------------------------- batch
@dataclass
class Batch:
    """Block-diagonal concatenation of independent systems."""
    nsys: int
    row_off: np.ndarray   # int64[nsys+1]
    nnz_off: np.ndarray   # int64[nsys+1]
    rowptr: np.ndarray    # int32[N+1], global offsets
    colind: np.ndarray    # int32[nnz], global column indices
    val: np.ndarray
    kinds: np.ndarray
    params: np.ndarray

    @property
    def n(self):
        return int(self.row_off[-1])

    @property
    def nnz(self):
        return int(self.nnz_off[-1])

    def system(self, k):
        r0, r1 = int(self.row_off[k]), int(self.row_off[k + 1])
        z0 = int(self.nnz_off[k])
        rp = (self.rowptr[r0:r1 + 1].astype(np.int64) - z0).astype(np.int32)
        z1 = int(self.nnz_off[k + 1])
        ci = (self.colind[z0:z1] - r0).astype(np.int32)
        return CSR(r1 - r0, r1 - r0, rp, ci, self.val[z0:z1].copy(), name=f"sys{k}")


def batch_params(nsys=512, seed=4, nmin=1000, nmax=65536, hmax=64):
    n = np.empty(nsys, dtype=np.int32)
    kind = np.empty(nsys, dtype=np.int32)
    h = np.empty(nsys, dtype=np.int32)
    lib().xg_batch_params(nsys, seed, nmin, nmax, hmax, _p(n), _p(kind), _p(h))
    return n, kind, h


def batch_system(k, n, kind, h, seed=4, lmin=5, lmax=50):
    sid = int(lib().xg_batch_sid(seed, k))
    if kind == 0:
        return banded(n, int(h), sid)
    return random_uniform_rows(n, sid, lmin, lmax)


def batch(nsys=512, seed=4, nmin=1000, nmax=65536, hmax=64, lmin=5, lmax=50):
    """Independent systems: k even -> dense band of half-width h ~ U{1..hmax},
    k odd -> random rows of U{lmin..lmax} entries; n_k log-uniform."""
    n, kind, h = batch_params(nsys, seed, nmin, nmax, hmax)
    mats = [batch_system(k, int(n[k]), int(kind[k]), int(h[k]), seed, lmin, lmax) for k in range(nsys)]
    row_off = np.zeros(nsys + 1, dtype=np.int64)
    nnz_off = np.zeros(nsys + 1, dtype=np.int64)
    for k, m in enumerate(mats):
        row_off[k + 1] = row_off[k] + m.n
        nnz_off[k + 1] = nnz_off[k] + m.nnz
    if nnz_off[-1] >= 2**31:
        raise ValueError("batch nnz does not fit int32")
    rp = np.empty(int(row_off[-1]) + 1, dtype=np.int32)
    ci = np.empty(int(nnz_off[-1]), dtype=np.int32)
    v = np.empty(int(nnz_off[-1]), dtype=np.float64)
    for k, m in enumerate(mats):
        r0, z0 = int(row_off[k]), int(nnz_off[k])
        rp[r0:r0 + m.n] = m.rowptr[:-1] + z0
        ci[z0:z0 + m.nnz] = m.colind + r0
        v[z0:z0 + m.nnz] = m.val
    rp[-1] = int(nnz_off[-1])
    return Batch(nsys, row_off, nnz_off, rp, ci, v, kind, h)


# ----------------------------------------------------------------- selector set
FAMILIES = ("stencil", "banded", "powerlaw", "blockdiag")


def selector_matrix(idx, seed, nmin=1e4, nmax=4e6):
    """Matrix `idx` of the learned-selector set.  Family = idx % 4.  Parameters
    come from substream (seed, 2^40 + idx); the matrix itself uses seed
    seed * 2^20 + idx for its row substreams."""
    fam = FAMILIES[idx % 4]
    sid = int(seed) * (1 << 20) + idx
    u = [((stream_u64(seed, (1 << 40) + idx, k) >> 11) * 2.0 ** -53) for k in range(4)]
    n = int(round(math.exp(math.log(nmin) + u[0] * (math.log(nmax) - math.log(nmin)))))
    lower = u[1] < 0.5
    if fam == "stencil":
        kinds = [(2, 5), (2, 9), (3, 7), (3, 27)]
        dim, npts = kinds[min(3, int(u[2] * 4))]
        g = max(2, int(round(n ** (1.0 / dim))))
        m = stencil(dim, npts, g, lower=lower, dominant=True, name=f"sel{idx}_st{dim}d{npts}_{g}")
    elif fam == "banded":
        h = 1 + min(63, int(u[2] * 64))
        m = banded(n, h, sid, lower=lower)
    elif fam == "powerlaw":
        mu = 1.0 + 2.0 * u[2]
        sigma = 0.5 + u[3]
        m = powerlaw(n, sid, mu, sigma)
        lower = False
    else:
        m = blockdiag(n, sid)
        lower = False
    m.meta = {"family": fam, "idx": idx}
    return m

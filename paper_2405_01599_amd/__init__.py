"""Python binding of libxab (the MI355X auto-tuned CSR SpMV / Krylov library).

Argument marshalling only: every step runs in the HIP library.  PyTorch
supplies device memory and the current HIP stream.  Importing this module
does not load the library; the first call does, and it raises if the
library has not been built (there is no fallback path).
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxab.so")

F64, F32 = 0, 1
TIME, STABLE, LEARNED, MEMORY, ACCURACY = 0, 1, 2, 3, 4
ROW, NNZ, BSS, SYM_S3, SYM_ATOMIC, XCB, SELL, BCSR = 0, 1, 2, 3, 4, 5, 6, 7
VARIANT_NAMES = {ROW: "row", NNZ: "nnz", BSS: "bss", SYM_S3: "sym_s3", SYM_ATOMIC: "sym_atomic", XCB: "xcb",
                 SELL: "sell", BCSR: "bcsr"}
GENERAL, SYM_LOWER, TRUST_INPUT, BATCH_TILES = 0, 1, 2, 4
NCLASSES = 15
GENERAL_CLASSES = tuple(range(9)) + (12, 13, 14)
SYM_CLASSES = (9, 10, 11)
NFEAT = 12
MLP_NPARAMS = 64 * 12 + 64 + 64 * 64 + 64 + NCLASSES * 64 + NCLASSES
MODE_FP64, MODE_IR = 0, 1
PRECOND_NONE, PRECOND_JACOBI = 0, 1
ORTHO_DGKS, ORTHO_CGS, ORTHO_MGS, ORTHO_BCGS, ORTHO_POLICY = 0, 1, 2, 3, 4
EIG_LARGEST, EIG_SMALLEST, EIG_MAGNITUDE = 0, 1, 2
NOALLOC_MAX_TILES = 262000  # XAB_NOALLOC_MAX_TILES

STATUS = {0: "ok", -1: "null", -2: "shape", -3: "dtype", -4: "struct", -5: "alias", -6: "unsupported",
          -7: "nomem", -8: "device", -9: "align", 1: "not_converged", 2: "breakdown", 3: "time_limit"}


class XabError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"xab status {status} ({STATUS.get(status, '?')}): {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("lanes_per_row", ctypes.c_int32), ("tile_nnz", ctypes.c_int32), ("j_per_lane", ctypes.c_int32),
                ("col_block", ctypes.c_int32), ("tile_rows", ctypes.c_int32), ("xcb_slices", ctypes.c_int32)]


class InitOpts(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("stream", ctypes.c_void_p), ("alloc", ctypes.c_void_p),
                ("free", ctypes.c_void_p), ("user", ctypes.c_void_p), ("policy", ctypes.c_int32)]


class SelectInfo(ctypes.Structure):
    _fields_ = [("chosen", ctypes.c_int32), ("time_ms", ctypes.c_float * NCLASSES), ("select_ms", ctypes.c_float),
                ("valid", ctypes.c_int32 * NCLASSES), ("bytes", ctypes.c_int64 * NCLASSES)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


class TrainInfo(ctypes.Structure):
    _fields_ = [("final_loss", ctypes.c_float), ("seconds", ctypes.c_float)]


class KrylovOpts(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("tol", ctypes.c_double), ("maxiter", ctypes.c_int64),
                ("max_time_s", ctypes.c_double), ("mode", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("graph", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("restart_step", ctypes.c_int32), ("m_max", ctypes.c_int32), ("mm_ratio", ctypes.c_double),
                ("ortho", ctypes.c_int32)]


class KrylovInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("restarts", ctypes.c_int64), ("refinements", ctypes.c_int64),
                ("true_relres", ctypes.c_double), ("seconds", ctypes.c_double), ("status", ctypes.c_int32),
                ("m_final", ctypes.c_int32), ("faults", ctypes.c_int32), ("ortho", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class EigOpts(ctypes.Structure):
    _fields_ = [("nev", ctypes.c_int32), ("m", ctypes.c_int32), ("tol", ctypes.c_double),
                ("maxiter", ctypes.c_int64), ("max_time_s", ctypes.c_double), ("which", ctypes.c_int32),
                ("restart_step", ctypes.c_int32), ("m_max", ctypes.c_int32), ("mm_ratio", ctypes.c_double),
                ("window", ctypes.c_int32)]


class EigInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("restarts", ctypes.c_int64), ("nconv", ctypes.c_int32),
                ("anrm", ctypes.c_double), ("max_resid", ctypes.c_double), ("seconds", ctypes.c_double),
                ("status", ctypes.c_int32), ("m_final", ctypes.c_int32), ("nret", ctypes.c_int32),
                ("faults", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = ctypes.c_void_p
_I32, _I64, _U32, _F, _D = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_float, ctypes.c_double
_PP = ctypes.POINTER(ctypes.c_void_p)

# symbol -> (restype, argtypes); every symbol declared in include/xab.h
SIGNATURES = {
    "xab_class_params": (ctypes.c_int, [_I32, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(Params)]),
    "xab_select_rule": (ctypes.c_int, [_P, _P, _I32, ctypes.POINTER(_I32)]),
    "xab_plan_refresh": (ctypes.c_int, [_P]),
    "xab_class_applies": (ctypes.c_int, [_I32, _I32]),
    "xab_init": (ctypes.c_int, [_PP, ctypes.POINTER(InitOpts)]),
    "xab_finalize": (None, [_P]),
    "xab_set_stream": (ctypes.c_int, [_P, _P]),
    "xab_last_error": (ctypes.c_char_p, [_P]),
    "xab_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "xab_matrix_csr": (ctypes.c_int, [_P, _I32, _I32, _I64, _P, _P, _P, ctypes.c_int, _U32, _PP]),
    "xab_matrix_add_values": (ctypes.c_int, [_P, _P, ctypes.c_int]),
    "xab_matrix_destroy": (None, [_P]),
    "xab_plan_fixed": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.POINTER(Params), _PP]),
    "xab_plan_destroy": (None, [_P]),
    "xab_plan_array": (ctypes.c_int, [_P, _I32, _P, ctypes.POINTER(_I64)]),
    "xab_plan_info": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(Params)]),
    "xab_plan_bytes": (ctypes.c_int64, [_P]),
    "xab_spmv_csr": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, _P, ctypes.c_int, ctypes.c_int]),
    "xab_spmv_sym": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, _P, ctypes.c_int, ctypes.c_int]),
    "xab_spmv_csr_noalloc": (ctypes.c_int, [_P, _I32, _I32, _I64, _P, _P, _P, _I32, _P, ctypes.c_int, _P,
                                            ctypes.c_int, ctypes.c_int]),
    "xab_time_spmv": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, _P, ctypes.c_int, ctypes.c_int, _I32, _I32,
                                     ctypes.POINTER(_F)]),
    "xab_select": (ctypes.c_int, [_P, _P, ctypes.c_int, _PP, ctypes.POINTER(SelectInfo)]),
    "xab_features": (ctypes.c_int, [_P, _P, _P, _P]),
    "xab_selector_set": (ctypes.c_int, [_P, _P, _P, _P]),
    "xab_selector_get": (ctypes.c_int, [_P, _P, _P, _P]),
    "xab_selector_save": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "xab_selector_load": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "xab_selector_train": (ctypes.c_int, [_P, _P, _P, _P, _I32, _P, ctypes.POINTER(TrainOpts), _P,
                                          ctypes.POINTER(TrainInfo)]),
    "xab_selector_forward": (ctypes.c_int, [_P, _P, _I32, _I32, _P]),
    "xab_selector_loss_grad": (ctypes.c_int, [_P, _P, _P, _P, _I32, _P, ctypes.POINTER(_F)]),
    "xab_gmres": (ctypes.c_int, [_P, _P, _P, _P, ctypes.POINTER(KrylovOpts), ctypes.POINTER(KrylovInfo)]),
    "xab_lanczos": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(EigOpts), _P, _P, ctypes.POINTER(EigInfo)]),
    "xab_arnoldi": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(EigOpts), _P, _P, _P, ctypes.POINTER(EigInfo)]),
    "xab_batch_csr": (ctypes.c_int, [_P, _I32, _P, _P, _P, _P, _P, ctypes.c_int, _U32, _PP]),
    "xab_batch_destroy": (None, [_P]),
    "xab_batch_layout": (ctypes.c_int, [_P]),
    "xab_batch_spmv": (ctypes.c_int, [_P, _P, _P, _P]),
    "xab_bicgstab": (ctypes.c_int, [_P, _P, _P, _P, ctypes.POINTER(KrylovOpts), _P, ctypes.POINTER(KrylovInfo)]),
}

_lib = None


def lib():
    """Load libxab.so (raises if it is missing: no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libxab.so not built at {LIB_PATH}; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name, None)
            if f is None:
                continue  # calling it raises AttributeError
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _torch():
    import torch
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dt(t):
    torch = _torch()
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def select_rule(time_ms, valid):
    """The TIME policy's decision on a given table: (status, chosen class)."""
    t = np.ascontiguousarray(time_ms, dtype=np.float32)
    v = np.ascontiguousarray(valid, dtype=np.int32)
    if t.shape != v.shape:
        raise ValueError("time_ms and valid differ in length")
    c = _I32()
    s = lib().xab_select_rule(t.ctypes.data_as(_P), v.ctypes.data_as(_P), t.size, ctypes.byref(c))
    return s, c.value


def class_applies(k, sym):
    return lib().xab_class_applies(k, 1 if sym else 0)


def class_params(k):
    v = ctypes.c_int()
    p = Params()
    s = lib().xab_class_params(k, ctypes.byref(v), ctypes.byref(p))
    if s != 0:
        raise XabError(s, f"class {k}")
    return v.value, p


class Context:
    """A library context bound to a device and (by default) torch's current stream."""

    def __init__(self, device=0, stream=None, policy=TIME):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("xab needs a HIP device")
        self.device = device
        torch.cuda.set_device(device)
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        opts = InitOpts(device=device, stream=ctypes.c_void_p(stream.cuda_stream), alloc=None, free=None, user=None,
                        policy=policy)
        h = ctypes.c_void_p()
        self._check(lib().xab_init(ctypes.byref(h), ctypes.byref(opts)), "xab_init", ctx=False)
        self.h = h
        self._has_model = False

    def _check(self, s, what, ctx=True):
        if s < 0:
            msg = lib().xab_last_error(self.h).decode() if ctx else what
            raise XabError(s, f"{what}: {msg}")
        return s

    def error(self):
        return lib().xab_last_error(self.h).decode()

    def close(self):
        if getattr(self, "h", None):
            lib().xab_finalize(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------- matrices
    def matrix(self, rowptr, colind, val, ncols=None, sym_lower=False, trust=False, val32=None):
        """Wrap device tensors (int32 rowptr/colind, float64 or float32 values)."""
        return Matrix(self, rowptr, colind, val, ncols, sym_lower, trust, val32)

    def matrix_from_csr(self, A, with_f32=False, with_f64=True, trust=False):
        """Upload a host CSR (gen.CSR) and wrap it."""
        torch = _torch()
        dev = f"cuda:{self.device}"
        rp = torch.from_numpy(np.ascontiguousarray(A.rowptr, dtype=np.int32)).to(dev)
        ci = torch.from_numpy(np.ascontiguousarray(A.colind, dtype=np.int32)).to(dev)
        v64 = torch.from_numpy(np.ascontiguousarray(A.val, dtype=np.float64)).to(dev) if with_f64 else None
        v32 = torch.from_numpy(np.ascontiguousarray(A.val, dtype=np.float32)).to(dev) if with_f32 else None
        first = v64 if v64 is not None else v32
        return Matrix(self, rp, ci, first, A.ncols, A.sym_lower, trust, v32 if v64 is not None else None)

    def plan(self, A, variant, **params):
        return Plan(self, A, variant, **params)

    def plan_class(self, A, k):
        v, p = class_params(k)
        return Plan(self, A, v, params=p)

    def select(self, A, policy=TIME):
        """Run the selector.  LEARNED uses the cost model last set, loaded or
        trained on this context, else the one shipped with the package."""
        if policy == LEARNED and not self._has_model:
            from .selector import MODEL_PATH
            self.selector_load(MODEL_PATH)
        h = ctypes.c_void_p()
        info = SelectInfo()
        self._check(lib().xab_select(self.h, A.h, policy, ctypes.byref(h), ctypes.byref(info)), "xab_select")
        pl = Plan.__new__(Plan)
        pl.ctx, pl.A, pl.h = self, A, h
        pl._load_info()
        return pl, info

    def features(self, A):
        out = np.zeros(NFEAT, dtype=np.float32)
        st = np.zeros(9, dtype=np.int64)
        self._check(lib().xab_features(self.h, A.h, out.ctypes.data_as(_P), st.ctypes.data_as(_P)), "xab_features")
        return out, st

    # ----------------------------------------------------------- SpMV
    def spmv(self, plan, x, y=None, acc=None, ydtype=None):
        """y = A x (general or symmetric), queued on the context stream."""
        torch = _torch()
        if y is None:
            ydtype = ydtype or x.dtype
            y = torch.empty(plan.A.n, dtype=ydtype, device=x.device)
        xt, yt = _dt(x), _dt(y)
        at = (F64 if (xt == F64 or yt == F64) else F32) if acc is None else acc
        fn = lib().xab_spmv_sym if plan.A.sym_lower else lib().xab_spmv_csr
        self._check(fn(self.h, plan.h, _ptr(x), xt, _ptr(y), yt, at), "spmv")
        return y

    def spmv_noalloc(self, rowptr, colind, val, x, y, j=8, ncols=None, acc=None):
        """y = A x for the CSR arrays (device tensors; values in x's precision)
        with no plan and no device allocation (xab_spmv_csr_noalloc).  The
        caller provides y."""
        xt, yt = _dt(x), _dt(y)
        at = (F64 if (xt == F64 or yt == F64) else F32) if acc is None else acc
        n = rowptr.numel() - 1
        nc = x.numel() if ncols is None else ncols
        self._check(lib().xab_spmv_csr_noalloc(self.h, n, nc, colind.numel(), _ptr(rowptr), _ptr(colind), _ptr(val), j,
                                               _ptr(x), xt, _ptr(y), yt, at), "xab_spmv_csr_noalloc")
        return y

    def time_spmv(self, plan, x, y, acc=None, warmup=3, reps=20):
        xt, yt = _dt(x), _dt(y)
        at = (F64 if (xt == F64 or yt == F64) else F32) if acc is None else acc
        ms = ctypes.c_float()
        self._check(lib().xab_time_spmv(self.h, plan.h, _ptr(x), xt, _ptr(y), yt, at, warmup, reps, ctypes.byref(ms)),
                    "xab_time_spmv")
        return ms.value

    # ----------------------------------------------------------- selector model
    def selector_set(self, params, mean, std):
        p = np.ascontiguousarray(params, dtype=np.float32)
        m = np.ascontiguousarray(mean, dtype=np.float32)
        s = np.ascontiguousarray(std, dtype=np.float32)
        assert p.size == MLP_NPARAMS and m.size == NFEAT and s.size == NFEAT
        self._check(lib().xab_selector_set(self.h, p.ctypes.data_as(_P), m.ctypes.data_as(_P), s.ctypes.data_as(_P)),
                    "xab_selector_set")
        self._has_model = True

    def selector_get(self):
        p = np.zeros(MLP_NPARAMS, dtype=np.float32)
        m = np.zeros(NFEAT, dtype=np.float32)
        s = np.zeros(NFEAT, dtype=np.float32)
        self._check(lib().xab_selector_get(self.h, p.ctypes.data_as(_P), m.ctypes.data_as(_P), s.ctypes.data_as(_P)),
                    "xab_selector_get")
        return p, m, s

    def selector_save(self, path):
        self._check(lib().xab_selector_save(self.h, str(path).encode()), "xab_selector_save")

    def selector_load(self, path):
        self._check(lib().xab_selector_load(self.h, str(path).encode()), "xab_selector_load")
        self._has_model = True

    def selector_train(self, feat, cost, valid, order, epochs=300, batch=128, lr=1e-3):
        torch = _torch()
        m = feat.shape[0]
        order = np.ascontiguousarray(order, dtype=np.int32)
        assert order.size == epochs * m
        opts = TrainOpts(epochs=epochs, batch=batch, lr=lr, beta1=0.9, beta2=0.999, eps=1e-8)
        info = TrainInfo()
        loss = np.zeros(epochs, dtype=np.float32)
        f = feat.to(torch.float32).contiguous()
        c = cost.to(torch.float32).contiguous()
        v = valid.to(torch.uint8).contiguous()
        self._check(lib().xab_selector_train(self.h, _ptr(f), _ptr(c), _ptr(v), m, order.ctypes.data_as(_P),
                                             ctypes.byref(opts), loss.ctypes.data_as(_P), ctypes.byref(info)),
                    "xab_selector_train")
        return loss, info

    def selector_forward(self, feat, raw=True):
        torch = _torch()
        f = feat.to(torch.float32).contiguous()
        out = torch.empty((f.shape[0], NCLASSES), dtype=torch.float32, device=f.device)
        self._check(lib().xab_selector_forward(self.h, _ptr(f), f.shape[0], int(raw), _ptr(out)),
                    "xab_selector_forward")
        return out

    def selector_loss_grad(self, feat, y, valid):
        torch = _torch()
        f = feat.to(torch.float32).contiguous()
        yy = y.to(torch.float32).contiguous()
        v = valid.to(torch.uint8).contiguous()
        g = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=f.device)
        loss = ctypes.c_float()
        self._check(lib().xab_selector_loss_grad(self.h, _ptr(f), _ptr(yy), _ptr(v), f.shape[0], _ptr(g),
                                                 ctypes.byref(loss)), "xab_selector_loss_grad")
        return loss.value, g

    # ----------------------------------------------------------- Krylov
    def gmres(self, plan, b, x=None, m=30, tol=1e-10, maxiter=100000, mode=MODE_FP64, precond=PRECOND_JACOBI,
              inner_tol=1e-6, max_time_s=0.0, restart_step=0, m_max=0, mm_ratio=0.0, ortho=0):
        torch = _torch()
        if x is None:
            x = torch.zeros_like(b)
        opts = KrylovOpts(m=m, tol=tol, maxiter=maxiter, max_time_s=max_time_s, mode=mode, precond=precond,
                          inner_tol=inner_tol, graph=0, check_every=0, restart_step=restart_step,
                          m_max=m_max if m_max else m, mm_ratio=mm_ratio, ortho=ortho)
        info = KrylovInfo()
        s = self._check(lib().xab_gmres(self.h, plan.h, _ptr(b), _ptr(x), ctypes.byref(opts), ctypes.byref(info)),
                        "xab_gmres")
        return x, info.as_dict(), s

    def lanczos(self, plan, v0, nev=10, m=30, tol=1e-8, maxiter=0, which=EIG_LARGEST, max_time_s=0.0,
                restart_step=0, m_max=0, mm_ratio=0.0, window=5):
        """Thick-restart Lanczos: (evals numpy[nev], evecs tensor [n, nev], info dict, status)."""
        torch = _torch()
        n = v0.numel()
        ev = np.zeros(nev, dtype=np.float64)
        X = torch.empty((nev, n), dtype=torch.float64, device=v0.device)  # column-major n x nev
        opts = EigOpts(nev=nev, m=m, tol=tol, maxiter=maxiter, max_time_s=max_time_s, which=which,
                       restart_step=restart_step, m_max=m_max if m_max else m, mm_ratio=mm_ratio, window=window)
        info = EigInfo()
        s = self._check(lib().xab_lanczos(self.h, plan.h, _ptr(v0), ctypes.byref(opts), ev.ctypes.data_as(_P),
                                          _ptr(X), ctypes.byref(info)), "xab_lanczos")
        return ev, X.t(), info.as_dict(), s

    def arnoldi(self, plan, v0, nev=10, m=30, tol=1e-8, maxiter=0, which=EIG_MAGNITUDE, max_time_s=0.0,
                restart_step=0, m_max=0, mm_ratio=0.0, window=5):
        """Implicitly restarted Arnoldi: (evals complex numpy[nret], evecs tensor
        [n, nret] (a complex pair as real and imaginary parts), info dict, status)."""
        torch = _torch()
        n = v0.numel()
        re = np.zeros(nev + 1, dtype=np.float64)
        im = np.zeros(nev + 1, dtype=np.float64)
        X = torch.empty((nev + 1, n), dtype=torch.float64, device=v0.device)  # column-major n x (nev + 1)
        opts = EigOpts(nev=nev, m=m, tol=tol, maxiter=maxiter, max_time_s=max_time_s, which=which,
                       restart_step=restart_step, m_max=m_max if m_max else m, mm_ratio=mm_ratio, window=window)
        info = EigInfo()
        s = self._check(lib().xab_arnoldi(self.h, plan.h, _ptr(v0), ctypes.byref(opts), re.ctypes.data_as(_P),
                                          im.ctypes.data_as(_P), _ptr(X), ctypes.byref(info)), "xab_arnoldi")
        k = info.nret
        return (re + 1j * im)[:k], X[:k].t(), info.as_dict(), s

    def batch(self, B, dtype="f64", trust=False, tiles=False):
        return Batch(self, B, dtype, trust, tiles)

    def bicgstab(self, batch, b, x=None, tol=1e-10, maxiter=10000, precond=PRECOND_JACOBI, graph=True,
                 check_every=8):
        torch = _torch()
        if x is None:
            x = torch.zeros_like(b)
        opts = KrylovOpts(m=0, tol=tol, maxiter=maxiter, max_time_s=0.0, mode=0, precond=precond, inner_tol=0.0,
                          graph=int(graph), check_every=check_every, restart_step=0, m_max=0, mm_ratio=0.0, ortho=0)
        infos = (KrylovInfo * batch.nsys)()
        allinfo = KrylovInfo()
        s = self._check(lib().xab_bicgstab(self.h, batch.h, _ptr(b), _ptr(x), ctypes.byref(opts),
                                           ctypes.cast(infos, _P), ctypes.byref(allinfo)), "xab_bicgstab")
        return x, [i.as_dict() for i in infos], allinfo.as_dict(), s


class Matrix:
    def __init__(self, ctx, rowptr, colind, val, ncols, sym_lower, trust, val32=None):
        torch = _torch()
        assert rowptr.dtype == torch.int32 and colind.dtype == torch.int32
        self.ctx = ctx
        self.rowptr, self.colind, self.val = rowptr, colind, val
        self.val32 = val32
        self.n = rowptr.numel() - 1
        self.ncols = self.n if ncols is None else ncols
        self.nnz = colind.numel()
        self.sym_lower = sym_lower
        flags = (SYM_LOWER if sym_lower else 0) | (TRUST_INPUT if trust else 0)
        h = ctypes.c_void_p()
        ctx._check(lib().xab_matrix_csr(ctx.h, self.n, self.ncols, self.nnz, _ptr(rowptr), _ptr(colind), _ptr(val),
                                        _dt(val), flags, ctypes.byref(h)), "xab_matrix_csr")
        self.h = h
        if val32 is not None:
            ctx._check(lib().xab_matrix_add_values(h, _ptr(val32), _dt(val32)), "xab_matrix_add_values")

    def add_values(self, v):
        self.ctx._check(lib().xab_matrix_add_values(self.h, _ptr(v), _dt(v)), "xab_matrix_add_values")
        if _dt(v) == F32:
            self.val32 = v
        else:
            self.val = v

    def close(self):
        if getattr(self, "h", None) and self.ctx.h:
            lib().xab_matrix_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    def __init__(self, ctx, A, variant, params=None, **kw):
        if params is None:
            params = Params(lanes_per_row=8, tile_nnz=2048, j_per_lane=8, col_block=256, tile_rows=2048)
        for k, v in kw.items():
            setattr(params, k, v)
        h = ctypes.c_void_p()
        ctx._check(lib().xab_plan_fixed(ctx.h, A.h, variant, ctypes.byref(params), ctypes.byref(h)), "xab_plan_fixed")
        self.ctx, self.A, self.h = ctx, A, h
        self._load_info()

    def _load_info(self):
        v = ctypes.c_int()
        p = Params()
        lib().xab_plan_info(self.h, ctypes.byref(v), ctypes.byref(p))
        self.variant, self.params = v.value, p

    @property
    def bytes(self):
        """Device bytes held by the plan's own arrays."""
        return int(lib().xab_plan_bytes(self.h))

    def array(self, which):
        n = _I64()
        self.ctx._check(lib().xab_plan_array(self.h, which, None, ctypes.byref(n)), "xab_plan_array")
        out = np.zeros(n.value, dtype=np.int32)
        if n.value:
            self.ctx._check(lib().xab_plan_array(self.h, which, out.ctypes.data_as(_P), ctypes.byref(n)),
                            "xab_plan_array")
        return out

    def refresh(self):
        """Re-read the matrix's values (changed in place) into the plan's copies."""
        self.ctx._check(lib().xab_plan_refresh(self.h), "xab_plan_refresh")

    def describe(self):
        p = self.params
        return dict(variant=VARIANT_NAMES[self.variant], lanes_per_row=p.lanes_per_row, tile_nnz=p.tile_nnz,
                    j_per_lane=p.j_per_lane, col_block=p.col_block, tile_rows=p.tile_rows, xcb_slices=p.xcb_slices)

    def close(self):
        if getattr(self, "h", None) and self.ctx.h:
            lib().xab_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    def __init__(self, ctx, B, dtype="f64", trust=False, tiles=False):
        torch = _torch()
        dev = f"cuda:{ctx.device}"
        self.ctx = ctx
        self.nsys = B.nsys
        self.n = B.n
        self.row_off = np.ascontiguousarray(B.row_off, dtype=np.int64)
        self.nnz_off = np.ascontiguousarray(B.nnz_off, dtype=np.int64)
        self.rowptr = torch.from_numpy(B.rowptr).to(dev)
        self.colind = torch.from_numpy(B.colind).to(dev)
        tdt = torch.float64 if dtype == "f64" else torch.float32
        self.val = torch.from_numpy(B.val).to(dev).to(tdt)
        self.dtype = tdt
        h = ctypes.c_void_p()
        ctx._check(lib().xab_batch_csr(ctx.h, self.nsys, self.row_off.ctypes.data_as(_P),
                                       self.nnz_off.ctypes.data_as(_P), _ptr(self.rowptr), _ptr(self.colind),
                                       _ptr(self.val), _dt(self.val),
                                       (TRUST_INPUT if trust else 0) | (BATCH_TILES if tiles else 0), ctypes.byref(h)),
                   "xab_batch_csr")
        self.h = h

    @property
    def layout(self):
        """'sell' when the SpMV runs on the batch's sliced ELLPACK copy, else 'tiles'."""
        return "sell" if lib().xab_batch_layout(self.h) == 1 else "tiles"

    def spmv(self, x, y=None):
        torch = _torch()
        if y is None:
            y = torch.empty(self.n, dtype=self.dtype, device=x.device)
        self.ctx._check(lib().xab_batch_spmv(self.ctx.h, self.h, _ptr(x), _ptr(y)), "xab_batch_spmv")
        return y

    def close(self):
        if getattr(self, "h", None) and self.ctx.h:
            lib().xab_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

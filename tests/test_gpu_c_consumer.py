"""The boundary used from plain C: a C99 program built against
include/xab.h and libxab.so alone (no Python in between) selects an SpMV
implementation, multiplies and solves; its results are checked against the
oracle."""
import os
import subprocess

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "host", "abi_consumer")
PKG = os.path.join(ROOT, "paper_2405_01599_amd")


def test_c_program_through_the_boundary(tmp_path):
    if not os.path.exists(EXE):
        pytest.fail("tests/host/abi_consumer is not built: run __graft_entry__.build()")
    A = gen.powerlaw(100_000, seed=5)
    x = gen.uniform_vec(A.n, 3)
    b = np.ones(A.n)
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        f.write(np.int32(A.n).tobytes() + np.int64(A.nnz).tobytes())
        for arr, dt in ((A.rowptr, np.int32), (A.colind, np.int32), (A.val, np.float64), (x, np.float64),
                        (b, np.float64)):
            f.write(np.ascontiguousarray(arr, dtype=dt).tobytes())
    env = dict(os.environ)
    env["LD_LIBRARY_PATH"] = PKG + (":" + env["LD_LIBRARY_PATH"] if env.get("LD_LIBRARY_PATH") else "")
    print(f"abi_consumer: power-law n={A.n} nnz={A.nnz}", flush=True)
    r = subprocess.run([EXE, str(inp), str(out)], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    raw = open(out, "rb").read()
    chosen, spmv_st, gm_st = np.frombuffer(raw[:12], dtype=np.int32)
    iters = int(np.frombuffer(raw[12:20], dtype=np.int64)[0])
    relres = float(np.frombuffer(raw[20:28], dtype=np.float64)[0])
    y = np.frombuffer(raw[28:28 + 8 * A.n], dtype=np.float64)
    s = np.frombuffer(raw[28 + 8 * A.n:28 + 16 * A.n], dtype=np.float64)
    import paper_2405_01599_amd as xab
    assert int(chosen) in xab.GENERAL_CLASSES
    assert spmv_st == 0 and gm_st == 0 and iters > 0
    yo, sa = oracle.spmv(A, x)
    assert np.all(np.abs(y - yo) <= 1e-12 * sa)
    res = np.linalg.norm(b - oracle.spmv(A, s)[0]) / np.linalg.norm(b)
    assert res <= 1e-10 and abs(res - relres) <= 1e-12

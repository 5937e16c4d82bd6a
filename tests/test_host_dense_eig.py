"""CPU checks of the library's host-side dense eigenvalue routines (the
Arnoldi driver's small projected problem), built through a C shim with g++:
Schur form against LAPACK's eigenvalues, orthogonality and the
similarity; Ritz vectors against the definition; implicit QR steps keep
the Hessenberg form, the spectrum and orthogonality, and an exact shift
deflates."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("shim") / "dense_eig_shim.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", out,
                    os.path.join(HERE, "host", "dense_eig_shim.cpp")], check=True)
    L = ctypes.CDLL(out)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    L.shim_schur.argtypes = [I, P, P, P, P]
    L.shim_schur.restype = I
    L.shim_ritz_vec.argtypes = [I, P, I, P, P]
    L.shim_qr_shift.argtypes = [I, P, P, I, D, D]
    return L


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def hess(n, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return np.triu(rng.standard_normal((n, n)) * scale, -1)


def schur(shim, H):
    n = H.shape[0]
    T = np.ascontiguousarray(H.copy())
    Z = np.zeros((n, n))
    wr, wi = np.zeros(n), np.zeros(n)
    assert shim.shim_schur(n, _p(T), _p(Z), _p(wr), _p(wi)) == 0
    return T, Z, wr + 1j * wi


@pytest.mark.parametrize("n,seed", [(3, 1), (8, 2), (30, 3), (63, 4)])
def test_schur_form(shim, n, seed):
    H = hess(n, seed)
    T, Z, lam = schur(shim, H)
    assert np.max(np.abs(Z.T @ Z - np.eye(n))) <= 1e-13
    assert np.max(np.abs(Z @ T @ Z.T - H)) <= 1e-12 * np.max(np.abs(H)) * n
    assert np.all(np.abs(np.tril(T, -2)) == 0.0)
    # 2 x 2 blocks only for complex pairs, never two in a row
    for i in range(n - 1):
        if T[i + 1, i] != 0.0:
            assert lam[i].imag > 0 and lam[i + 1] == np.conj(lam[i])
            assert i + 2 >= n or T[i + 2, i + 1] == 0.0
        elif lam[i].imag == 0.0:
            assert lam[i].real == T[i, i]
    ref = np.linalg.eigvals(H)
    assert np.max(np.abs(np.sort_complex(lam) - np.sort_complex(ref))) <= 1e-10 * np.max(np.abs(ref))


def test_schur_symmetric_tridiagonal_real(shim):
    n = 20
    H = np.diag(np.full(n, 2.0)) + np.diag(np.full(n - 1, -1.0), 1) + np.diag(np.full(n - 1, -1.0), -1)
    T, Z, lam = schur(shim, H)
    assert np.all(lam.imag == 0.0)
    want = 2.0 - 2.0 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    assert np.max(np.abs(np.sort(lam.real) - np.sort(want))) <= 1e-13


@pytest.mark.parametrize("seed", [5, 6, 7])
def test_ritz_vectors(shim, seed):
    n = 25
    T, Z, lam = schur(shim, hess(n, seed))
    for p in range(n):
        if lam[p].imag < 0:
            continue  # the second of a pair: the first carries the vector
        xr, xi = np.zeros(n), np.zeros(n)
        shim.shim_ritz_vec(n, _p(np.ascontiguousarray(T)), p, _p(xr), _p(xi))
        x = xr + 1j * xi
        assert np.linalg.norm(T @ x - lam[p] * x) <= 1e-11 * np.linalg.norm(x) * np.max(np.abs(T))


def test_qr_steps(shim):
    n = 12
    H0 = hess(n, 8)
    lam = np.linalg.eigvals(H0)
    for kind, s, t in ((1, 0.3, 0.0), (2, 1.0, 2.5)):
        H, Q = H0.copy(), np.eye(n)
        shim.shim_qr_shift(n, _p(H), _p(Q), kind, s, t)
        assert np.max(np.abs(np.tril(H, -2))) == 0.0
        assert np.max(np.abs(Q.T @ Q - np.eye(n))) <= 1e-14
        assert np.max(np.abs(Q.T @ H0 @ Q - H)) <= 1e-13 * np.max(np.abs(H0)) * n
        assert np.max(np.abs(np.sort_complex(np.linalg.eigvals(H)) - np.sort_complex(lam))) <= 1e-10
    # an exact real shift: the last subdiagonal entry vanishes
    real = lam[np.abs(lam.imag) == 0][0].real
    H, Q = H0.copy(), np.eye(n)
    shim.shim_qr_shift(n, _p(H), _p(Q), 1, real, 0.0)
    assert abs(H[n - 1, n - 2]) <= 1e-8 * np.max(np.abs(H0))
    assert abs(H[n - 1, n - 1] - real) <= 1e-8 * np.max(np.abs(H0))
    # an exact complex pair: the trailing 2 x 2 block decouples
    cz = lam[lam.imag > 0][0]
    H, Q = H0.copy(), np.eye(n)
    shim.shim_qr_shift(n, _p(H), _p(Q), 2, 2 * cz.real, abs(cz) ** 2)
    assert abs(H[n - 2, n - 3]) <= 1e-7 * np.max(np.abs(H0))

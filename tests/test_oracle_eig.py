"""Pins of the oracle's thick-restart Lanczos against closed forms, a library
eigensolver and invariants (no GPU)."""
import numpy as np
import pytest

import gen
from oracle import eig


def lap1d(n):
    """tridiag(-1, 2, -1): eigenvalues 2 - 2 cos(k pi / (n + 1)), all simple."""
    rp = [0]
    ci, v = [], []
    for i in range(n):
        for j, a in ((i - 1, -1.0), (i, 2.0), (i + 1, -1.0)):
            if 0 <= j < n:
                ci.append(j)
                v.append(a)
        rp.append(len(ci))
    return gen.CSR(n, n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(v), name=f"lap1d_{n}")


def from_dense(D, lower=False):
    n = D.shape[0]
    rp, ci, v = [0], [], []
    for i in range(n):
        for j in range(n):
            if D[i, j] != 0.0 and (not lower or j <= i):
                ci.append(j)
                v.append(D[i, j])
        rp.append(len(ci))
    return gen.CSR(n, n, np.array(rp, np.int32), np.array(ci, np.int32), np.array(v), sym_lower=lower,
                   name="dense")


def st27_eigs(g):
    """Closed-form spectrum of 28 I - T (x) T (x) T, T = tridiag(1, 1, 1) of order g
    (the 27-point stencil with 27 on the diagonal and -1 off it)."""
    t = 1.0 + 2.0 * np.cos(np.arange(1, g + 1) * np.pi / (g + 1))
    return np.sort((28.0 - np.einsum("i,j,k->ijk", t, t, t)).ravel())


@pytest.mark.parametrize("which", [eig.LARGEST, eig.SMALLEST])
def test_lap1d_closed_form(which):
    n = 400
    A = lap1d(n)
    r = eig.lanczos(A, 10, 30, gen.uniform_vec(n, 1), tol=1e-8, which=which)
    assert r["status"] == eig.OK and r["restarts"] > 5  # the restart path is exercised
    k = np.arange(1, n + 1)
    lam = 2.0 - 2.0 * np.cos(k * np.pi / (n + 1))
    want = np.sort(lam)[::-1][:10] if which == eig.LARGEST else np.sort(lam)[:10]
    assert np.max(np.abs(r["evals"] - want)) <= 1e-10 * r["anrm"]
    # eigenvectors: sin(k j pi / (n + 1)), normalised, up to sign
    for i in range(10):
        kk = int(np.argmin(np.abs(lam - r["evals"][i]))) + 1
        u = np.sin(kk * np.arange(1, n + 1) * np.pi / (n + 1))
        u /= np.linalg.norm(u)
        assert abs(abs(u @ r["evecs"][:, i]) - 1.0) <= 1e-8
    assert np.max(r["resid"]) <= 1.5e-8 * r["anrm"]


def test_diagonal_distinct():
    d = np.linspace(1.0, 3.0, 300) ** 2
    A = from_dense(np.diag(d))
    r = eig.lanczos(A, 10, 24, gen.uniform_vec(300, 2), tol=1e-10)
    assert r["status"] == eig.OK
    assert np.max(np.abs(r["evals"] - np.sort(d)[::-1][:10])) <= 1e-12 * r["anrm"]
    top = np.argsort(-d)[:10]
    for i in range(10):
        assert abs(abs(r["evecs"][top[i], i]) - 1.0) <= 1e-8


def test_full_space_one_cycle_matches_eigh():
    """m = n: the Krylov space is the whole space after one cycle, so every
    Ritz value equals an eigenvalue of the dense matrix (LAPACK's)."""
    rng = np.random.default_rng(3)
    M = rng.standard_normal((40, 40))
    D = M + M.T
    r = eig.lanczos(from_dense(D), 6, 40, rng.standard_normal(40), tol=1e-12)
    assert r["status"] == eig.OK and r["restarts"] == 0
    ref = np.linalg.eigvalsh(D)[::-1][:6]
    assert np.max(np.abs(r["evals"] - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_random_sparse_vs_eigh_and_lower_equals_full():
    rng = np.random.default_rng(4)
    n = 300
    D = np.zeros((n, n))
    for i in range(n):
        for j in rng.choice(n, 6, replace=False):
            D[i, j] = D[j, i] = rng.standard_normal()
    D += np.diag(rng.uniform(-2, 2, n))
    v0 = gen.uniform_vec(n, 9)
    full = eig.lanczos(from_dense(D), 8, 32, v0, tol=1e-9)
    low = eig.lanczos(from_dense(D, lower=True), 8, 32, v0, tol=1e-9)
    ref = np.linalg.eigvalsh(D)[::-1][:8]
    for r in (full, low):
        assert r["status"] == eig.OK
        assert np.max(np.abs(r["evals"] - ref)) <= 1e-9 * r["anrm"]
        X = r["evecs"]
        assert np.max(np.abs(X.T @ X - np.eye(8))) <= 1e-10
        assert np.max(r["resid"]) <= 1.5e-9 * r["anrm"]
    assert np.max(np.abs(full["evals"] - low["evals"])) <= 1e-11 * full["anrm"]


def test_st27_values_are_eigenvalues():
    """The lower-stored 27-point stencil on a 12^3 grid has eigenvalues of
    multiplicity 3 and 6, so which copies a single-vector Lanczos finds is
    rounding-dependent; what is fixed: the first value is the largest
    eigenvalue, every value is one of the closed form's, and each Ritz pair
    meets the residual bound."""
    g = 12
    A = gen.stencil27(g)
    r = eig.lanczos(A, 10, 40, gen.uniform_vec(A.n, 5), tol=1e-8)
    assert r["status"] == eig.OK
    lam = st27_eigs(g)
    assert abs(r["evals"][0] - lam[-1]) <= 1e-9 * r["anrm"]
    for t in r["evals"]:
        assert np.min(np.abs(lam - t)) <= 1e-9 * r["anrm"]
    assert np.all(np.diff(r["evals"]) <= 0)
    assert np.max(r["resid"]) <= 1.5e-8 * r["anrm"]


def test_breakdown_small_invariant_space():
    """A start vector inside a 3-dimensional eigenspace sum: the recurrence
    stops at 3 vectors, fewer than nev = 4, which is a breakdown."""
    d = np.arange(1.0, 31.0)
    A = from_dense(np.diag(d))
    v0 = np.zeros(30)
    v0[[2, 7, 11]] = 1.0
    r = eig.lanczos(A, 4, 10, v0)
    assert r["status"] == eig.BREAKDOWN
    r = eig.lanczos(A, 2, 10, v0)  # nev within the invariant space: exact
    assert r["status"] == eig.OK
    assert np.allclose(r["evals"], [12.0, 8.0], atol=1e-13)


def test_kept_count():
    assert eig.kept_count(10, 30) == 20
    assert eig.kept_count(10, 11) == 10


def test_restart_tuning_off_is_plain():
    A = lap1d(300)
    v0 = gen.uniform_vec(300, 3)
    a = eig.lanczos(A, 6, 16, v0)
    b = eig.lanczos(A, 6, 16, v0, step=0, m_max=40, ratio=100.0)
    assert a["matvecs"] == b["matvecs"] and np.array_equal(a["evals"], b["evals"])
    assert set(b["m_hist"]) == {16}


def test_restart_tuning_rule_extremes():
    """ratio = inf: every window of samples is 'stagnant', so m grows by step
    after each `window` cycles until m_max; ratio = 0: never (eq. (1) is >= 1)."""
    A = lap1d(400)
    v0 = gen.uniform_vec(400, 1)
    r = eig.lanczos(A, 10, 12, v0, step=5, m_max=30, ratio=np.inf, window=3)
    h = r["m_hist"]
    want = [12] * 3 + [17] * 3 + [22] * 3 + [27] * 3
    assert h[:12] == want and all(m == 30 for m in h[12:]) and r["m_final"] == 30
    assert r["status"] == eig.OK
    r0 = eig.lanczos(A, 10, 12, v0, step=5, m_max=30, ratio=0.0, window=3, maxiter=400)
    assert set(r0["m_hist"]) == {12}


def test_restart_tuning_cures_slow_convergence():
    """Basis of 12 for 10 wanted pairs restarts with little room; the MM-ratio
    rule grows it and the solve needs fewer products, same eigenvalues."""
    n = 400
    A = lap1d(n)
    v0 = gen.uniform_vec(n, 1)
    fixed = eig.lanczos(A, 10, 12, v0, maxiter=20000)
    tuned = eig.lanczos(A, 10, 12, v0, step=5, m_max=40, ratio=2.0, window=5, maxiter=20000)
    assert tuned["status"] == eig.OK and tuned["m_final"] > 12
    assert tuned["matvecs"] < fixed["matvecs"]
    lam = np.sort(2.0 - 2.0 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1)))[::-1][:10]
    assert np.max(np.abs(tuned["evals"] - lam)) <= 1e-10 * tuned["anrm"]


# ------------------------------------------------------------- Arnoldi
def triangular_permuted(n, seed):
    """P (D + U) P^T: D diagonal with distinct entries, U sparse strictly
    upper triangular; the eigenvalues are exactly the diagonal entries."""
    rng = np.random.default_rng(seed)
    d = np.linspace(0.0, 10.0, n) ** 1.5
    U = np.triu(rng.standard_normal((n, n)) * (rng.random((n, n)) < 0.01), 1) * 0.3
    P = np.eye(n)[rng.permutation(n)]
    return from_dense(P @ (np.diag(d) + U) @ P.T), d


def rotation_blocks(nb, seed):
    """Block-diagonal 2x2 rotation-scalings [[r, -s], [s, r]], permuted: a
    normal matrix with eigenvalues r_i +- i s_i."""
    rng = np.random.default_rng(seed)
    rs, ss = np.linspace(0.1, 3.0, nb), np.linspace(0.5, 1.0, nb)
    D = np.zeros((2 * nb, 2 * nb))
    for i in range(nb):
        D[2 * i:2 * i + 2, 2 * i:2 * i + 2] = [[rs[i], -ss[i]], [ss[i], rs[i]]]
    P = np.eye(2 * nb)[rng.permutation(2 * nb)]
    return from_dense(P @ D @ P.T), rs, ss


def dense_of_csr(A):
    D = np.zeros((A.n, A.ncols))
    for i in range(A.n):
        D[i, A.colind[A.rowptr[i]:A.rowptr[i + 1]]] += A.val[A.rowptr[i]:A.rowptr[i + 1]]
    return D


@pytest.mark.parametrize("which", [eig.LR, eig.SR, eig.LM])
def test_arnoldi_triangular_closed_form(which):
    A, d = triangular_permuted(500, 7)
    r = eig.arnoldi(A, 8, 30, gen.uniform_vec(500, 1), tol=1e-9, which=which)
    assert r["status"] == eig.OK and r["restarts"] > 5
    want = np.sort(d)[::-1][:8] if which != eig.SR else np.sort(d)[:8]
    assert np.max(np.abs(r["evals"] - want)) <= 1e-9 * r["anrm"]
    assert np.max(r["resid"]) <= 1.5e-9 * r["anrm"]


def test_arnoldi_complex_pairs():
    """nev = 5 cuts a complex pair, so both members are returned; the pair's
    vector comes back as real and imaginary parts (dgeev's convention)."""
    A, rs, ss = rotation_blocks(150, 3)
    r = eig.arnoldi(A, 5, 30, gen.uniform_vec(300, 2), tol=1e-10, which=eig.LR)
    assert r["status"] == eig.OK and r["evals"].size == 6
    want = np.array([rs[-1 - i // 2] + (1j if i % 2 == 0 else -1j) * ss[-1 - i // 2] for i in range(6)])
    got = np.sort_complex(r["evals"])
    assert np.max(np.abs(got - np.sort_complex(want))) <= 1e-10 * r["anrm"]
    D = dense_of_csr(A)
    for i in (0, 2, 4):
        lam = r["evals"][i]
        x = r["evecs"][:, i] + 1j * r["evecs"][:, i + 1]
        assert np.linalg.norm(D @ x - lam * x) / np.linalg.norm(x) <= 1e-9 * r["anrm"]


def test_arnoldi_mild_toeplitz_closed_form():
    """tridiag(a, b, c) with a c > 0 has the eigenvalues b + 2 sqrt(ac) cos(k pi / (n + 1));
    a / c close to 1 keeps them well conditioned at n = 60."""
    n, a, b, c = 60, -1.025, 2.0, -0.975
    T = np.diag(np.full(n, b)) + np.diag(np.full(n - 1, a), -1) + np.diag(np.full(n - 1, c), 1)
    lam = b + 2.0 * np.sqrt(a * c) * np.cos(np.arange(1, n + 1) * np.pi / (n + 1))
    r = eig.arnoldi(from_dense(T), 4, 20, gen.uniform_vec(n, 3), tol=1e-10, which=eig.LR)
    assert r["status"] == eig.OK
    assert np.max(np.abs(r["evals"] - np.sort(lam)[::-1][:4])) <= 1e-11


def test_arnoldi_full_space_matches_lapack():
    rng = np.random.default_rng(3)
    M = rng.standard_normal((40, 40))
    r = eig.arnoldi(from_dense(M), 5, 40, rng.standard_normal(40), tol=1e-12, which=eig.LM)
    assert r["status"] == eig.OK and r["restarts"] == 0
    ref = np.linalg.eigvals(M)
    ref = ref[np.argsort(-np.abs(ref), kind="stable")][:r["evals"].size]
    assert np.max(np.abs(np.sort_complex(r["evals"]) - np.sort_complex(ref))) <= 1e-11 * np.abs(ref[0])


def test_arnoldi_symmetric_is_lanczos_closed_form():
    n = 400
    A = lap1d(n)
    r = eig.arnoldi(A, 6, 30, gen.uniform_vec(n, 1), tol=1e-9, which=eig.LR)
    lam = np.sort(2.0 - 2.0 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1)))[::-1][:6]
    assert r["status"] == eig.OK
    assert np.max(np.abs(r["evals"] - lam)) <= 1e-10 * r["anrm"]


def test_arnoldi_breakdown_and_tuning():
    A = from_dense(np.diag(np.arange(1.0, 31.0)))
    v0 = np.zeros(30)
    v0[[2, 7, 11]] = 1.0
    assert eig.arnoldi(A, 4, 10, v0)["status"] == eig.BREAKDOWN
    r = eig.arnoldi(A, 2, 10, v0, which=eig.LR)
    assert r["status"] == eig.OK and np.allclose(r["evals"], [12.0, 8.0], atol=1e-12)
    T, d = triangular_permuted(500, 7)
    r = eig.arnoldi(T, 8, 12, gen.uniform_vec(500, 1), tol=1e-9, step=5, m_max=30, ratio=np.inf, window=3)
    assert r["m_hist"][:9] == [12] * 3 + [17] * 3 + [22] * 3
    r0 = eig.arnoldi(T, 8, 12, gen.uniform_vec(500, 1), tol=1e-9, step=5, m_max=30, ratio=0.0, window=3,
                     maxiter=300)
    assert set(r0["m_hist"]) == {12}


def convdiff_eigs(g, beta):
    k = np.arange(1, g + 1)
    lx = 2.0 + 2.0 * np.sqrt(1.0 - beta * beta) * np.cos(k * np.pi / (g + 1))
    ly = 2.0 - 2.0 * np.cos(k * np.pi / (g + 1))
    return np.sort((lx[:, None, None] + ly[None, :, None] + ly[None, None, :]).ravel())


def test_convdiff_generator_spectrum():
    """The generator's convection-diffusion matrix has the stated closed-form
    (real) spectrum: checked against LAPACK on an 8^3 grid."""
    A = gen.convdiff3d(8, 0.3)
    ev = np.linalg.eigvals(dense_of_csr(A))
    assert np.max(np.abs(ev.imag)) <= 1e-10
    assert np.max(np.abs(np.sort(ev.real) - convdiff_eigs(8, 0.3))) <= 1e-11


def test_arnoldi_convdiff_values_in_closed_form():
    g, beta = 12, 0.02
    A = gen.convdiff3d(g, beta)
    r = eig.arnoldi(A, 6, 30, gen.uniform_vec(A.n, 5), tol=1e-8, which=eig.LR)
    lam = convdiff_eigs(g, beta)
    assert r["status"] == eig.OK
    assert abs(r["evals"][0].real - lam[-1]) <= 1e-9 * r["anrm"]
    for v in r["evals"]:
        assert abs(v.imag) <= 1e-9 * r["anrm"] and np.min(np.abs(lam - v.real)) <= 1e-9 * r["anrm"]

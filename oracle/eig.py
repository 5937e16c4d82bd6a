"""CPU oracle for the restarted Lanczos eigensolver -- TEST INFRASTRUCTURE ONLY.

Imported by the test suite and the benchmark's checks, never by the product
path.  Plain FP64 numpy; the products with A use the oracle's compensated
SpMV, the small projected eigenproblem uses numpy.linalg.eigh.

What it computes (section 2.2 lists a restarted Lanczos method for the
symmetric standard eigenproblem; section 4.3 asks for 10 eigenpairs to an
accuracy of 1e-8).  The paper does not say which restart scheme its Lanczos
uses; this is the thick restart of Wu and Simon (2000):

* A basis Q = [q_0 .. q_{m-1}] with orthonormal columns, built by the
  Lanczos recurrence with full re-orthogonalisation (two classical
  Gram-Schmidt passes against every basis vector).  T = Q^T A Q is kept in
  its structured form: after a restart with k kept vectors, T[:k, :k] =
  diag(theta_0 .. theta_{k-1}), row/column k couples q_k to every kept
  vector (s_i), and from column k on T is tridiagonal with alpha_j on the
  diagonal and beta_j = ||w_j|| (the norm left after orthogonalisation)
  below it.
* After m vectors: T = Y diag(theta) Y^T.  Ritz pairs (theta_i, Q y_i) are
  ordered from the wanted end (largest or smallest algebraic).  The
  residual norm of Ritz pair i is |beta_{m-1} * Y[m-1, i]| (exact in exact
  arithmetic because A Q = Q T + beta q_m e_m^T).
* Converged: the first nev residual norms are all <= tol * anrm, where
  anrm is the largest |theta| seen so far (an estimate of ||A||_2).
* Otherwise keep k = nev + (m - nev) // 2 Ritz vectors Q Y[:, :k], append
  q_m as q_k, set s_i = beta_{m-1} * Y[m-1, i] and continue from step k.
* Restart-length tuning (the MM ratio of eq. (1) in the manner of
  section 3.2.1, with the section 4.3 growth rule), when step > 0: after
  every cycle the worst residual estimate of the nev wanted pairs relative
  to anrm is sampled; once `window` samples exist since the last change of
  m, and their MM ratio (max / min over the last `window`) is below
  `ratio`, convergence is judged stagnant and m grows by `step` up to m_max
  (the samples then start afresh).
* beta_j <= 1e-14 * (the largest |alpha|, beta or |theta| met so far) is
  taken as an invariant subspace: the cycle ends at j + 1 vectors with
  exact Ritz pairs; if fewer than nev exist then, the solve reports a
  breakdown.
"""
import numpy as np
import scipy.linalg

from . import mm_ratio, spmv

OK, NOT_CONVERGED, BREAKDOWN = 0, 1, 2
LARGEST, SMALLEST = 0, 1
# Arnoldi targets: largest / smallest real part, largest magnitude
LR, SR, LM = 0, 1, 2


def kept_count(nev, m):
    """Ritz vectors kept at a thick restart."""
    return nev + (m - nev) // 2


def _order(theta, which):
    return np.argsort(-theta, kind="stable") if which == LARGEST else np.argsort(theta, kind="stable")


def _cgs2(Q, j, w):
    """Two classical Gram-Schmidt passes of w against Q[:, :j+1]; returns
    the accumulated coefficients and the orthogonalised w."""
    B = Q[:, :j + 1]
    h = B.T @ w
    w = w - B @ h
    h2 = B.T @ w
    w = w - B @ h2
    return h + h2, w


def lanczos(A, nev, m, v0, tol=1e-8, maxiter=100000, which=LARGEST, matvec=None, step=0, m_max=0,
            ratio=0.0, window=5):
    """Thick-restart Lanczos for a symmetric A (CSR, general or lower-stored).

    Returns dict(evals[nev], evecs[n, nev], status, matvecs, restarts, anrm,
    est[nev] (residual estimates), resid[nev] (true ||A x - theta x||),
    m_hist (m of every cycle), m_final)."""
    n = A.n
    if matvec is None:
        def matvec(x):
            return spmv(A, x)[0]
    m_max = max(m, m_max) if step > 0 else m
    if not 1 <= nev < m <= m_max <= n:
        raise ValueError("need 1 <= nev < m <= m_max <= n")
    Q = np.zeros((n, m_max + 1))
    T = np.zeros((m_max, m_max))
    m_hist, samples = [], []
    Q[:, 0] = v0 / np.linalg.norm(v0)
    k = 0                 # kept Ritz vectors at the start of the cycle
    anrm = 0.0
    tscale = 0.0          # largest |alpha|, beta, |theta| so far (the invariance test's scale)
    matvecs = restarts = 0
    status = NOT_CONVERGED
    while True:
        mm = m
        beta = 0.0
        for j in range(k, m):
            w = matvec(Q[:, j])
            matvecs += 1
            h, w = _cgs2(Q, j, w)
            T[j, j] = h[j]
            beta = float(np.linalg.norm(w))
            tscale = max(tscale, abs(h[j]), beta)
            if beta <= 1e-14 * tscale:
                beta = 0.0
                mm = j + 1
                break
            if j + 1 < m:
                T[j + 1, j] = T[j, j + 1] = beta
            Q[:, j + 1] = w / beta
        m_hist.append(m)
        theta, Y = np.linalg.eigh(T[:mm, :mm])
        order = _order(theta, which)
        theta, Y = theta[order], Y[:, order]
        anrm = max(anrm, float(np.max(np.abs(theta))))
        tscale = max(tscale, anrm)
        est = np.abs(beta * Y[mm - 1, :])
        samples.append(float(np.max(est[:nev])) / anrm if mm >= nev else 0.0)
        if mm < nev:
            status = BREAKDOWN
            break
        if np.all(est[:nev] <= tol * anrm) or beta == 0.0:
            status = OK
            break
        if matvecs >= maxiter:
            break
        # thick restart (kept count from the length of the cycle just ended)
        k = kept_count(nev, m)
        Qk = Q[:, :mm] @ Y[:, :k]
        qn = Q[:, mm].copy()
        Q[:, :k] = Qk
        Q[:, k] = qn
        T[:] = 0.0
        T[np.arange(k), np.arange(k)] = theta[:k]
        T[k, :k] = T[:k, k] = beta * Y[mm - 1, :k]
        restarts += 1
        # restart-length judgment on the samples since the last change of m
        if step > 0 and m < m_max and len(samples) >= window and \
                mm_ratio(samples, len(samples), window) < ratio:
            m = min(m + step, m_max)
            samples = []
    nret = min(nev, mm)
    X = Q[:, :mm] @ Y[:, :nret]
    resid = np.array([np.linalg.norm(matvec(X[:, i]) - theta[i] * X[:, i]) for i in range(nret)])
    return {"evals": theta[:nret].copy(), "evecs": X, "status": status, "matvecs": matvecs,
            "restarts": restarts, "anrm": anrm, "est": est[:nret].copy(), "resid": resid, "m_hist": m_hist,
            "m_final": m}


# --------------------------------------------------------------- Arnoldi
def _arnoldi_key(lam, which):
    """Sort key (ascending = wanted first)."""
    if which == LR:
        return -lam.real
    if which == SR:
        return lam.real
    return -np.abs(lam)


def arnoldi(A, nev, m, v0, tol=1e-8, maxiter=100000, which=LM, matvec=None, step=0, m_max=0, ratio=0.0,
            window=5):
    """Restarted Arnoldi for a general A, Krylov-Schur restart (Stewart 2001).

    The paper names a restarted Arnoldi for unsymmetric matrices (section
    2.2) and tunes its restart frequency (section 4.4.2); the restart scheme
    is not given, so this follows Krylov-Schur:

    * Q[:, :m] orthonormal, built by the Arnoldi recurrence with full
      re-orthogonalisation (two classical Gram-Schmidt passes); H = Q^T A Q
      holds every coefficient of both passes, and beta_j = ||w_j|| after
      them goes below the diagonal.
    * After m vectors: the Ritz values are the eigenvalues of H; the wanted
      ones come first by `which` (LR, SR or LM).  The residual norm of a
      Ritz pair (lam, y), ||y|| = 1, is |beta * y[m-1]|.
    * Converged when the first nev (nev + 1 if the nev-th is one of a
      complex pair whose partner comes next) residual norms are all
      <= tol * anrm, anrm the largest |Ritz value| seen.
    * Otherwise: the real Schur form H = Z T Z^T ordered so that the k
      wanted Ritz values lead, k = nev + (m - nev) // 2 (one more when the
      cut would split a complex pair); keep Q Z[:, :k], continue from q_m
      with T[:k, :k] and the coupling row beta * Z[m-1, :k].
    * Invariance (beta <= 1e-14 * scale) and restart-length tuning as in
      the Lanczos oracle.

    Returns dict(evals (complex), evecs (real, a complex pair as its real
    and imaginary parts in two columns, like LAPACK's dgeev), status,
    matvecs, restarts, anrm, est, resid (true ||A x - lam x|| per
    eigenvalue), m_final, m_hist)."""
    n = A.n
    if matvec is None:
        def matvec(x):
            return spmv(A, x)[0]
    m_max = max(m, m_max) if step > 0 else m
    if not (1 <= nev < m - 1 and m <= m_max <= n):
        raise ValueError("need 1 <= nev < m - 1, m <= m_max <= n")
    Q = np.zeros((n, m_max + 1))
    H = np.zeros((m_max + 1, m_max))
    Q[:, 0] = v0 / np.linalg.norm(v0)
    k = 0
    anrm = tscale = 0.0
    matvecs = restarts = 0
    status = NOT_CONVERGED
    m_hist, samples = [], []
    while True:
        mm = m
        beta = 0.0
        for j in range(k, m):
            w = matvec(Q[:, j])
            matvecs += 1
            h, w = _cgs2(Q, j, w)
            H[:j + 1, j] = h
            beta = float(np.linalg.norm(w))
            tscale = max(tscale, float(np.max(np.abs(h))), beta)
            if beta <= 1e-14 * tscale:
                beta = 0.0
                mm = j + 1
                break
            H[j + 1, j] = beta
            Q[:, j + 1] = w / beta
        m_hist.append(m)
        Hm = H[:mm, :mm]
        lam, Y = np.linalg.eig(Hm)
        order = np.argsort(_arnoldi_key(lam, which), kind="stable")
        lam, Y = lam[order], Y[:, order]
        Y = Y / np.linalg.norm(Y, axis=0)
        anrm = max(anrm, float(np.max(np.abs(lam))))
        tscale = max(tscale, anrm)
        est = np.abs(beta * Y[mm - 1, :])
        ne = nev
        if ne < mm and lam[ne - 1].imag != 0.0 and np.isclose(lam[ne], np.conj(lam[ne - 1])):
            ne += 1
        samples.append(float(np.max(est[:ne])) / anrm if mm >= ne else 0.0)
        if mm < ne:
            status = BREAKDOWN
            break
        if np.all(est[:ne] <= tol * anrm) or beta == 0.0:
            status = OK
            break
        if matvecs >= maxiter:
            break
        # Krylov-Schur restart: the k wanted Ritz values lead the Schur form
        kk = nev + (m - nev) // 2
        if lam[kk - 1].imag != 0.0 and np.isclose(lam[kk], np.conj(lam[kk - 1])):
            kk += 1
        keys = _arnoldi_key(lam, which)
        cut = keys[kk - 1]
        T, Z, sdim = scipy.linalg.schur(Hm, output="real",
                                        sort=lambda re, im: _arnoldi_key(np.array([re + 1j * im]), which)[0]
                                        <= cut + 1e-12 * max(1.0, abs(cut)))
        kk = int(sdim)
        Qk = Q[:, :mm] @ Z[:, :kk]
        qn = Q[:, mm].copy()
        Q[:, :kk] = Qk
        Q[:, kk] = qn
        H[:] = 0.0
        H[:kk, :kk] = T[:kk, :kk]
        H[kk, :kk] = beta * Z[mm - 1, :kk]
        k = kk
        restarts += 1
        if step > 0 and m < m_max and len(samples) >= window and \
                mm_ratio(samples, len(samples), window) < ratio:
            m = min(m + step, m_max)
            samples = []
    ne = min(ne, mm)
    X = np.zeros((n, ne))
    resid = np.zeros(ne)
    i = 0
    while i < ne:
        x = Q[:, :mm] @ Y[:, i]
        if lam[i].imag == 0.0 or i + 1 >= ne:
            X[:, i] = x.real
            resid[i] = np.linalg.norm(matvec(x.real) - lam[i].real * x.real) if lam[i].imag == 0.0 else \
                np.linalg.norm(matvec(x.real) + 1j * matvec(x.imag) - lam[i] * x)
            i += 1
        else:
            X[:, i], X[:, i + 1] = x.real, x.imag
            r = np.linalg.norm(matvec(x.real) + 1j * matvec(x.imag) - lam[i] * x)
            resid[i] = resid[i + 1] = r
            i += 2
    return {"evals": lam[:ne].copy(), "evecs": X, "status": status, "matvecs": matvecs, "restarts": restarts,
            "anrm": anrm, "est": est[:ne].copy(), "resid": resid, "m_final": m, "m_hist": m_hist}

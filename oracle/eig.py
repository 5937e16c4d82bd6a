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

from . import mm_ratio, spmv

OK, NOT_CONVERGED, BREAKDOWN = 0, 1, 2
LARGEST, SMALLEST = 0, 1


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

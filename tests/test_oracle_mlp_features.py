"""Pins for the oracle's selector features and MLP (CPU only)."""
import math

import numpy as np
import pytest

import gen
import oracle

K = 12
F = oracle.F_FEATURES
H = oracle.HIDDEN


def _numpy_stats(A):
    """The same statistics computed independently with vectorised numpy."""
    ln = np.diff(A.rowptr.astype(np.int64))
    rows = np.repeat(np.arange(A.n, dtype=np.int64), ln)
    d = np.abs(rows - A.colind.astype(np.int64))
    nnz = int(A.nnz)
    return np.array([A.n, nnz, int((ln * ln).sum()), int(ln.max(initial=0)), int(d.max(initial=0)),
                     int((ln == 0).sum()), int((ln > 64).sum()), int(d.sum()),
                     int(ln[ln * A.n > 4 * nnz].sum())], dtype=np.int64)


@pytest.mark.parametrize("make", [
    lambda: gen.laplacian2d(64),
    lambda: gen.stencil27(10, lower=True),
    lambda: gen.powerlaw(30_000, seed=2),
    lambda: gen.trans4_like(),
    lambda: gen.blockdiag(5000, 3),
    lambda: gen.banded(4000, 17, 5, lower=True),
])
def test_feature_stats_match_numpy(make):
    A = make()
    st, f = oracle.features(A)
    assert np.array_equal(st, _numpy_stats(A))
    assert f.shape == (12,) and np.all(np.isfinite(f))
    assert f[7] == (1.0 if A.sym_lower else 0.0)


def test_features_closed_form_identity():
    n = 1024
    A = gen.CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))
    st, f = oracle.features(A)
    assert f[0] == 10.0 and f[1] == 10.0 and f[2] == 1.0 and f[3] == 0.0
    assert f[4] == 0.0 and f[5] == 0.0 and f[6] == 0.0 and f[8] == 0.0 and f[9] == 0.0
    assert f[10] == 0.0 and f[11] == 0.0


def test_features_closed_form_laplacian():
    A = gen.laplacian2d(64)
    _, f = oracle.features(A)
    assert f[0] == 12.0
    assert f[2] == 20224 / 4096
    assert f[6] == 64 / 4096             # bandwidth of the 5-point stencil
    assert f[4] == math.log2(5)


def _params(seed=5, K=K):
    """He-uniform init from the fixture generator (bounds sqrt(6/fan_in))."""
    shapes = [(H, F), (H,), (H, H), (H,), (K, H), (K,)]
    out = []
    for idx, s in enumerate(shapes):
        size = int(np.prod(s))
        if len(s) == 2:
            bound = math.sqrt(6.0 / s[1])
            out.append(gen.uniform_vec(size, seed * 16 + idx, -bound, bound))
        else:
            out.append(np.full(size, 0.01))
    return np.concatenate(out)


def _data(B=7, seed=2):
    rng = np.random.default_rng(seed)
    feat = rng.standard_normal((B, F))
    y = rng.standard_normal((B, K))
    mask = (rng.random((B, K)) < 0.8).astype(np.uint8)
    return feat, y, mask


def test_mlp_gradient_vs_finite_differences():
    p = _params()
    feat, y, mask = _data()
    loss, g = oracle.mlp_loss_grad(p, feat, y, mask, K)
    h = 1e-6
    rng = np.random.default_rng(0)
    idx = rng.choice(p.size, 200, replace=False)
    fd = np.empty(idx.size)
    for t, i in enumerate(idx):
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd[t] = (oracle.mlp_loss_grad(pp, feat, y, mask, K)[0] - oracle.mlp_loss_grad(pm, feat, y, mask, K)[0]) / (2 * h)
    err = np.linalg.norm(fd - g[idx]) / np.linalg.norm(fd)
    assert err <= 1e-6


def test_mlp_forward_vs_matrix_form():
    p = _params()
    feat, _, _ = _data(B=9)
    o = oracle.mlp_forward(p, feat, K)
    W1 = p[:H * F].reshape(H, F); off = H * F
    b1 = p[off:off + H]; off += H
    W2 = p[off:off + H * H].reshape(H, H); off += H * H
    b2 = p[off:off + H]; off += H
    W3 = p[off:off + K * H].reshape(K, H); off += K * H
    b3 = p[off:off + K]
    relu = lambda z: np.maximum(z, 0)
    ref = relu(relu(feat @ W1.T + b1) @ W2.T + b2) @ W3.T + b3
    assert np.allclose(o, ref, rtol=1e-13, atol=1e-13)


def test_mlp_zero_weights_closed_form():
    p = np.zeros(oracle.mlp_nparams(K))
    b3 = np.linspace(-1, 1, K)
    p[-K:] = b3
    feat, y, mask = _data(B=5)
    o = oracle.mlp_forward(p, feat, K)
    assert np.array_equal(o, np.tile(b3, (5, 1)))
    loss, g = oracle.mlp_loss_grad(p, feat, y, mask, K)
    cnt = mask.sum()
    assert np.all(g[:H * F] == 0.0)                                      # dW1 = 0
    assert np.allclose(g[-K:], (2 * (b3 - y) * mask).sum(0) / cnt, rtol=1e-14, atol=0)
    assert math.isclose(loss, float((((b3 - y) ** 2) * mask).sum() / cnt), rel_tol=1e-14)


def test_adam_first_step_closed_form():
    """After one step with zero moments the bias-corrected update is
    lr * g / (|g| + eps)."""
    rng = np.random.default_rng(4)
    p0 = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    oracle.adam_step(p, g, m, v, 1, lr=1e-3)
    assert np.allclose(p, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_mlp_training_learns_linear_costs():
    rng = np.random.default_rng(9)
    M = 256
    feat = rng.standard_normal((M, F))
    Wt = rng.standard_normal((K, F)) * 0.3
    y = feat @ Wt.T
    mask = np.ones((M, K), dtype=np.uint8)
    order = np.concatenate([rng.permutation(M) for _ in range(60)]).astype(np.int32)
    p, losses = oracle.mlp_train(_params(), feat, y, mask, order, 60, 32, 3e-3, K)
    assert losses[-1] < 0.1 * losses[0]


def test_adam_constant_gradient_closed_form():
    """Kingma & Ba's bias correction makes a constant gradient g give
    m_hat = g and v_hat = g^2 at every step t, so after t steps
    p_t = p_0 - t * lr * g / (|g| + eps).  A correction frozen at t = 1, or a
    step counter that does not advance, leaves m_hat != g from t = 2 on."""
    rng = np.random.default_rng(11)
    p0 = rng.standard_normal(64)
    g = rng.standard_normal(64) * np.exp(rng.uniform(-4, 4, 64))
    p, m, v = p0.copy(), np.zeros(64), np.zeros(64)
    lr = 1e-3
    for t in range(1, 13):
        oracle.adam_step(p, g, m, v, t, lr=lr)
        ref = p0 - t * lr * g / (np.abs(g) + 1e-8)
        assert np.allclose(p, ref, rtol=0, atol=t * 4e-16 * (np.abs(p0) + 1)), t
        # the raw moments are the geometric sums (1 - beta^t) g and (1 - beta^t) g^2
        assert np.allclose(m, (1 - 0.9 ** t) * g, rtol=1e-13, atol=0)
        assert np.allclose(v, (1 - 0.999 ** t) * g * g, rtol=1e-12, atol=0)


def test_adam_alternating_gradient_closed_form():
    """With g_s = (-1)^(s-1) g the first moment is a geometric series in -beta1:
    m_t = (1 - beta1) g sum_{s=1..t} beta1^(t-s) (-1)^(s-1)
        = (-1)^(t-1) g (1 - beta1)(1 - (-beta1)^t) / (1 + beta1),
    the second is (1 - beta2^t) g^2 as before; the update of step t is
    lr * m_t / (1 - beta1^t) / (|g| + eps)."""
    rng = np.random.default_rng(12)
    p0 = rng.standard_normal(40)
    g = rng.standard_normal(40)
    p, m, v = p0.copy(), np.zeros(40), np.zeros(40)
    b1, b2, lr = 0.9, 0.999, 2e-3
    ref = p0.copy()
    for t in range(1, 9):
        gt = g if t % 2 == 1 else -g
        oracle.adam_step(p, gt, m, v, t, lr=lr)
        mt = (-1) ** (t - 1) * g * (1 - b1) * (1 - (-b1) ** t) / (1 + b1)
        assert np.allclose(m, mt, rtol=1e-13, atol=1e-17), t
        assert np.allclose(v, (1 - b2 ** t) * g * g, rtol=1e-12, atol=0), t
        ref = ref - lr * (mt / (1 - b1 ** t)) / (np.abs(g) + 1e-8)
        assert np.allclose(p, ref, rtol=0, atol=1e-14), t


def test_mlp_train_is_minibatch_adam_in_the_given_order():
    """Mini-batch training = for each epoch e, batches of `batch` consecutive
    positions of order[e*M : (e+1)*M] (the last one short), each followed by
    one Adam step with a step counter that runs on across epochs.  Composed
    here from the separately pinned loss gradient and Adam step, on M = 5
    samples with batch 2 (batches 2, 2, 1) over 3 epochs with different
    orders; the epoch loss is the mean of its batch losses."""
    M, batch, epochs, lr = 5, 2, 3, 1e-2
    feat, y, mask = _data(B=M, seed=21)
    rng = np.random.default_rng(22)
    order = np.concatenate([rng.permutation(M) for _ in range(epochs)]).astype(np.int32)
    p0 = _params(seed=7)
    p_orc, losses_orc = oracle.mlp_train(p0, feat, y, mask, order, epochs, batch, lr, K)

    def compose(order_of_epoch):
        p, m, v = p0.copy(), np.zeros(p0.size), np.zeros(p0.size)
        t, losses = 0, []
        for e in range(epochs):
            idx = order_of_epoch(e)
            bl = []
            for s0 in range(0, M, batch):
                sel = idx[s0:s0 + batch]
                loss, g = oracle.mlp_loss_grad(p, feat[sel], y[sel], mask[sel], K)
                t += 1
                oracle.adam_step(p, g, m, v, t, lr=lr)
                bl.append(loss)
            losses.append(np.mean(bl))
        return p, np.array(losses)

    p_ref, losses_ref = compose(lambda e: order[e * M:(e + 1) * M])
    assert np.array_equal(p_orc, p_ref)
    assert np.allclose(losses_orc, losses_ref, rtol=1e-15, atol=0)
    # the case is sensitive to the epoch offset and to the short batch: the
    # first epoch's order reused, or the short batch dropped, change the result
    p_bad, _ = compose(lambda e: order[:M])
    assert not np.allclose(p_bad, p_orc, rtol=1e-9, atol=0)
    p_drop, _ = compose(lambda e: order[e * M:e * M + 4])
    assert not np.allclose(p_drop, p_orc, rtol=1e-9, atol=0)


def test_mlp_train_bias_only_closed_form():
    """All weights and hidden biases zero: h1 = h2 = 0 (ReLU'(0) = 0), so only
    b3 learns, with gradient 2 (b3 - c) / K for targets y = c in every sample
    (mask all ones, cnt = B K); the closed-form Adam trajectory of a gradient
    that is constant within each step then applies componentwise.  Checked
    against a scalar Adam recurrence run here in plain Python."""
    M, batch, epochs, lr = 7, 3, 4, 5e-2
    c = np.linspace(-2.0, 3.0, K)
    feat = np.random.default_rng(3).standard_normal((M, F))
    y = np.tile(c, (M, 1))
    mask = np.ones((M, K), dtype=np.uint8)
    order = np.tile(np.arange(M, dtype=np.int32), epochs)
    p0 = np.zeros(oracle.mlp_nparams(K))
    p, _ = oracle.mlp_train(p0, feat, y, mask, order, epochs, batch, lr, K)
    assert np.all(p[:-K] == 0.0)
    nsteps = epochs * ((M + batch - 1) // batch)
    b3 = np.zeros(K)
    mm, vv = np.zeros(K), np.zeros(K)
    for t in range(1, nsteps + 1):
        g = 2.0 * (b3 - c) / K
        mm = 0.9 * mm + 0.1 * g
        vv = 0.999 * vv + 0.001 * g * g
        b3 = b3 - lr * (mm / (1 - 0.9 ** t)) / (np.sqrt(vv / (1 - 0.999 ** t)) + 1e-8)
    assert np.allclose(p[-K:], b3, rtol=1e-12, atol=1e-14)

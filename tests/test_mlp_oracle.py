"""Pins of the CPU reference MLP used by the learned warm start (no GPU)."""
import numpy as np

from oracle import mlp_oracle as mo
from oracle import ntf_oracle as orc


def test_backward_matches_central_differences():
    F, H = 3, 8
    rng = np.random.default_rng(1)
    p = mo.init_params(F, H, seed=2) + 0.05 * rng.standard_normal(mo.layout(F, H)["_total"][0])
    X = rng.standard_normal((5, F * (F + 1) // 2 + F))
    T = np.abs(rng.standard_normal((5, F)))

    def loss(q):
        y, _ = mo.forward(q, X, F, H)
        return mo.mse_loss(y, T)

    y, cache = mo.forward(p, X, F, H)
    g = mo.backward(p, cache, (y - T) / y.shape[0], F, H)
    h = 1e-6
    for idx in rng.choice(p.size, 60, replace=False):
        e = np.zeros_like(p)
        e[idx] = h
        fd = (loss(p + e) - loss(p - e)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(fd)), idx


def test_adam_first_step_closed_form():
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 0.0])
    p1, m, v = mo.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=0.1)
    # step 1: m_hat = g, v_hat = g^2  ->  update = lr * g / (|g| + eps)
    np.testing.assert_allclose(p1, p - 0.1 * g / (np.abs(g) + 1e-8), rtol=1e-15)


def test_features_make_prediction_scale_equivariant():
    # NNLS: h*(aG, bw) = (b/a) h*(G, w); the normalised inputs carry this over.
    F = 4
    rng = np.random.default_rng(3)
    M = rng.random((6, F))
    G = M.T @ M
    W = rng.standard_normal((7, F))
    p = mo.init_params(F, 16, seed=4)
    rho = orc.rho_trace(G)
    h1 = mo.predict_rows(p, G, W, rho, 16)
    a, b = 3.0, 0.25
    h2 = mo.predict_rows(p, a * G, b * W, orc.rho_trace(a * G), 16)
    np.testing.assert_allclose(h2, (b / a) * h1, rtol=1e-12, atol=1e-14)
    # and the NNLS solutions themselves obey it (pinned by the exhaustive solver)
    for i in range(3):
        np.testing.assert_allclose(orc.nnls_bruteforce(a * G, b * W[i]),
                                   (b / a) * orc.nnls_bruteforce(G, W[i]), atol=1e-12)


def test_judge_keeps_the_better_candidate():
    F = 3
    G = np.diag([2.0, 1.0, 4.0])
    W = np.array([[2.0, 1.0, 4.0], [-1.0, -1.0, -1.0]])
    hstar = np.array([[1.0, 1.0, 1.0], [0.0, 0.0, 0.0]])
    assert np.allclose(mo.kkt_violation(G, W, hstar), 0.0)
    p = np.zeros(mo.layout(F, 8)["_total"][0])          # predicts h = 0 everywhere
    Hprev = np.array([[0.9, 1.1, 1.0], [0.5, 0.0, 0.0]])
    Hs, Us, take = mo.warm_start(p, G, W, 3.0, Hprev, np.zeros_like(Hprev), 8)
    # row 0: h = 0 violates KKT more than the previous iterate; row 1: h = 0 is optimal
    assert list(take) == [False, True]
    np.testing.assert_array_equal(Hs[0], Hprev[0])
    np.testing.assert_array_equal(Hs[1], np.zeros(3))
    np.testing.assert_allclose(Us[1], np.maximum(-W[1] / 3.0, 0))

"""Pins of the FP64 bracket-MLP oracle (no GPU): its gradient equals central
finite differences of its loss; the forward equals a direct numpy
evaluation of the layer definitions."""
import numpy as np


def _rand_params(rng, D, H, orc):
    P = orc.mlp_num_params(D, H)
    return rng.normal(0, 0.4, size=P)


def test_forward_matches_layer_definition(orc):
    rng = np.random.default_rng(1)
    D, H, n = 10, 64, 50
    p = _rand_params(rng, D, H, orc)
    X = rng.normal(size=(n, D))
    o = 0
    W1 = p[o:o + H * D].reshape(H, D); o += H * D
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    ref = np.maximum(np.maximum(X @ W1.T + b1, 0) @ W2.T + b2, 0) @ w3 + b3
    assert np.allclose(orc.mlp_forward(p, X, H), ref, rtol=1e-12, atol=1e-12)


def test_gradient_matches_finite_differences(orc):
    rng = np.random.default_rng(2)
    for D, H, delta in [(10, 64, 1.0), (16, 8, 0.5)]:
        p = _rand_params(rng, D, H, orc)
        X = rng.normal(size=(40, D))
        y = rng.normal(scale=3.0, size=40)
        loss, g = orc.mlp_loss_grad(p, X, y, delta, H)
        idx = rng.choice(p.size, 60, replace=False)
        idx = np.concatenate([idx, [p.size - 1, 0, H * D]])   # b3, W1[0,0], b1[0]
        eps = 1e-6
        for i in idx:
            pp, pm = p.copy(), p.copy()
            pp[i] += eps
            pm[i] -= eps
            fd = (orc.mlp_loss_grad(pp, X, y, delta, H)[0] -
                  orc.mlp_loss_grad(pm, X, y, delta, H)[0]) / (2 * eps)
            assert abs(fd - g[i]) <= 1e-5 * max(1.0, abs(fd)), (D, H, i, fd, g[i])
        # the loss is the Huber sum of the residuals
        r = orc.mlp_forward(p, X, H) - y
        a = np.abs(r)
        hub = np.where(a <= delta, 0.5 * r * r, delta * (a - 0.5 * delta)).sum()
        assert abs(loss - hub) <= 1e-9 * max(1.0, hub)

"""Pins of the FP64 bracket-MLP oracle (no GPU): its gradient equals central
finite differences of its loss; the forward equals a direct numpy
evaluation of the layer definitions; with the first layer's activations
rounded to bfloat16, forward and straight-through gradient equal the same
definitions with torch's bfloat16 conversion (round to nearest even)."""
import numpy as np
import pytest


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


def _layers(p, D, H):
    o = 0
    W1 = p[o:o + H * D].reshape(H, D); o += H * D
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    return W1, b1, W2, b2, w3, p[o]


def test_bf16_activations_match_definition(orc):
    """round_act: a1 = bf16(relu(W1 x + b1)) (binary32 first, then to
    bfloat16 with ties to even, which torch's conversion implements), used
    by the second layer and by the W2 gradient; the first layer's mask and
    the rest of the backward pass are unchanged (straight-through)."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    D, H, n, delta = 10, 64, 200, 1.0
    p = _rand_params(rng, D, H, orc)
    X = rng.normal(size=(n, D))
    y = rng.normal(scale=3.0, size=n)
    W1, b1, W2, b2, w3, b3 = _layers(p, D, H)
    z1 = X @ W1.T + b1
    a1 = torch.from_numpy(np.maximum(z1, 0).astype(np.float32)).bfloat16().double().numpy()
    assert np.any(a1 != np.maximum(z1, 0))           # the rounding is active
    z2 = a1 @ W2.T + b2
    out = np.maximum(z2, 0) @ w3 + b3
    assert np.allclose(orc.mlp_forward(p, X, H, round_act=True), out, rtol=1e-12, atol=1e-12)
    r = out - y
    g = np.where(np.abs(r) <= delta, r, np.sign(r) * delta)
    d2 = (z2 > 0) * (g[:, None] * w3[None, :])
    d1 = (z1 > 0) * (d2 @ W2)
    ref = np.concatenate([(d1.T @ X).ravel(), d1.sum(0), (d2.T @ a1).ravel(), d2.sum(0),
                          np.maximum(z2, 0).T @ g, [g.sum()]])
    loss, grad = orc.mlp_loss_grad(p, X, y, delta, H, round_act=True)
    assert np.allclose(grad, ref, rtol=1e-10, atol=1e-10)
    a = np.abs(r)
    assert abs(loss - np.where(a <= delta, 0.5 * r * r, delta * (a - 0.5 * delta)).sum()) <= 1e-9

"""Pins of the oracle's EoS surrogate network (forward pass and backpropagation), which the GPU
training kernels' gradients are checked against."""
import numpy as np
import pytest

import oracle

NP = oracle.MLP_NPARAM
H = 64
# flat parameter layout: W1[64][2], b1[64], W2[64][64], b2, W3[64][64], b3, W4[2][64], b4[2]
OFF = {"W1": 0, "b1": 128, "W2": 192, "b2": 4288, "W3": 4352, "b3": 8448, "W4": 8512, "b4": 8640}


def _silu(z):
    return z / (1.0 + np.exp(-z))


def _random_params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, NP)


def test_parameter_count():
    assert NP == 2 * H + H + H * H + H + H * H + H + 2 * H + 2


def test_output_layer_only_network():
    # with every hidden weight zero, each hidden unit sees only its bias and the output is an
    # affine map of silu(silu(silu(b))) -- checked against the closed form
    w = np.zeros(NP)
    rng = np.random.default_rng(3)
    b1, b2, b3 = rng.normal(size=(3, H))
    W4 = rng.normal(size=(2, H))
    b4 = rng.normal(size=2)
    w[OFF["b1"]:OFF["b1"] + H] = b1
    w[OFF["b2"]:OFF["b2"] + H] = b2
    w[OFF["b3"]:OFF["b3"] + H] = b3
    w[OFF["W4"]:OFF["W4"] + 2 * H] = W4.ravel()
    w[OFF["b4"]:] = b4
    x = rng.uniform(-1, 1, (5, 2))
    y = oracle.mlp_forward(w, x)
    h3 = _silu(b3)          # W3 = 0: layer 3 sees only b3; likewise layers 1-2 are irrelevant
    expect = W4 @ h3 + b4
    assert np.allclose(y, expect[None, :], rtol=0, atol=1e-14)


def test_single_path_network():
    # one active unit per layer: y0 = w4 silu(w3 silu(w2 silu(w1 x0 + b1) + b2) + b3) + b4
    w = np.zeros(NP)
    w1, b1, w2, b2, w3, b3, w4, b4 = 0.7, -0.2, 1.3, 0.1, -0.9, 0.4, 2.0, 0.5
    w[OFF["W1"] + 0] = w1                 # W1[0][0]
    w[OFF["b1"] + 0] = b1
    w[OFF["W2"] + 0] = w2                 # W2[0][0]
    w[OFF["b2"] + 0] = b2
    w[OFF["W3"] + 0] = w3
    w[OFF["b3"] + 0] = b3
    w[OFF["W4"] + 0] = w4                 # W4[0][0]
    w[OFF["b4"] + 0] = b4
    x = np.array([[0.3, -0.8], [-1.0, 1.0]])
    y = oracle.mlp_forward(w, x)
    # units 1..63 carry silu(0) = 0 into the next layer, so only unit 0 matters
    for s in range(2):
        v = b4 + w4 * _silu(w3 * _silu(w2 * _silu(w1 * x[s, 0] + b1) + b2) + b3)
        assert abs(y[s, 0] - v) < 1e-15
        assert y[s, 1] == 0.0


def test_loss_value():
    w = _random_params(1)
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, (17, 2))
    t = rng.uniform(-1, 1, (17, 2))
    loss, _ = oracle.mlp_loss_grad(w, x, t)
    y = oracle.mlp_forward(w, x)
    assert abs(loss - 0.5 * np.mean(np.sum((y - t) ** 2, axis=1))) < 1e-14


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_central_differences(seed):
    w = _random_params(seed)
    rng = np.random.default_rng(10 + seed)
    x = rng.uniform(-1, 1, (9, 2))
    t = rng.uniform(-1, 1, (9, 2))
    _, g = oracle.mlp_loss_grad(w, x, t)
    # every parameter block, several entries each
    idx = []
    for k, o in OFF.items():
        size = {"W1": 128, "b1": 64, "W2": 4096, "b2": 64, "W3": 4096, "b3": 64, "W4": 128, "b4": 2}[k]
        idx += list(o + rng.choice(size, min(size, 12), replace=False))
    eps = 1e-6
    fd = np.zeros(len(idx))
    for j, i in enumerate(idx):
        wp = w.copy(); wp[i] += eps
        wm = w.copy(); wm[i] -= eps
        fd[j] = (oracle.mlp_loss_grad(wp, x, t)[0] - oracle.mlp_loss_grad(wm, x, t)[0]) / (2 * eps)
    an = g[idx]
    err = np.abs(fd - an) / np.maximum(np.abs(an), 1e-3 * np.max(np.abs(an)))
    assert np.max(err) < 1e-6, (np.max(err), idx[int(np.argmax(err))])


def test_readout_fit_is_the_least_squares_minimiser():
    # the least-squares readout minimises the loss over W4, b4 for fixed hidden layers: the loss
    # gradient (backpropagation, pinned above by finite differences) vanishes in those two blocks,
    # the loss does not rise, the hidden layers are untouched, and the output is W4 h + b4 of the
    # network's own last hidden layer
    w = _random_params(11)
    rng = np.random.default_rng(12)
    x = rng.uniform(-1, 1, (400, 2))
    t = np.stack([np.sin(2 * x[:, 0]) + x[:, 1] ** 2, np.cos(x[:, 0] * x[:, 1])], axis=1)
    l0, g0 = oracle.mlp_loss_grad(w, x, t)
    wf = oracle.mlp_fit_readout(w, x, t, 0.0)
    l1, g1 = oracle.mlp_loss_grad(wf, x, t)
    assert l1 < l0
    assert np.array_equal(wf[:OFF["W4"]], w[:OFF["W4"]])
    ro = slice(OFF["W4"], NP)
    assert np.max(np.abs(g1[ro])) < 1e-9 * np.max(np.abs(g0[ro]))
    h = oracle.mlp_features(wf, x)
    y = h @ wf[OFF["W4"]:OFF["b4"]].reshape(2, H).T + wf[OFF["b4"]:]
    assert np.max(np.abs(y - oracle.mlp_forward(wf, x))) < 1e-12
    # a ridge term shrinks the readout towards zero
    wr = oracle.mlp_fit_readout(w, x, t, 1e-2)
    assert np.linalg.norm(wr[ro]) < np.linalg.norm(wf[ro])

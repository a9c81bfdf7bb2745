"""Pins for the oracle MLP: closed forms and finite differences."""
import math

import numpy as np
import pytest

from oracle import mlp


def test_bf16_rounding_known_values():
    # exactly representable values stay; ties round to even; 1 + 2^-8 is a tie
    x = np.array([1.0, -2.5, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 3.0e38, 0.0,
                  1.0 + 2.0 ** -8 + 2.0 ** -20])
    r = mlp.bf16_round(x)
    assert r[0] == 1.0 and r[1] == -2.5 and r[5] == 0.0
    assert r[2] == 1.0                      # tie -> even mantissa (1.0)
    assert r[3] == 1.0 + 4 * 2.0 ** -8      # tie -> even (1 + 2^-6)
    assert r[6] == 1.0 + 2 * 2.0 ** -8      # above the tie rounds up
    assert np.isinf(mlp.bf16_round(np.array([3.4e38]))[0])
    rel = np.abs(mlp.bf16_round(np.linspace(0.1, 100, 1000)) / np.linspace(0.1, 100, 1000) - 1)
    assert rel.max() <= 2.0 ** -8


def test_gelu_closed_form_and_derivative():
    z = np.array([-3.0, -1.0, 0.0, 0.5, 2.0])
    Phi = 0.5 * (1 + np.array([math.erf(v / math.sqrt(2)) for v in z]))
    assert np.allclose(mlp.gelu(z), z * Phi, rtol=0, atol=1e-15)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(z), fd, rtol=1e-8, atol=1e-10)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0 and mlp.gelu_grad(np.array([0.0]))[0] == 0.5


def make_params(rng, sizes):
    return [(rng.standard_normal((o, i)) / math.sqrt(i), 0.1 * rng.standard_normal(o))
            for i, o in zip(sizes[:-1], sizes[1:])]


def skip_params(rng, sizes):
    """Parameters of a skip network: the last layer reads hidden + input."""
    p = make_params(rng, sizes)
    W, b = p[-1]
    p[-1] = (np.concatenate([W, rng.standard_normal((W.shape[0], sizes[0])) / 3.0], axis=1), b)
    return p


@pytest.mark.parametrize("skip", [False, True])
def test_backward_matches_central_differences(skip):
    rng = np.random.default_rng(0)
    sizes = [5, 7, 6, 4]
    net = mlp.MLP(skip_params(rng, sizes) if skip else make_params(rng, sizes), skip=skip)
    x = rng.standard_normal((3, 5))
    t = rng.standard_normal((3, 4))
    loss, grads = net.backward(x, t)
    h = 1e-6
    for l, (W, b) in enumerate(net.params):
        for arr, g in ((W, grads[l][0]), (b, grads[l][1])):
            flat = arr.reshape(-1)
            gflat = g.reshape(-1)
            for idx in range(0, flat.size, max(1, flat.size // 7)):
                old = flat[idx]
                flat[idx] = old + h
                lp = net.loss(x, t)
                flat[idx] = old - h
                lm = net.loss(x, t)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - gflat[idx]) <= 1e-6 * max(1.0, abs(fd)), (l, idx, fd, gflat[idx])


def test_linear_network_gradient_is_least_squares_gradient():
    """One linear layer: dL/dW = 2 (xW^T + b - t)^T x / n exactly."""
    rng = np.random.default_rng(1)
    W = rng.standard_normal((3, 4))
    b = rng.standard_normal(3)
    net = mlp.MLP([(W, b)])
    x = rng.standard_normal((5, 4))
    t = rng.standard_normal((5, 3))
    _, g = net.backward(x, t)
    r = x @ W.T + b - t
    assert np.allclose(g[0][0], 2 * r.T @ x / r.size, rtol=1e-14)
    assert np.allclose(g[0][1], 2 * r.sum(axis=0) / r.size, rtol=1e-14)


def test_adam_first_step_moves_by_lr_times_sign():
    """With bias correction, the first Adam step is -lr * g / (|g| + eps')."""
    p = [(np.array([[1.0, -2.0]]), np.array([0.5]))]
    g = [(np.array([[0.3, -4.0]]), np.array([1e-3]))]
    st = {}
    out = mlp.adam_step(p, g, st, lr=0.01)
    assert np.allclose(out[0][0], [[1.0 - 0.01, -2.0 + 0.01]], rtol=0, atol=1e-9)
    assert np.allclose(out[0][1], [0.5 - 0.01], rtol=0, atol=1e-7)
    assert st["t"] == 1


def test_bf16_mode_rounds_operands():
    rng = np.random.default_rng(2)
    params = make_params(rng, [4, 3])
    x = rng.standard_normal((2, 4))
    y16, _ = mlp.MLP(params, bf16=True).forward(x)
    W, b = params[0]
    ref = mlp.bf16_round(x) @ mlp.bf16_round(W).T + b
    assert np.array_equal(y16, ref)


def test_skip_network_with_silent_trunk_is_the_linear_map():
    """Zero weights on the hidden part of the last layer leave y = x S^T + b,
    with S the input block of that layer: the order of the concatenation."""
    rng = np.random.default_rng(3)
    sizes = [6, 8, 8, 5]
    p = skip_params(rng, sizes)
    W, b = p[-1]
    W[:, :8] = 0.0
    net = mlp.MLP(p, skip=True)
    x = rng.standard_normal((4, 6))
    y, _ = net.forward(x)
    assert np.allclose(y, x @ W[:, 8:].T + b, rtol=0, atol=1e-14)
    # and its gradient reaches only the last layer
    _, g = net.backward(x, np.zeros((4, 5)))
    assert all(np.all(gW == 0) and np.all(gb == 0) for gW, gb in g[:-1])

"""Pins of the surrogate-network oracle (no GPU): finite differences of the
loss on every weight, finite differences of the output on the CVs, an
independent reverse-mode input gradient, closed forms, periodicity, Adam's
first step, and bfloat16 rounding on exactly representable cases."""
import numpy as np
import pytest

from oracle import mlp

rng = np.random.default_rng(77)


def rand_params(H, F, scale=0.8):
    P = mlp.init_params(H, F, 3)
    for k in P:
        P[k] = P[k] + scale * rng.normal(size=P[k].shape) * 0.3
    return P


@pytest.mark.parametrize("periodic", [[True, True], [False, False, False], [True, False]])
def test_input_gradient_fd_and_reverse(periodic):
    D = len(periodic)
    H, F = 9, 2 * D
    P = rand_params(H, F)
    mu, s = np.full(D, 0.3), np.full(D, 1.7)
    xi = rng.uniform(-2, 2, size=(7, D))
    y, dy, _ = mlp.forward(P, xi, periodic, mu, s)
    assert np.allclose(dy, mlp.input_grad_reverse(P, xi, periodic, mu, s), rtol=1e-12, atol=1e-13)
    for d in range(D):
        e = np.zeros(D)
        e[d] = 1e-6
        fd = (mlp.forward(P, xi + e, periodic, mu, s)[0] - mlp.forward(P, xi - e, periodic, mu, s)[0]) / 2e-6
        assert np.max(np.abs(fd - dy[:, d])) < 1e-8


def test_loss_gradients_fd_every_weight():
    periodic = [True, False]
    D, H = 2, 6
    F = 2 * D
    P = rand_params(H, F)
    mu, s = np.array([0.0, 0.5]), np.array([1.0, 0.8])
    xi = rng.uniform(-2, 2, size=(11, D))
    V = rng.normal(size=11)
    G = rng.normal(size=(11, D))
    L, g, _, _ = mlp.loss_and_grads(P, xi, V, G, 0.7, 1.3, periodic, mu, s)
    for k in P:
        for idx in np.ndindex(P[k].shape):
            Pp = {q: P[q].copy() for q in P}
            Pm = {q: P[q].copy() for q in P}
            Pp[k][idx] += 1e-6
            Pm[k][idx] -= 1e-6
            fd = (mlp.loss_and_grads(Pp, xi, V, G, 0.7, 1.3, periodic, mu, s)[0] -
                  mlp.loss_and_grads(Pm, xi, V, G, 0.7, 1.3, periodic, mu, s)[0]) / 2e-6
            assert abs(fd - g[k][idx]) < 1e-7 * max(1.0, abs(fd)), (k, idx, fd, g[k][idx])


def test_closed_forms_and_periodicity():
    H, F = 5, 4
    Z = {k: np.zeros_like(v) for k, v in mlp.init_params(H, F, 0).items()}
    Z["b3"] = np.array([2.5])
    xi = rng.uniform(-3, 3, size=(4, 2))
    y, dy, _ = mlp.forward(Z, xi, [True, True])
    assert np.all(y == 2.5) and np.all(dy == 0)
    # one hidden unit path: y = w3 tanh(W2 tanh(W1 f))
    P = rand_params(H, F)
    y1, dy1, _ = mlp.forward(P, xi, [True, True])
    y2, dy2, _ = mlp.forward(P, xi + 2 * np.pi * np.array([1, -2]), [True, True])
    assert np.allclose(y1, y2, atol=1e-12) and np.allclose(dy1, dy2, atol=1e-12)
    f, _ = mlp.features(xi, [True, True])
    a1 = np.tanh(f @ P["W1"].T + P["b1"])
    a2 = np.tanh(a1 @ P["W2"].T + P["b2"])
    assert np.allclose(y1, a2 @ P["w3"] + P["b3"][0], atol=1e-15)


def test_adam_first_step_and_recurrence():
    P = {"w": np.array([1.0, -2.0, 0.5])}
    g = {"w": np.array([0.3, -4.0, 0.0])}
    m = {"w": np.zeros(3)}
    v = {"w": np.zeros(3)}
    P1, m1, v1 = mlp.adam_step(P, g, m, v, 1, 0.01)
    # t = 1: bias-corrected moments are g and g^2, so the step is lr * sign(g)
    assert np.allclose(P1["w"], [1.0 - 0.01 * 0.3 / (0.3 + 1e-8), -2.0 + 0.01 * 4 / (4 + 1e-8), 0.5])
    assert np.allclose(m1["w"], 0.1 * g["w"]) and np.allclose(v1["w"], 0.001 * g["w"] ** 2)
    P2, m2, v2 = mlp.adam_step(P1, g, m1, v1, 2, 0.01)
    mh = (0.9 * m1["w"] + 0.1 * g["w"]) / (1 - 0.81)
    vh = (0.999 * v1["w"] + 0.001 * g["w"] ** 2) / (1 - 0.999 ** 2)
    assert np.allclose(P2["w"], P1["w"] - 0.01 * mh / (np.sqrt(vh) + 1e-8))


def test_bf16_rounding():
    # exactly representable values survive; ties round to even
    assert mlp.round_bf16(1.0) == 1.0 and mlp.round_bf16(-0.5) == -0.5
    assert mlp.round_bf16(1.0 + 2 ** -7) == 1.0 + 2 ** -7
    assert mlp.round_bf16(1.0 + 2 ** -8) == 1.0          # tie -> even (1.0)
    assert mlp.round_bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6  # tie -> even (1 + 2^-6)
    x = rng.normal(size=1000)
    r = mlp.round_bf16(x)
    assert np.max(np.abs(r - x) / np.abs(x)) <= 2 ** -8


def test_bf16_pair_rounding():
    # values with at most 16 significant bits (8 + 8, both halves exact) survive
    for v in [1.0 + 2 ** -7 + 2 ** -15, -(3.0 + 2 ** -12), 0.75 + 2 ** -20]:
        assert mlp.round_bf16x2(v) == v
    x = rng.normal(size=5000)
    r = mlp.round_bf16x2(x)
    # hi carries 8 bits, lo rounds the remainder (< half an ulp of hi) to 8 bits
    assert np.max(np.abs(r - x) / np.abs(x)) <= 2.0 ** -16
    assert np.max(np.abs(r - x) / np.abs(x)) > 2.0 ** -20  # not the identity
    # the pair is at least as close as the single bf16 value
    assert np.all(np.abs(r - x) <= np.abs(mlp.round_bf16(x) - x))

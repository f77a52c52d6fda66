"""Pins for the float64 MLP oracle: central finite differences, the linear
layer's closed-form gradient, and a hand-computed one-neuron case."""
import numpy as np

from oracle import mlp_ref


def init(sizes, seed=0):
    g = np.random.default_rng(seed)
    return [(g.standard_normal((o, i)) / np.sqrt(i), g.standard_normal(o) * 0.1) for i, o in zip(sizes, sizes[1:])]


def test_gradients_match_central_differences():
    sizes = [7, 16, 16, 16, 48]
    params = init(sizes)
    g = np.random.default_rng(1)
    X = g.standard_normal((40, 7))
    T = g.standard_normal((40, 48))
    M = (g.random((40, 48)) < 0.6).astype(np.float64)
    _, grads = mlp_ref.loss_and_grads(params, X, T, M)
    h = 1e-6
    for l, (W, b) in enumerate(params):
        for idx in [(0, 0), (3, 5), (W.shape[0] - 1, W.shape[1] - 1)]:
            Wp = [list(p) for p in params]
            Wp[l][0] = W.copy(); Wp[l][0][idx] += h
            Lp, _ = mlp_ref.loss_and_grads([tuple(p) for p in Wp], X, T, M)
            Wp[l][0] = W.copy(); Wp[l][0][idx] -= h
            Lm, _ = mlp_ref.loss_and_grads([tuple(p) for p in Wp], X, T, M)
            num = (Lp - Lm) / (2 * h)
            assert abs(num - grads[l][0][idx]) <= 1e-7 * max(1.0, abs(num)), (l, idx)
        j = b.shape[0] // 2
        bp = [list(p) for p in params]
        bp[l][1] = b.copy(); bp[l][1][j] += h
        Lp, _ = mlp_ref.loss_and_grads([tuple(p) for p in bp], X, T, M)
        bp[l][1] = b.copy(); bp[l][1][j] -= h
        Lm, _ = mlp_ref.loss_and_grads([tuple(p) for p in bp], X, T, M)
        assert abs((Lp - Lm) / (2 * h) - grads[l][1][j]) <= 1e-7


def test_linear_layer_closed_form():
    # One linear layer, unmasked: L = |X W^T + b - T|^2 / N gives
    # dW = (2/N) (P - T)^T X and db = (2/N) sum_rows (P - T).
    g = np.random.default_rng(2)
    X = g.standard_normal((9, 4))
    W = g.standard_normal((3, 4))
    b = g.standard_normal(3)
    T = g.standard_normal((9, 3))
    M = np.ones((9, 3))
    L, grads = mlp_ref.loss_and_grads([(W, b)], X, T, M)
    P = X @ W.T + b
    assert np.allclose(L, ((P - T) ** 2).sum() / 27)
    assert np.allclose(grads[0][0], 2.0 / 27 * (P - T).T @ X)
    assert np.allclose(grads[0][1], 2.0 / 27 * (P - T).sum(axis=0))


def test_hand_computed_relu_case():
    # x = 2; hidden z = 1.5 x - 1 = 2 (active), output p = -0.5 z + 1 = 0,
    # target 1, mask 1: L = 1, dL/dp = -2, dL/dw2 = -2 z = -4, dL/dz = 1,
    # dL/dw1 = x = 2, and a hidden unit with negative z passes no gradient.
    params = [(np.array([[1.5], [-1.0]]), np.array([-1.0, 0.0])), (np.array([[-0.5, 3.0]]), np.array([1.0]))]
    L, grads = mlp_ref.loss_and_grads(params, np.array([[2.0]]), np.array([[1.0]]), np.array([[1.0]]))
    assert L == 1.0
    assert np.allclose(grads[1][0], [[-4.0, 0.0]]) and np.allclose(grads[1][1], [-2.0])
    assert np.allclose(grads[0][0], [[2.0], [0.0]]) and np.allclose(grads[0][1], [1.0, 0.0])


def test_adam_first_step_is_sign_times_lr():
    p, m, v = mlp_ref.adam(np.array([1.0, -2.0]), np.array([0.3, -5.0]), np.zeros(2), np.zeros(2), 1, lr=0.01)
    assert np.allclose(p, [1.0 - 0.01, -2.0 + 0.01], atol=1e-9)

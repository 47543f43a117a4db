"""The FP64 reference of the screener network: backward pinned by central finite differences,
Adam against its closed-form first step, constant-gradient steps and a two-step case by hand."""
import numpy as np

from oracle import mlp_ref as M


def _data(n=37, seed=1):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 16))
    t = rng.normal(size=n) * 2.0
    return X, t


def test_backward_matches_central_differences():
    p = M.init_params(3)
    X, t = _data()
    y, cache = M.forward(p, X)
    g = M.backward(p, cache, y, t)
    h = 1e-6
    rng = np.random.default_rng(0)
    for k in p:
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in p[k].shape)
            q = {kk: vv.copy() for kk, vv in p.items()}
            q[k][idx] += h
            lp = M.loss(M.forward(q, X)[0], t)
            q[k][idx] -= 2 * h
            lm = M.loss(M.forward(q, X)[0], t)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k][idx]) <= 1e-7 * max(1.0, abs(fd)), (k, idx, fd, g[k][idx])


def test_underprediction_weight():
    # the loss penalises predictions below the target ten times harder
    assert M.loss(np.array([0.0]), np.array([1.0])) == 10.0
    assert M.loss(np.array([2.0]), np.array([1.0])) == 1.0


def test_adam_first_step_is_sign_step():
    p = M.init_params(0)
    g = {k: np.random.default_rng(1).normal(size=v.shape) for k, v in p.items()}
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(vv) for k, vv in p.items()}
    q = {k: vv.copy() for k, vv in p.items()}
    M.adam_step(q, g, m, v, 1, lr=0.01)
    for k in p:
        # bias-corrected first step: -lr * g / (|g| + eps) = -lr * sign(g)
        assert np.allclose(q[k] - p[k], -0.01 * g[k] / (np.abs(g[k]) + 1e-8), atol=1e-12)


def test_flatten_roundtrip():
    p = M.init_params(5)
    v = M.flatten(p)
    assert v.shape == (M.NPARAM,)
    q = M.unflatten(v)
    for k in p:
        assert np.array_equal(p[k], q[k])


def test_adam_constant_gradient_steps_are_sign_steps():
    # With a constant gradient g the first moment after t steps is g (1 - b1^t) and the second
    # g^2 (1 - b2^t); bias correction divides exactly these factors out, so every step of
    # t = 1..5 moves a parameter by -lr g / (|g| + eps).  A bias correction with the wrong
    # power of b1 or b2 fails from t = 2 on.
    p = M.init_params(2)
    g = {k: np.random.default_rng(4).normal(size=v.shape) for k, v in p.items()}
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(vv) for k, vv in p.items()}
    q = {k: vv.copy() for k, vv in p.items()}
    lr = 0.003
    for t in range(1, 6):
        prev = {k: vv.copy() for k, vv in q.items()}
        M.adam_step(q, g, m, v, t, lr=lr)
        for k in p:
            assert np.allclose(q[k] - prev[k], -lr * g[k] / (np.abs(g[k]) + 1e-8), rtol=1e-9, atol=1e-15), (t, k)
            assert np.allclose(m[k], g[k] * (1 - 0.9 ** t), rtol=1e-12, atol=0)
            assert np.allclose(v[k], g[k] ** 2 * (1 - 0.999 ** t), rtol=1e-12, atol=0)


def test_adam_two_steps_by_hand():
    # gradients 1 then -2 on one parameter, b1 = 0.9, b2 = 0.999, computed with exact fractions:
    #   m1 = 1/10, v1 = 1/1000; m2 = 9/100 - 2/10 = -11/100, v2 = 999/10^6 + 4/1000 = 4999/10^6
    #   m2 / (1 - 0.81) = -11/19, v2 / (1 - 0.998001) = 4999/1999
    # so the second step is -lr (-11/19) / (sqrt(4999/1999) + eps) = +0.366103527... lr.
    lr = 0.01
    p = {"w": np.array([0.5])}
    m = {"w": np.zeros(1)}
    v = {"w": np.zeros(1)}
    M.adam_step(p, {"w": np.array([1.0])}, m, v, 1, lr=lr)
    assert abs(p["w"][0] - (0.5 - lr * 1.0 / (1.0 + 1e-8))) < 1e-15
    w1 = p["w"][0]
    M.adam_step(p, {"w": np.array([-2.0])}, m, v, 2, lr=lr)
    assert abs(m["w"][0] - (-0.11)) < 1e-15
    assert abs(v["w"][0] - 0.004999) < 1e-17
    assert abs((p["w"][0] - w1) - lr * (11 / 19) / (np.sqrt(4999 / 1999) + 1e-8)) < 1e-15

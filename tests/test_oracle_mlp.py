"""The FP64 reference of the screener network: backward pinned by central finite differences,
Adam against its closed-form first step."""
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

"""Pins of the learned-guess oracle (oracle/mlp.py) against what mathematics fixes:
finite differences for the gradient, rotation and scale invariance and closed forms for the
features, the eigenpair of a boosted perfect fluid for the targets, the defining property of
Adam's first step, and loss reduction on a smooth target."""
import numpy as np

import oracle
from oracle import mlp
from paper_1508_03452_amd import workloads as W


def _params(seed=7):
    return mlp.unflatten(W.mlp_init(seed))


def test_parameter_count_and_order():
    assert mlp.N_PARAMS == 1346
    v = np.arange(mlp.N_PARAMS, dtype=np.float64)
    assert np.array_equal(mlp.flatten(mlp.unflatten(v)), v)
    P = mlp.unflatten(v)
    assert P["W1"][1, 0] == 6 and P["b1"][0] == 192 and P["W2"][0, 1] == 225 and P["b3"][1] == 1345


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    P = _params()
    for k in P:
        P[k] = P[k] + 0.1 * rng.normal(size=P[k].shape)   # nonzero biases too
    X = rng.normal(size=(40, 6))
    Yt = rng.normal(size=(40, 2))
    _, G = mlp.loss_and_grad(P, X, Yt)
    g = mlp.flatten(G)
    v = mlp.flatten(P)
    h = 1e-6
    idx = rng.choice(mlp.N_PARAMS, size=120, replace=False)
    for i in idx:
        vp, vm = v.copy(), v.copy()
        vp[i] += h
        vm[i] -= h
        fd = (mlp.loss_and_grad(mlp.unflatten(vp), X, Yt)[0] - mlp.loss_and_grad(mlp.unflatten(vm), X, Yt)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(fd), np.abs(g).max() * 1e-3), (i, fd, g[i])


def _tensor(rng, n):
    Ef = rng.uniform(1.0, 5.0, n)
    S = rng.normal(size=(n, 3)) * 0.3
    A = rng.normal(size=(n, 3, 3)) * 0.4
    Pi = A + np.transpose(A, (0, 2, 1)) + 2.0 * np.eye(3)
    N0 = rng.uniform(0.2, 2.0, n)
    return Ef, S, Pi, N0


def test_features_are_rotation_and_scale_invariant():
    rng = np.random.default_rng(5)
    Ef, S, Pi, N0 = _tensor(rng, 50)
    F = mlp.features(Ef, S, Pi, N0)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    Fr = mlp.features(Ef, S @ Q.T, np.einsum("ab,nbc,dc->nad", Q, Pi, Q), N0)
    assert np.abs(Fr - F).max() < 1e-13
    Fs = mlp.features(7.5 * Ef, 7.5 * S, 7.5 * Pi, 7.5 * N0)
    assert np.abs(Fs - F).max() < 1e-14


def test_features_of_a_fluid_at_rest():
    eps, p, n = 3.0, 0.7, 1.4
    F = mlp.features(np.array([eps]), np.zeros((1, 3)), p * np.eye(3)[None], np.array([n]))[0]
    assert np.allclose(F, [0.0, 0.0, 3 * p / eps, 0.0, np.sqrt(3) * p / eps, n / eps], rtol=0, atol=1e-15)


def test_targets_of_a_boosted_perfect_fluid():
    """T_fl = (eps + p) gamma^2 (1, beta)(1, beta) - p eta: the recovery returns eps and beta, so the
    targets are (eps / T^00, |beta|) with T^00 = gamma^2 (eps + p) - p."""
    rng = np.random.default_rng(9)
    for _ in range(10):
        eps, p = rng.uniform(1, 4), rng.uniform(0.1, 1.0)
        d = rng.normal(size=3)
        beta = d / np.linalg.norm(d) * rng.uniform(0, 0.8)
        g2 = 1 / (1 - beta @ beta)
        U = np.r_[1.0, beta]
        T = (eps + p) * g2 * np.outer(U, U) - p * np.diag([1.0, -1, -1, -1])
        r = oracle.recover(T, 1.0, np.zeros(3), np.zeros(3))
        t = mlp.targets(np.array([r["eps"]]), r["beta"][None], np.array([T[0, 0]]))[0]
        assert abs(t[0] - eps / (g2 * (eps + p) - p)) < 1e-13 and abs(t[1] - np.linalg.norm(beta)) < 1e-13


def test_first_adam_step_is_lr_times_sign():
    """With zero moments the bias-corrected first update is lr * g / (|g| + eps): lr * sign(g)."""
    rng = np.random.default_rng(1)
    P = _params()
    X, Yt = rng.normal(size=(16, 6)), rng.normal(size=(16, 2))
    _, G = mlp.loss_and_grad(P, X, Yt)
    before = mlp.flatten(P)
    mlp.adam_step(P, G, mlp.adam_state(), lr=1e-3)
    step = mlp.flatten(P) - before
    g = mlp.flatten(G)
    big = np.abs(g) > 1e-4
    assert np.allclose(step[big], -1e-3 * np.sign(g[big]), rtol=1e-3)


def test_training_fits_a_smooth_map():
    rng = np.random.default_rng(2)
    F = rng.uniform(-1, 1, size=(2048, 6))
    T = np.stack([np.sin(F[:, 0]) + 0.5 * F[:, 1] * F[:, 2], np.cos(F[:, 3]) * F[:, 4]], axis=1)
    P, norm, losses = mlp.train(F, T, _params(), iters=300, batch=256, lr=3e-3, stride=7)
    assert losses[-20:].mean() < 0.1 * losses[:5].mean()


def test_features_of_oracle_cells_are_finite_and_scale_free():
    """Features of the recovery inputs of a KH slab: finite, and f6 = N0 / E_f below 1 / c^2."""
    w = W.kh(nx=16, ny=40, v0=0.4, ratio=10.0, sigma=100.0)
    o = oracle.Oracle(w.shape, w.bc, **w.params)
    o.init(w.fields)
    o.step(5)
    ft = o.fluid_tensor()
    F = mlp.features(ft["Ef"], ft["S"], ft["Pi"], ft["N0"])
    T = mlp.targets(ft["eps"], ft["beta"], ft["Ef"])
    assert np.isfinite(F).all() and np.isfinite(T).all()
    assert (F[:, 5] < 1.0).all() and (T[:, 0] <= 1.0 + 1e-15).all() and (T[:, 1] < 1).all()

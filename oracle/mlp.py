"""Oracle of the learned recovery guess: a 6 -> 32 -> 32 -> 2 multilayer
perceptron that predicts the Landau-frame eigenvalue of a cell from rotation
and scale invariants of its fluid tensor.

TEST INFRASTRUCTURE ONLY.  Plain numpy in float64, written from the
definitions below; only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import it.  It shares no code with the HIP library.

This form is not in the paper: the paper recovers eps and u from T_fl by the
power method (Sec. III, coupling subsection).  The network only seeds the
Newton iteration that finds the same eigenvalue; it never replaces it.

Definitions (the library follows the same ones):
  inputs, from E_f = T_fl^00, S^a = T_fl^0a, Pi^ab = T_fl^ab, N^0, with
  S_hat = S / |S| (0 when S = 0):
    f1 = |S| / E_f          f2 = S_hat . Pi S_hat / E_f     f3 = tr Pi / E_f
    f4 = |Pi S_hat - (S_hat . Pi S_hat) S_hat| / E_f         f5 = |Pi|_F / E_f
    f6 = N^0 / E_f
  then x = (f - mu_x) / sd_x with statistics of the training set;
  targets t = (lambda / E_f, |beta|), normalised as y = (t - mu_t) / sd_t;
  network y = W3 tanh(W2 tanh(W1 x + b1) + b2) + b3;
  loss L = (1 / (2 n)) sum over the batch and both outputs of (y - y_target)^2;
  Adam (Kingma and Ba, 2015) with bias correction.
Parameters in the order W1 (32 x 6), b1, W2 (32 x 32), b2, W3 (2 x 32), b3:
1346 values.
"""
import numpy as np

N_IN, N_H, N_OUT = 6, 32, 2
SHAPES = (("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)), ("W3", (N_OUT, N_H)),
          ("b3", (N_OUT,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def flatten(P):
    return np.concatenate([np.asarray(P[k], dtype=np.float64).reshape(-1) for k, _ in SHAPES])


def unflatten(v):
    v = np.asarray(v, dtype=np.float64)
    P, o = {}, 0
    for k, s in SHAPES:
        n = int(np.prod(s))
        P[k] = v[o:o + n].reshape(s).copy()
        o += n
    return P


def features(Ef, S, Pi, N0):
    """Six invariants per cell.  Ef (n,), S (n, 3), Pi (n, 3, 3) symmetric, N0 (n,)."""
    Ef = np.asarray(Ef, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    Pi = np.asarray(Pi, dtype=np.float64)
    s = np.linalg.norm(S, axis=1)
    sh = np.where(s[:, None] > 0, S / np.where(s > 0, s, 1.0)[:, None], 0.0)
    PS = np.einsum("nab,nb->na", Pi, sh)
    sps = np.einsum("na,na->n", sh, PS)
    perp = np.linalg.norm(PS - sps[:, None] * sh, axis=1)
    tr = np.trace(Pi, axis1=1, axis2=2)
    fro = np.sqrt(np.einsum("nab,nab->n", Pi, Pi))
    return np.stack([s / Ef, sps / Ef, tr / Ef, perp / Ef, fro / Ef, np.asarray(N0) / Ef], axis=1)


def targets(lam, beta, Ef):
    return np.stack([np.asarray(lam) / np.asarray(Ef), np.linalg.norm(np.asarray(beta), axis=1)], axis=1)


def forward(P, X):
    """Network outputs for normalised inputs X (n, 6); returns (Y, cache)."""
    Z1 = X @ P["W1"].T + P["b1"]
    H1 = np.tanh(Z1)
    Z2 = H1 @ P["W2"].T + P["b2"]
    H2 = np.tanh(Z2)
    Y = H2 @ P["W3"].T + P["b3"]
    return Y, (X, H1, H2)


def loss_and_grad(P, X, Yt):
    """L = sum (Y - Yt)^2 / (2 n) and its gradient with respect to every parameter (backpropagation)."""
    Y, (X, H1, H2) = forward(P, X)
    n = X.shape[0]
    R = Y - Yt
    L = 0.5 * np.sum(R * R) / n
    dY = R / n
    G = {"W3": dY.T @ H2, "b3": dY.sum(axis=0)}
    dZ2 = (dY @ P["W3"]) * (1.0 - H2 * H2)
    G["W2"] = dZ2.T @ H1
    G["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ P["W2"]) * (1.0 - H1 * H1)
    G["W1"] = dZ1.T @ X
    G["b1"] = dZ1.sum(axis=0)
    return L, G


def adam_step(P, G, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place.  state holds m, v (dicts) and t."""
    state["t"] += 1
    t = state["t"]
    for k, _ in SHAPES:
        state["m"][k] = b1 * state["m"][k] + (1 - b1) * G[k]
        state["v"][k] = b2 * state["v"][k] + (1 - b2) * G[k] * G[k]
        mh = state["m"][k] / (1 - b1 ** t)
        vh = state["v"][k] / (1 - b2 ** t)
        P[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)
    return P


def adam_state():
    return {"t": 0, "m": {k: np.zeros(s) for k, s in SHAPES}, "v": {k: np.zeros(s) for k, s in SHAPES}}


def normalisation(F, T):
    """Feature and target statistics of a training set (mean, population standard deviation, floor 1e-6)."""
    mu_x, sd_x = F.mean(axis=0), np.maximum(F.std(axis=0), 1e-6)
    mu_t, sd_t = T.mean(axis=0), np.maximum(T.std(axis=0), 1e-6)
    return mu_x, sd_x, mu_t, sd_t


def train(F, T, P0, iters, batch, lr, stride):
    """Adam on minibatches: batch b takes samples (b * batch + i) * stride mod n, i < batch.
    Returns the trained parameters, the normalisation and the loss per iteration."""
    mu_x, sd_x, mu_t, sd_t = normalisation(F, T)
    X = (F - mu_x) / sd_x
    Y = (T - mu_t) / sd_t
    P = {k: np.array(v, dtype=np.float64) for k, v in P0.items()}
    st = adam_state()
    n = X.shape[0]
    losses = []
    for b in range(iters):
        idx = ((b * batch + np.arange(batch)) * stride) % n
        L, G = loss_and_grad(P, X[idx], Y[idx])
        losses.append(L)
        adam_step(P, G, st, lr)
    return P, (mu_x, sd_x, mu_t, sd_t), np.array(losses)

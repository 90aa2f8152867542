"""The learned recovery guess on the GPU, through the C ABI: MFMA forward and backward against the
FP64 oracle network (oracle/mlp.py) on the same FP16-rounded weights and inputs, sampled features
against the oracle's own cells, training, and the step with the guess against the plain oracle."""
import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_1508_03452_amd import workloads as W

from .parity_util import field_errors, field_scale, gpu_moments_np, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _f16(a):
    return np.asarray(a, dtype=np.float16).astype(np.float64)


def test_mfma_forward_and_gradient_match_the_oracle_network():
    """FP16 weights and inputs (biases FP32), FP32 accumulation: outputs, loss and every gradient
    tensor within 1e-2 of the FP64 oracle evaluated on the same rounded numbers (max-norm relative)."""
    torch = _torch_cuda()
    from paper_1508_03452_amd.rmhdlb import mlp_eval
    rng = np.random.default_rng(21)
    w = W.mlp_init(5).astype(np.float32)
    w[mlp.N_PARAMS - 2:] = [0.1, -0.2]
    n = 384
    X = rng.normal(size=(n, 6)).astype(np.float32)
    Yt = rng.normal(size=(n, 2)).astype(np.float32)
    Y, g, loss = mlp_eval(w, torch.from_numpy(X).cuda(), torch.from_numpy(Yt).cuda())
    Y, g, loss = Y.cpu().numpy(), g.cpu().numpy(), float(loss.cpu().numpy()[0])
    P = mlp.unflatten(w.astype(np.float64))
    for k in ("W1", "W2", "W3"):
        P[k] = _f16(P[k])
    Yo, _ = mlp.forward(P, _f16(X))
    Lo, Go = mlp.loss_and_grad(P, _f16(X), Yt.astype(np.float64))
    print(f"[guess] forward max rel {np.abs(Y - Yo).max() / np.abs(Yo).max():.2e}", flush=True)
    assert np.abs(Y - Yo).max() <= 1e-2 * np.abs(Yo).max()
    assert abs(loss - Lo) <= 1e-2 * Lo
    G = mlp.unflatten(g.astype(np.float64))
    for k, _ in mlp.SHAPES:
        err = np.abs(G[k] - Go[k]).max() / np.abs(Go[k]).max()
        print(f"[guess] grad {k} rel {err:.2e}", flush=True)
        assert err <= 1e-2, k


def test_sampled_features_and_targets_match_the_oracle_cells():
    _torch_cuda()
    w = W.kh(nx=96, ny=160, v0=0.4, ratio=10.0, sigma=1e3)
    o = run_oracle(w, 5)
    s = run_gpu(w, 5)
    ns = 1000
    F, T, rc = s.guess_samples(ns)
    assert rc == 0
    ft = o.fluid_tensor()
    cells = (np.arange(ns, dtype=np.int64) * w.ncells) // ns
    Fo = mlp.features(ft["Ef"][cells], ft["S"][cells], ft["Pi"][cells], ft["N0"][cells])
    To = mlp.targets(ft["eps"][cells], ft["beta"][cells], ft["Ef"][cells])
    ef = np.abs(F.cpu().numpy() - Fo).max() / np.abs(Fo).max()
    et = np.abs(T.cpu().numpy() - To).max()
    print(f"[guess] features {ef:.2e} targets {et:.2e}", flush=True)
    assert ef < 1e-12 and et < 1e-12


def _trained_solver(w, steps, storage="f64", iters=400):
    s = run_gpu(w, steps, storage=storage)
    weights, losses = s.train_guess(W.mlp_init(11), n_samples=min(w.ncells, 16384), iters=iters, batch=512,
                                    lr=3e-3)
    return s, weights, losses


def test_training_reduces_the_loss():
    _torch_cuda()
    s, weights, losses = _trained_solver(W.kh(nx=96, ny=160, v0=0.4, ratio=10.0, sigma=1e3), 10)
    print(f"[guess] loss {losses[:3]} -> {losses[-3:]}", flush=True)
    assert np.isfinite(losses).all()
    assert losses[-20:].mean() < 0.2 * losses[:5].mean()
    assert np.isfinite(weights["w"]).all() and (weights["sd_x"] > 0).all()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_step_with_learned_guess_matches_the_plain_oracle(storage):
    """Newton from the network's guess reaches the same root: the FP64 state agrees with the plain
    oracle to the plain bound; the FP32 (one lane per cell) and FP16-shifted forms stay within their
    stated bounds.  The iteration
    counts with and without the guess are reported (the gain test)."""
    _torch_cuda()
    w = W.kh(nx=96, ny=160, v0=0.4, ratio=10.0, sigma=1e3)
    s, weights, _ = _trained_solver(w, 10, storage)
    plain = run_gpu(w, 10, storage=storage)
    s.set_guess(True)
    s.step(10)
    plain.step(10)
    o = run_oracle(w, 20)
    mo = o.moments()
    mg = gpu_moments_np(s)
    mp = gpu_moments_np(plain)
    dg, dp = mg["diag"], mp["diag"]
    assert dg["n_failed"] == 0
    print(f"[guess] {storage} mean Newton iterations: guess {dg['mean_iters']:.3f} "
          f"(fallbacks {dg['n_fallback']}) vs plain {dp['mean_iters']:.3f}; "
          f"hist guess {dg['newton_hist'][:8].tolist()} plain {dp['newton_hist'][:8].tolist()}", flush=True)
    errs = field_errors(mo, mg, field_scale(w))
    worst = max(errs, key=errs.get)
    print(f"[guess] {storage} vs oracle worst {worst}={errs[worst]:.2e}", flush=True)
    if storage == "f64":
        assert errs[worst] <= TOL, (worst, errs[worst])
    else:
        e_plain = field_errors(mo, mp, field_scale(w))
        # same stated bound as the plain form of this storage (the root is the same; only rounding differs)
        for k in errs:
            assert errs[k] <= max(5e-2 if k in ("Jx", "Jy", "Jz", "rho_c") else 5e-3, 2 * e_plain[k]), k
    assert dg["n_fallback"] < 0.05 * w.ncells


def test_learned_guess_gains_on_fast_flows():
    """The gain test.  On a fast smooth random flow (64 x 64 x 32, |u| up to 0.72c; tau = 3 keeps the
    explicit collision stable there) plain Newton from E_f needs about five iterations per cell.  The
    network, trained on the GPU on cells of the same state, seeds Newton near the root: the recovered
    fields are the plain ones to 1e-12 and the mean Newton iteration count drops.  The time of five
    steps with and without the guess is reported beside it."""
    torch = _torch_cuda()
    w = W.random_state(shape=(64, 64, 32), seed=31, vmax=1.0, modes=1, Bmag=0.1, Emag=0.01, sigma=10.0, tau=3.0)
    s, _, losses = _trained_solver(w, 0)
    plain = run_gpu(w, 0)
    mp = gpu_moments_np(plain)
    s.set_guess(True)
    mg = gpu_moments_np(s)
    dp, dg = mp["diag"], mg["diag"]
    assert dp["n_failed"] == 0 and dg["n_failed"] == 0
    errs = field_errors(mp, mg, field_scale(w))
    worst = max(errs, key=errs.get)
    times = {}
    for name, sol in (("plain", plain), ("guess", s)):
        sol.step(1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(sol.stream)
        sol.step(5)
        e1.record(sol.stream)
        torch.cuda.synchronize()
        times[name] = e0.elapsed_time(e1) / 5
    print(f"[guess] fast flow: mean Newton iterations plain {dp['mean_iters']:.3f} -> guess {dg['mean_iters']:.3f} "
          f"(fallbacks {dg['n_fallback']} of {w.ncells}); hist plain {dp['newton_hist'][:10].tolist()} "
          f"guess {dg['newton_hist'][:10].tolist()}; step {times['plain']:.4f} ms plain, {times['guess']:.4f} ms "
          f"guess; worst field gap {worst}={errs[worst]:.1e}; loss {losses[0]:.3f} -> {losses[-1]:.4f}", flush=True)
    assert errs[worst] <= TOL, (worst, errs[worst])
    assert dg["mean_iters"] <= 0.8 * dp["mean_iters"], (dg["mean_iters"], dp["mean_iters"])
    assert dg["n_fallback"] < 0.05 * w.ncells


@pytest.mark.parametrize("storage", ["f64", "f16"])
def test_guess_gate_closes_on_slow_flows(storage):
    """On a slow flow (flare box 32 x 32 x 32, drive 0.1c: every cell's |S| / E_f stays below the gate of
    0.1) the network runs in the first step only (the gate opens when the guess is enabled and closes
    when a step meets no cell above it); the other steps take the plain recovery, so the state is
    that of the plain form to rounding (the network and monitor kernels are other instantiations of the
    same cell code: bitwise in FP16, within the plain parity bound 1e-12 of each state array's scale in
    FP64, measured 6e-14), and the diagnostics count one network step."""
    _torch_cuda()
    w = W.flare(nx=32, ny=32, nz=32, Lz=6.0)
    s, _, _ = _trained_solver(w, 2, storage)
    plain = run_gpu(w, 2, storage=storage)
    s.set_guess(True)
    s.step(6)
    plain.step(6)
    dg = s.moments(fields=())["diag"]
    assert dg["guess_steps"] == 1 and dg["n_failed"] == 0, dg["guess_steps"]
    a, b = s.get_state().cpu().numpy(), plain.get_state().cpu().numpy()
    scale = np.abs(b).reshape(b.shape[0], -1).max(axis=1)
    gap = (np.abs(a - b).reshape(b.shape[0], -1).max(axis=1) / np.maximum(scale, 1e-300)).max()
    print(f"[guess] gate closed, {storage}: largest state gap to the plain form {gap:.1e}", flush=True)
    assert gap <= TOL, gap


def test_guess_gate_stays_open_on_fast_flows():
    """On the KH layer at v0 = 0.4 (|S| / E_f near 0.4 away from the layer) every step runs the network,
    and init_fields resets the count."""
    _torch_cuda()
    w = W.kh(nx=96, ny=160, v0=0.4, ratio=10.0, sigma=1e3)
    s, _, _ = _trained_solver(w, 3)
    s.set_guess(True)
    s.step(5)
    d = s.moments(fields=())["diag"]
    assert d["guess_steps"] == 5 and d["step"] == 8, (d["guess_steps"], d["step"])
    s.init_fields(w.fields)
    s.step(2)
    d = s.moments(fields=())["diag"]
    assert d["guess_steps"] == 2 and d["step"] == 2

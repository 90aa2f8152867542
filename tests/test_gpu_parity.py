"""Parity of the HIP library (called through the C ABI) with the oracle.

Plain FP64 path, per-field error = max |gpu - oracle| / max(max |oracle|,
floor), floors c for u and the run's field scale for E, B, J, rho_c.

Tolerance: 1e-12 at the stated step counts.  For the longer stiff or
shearing runs ("conditioned") the bound of a field is max(1e-12, 4 s), where
s is the oracle's own sensitivity: the difference between two oracle runs
whose initial states differ by one ulp (relative 2^-52 noise, keeping the
workload's symmetry).  No implementation can agree with the oracle more
closely than the oracle agrees with itself under rounding, and an
implementation that rounds differently at every step lands about one to two
s away (one-ulp noise injected at every step of the oracle gives the same s
as one initial ulp); for the stiff high-sigma and shear-layer runs that
floor passes 1e-12 after a few hundred steps.  Floors of the
per-field error: c for u, the field scale for E, B, J, rho_c, the largest
eps for p and eps.  Diagnostics (sums in another order) agree to 1e-13
relative.
"""
import numpy as np
import pytest

import oracle
from paper_1508_03452_amd import workloads as W

from .parity_util import field_errors, field_scale, gpu_moments_np, run_gpu, run_oracle, state_errors

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def oracle_sensitivity(w, steps, o_ref, symmetric):
    """Per-field and per-state-group difference between the oracle and the
    oracle started from a one-ulp perturbed state."""
    b = oracle.Oracle(w.shape, w.bc, **w.params)
    b.init(w.fields)
    if w.driven is not None:
        b.set_driven(w.driven)
    if w.force is not None:
        b.set_force(*w.force)
    st = b.get_state()
    rng = np.random.default_rng(1234)
    shp = (st.shape[0], 1, 1, st.shape[3]) if symmetric else st.shape
    b.set_state(st * (1 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=shp)))
    b.step(steps)
    return (field_errors(o_ref.moments(), b.moments(), field_scale(w)),
            state_errors(o_ref.get_state(), b.get_state(), field_scale(w)),
            abs(b.diagnostics()["charge"] - o_ref.diagnostics()["charge"]))


def check_case(w, steps, conditioned=False, symmetric=False):
    _torch_cuda()
    print(f"[parity] {w.name} shape={w.shape} steps={steps}", flush=True)
    o = run_oracle(w, steps)
    s = run_gpu(w, steps)
    mo = o.moments()
    mg = gpu_moments_np(s)
    assert mo["n_failed"] == 0 and mg["diag"]["n_failed"] == 0
    errs = field_errors(mo, mg, field_scale(w))
    serr = state_errors(o.get_state(), s.get_state().cpu().numpy(), field_scale(w))
    ctol = 1e-12 * max(1.0, w.ncells * 1e-3)
    if conditioned:
        fs, ss, cs = oracle_sensitivity(w, steps, o, symmetric)
        ftol = {k: max(TOL, 4 * v) for k, v in fs.items()}
        stol = {k: max(TOL, 4 * v) for k, v in ss.items()}
        # the charge is the sum of the rho_c field: its bound follows from the per-cell one
        rho_den = max(np.abs(mo["rho_c"]).max(), field_scale(w))
        ctol = max(ctol, 4 * cs, ftol["rho_c"] * rho_den * w.ncells)
        print("[parity] oracle self-sensitivity: " + " ".join(f"{k}={v:.1e}" for k, v in fs.items()) +
              f" charge={cs:.1e}", flush=True)
    else:
        ftol = {k: TOL for k in errs}
        stol = {k: TOL for k in serr}
    print("[parity] gpu vs oracle: " + " ".join(f"{k}={v:.1e}" for k, v in errs.items()), flush=True)
    print(f"[parity] state {serr}", flush=True)
    bad = {k: (v, ftol[k]) for k, v in errs.items() if v > ftol[k]}
    assert not bad, bad
    bad = {k: (v, stol[k]) for k, v in serr.items() if v > stol[k]}
    assert not bad, bad
    # global sums: 1e-13 for the different summation order, or the state-level
    # bound of this case when that is larger (they sum per-cell differences)
    dtol = max(1e-13, max(stol.values()))
    do, dg = o.diagnostics(), mg["diag"]
    for k in ("energy", "mass", "em_energy"):
        assert abs(dg[k] - do[k]) <= dtol * abs(do[k]), (k, dg[k], do[k])
    assert np.abs(dg["momentum"] - do["momentum"]).max() <= dtol * abs(do["energy"])
    assert abs(dg["charge"] - do["charge"]) <= ctol, (dg["charge"], do["charge"], ctol)
    # the GPU's charge is the sum of its own rho_c field (summation order only)
    assert abs(dg["charge"] - mg["rho_c"].sum()) <= 1e-13 * max(np.abs(mg["rho_c"]).sum(), 1e-300) + 1e-300
    # div B is a difference quotient: its natural scale is |B| / dx
    assert abs(dg["max_divB"] - do["max_divB"]) <= 1e-12 * max(do["max_divB"], field_scale(w) / w.params["dx"])
    check_null_point(w, mo, mg, do, dg, ftol)
    check_newton_histogram(w, dg)
    return errs


def check_null_point(w, mo, mg, do, dg, ftol):
    """Reconnection rate: same null cell as the oracle, or (near-tie) a cell whose key is the band minimum
    to rounding; R within the E_z bound divided by B0."""
    assert abs(dg["B0"] - do["B0"]) <= 1e-15 * max(do["B0"], 1e-300)
    assert dg["null_index"] >= 0 and do["null_index"] >= 0
    key = mo["Bx"] ** 2 + mo["By"] ** 2
    flat = key.reshape(-1)
    if dg["null_index"] != do["null_index"]:
        assert flat[dg["null_index"]] <= flat[do["null_index"]] * (1 + 1e-11) + 1e-300, (dg["null_index"],
                                                                                             do["null_index"])
        ez = mo["Ez"].reshape(-1)[dg["null_index"]]
        ref = (ez - w.fields["E"][2].reshape(-1)[dg["null_index"]]) / do["B0"]
    else:
        ref = do["recon_rate"]
    tol = max(ftol["Ez"], TOL) * max(np.abs(mo["Ez"]).max(), field_scale(w)) / do["B0"]
    print(f"[parity] null {dg['null_index']} / {do['null_index']}: R {dg['recon_rate']:.6e} vs {ref:.6e}", flush=True)
    assert abs(dg["recon_rate"] - ref) <= tol, (dg["recon_rate"], ref, tol)


def check_newton_histogram(w, dg):
    """Every cell is counted once, and the histogram carries the mean iteration count."""
    h = dg["newton_hist"]
    assert h.sum() == w.ncells and (h >= 0).all()
    if h[15] == 0:
        assert abs((h * np.arange(16)).sum() / w.ncells - dg["mean_iters"]) <= 1e-12 * max(dg["mean_iters"], 1.0)


def test_init_round_trip():
    w = W.random_state(shape=(70, 6, 3), seed=1, vmax=0.1, Bmag=0.2, Emag=0.02, sigma=3.0)
    check_case(w, 0)


def test_random_3d_periodic_ragged_tiles():
    # 70 x 6 x 3 spans two 64 x 4 tiles per axis with ragged tails
    w = W.random_state(shape=(70, 6, 3), seed=2, vmax=0.1, Bmag=0.2, Emag=0.02, sigma=3.0)
    check_case(w, 12)


def test_printed_collision_random_3d_ragged_tiles():
    """The printed semi-implicit f collision (collision = 1), 12 steps of a ragged periodic 3-D state."""
    w = W.random_state(shape=(70, 6, 3), seed=2, vmax=0.1, Bmag=0.2, Emag=0.02, sigma=3.0)
    w.params["collision"] = 1
    check_case(w, 12)


def test_printed_collision_supersonic_kh():
    """The paper's KH set-up at U0 = 0.6c on 64 x 64 cells (x periodic, y open) with the printed
    collision, a 60-step prefix (the supersonic shear amplifies rounding about a million-fold over
    300 steps); conditioning-derived bound."""
    w = W.kh_box(n_cells=64, U0=0.6, sigma=100.0)
    w.params["collision"] = 1
    check_case(w, 60, conditioned=True)


def test_lax_wendroff_flux_random_3d_ragged_tiles():
    """The limited Lax-Wendroff face values (flux = 1), 12 steps of a ragged periodic 3-D state."""
    w = W.random_state(shape=(70, 6, 3), seed=2, vmax=0.1, Bmag=0.2, Emag=0.02, sigma=3.0)
    w.params["flux"] = 1
    check_case(w, 12)


def test_lax_wendroff_flux_with_printed_collision_open_faces():
    """Both alternative readings together on a box open on every face, 10 steps."""
    w = W.random_state(shape=(20, 9, 7), seed=3, vmax=0.05, Bmag=0.2, Emag=0.02, sigma=30.0, solenoidal=True,
                       bc=(("open", "open"),) * 3)
    w.params.update(flux=1, collision=1)
    check_case(w, 10)


def _random_force(w, seed, amp):
    rng = np.random.default_rng(seed)
    nx, ny, nz = w.shape
    x, y, z = np.meshgrid(np.arange(nx) / nx, np.arange(ny) / ny, np.arange(nz) / nz, indexing="xy")
    F = []
    for a in range(3):
        k = rng.integers(1, 3, size=3)
        ph = rng.uniform(0, 2 * np.pi, size=3)
        f = amp * np.sin(2 * np.pi * k[0] * x + ph[0]) * np.cos(2 * np.pi * k[1] * y + ph[1]) * np.sin(
            2 * np.pi * k[2] * z + ph[2])
        F.append(np.ascontiguousarray(np.transpose(f, (2, 0, 1))))      # (nz, ny, nx)
    return tuple(F)


def test_external_force_random_3d_ragged_tiles():
    """The external force (Reading R26), always on, with a smooth random force field: 12 steps of a
    ragged periodic 3-D state."""
    w = W.random_state(shape=(70, 6, 3), seed=2, vmax=0.1, Bmag=0.2, Emag=0.02, sigma=3.0)
    w.force = (_random_force(w, 5, 0.02), 0.0)
    check_case(w, 12)


def test_external_force_gate_closes():
    """A gate below the state's velocities: the force acts in the first step only (the gate reads the
    previous step's largest |beta|, zero before the first step), on a box open on every face."""
    w = W.random_state(shape=(20, 9, 7), seed=3, vmax=0.05, Bmag=0.2, Emag=0.02, sigma=30.0, solenoidal=True,
                       bc=(("open", "open"),) * 3)
    w.force = (_random_force(w, 6, 0.05), 1e-6)
    check_case(w, 8)


def test_autotune_keeps_the_force_gate():
    """Timing a forced context runs forced steps, whose per-step maximum of |beta| feeds the gate of the
    next step: the tuner must leave the gate at the value of the last real step (open right after init).
    The gated run of test_external_force_gate_closes, autotuned before its first step, still equals the
    oracle."""
    _torch_cuda()
    w = W.random_state(shape=(20, 9, 7), seed=3, vmax=0.05, Bmag=0.2, Emag=0.02, sigma=30.0, solenoidal=True,
                       bc=(("open", "open"),) * 3)
    w.force = (_random_force(w, 6, 0.05), 1e-6)
    s = run_gpu(w, 0)
    print(f"[parity] forced gate, autotuned shape {s.autotune()}", flush=True)
    s.step(8)
    o = run_oracle(w, 8)
    serr = state_errors(o.get_state(), s.get_state().cpu().numpy(), field_scale(w))
    print(f"[parity] state {serr}", flush=True)
    assert max(serr.values()) <= TOL, serr


def test_external_force_with_printed_collision():
    """The external force together with the printed semi-implicit collision, 12 steps."""
    w = W.random_state(shape=(70, 6, 3), seed=2, vmax=0.1, Bmag=0.2, Emag=0.02, sigma=3.0)
    w.params["collision"] = 1
    w.force = (_random_force(w, 7, 0.02), 0.0)
    check_case(w, 12)


def test_flare_set_up_of_the_paper_with_its_force():
    """The stellar-flare set-up of Sec. IV at 32^3 (dx = 0.1875, c = 2.5, all faces open, initial E from
    the steady resistive balance, the force in the bottom band), 40 steps."""
    w = W.flare_box(n=32)
    check_case(w, 40, conditioned=True)


def test_printed_collision_limits():
    """The printed collision has 64-wide tiles and no learned guess or batches."""
    torch = _torch_cuda()
    from paper_1508_03452_amd.rmhdlb import Batch, RmhdlbError
    w = W.random_state(shape=(20, 9, 7), seed=3, vmax=0.05, Bmag=0.2, Emag=0.02, sigma=30.0)
    w.params["collision"] = 1
    s = run_gpu(w, 0)
    with pytest.raises(RmhdlbError):
        s.set_tuning(32, 4)
    assert s.autotune()[0] == 64
    with pytest.raises(RmhdlbError):
        Batch([(w.shape, w.bc, w.params)], storage="f32", stream=torch.cuda.current_stream())
    s.set_guess_weights(dict(w=W.mlp_init(11).astype(np.float32), mu_x=np.zeros(6), sd_x=np.ones(6),
                             mu_t=np.zeros(2), sd_t=np.ones(2)))
    with pytest.raises(RmhdlbError):
        s.set_guess(True)
    s.step(1)
    assert s.moments(fields=())["diag"]["n_failed"] == 0


def test_previous_B_reading_random_3d_ragged_tiles():
    """The previous step's B in the recovery and f_eq (b_prev = 1, the paper's wording), carried as
    B_prev in the state: 12 steps of the ragged periodic 3-D state, every state group to 1e-12."""
    w = W.random_state(shape=(70, 6, 3), seed=2, vmax=0.1, Bmag=0.2, Emag=0.02, sigma=3.0)
    w.params["b_prev"] = 1
    check_case(w, 12)


def test_previous_B_reading_driven_and_open_faces():
    """b_prev = 1 with the driven low-z face and open y faces (the ghost planes carry B_prev too)."""
    w = _driven_case()
    w.params["b_prev"] = 1
    check_case(w, 15)


def test_previous_B_reading_limits():
    """The previous-B reading has 64-wide tiles and no learned guess, force or batches."""
    torch = _torch_cuda()
    from paper_1508_03452_amd.rmhdlb import Batch, RmhdlbError
    w = W.random_state(shape=(20, 9, 7), seed=3, vmax=0.05, Bmag=0.2, Emag=0.02, sigma=30.0)
    w.params["b_prev"] = 1
    s = run_gpu(w, 0)
    assert s.state_len() == 69 * w.ncells
    with pytest.raises(RmhdlbError):
        s.set_tuning(32, 4)
    assert s.autotune()[0] == 64
    with pytest.raises(RmhdlbError):
        Batch([(w.shape, w.bc, w.params)], storage="f32", stream=torch.cuda.current_stream())
    with pytest.raises(RmhdlbError):
        s.set_force(_random_force(w, 5, 0.02), 0.0)
    s.step(1)
    assert s.moments(fields=())["diag"]["n_failed"] == 0


@pytest.mark.parametrize("nu", [4.5, 27 ** 0.25])
def test_lattice_nu_other_than_sqrt27(nu):
    """nu enters the g weights, the g equilibrium's coefficients and the g collision rate
    nu^2 / (sqrt 27 tau) (Readings R1, R12): a 12-step parity run at nu = 4.5 and at 27^(1/4) (where two
    g weights are negative; stable over these steps)."""
    w = W.random_state(shape=(70, 6, 3), seed=2, vmax=0.1, Bmag=0.2, Emag=0.02, sigma=3.0)
    w.params["nu"] = nu
    check_case(w, 12)


def test_torch_and_library_workspaces_step_identically():
    """The same run with the device memory allocated by torch (the binding's default: a workspace
    tensor of rmhdlb_workspace_bytes) and by the library itself: bitwise the same states."""
    torch = _torch_cuda()
    from paper_1508_03452_amd.rmhdlb import Solver
    w = _driven_case()
    states = []
    for ws in ("torch", "library"):
        s = Solver(w.shape, w.bc, workspace=ws, **w.params)
        assert (s.workspace is not None) == (ws == "torch")
        s.init_fields(w.fields)
        s.set_driven_face(w.driven)
        s.step(9)
        states.append(s.get_state())
    assert torch.equal(states[0], states[1])


def test_calls_before_the_state_is_set_report_estate():
    """rmhdlb_step, rmhdlb_moments, rmhdlb_get_state and rmhdlb_autotune before rmhdlb_init_fields (or
    rmhdlb_set_state) return RMHDLB_ESTATE; set_state then makes the context usable."""
    _torch_cuda()
    from paper_1508_03452_amd.rmhdlb import RMHDLB_ESTATE, RmhdlbError, Solver
    w = W.random_state(shape=(8, 6, 4), seed=5, vmax=0.05)
    s = Solver(w.shape, w.bc, **w.params)
    for call in (lambda: s.step(1), lambda: s.moments(), lambda: s.get_state(), lambda: s.autotune()):
        with pytest.raises(RmhdlbError) as e:
            call()
        assert e.value.code == RMHDLB_ESTATE
    ref = run_gpu(w, 0)
    s.set_state(ref.get_state())
    s.step(2)
    ref.step(2)
    import torch
    assert torch.equal(s.get_state(), ref.get_state())


def test_random_3d_open_faces():
    """Open faces on every axis with the normal-B adjustment (div B = 0 on the faces)."""
    w = W.random_state(shape=(20, 9, 7), seed=3, vmax=0.05, Bmag=0.2, Emag=0.02, sigma=30.0,
                       bc=(("open", "open"),) * 3, divb_fix=1)
    check_case(w, 10)


def test_solenoidal_box_open_on_every_face_40_steps():
    w = W.random_state(shape=(20, 9, 7), seed=3, vmax=0.05, Bmag=0.1, sigma=30.0, bc=(("open", "open"),) * 3,
                       solenoidal=True, divb_fix=1)
    check_case(w, 40)


def test_random_3d_open_faces_without_divb_fix():
    w = W.random_state(shape=(20, 9, 7), seed=3, vmax=0.05, Bmag=0.2, Emag=0.02, sigma=30.0,
                       bc=(("open", "open"),) * 3, divb_fix=0)
    check_case(w, 10)


def _driven_case(shape=(20, 9, 12), seed=5, v_drive=0.15, storage="f64"):
    bc = (("periodic", "periodic"), ("open", "open"), ("driven", "open"))
    w = W.random_state(shape=shape, seed=seed, vmax=0.05, Bmag=0.2, Emag=0.02, sigma=30.0, bc=bc)
    nx, ny, _ = shape
    rng = np.random.default_rng(seed)
    yy = (np.arange(ny) + 0.5 - ny / 2)[:, None] * np.ones((1, nx))
    w.driven = dict(n=w.fields["n"][0].copy(), p=w.fields["p"][0].copy(),
                    u=(v_drive * np.tanh(yy / 2.0) * (1 + 1e-3 * rng.uniform(-1, 1, (ny, nx))),
                       np.zeros((ny, nx)), np.zeros((ny, nx))),
                    B=tuple(b[0].copy() for b in w.fields["B"]))
    return w


def test_driven_bottom_face():
    """Driven low-z face (fixed equilibrium ghost planes of a prescribed shear) under open y faces."""
    check_case(_driven_case(), 15)


def test_driven_face_rejects_invalid_fields():
    from paper_1508_03452_amd.rmhdlb import RmhdlbError
    _torch_cuda()
    w = _driven_case(shape=(8, 6, 5))
    s = run_gpu(w, 0)
    bad = dict(w.driven)
    bad["u"] = (np.full((6, 8), 1.0), np.zeros((6, 8)), np.zeros((6, 8)))
    with pytest.raises(RmhdlbError):
        s.set_driven_face(bad)
    s.step(2)  # the ghost planes kept the valid fields
    assert s.moments(fields=())["diag"]["n_failed"] == 0


def test_alfven_wave_500_steps():
    """Ideal-limit Alfven wave, periodic 256x4x4, sigma = 1e6, 500 steps (J amplifies the rounding of
    E by sigma, so the bound is conditioning-derived)."""
    check_case(W.alfven(), 500, conditioned=True, symmetric=True)


@pytest.mark.parametrize("steps", [283, 425])
def test_alfven_wave_of_the_paper(steps):
    """The paper's Alfven set-up: 400 cells on [-1, 1] (dx = 0.005), open ends, sigma = 1e5, initial
    charge from Gauss's law, to the two times it is compared at, t = 1 and 1.5 (283 and 425 steps);
    conditioning-derived bound (stiff Ohm coupling)."""
    check_case(W.alfven_box(), steps, conditioned=True, symmetric=True)


@pytest.mark.parametrize("sigma", [100.0, 50.0])
def test_current_sheet_of_the_paper(sigma):
    """The paper's current-sheet set-up: 100 cells on [-1.5, 1.5] (dx = 0.03), open ends, p = 50,
    run to t = 9 (377 steps).  As in the sigma = 1000 sheet, the charge mode is not damped and carries
    the rounding of every step: conditioning-derived bound."""
    check_case(W.sheet_box(100, sigma), 377, conditioned=True, symmetric=True)


def test_current_sheet_sigma10():
    """Resistive current sheet, 1024x4x4, x open, p = 50, sigma = 10, a 300-step prefix."""
    check_case(W.sheet(sigma=10.0), 300)


def test_current_sheet_sigma1000():
    """sigma = 1000: the stiff charge mode is undamped, conditioning-derived bound."""
    check_case(W.sheet(sigma=1000.0), 300, conditioned=True, symmetric=True)


def test_kh_prefix_20_steps():
    """Kelvin-Helmholtz shear layer (x periodic, y open, v0 = 0.4, ratio 10, sigma = 1e3), 96x160x1."""
    check_case(W.kh(nx=96, ny=160, v0=0.4, ratio=10.0, sigma=1e3), 20)


def test_kh_prefix_100_steps():
    check_case(W.kh(nx=96, ny=160, v0=0.4, ratio=10.0, sigma=1e3), 100, conditioned=True)


def test_degenerate_single_cell_and_line():
    for shape in ((1, 1, 1), (5, 1, 1), (1, 7, 1)):
        w = W.random_state(shape=shape, seed=4, vmax=0.05, Bmag=0.1, Emag=0.01, modes=1)
        check_case(w, 5)


def test_recovery_failure_is_reported():
    """A superluminal cell is invalid input: the step propagates NaN there and rmhdlb_moments reports it."""
    torch = _torch_cuda()
    w = W.random_state(shape=(8, 8, 4), seed=5, vmax=0.05)
    f = dict(w.fields)
    ux = f["u"][0].copy()
    ux[1, 2, 3] = 1.5
    f["u"] = (ux, f["u"][1], f["u"][2])
    from paper_1508_03452_amd.rmhdlb import RMHDLB_ERECOVERY, Solver
    s = Solver(w.shape, w.bc, **w.params)
    s.init_fields(f)
    m = s.moments()
    assert m["rc"] == RMHDLB_ERECOVERY and m["diag"]["n_failed"] >= 1
    assert torch.isnan(m["n"][1, 2, 3])


def test_checkpoint_restart_bitwise():
    _torch_cuda()
    w = W.random_state(shape=(16, 8, 4), seed=6, vmax=0.05, Bmag=0.2, Emag=0.02)
    a = run_gpu(w, 10)
    b = run_gpu(w, 5)
    st = b.get_state()
    from paper_1508_03452_amd.rmhdlb import Solver
    c = Solver(w.shape, w.bc, **w.params)
    c.set_state(st)
    c.step(5)
    import torch
    assert torch.equal(a.get_state(), c.get_state())


# --------------------------------------------- full sizes, sampled cells ---

def _sub_state(state, shape, cx, cy, cz, r=2):
    """Cut a (2r+1)^3 block (periodic wrap on every axis, clipped to one cell on
    axes of length 1) centred on (cx, cy, cz) out of a (66, nz, ny, nx) state."""
    nx, ny, nz = shape
    def idx(c, n):
        return np.array([0]) if n == 1 else (np.arange(c - r, c + r + 1) % n)
    ix, iy, iz = idx(cx, nx), idx(cy, ny), idx(cz, nz)
    return state[:, iz][:, :, iy][:, :, :, ix], (len(ix), len(iy), len(iz))


@pytest.mark.parametrize("name,prefix", [("kh", 3), ("flare", 3), ("kh", 199), ("flare", 199)])
def test_full_size_sampled_cells_one_step(name, prefix):
    """At the full benchmark sizes (KH slab 1024x2048x1, flare box 256x256x512)
    and the benchmark's launch configuration: take the GPU state after 3 or 199
    steps (the KH slab's 200-step prefix), cut the stencil neighbourhood of
    sampled interior cells, advance it one step with the oracle, and compare the
    sampled cells' new state with the GPU's own next step."""
    torch = _torch_cuda()
    w = W.kh() if name == "kh" else W.flare()
    s = run_gpu(w, 0)
    shape = s.autotune()   # the launch shape bench.py times (the state is not advanced)
    print(f"[parity] {name} full size, autotuned shape {shape}, after {prefix} steps", flush=True)
    s.step(prefix)
    st = s.get_state()
    s.step(1)
    st1 = s.get_state()
    # the same steps in the default shape (one block per column walk of 4
    # planes): the launch shape changes the order of work, not one bit
    d = run_gpu(w, prefix + 1)
    assert torch.equal(d.get_state(), st1)
    d.close()
    del d
    rng = np.random.default_rng(11)
    nx, ny, nz = w.shape
    worst = 0.0
    for _ in range(24):
        cx = int(rng.integers(3, nx - 3))
        cy = int(rng.integers(3, ny - 3))
        cz = int(rng.integers(3, nz - 3)) if nz > 6 else 0
        ix = np.arange(cx - 2, cx + 3)
        iy = np.arange(cy - 2, cy + 3)
        iz = np.arange(cz - 2, cz + 3) if nz > 1 else np.array([0])
        sub = st[:, torch.as_tensor(iz, device="cuda")][:, :, torch.as_tensor(iy, device="cuda")][
            :, :, :, torch.as_tensor(ix, device="cuda")].cpu().numpy()
        shp = (5, 5, len(iz))
        bc = (("periodic", "periodic"),) * 3
        o = oracle.Oracle(shp, bc, **w.params)
        o.set_state(np.ascontiguousarray(sub))
        o.step(1)
        got = st1[:, cz, cy, cx].cpu().numpy()
        ref = o.get_state()[:, len(iz) // 2, 2, 2]
        for sl in (slice(0, 19), slice(19, 38), slice(38, 63), slice(63, 66)):
            scale = max(np.abs(ref[sl]).max(), 1e-3 * field_scale(w))
            worst = max(worst, np.abs(got[sl] - ref[sl]).max() / scale)
    print(f"[parity] {name} full-size sampled-cell worst {worst:.2e} after {prefix} steps", flush=True)
    assert worst <= TOL


# One step of a reduced storage form from its own state, against the FP64 oracle's step from the same
# (widened) state, per state group relative to the group's largest value: the form's arithmetic and
# the rounding of the stored deviations in that one step: a few units of the storage's rounding
# (FP32 6e-8, FP16 4.9e-4 of the stored deviation).  Measured on the KH slab and the flare box: FP32
# 2.1e-7, FP16 5.6e-4.
ONE_STEP_TOL = {"f32": 1e-6, "f16": 2e-3}


@pytest.mark.parametrize("name,storage", [("kh", "f32"), ("kh", "f16"), ("flare", "f32"), ("flare", "f16")])
def test_full_size_sampled_cells_one_step_reduced_forms(name, storage):
    """The FP32 and FP16 forms at the full benchmark sizes in their tuned launch shapes (quad and
    double-quad layouts, one lane per cell): sampled interior cells after 3 steps, one step by the
    oracle from the form's own state against the form's next step."""
    torch = _torch_cuda()
    w = W.kh() if name == "kh" else W.flare()
    s = run_gpu(w, 0, storage=storage)
    shape = s.autotune()
    s.step(3)
    st = s.get_state()
    s.step(1)
    st1 = s.get_state()
    rng = np.random.default_rng(12)
    nx, ny, nz = w.shape
    worst = {g: 0.0 for g in ("F", "G", "h", "E")}
    for _ in range(24):
        cx = int(rng.integers(3, nx - 3))
        cy = int(rng.integers(3, ny - 3))
        cz = int(rng.integers(3, nz - 3)) if nz > 6 else 0
        ix = np.arange(cx - 2, cx + 3)
        iy = np.arange(cy - 2, cy + 3)
        iz = np.arange(cz - 2, cz + 3) if nz > 1 else np.array([0])
        sub = st[:, torch.as_tensor(iz, device="cuda")][:, :, torch.as_tensor(iy, device="cuda")][
            :, :, :, torch.as_tensor(ix, device="cuda")].cpu().numpy()
        o = oracle.Oracle((5, 5, len(iz)), (("periodic", "periodic"),) * 3, **w.params)
        o.set_state(np.ascontiguousarray(sub))
        o.step(1)
        got = st1[:, cz, cy, cx].cpu().numpy()
        ref = o.get_state()[:, len(iz) // 2, 2, 2]
        for g, sl in (("F", slice(0, 19)), ("G", slice(19, 38)), ("h", slice(38, 63)), ("E", slice(63, 66))):
            scale = max(np.abs(ref[sl]).max(), 1e-3 * field_scale(w))
            worst[g] = max(worst[g], float(np.abs(got[sl] - ref[sl]).max() / scale))
    print(f"[parity] {name} {storage} full size, shape {shape}, one step from its own state: " +
          " ".join(f"{g} {v:.1e}" for g, v in worst.items()), flush=True)
    assert max(worst.values()) <= ONE_STEP_TOL[storage], worst


@pytest.mark.parametrize("divb_fix", [0, 1])
def test_full_size_sampled_face_cells_one_step(divb_fix):
    """The flare box at full size: cells on the open x-low, y-high and z-high faces (with and
    without the normal-B adjustment) and on the driven bottom face, each advanced one step by the
    oracle on a 5x5x5 window that keeps the face (and, for the bottom, the prescribed face fields)."""
    torch = _torch_cuda()
    w = W.flare()
    w.params["divb_fix"] = divb_fix
    s = run_gpu(w, 0)
    print(f"[parity] flare faces divb_fix={divb_fix}, autotuned shape {s.autotune()}", flush=True)
    s.step(3)
    st = s.get_state()
    s.step(1)
    st1 = s.get_state()
    rng = np.random.default_rng(12)
    nx, ny, nz = w.shape
    worst = 0.0
    for face in ("x_lo", "y_hi", "z_hi", "z_lo"):
        for _ in range(6):
            c = [int(rng.integers(3, nx - 3)), int(rng.integers(3, ny - 3)), int(rng.integers(3, nz - 3))]
            ax, hi = {"x_lo": (0, 0), "y_hi": (1, 1), "z_hi": (2, 1), "z_lo": (2, 0)}[face]
            n_ax = w.shape[ax]
            c[ax] = n_ax - 1 if hi else 0
            win = []
            for a in range(3):
                if a == ax:
                    win.append(np.arange(n_ax - 5, n_ax) if hi else np.arange(0, 5))
                else:
                    win.append(np.arange(c[a] - 2, c[a] + 3))
            ix, iy, iz = win
            sub = st[:, torch.as_tensor(iz, device="cuda")][:, :, torch.as_tensor(iy, device="cuda")][
                :, :, :, torch.as_tensor(ix, device="cuda")].cpu().numpy()
            bc = [["periodic", "periodic"] for _ in range(3)]
            bc[ax] = ["driven", "open"] if face == "z_lo" else ["open", "open"]
            o = oracle.Oracle((5, 5, 5), tuple(tuple(b) for b in bc), **w.params)
            o.set_state(np.ascontiguousarray(sub))
            if face == "z_lo":
                d = w.driven
                cut = lambda a: np.ascontiguousarray(a[np.ix_(iy, ix)])
                o.set_driven(dict(n=cut(d["n"]), p=cut(d["p"]), u=tuple(cut(v) for v in d["u"]),
                                  B=tuple(cut(v) for v in d["B"])))
            o.step(1)
            li = [int(np.where(win[a] == c[a])[0][0]) for a in range(3)]
            got = st1[:, c[2], c[1], c[0]].cpu().numpy()
            ref = o.get_state()[:, li[2], li[1], li[0]]
            for sl in (slice(0, 19), slice(19, 38), slice(38, 63), slice(63, 66)):
                scale = max(np.abs(ref[sl]).max(), 1e-3 * field_scale(w))
                worst = max(worst, np.abs(got[sl] - ref[sl]).max() / scale)
    print(f"[parity] flare full-size sampled face cells worst {worst:.2e}", flush=True)
    assert worst <= TOL


# ------------------------------------------------ mixed storage forms (a10) ---

# Stated per-field bounds against the FP64 oracle (max error over the field's
# max, same floors as above): FP32 storage + FP32 arithmetic, and FP16-shifted
# storage + FP32 arithmetic, with the recovery and Ohm solve in FP64.  The
# current J = sigma * (E + v x B - ...) and the charge eps0 div E are derived
# fields: J amplifies the storage rounding of E, v and B by sigma (a difference
# of nearly cancelling terms in the ideal limit) and rho_c by 1/dx, so they
# carry a bound ten times looser than the primary fields n, p, eps, u, E, B.
MIXED_TOL = {"f32": 5e-5, "f16": 5e-3}
DERIVED = ("Jx", "Jy", "Jz", "rho_c")


def _mixed_tol(storage, field):
    return MIXED_TOL[storage] * (10.0 if field in DERIVED else 1.0)


def _mixed_case(w, steps, storage):
    _torch_cuda()
    o = run_oracle(w, steps)
    s = run_gpu(w, steps, storage=storage)
    mo = o.moments()
    mg = gpu_moments_np(s)
    assert mg["diag"]["n_failed"] == 0
    errs = field_errors(mo, mg, field_scale(w))
    print(f"[mixed] {storage} {w.name} {w.shape} steps={steps}: " +
          " ".join(f"{k}={v:.1e}" for k, v in errs.items()), flush=True)
    bad = {k: v for k, v in errs.items() if v > _mixed_tol(storage, k)}
    assert not bad, bad
    do, dg = o.diagnostics(), mg["diag"]
    # global sums stay close: FP32 arithmetic per cell, FP64 sums
    assert abs(dg["energy"] - do["energy"]) <= MIXED_TOL[storage] * abs(do["energy"])
    assert abs(dg["mass"] - do["mass"]) <= MIXED_TOL[storage] * abs(do["mass"])
    return errs


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_mixed_random_3d(storage):
    w = W.random_state(shape=(70, 6, 3), seed=2, vmax=0.1, Bmag=0.2, Emag=0.02, sigma=3.0)
    _mixed_case(w, 12, storage)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_mixed_current_sheet(storage):
    _mixed_case(W.sheet(sigma=10.0), 300, storage)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_mixed_kh_prefix(storage):
    _mixed_case(W.kh(nx=96, ny=160, v0=0.4, ratio=10.0, sigma=1e3), 20, storage)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_mixed_driven_face(storage):
    """Ghost planes of the driven face are stored as shifted deviations like the interior."""
    _mixed_case(_driven_case(), 15, storage)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_mixed_alternative_readings(storage):
    """The printed collision with the Lax-Wendroff faces in the reduced storage forms."""
    w = W.random_state(shape=(70, 6, 3), seed=2, vmax=0.1, Bmag=0.2, Emag=0.02, sigma=3.0)
    w.params.update(collision=1, flux=1)
    _mixed_case(w, 12, storage)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_mixed_external_force(storage):
    """The external force in the reduced storage forms (the source enters the stored deviations)."""
    w = W.random_state(shape=(70, 6, 3), seed=2, vmax=0.1, Bmag=0.2, Emag=0.02, sigma=3.0)
    w.force = (_random_force(w, 5, 0.02), 0.0)
    _mixed_case(w, 12, storage)


@pytest.mark.parametrize("storage", ["f32", "f16"])
def test_mixed_conserves_mass_exactly_in_fp64_sums(storage):
    """The collisions conserve N^0 exactly; with FP32 arithmetic per cell the
    total mass on a periodic box drifts only by rounding."""
    torch = _torch_cuda()
    w = W.random_state(shape=(16, 12, 8), seed=7, vmax=0.05, Bmag=0.1, Emag=0.01)
    s = run_gpu(w, 0, storage=storage)
    d0 = s.moments(fields=())["diag"]
    s.step(50)
    d1 = s.moments(fields=())["diag"]
    drift = abs(d1["mass"] - d0["mass"]) / d0["mass"]
    print(f"[mixed] {storage} mass drift over 50 steps {drift:.1e}", flush=True)
    assert drift <= (1e-6 if storage == "f32" else 1e-3)


def test_device_copy_copies_and_checks_its_arguments():
    """rmhdlb_device_copy, the plain copy kernel the benchmark reads the HBM rate from: exact copies of a
    ragged length (not a multiple of the 1024 words a block moves), and RMHDLB_EINVAL for a length or an
    address that is not 16-byte aligned and for overlapping ranges, with nothing written."""
    torch = _torch_cuda()
    from paper_1508_03452_amd.rmhdlb import RMHDLB_EINVAL, device_copy, load
    import ctypes
    a = torch.arange(3 * 1024 * 16 + 6, dtype=torch.float64, device="cuda")       # 49158 doubles, 16 B multiple
    b = torch.zeros_like(a)
    device_copy(b, a)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    L = load()
    c = torch.zeros_like(a)
    p = lambda t, off=0: ctypes.c_void_p(t.data_ptr() + off)
    assert L.rmhdlb_device_copy(p(c), p(a), 8, None) == RMHDLB_EINVAL           # not a multiple of 16
    assert L.rmhdlb_device_copy(p(c, 8), p(a), 16, None) == RMHDLB_EINVAL       # misaligned destination
    assert L.rmhdlb_device_copy(p(a, 16), p(a), 64, None) == RMHDLB_EINVAL      # overlapping
    torch.cuda.synchronize()
    assert not c.any()

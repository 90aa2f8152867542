"""Launch shapes, the autotuner and batched sweeps on the GPU, through the C ABI.

Every cell's arithmetic is independent of the block shape and of the other instances of a batch,
so a different tile shape, a batched launch or a replayed hipGraph must give the same state bit
for bit; the plain path itself is pinned to the oracle in test_gpu_parity.py."""
import numpy as np
import pytest

from paper_1508_03452_amd import workloads as W

from .parity_util import run_gpu

pytestmark = pytest.mark.gpu


def _torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _state(s):
    return s.get_state().cpu().numpy()


# zg > 1: interleaved walks, with chunks of zg * zb planes that do not divide
# nz = 9 (the last chunk is ragged and some walks are empty); yw > 1: row
# groups stacked along y, with ny = 13 leaving the last tile's groups partly
# or wholly outside the grid
@pytest.mark.parametrize("px,zb,zg,yw", [(32, 1, 1, 1), (16, 2, 1, 1), (64, 8, 1, 1), (64, 2, 2, 1), (64, 2, 4, 1),
                                         (32, 1, 4, 1), (64, 16, 2, 1), (64, 1, 1, 2), (32, 2, 1, 2),
                                         (16, 1, 1, 4), (64, 4, 2, 4)])
def test_tile_shapes_give_identical_states(px, zb, zg, yw):
    _torch_cuda()
    w = W.random_state(shape=(70, 13, 9), seed=6, vmax=0.1, Bmag=0.2, Emag=0.02, sigma=3.0,
                       bc=(("open", "open"), ("periodic", "periodic"), ("open", "open")))
    a = run_gpu(w, 0)
    b = run_gpu(w, 0)
    b.set_tuning(px, zb, zg, yw)
    a.step(6)
    b.step(6)
    assert np.array_equal(_state(a), _state(b))


def test_autotune_picks_a_valid_shape_and_keeps_the_state():
    _torch_cuda()
    w = W.kh(nx=192, ny=256, v0=0.3, ratio=5.0, sigma=1e3)
    s = run_gpu(w, 2)
    before = _state(s)
    px, zb, zg, yw = s.autotune()
    print(f"[batch] autotune kh 192x256x1 -> px {px} zb {zb} zg {zg} yw {yw}", flush=True)
    assert px in (64, 32, 16) and zb >= 1 and zg == 1 and yw in (1, 2, 4)   # nz = 1: no interleaved walks
    assert np.array_equal(before, _state(s))   # timing does not advance the state
    assert s.autotune() == (px, zb, zg, yw)    # cached
    ref = run_gpu(w, 2)
    s.step(3)
    ref.step(3)
    assert np.array_equal(_state(s), _state(ref))


def test_autotune_3d_with_interleaved_candidates():
    """On a box deep enough for the interleaved walks the tuner times them
    too; whatever it picks leaves the state alone and steps as the default."""
    _torch_cuda()
    w = W.random_state(shape=(64, 8, 64), seed=8, vmax=0.1, Bmag=0.2, Emag=0.02, sigma=3.0,
                       bc=(("periodic", "periodic"), ("open", "open"), ("open", "open")))
    s = run_gpu(w, 0)
    before = _state(s)
    px, zb, zg, yw = s.autotune()
    print(f"[batch] autotune random 64x8x64 -> px {px} zb {zb} zg {zg} yw {yw}", flush=True)
    assert px in (64, 32, 16) and zb >= 1 and zg in (1, 2, 4) and (zg == 1 or px == 64) and yw == 1
    assert np.array_equal(before, _state(s))
    ref = run_gpu(w, 0)
    s.step(4)
    ref.step(4)
    assert np.array_equal(_state(s), _state(ref))


def test_interleaved_walks_not_with_force():
    """With an external force the step keeps one walk per column (zg = 1)."""
    _torch_cuda()
    from paper_1508_03452_amd.rmhdlb import RmhdlbError
    w = W.random_state(shape=(20, 9, 16), seed=4, vmax=0.05, Bmag=0.2, Emag=0.02, sigma=30.0)
    s = run_gpu(w, 0)
    nx, ny, nz = w.shape
    s.set_force([np.full((nz, ny, nx), 0.01) for _ in range(3)], 0.0)
    with pytest.raises(RmhdlbError):
        s.set_tuning(64, 2, 2)
    assert s.autotune()[2] == 1


def _sweep_workloads(n=5, seed=3):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        nx, ny = int(rng.choice([48, 64, 96, 130])), int(rng.choice([40, 64, 100]))
        out.append(W.kh(nx=nx, ny=ny, v0=float(rng.uniform(0.05, 0.4)), ratio=float(rng.uniform(1, 10)),
                        sigma=float(10 ** rng.uniform(2, 4)), seed=i))
    out.append(W.random_state(shape=(20, 9, 7), seed=9, vmax=0.05, Bmag=0.1, sigma=30.0, solenoidal=True,
                              bc=(("open", "open"),) * 3))
    return out


def _batch(ws, storage, stream):
    from paper_1508_03452_amd.rmhdlb import Batch
    b = Batch([(w.shape, w.bc, w.params) for w in ws], storage=storage, stream=stream)
    for w, s in zip(ws, b.instances):
        s.init_fields(w.fields)
    return b


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_batch_matches_instances_stepped_alone(storage):
    """Uneven 2-D KH slabs (ragged tiles) plus a 3-D box with open faces: 7 batched steps (graph
    replays and an eager remainder) equal 7 steps of each instance alone, bit for bit."""
    torch = _torch_cuda()
    ws = _sweep_workloads()
    st = torch.cuda.Stream()
    b = _batch(ws, storage, st)
    b.step(7)
    st.synchronize()
    for w, s in zip(ws, b.instances):
        ref = run_gpu(w, 7, storage=storage)
        assert np.array_equal(_state(s), _state(ref)), w.shape
        assert s.moments(fields=())["diag"]["step"] == 7
    b.close()


def test_batch_graph_replays_match_eager_steps():
    """The captured two-step graph replayed three times, with eager work and synchronisation between
    the replays, against the same batch stepped eagerly on the default stream (no capture)."""
    torch = _torch_cuda()
    ws = _sweep_workloads(n=3, seed=4)
    st = torch.cuda.Stream()
    g = _batch(ws, "f32", st)
    e = _batch(ws, "f32", torch.cuda.default_stream())
    for r in range(3):
        g.step(2)
        e.step(2)
        scratch = torch.ones(1 << 20, device="cuda", dtype=torch.float32).sum()   # unrelated eager work
        torch.cuda.synchronize()
        assert float(scratch) == float(1 << 20)
        for sg, se in zip(g.instances, e.instances):
            assert np.array_equal(_state(sg), _state(se)), r
    g.close()
    e.close()


def test_batch_rejects_mixed_parity_and_autotunes():
    torch = _torch_cuda()
    from paper_1508_03452_amd.rmhdlb import RmhdlbError
    ws = _sweep_workloads(n=3, seed=5)
    st = torch.cuda.Stream()
    b = _batch(ws, "f32", st)
    before = [_state(s) for s in b.instances]
    px, yw, waves = b.autotune()
    print(f"[batch] batch autotune -> px {px} yw {yw} waves {waves}", flush=True)
    assert (px, yw) in BATCH_TILES and waves in (2, 3)
    for s, x in zip(b.instances, before):
        assert np.array_equal(_state(s), x)   # timing does not advance the state
    assert b.autotune() == (px, yw, waves)    # cached
    b.instances[0].step(1)                    # one instance stepped alone: parities differ
    from paper_1508_03452_amd.rmhdlb import RMHDLB_ESTATE
    with pytest.raises(RmhdlbError) as e:
        b.step(1)
    assert e.value.code == RMHDLB_ESTATE
    b.close()


# the batch tuner's tiles (px, yw) of both layouts: px x (R / px) yw cells, R = 128 (FP64), 256 (FP32, FP16)
BATCH_TILES = ((64, 1), (32, 1), (16, 1), (128, 1), (64, 2), (32, 2), (128, 2), (16, 2), (64, 4))


@pytest.mark.parametrize("px,yw", BATCH_TILES)
@pytest.mark.parametrize("waves", [2, 3])
def test_batch_tiles_and_occupancies_match_instances(px, yw, waves):
    """Every tile shape and occupancy variant of the batched FP32 step gives each instance exactly the
    state of stepping it alone (uneven slabs with ragged tiles in x and y, and a 3-D open box)."""
    torch = _torch_cuda()
    ws = _sweep_workloads(n=4, seed=6)
    st = torch.cuda.Stream()
    b = _batch(ws, "f32", st)
    b.set_tuning(px, yw, waves)
    b.step(5)
    st.synchronize()
    for w, s in zip(ws, b.instances):
        ref = run_gpu(w, 5, storage="f32")
        assert np.array_equal(_state(s), _state(ref)), (w.shape, px, yw, waves)
    b.close()


def test_batch_long_graph_replays_match_instances():
    """131 batched steps from parity 0: two replays of the captured 64-step graph, one of the two-step
    graph and one eager step, against each instance stepped alone (eager launches)."""
    torch = _torch_cuda()
    ws = _sweep_workloads(n=3, seed=7)
    st = torch.cuda.Stream()
    b = _batch(ws, "f32", st)
    b.step(131)
    st.synchronize()
    for w, s in zip(ws, b.instances):
        ref = run_gpu(w, 131, storage="f32")
        assert np.array_equal(_state(s), _state(ref)), w.shape
        assert s.moments(fields=())["diag"]["step"] == 131
    b.close()


def test_batch_recaptures_when_an_instance_is_retuned():
    """The captured graphs hold the launch grid.  Retuning an instance of the batch (its z-walk, which
    changes its block count) must make the batch capture again: the steps after the retune still equal
    each instance stepped alone (a stale graph would skip the added blocks)."""
    torch = _torch_cuda()
    ws = _sweep_workloads(n=2, seed=8)            # two slabs and the 3-D box (nz = 7) last
    st = torch.cuda.Stream()
    b = _batch(ws, "f32", st)
    b.step(4)                                     # captures the two-step graph with zb = 4
    b.instances[-1].set_tuning(64, 1)             # zb = 1: seven blocks per column instead of two
    b.step(4)
    b.instances[-1].set_tuning(64, 8)
    b.step(70)                                    # and the long graph with yet another grid
    st.synchronize()
    for w, s in zip(ws, b.instances):
        ref = run_gpu(w, 78, storage="f32")
        assert np.array_equal(_state(s), _state(ref)), w.shape
    b.close()


def test_batched_sweep_instances_against_the_oracle():
    """The batched sweep's instances against the oracle: six KH slabs drawn by the sweep generator (seed
    64, uneven sizes that leave ragged tiles in x and y; sigma 1e2 .. 1e5, shear 0.05 .. 0.4c, density
    ratio 1 .. 10), stepped 20 times as one FP64 batch in the tuner's chosen tile; every instance's
    fields and raw state within 1e-12 of the oracle's run of that instance."""
    torch = _torch_cuda()
    from .parity_util import field_errors, field_scale, gpu_moments_np, run_oracle, state_errors
    specs = W.sweep_specs(n=6, seed=64, sizes=(72, 96, 130, 160, 200))
    ws = [W.sweep_instance(sp) for sp in specs]
    st = torch.cuda.Stream()
    b = _batch(ws, "f64", st)
    print(f"[batch] sweep of {len(ws)} KH slabs {[w.shape[:2] for w in ws]}, tile {b.autotune()}", flush=True)
    b.step(20)
    st.synchronize()
    for w, s in zip(ws, b.instances):
        o = run_oracle(w, 20)
        mg = gpu_moments_np(s)
        assert mg["diag"]["n_failed"] == 0
        errs = field_errors(o.moments(), mg, field_scale(w))
        serr = state_errors(o.get_state(), _state(s), field_scale(w))
        worst = max(errs, key=errs.get)
        print(f"[batch] {w.shape[:2]} sigma {w.params['sigma']:.3g}: worst field {worst}={errs[worst]:.1e}, "
              f"state {max(serr.values()):.1e}", flush=True)
        assert errs[worst] <= 1e-12 and max(serr.values()) <= 1e-12, (w.shape, errs[worst], serr)
    b.close()


def _sync():
    """The graph-replay batch finishes before the persistent one starts: a cooperative launch needs all
    of its blocks resident together, so the two are not left to overlap on the device."""
    import torch
    torch.cuda.synchronize()


def _pair_batches(ws, storage, waves=2):
    """The same instances as two batches on their own streams: graph replays, and persistent mode."""
    torch = _torch_cuda()
    g = _batch(ws, storage, torch.cuda.Stream())
    p = _batch(ws, storage, torch.cuda.Stream())
    for b in (g, p):
        b.set_tuning(64, 1, waves)
    p.set_persistent(True)
    return g, p


def _assert_batches_equal(g, p, steps):
    import torch
    torch.cuda.synchronize()
    for sg, sp in zip(g.instances, p.instances):
        assert np.array_equal(_state(sg), _state(sp), equal_nan=True)
        assert sp.moments(fields=())["diag"]["step"] == steps


@pytest.mark.parametrize("storage,waves", [("f64", 2), ("f32", 2), ("f32", 3), ("f16", 2)])
def test_persistent_batch_matches_graph_replays(storage, waves):
    """Persistent mode (one cooperative launch per call, grid barriers between the steps) against graph
    replays, bit for bit: six KH slabs of 384-512 x 256-320 cells, about 3,800 tiles, more than the
    blocks resident at once, so that every block takes several tiles per step; calls of 1, 6 and 5
    steps start from both buffer parities."""
    rng = np.random.default_rng(11)
    ws = [W.kh(nx=int(rng.choice([384, 448, 512])), ny=int(rng.choice([256, 320])), v0=float(rng.uniform(0.05, 0.4)),
               ratio=float(rng.uniform(1, 10)), sigma=float(10 ** rng.uniform(2, 4)), seed=20 + i) for i in range(6)]
    print(f"[batch] persistent {storage} waves {waves}: {sum(w.ncells for w in ws)} cells", flush=True)
    g, p = _pair_batches(ws, storage, waves)
    done = 0
    for k in (1, 6, 5):
        g.step(k)
        _sync()
        p.step(k)
        done += k
        _assert_batches_equal(g, p, done)
    g.close()
    p.close()


@pytest.mark.skip(reason="a GPU memory fault (aperture violation) was reported during this test with a per-wavefront "
                         "variant of the persistent kernel; its cause was not found, so the variant was removed and the "
                         "persistent kernel's face pass switched off (persistent mode refuses such batches)")
def test_persistent_batch_with_the_open_face_adjustment():
    """An instance with the open-face div B adjustment makes the persistent kernel run the face pass
    (its own phase and grid barrier) before each step: uneven slabs, the 3-D open box and a KH slab with
    the adjustment on, 7 steps in calls of 3 and 4, against graph replays bit for bit."""
    ws = _sweep_workloads(n=3, seed=12)
    kh = W.kh(nx=96, ny=64, v0=0.2, ratio=4.0, sigma=1e3, seed=5)
    kh.params = dict(kh.params, divb_fix=1)
    ws.append(kh)
    g, p = _pair_batches(ws, "f32")
    for k in (3, 4):
        g.step(k)
        _sync()
        p.step(k)
    _assert_batches_equal(g, p, 7)
    g.close()
    p.close()


def test_persistent_mode_refuses_the_face_pass():
    """A batch with an instance that adjusts its open faces has no face pass in persistent mode: the step is
    refused before any launch (RMHDLB_EUNSUPPORTED), the state is left alone, and graph replays step it."""
    torch = _torch_cuda()
    from paper_1508_03452_amd.rmhdlb import RmhdlbError
    kh = W.kh(nx=96, ny=64, v0=0.2, ratio=4.0, sigma=1e3, seed=5)
    kh.params = dict(kh.params, divb_fix=1)
    b = _batch([kh], "f32", torch.cuda.Stream())
    before = _state(b.instances[0])
    b.set_persistent(True)
    with pytest.raises(RmhdlbError):
        b.step(2)
    assert np.array_equal(before, _state(b.instances[0]))
    b.set_persistent(False)
    b.step(2)
    torch.cuda.synchronize()
    assert b.instances[0].moments(fields=())["diag"]["step"] == 2
    b.close()

"""Host logic of bench.py: the JSON contract pieces that need no GPU."""
import json
import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]
sys.path.insert(0, str(ROOT))

import bench  # noqa: E402


def test_multi_gpu_request_exits_with_a_message():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_algorithmic_bytes_per_cell():
    # read + write of 63 distributions and 3 E_prev values per cell
    assert bench.alg_bytes_per_step("f64", 1) == 2 * 66 * 8
    assert bench.alg_bytes_per_step("f32", 1) == 2 * 66 * 4
    assert bench.alg_bytes_per_step("f16", 1) == 2 * (63 * 2 + 3 * 4)


def test_traffic_lookup_is_keyed_by_kernel_hash_and_shape():
    keys = list(bench.MEASURED_TRAFFIC)
    assert keys and len({k[2] for k in keys}) == 1      # one kernel version per table
    wl, form, h, shape = keys[0]
    if h == bench.kernel_hash():
        assert bench.measured_traffic(wl, form, [int(v) for v in shape.split(",")]) == bench.MEASURED_TRAFFIC[keys[0]]
    assert bench.measured_traffic(wl, form, [16, 1, 1]) is None   # a shape never counted
    assert bench.measured_traffic("nowhere", form, [64, 16, 4]) is None


def test_tile_text():
    assert bench.tile_text((64, 16, 1)) == "64x2 cells, 16 z-planes per block"
    assert "4 blocks per column" in bench.tile_text((64, 32, 4))


def test_rate_fits_recover_their_laws():
    """The KH study's fits: a pure power law is recovered with its exponent and no residual, a pure
    1 / ln sigma law has no residual in its own fit and a visible one in the power law, and signs are
    ignored (the rate at the null is negative in these runs)."""
    import numpy as np
    sig = [20.0, 40.0, 60.0, 80.0, 100.0]
    f = bench.fit_rates(sig, [-0.3 * s ** -0.5 for s in sig])
    assert abs(f["power_law"]["k"] + 0.5) < 1e-4 and f["power_law"]["max_rel_residual"] < 1e-4
    assert abs(f["power_law"]["a"] - 0.3) < 1e-9
    g = bench.fit_rates(sig, [0.1 / np.log(s) for s in sig])
    assert abs(g["inv_log"]["b"] - 0.1) < 1e-12 and g["inv_log"]["max_rel_residual"] < 1e-12
    assert g["power_law"]["max_rel_residual"] > 1e-3
    assert bench.fit_rates(sig[:2], [0.1, 0.2]) is None


def test_window_mean():
    series = [(1.0, 5.0), (2.0, 1.0), (5.0, 2.0), (8.0, 3.0), (9.0, 7.0)]
    assert bench.window_mean(series) == 2.0
    assert bench.window_mean([(1.0, 1.0)]) is None


def test_halo_of_a_slab_face():
    """The exchange a z-slab of the flare box would need per face and step: 59 values per face cell, 31 MB
    for a 256 x 256 face in FP64, about 0.2 ms over one 153 GB/s xGMI link."""
    n = bench.halo_values_per_face_cell()
    assert n == 59
    face = n * 256 * 256 * 8
    assert abs(face / 1e6 - 30.93) < 0.01
    assert abs(face / 153e9 * 1e3 - 0.202) < 0.001

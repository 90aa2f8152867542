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

"""Writes flare64_oracle.npz: the FP64 oracle after 1000 steps of the 64^3 instance of the flare box
(workloads.flare(64, 64, 64, Lz=12): arcade plus flux rope, stratified density, driven shearing bottom
face, open faces elsewhere, sigma = 1e3).

Stored: the primitive fields n, p, eps, u, E, B on six z-planes (0, 1, 3, 8, 24, 63) at every second cell
in x and y; each field's largest magnitude over the whole box; the global diagnostics; and the oracle's
own sensitivity per field and for the total energy and mass, which bounds how closely any other implementation can agree after these
steps: the largest difference, over the whole box, to the reference run of two other runs, one started
from a density one ulp larger and one of the oracle built with contracted (fused) multiply-adds, the
rounding a GPU compiler's contraction gives at every step.

Only oracle/ and the seeded generator are called (three oracle runs, one per process, about 10 minutes
each on one core).  Run from the repository root: python tests/golden/make_flare64.py
"""
import multiprocessing as mp
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

STEPS = 1000
PLANES = (0, 1, 3, 8, 24, 63)
FIELDS = ("n", "p", "eps", "ux", "uy", "uz", "Ex", "Ey", "Ez", "Bx", "By", "Bz")
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "flare64_oracle.npz")


def workload():
    from paper_1508_03452_amd import workloads as W
    return W.flare(nx=64, ny=64, nz=64, Lz=12.0)


def run(mode):
    """mode 0: the reference; 1: initial density one ulp larger; 2: the oracle built with fused
    multiply-adds (set before the oracle library is loaded in this worker process)."""
    if mode == 2:
        os.environ["RMHDLB_ORACLE_FMA"] = "1"
    import oracle
    w = workload()
    fields = dict(w.fields)
    if mode == 1:
        fields["n"] = np.nextafter(np.asarray(w.fields["n"]), np.inf)
    o = oracle.Oracle(w.shape, w.bc, **w.params)
    o.init(fields)
    o.set_driven(w.driven)
    for done in range(100, STEPS + 1, 100):
        o.step(100)
        print(f"run {mode}: {done} steps", flush=True)
    m = o.moments()
    return {k: m[k] for k in FIELDS}, o.diagnostics(), m["n_failed"]


def main():
    with mp.get_context("spawn").Pool(3) as pool:     # fresh workers: each loads its own oracle build
        results = pool.map(run, [0, 1, 2])
    (ref, diag, failed) = results[0]
    assert all(r[2] == 0 for r in results)
    scale = max(max(np.abs(b).max() for b in workload().fields["B"]), 1e-3)
    eps_ref = float(np.abs(ref["eps"]).max())
    sens = {}
    for k in FIELDS:
        floor = 1.0 if k[0] == "u" else (scale if k[0] in "EB" else (eps_ref if k in ("p", "eps") else 1e-300))
        den = max(np.abs(ref[k]).max(), floor)
        sens[k] = max(float(np.abs(per[k] - ref[k]).max() / den) for per, _, _ in results[1:])
    out = {"steps": np.int64(STEPS), "planes": np.array(PLANES), "field_scale": np.float64(scale)}
    for k in FIELDS:
        out[k] = np.ascontiguousarray(ref[k][list(PLANES), ::2, ::2])
        out["max_" + k] = np.float64(np.abs(ref[k]).max())
        out["sens_" + k] = np.float64(sens[k])
    for k in ("energy", "mass", "em_energy", "charge", "max_divB"):
        out["diag_" + k] = np.float64(diag[k])
    for k in ("energy", "mass"):   # the same sensitivity for the global sums
        out["sens_diag_" + k] = np.float64(max(abs(d[k] - diag[k]) / abs(diag[k]) for _, d, _ in results[1:]))
    out["diag_momentum"] = np.asarray(diag["momentum"], dtype=np.float64)
    np.savez_compressed(OUT, **out)
    print("sensitivity: " + " ".join(f"{k}={v:.1e}" for k, v in sens.items()) +
          f" energy={float(out['sens_diag_energy']):.1e} mass={float(out['sens_diag_mass']):.1e}")
    print(f"wrote {OUT} ({os.path.getsize(OUT)} bytes)")


if __name__ == "__main__":
    main()

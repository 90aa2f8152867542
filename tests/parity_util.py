"""Helpers for comparing the HIP library with the oracle (test infrastructure)."""
import numpy as np

import oracle

VEC = ("u", "E", "B", "J")


def field_errors(ref, got, scale_B, eps_ref=None):
    """Per-field error: max |got - ref| / max(max |ref|, floor).  Floors: c for
    velocities, the field scale for E, B, J (their natural size in the run),
    the energy scale eps_ref (default: max |eps| of ref) for p and eps."""
    errs = {}
    if eps_ref is None and "eps" in ref:
        eps_ref = float(np.abs(ref["eps"]).max())
    for k, r in ref.items():
        if k not in got or k in ("n_failed", "diag") or not hasattr(r, "shape"):
            continue
        g = got[k]
        if k[0] == "u" and len(k) == 2:
            floor = 1.0
        elif (k[0] in "EBJ" and len(k) == 2) or k == "rho_c":
            floor = scale_B             # rho_c ~ eps0 div E ~ eps0 c |B| / dx
        elif k in ("p", "eps") and eps_ref is not None:
            floor = eps_ref
        else:
            floor = 1e-300
        den = max(np.abs(r).max(), floor)
        errs[k] = float(np.abs(g - r).max() / den)
    return errs


def state_errors(ref, got, scale_B=None):
    """Per-group error of the raw state (F, G, h*, E_prev and, with the previous-B reading, B_prev),
    relative to each group's max; the field groups E_prev and B_prev with the floor scale_B of the
    field errors (their natural size in the run), when given."""
    groups = dict(F=slice(0, 19), G=slice(19, 38), h=slice(38, 63), E=slice(63, 66))
    if ref.shape[0] == 69:
        groups["Bp"] = slice(66, 69)
    out = {}
    for k, s in groups.items():
        r, g = ref[s], got[s]
        floor = scale_B if (k in ("E", "Bp") and scale_B is not None) else 1e-300
        out[k] = float(np.abs(g - r).max() / max(np.abs(r).max(), floor))
    return out


def run_oracle(w, steps):
    o = oracle.Oracle(w.shape, w.bc, **w.params)
    o.init(w.fields)
    if w.driven is not None:
        o.set_driven(w.driven)
    if w.force is not None:
        o.set_force(*w.force)
    if steps:
        o.step(steps)
    return o


def run_gpu(w, steps, storage="f64"):
    from paper_1508_03452_amd.rmhdlb import Solver
    s = Solver(w.shape, w.bc, storage=storage, **w.params)
    s.init_fields(w.fields)
    if w.driven is not None:
        s.set_driven_face(w.driven)
    if w.force is not None:
        s.set_force(*w.force)
    if steps:
        s.step(steps)
    return s


def gpu_moments_np(s):
    m = s.moments()
    out = {k: v.cpu().numpy() for k, v in m.items() if hasattr(v, "cpu")}
    out["diag"] = m["diag"]
    return out


def field_scale(w):
    return max(max(np.abs(b).max() for b in w.fields["B"]), 1e-3)

"""rmhdlb_guess_samples_noalloc (the entry point that allocates no device memory) against
rmhdlb_guess_samples, both called through the C ABI: the same kernels with the partial sums in the
library's fixed per-device array instead of a fresh allocation, so the outputs must agree bit for bit,
also on a second call with fewer samples (the array keeps the first call's larger contents)."""
import ctypes

import numpy as np
import pytest

from paper_1508_03452_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_noalloc_sampling_matches_the_allocating_call():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1508_03452_amd.rmhdlb import (NOALLOC_MAX_SAMPLES, RMHDLB_ELIMIT, RMHDLB_OK, Solver, _dptr,
                                             load)
    L = load()
    w = W.kh(nx=200, ny=300, v0=0.3, ratio=5.0, sigma=1e3)
    s = Solver(w.shape, w.bc, **w.params)
    s.init_fields(w.fields)
    s.step(3)
    for ns in (60000, 50000, 777):           # repeated calls, each later one smaller
        print(f"[noalloc] kh 200x300, {ns} samples", flush=True)
        out = []
        for fn in (L.rmhdlb_guess_samples, L.rmhdlb_guess_samples_noalloc):
            F = torch.full((ns, 6), float("nan"), dtype=torch.float64, device="cuda")
            T = torch.full((ns, 2), float("nan"), dtype=torch.float64, device="cuda")
            rc = fn(s._h, ns, _dptr(F), _dptr(T))
            assert rc == RMHDLB_OK, (fn.__name__, rc)
            out.append((F, T))
        (F0, T0), (F1, T1) = out
        assert torch.isfinite(F1).all() and torch.isfinite(T1).all()
        assert torch.equal(F0, F1) and torch.equal(T0, T1), ns
    # beyond the fixed array: a clear error, nothing written
    F = torch.zeros((8, 6), dtype=torch.float64, device="cuda")
    T = torch.zeros((8, 2), dtype=torch.float64, device="cuda")
    assert L.rmhdlb_guess_samples_noalloc(s._h, NOALLOC_MAX_SAMPLES + 1, _dptr(F), _dptr(T)) == RMHDLB_ELIMIT
    assert not F.any() and not T.any()
    s.close()

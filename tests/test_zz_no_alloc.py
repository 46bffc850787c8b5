"""fwi_lbfgs_apply_noalloc (the two-loop recursion with the library's static
scratch, for callers that cannot allocate) against fwi_lbfgs_apply through
the C-ABI: bit-identical results on two calls in a row, the second on a
smaller problem (fewer elements, fewer stored pairs, FP64 after FP32 on the
same device array), and a history larger than the static scratch rejected
before any launch."""

import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _history(n, m, npair, dt, seed):
    from paper_2102_00755_amd.slbfgs import LbfgsHistory, VecOps
    dev = torch.device("cuda", 0)
    ops = VecOps(dev, dt)
    rng = np.random.default_rng(seed)
    hist = LbfgsHistory(n, m, ops)
    for _ in range(npair):           # npair > m wraps the ring
        s = rng.standard_normal(n)
        y = s + 0.1 * rng.standard_normal(n)
        hist.push(torch.tensor(s, device=dev, dtype=dt), torch.tensor(y, device=dev, dtype=dt))
    g = torch.tensor(rng.standard_normal(n), device=dev, dtype=dt)
    return hist, g


def test_noalloc_matches_apply_two_calls_second_smaller():
    cases = [(200003, 12, 15, torch.float32, 5, 0.7),    # several reduction blocks, ring wrapped
             (1531, 3, 2, torch.float64, 6, 1.3)]        # smaller: fewer elements and pairs
    for n, m, npair, dt, seed, h0 in cases:
        print(f"noalloc case n={n} m={m} pairs={npair} dtype={dt}", flush=True)
        hist, g = _history(n, m, npair, dt, seed)
        want = hist.apply(g, torch.empty_like(g), h0)
        # poison the output so that an unwritten element shows
        got = hist.apply_noalloc(g, torch.full_like(g, float("nan")), h0)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (n, m)
        assert torch.isfinite(got).all()
        # r may alias g, as for fwi_lbfgs_apply
        g2 = g.clone()
        hist.apply_noalloc(g2, g2, h0)
        assert torch.equal(g2, want)
        hist.close()


def test_noalloc_rejects_history_beyond_static_scratch():
    from paper_2102_00755_amd import _lib
    lib = _lib.load()
    hist, g = _history(64, _lib.FWI_NOALLOC_MAX_PAIRS + 1, 1, torch.float32, 7)
    r = torch.full_like(g, 3.0)
    rc = lib.fwi_lbfgs_apply_noalloc(hist._h, ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(r.data_ptr()),
                                     1.0, None)
    assert rc == _lib.FWI_ERR_INVALID_ARG
    assert b"static scratch" in lib.fwi_last_error()
    torch.cuda.synchronize()
    assert torch.all(r == 3.0)       # nothing launched
    hist.close()

"""GPU parity of the grid transfers (Sec. 2.4, App. C) with the oracle:
Fourier interpolation between handles of the same box (eta = 2 and 1.5,
with and without the Blackman window) and windowed-sinc time resampling."""

import numpy as np
import pytest
import torch

from oracle import multigrid as omg
from synth import make_small

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _handle(shape, dx, precision):
    from paper_2102_00755_amd.fwi import Handle
    prob = make_small(shape=shape, dx=dx, nt=4, pml=2, layer=1, precision=precision, r_transducer=3.0,
                      r_gamma=2.0, n_src=1, n_rec=2)
    return Handle.from_problem(prob, precision=precision)


@pytest.mark.parametrize("precision", [8, 4])
@pytest.mark.parametrize("shapes", [((24, 32, 32), (48, 64, 64)), ((32, 32, 32), (48, 48, 48)),
                                    ((12, 16, 24), (12, 16, 24))])
@pytest.mark.parametrize("window", ["blackman", "none"])
def test_interp_up_matches_oracle(precision, shapes, window):
    from paper_2102_00755_amd import multigrid as mg
    (sc, sf) = shapes
    dx_f = 0.5e-3
    dx_c = dx_f * sf[2] / sc[2]
    hc = _handle(sc, dx_c, precision)
    hf = _handle(sf, dx_f, precision)
    rng = np.random.default_rng(7)
    u = 1500 + 30 * rng.standard_normal(sc)
    print("interp", sc, sf, window, precision, flush=True)
    got = mg.interp_up(hc, hf, torch.from_numpy(u), window=window).cpu().numpy()
    want = omg.interp_up(u, sf, window=window)
    assert rel(got, want) < (1e-12 if precision == 8 else 2e-6)
    hc.close()
    hf.close()


def test_interp_up_rejects_other_boxes():
    from paper_2102_00755_amd import multigrid as mg
    from paper_2102_00755_amd.fwi import FwiError
    hc = _handle((24, 32, 32), 1.0e-3, 8)
    hf = _handle((48, 64, 64), 0.6e-3, 8)
    with pytest.raises(FwiError):
        mg.interp_up(hc, hf, torch.zeros(24, 32, 32, dtype=torch.float64))
    hc.close()
    hf.close()


@pytest.mark.parametrize("precision", [8, 4])
def test_resample_time_matches_oracle(precision):
    from paper_2102_00755_amd import multigrid as mg
    rng = np.random.default_rng(8)
    dt_f = 83.3e-9
    eta = 2.0
    nt_f = 300
    dt_c, nt_c = mg.coarse_level(dt_f, nt_f, eta)
    f = rng.standard_normal((nt_f, 5))
    fc = mg.coarse_cutoff(1350.0, 1.0e-3)
    dtype = torch.float64 if precision == 8 else torch.float32
    got = mg.resample_time(torch.tensor(f, device="cuda", dtype=dtype), dt_f, dt_c, nt_c, fc, beta=8.0,
                           t_window=12 * dt_c, scale=mg.data_scale(eta)).cpu().numpy()
    want = omg.resample_time(f, dt_f, dt_c, nt_c, fc, 8.0, 12 * dt_c, scale=eta ** 2)
    assert got.shape == (150, 5)
    assert rel(got, want) < (1e-12 if precision == 8 else 1e-5)

"""Host-side checks of the C-ABI library (no GPU needed).

* the library loads and exports every entry point declared in include/fwi.h;
* the host-only entry points behave: Rademacher weights bit-exact against
  the oracle's SplitMix64, workspace query, argument validation.
"""

import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from synth import make_config, make_small

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2102_00755_amd import _lib as L
    return L, L.load()


def test_library_exports_every_declared_symbol():
    L, lib = _lib()
    hdr = open(os.path.join(ROOT, "include", "fwi.h")).read()
    declared = set(re.findall(r"\b(fwi_[a-z_]+)\s*\(", hdr))
    assert declared == set(L.EXPORTED)
    for name in declared:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("seed", [0, 1, 1005, 2 ** 63 + 12345])
def test_rademacher_bit_exact_with_oracle(seed):
    from paper_2102_00755_amd.fwi import rademacher
    n = 2048
    assert np.array_equal(rademacher(seed, n), oracle.rademacher(seed, n))


def test_workspace_query_and_validation():
    from paper_2102_00755_amd import fwi
    prob = make_small(shape=(16, 24, 32), nt=10, precision=4)
    kw = fwi.problem_kwargs(prob)
    b1 = fwi.workspace_bytes(**dict(kw), batch=1)
    b2 = fwi.workspace_bytes(**dict(kw), batch=2)
    nfield = 16 * 24 * 32
    assert b1 > 6 * nfield * 4 * 2           # two slots of six fields at least
    assert b2 > b1
    bad = dict(kw)
    bad["shape"] = (16, 24, 30)              # nx/2 = 15 is not a supported length
    assert fwi.workspace_bytes(**bad) == 0
    bad = dict(kw)
    bad["gamma"] = np.zeros_like(prob.gamma)  # dGamma outside Gamma
    assert fwi.workspace_bytes(**bad) == 0


def test_full_size_workspace_fits_one_gpu():
    from paper_2102_00755_amd import fwi
    prob = make_config("full")
    nbytes = fwi.workspace_bytes(**fwi.problem_kwargs(prob), batch=1)
    # tape (2200 steps x |dGamma|) + two slots of state and spectra
    tape = 2200 * int(prob.boundary.sum()) * 4
    assert tape < nbytes < 24e9


@pytest.mark.parametrize("seed,tau", [(0, 0), (7, 100), (1005, 2200)])
def test_delays_bit_exact_with_oracle(seed, tau):
    from paper_2102_00755_amd.fwi import delays
    got = delays(seed, 1024, tau)
    want = oracle.delays(seed, 1024, tau)
    assert np.array_equal(got, want)
    assert got.min() >= 0 and got.max() <= tau
    if tau:
        assert abs(got.mean() / tau - 0.5) < 0.05     # d_i ~ U[0,1)


def test_set_delays_rejects_null_handle():
    L, lib = _lib()
    assert lib.fwi_set_delays(None, 0, None) == L.FWI_ERR_INVALID_ARG


def test_set_tuning_rejects_null_handle_and_bad_values():
    L, lib = _lib()
    t = L.FwiTuning(128, 128, 128)
    assert lib.fwi_set_tuning(None, ctypes.byref(t)) == L.FWI_ERR_INVALID_ARG
    assert lib.fwi_get_tuning(None, ctypes.byref(t)) == L.FWI_ERR_INVALID_ARG


def test_set_absorption_rejects_null_handle_and_db_conversion_matches_oracle():
    L, lib = _lib()
    assert lib.fwi_set_absorption(None, 1e-3, 1.5, None, 1) == L.FWI_ERR_INVALID_ARG
    from oracle import lossy
    from paper_2102_00755_amd.fwi import db_to_neper
    for a_db, y in ((0.75, 1.5), (15.0, 0.6), (0.5, 1.1)):
        want = lossy.db_to_neper(a_db, y)
        assert abs(db_to_neper(a_db, y) - want) <= 1e-15 * want


def test_autotune_choice_and_cache(tmp_path):
    from paper_2102_00755_amd import autotune
    per = {64: {"y_fwd": 1.0, "y_inv": 1.0, "y_vel_q": 1.0, "z_minus": 2.0, "z_plus": 1.0},
           128: {"y_fwd": 0.9, "y_inv": 0.9, "y_vel_q": 1.0, "z_minus": 2.5, "z_plus": 0.5}}
    assert autotune.choose(per) == {"y_tile_bytes": 128, "zm_tile_bytes": 64, "zp_tile_bytes": 128}
    path = str(tmp_path / "sub" / "tuning.json")
    assert autotune.load_cache(path) == {}
    key = autotune.cache_key("AMD Instinct MI355X", 4, (224, 448, 448), 1)
    assert key == "AMD Instinct MI355X|fp32|224x448x448|B1"
    autotune.save_cache({key: {"y_tile_bytes": 128}}, path)
    assert autotune.load_cache(path) == {key: {"y_tile_bytes": 128}}
    with open(path, "w") as f:
        f.write("not json")
    assert autotune.load_cache(path) == {}


def _create_status(mutate_params=None, mutate_geo=None):
    """fwi_create status for a valid small problem with one change; the
    argument checks run before any device call, so this needs no GPU."""
    from paper_2102_00755_amd import fwi
    L, lib = _lib()
    prob = make_small(shape=(16, 24, 32), nt=10, precision=4)
    kw = fwi.problem_kwargs(prob)
    geo_kw = dict(src=np.array(kw["src_ijk"]), rec=np.array(kw["rec_ijk"]), gamma=kw["gamma"].copy(),
                  boundary=kw["boundary"].copy())
    if mutate_geo:
        mutate_geo(geo_kw, prob)
    p = fwi._params(kw["shape"], kw["dx"], kw["dt"], kw["nt"], kw["c_ref"], kw["c_min"], kw["c_max"], kw["rho0"],
                    kw["pml"], kw["pml_alpha"], kw["precision"], 1)
    if mutate_params:
        mutate_params(p)
    geo = fwi._Geometry(geo_kw["src"], geo_kw["rec"], geo_kw["gamma"], geo_kw["boundary"])
    h = ctypes.c_void_p(None)
    rc = lib.fwi_create(ctypes.byref(p), ctypes.byref(geo.c), 0, ctypes.byref(h))
    assert not h.value or rc == L.FWI_OK
    return rc, L


def test_create_rejects_invalid_arguments_before_any_device_call():
    rc, L = _create_status(lambda p: setattr(p, "nx", 30))
    assert rc == L.FWI_ERR_UNSUPPORTED                       # nx/2 = 15 not a supported length
    assert _create_status(lambda p: setattr(p, "precision", 5))[0] == L.FWI_ERR_INVALID_ARG
    assert _create_status(lambda p: setattr(p, "nx", 31))[0] == L.FWI_ERR_INVALID_ARG   # odd nx
    assert _create_status(lambda p: setattr(p, "nt", 0))[0] == L.FWI_ERR_INVALID_ARG
    assert _create_status(lambda p: setattr(p, "c_min", -1.0))[0] == L.FWI_ERR_INVALID_ARG
    assert _create_status(lambda p: setattr(p, "dt", 1e-5))[0] == L.FWI_ERR_INVALID_ARG  # kappa argument too large

    def src_in_pml(g, prob):
        g["src"][0] = (0, 0, 0)
    assert _create_status(mutate_geo=src_in_pml)[0] == L.FWI_ERR_INVALID_ARG

    def dup_rec(g, prob):
        g["rec"][1] = g["rec"][0]
    assert _create_status(mutate_geo=dup_rec)[0] == L.FWI_ERR_INVALID_ARG

    def bnd_outside(g, prob):
        g["boundary"][0, 0, 0] = 1
    assert _create_status(mutate_geo=bnd_outside)[0] == L.FWI_ERR_INVALID_ARG

    def gamma_in_pml(g, prob):
        g["gamma"][0, :, :] = 1
    assert _create_status(mutate_geo=gamma_in_pml)[0] == L.FWI_ERR_INVALID_ARG

    def src_in_gamma(g, prob):
        z, y, x = np.argwhere(prob.gamma)[0]
        g["src"][0] = (x, y, z)
    assert _create_status(mutate_geo=src_in_gamma)[0] == L.FWI_ERR_INVALID_ARG

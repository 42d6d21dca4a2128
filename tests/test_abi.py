"""Host-side checks of the C ABI: librmhd.so loads, exports every function declared in
include/rmhd.h, and validates parameters (no GPU work is issued)."""
import ctypes
import os
import re

import pytest

from paper_1808_09721_amd import rmhd as R
from paper_1808_09721_amd import workloads as WL

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in sorted(os.listdir(inc)):
        if f.endswith(".h"):
            src = re.sub(r"/\*.*?\*/", "", open(os.path.join(inc, f)).read(), flags=re.S)
            names |= set(re.findall(r"\b(rmhd_\w+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(R.LIB_PATH):
        pytest.skip("librmhd.so not built")
    names = declared_functions()
    assert names, "no declarations found"
    lib = ctypes.CDLL(R.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(R.EXPORTS) == names


def test_layout_of_pads_rows_and_counts_variables():
    p = R.params_from(WL.kelvin_helmholtz_2d(10, 7, steps=1))
    L = R.rmhd_layout_of(p)
    assert (L.nxg, L.nyg) == (14, 11)
    assert L.pitch == 16 and L.plane == 16 * 11
    assert (L.ncons, L.nprim) == (14, 5)
    p = R.params_from(WL.two_fluid_sheet_2d(12, 8, steps=1))
    L = R.rmhd_layout_of(p)
    assert (L.pitch, L.nyg, L.ncons, L.nprim) == (16, 12, 18, 10)
    p = R.params_from(WL.brio_wu_1d(400))
    L = R.rmhd_layout_of(p)
    assert (L.nxg, L.nyg, L.pitch, L.plane) == (404, 1, 408, 408)


def test_layout_of_3d_grids():
    p = R.params_from(WL.kelvin_helmholtz_3d(10, 6, 5, steps=1))
    L = R.rmhd_layout_of(p)
    assert (L.nxg, L.nyg, L.nzg, L.pitch) == (14, 10, 9, 16)
    assert L.slab == 16 * 10 and L.plane == 16 * 10 * 9
    # below 3-D there is one z plane
    L2 = R.rmhd_layout_of(R.params_from(WL.kelvin_helmholtz_2d(10, 7, steps=1)))
    assert (L2.nzg, L2.slab) == (1, L2.plane)


@pytest.mark.parametrize("field,value,msg", [("nz", 3, "nz >= 4"), ("ndim", 4, "ndim"), ("reserved_", 1, "reserved_"),
                                             ("z1", -0.5, "empty domain")])
def test_layout_of_rejects_bad_3d_parameters(field, value, msg):
    p = R.params_from(WL.kelvin_helmholtz_3d(8, 8, 8, steps=1))
    setattr(p, field, value)
    with pytest.raises(R.RmhdError, match=msg):
        R.rmhd_layout_of(p)
    p2 = R.params_from(WL.kelvin_helmholtz_2d(8, 8, steps=1))
    p2.nz = 5
    with pytest.raises(R.RmhdError, match="nz"):
        R.rmhd_layout_of(p2)


@pytest.mark.parametrize("field,value,msg", [("nx", 2, "nx >= 4"), ("model", 5, "model"), ("gamma_eos", 2.5, "gamma"),
                                             ("bc", 3, "bc"), ("max_newton_iter", 0, "iteration")])
def test_layout_of_rejects_bad_parameters(field, value, msg):
    p = R.params_from(WL.kelvin_helmholtz_2d(16, 16, steps=1))
    setattr(p, field, value)
    with pytest.raises(R.RmhdError, match=msg):
        R.rmhd_layout_of(p)


def test_two_fluid_needs_distinct_charge_to_mass_ratios():
    wl = WL.two_fluid_sheet_2d(16, 16, steps=1)
    p = R.params_from(wl)
    p.mu2 = p.mu1
    with pytest.raises(R.RmhdError, match="mu1 != mu2"):
        R.rmhd_layout_of(p)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(R, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(R, "_lib", None)
    with pytest.raises(R.RmhdError, match="missing"):
        R.lib()


def _batch_create_error(params):
    lib = R.lib()
    arr = (R.rmhd_params * len(params))(*params)
    b = ctypes.c_void_p()
    rc = lib.rmhd_batch_create(arr, len(params), None, ctypes.byref(b))
    msg = lib.rmhd_batch_last_error(b).decode()
    lib.rmhd_batch_destroy(b)
    return rc, msg


def test_batch_create_validates_before_touching_the_gpu():
    if not os.path.exists(R.LIB_PATH):
        pytest.skip("librmhd.so not built")
    ok = R.params_from(WL.brio_wu_1d(128))
    tf = R.params_from(WL.two_fluid_sheet_2d(16, 16, steps=1))
    rc, msg = _batch_create_error([ok, tf])
    assert rc == -1 and "single-fluid" in msg
    bad = R.params_from(WL.brio_wu_1d(128))
    bad.nx = 2
    rc, msg = _batch_create_error([ok, bad])
    assert rc == -1 and "domain 1" in msg
    lib = R.lib()
    b = ctypes.c_void_p()
    assert lib.rmhd_batch_create(None, 0, None, ctypes.byref(b)) == -1
    lib.rmhd_batch_destroy(b)


def test_batched_domains_recipe_is_seeded():
    a = WL.batched_domains(seed=4)
    b = WL.batched_domains(seed=4)
    assert len(a) == 64 and sum(w.ndim == 1 for w in a) == 32
    assert [(w.nx, w.ny, w.sigma) for w in a] == [(w.nx, w.ny, w.sigma) for w in b]
    assert all(128 <= w.nx <= 4096 for w in a if w.ndim == 1)
    assert all(64 <= w.nx <= 512 and 64 <= w.ny <= 512 for w in a if w.ndim == 2)
    assert all(10.0 <= w.sigma <= 1e6 for w in a)


def test_newton_percentile_from_histogram():
    st = {"newton_hist": [0, 0, 70, 29, 1] + [0] * 11}
    assert R.newton_percentile(st, 0.5) == 2
    assert R.newton_percentile(st, 0.7) == 2
    assert R.newton_percentile(st, 0.99) == 3
    assert R.newton_percentile(st, 1.0) == 4
    assert R.newton_percentile({"newton_hist": [0] * 16}, 0.5) == 15


def test_stats_record_matches_header():
    """The ctypes mirror of rmhd_stats has the header's fields in the header's order."""
    src = open(os.path.join(ROOT, "include", "rmhd.h")).read()
    body = src[src.index("typedef struct rmhd_stats {"):src.index("} rmhd_stats;")]
    names = re.findall(r"\b(\w+)(?:\[\d+\])?;", re.sub(r"/\*.*?\*/", "", body, flags=re.S))
    assert names == [n for n, _ in R.rmhd_stats._fields_]


def test_recovery_fallback_switch_is_validated():
    p = R.params_from(WL.kelvin_helmholtz_2d(16, 16, steps=1), c2p_primary_only=2)
    with pytest.raises(R.RmhdError, match="c2p_primary_only"):
        R.rmhd_layout_of(p)
    for v in (0, 1):
        R.rmhd_layout_of(R.params_from(WL.kelvin_helmholtz_2d(16, 16, steps=1), c2p_primary_only=v))


def test_integrator_is_validated_and_batch_rejects_ssp3():
    p = R.params_from(WL.kelvin_helmholtz_2d(16, 16, steps=1), integrator=2)
    with pytest.raises(R.RmhdError, match="integrator"):
        R.rmhd_layout_of(p)
    if not os.path.exists(R.LIB_PATH):
        pytest.skip("librmhd.so not built")
    ok = R.params_from(WL.brio_wu_1d(128))
    s3 = R.params_from(WL.brio_wu_1d(128), integrator=R.SSP3_332)
    rc, msg = _batch_create_error([ok, s3])
    assert rc == -1 and "SSP2" in msg

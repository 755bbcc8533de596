"""The C ABI library loads, exports every declared entry point, and validates
arguments on the host (no GPU needed for any of this)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "hamlet.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hamlet_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for required in ("hamlet_plan_create", "hamlet_logpost_grad", "hamlet_leapfrog", "hamlet_hmc_run",
                     "hamlet_plan_destroy", "hamlet_plan_footprint_bytes", "hamlet_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2203_02369_amd import _capi
    lib = _capi.load()
    for name in _declared_functions():
        assert hasattr(lib, name), name
    assert set(_declared_functions()) == set(_capi.SIGNATURES)


def test_footprint_query_is_host_only():
    from paper_2203_02369_amd import hamlet
    small = hamlet.footprint_bytes(32, 1000, "fp64")
    big = hamlet.footprint_bytes(256, 30000, "fp32")
    assert 0 < small < big
    # five FP32 spectral arrays and four FP64 mode arrays dominate at 256^3
    nm = 256 * 256 * 128
    assert big > nm * (5 * 8 + 4 * 16)
    assert hamlet.footprint_bytes(256, 30000, "fp64") > big


def test_invalid_arguments_are_rejected_on_the_host():
    from paper_2203_02369_amd import _capi, hamlet
    lib = _capi.load()
    out = ctypes.c_size_t()
    pk = np.ones(3 * 16 * 16 + 1)
    desc = _capi.PlanDesc(n_grid=24, precision=0, box=100.0, omega_m=0.3, h=0.7, f_growth=0.5, sigma_v=300.0,
                          pk_n2=pk.ctypes.data_as(_capi.c_double_p), n_pk=len(pk), hist_width=5.0,
                          sample_distances=1, sample_sigma_nl=1)
    assert lib.hamlet_plan_footprint_bytes(ctypes.byref(desc), 10, ctypes.byref(out)) == -4
    assert b"n_grid" in lib.hamlet_last_error()
    desc.n_grid = 32
    assert lib.hamlet_plan_footprint_bytes(ctypes.byref(desc), 10, ctypes.byref(out)) == 0
    desc.n_pk = 5
    assert lib.hamlet_plan_footprint_bytes(ctypes.byref(desc), 10, ctypes.byref(out)) == -1
    desc.n_pk = len(pk)
    desc.sigma_v = -1.0
    assert lib.hamlet_plan_footprint_bytes(ctypes.byref(desc), 10, ctypes.byref(out)) == -1
    assert lib.hamlet_plan_create(None, None, None, ctypes.byref(ctypes.c_void_p())) == -1
    with pytest.raises(_capi.HamletError):
        _capi.check(-1)


def test_batch_entry_points_reject_bad_plan_lists_on_the_host():
    from paper_2203_02369_amd import _capi
    lib = _capi.load()
    fake = ctypes.c_void_p(0x1000)     # never dereferenced: the list check comes first
    plans = (ctypes.c_void_p * 2)(fake, fake)
    null_ptrs = (ctypes.c_void_p * 2)()
    dnull = (_capi.c_double_p * 2)()
    assert lib.hamlet_logpost_grad(plans, 0, null_ptrs, dnull, dnull, null_ptrs, dnull, dnull, dnull) == -1
    assert b"at least one plan" in lib.hamlet_last_error()
    assert lib.hamlet_logpost_grad(plans, 2, null_ptrs, dnull, dnull, null_ptrs, dnull, dnull, dnull) == -1
    assert b"same plan" in lib.hamlet_last_error()
    one = (ctypes.c_void_p * 1)(None)
    assert lib.hamlet_hmc_run(one, 1, None, null_ptrs, dnull, dnull, None, None, None, None) == -1
    assert b"NULL" in lib.hamlet_last_error()


def test_server_entry_points_validate_on_the_host():
    from paper_2203_02369_amd import _capi
    lib = _capi.load()
    out = ctypes.c_void_p()
    desc = _capi.ServerDesc(hbm_budget=0, max_running=0, ticks_ahead=0)
    assert lib.hamlet_server_create(ctypes.byref(desc), None, ctypes.byref(out)) == -1
    assert b"hbm_budget" in lib.hamlet_last_error()
    assert lib.hamlet_server_create(None, None, ctypes.byref(out)) == -1
    assert lib.hamlet_server_tick(None, None) == -1
    state = ctypes.c_int32()
    assert lib.hamlet_server_job_state(None, 1, ctypes.byref(state)) == -1
    assert lib.hamlet_server_take(None, 1, None, None, None, None, None, None, None) == -1
    assert lib.hamlet_server_destroy(None) == 0


def test_velocity_field_validates_on_the_host():
    from paper_2203_02369_amd import _capi
    lib = _capi.load()
    assert lib.hamlet_velocity_field(None, None, None) == -1
    assert b"NULL" in lib.hamlet_last_error()
    assert lib.hamlet_density_field(None, None, None) == -1
    assert lib.hamlet_field_stats_accumulate(None, None, None) == -1
    assert lib.hamlet_shell_stats(None, None, None, 10.0, 4, None) == -1


def test_sphere_moments_validate_on_the_host():
    from paper_2203_02369_amd import _capi
    lib = _capi.load()
    radii = (ctypes.c_double * 2)(10.0, 20.0)
    assert lib.hamlet_sphere_moments(None, None, radii, 2, None) == -1
    assert b"NULL" in lib.hamlet_last_error()


def test_flat_vector_entry_points_validate_on_the_host():
    from paper_2203_02369_amd import _capi
    lib = _capi.load()
    n = ctypes.c_int64()
    assert lib.hamlet_flat_size(None, ctypes.byref(n)) == -1
    assert b"NULL" in lib.hamlet_last_error()
    assert lib.hamlet_pack_flat(None, None, None, None, None) == -1
    assert lib.hamlet_unpack_flat(None, None, None, None, None) == -1


def test_refined_mock_keeps_the_field_on_the_coarse_nodes():
    # the input generator's finer-grid copy of a universe (used at 512^3)
    import numpy as np
    from paper_2203_02369_amd import mocks
    m = mocks.make_mock(16, 200.0, 50, 80.0, seed=3)
    r = mocks.refine(m, 32)
    coarse = np.fft.irfftn(m.dhat_true, s=(16, 16, 16), axes=(0, 1, 2))
    fine = np.fft.irfftn(r.dhat_true, s=(32, 32, 32), axes=(0, 1, 2))
    assert np.abs(fine[::2, ::2, ::2] - coarse).max() <= 1e-12 * np.abs(coarse).max()
    assert r.n_grid == 32 and len(r.pk_n2) == 3 * 16 ** 2 + 1 and r.n_gal == m.n_gal

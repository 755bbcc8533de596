"""Sphere moments of the velocity field (hamlet_sphere_moments) against the
oracle (oracle/analysis.py), through the C ABI.

Tolerance: the moments are signed sums over all modes in FP64 on both
sides, in different orders; each value must agree within 1e-12 times the
sum of the absolute values of its terms (the scale of the rounding error).
"""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import analysis, hmc
from paper_2203_02369_amd import mocks

from helpers import oracle_problem, start_modes, to_lib_layout

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def hl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_02369_amd import hamlet
    return hamlet


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _check(got, prob, dhat, radii):
    mono, dip = analysis.sphere_moments(prob, dhat, radii)
    ref = np.concatenate([mono[:, None], dip], axis=1)
    scale = analysis.sphere_moments_abs(prob, dhat, radii)
    err = np.abs(got - ref)
    assert np.all(err <= TOL * scale + 1e-300), (np.max(err / scale), got, ref)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_moments_match_the_oracle(hl, precision):
    m = mocks.plain_fp64_32()
    prob = oracle_problem(m)
    rng = np.random.default_rng(11)
    shape = (32, 32, 17)
    dhat = hmc.symmetrise(32, 1e3 * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)))
    # below the series switch (|k| R < 1/2 for every mode), across it, and out to the box size
    radii = [0.05, 3.0, 12.5, 40.0, 90.0, 150.0, 199.0, 260.0, 380.0]
    say("moments 32^3", precision)
    plan = hl.Plan.from_mock(m, precision=precision)
    q = torch.from_numpy(to_lib_layout(dhat)).to(plan.device)
    out = hl.sphere_moments(plan, q, radii)
    torch.cuda.synchronize()
    _check(out.cpu().numpy(), prob, dhat, radii)
    plan.close()


def test_moments_are_bit_identical_across_reruns_and_precisions(hl):
    m = mocks.plain_fp64_32()
    dhat = start_modes(m)
    radii = [7.0, 30.0, 100.0, 150.0, 170.0]
    say("moments determinism")
    outs = []
    for precision in ("fp64", "fp32", "fp64"):
        plan = hl.Plan.from_mock(m, precision=precision)
        q = torch.from_numpy(to_lib_layout(dhat)).to(plan.device)
        outs.append(hl.sphere_moments(plan, q, radii).cpu().numpy())
        plan.close()
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_moments_at_the_paper_scale(hl):
    # the mock field of the 256^3 benchmark, sixteen radii (four passes)
    m = mocks.paper_scale_256()
    prob = oracle_problem(m)
    dhat = start_modes(m)
    radii = [5.0 + 15.0 * j for j in range(16)]
    say("moments 256^3")
    plan = hl.Plan.from_mock(m, precision="fp32")
    q = torch.from_numpy(to_lib_layout(dhat)).to(plan.device)
    out = hl.sphere_moments(plan, q, radii).cpu().numpy()
    plan.close()
    say("oracle 256^3")
    _check(out, prob, dhat, radii)


def test_moments_validate_their_arguments(hl):
    from paper_2203_02369_amd import _capi
    m = mocks.make_mock(16, 200.0, 50, 80.0, seed=5)
    plan = hl.Plan.from_mock(m, precision="fp64")
    q = torch.zeros(plan.mode_shape, dtype=torch.complex128, device=plan.device)
    say("moments validation")
    for bad in ([0.0], [-3.0], [math.nan], [math.inf], [10.0] * 17):
        with pytest.raises(Exception):
            hl.sphere_moments(plan, q, bad)
    assert b"radius" in _capi.load().hamlet_last_error() or b"n_radii" in _capi.load().hamlet_last_error()
    # no radii: nothing to do
    assert hl.sphere_moments(plan, q, []).numel() == 0
    # a zero field has zero moments
    out = hl.sphere_moments(plan, q, [10.0, 50.0])
    assert torch.count_nonzero(out).item() == 0
    plan.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [32, 64])
def test_velocity_field_matches_the_oracle(hl, precision, n):
    # the whole field of a state on every node (hamlet_velocity_field)
    # against the oracle's velocity grids (eq:vel-field)
    from oracle import model
    m = mocks.plain_fp64_32() if n == 32 else mocks.make_mock(64, 500.0, 2000, 250.0, "inv_r", seed=33)
    prob = oracle_problem(m)
    dhat = start_modes(m)
    ref = model.velocity_grids(prob, dhat)
    say("velocity field", n, precision)
    plan = hl.Plan.from_mock(m, precision=precision)
    q = torch.from_numpy(to_lib_layout(dhat)).to(plan.device)
    v = hl.velocity_field(plan, q).double().cpu().numpy()
    plan.close()
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert np.abs(v - ref).max() <= tol * np.abs(ref).max(), np.abs(v - ref).max() / np.abs(ref).max()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [32, 64])
def test_density_field_matches_the_oracle(hl, precision, n):
    # the density contrast of a state on every node (hamlet_density_field)
    # against the oracle's density grid
    from oracle import model
    m = mocks.plain_fp64_32() if n == 32 else mocks.make_mock(64, 500.0, 2000, 250.0, "inv_r", seed=33)
    prob = oracle_problem(m)
    dhat = start_modes(m)
    ref = model.density_grid(prob, dhat)
    say("density field", n, precision)
    plan = hl.Plan.from_mock(m, precision=precision)
    q = torch.from_numpy(to_lib_layout(dhat)).to(plan.device)
    dens = hl.density_field(plan, q).double().cpu().numpy()
    plan.close()
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert np.abs(dens - ref).max() <= tol * np.abs(ref).max(), np.abs(dens - ref).max() / np.abs(ref).max()


def test_fields_at_the_paper_scale(hl):
    # the velocity and density fields of a state of the 256^3 benchmark,
    # every node, in the precision the benchmark runs (FP32 fields)
    from oracle import model
    m = mocks.paper_scale_256()
    prob = oracle_problem(m)
    dhat = start_modes(m)
    say("fields 256^3 fp32")
    plan = hl.Plan.from_mock(m, precision="fp32")
    q = torch.from_numpy(to_lib_layout(dhat)).to(plan.device)
    v = hl.velocity_field(plan, q).double().cpu().numpy()
    dens = hl.density_field(plan, q).double().cpu().numpy()
    plan.close()
    say("oracle density 256^3")
    ref = model.density_grid(prob, dhat)
    assert np.abs(dens - ref).max() <= 1e-5 * np.abs(ref).max(), np.abs(dens - ref).max() / np.abs(ref).max()
    del dens, ref
    say("oracle velocity 256^3")
    ref = model.velocity_grids(prob, dhat)
    assert np.abs(v - ref).max() <= 1e-5 * np.abs(ref).max(), np.abs(v - ref).max() / np.abs(ref).max()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [32, 64])
def test_field_stats_match_the_oracle(hl, precision, n):
    # three states added to the running sums of delta, v_r and their squares
    # (hamlet_field_stats_accumulate), against the oracle's sums
    m = mocks.plain_fp64_32() if n == 32 else mocks.make_mock(64, 500.0, 2000, 250.0, "inv_r", seed=33)
    prob = oracle_problem(m)
    a = start_modes(m)
    rng = np.random.default_rng(40 + n)
    amp = np.abs(a).std()
    shape = a.shape
    b = hmc.symmetrise(n, amp * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)))
    states = [a, b, -0.5 * a]
    say("field stats", n, precision)
    plan = hl.Plan.from_mock(m, precision=precision)
    acc = None
    for s in states:
        acc = hl.field_stats_accumulate(plan, torch.from_numpy(to_lib_layout(s)).to(plan.device), acc)
    got = acc.cpu().numpy()
    plan.close()
    from oracle import model
    ref = analysis.field_sums(prob, states)
    tol = 1e-12 if precision == "fp64" else 1e-5
    dmax = [np.abs(model.density_grid(prob, s)).max() for s in states]
    vmax = [np.abs(analysis.radial_velocity_grid(prob, s)).max() for s in states]
    for i, (scale, tl) in enumerate([(sum(dmax), tol), (sum(d * d for d in dmax), 2.5 * tol),
                                     (sum(vmax), tol), (sum(v * v for v in vmax), 2.5 * tol)]):
        err = np.abs(got[i] - ref[i]).max()
        assert err <= tl * scale, (i, err / scale)


def _shell_inputs(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n, n))
    b = 0.6 * a + 0.8 * rng.standard_normal((n, n, n))
    return a, b


def _check_shells(got, ref, a, b):
    assert np.array_equal(got[:, 0], ref[:, 0])
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref)
    scale = np.array([1.0, np.abs(a).max(), np.abs(a).max(), np.abs(b).max(), np.abs(b).max(), 1.0])
    err = np.where(ok, np.abs(got - ref), 0.0) / scale
    assert err[:, 1:5].max() <= 1e-12 and err[:, 5].max() <= 1e-10, err.max(axis=0)


def _margin(prob, width):
    # no node sits within rounding of a shell boundary unless exactly on it
    f = analysis.node_distances(prob) / width
    d = np.abs(f - np.round(f))
    assert d[d > 0].min() > 1e-9


@pytest.mark.parametrize("n", [32, 64])
def test_shell_stats_match_the_oracle(hl, n):
    # hamlet_shell_stats on seeded fields against the oracle, shells out past
    # the box corner (the last ones empty)
    m = mocks.plain_fp64_32() if n == 32 else mocks.make_mock(64, 500.0, 2000, 250.0, "inv_r", seed=33)
    prob = oracle_problem(m)
    a, b = _shell_inputs(n, 50 + n)
    plan = hl.Plan.from_mock(m, precision="fp64")
    ta, tb = torch.from_numpy(a).to(plan.device), torch.from_numpy(b).to(plan.device)
    rmax = analysis.node_distances(prob).max()
    for width in ([7.3, 23.1, 10.0] if n == 32 else [10.0, 17.9]):
        _margin(prob, width)
        n_shells = int(math.ceil(rmax / width)) + 2
        say("shell stats", n, width, n_shells)
        got = hl.shell_stats(plan, ta, tb, width, n_shells).cpu().numpy()
        _check_shells(got, analysis.shell_stats(prob, a, b, width, n_shells), a, b)
        again = hl.shell_stats(plan, ta, tb, width, n_shells).cpu().numpy()
        assert np.array_equal(np.nan_to_num(again, nan=7.0), np.nan_to_num(got, nan=7.0))
    # b absent: its statistics are those of a zero field
    got = hl.shell_stats(plan, ta, None, 23.1 if n == 32 else 17.9, 8).cpu().numpy()
    _check_shells(got, analysis.shell_stats(prob, a, None, 23.1 if n == 32 else 17.9, 8), a, np.ones(1))
    plan.close()


def test_shell_stats_at_the_paper_scale(hl):
    # 256^3 grid, shells of 10 Mpc/h out past the corner of the 500 Mpc/h box
    m = mocks.paper_scale_256()
    prob = oracle_problem(m)
    a, b = _shell_inputs(256, 256)
    _margin(prob, 10.0)
    say("shell stats 256^3")
    plan = hl.Plan.from_mock(m, precision="fp32")
    got = hl.shell_stats(plan, torch.from_numpy(a).to(plan.device), torch.from_numpy(b).to(plan.device), 10.0, 45)
    got = got.cpu().numpy()
    plan.close()
    say("oracle shells 256^3")
    _check_shells(got, analysis.shell_stats(prob, a, b, 10.0, 45), a, b)


def test_shell_stats_validate_their_arguments(hl):
    m = mocks.make_mock(16, 200.0, 50, 80.0, seed=5)
    plan = hl.Plan.from_mock(m, precision="fp64")
    a = torch.zeros((16, 16, 16), dtype=torch.float64, device=plan.device)
    say("shell stats validation")
    for width, ns in ((0.0, 4), (-1.0, 4), (math.nan, 4), (math.inf, 4), (10.0, -1), (10.0, 5000)):
        with pytest.raises(Exception):
            hl.shell_stats(plan, a, a, width, ns)
    with pytest.raises(ValueError):
        hl.shell_stats(plan, a.float(), a, 10.0, 4)
    assert hl.shell_stats(plan, a, a, 10.0, 0).numel() == 0
    # a constant field: mean the constant, no scatter, no correlation
    got = hl.shell_stats(plan, a + 2.5, a, 30.0, 3).cpu().numpy()
    assert np.all(got[:, 1] == 2.5) and np.all(got[:, 2] == 0.0) and np.all(np.isnan(got[:, 5]))
    plan.close()

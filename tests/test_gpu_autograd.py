"""The adjoint behind torch.autograd.Function: gradcheck, finite differences
on random modes at the paper scale, and the oracle gradient at 256^3."""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import hmc, model
from paper_2203_02369_amd import mocks

from helpers import from_lib_layout, oracle_problem, rel_inf, start_modes, to_lib_layout

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_02369_amd import autograd, hamlet
    return hamlet, autograd


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _inputs(plan, m, dhat, d, s, grad=True):
    dev = plan.device
    q = torch.from_numpy(to_lib_layout(dhat)).to(dev).requires_grad_(grad)
    qd = torch.from_numpy(np.ascontiguousarray(d)).to(dev).requires_grad_(grad)
    qs = plan.scalar(s).requires_grad_(grad)
    return q, qd, qs


def test_gradcheck_fp64_small(lib):
    hamlet, ag = lib
    m = mocks.make_mock(16, 200.0, 120, 70.0, "sphere", (0.2, 0.2), seed=51)
    dhat = start_modes(m)
    rng = np.random.default_rng(3)
    d = m.d_true * (1 + 0.01 * rng.standard_normal(m.n_gal))
    say("gradcheck fp64 16^3")
    plan = hamlet.Plan.from_mock(m, precision="fp64")
    q, qd, qs = _inputs(plan, m, dhat, d, 1.2)
    fn = lambda a, b, c: ag.hamlet_logpost(plan, a, b, c)
    assert torch.autograd.gradcheck(fn, (q, qd, qs), eps=1e-6, atol=1e-6, rtol=1e-5, fast_mode=True)
    plan.close()


def test_backward_matches_oracle_per_entry_convention(lib):
    # d Psi / d(stored entry) = oracle gradient, halved on the kz = 0 plane
    hamlet, ag = lib
    m = mocks.plain_fp64_32()
    prob = oracle_problem(m)
    dhat = start_modes(m)
    d = m.d_true.copy()
    psi_r, g_r, gd_r, gs_r = model.logpost_grad(prob, dhat, d, 1.3)
    say("backward fp64 32^3")
    plan = hamlet.Plan.from_mock(m, precision="fp64")
    q, qd, qs = _inputs(plan, m, dhat, d, 1.3)
    psi = ag.hamlet_logpost(plan, q, qd, qs)
    (2.0 * psi).backward()
    assert abs(psi.item() - psi_r) <= 1e-12 * abs(psi_r)
    half = np.ones(g_r.shape)
    half[:, :, 0] = 0.5
    assert rel_inf(from_lib_layout(q.grad.cpu().numpy()), 2.0 * half * g_r) <= 1e-12
    assert rel_inf(qd.grad.cpu().numpy(), 2.0 * gd_r) <= 1e-12
    assert abs(qs.grad.item() - 2.0 * gs_r) <= 1e-12 * abs(gs_r)
    plan.close()


def _fd_modes(hamlet, plan, dhat, d, s, picks, hscale):
    """Central differences of Psi in single independent mode coordinates."""
    n = plan.n_grid
    dev = plan.device
    var = plan_var(n, plan)
    base = torch.from_numpy(to_lib_layout(dhat)).to(dev)
    qd = torch.from_numpy(np.ascontiguousarray(d)).to(dev)
    qs = plan.scalar(s)
    g, gd, gs, psi = plan.zeros_modes(), plan.zeros_dist(), plan.scalar(), plan.scalar()
    out = []
    for (ix, iy, iz, comp) in picks:
        h = hscale * math.sqrt(var[ix, iy, iz])
        vals = []
        for sgn in (+1, -1):
            q = base.clone()
            delta = complex(h * sgn * (1.0 if comp == 0 else 1j))
            q[ix, iy, iz] += delta
            if iz == 0:        # keep the kz = 0 plane Hermitian: move the partner too
                q[(-ix) % n, (-iy) % n, 0] += complex(delta).conjugate()
            hamlet.logpost_grad([plan], [q], [qd], [qs], [g], [gd], [gs], [psi])
            vals.append(psi.item())
        out.append((vals[0] - vals[1]) / (2 * h))
    return np.array(out)


_VAR = {}


def plan_var(n, plan):
    return _VAR[n]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_finite_differences_64_modes_256(lib, precision):
    # Psi is quadratic in any single mode coordinate, so the central
    # difference is exact up to rounding even for a step of the prior scale.
    hamlet, ag = lib
    m = mocks.paper_scale_256()
    prob = oracle_problem(m)
    _VAR[256] = model.mode_variance(prob)
    n = 256
    dhat = m.dhat_true
    d = m.d_true.copy()
    s = 1.5
    rng = np.random.default_rng(64)
    keep = hmc.canonical_mask(n)
    cand = np.argwhere(keep[:, :, : n // 2])
    picks = [tuple(cand[i]) + (int(rng.integers(2)),) for i in rng.choice(len(cand), 56, replace=False)]
    plane = np.argwhere(keep[:, :, :1])
    picks += [tuple(plane[i]) + (int(rng.integers(2)),) for i in rng.choice(len(plane), 8, replace=False)]
    say("fd 64 modes 256^3", precision)
    plan = hamlet.Plan.from_mock(m, precision=precision)
    q, qd, qs = _inputs(plan, m, dhat, d, s, grad=False)
    g, gd, gs, psi = plan.zeros_modes(), plan.zeros_dist(), plan.scalar(), plan.scalar()
    hamlet.logpost_grad([plan], [q], [qd], [qs], [g], [gd], [gs], [psi])
    gg = g.cpu().numpy()
    an = np.array([gg[ix, iy, iz].real if c == 0 else gg[ix, iy, iz].imag for ix, iy, iz, c in picks])
    fd = _fd_modes(hamlet, plan, dhat, d, s, picks, hscale=1.0)
    scale = np.abs(an).max()
    # FP32 fields: the rounding of Psi's field part does not cancel between
    # the two evaluations; the FP32 gradient itself is checked against the
    # oracle at 1e-4 in test_paper_scale_gradient_matches_oracle_fp32
    tol = 1e-7 if precision == "fp64" else 1e-2
    say("max |fd - grad| / max |grad| =", np.abs(fd - an).max() / scale)
    assert np.abs(fd - an).max() <= tol * scale
    plan.close()


def test_paper_scale_gradient_matches_oracle_fp32(lib):
    # 256^3, 30 000 points, the launch configuration the benchmark times.
    hamlet, ag = lib
    m = mocks.paper_scale_256()
    prob = oracle_problem(m)
    dhat = m.dhat_true
    d = m.d_true.copy()
    s = 1.5
    say("oracle 256^3 (one evaluation on the host)")
    psi_r, g_r, gd_r, gs_r = model.logpost_grad(prob, dhat, d, s)
    say("gpu 256^3 fp32")
    plan = hamlet.Plan.from_mock(m, precision="fp32")
    q, qd, qs = _inputs(plan, m, dhat, d, s, grad=False)
    g, gd, gs, psi = plan.zeros_modes(), plan.zeros_dist(), plan.scalar(), plan.scalar()
    hamlet.logpost_grad([plan], [q], [qd], [qs], [g], [gd], [gs], [psi])
    torch.cuda.synchronize()
    assert abs(psi.item() - psi_r) <= 2e-5 * abs(psi_r)
    assert rel_inf(from_lib_layout(g.cpu().numpy()), g_r) <= 1e-4
    assert rel_inf(gd.cpu().numpy(), gd_r) <= 1e-4
    assert abs(gs.item() - gs_r) <= 1e-4 * abs(gs_r)
    plan.close()

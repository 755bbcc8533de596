"""Batched execution through the C ABI: plans of one grid size and
precision share every kernel launch (blockIdx.z selects the plan).

A chain's numbers must not depend on which other chains share its launches:
every output of a batched call is compared bit for bit with the same plan
called alone, for batches that mix grid sizes, precisions, catalogue sizes
(including an empty catalogue), leapfrog lengths and HIP streams, and for
more plans than one launch holds.  The batched gradients are also checked
against the oracle.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import hmc, model
from paper_2203_02369_amd import _capi, mocks

from helpers import from_lib_layout, oracle_problem, rel_inf, start_modes, to_lib_layout

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_02369_amd import hamlet
    return hamlet


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _empty(m):
    for key in ("mu", "sigma_mu", "cz", "sigma_cz", "d_init", "d_true"):
        setattr(m, key, np.zeros(0))
    m.rhat = np.zeros((0, 3))
    return m


# (mock, precision): two grid sizes, both precisions, uneven catalogues.
def _members():
    return [
        (mocks.make_mock(16, 200.0, 300, 80.0, "sphere", (0.2, 0.2), seed=31), "fp64"),
        (mocks.make_mock(32, 400.0, 400, 120.0, "sphere", (0.2, 0.2), seed=41), "fp64"),
        (mocks.make_mock(16, 200.0, 120, 70.0, "inv_r", (0.15, 0.25), seed=35), "fp64"),
        (mocks.make_mock(16, 200.0, 300, 80.0, "sphere", (0.2, 0.2), seed=36), "fp32"),
        (_empty(mocks.make_mock(16, 200.0, 5, 50.0, seed=3)), "fp64"),
        (mocks.make_mock(32, 400.0, 700, 120.0, "inv_r", (0.2, 0.2), seed=44), "fp32"),
        (mocks.make_mock(16, 200.0, 200, 80.0, "sphere", (0.2, 0.2), seed=37), "fp64"),
    ]


_mem = {}


def members():
    if "m" not in _mem:
        out = []
        for k, (m, prec) in enumerate(_members()):
            rng = np.random.default_rng(100 + k)
            d = m.d_true * (1.0 + 0.02 * rng.standard_normal(m.n_gal))
            out.append((m, prec, start_modes(m), d, 1.2 + 0.05 * k))
        _mem["m"] = out
    return _mem["m"]


def _state(plan, dhat, d, s):
    dev = plan.device
    return (torch.from_numpy(to_lib_layout(dhat)).to(dev), torch.from_numpy(d.copy()).to(dev), plan.scalar(s))


def _grad(hl, plans, states):
    outs = [(p.zeros_modes(), p.zeros_dist(), p.scalar(), p.scalar()) for p in plans]
    hl.logpost_grad(plans, [s[0] for s in states], [s[1] for s in states], [s[2] for s in states],
                    [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs], [o[3] for o in outs])
    torch.cuda.synchronize()
    return [tuple(t.cpu().numpy() for t in o) for o in outs]


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def test_batched_gradient_equals_alone_and_oracle(hl):
    mem = members()
    plans = [hl.Plan.from_mock(m, precision=prec) for (m, prec, _, _, _) in mem]
    states = [_state(p, dh, d, s) for p, (_, _, dh, d, s) in zip(plans, mem)]
    say("batched gradient, %d plans" % len(plans))
    together = _grad(hl, plans, states)
    for j, p in enumerate(plans):
        say("alone", j, p.n_grid, p.precision, p.n_gal)
        alone = _grad(hl, [p], [states[j]])[0]
        assert _same(together[j], alone), "plan %d differs when batched" % j
    for j, (m, prec, dhat, d, s) in enumerate(mem):
        ref = model.logpost_grad(oracle_problem(m), dhat, d, s)
        assert np.isfinite(ref[0]), "test input %d outside the posterior's domain" % j
        g, gd, gs, psi = together[j]
        tol_psi, tol_g = (1e-12, 1e-12) if prec == "fp64" else (2e-5, 1e-4)
        assert abs(psi[0] - ref[0]) <= tol_psi * abs(ref[0])
        assert rel_inf(from_lib_layout(g), ref[1]) <= tol_g
        if m.n_gal:
            assert rel_inf(gd, ref[2]) <= tol_g
            assert abs(gs[0] - ref[3]) <= tol_g * abs(ref[3])
        else:
            assert gs[0] == 0.0
    for p in plans:
        p.close()


def _momenta(plan, seed):
    rng = np.random.default_rng(seed)
    n = plan.n_grid
    pm = hmc.symmetrise(n, (rng.standard_normal((n, n, n // 2 + 1)) + 1j * rng.standard_normal((n, n, n // 2 + 1)))
                        * 1e-3)
    return to_lib_layout(pm), rng.standard_normal(plan.n_gal), float(rng.standard_normal())


def _leap(hl, plans, states, moms, eps, steps):
    qs, ps = [], []
    for p, st, mo in zip(plans, states, moms):
        qs.append([t.clone() for t in st])
        ps.append((torch.from_numpy(mo[0]).to(p.device), torch.from_numpy(mo[1].copy()).to(p.device),
                   p.scalar(mo[2])))
    psi = [p.scalar() for p in plans]
    hl.leapfrog(plans, eps, steps, [q[0] for q in qs], [q[1] for q in qs], [q[2] for q in qs],
                [x[0] for x in ps], [x[1] for x in ps], [x[2] for x in ps], psi)
    torch.cuda.synchronize()
    return [tuple(t.cpu().numpy() for t in (*q, *x, y)) for q, x, y in zip(qs, ps, psi)]


def test_batched_leapfrog_equals_alone(hl):
    mem = members()
    plans = [hl.Plan.from_mock(m, precision=prec) for (m, prec, _, _, _) in mem]
    states = [_state(p, dh, d, s) for p, (_, _, dh, d, s) in zip(plans, mem)]
    moms = [_momenta(p, 7 + j) for j, p in enumerate(plans)]
    eps = [1e-3 * (1 + 0.1 * j) for j in range(len(plans))]
    steps = [3, 3, 2, 3, 0, 1, 3]        # groups split by trajectory length too
    say("batched leapfrog")
    together = _leap(hl, plans, states, moms, eps, steps)
    for j, p in enumerate(plans):
        say("alone", j)
        alone = _leap(hl, [p], [states[j]], [moms[j]], [eps[j]], [steps[j]])[0]
        assert _same(together[j], alone), "plan %d differs when batched" % j
    for p in plans:
        p.close()


def _chains(hl, plans, starts, n_iter, n_lf, seeds, warmup=0, resume=False, runs=None):
    runs = runs or [dict(q=[t.clone() for t in st], msum=p.zeros_modes(),
                         dh=torch.zeros(n_iter, dtype=torch.float64, device=p.device),
                         acc=torch.zeros(n_iter, dtype=torch.int32, device=p.device))
                    for p, st in zip(plans, starts)]
    eps = hl.hmc_run(plans, [r["q"][0] for r in runs], [r["q"][1] for r in runs], [r["q"][2] for r in runs],
                     n_iter=n_iter, n_leapfrog=n_lf, eps0=2e-3, seed=0, seeds=seeds, warmup=warmup, jitter=True,
                     mode_sum=[r["msum"] for r in runs], dh=[r["dh"] for r in runs],
                     accepted=[r["acc"] for r in runs], resume=resume)
    torch.cuda.synchronize()
    return runs, eps


def _pull(run):
    return tuple(t.cpu().numpy() for t in (*run["q"], run["msum"], run["dh"], run["acc"]))


def test_batched_chains_equal_alone(hl):
    mem = members()
    plans = [hl.Plan.from_mock(m, precision=prec) for (m, prec, _, _, _) in mem]
    starts = [_state(p, dh, d, s) for p, (_, _, dh, d, s) in zip(plans, mem)]
    seeds = [1000 + 17 * j for j in range(len(plans))]
    n_iter, n_lf = 6, 4
    say("batched chains")
    runs, eps = _chains(hl, plans, starts, n_iter, n_lf, seeds, warmup=3)
    for j, p in enumerate(plans):
        say("alone", j)
        r1, e1 = _chains(hl, [p], [starts[j]], n_iter, n_lf, [seeds[j]], warmup=3)
        assert _same(_pull(runs[j]), _pull(r1[0])), "chain %d differs when batched" % j
        assert eps[j] == e1[0]
    for p in plans:
        p.close()


def test_batched_chain_matches_oracle(hl):
    # the second chain of a batch (key seeds[1]) against the oracle chain
    mem = members()
    picks = [0, 2, 6]
    plans = [hl.Plan.from_mock(mem[k][0], precision="fp64") for k in picks]
    starts = [_state(p, mem[k][2], mem[k][3], mem[k][4]) for p, k in zip(plans, picks)]
    seeds = [5, 2203, 9]
    n_iter, n_lf, eps0 = 5, 4, 2e-3
    say("batched chain vs oracle")
    runs, _ = _chains(hl, plans, starts, n_iter, n_lf, seeds)
    m, _, dhat, d, s = mem[picks[1]]
    res = hmc.hmc_run(oracle_problem(m), hmc.State(dhat, d.copy(), s), n_iter, n_lf, eps0, seeds[1], jitter=True)
    q, qd, qs, msum, dh, acc = _pull(runs[1])
    assert np.array_equal(acc, res.accepted)
    errs = {"modes": rel_inf(from_lib_layout(q), res.state.modes), "dist": rel_inf(qd, res.state.dist),
            "mode_sum": rel_inf(from_lib_layout(msum), res.mode_sum)}
    say("batched chain errors against the oracle", errs)
    for k, e in errs.items():
        assert e <= 1e-12, (k, e)
    for p in plans:
        p.close()


_big = {}


def _big_members(n_grid):
    """Three problems at one of the benchmark's grid sizes (box 500 Mpc/h,
    n ~ 1/r, zone of avoidance): two FP32 plans that share launches and one
    FP64 plan, a group of its own that runs beside them.  At 64^3 the
    30 000-point catalogue crowds its columns (the scatter's dense path)."""
    if n_grid not in _big:
        sizes = {64: (30000, 4000, 9000), 128: (10000, 2500, 6000), 256: (30000, 5000, 12000)}[n_grid]
        out = []
        for k, (ng, prec) in enumerate(zip(sizes, ("fp32", "fp32", "fp64"))):
            m = mocks.paper_scale_256(n_gal=ng, n_grid=n_grid, seed=mocks.config_seed(4) + 50 * k + n_grid)
            rng = np.random.default_rng(400 + k)
            out.append((m, prec, start_modes(m), m.d_true * (1.0 + 0.02 * rng.standard_normal(m.n_gal)),
                        1.1 + 0.1 * k))
        _big[n_grid] = out
    return _big[n_grid]


@pytest.mark.parametrize("n_grid", [64, 128, 256])
def test_shared_launches_at_benchmark_grids(hl, n_grid):
    # The tile widths, thread counts and scatter paths of the benchmark's
    # instantiations in shared launches: gradients and a two-step leapfrog
    # of the batch bit-identical to each plan alone, gradients against the
    # oracle, and at 64^3 and 128^3 the leapfrog too.
    mem = _big_members(n_grid)
    plans = [hl.Plan.from_mock(m, precision=prec) for (m, prec, _, _, _) in mem]
    states = [_state(p, dh, d, s) for p, (_, _, dh, d, s) in zip(plans, mem)]
    say("shared launches at %d^3: gradient" % n_grid)
    together = _grad(hl, plans, states)
    for j, p in enumerate(plans):
        assert _same(together[j], _grad(hl, [p], [states[j]])[0]), "plan %d differs when batched" % j
    moms = [_momenta(p, 70 + j) for j, p in enumerate(plans)]
    eps = [2e-4, 3e-4, 2e-4]
    say("shared launches at %d^3: leapfrog" % n_grid)
    lf_together = _leap(hl, plans, states, moms, eps, [2, 2, 2])
    for j, p in enumerate(plans):
        assert _same(lf_together[j], _leap(hl, [p], [states[j]], [moms[j]], [eps[j]], [2])[0]), \
            "plan %d leapfrog differs when batched" % j
    for j, (m, prec, dhat, d, s) in enumerate(mem):
        say("oracle gradient %d at %d^3" % (j, n_grid))
        prob = oracle_problem(m)
        ref = model.logpost_grad(prob, dhat, d, s)
        g, gd, gs, psi = together[j]
        tol_psi, tol_g = (1e-12, 1e-12) if prec == "fp64" else (2e-5, 1e-4)
        errs = {"psi": abs(psi[0] - ref[0]) / abs(ref[0]), "modes": rel_inf(from_lib_layout(g), ref[1]),
                "dist": rel_inf(gd, ref[2]), "s": abs(gs[0] - ref[3]) / abs(ref[3])}
        say("  errors", prec, errs)
        assert errs["psi"] <= tol_psi
        assert max(errs["modes"], errs["dist"], errs["s"]) <= tol_g
        if n_grid <= 128 and j in (0, 2):
            pm, pd, ps = moms[j]
            q0 = hmc.State(dhat, d.copy(), s)
            p0 = hmc.State(from_lib_layout(pm), pd.copy(), ps)
            q1, p1, c1 = hmc.leapfrog(prob, q0, p0, eps[j], 2)
            got = lf_together[j]
            lerrs = {"modes": rel_inf(from_lib_layout(got[0]) - q0.modes, q1.modes - q0.modes),
                     "dist": rel_inf(got[1] - q0.dist, q1.dist - q0.dist),
                     "p_modes": rel_inf(from_lib_layout(got[3]) - p0.modes, p1.modes - p0.modes),
                     "p_dist": rel_inf(got[4] - p0.dist, p1.dist - p0.dist)}
            say("  leapfrog displacement errors", prec, lerrs)
            assert max(lerrs.values()) <= tol_g
            assert abs(got[6][0] - c1[0]) <= tol_psi * abs(c1[0])
    for p in plans:
        p.close()


def test_resumed_chain_equals_one_run(hl):
    m, prec, dhat, d, s = members()[1]
    plan = hl.Plan.from_mock(m, precision=prec)
    start = _state(plan, dhat, d, s)
    n_iter, n_lf = 6, 3
    say("resume")
    whole, e_whole = _chains(hl, [plan], [start], n_iter, n_lf, [77], warmup=4)
    parts, _ = _chains(hl, [plan], [start], 2, n_lf, [77], warmup=4, runs=[dict(
        q=[t.clone() for t in start], msum=plan.zeros_modes(),
        dh=torch.zeros(n_iter, dtype=torch.float64, device=plan.device),
        acc=torch.zeros(n_iter, dtype=torch.int32, device=plan.device))])
    parts, e_parts = _chains(hl, [plan], None, 4, n_lf, [77], warmup=4, resume=True, runs=parts)
    assert _same(_pull(whole[0]), _pull(parts[0]))
    assert e_whole[0] == e_parts[0]
    plan.close()


def test_more_plans_than_one_launch(hl):
    # 34 small plans of one size: two shared launches per kernel
    base = [mocks.make_mock(16, 200.0, 40 + 3 * j, 70.0, "sphere", (0.2, 0.2), seed=200 + j) for j in range(34)]
    plans = [hl.Plan.from_mock(m, precision="fp32") for m in base]
    states = [_state(p, start_modes(m), m.d_true.copy(), 1.0) for p, m in zip(plans, base)]
    say("34 plans")
    together = _grad(hl, plans, states)
    for j in (0, 31, 32, 33):
        assert _same(together[j], _grad(hl, [plans[j]], [states[j]])[0])
    for p in plans:
        p.close()


def test_plans_on_different_streams(hl):
    mem = members()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    plans = [hl.Plan.from_mock(mem[0][0], precision="fp64", stream=s1),
             hl.Plan.from_mock(mem[2][0], precision="fp64", stream=s2)]
    states = [_state(p, mem[k][2], mem[k][3], mem[k][4]) for p, k in zip(plans, (0, 2))]
    torch.cuda.synchronize()
    say("two streams")
    together = _grad(hl, plans, states)
    for j in range(2):
        assert _same(together[j], _grad(hl, [plans[j]], [states[j]])[0])
    for p in plans:
        p.close()


def test_same_plan_twice_is_rejected(hl):
    m, prec, dhat, d, s = members()[0]
    plan = hl.Plan.from_mock(m, precision=prec)
    st = _state(plan, dhat, d, s)
    with pytest.raises(_capi.HamletError, match="same plan"):
        _grad(hl, [plan, plan], [st, st])
    plan.close()

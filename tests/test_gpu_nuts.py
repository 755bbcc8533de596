"""The No-U-Turn sampler on the GPU (hamlet_nuts_run) against the oracle's
(oracle/nuts.py), through the C ABI.

Under the shared counter-based stream both build the same trees: the
doublings of every iteration, its leapfrog steps and the leaf the chain moves
to must be identical in FP64, and the states within 1e-12 (with an adapted
step, within the bound that the step's sensitivity to dH gives, as for HMC).
In FP32 the trees must agree up to the first decision that differs, and
that decision must be a near-tie of the FP32 Hamiltonian.  Chains sharing
launches equal the same chains run alone, bit for bit.
"""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import hmc, model, nuts
from paper_2203_02369_amd import mocks

from helpers import TOL64, from_lib_layout, oracle_problem, path_length, rel_inf, start_modes, to_lib_layout

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


def _m16():
    return mocks.make_mock(16, 200.0, 300, 80.0, "sphere", (0.2, 0.2), seed=31)


# (mock, plan and problem overrides, step, most doublings): trees that end by
# the whole trajectory turning back, by a subtree turning back or leaving the
# slice part-way through a doubling, and by the depth cap.
CASES = {
    "16^3 frozen d, trajectory U-turns": (_m16, dict(sample_distances=False), 0.05, 9),
    "16^3 frozen d, subtree stops": (_m16, dict(sample_distances=False), 0.1, 6),
    "32^3 depth cap": (mocks.plain_fp64_32, {}, 0.02, 6),
}


def _start(m, k):
    rng = np.random.default_rng(600 + k)
    return start_modes(m), m.d_true * (1.0 + 0.01 * rng.standard_normal(m.n_gal)), 1.2 + 0.05 * k


def _gpu_state(plan, dhat, d, s):
    dev = plan.device
    return (torch.from_numpy(to_lib_layout(dhat)).to(dev), torch.from_numpy(np.ascontiguousarray(d)).to(dev),
            plan.scalar(s))


def _oracle(m, start, n_iter, eps, seed, warmup=0, max_depth=6, **over):
    prob = oracle_problem(m, **over)
    q0 = hmc.State(start[0], start[1].copy(), start[2])
    return prob, q0, nuts.nuts_run(nuts.PosteriorTarget(prob), q0, n_iter, eps, seed, warmup=warmup,
                                   max_depth=max_depth)


def _compare_trees(got, res):
    say("depth gpu", got["depth"].tolist(), "oracle", res.depth.tolist())
    say("where gpu", got["where"].tolist(), "oracle", res.where.tolist())
    assert np.array_equal(got["depth"], res.depth)
    assert np.array_equal(got["leaves"], res.leaves)
    assert np.array_equal(got["where"], res.where)


@pytest.mark.parametrize("name", list(CASES))
def test_nuts_fp64_matches_oracle(hl, name):
    mk, over, eps, depth = CASES[name]
    m = mk()
    start = _start(m, 0)
    n_iter, seed = 6, 4242
    prob, q0, res = _oracle(m, start, n_iter, eps, seed, max_depth=depth, **over)
    say("oracle trees", res.depth.tolist(), res.leaves.tolist())
    assert res.depth.max() >= 2 and np.any(res.where[:, 0] >= 0)   # the trees grow and the chain moves
    say("nuts fp64", name)
    plan = hl.Plan.from_mock(m, precision="fp64", **over)
    q, qd, qs = _gpu_state(plan, *start)
    msum = plan.zeros_modes()
    got = hl.nuts_run([plan], [q], [qd], [qs], n_iter=n_iter, eps0=eps, seed=seed, max_depth=depth,
                      mode_sum=[msum])[0]
    torch.cuda.synchronize()
    _compare_trees(got, res)
    # alpha = mean of exp(H0 - H) over the leaves: its error is that of the
    # energy differences, TOL64 of H each
    h_scale = abs(model.logpost(prob, q0.modes, q0.dist, q0.s))
    errs = {"alpha": float(np.abs(got["alpha"] - res.alpha).max()) / (2.0 * h_scale),
            "modes": rel_inf(from_lib_layout(q.cpu().numpy()), res.state.modes),
            "dist": rel_inf(qd.cpu().numpy(), res.state.dist),
            "s": abs(qs.item() - res.state.s) / abs(res.state.s),
            "mode_sum": rel_inf(from_lib_layout(msum.cpu().numpy()), res.mode_sum)}
    say("nuts fp64 errors", errs)
    for k, e in errs.items():
        assert e <= TOL64, (k, e)
    plan.close()


def test_nuts_fp64_dual_averaging_matches_oracle(hl):
    m = _m16()
    start = _start(m, 1)
    n_iter, warm, eps0, seed = 10, 6, 0.1, 77
    path = [start[0]]
    prob = oracle_problem(m)
    q0 = hmc.State(start[0], start[1].copy(), start[2])
    res = nuts.nuts_run(nuts.PosteriorTarget(prob), q0, n_iter, eps0, seed, warmup=warm, max_depth=6,
                        callback=lambda it, q, st: path.append(q.modes.copy()))
    say("nuts fp64 with dual averaging")
    plan = hl.Plan.from_mock(m, precision="fp64")
    q, qd, qs = _gpu_state(plan, *start)
    got = hl.nuts_run([plan], [q], [qd], [qs], n_iter=n_iter, eps0=eps0, seed=seed, warmup=warm, max_depth=6)[0]
    torch.cuda.synchronize()
    _compare_trees(got, res)
    # the step is a function of the acceptance statistics alpha / n_alpha:
    # |d ln eps| <= (sqrt(W) / gamma) max |d alpha| (as for HMC)
    a_err = float(np.abs(got["alpha"] - res.alpha).max())
    a_tol = 2.0 * TOL64 * abs(model.logpost(prob, q0.modes, q0.dist, q0.s))
    e_err = abs(got["eps"] - res.eps) / res.eps
    e_tol = TOL64 + math.sqrt(warm) / 0.05 * a_err
    s_err = rel_inf(from_lib_layout(q.cpu().numpy()), res.state.modes)
    s_tol = TOL64 + 2.0 * e_err * path_length(path)
    say("nuts dual averaging: alpha err %.3g (tol %.3g), eps err %.3g (tol %.3g), state err %.3g (tol %.3g)"
        % (a_err, a_tol, e_err, e_tol, s_err, s_tol))
    assert a_err <= a_tol and e_err <= e_tol and s_err <= s_tol
    plan.close()


def test_nuts_shared_launches_equal_alone(hl):
    ms = [(_m16(), "fp64"), (mocks.make_mock(16, 200.0, 150, 70.0, "inv_r", (0.15, 0.25), seed=35), "fp64"),
          (mocks.plain_fp64_32(), "fp32"), (mocks.make_mock(16, 200.0, 200, 80.0, "sphere", (0.2, 0.2), seed=36),
                                            "fp32")]
    plans = [hl.Plan.from_mock(m, precision=p) for m, p in ms]
    starts = [_start(m, k) for k, (m, _) in enumerate(ms)]
    seeds = [11, 12, 13, 14]

    def run(idx):
        st = [_gpu_state(plans[k], *starts[k]) for k in idx]
        out = hl.nuts_run([plans[k] for k in idx], [s[0] for s in st], [s[1] for s in st], [s[2] for s in st],
                          n_iter=4, eps0=0.03, seed=0, seeds=[seeds[k] for k in idx], max_depth=5)
        torch.cuda.synchronize()
        return [(o, tuple(t.cpu().numpy() for t in s)) for o, s in zip(out, st)]
    say("nuts shared launches")
    together = run(range(len(plans)))
    for k in range(len(plans)):
        alone = run([k])[0]
        for key in ("depth", "leaves", "where", "alpha"):
            assert np.array_equal(together[k][0][key], alone[0][key]), (k, key)
        for a, b in zip(together[k][1], alone[1]):
            assert np.array_equal(a, b), k
    for p in plans:
        p.close()


def test_nuts_fp32_trees_match_oracle_up_to_near_ties(hl):
    # The FP32 fields move H by ~1e-6 relative: the trees must be the
    # oracle's until the first decision that differs, and that decision must
    # be a near-tie (a slice test within the FP32 H error, or an iteration
    # whose tree the oracle built differently only after such a leaf).
    m = mocks.plain_fp64_32()
    start = _start(m, 2)
    n_iter, eps, seed = 8, 0.02, 5150
    prob, q0, res = _oracle(m, start, n_iter, eps, seed)
    say("nuts fp32")
    plan = hl.Plan.from_mock(m, precision="fp32")
    q, qd, qs = _gpu_state(plan, *start)
    got = hl.nuts_run([plan], [q], [qd], [qs], n_iter=n_iter, eps0=eps, seed=seed, max_depth=6)[0]
    torch.cuda.synchronize()
    plan.close()
    same = (got["depth"] == res.depth) & (got["leaves"] == res.leaves) & np.all(got["where"] == res.where, axis=1)
    upto = int(np.cumprod(same).sum())
    say("fp32 trees equal to the oracle's for %d of %d iterations" % (upto, n_iter))
    a_err = float(np.abs(got["alpha"][:upto] - res.alpha[:upto]).max()) if upto else 0.0
    say("fp32 alpha error over those: %.3g" % a_err)
    assert a_err <= 1e-3
    # at paper-like smoothness a flip needs a tie; over 8 iterations of a
    # few dozen leaves none is expected, and at most one is accepted
    assert upto >= n_iter - 1, (got["depth"], res.depth)

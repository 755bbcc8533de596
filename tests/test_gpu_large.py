"""The 512^3 grid (through the C ABI): the 256^3 benchmark's catalogue on a
grid twice as fine, modes drawn from the prior.

Both paths are compared with the oracle on sampled outputs: Psi, the
gradient in every distance and in s, and the mode gradient at 64 entries
(the oracle's velocity field is its full inverse transform; its adjoint is
summed directly at the sampled modes).  Besides, properties that hold at any
size: the gradient against central differences of Psi (exact up to
rounding: Psi is quadratic in a single mode coordinate), the FP32 path
against the FP64 path, bit-identical reruns, and the reversibility of the
leapfrog map.
"""
import math
import sys

import numpy as np
import pytest
import torch

from paper_2203_02369_amd import mocks

from helpers import from_lib_layout, rel_inf

pytestmark = pytest.mark.gpu

N = 512


@pytest.fixture(scope="module")
def hl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2203_02369_amd import hamlet
    return hamlet


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


_cache = {}


def problem():
    """(problem kwargs, modes in the library layout, distances, sigma_k^2)."""
    if not _cache:
        m = mocks.paper_scale_256()
        kw = m.problem_kwargs()
        kw["n_grid"] = N
        pk = mocks.PowerSpectrum(omega_m=m.omega_m, h=m.h).table_n2(N, m.box)
        kw["pk_n2"] = pk
        # modes from the prior on kz >= 1 (the kz = 0 plane left at zero, so
        # the state is Hermitian by construction), Nyquist rows excluded
        rng = np.random.default_rng(512)
        s = np.where(np.arange(N) < N // 2, np.arange(N), np.arange(N) - N)
        kz = np.arange(N // 2)
        n2 = s[:, None, None] ** 2 + s[None, :, None] ** 2 + kz[None, None, :] ** 2
        var = (float(N) ** 6 / m.box ** 3) * pk[n2]
        keep = (np.abs(s)[:, None, None] != N // 2) & (np.abs(s)[None, :, None] != N // 2) & (kz[None, None, :] > 0)
        amp = np.where(keep, np.sqrt(0.5 * var), 0.0)
        q = amp * rng.standard_normal(n2.shape) + 1j * (amp * rng.standard_normal(n2.shape))
        _cache.update(kw=kw, q=q, d=m.d_true.copy(), var=np.where(keep, var, 0.0))
    return _cache["kw"], _cache["q"], _cache["d"], _cache["var"]


def evaluate(hl, plan, q, qd, qs):
    g, gd, gs, psi = plan.zeros_modes(), plan.zeros_dist(), plan.scalar(), plan.scalar()
    hl.logpost_grad([plan], [q], [qd], [qs], [g], [gd], [gs], [psi])
    torch.cuda.synchronize()
    return psi.item(), g, gd, gs.item()


_oracle = {}


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_512_gradient_against_sampled_oracle(hl, precision):
    from oracle import model
    kw, qn, d, var = problem()
    s = 1.5
    if not _oracle:
        rng = np.random.default_rng(5120)
        sx = np.where(np.arange(N) < N // 2, np.arange(N), np.arange(N) - N)
        ok = np.abs(sx) != N // 2
        # 48 entries with kz > 0 and 16 on the kz = 0 plane, none excluded
        ix = rng.choice(np.nonzero(ok)[0], 64)
        iy = rng.choice(np.nonzero(ok)[0], 64)
        iz = np.concatenate([rng.integers(1, N // 2, 48), np.zeros(16, dtype=np.int64)])
        iz[48:][(ix[48:] == 0) & (iy[48:] == 0)] = 1
        prob = model.Problem(**kw)
        say("oracle 512^3: full inverse transforms, adjoint at 64 modes (about a minute)")
        _oracle.update(kidx=(ix, iy, iz), ref=model.logpost_grad_sampled(prob, from_lib_layout(qn), d, s,
                                                                          (ix, iy, iz)))
    kidx, ref = _oracle["kidx"], _oracle["ref"]
    say("512^3 %s plan" % precision)
    plan = hl.Plan(**kw, precision=precision)
    q = torch.from_numpy(qn).to(plan.device)
    qd = torch.from_numpy(d).to(plan.device)
    psi, g, gd, gs = evaluate(hl, plan, q, qd, plan.scalar(s))
    gg = g.cpu().numpy()
    plan.close()
    # the mode gradient's error relative to its largest entry over the grid
    gmax = float(np.abs(gg).max())
    errs = {"psi": abs(psi - ref[0]) / abs(ref[0]),
            "modes": float(np.abs(gg[kidx] - ref[1]).max()) / gmax,
            "dist": rel_inf(gd.cpu().numpy(), ref[2]), "s": abs(gs - ref[3]) / abs(ref[3])}
    say("512^3 %s errors against the oracle" % precision, errs)
    tol_psi, tol_g = (1e-12, 1e-12) if precision == "fp64" else (2e-5, 1e-4)
    assert errs["psi"] <= tol_psi
    assert max(errs["modes"], errs["dist"], errs["s"]) <= tol_g


def test_512_gradient_against_central_differences_fp64(hl):
    kw, qn, d, var = problem()
    say("512^3 fp64 plan")
    plan = hl.Plan(**kw, precision="fp64")
    q = torch.from_numpy(qn).to(plan.device)
    qd = torch.from_numpy(d).to(plan.device)
    qs = plan.scalar(1.5)
    psi, g, gd, gs = evaluate(hl, plan, q, qd, qs)
    assert math.isfinite(psi)
    gg = g.cpu().numpy()
    rng = np.random.default_rng(3)
    picks = []
    while len(picks) < 24:
        ix, iy, iz = (int(v) for v in rng.integers(0, (N, N, N // 2)))
        if var[ix, iy, iz] > 0 and (ix, iy, iz) not in [t[:3] for t in picks]:
            picks.append((ix, iy, iz, int(rng.integers(2))))
    an, fd = [], []
    for (ix, iy, iz, comp) in picks:
        h = math.sqrt(var[ix, iy, iz])
        v0 = q[ix, iy, iz].item()
        vals = []
        for sgn in (+1, -1):
            q[ix, iy, iz] = v0 + h * sgn * (1.0 if comp == 0 else 1j)
            vals.append(evaluate(hl, plan, q, qd, qs)[0])
        q[ix, iy, iz] = v0
        fd.append((vals[0] - vals[1]) / (2 * h))
        an.append(gg[ix, iy, iz].real if comp == 0 else gg[ix, iy, iz].imag)
    an, fd = np.array(an), np.array(fd)
    say("modes: max |fd - grad| / max |grad| =", np.abs(fd - an).max() / np.abs(an).max())
    assert np.abs(fd - an).max() <= 1e-7 * np.abs(an).max()
    # s: Psi is smooth in s
    h = 1e-4
    vals = []
    for sgn in (+1, -1):
        vals.append(evaluate(hl, plan, q, qd, plan.scalar(1.5 + sgn * h))[0])
    fds = (vals[0] - vals[1]) / (2 * h)
    assert abs(fds - gs) <= 1e-6 * abs(gs), (fds, gs)
    plan.close()


def test_512_fp32_path_matches_fp64_path_and_reruns(hl):
    kw, qn, d, _ = problem()
    out = {}
    for precision in ("fp64", "fp32"):
        say("512^3", precision)
        plan = hl.Plan(**kw, precision=precision)
        q = torch.from_numpy(qn).to(plan.device)
        qd = torch.from_numpy(d).to(plan.device)
        qs = plan.scalar(1.5)
        a = evaluate(hl, plan, q, qd, qs)
        out[precision] = (a[0], a[1].cpu().numpy(), a[2].cpu().numpy(), a[3])
        if precision == "fp32":
            b = evaluate(hl, plan, q, qd, qs)
            assert a[0] == b[0] and a[3] == b[3]
            assert torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])
        plan.close()
    p64, g64, gd64, gs64 = out["fp64"]
    p32, g32, gd32, gs32 = out["fp32"]
    assert abs(p32 - p64) <= 2e-5 * abs(p64), (p32, p64)
    assert rel_inf(g32, g64) <= 1e-4, rel_inf(g32, g64)
    assert rel_inf(gd32, gd64) <= 1e-4, rel_inf(gd32, gd64)
    assert abs(gs32 - gs64) <= 1e-4 * abs(gs64), (gs32, gs64)


def test_512_leapfrog_is_reversible_fp64(hl):
    kw, qn, d, var = problem()
    say("512^3 fp64 leapfrog there and back")
    plan = hl.Plan(**kw, precision="fp64")
    dev = plan.device
    rng = np.random.default_rng(9)
    sc = np.sqrt(2.0 / np.where(var > 0, var, 1.0)) * (var > 0)
    p0 = sc * rng.standard_normal(var.shape) + 1j * (sc * rng.standard_normal(var.shape))
    q = torch.from_numpy(qn).to(dev)
    qd = torch.from_numpy(d).to(dev)
    qs = plan.scalar(1.5)
    p = torch.from_numpy(p0).to(dev)
    pd = torch.from_numpy(0.3 * rng.standard_normal(len(d))).to(dev)
    ps = plan.scalar(0.2)
    psi = plan.scalar()
    eps = 5e-5
    hl.leapfrog([plan], [eps], [3], [q], [qd], [qs], [p], [pd], [ps], [psi])
    p.neg_(), pd.neg_(), ps.neg_()
    hl.leapfrog([plan], [eps], [3], [q], [qd], [qs], [p], [pd], [ps], [psi])
    torch.cuda.synchronize()
    assert rel_inf(q.cpu().numpy(), qn) <= 1e-10
    assert rel_inf(qd.cpu().numpy(), d) <= 1e-10
    assert abs(qs.item() - 1.5) <= 1e-10
    plan.close()


@pytest.mark.timeout(600)
def test_512_fp32_chain_matches_fp64_chain(hl):
    # Above 256^3 the FP32 chain updates its complex64 state one mode per
    # lane (below, two).  Same start, same Philox stream: the FP32 chain's
    # dH differs from the FP64 chain's by the FP32 fields (1e-3 allowed, as
    # at 256^3) plus the rounding of its stored state, about sqrt(D) 2^-24
    # per update of all D real mode coordinates, seven updates per 3-step
    # trajectory, allowed at four standard deviations; the accept decisions
    # agree unless |ln u + dH| is within that bound.  The retained modes
    # come back as complex64 values.
    from oracle import philox
    kw, qn, d, var = problem()
    n_iter, n_lf, eps, seed = 2, 3, 1.2e-4, 5120
    res = {}
    for precision in ("fp64", "fp32"):
        say("512^3 %s chain" % precision)
        plan = hl.Plan(**kw, precision=precision)
        dev = plan.device
        q = torch.from_numpy(qn).to(dev)
        qd = torch.from_numpy(d).to(dev)
        qs = plan.scalar(1.5)
        dh = torch.zeros(n_iter, dtype=torch.float64, device=dev)
        acc = torch.zeros(n_iter, dtype=torch.int32, device=dev)
        hl.hmc_run([plan], [q], [qd], [qs], n_iter=n_iter, n_leapfrog=n_lf, eps0=eps, seed=seed, dh=[dh],
                   accepted=[acc])
        torch.cuda.synchronize()
        res[precision] = (dh.cpu().numpy(), acc.cpu().numpy(), q.cpu().numpy())
        plan.close()
    dh64, acc64, _ = res["fp64"]
    dh32, acc32, q32 = res["fp32"]
    n_real = 2 * int(np.count_nonzero(var))
    bound = 1e-3 + 4.0 * math.sqrt(7 * n_real) * 2.0 ** -24
    err = float(np.abs(dh32 - dh64).max())
    say("512^3 chains: dH fp64 %s fp32 %s, max difference %.3g (bound %.3g); decisions %s %s"
        % (dh64.tolist(), dh32.tolist(), err, bound, acc64.tolist(), acc32.tolist()))
    assert np.all(np.isfinite(dh64)) and err <= bound
    for it in range(n_iter):
        if acc32[it] != acc64[it]:
            ln_u = math.log(float(philox.uniform53(*philox.draw_words(seed, it, philox.PURPOSE_ACCEPT, [0])[0, :2])))
            assert abs(ln_u + dh64[it]) <= bound, "a decision away from a tie differs"
            break
    keep = var > 0
    r = q32[keep]
    assert np.array_equal(r, r.astype(np.complex64).astype(np.complex128))

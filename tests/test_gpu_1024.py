"""The 1024^3 grid (through the C ABI): the 256^3 benchmark's catalogue on a
grid four times as fine, modes drawn from the prior on the device (each
complex128 mode array is 8 GiB; an FP64 plan holds about 76 GiB).

The oracle's full transforms at this size are out of reach on the host, so
the checks are properties that hold at any size:
  * with no points, Psi is the prior energy E = (1/2) sum_k w_k |q_k|^2 /
    sigma_k^2 over the stored half spectrum (w_k = 2 off the kz = 0 plane,
    whose partners -k are not stored; 1 on it) and the mode gradient is
    2 q_k / sigma_k^2 (eq:prior-k): closed forms, summed here by torch on
    the device (the state has q = 0 on the kz = 0 plane);
  * the gradient against central differences of Psi in sampled modes and
    in s (Psi is quadratic in one mode coordinate, so the central difference
    is exact up to rounding);
  * the FP32 path against the FP64 path, and bit-identical reruns;
  * the reversibility of the leapfrog map.
"""
import math
import sys

import numpy as np
import pytest
import torch

from paper_2203_02369_amd import mocks

pytestmark = pytest.mark.gpu

N = 1024


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
    """(problem kwargs, modes on the device in the library layout, distances,
    sigma_k^2 on the device).  Modes from the prior on kz >= 1 (the kz = 0
    plane left at zero, so the state is Hermitian by construction), Nyquist
    rows excluded."""
    if not _cache:
        m = mocks.paper_scale_256()
        kw = m.problem_kwargs()
        kw["n_grid"] = N
        pk = mocks.PowerSpectrum(omega_m=m.omega_m, h=m.h).table_n2(N, m.box)
        kw["pk_n2"] = pk
        dev = torch.device("cuda", 0)
        say("1024^3: drawing the modes on the device")
        s = torch.arange(N, device=dev, dtype=torch.int64)
        s = torch.where(s < N // 2, s, s - N)
        kz = torch.arange(N // 2, device=dev, dtype=torch.int64)
        n2 = s[:, None, None] ** 2 + s[None, :, None] ** 2 + kz[None, None, :] ** 2
        var = (float(N) ** 6 / m.box ** 3) * torch.from_numpy(pk).to(dev)[n2]
        del n2
        keep = (s.abs()[:, None, None] != N // 2) & (s.abs()[None, :, None] != N // 2) & (kz[None, None, :] > 0)
        var = torch.where(keep, var, torch.zeros((), dtype=torch.float64, device=dev))
        del keep
        gen = torch.Generator(device=dev)
        gen.manual_seed(1024)
        amp = torch.sqrt(0.5 * var)
        q = torch.complex(amp * torch.randn(var.shape, generator=gen, device=dev, dtype=torch.float64),
                          amp * torch.randn(var.shape, generator=gen, device=dev, dtype=torch.float64))
        del amp
        torch.cuda.synchronize()
        _cache.update(kw=kw, q=q, d=m.d_true.copy(), var=var, mock=m)
    return _cache["kw"], _cache["q"], _cache["d"], _cache["var"]


def evaluate(hl, plan, q, qd, qs):
    g, gd, gs, psi = plan.zeros_modes(), plan.zeros_dist(), plan.scalar(), plan.scalar()
    hl.logpost_grad([plan], [q], [qd], [qs], [g], [gd], [gs], [psi])
    torch.cuda.synchronize()
    return psi.item(), g, gd, gs.item()


def rel_inf_dev(a, b):
    return float((a - b).abs().max() / b.abs().max())


def release(plan):
    plan.close()
    torch.cuda.empty_cache()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_1024_prior_only_against_closed_form(hl, precision):
    kw, q, _, var = problem()
    kw0 = dict(kw)
    for k in ("rhat", "mu", "sigma_mu", "cz", "sigma_cz"):
        kw0[k] = kw0[k][:0]
    say("1024^3 %s plan without points" % precision)
    plan = hl.Plan(**kw0, precision=precision)
    assert plan.n_gal == 0
    psi, g, _, _ = evaluate(hl, plan, q, plan.zeros_dist(), plan.scalar(1.5))
    release(plan)
    inv = torch.where(var > 0, 1.0 / torch.where(var > 0, var, torch.ones_like(var)), torch.zeros_like(var))
    e_ref = float(0.5 * 2.0 * ((q.real ** 2 + q.imag ** 2) * inv).sum())   # w = 2: q = 0 on kz = 0
    say("1024^3 %s prior energy: library %.17g, torch %.17g" % (precision, psi, e_ref))
    assert abs(psi - e_ref) <= 1e-12 * abs(e_ref)
    g_ref = 2.0 * q * inv
    err = rel_inf_dev(g, g_ref)
    say("1024^3 %s prior gradient: max error / max entry %.3g" % (precision, err))
    assert err <= 1e-14
    del g, g_ref, inv


@pytest.mark.timeout(600)
def test_1024_gradient_against_central_differences_fp64(hl):
    kw, q, d, var = problem()
    say("1024^3 fp64 plan")
    plan = hl.Plan(**kw, precision="fp64")
    qd = torch.from_numpy(d).to(plan.device)
    qs = plan.scalar(1.5)
    psi, g, gd, gs = evaluate(hl, plan, q, qd, qs)
    assert math.isfinite(psi)
    rng = np.random.default_rng(3)
    picks = []
    while len(picks) < 16:
        ix, iy, iz = (int(v) for v in rng.integers(0, (N, N, N // 2)))
        if var[ix, iy, iz].item() > 0 and (ix, iy, iz) not in [t[:3] for t in picks]:
            picks.append((ix, iy, iz, int(rng.integers(2))))
    gmax = float(g.abs().max())
    an, fd = [], []
    for (ix, iy, iz, comp) in picks:
        h = math.sqrt(var[ix, iy, iz].item())
        v0 = q[ix, iy, iz].item()
        vals = []
        for sgn in (+1, -1):
            q[ix, iy, iz] = v0 + h * sgn * (1.0 if comp == 0 else 1j)
            vals.append(evaluate(hl, plan, q, qd, qs)[0])
        q[ix, iy, iz] = v0
        fd.append((vals[0] - vals[1]) / (2 * h))
        gv = g[ix, iy, iz].item()
        an.append(gv.real if comp == 0 else gv.imag)
    an, fd = np.array(an), np.array(fd)
    say("1024^3 modes: max |fd - grad| / max |grad| =", np.abs(fd - an).max() / gmax)
    assert np.abs(fd - an).max() <= 1e-7 * gmax
    # s: Psi is smooth in s
    h = 1e-4
    vals = [evaluate(hl, plan, q, qd, plan.scalar(1.5 + sgn * h))[0] for sgn in (+1, -1)]
    fds = (vals[0] - vals[1]) / (2 * h)
    say("1024^3 s: fd %.12g grad %.12g" % (fds, gs))
    assert abs(fds - gs) <= 1e-6 * abs(gs), (fds, gs)
    del g
    release(plan)


@pytest.mark.timeout(600)
def test_1024_fp32_path_matches_fp64_path_and_reruns(hl):
    kw, q, d, _ = problem()
    out = {}
    for precision in ("fp64", "fp32"):
        say("1024^3", precision)
        plan = hl.Plan(**kw, precision=precision)
        qd = torch.from_numpy(d).to(plan.device)
        qs = plan.scalar(1.5)
        a = evaluate(hl, plan, q, qd, qs)
        if precision == "fp32":
            b = evaluate(hl, plan, q, qd, qs)
            assert a[0] == b[0] and a[3] == b[3]
            assert torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])
            del b
        out[precision] = a
        release(plan)
    p64, g64, gd64, gs64 = out["fp64"]
    p32, g32, gd32, gs32 = out["fp32"]
    errs = {"psi": abs(p32 - p64) / abs(p64), "modes": rel_inf_dev(g32, g64), "dist": rel_inf_dev(gd32, gd64),
            "s": abs(gs32 - gs64) / abs(gs64)}
    say("1024^3 fp32 against fp64", errs)
    assert errs["psi"] <= 2e-5
    assert max(errs["modes"], errs["dist"], errs["s"]) <= 1e-4


@pytest.mark.timeout(600)
def test_1024_leapfrog_is_reversible_fp64(hl):
    kw, q0, d, var = problem()
    say("1024^3 fp64 leapfrog there and back")
    plan = hl.Plan(**kw, precision="fp64")
    dev = plan.device
    gen = torch.Generator(device=dev)
    gen.manual_seed(9)
    sc = torch.sqrt(2.0 / torch.where(var > 0, var, torch.ones_like(var))) * (var > 0)
    p = torch.complex(sc * torch.randn(var.shape, generator=gen, device=dev, dtype=torch.float64),
                      sc * torch.randn(var.shape, generator=gen, device=dev, dtype=torch.float64))
    del sc
    q = q0.clone()
    qd = torch.from_numpy(d).to(dev)
    qs = plan.scalar(1.5)
    rng = np.random.default_rng(9)
    pd = torch.from_numpy(0.3 * rng.standard_normal(len(d))).to(dev)
    ps = plan.scalar(0.2)
    psi = plan.scalar()
    eps = 5e-5
    hl.leapfrog([plan], [eps], [3], [q], [qd], [qs], [p], [pd], [ps], [psi])
    p.neg_(), pd.neg_(), ps.neg_()
    hl.leapfrog([plan], [eps], [3], [q], [qd], [qs], [p], [pd], [ps], [psi])
    torch.cuda.synchronize()
    eq, ed = rel_inf_dev(q, q0), float(np.abs(qd.cpu().numpy() - d).max() / np.abs(d).max())
    say("1024^3 leapfrog there and back: modes %.3g, distances %.3g" % (eq, ed))
    assert eq <= 1e-10
    assert ed <= 1e-10
    del p, q
    release(plan)

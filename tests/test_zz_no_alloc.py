"""hamlet_shell_stats_static, the allocation-free variant of
hamlet_shell_stats (its partial sums in a static device array), against the
allocating entry point, through the C ABI.

Two calls in a row, the second with a smaller input (a smaller grid and
fewer shells, after the first left its partials in the shared array): each
result must equal hamlet_shell_stats bit for bit (same kernels, same order
of summation; NaN where both are undefined).  A call whose partials exceed
the static array is refused before anything is enqueued.
"""
import ctypes
import sys

import numpy as np
import pytest
import torch

from paper_2203_02369_amd import _capi, mocks

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


def _call(name, plan, a, b, width, n_shells, out):
    fn = getattr(_capi.load(), name)
    return fn(plan.handle, ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr() if b is not None else None),
              float(width), int(n_shells), ctypes.c_void_p(out.data_ptr()))


def _fields(n, dev, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n, n))
    b = 0.5 * a + rng.standard_normal((n, n, n))
    return torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)


def test_static_scratch_equals_the_allocating_call(hl):
    # (grid, box, shell width, shells, with b): the second call is smaller
    cases = [(64, 500.0, 9.3, 45, True), (32, 400.0, 13.7, 20, False)]
    for n, box, width, n_shells, with_b in cases:
        say("static scratch: %d^3, %d shells of %.1f Mpc/h" % (n, n_shells, width))
        m = mocks.make_mock(n, box, 10, 50.0, seed=3)
        plan = hl.Plan.from_mock(m, precision="fp64")
        a, b = _fields(n, plan.device, 100 + n)
        if not with_b:
            b = None
        got = torch.full((n_shells, 6), -7.0, dtype=torch.float64, device=plan.device)
        ref = torch.full((n_shells, 6), -7.0, dtype=torch.float64, device=plan.device)
        torch.cuda.synchronize()
        _capi.check(_call("hamlet_shell_stats_static", plan, a, b, width, n_shells, got))
        _capi.check(_call("hamlet_shell_stats", plan, a, b, width, n_shells, ref))
        torch.cuda.synchronize()
        g, r = got.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(np.isnan(g), np.isnan(r))
        assert np.array_equal(g[~np.isnan(g)], r[~np.isnan(r)])
        assert g[:, 0].sum() > 0 and not np.any(g == -7.0)
        plan.close()


def test_static_scratch_refuses_oversized_partials(hl):
    # 4096 shells of 0.01 Mpc/h on 64^3: one partial per shell and x plane,
    # 4096 x 64 x 24 bytes > 4 MiB
    m = mocks.make_mock(64, 500.0, 10, 50.0, seed=3)
    plan = hl.Plan.from_mock(m, precision="fp64")
    a, b = _fields(64, plan.device, 7)
    out = torch.full((4096, 6), -7.0, dtype=torch.float64, device=plan.device)
    torch.cuda.synchronize()
    st = _call("hamlet_shell_stats_static", plan, a, b, 0.01, 4096, out)
    assert st == -1
    msg = _capi.load().hamlet_last_error().decode()
    say("refused:", msg)
    assert "static scratch" in msg
    torch.cuda.synchronize()
    assert np.all(out.cpu().numpy() == -7.0)   # nothing was enqueued
    plan.close()

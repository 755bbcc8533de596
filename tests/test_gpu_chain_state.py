"""The FP32 path's chain state in complex64, at the boundary of
hamlet_hmc_run (through the C ABI).

A chain of an FP32 plan runs on a complex64 copy of the caller's modes:
the modes are rounded to complex64 on entry, the retained modes of the last
state are written back (widened exactly, so each is a complex64 value), and
the caller's other entries (k = 0, the Nyquist rows, which no kernel reads)
keep their values bit for bit.  A chain of no iterations therefore returns
the rounded start; an FP64 plan's chain returns its start unchanged.  The
mode sum stays FP64: it adds the complex64 states exactly.
"""
import sys

import numpy as np
import pytest
import torch

from paper_2203_02369_amd import mocks

from helpers import start_modes, to_lib_layout

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


def _retained_mask(n):
    s = np.arange(n)
    s = np.where(s < n // 2, s, s - n)
    kz = np.arange(n // 2)
    ok = (s[:, None, None] != -n // 2) & (s[None, :, None] != -n // 2)
    nonzero = (s[:, None, None] != 0) | (s[None, :, None] != 0) | (kz[None, None, :] != 0)
    return ok & nonzero


def _start(m, seed):
    """Library-layout modes with FP64 values off the complex64 grid, and
    arbitrary values on the excluded entries."""
    q = to_lib_layout(start_modes(m)).copy()
    rng = np.random.default_rng(seed)
    q *= 1.0 + 1e-3 * rng.standard_normal(q.shape)          # not representable in FP32
    ex = ~_retained_mask(m.n_grid)
    q[ex] = rng.standard_normal(int(ex.sum())) + 1j * rng.standard_normal(int(ex.sum()))
    return q


def _run(hl, plan, m, q_host, n_iter, seed=11):
    dev = plan.device
    q = torch.from_numpy(q_host.copy()).to(dev)
    qd = torch.from_numpy(m.d_true.copy()).to(dev)
    qs = plan.scalar(1.3)
    msum = plan.zeros_modes()
    hl.hmc_run([plan], [q], [qd], [qs], n_iter=n_iter, n_leapfrog=3, eps0=2e-3, seed=seed, jitter=True,
               mode_sum=[msum])
    torch.cuda.synchronize()
    return q.cpu().numpy(), msum.cpu().numpy()


@pytest.mark.parametrize("n_iter", [0, 3])
def test_fp32_chain_state_is_complex64_at_the_boundary(hl, n_iter):
    m = mocks.make_mock(32, 400.0, 600, 120.0, "inv_r", (0.2, 0.2), seed=44)
    plan = hl.Plan.from_mock(m, precision="fp32")
    q0 = _start(m, 5)
    say("fp32 chain, %d iterations" % n_iter)
    q1, msum = _run(hl, plan, m, q0, n_iter)
    plan.close()
    keep = _retained_mask(m.n_grid)
    # the caller's excluded entries are untouched
    assert np.array_equal(q1[~keep], q0[~keep])
    # every retained mode is a complex64 value, widened exactly
    r = q1[keep]
    assert np.array_equal(r, r.astype(np.complex64).astype(np.complex128))
    if n_iter == 0:
        # no iterations: the rounded start
        assert np.array_equal(r, q0[keep].astype(np.complex64).astype(np.complex128))
        assert not np.any(msum)
    else:
        assert not np.array_equal(r, q0[keep].astype(np.complex64).astype(np.complex128))   # the chain moved
        assert np.all(np.isfinite(msum))


def test_fp64_chain_state_stays_complex128(hl):
    m = mocks.make_mock(16, 200.0, 200, 80.0, "sphere", (0.2, 0.2), seed=36)
    plan = hl.Plan.from_mock(m, precision="fp64")
    q0 = _start(m, 6)
    say("fp64 chain, no iterations")
    q1, _ = _run(hl, plan, m, q0, 0)
    plan.close()
    assert np.array_equal(q1, q0)

"""Python binding of libhamlet: plans and the four entry points.

Argument marshalling only.  Device buffers are torch tensors (PyTorch
provides device memory and streams); every step of the computation runs in
the library's HIP kernels.  Shapes and dtypes:
    modes, gradients, momenta   complex128 (N, N, N/2)   [kx][ky][kz < N/2]
    distances                   float64 (n,)
    s = sigma_NL / 100 km/s     float64 (1,)
    Psi                         float64 (1,)
"""
import ctypes

import numpy as np
import torch

from . import _capi
from ._capi import HmcOpts, c_double_p

PRECISIONS = {"fp64": _capi.HAMLET_FP64, "fp32": _capi.HAMLET_FP32_FP64E}


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _dptr(a):
    return a.ctypes.data_as(c_double_p)


def _stream_handle(stream, device):
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


def _problem(n_grid, box, omega_m, h, f_growth, sigma_v, pk_n2, rhat, mu, sigma_mu, cz, sigma_cz, hist_width,
             precision, sample_distances, sample_sigma_nl, sample_cosmology=False):
    """hamlet_plan_desc and hamlet_catalog of a problem, and the arrays they point into."""
    pk = _f64(pk_n2)
    rh = _f64(rhat).reshape(-1)
    arrays = [_f64(mu), _f64(sigma_mu), _f64(cz), _f64(sigma_cz)]
    n = len(arrays[0])
    if rh.size != 3 * n or any(len(a) != n for a in arrays):
        raise ValueError("catalogue arrays must all have length n (rhat: n x 3)")
    desc = _capi.PlanDesc(n_grid=int(n_grid), precision=PRECISIONS[precision], box=float(box),
                          omega_m=float(omega_m), h=float(h), f_growth=float(f_growth),
                          sigma_v=float(sigma_v), pk_n2=_dptr(pk), n_pk=len(pk),
                          hist_width=float(hist_width), sample_distances=int(bool(sample_distances)),
                          sample_sigma_nl=int(bool(sample_sigma_nl)), sample_cosmology=int(bool(sample_cosmology)))
    cat = _capi.Catalog(n=n, rhat=_dptr(rh), mu=_dptr(arrays[0]), sigma_mu=_dptr(arrays[1]),
                        cz=_dptr(arrays[2]), sigma_cz=_dptr(arrays[3]))
    return desc, cat, n, (pk, rh, arrays)


class Plan:
    """A reconstruction problem resident on one GPU (hamlet_plan_create)."""

    def __init__(self, *, n_grid, box, omega_m, h, f_growth, sigma_v, pk_n2, rhat, mu, sigma_mu, cz, sigma_cz,
                 hist_width=5.0, precision="fp32", sample_distances=True, sample_sigma_nl=True,
                 sample_cosmology=False, stream=None, device=None):
        lib = _capi.load()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.n_grid = int(n_grid)
        self.precision = precision
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        desc, cat, n, _keep = _problem(n_grid, box, omega_m, h, f_growth, sigma_v, pk_n2, rhat, mu, sigma_mu, cz,
                                       sigma_cz, hist_width, precision, sample_distances, sample_sigma_nl,
                                       sample_cosmology)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _capi.check(lib.hamlet_plan_create(ctypes.byref(desc), ctypes.byref(cat),
                                               ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(handle)))
        self._handle = handle
        self.n_gal = n
        self.mode_shape = (self.n_grid, self.n_grid, self.n_grid // 2)
        # small coordinates: s, and u8 = sigma_8 / sigma_8,fid, phi = f / f_fid,
        # eta = h / h_fid when sampled
        self.n_small = 4 if sample_cosmology else 1

    @classmethod
    def from_mock(cls, mock, **kw):
        args = mock.problem_kwargs()
        args.update(kw)
        return cls(**args)

    @property
    def handle(self):
        if self._handle is None:
            raise RuntimeError("plan is closed")
        return self._handle.value

    def close(self):
        if getattr(self, "_handle", None) is not None and self._handle.value:
            _capi.check(_capi.load().hamlet_plan_destroy(self._handle))
        self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- buffers ---------------------------------------------------------------
    def zeros_modes(self):
        return torch.zeros(self.mode_shape, dtype=torch.complex128, device=self.device)

    def zeros_dist(self):
        return torch.zeros(max(self.n_gal, 0), dtype=torch.float64, device=self.device)

    def scalar(self, value=0.0):
        return torch.full((1,), float(value), dtype=torch.float64, device=self.device)

    def small(self, s=0.0, u8=1.0, phi=1.0, eta=1.0):
        """The small coordinates of a state (or momenta, gradient): (s,) or
        (s, u8, phi, eta) when the plan samples the cosmological parameters."""
        vals = [s, u8, phi, eta][: self.n_small]
        return torch.tensor(vals, dtype=torch.float64, device=self.device)


def footprint_bytes(n_grid, n_gal, precision="fp32", pk_len=None):
    """Device bytes a plan of this size would own (hamlet_plan_footprint_bytes)."""
    lib = _capi.load()
    npk = 3 * (n_grid // 2) ** 2 + 1 if pk_len is None else pk_len
    pk = np.ones(npk)
    desc = _capi.PlanDesc(n_grid=int(n_grid), precision=PRECISIONS[precision], box=500.0, omega_m=0.3, h=0.7,
                          f_growth=0.5, sigma_v=300.0, pk_n2=_dptr(pk), n_pk=npk, hist_width=5.0,
                          sample_distances=1, sample_sigma_nl=1)
    out = ctypes.c_size_t()
    _capi.check(lib.hamlet_plan_footprint_bytes(ctypes.byref(desc), int(n_gal), ctypes.byref(out)))
    return out.value


# -- checks and pointer arrays -------------------------------------------------

def _check(t, plan, kind, name):
    if t is None:
        return 0
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("%s must be a CUDA tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if kind == "modes":
        if t.dtype != torch.complex128 or tuple(t.shape) != plan.mode_shape:
            raise ValueError("%s must be complex128 %s" % (name, plan.mode_shape))
    elif kind == "dist":
        if t.dtype != torch.float64 or t.numel() != plan.n_gal:
            raise ValueError("%s must be float64 (%d,)" % (name, plan.n_gal))
    elif kind == "scalar":
        if t.dtype != torch.float64 or t.numel() < 1:
            raise ValueError("%s must be float64 (1,)" % name)
    elif kind == "small":
        if t.dtype != torch.float64 or t.numel() < plan.n_small:
            raise ValueError("%s must be float64 (%d,)" % (name, plan.n_small))
    elif kind == "iter_f64":
        if t.dtype != torch.float64:
            raise ValueError("%s must be float64" % name)
    elif kind == "iter_i32":
        if t.dtype != torch.int32:
            raise ValueError("%s must be int32" % name)
    return t.data_ptr()


def _vp(addrs):
    return (ctypes.c_void_p * len(addrs))(*[a or None for a in addrs])


def _dpp(addrs):
    arr = (c_double_p * len(addrs))()
    for i, a in enumerate(addrs):
        arr[i] = ctypes.cast(ctypes.c_void_p(a), c_double_p) if a else c_double_p()
    return arr


def _ipp(addrs):
    arr = (_capi.c_int32_p * len(addrs))()
    for i, a in enumerate(addrs):
        arr[i] = ctypes.cast(ctypes.c_void_p(a), _capi.c_int32_p) if a else _capi.c_int32_p()
    return arr


def _plans(plans):
    plans = list(plans)
    return plans, _vp([p.handle for p in plans])


def logpost_grad(plans, q_modes, q_dist, q_snl, g_modes, g_dist, g_snl, psi, per_entry=False):
    """Psi and its gradient for a batch of plans (hamlet_logpost_grad, or
    hamlet_logpost_grad_entries with per_entry=True)."""
    plans, hp = _plans(plans)
    args = []
    for kind, name, ts in (("modes", "q_modes", q_modes), ("dist", "q_dist", q_dist), ("small", "q_snl", q_snl),
                           ("modes", "g_modes", g_modes), ("dist", "g_dist", g_dist), ("small", "g_snl", g_snl),
                           ("scalar", "psi", psi)):
        args.append([_check(t, p, kind, name) for t, p in zip(ts, plans)])
    lib = _capi.load()
    fn = lib.hamlet_logpost_grad_entries if per_entry else lib.hamlet_logpost_grad
    _capi.check(fn(hp, len(plans), _vp(args[0]), _dpp(args[1]), _dpp(args[2]),
                   _vp(args[3]), _dpp(args[4]), _dpp(args[5]), _dpp(args[6])))


def _ptr(addr):
    return ctypes.cast(ctypes.c_void_p(addr), c_double_p) if addr else c_double_p()


def flat_size(plan):
    """Length 2m + n + 1 of the plan's flat parameter vector (hamlet_flat_size)."""
    out = ctypes.c_int64()
    _capi.check(_capi.load().hamlet_flat_size(plan.handle, ctypes.byref(out)))
    return out.value


def pack_flat(plan, modes, dist, snl, flat=None):
    """The paper's flat vector (Re, Im of the independent modes, distances, s)
    of a state or a gradient, on the plan's stream (hamlet_pack_flat)."""
    if flat is None:
        flat = torch.empty(flat_size(plan), dtype=torch.float64, device=plan.device)
    elif flat.dtype != torch.float64 or flat.numel() != flat_size(plan) or not flat.is_contiguous():
        raise ValueError("flat must be contiguous float64 (%d,)" % flat_size(plan))
    m, d, s = _check(modes, plan, "modes", "modes"), _check(dist, plan, "dist", "dist"), _check(snl, plan, "small", "snl")
    _capi.check(_capi.load().hamlet_pack_flat(plan.handle, ctypes.c_void_p(m), _ptr(d), _ptr(s),
                                              _ptr(_check(flat, plan, "iter_f64", "flat"))))
    return flat


def unpack_flat(plan, flat, modes, dist, snl):
    """Writes the state (modes with mirror entries and excluded modes filled,
    distances, s) of a flat vector, on the plan's stream (hamlet_unpack_flat)."""
    if flat.dtype != torch.float64 or flat.numel() != flat_size(plan) or not flat.is_contiguous():
        raise ValueError("flat must be contiguous float64 (%d,)" % flat_size(plan))
    m, d, s = _check(modes, plan, "modes", "modes"), _check(dist, plan, "dist", "dist"), _check(snl, plan, "small", "snl")
    _capi.check(_capi.load().hamlet_unpack_flat(plan.handle, _ptr(_check(flat, plan, "iter_f64", "flat")),
                                                ctypes.c_void_p(m), _ptr(d), _ptr(s)))


def velocity_field(plan, modes, out=None):
    """The velocity field v_c (km/s) of a state's modes on every grid node, on
    the plan's stream (hamlet_velocity_field): a device tensor (3, N, N, N) of
    the plan's real type."""
    n = plan.n_grid
    dt = torch.float64 if plan.precision == "fp64" else torch.float32
    if out is None:
        out = torch.empty((3, n, n, n), dtype=dt, device=plan.device)
    elif out.dtype != dt or tuple(out.shape) != (3, n, n, n) or not out.is_contiguous():
        raise ValueError("out must be contiguous %s (3, %d, %d, %d)" % (dt, n, n, n))
    m = _check(modes, plan, "modes", "modes")
    _capi.check(_capi.load().hamlet_velocity_field(plan.handle, ctypes.c_void_p(m), ctypes.c_void_p(out.data_ptr())))
    return out


def density_field(plan, modes, out=None):
    """The density contrast of a state's modes on every grid node, on the
    plan's stream (hamlet_density_field): a device tensor (N, N, N) of the
    plan's real type."""
    n = plan.n_grid
    dt = torch.float64 if plan.precision == "fp64" else torch.float32
    if out is None:
        out = torch.empty((n, n, n), dtype=dt, device=plan.device)
    elif out.dtype != dt or tuple(out.shape) != (n, n, n) or not out.is_contiguous():
        raise ValueError("out must be contiguous %s (%d, %d, %d)" % (dt, n, n, n))
    m = _check(modes, plan, "modes", "modes")
    _capi.check(_capi.load().hamlet_density_field(plan.handle, ctypes.c_void_p(m), ctypes.c_void_p(out.data_ptr())))
    return out


def field_stats_accumulate(plan, modes, acc=None):
    """Add a state's density contrast and radial velocity on every node, and
    their squares, to running sums on the plan's stream
    (hamlet_field_stats_accumulate): acc is a float64 device tensor
    (4, N, N, N) = [sum delta, sum delta^2, sum v_r, sum v_r^2], zeros when
    None; returned."""
    n = plan.n_grid
    if acc is None:
        acc = torch.zeros((4, n, n, n), dtype=torch.float64, device=plan.device)
    elif acc.dtype != torch.float64 or tuple(acc.shape) != (4, n, n, n) or not acc.is_contiguous():
        raise ValueError("acc must be contiguous float64 (4, %d, %d, %d)" % (n, n, n))
    elif acc.device != plan.device:
        raise ValueError("acc must be on %s" % plan.device)
    m = _check(modes, plan, "modes", "modes")
    _capi.check(_capi.load().hamlet_field_stats_accumulate(plan.handle, ctypes.c_void_p(m),
                                                           ctypes.c_void_p(acc.data_ptr())))
    return acc


def shell_stats(plan, a, b, width, n_shells, out=None, static_scratch=False):
    """Statistics of float64 grids a and b (N, N, N) in spherical shells of
    the given width (Mpc/h) about the observer, on the plan's stream
    (hamlet_shell_stats): a float64 device tensor (n_shells, 6) of (count,
    mean a, scatter a, mean b, scatter b, correlation) per shell; b may be
    None.  static_scratch=True calls hamlet_shell_stats_static, which
    allocates nothing (pass `out` as well to keep the call free of torch
    allocations)."""
    n = plan.n_grid
    for name, g in (("a", a), ("b", b)):
        if g is None and name == "b":
            continue
        if (not isinstance(g, torch.Tensor) or g.dtype != torch.float64 or tuple(g.shape) != (n, n, n)
                or not g.is_contiguous() or g.device != plan.device):
            raise ValueError("%s must be a contiguous float64 (%d, %d, %d) tensor on %s" % (name, n, n, n, plan.device))
    n_shells = int(n_shells)
    if out is None:
        out = torch.empty((max(n_shells, 0), 6), dtype=torch.float64, device=plan.device)
    elif out.dtype != torch.float64 or out.numel() != 6 * n_shells or not out.is_contiguous() or out.device != plan.device:
        raise ValueError("out must be contiguous float64 (%d, 6) on %s" % (n_shells, plan.device))
    lib = _capi.load()
    fn = lib.hamlet_shell_stats_static if static_scratch else lib.hamlet_shell_stats
    _capi.check(fn(plan.handle, ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr() if b is not None else None),
                   float(width), n_shells, ctypes.c_void_p(out.data_ptr())))
    return out


def sphere_moments(plan, modes, radii, out=None):
    """Monopole and dipole of the velocity field in spheres of the given radii
    (Mpc/h) about the observer, on the plan's stream (hamlet_sphere_moments):
    a float64 device tensor (len(radii), 4) of (M, Dx, Dy, Dz) per radius."""
    r = [float(x) for x in radii]
    if out is None:
        out = torch.empty((len(r), 4), dtype=torch.float64, device=plan.device)
    elif out.dtype != torch.float64 or out.numel() != 4 * len(r) or not out.is_contiguous():
        raise ValueError("out must be contiguous float64 (%d, 4)" % len(r))
    m = _check(modes, plan, "modes", "modes")
    rr = (ctypes.c_double * max(len(r), 1))(*r)
    _capi.check(_capi.load().hamlet_sphere_moments(plan.handle, ctypes.c_void_p(m), rr, len(r),
                                                   _ptr(_check(out, plan, "iter_f64", "out"))))
    return out


def leapfrog(plans, eps, n_steps, q_modes, q_dist, q_snl, p_modes, p_dist, p_snl, psi):
    """n_steps kick-drift-kick steps in place (hamlet_leapfrog)."""
    plans, hp = _plans(plans)
    args = []
    for kind, name, ts in (("modes", "q_modes", q_modes), ("dist", "q_dist", q_dist), ("small", "q_snl", q_snl),
                           ("modes", "p_modes", p_modes), ("dist", "p_dist", p_dist), ("small", "p_snl", p_snl),
                           ("scalar", "psi", psi)):
        args.append([_check(t, p, kind, name) for t, p in zip(ts, plans)])
    e = (ctypes.c_double * len(plans))(*[float(x) for x in eps])
    s = (ctypes.c_int32 * len(plans))(*[int(x) for x in n_steps])
    lib = _capi.load()
    _capi.check(lib.hamlet_leapfrog(hp, len(plans), e, s, _vp(args[0]), _dpp(args[1]), _dpp(args[2]),
                                    _vp(args[3]), _dpp(args[4]), _dpp(args[5]), _dpp(args[6])))


def hmc_run(plans, q_modes, q_dist, q_snl, *, n_iter, n_leapfrog, eps0, seed, warmup=0, jitter=False,
            target_accept=0.65, mode_sum=None, dh=None, accepted=None, want_eps=True, seeds=None, resume=False):
    """Runs the HMC chains (hamlet_hmc_run); returns the post-warm-up steps.

    Chain j's key is seeds[j] when given, else seed + j.  resume=True
    continues each plan's chain from its previous run (then dh/accepted are
    indexed by the chain's own iteration count).  An FP32 plan's chain runs
    on complex64 modes: its retained modes come back rounded to complex64,
    its other entries as given."""
    plans, hp = _plans(plans)
    nplan = len(plans)
    qm = [_check(t, p, "modes", "q_modes") for t, p in zip(q_modes, plans)]
    qd = [_check(t, p, "dist", "q_dist") for t, p in zip(q_dist, plans)]
    qs = [_check(t, p, "small", "q_snl") for t, p in zip(q_snl, plans)]
    ms = [_check(t, p, "modes", "mode_sum") for t, p in zip(mode_sum, plans)] if mode_sum else None
    dd = [_check(t, p, "iter_f64", "dh") for t, p in zip(dh, plans)] if dh else None
    aa = [_check(t, p, "iter_i32", "accepted") for t, p in zip(accepted, plans)] if accepted else None
    for lst, what in ((dh, "dh"), (accepted, "accepted")):
        if lst:
            for t in lst:
                if t.numel() < n_iter:
                    raise ValueError("%s needs n_iter entries" % what)
    opts = HmcOpts(n_iter=int(n_iter), n_leapfrog=int(n_leapfrog), warmup=int(warmup), jitter_eps=int(bool(jitter)),
                   eps0=float(eps0), target_accept=float(target_accept), seed=int(seed) & 0xFFFFFFFFFFFFFFFF,
                   resume=int(bool(resume)))
    if seeds is not None:
        if len(seeds) != nplan:
            raise ValueError("seeds needs one key per plan")
        keys = (ctypes.c_uint64 * nplan)(*[int(k) & 0xFFFFFFFFFFFFFFFF for k in seeds])
        opts.seeds = ctypes.cast(keys, ctypes.POINTER(ctypes.c_uint64))
    eps_out = (ctypes.c_double * nplan)() if want_eps else None
    lib = _capi.load()
    _capi.check(lib.hamlet_hmc_run(hp, nplan, ctypes.byref(opts), _vp(qm), _dpp(qd), _dpp(qs),
                                   _vp(ms) if ms else None, _dpp(dd) if dd else None,
                                   _ipp(aa) if aa else None,
                                   ctypes.cast(eps_out, c_double_p) if want_eps else None))
    return list(eps_out) if want_eps else None


def nuts_run(plans, q_modes, q_dist, q_snl, *, n_iter, eps0, seed, warmup=0, max_depth=10, target_accept=0.65,
             mode_sum=None, seeds=None):
    """Runs the No-U-Turn chains (hamlet_nuts_run); the state tensors are
    updated in place.  Returns, per plan, a dict of numpy arrays over the
    iterations: depth (doublings), leaves (leapfrog steps), where (n_iter, 2:
    doubling and position of the leaf moved to, (-1, 0) if none), alpha (the
    acceptance statistic), and eps, the step after warm-up."""
    plans, hp = _plans(plans)
    nplan = len(plans)
    n_iter = int(n_iter)
    qm = [_check(t, p, "modes", "q_modes") for t, p in zip(q_modes, plans)]
    qd = [_check(t, p, "dist", "q_dist") for t, p in zip(q_dist, plans)]
    qs = [_check(t, p, "small", "q_snl") for t, p in zip(q_snl, plans)]
    ms = [_check(t, p, "modes", "mode_sum") for t, p in zip(mode_sum, plans)] if mode_sum else None
    opts = _capi.NutsOpts(n_iter=n_iter, warmup=int(warmup), max_depth=int(max_depth), reserved=0, eps0=float(eps0),
                          target_accept=float(target_accept), seed=int(seed) & 0xFFFFFFFFFFFFFFFF)
    if seeds is not None:
        if len(seeds) != nplan:
            raise ValueError("seeds needs one key per plan")
        keys = (ctypes.c_uint64 * nplan)(*[int(k) & 0xFFFFFFFFFFFFFFFF for k in seeds])
        opts.seeds = ctypes.cast(keys, ctypes.POINTER(ctypes.c_uint64))
    outs = [dict(depth=np.zeros(max(n_iter, 1), dtype=np.int32), leaves=np.zeros(max(n_iter, 1), dtype=np.int32),
                 where=np.zeros((max(n_iter, 1), 2), dtype=np.int32), alpha=np.zeros(max(n_iter, 1)))
            for _ in plans]

    def host_ptrs(key, ctype):
        arr = (ctypes.POINTER(ctype) * nplan)()
        for i, o in enumerate(outs):
            arr[i] = o[key].ctypes.data_as(ctypes.POINTER(ctype))
        return arr
    eps_out = (ctypes.c_double * nplan)()
    _capi.check(_capi.load().hamlet_nuts_run(hp, nplan, ctypes.byref(opts), _vp(qm), _dpp(qd), _dpp(qs),
                                             _vp(ms) if ms else None, host_ptrs("depth", ctypes.c_int32),
                                             host_ptrs("leaves", ctypes.c_int32), host_ptrs("where", ctypes.c_int32),
                                             host_ptrs("alpha", ctypes.c_double),
                                             ctypes.cast(eps_out, c_double_p)))
    for i, o in enumerate(outs):
        for k in ("depth", "leaves", "where", "alpha"):
            o[k] = o[k][:n_iter]
        o["eps"] = eps_out[i]
    return outs


# -- serving ---------------------------------------------------------------------

SERVER_STATES = {-1: "failed", 0: "queued", 1: "running", 2: "finished"}


class Server:
    """Continuous batching of independent reconstruction jobs on one GPU
    (hamlet_server_*): submit() queues a job, tick() admits what fits the
    device budget and advances every running job by one leapfrog step,
    take() returns a finished job's results as numpy arrays."""

    def __init__(self, hbm_budget, *, max_running=0, ticks_ahead=2, stream=None, device=None):
        lib = _capi.load()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        desc = _capi.ServerDesc(hbm_budget=int(hbm_budget), max_running=int(max_running),
                                ticks_ahead=int(ticks_ahead))
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _capi.check(lib.hamlet_server_create(ctypes.byref(desc), ctypes.c_void_p(self.stream.cuda_stream),
                                                 ctypes.byref(handle)))
        self._handle = handle
        self._jobs = {}

    @property
    def handle(self):
        if self._handle is None:
            raise RuntimeError("server is closed")
        return self._handle.value

    def submit(self, *, n_iter, n_leapfrog, eps0, seed, warmup=0, jitter=False, target_accept=0.65,
               q_modes=None, q_dist=None, q_snl=1.0, precision="fp32", hist_width=5.0, sample_distances=True,
               sample_sigma_nl=True, sample_cosmology=False, **problem):
        """Queue a job; `problem` holds the Plan keywords (n_grid, box, ...,
        sigma_cz).  q_modes: complex (N, N, N/2) or None (zero field); q_dist:
        (n,) or None (redshift distances)."""
        desc, cat, n, _keep = _problem(hist_width=hist_width, precision=precision,
                                       sample_distances=sample_distances, sample_sigma_nl=sample_sigma_nl,
                                       sample_cosmology=sample_cosmology, **problem)
        ng = int(problem["n_grid"])
        opts = HmcOpts(n_iter=int(n_iter), n_leapfrog=int(n_leapfrog), warmup=int(warmup),
                       jitter_eps=int(bool(jitter)), eps0=float(eps0), target_accept=float(target_accept),
                       seed=int(seed) & 0xFFFFFFFFFFFFFFFF)
        qm = None
        if q_modes is not None:
            qm = np.ascontiguousarray(np.asarray(q_modes, dtype=np.complex128))
            if qm.shape != (ng, ng, ng // 2):
                raise ValueError("q_modes must be complex (N, N, N/2)")
        qd = None
        if q_dist is not None:
            qd = _f64(q_dist)
            if qd.shape != (n,):
                raise ValueError("q_dist must have n entries")
        job = ctypes.c_int64()
        _capi.check(_capi.load().hamlet_server_submit(
            self.handle, ctypes.byref(desc), ctypes.byref(cat), ctypes.byref(opts),
            qm.ctypes.data_as(c_double_p) if qm is not None else None,
            _dptr(qd) if qd is not None else None, float(q_snl), ctypes.byref(job)))
        self._jobs[job.value] = (ng, n, int(n_iter))
        return job.value

    def tick(self):
        st = _capi.ServerStats()
        _capi.check(_capi.load().hamlet_server_tick(self.handle, ctypes.byref(st)))
        return {"queued": st.queued, "running": st.running, "finished": st.finished, "ticks": st.ticks,
                "bytes_in_use": st.bytes_in_use}

    def state(self, job):
        out = ctypes.c_int32()
        _capi.check(_capi.load().hamlet_server_job_state(self.handle, int(job), ctypes.byref(out)))
        return SERVER_STATES[out.value]

    TAKE_ALL = ("mode_sum", "q_modes", "q_dist", "q_snl", "dh", "accepted", "eps")

    def take(self, job, outputs=TAKE_ALL):
        """Results of a finished job (the listed ones) as numpy arrays; releases the job."""
        ng, n, n_iter = self._jobs.pop(job)
        shapes = {"mode_sum": ((ng, ng, ng // 2), np.complex128), "q_modes": ((ng, ng, ng // 2), np.complex128),
                  "q_dist": ((n,), np.float64), "q_snl": ((1,), np.float64), "dh": ((n_iter,), np.float64),
                  "accepted": ((n_iter,), np.int32), "eps": ((1,), np.float64)}
        res = {k: np.zeros(*shapes[k]) for k in outputs}

        def ptr(k, typ=c_double_p):
            return res[k].ctypes.data_as(typ) if k in res else None
        _capi.check(_capi.load().hamlet_server_take(
            self.handle, int(job), ptr("mode_sum"), ptr("q_modes"), ptr("q_dist"), ptr("q_snl"), ptr("dh"),
            ptr("accepted", _capi.c_int32_p), ptr("eps")))
        for k in ("q_snl", "eps"):
            if k in res:
                res[k] = float(res[k][0])
        return res

    def close(self):
        if getattr(self, "_handle", None) is not None and self._handle.value:
            _capi.check(_capi.load().hamlet_server_destroy(self._handle))
        self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# -- measurement ---------------------------------------------------------------

def schedule(n_grid, precision="fp32"):
    """The kernel schedule the loaded library uses for a grid size and
    precision (hamlet_schedule_get), as a dict; the radix plan as its
    radices ("16x16")."""
    out = _capi.Schedule()
    prec = 0 if precision == "fp64" else 1
    _capi.check(_capi.load().hamlet_schedule_get(prec, int(n_grid), ctypes.byref(out)))
    res = {name: int(getattr(out, name)) for name, _ in _capi.Schedule._fields_ if name != "radix"}
    res["radix"] = "x".join(str(r) for r in out.radix if r)
    return res


PROFILE_KERNELS = {"bin": 0, "inv_x": 1, "inv_y": 2, "inv_z_gather": 3, "like": 4, "fwd_z_scatter": 5,
                   "fwd_y": 6, "fwd_x": 7}


class KernelTimer:
    """HIP-event timing of one kernel kind of a plan (hamlet_profile_*)."""

    def __init__(self, plan, kind):
        self.plan = plan
        self.kind = int(kind)

    def start(self):
        _capi.check(_capi.load().hamlet_profile_start(ctypes.c_void_p(self.plan.handle), self.kind))

    def stop(self):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _capi.check(_capi.load().hamlet_profile_stop(ctypes.c_void_p(self.plan.handle), ctypes.byref(ms),
                                                     ctypes.byref(n)))
        return ms.value, n.value

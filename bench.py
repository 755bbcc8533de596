"""Throughput of the HAMLET hot path on one MI355X.

A step is one HMC iteration of the paper-scale problem (256^3 grid, box
500 Mpc/h, 30 000 points with number density ~ 1/r to 250 Mpc/h and a zone
of avoidance |b| < 10 deg, lognormal distance errors 15-25 %): momentum
refresh, 20 leapfrog steps (each one log-posterior-and-gradient evaluation:
binning, three inverse FFTs with the CIC gather, likelihood, CIC scatter,
three forward FFTs, adjoint multiply), kinetic energies and the
Metropolis-Hastings test, all on the device.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  value = gradient evaluations per second of the
FP32-field / FP64-Hamiltonian path; the plain FP64 path is timed beside it
with the same step size and seed ("fp64_path"), and the FP64 oracle is
timed on the host cores ("cpu_baseline").

    python bench.py --workload batched

16 independent chains of uneven size (grids 64^3, 128^3, 256^3 in turn,
2000 to 30 000 points) advanced together: chains of one grid size share
every kernel launch.  value = gradient evaluations per second summed over
the chains; the same chains advanced one at a time are timed beside it.

    python bench.py --workload served [--jobs J] [--rate R]

A seeded Poisson stream of J reconstruction requests at R per second (grid
64^3, 128^3 or 256^3, 1000 to 30 000 points, 100 HMC iterations of 20
leapfrog steps each) served by continuous batching with admission by device
footprint.  value = gradient evaluations per second over the run; p50 and
p99 job latency (arrival to results) are reported beside those of the same
stream served by the plain FP64 path one job at a time.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM traffic of k_x_pass<float, 256> per launch in a chain (complex64 chain
# state), from two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE) of this
# script at 256^3 with 30 000 points, each scaled by what the counter reads
# for a plain 1 GiB device copy (--copy-calibration: FETCH_SIZE x 1.9999,
# WRITE_SIZE x 1.0000).  Bytes read and written per launch for the
# plain-gradient, first, middle and last variants.  Valid only for the kernel
# sources and the 256^3 FP32 schedule they were taken on (hash below).
X_TRAFFIC_SOURCES_SHA1 = "292591d7715e997f34387e643bd6acda08ee0ac6"
X_TRAFFIC = {"grad": (268546554, 67108864), "first": (201956190, 402810088),
             "mid": (335814340, 268505895), "last": (335732854, 134283763)}

# below this acceptance rate a chain hardly samples: the comparison of the two
# paths "at equal acceptance" would be void, and the run reports failure
MIN_ACCEPTANCE = 0.3


def kernel_sources_sha1(sched):
    """Hash of the kernel sources and of the launch schedule the library runs
    for the grid (threads, tiles, radix plan): together they fix the code of
    that grid's kernels, whatever the schedules of other grids."""
    import hashlib
    import json
    h = hashlib.sha1()
    for f in ("passes.hpp", "fft.hpp", "common.hpp", "workspace.hpp", "random.hpp", "schedule.hpp"):
        with open(os.path.join(ROOT, "paper_2203_02369_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    h.update(json.dumps(sched, sort_keys=True).encode())
    return h.hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5,
                    help="untimed HMC iterations at the adapted step, after the adaptation")
    ap.add_argument("--adapt", type=int, default=50,
                    help="untimed dual-averaging iterations that set the step (target acceptance 0.65)")
    ap.add_argument("--leapfrog", type=int, default=20)
    ap.add_argument("--fp64-steps", type=int, default=20)
    ap.add_argument("--n-grid", type=int, default=256)
    ap.add_argument("--n-gal", type=int, default=30000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="oracle processes of the all-cores CPU leg (0: the usable cores, at most 16)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--nuts-iters", type=int, default=4, help="No-U-Turn iterations timed on the same chain (0: none)")
    ap.add_argument("--nuts-depth", type=int, default=6, help="most doublings per No-U-Turn iteration")
    ap.add_argument("--served-jobs", type=int, default=16, help="paper workload: requests of the short served stream")
    ap.add_argument("--workload", choices=("paper", "batched", "served"), default="paper")
    ap.add_argument("--jobs", type=int, default=64, help="served: number of requests")
    # about 0.7 x the service capacity of the shared launches: the 16-chain
    # workload sustains ~5800 grad evals/s, ~2.9 requests of 100 x 20 steps/s
    ap.add_argument("--rate", type=float, default=2.0, help="served: requests per second")
    ap.add_argument("--max-running", type=int, default=0,
                    help="served: most jobs advanced together (0: as many as the device memory budget admits)")
    ap.add_argument("--iters", type=int, default=100, help="served: HMC iterations per request")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one plain 1 GiB device-to-device copy (reference for traffic counters)")
    ap.add_argument("--oracle-worker", default=None, help=argparse.SUPPRESS)
    return ap.parse_args()


def touched_pencil_fraction(mock, d):
    """Fraction of the real-space pencils (x, y) that some point's CIC
    stencil reaches (columns x - ox, y - oy, ox, oy in {0, 1}, hold a point);
    the y and z passes move only their rows."""
    import numpy as np
    n = mock.n_grid
    pos = np.mod(0.5 * mock.box + d[:, None] * mock.rhat, mock.box)
    cell = np.floor(pos[:, :2] * (n / mock.box)).astype(np.int64) % n
    occ = np.zeros((n, n), dtype=bool)
    occ[cell[:, 0], cell[:, 1]] = True
    reach = occ | np.roll(occ, 1, axis=0) | np.roll(occ, 1, axis=1) | np.roll(occ, (1, 1), axis=(0, 1))
    return float(reach.mean())


# ---------------------------------------------------------------------------
# CPU baseline: the oracle on the host cores
# ---------------------------------------------------------------------------
PROBLEM_KEYS = ("n_grid", "box", "omega_m", "h", "f_growth", "sigma_v", "pk_n2", "rhat", "mu", "sigma_mu", "cz",
                "sigma_cz")


def host_info():
    """CPU model and the cores this process may run on (at most 16 are used:
    the share of the host that comes with one GPU)."""
    model_name = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model_name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return model_name, usable


def oracle_worker(path):
    """One oracle evaluation in a child process (all-cores leg): loads the
    problem and the state, reports ready, waits for the go line on stdin,
    evaluates, reports its start and end times."""
    import numpy as np

    from oracle import model
    z = np.load(path)
    kw = {k: (z[k] if z[k].ndim else z[k].item()) for k in PROBLEM_KEYS}
    kw["n_grid"] = int(kw["n_grid"])
    prob = model.Problem(**kw)
    dh, d, s = z["dhat"], z["d"], float(z["s"])
    print("ready", flush=True)
    sys.stdin.readline()
    t0 = time.time()
    model.logpost_grad(prob, dh, d, s)
    print("done %.6f %.6f" % (t0, time.time()), flush=True)


def cpu_all_cores(mock, dh, d, s, workers):
    """Oracle evaluations of the same state in `workers` processes at once:
    grad evals/s of the whole host (each process one thread)."""
    import subprocess
    import tempfile

    import numpy as np
    path = os.path.join(tempfile.gettempdir(), "hamlet_oracle_state_%d.npz" % os.getpid())
    kw = mock.problem_kwargs()
    np.savez(path, dhat=dh, d=d, s=s, **{k: np.asarray(kw[k]) for k in PROBLEM_KEYS})
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    procs = []
    try:
        for _ in range(workers):
            procs.append(subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-worker", path],
                                          stdin=subprocess.PIPE, stdout=subprocess.PIPE, env=env, text=True))
        for p in procs:
            if not p.stdout.readline().startswith("ready"):
                raise RuntimeError("oracle worker failed to start")
        t_go = time.time()
        for p in procs:
            p.stdin.write("go\n")
            p.stdin.flush()
        ends = []
        for p in procs:
            line = p.stdout.readline().split()
            if not line or line[0] != "done":
                raise RuntimeError("oracle worker failed")
            ends.append(float(line[2]))
        for p in procs:
            p.wait(timeout=120)
    finally:
        for p in procs:
            if p.poll() is None:
                p.kill()
                p.wait()
        if os.path.exists(path):
            os.remove(path)
    wall = max(ends) - t_go
    return workers / wall, wall


def cpu_baseline(args, mock, dh, d, s):
    """The oracle as it stands on the host: one evaluation of the timed
    state on one thread (its result also gives the GPU paths' errors), the
    same on every usable core at once, config 1's whole chain (32^3, 1000
    points, 20 iterations of 10 leapfrog steps) and five config 2 gradients
    (128^3, 10 000 points)."""
    from oracle import hmc, model
    from paper_2203_02369_amd import mocks
    cpu_name, usable = host_info()
    prob = model.Problem(**mock.problem_kwargs())
    log("cpu oracle: one evaluation at %d^3 on one thread" % mock.n_grid)
    tc = time.perf_counter()
    ref = model.logpost_grad(prob, dh, d, s)
    t1 = time.perf_counter() - tc
    log("cpu oracle: %.1f s per gradient (one thread)" % t1)
    workers = args.cpu_workers if args.cpu_workers > 0 else min(16, usable)
    all_cores = None
    if workers > 1:
        log("cpu oracle: %d evaluations at once in %d processes" % (workers, workers))
        try:
            v_all, wall = cpu_all_cores(mock, dh, d, s, workers)
            all_cores = {"value": round(v_all, 5), "cores": workers, "wall_s": round(wall, 2)}
            log("cpu oracle, all cores: %.4f grad evals/s (%d in %.1f s)" % (v_all, workers, wall))
        except Exception as e:   # reported, not fatal: the single-thread figure stands
            all_cores = {"error": str(e)}
            log("cpu oracle, all cores: failed: %s" % e)
    # config 1: the plain FP64 chain of the smallest configuration, whole
    m1 = mocks.plain_fp64_32()
    p1 = model.Problem(**m1.problem_kwargs())
    q1 = hmc.State(hmc.symmetrise(32, m1.dhat_true), m1.d_true.copy(), 1.5)
    tc = time.perf_counter()
    hmc.hmc_run(p1, q1, 20, 10, 0.02, mocks.config_seed(1) + 3, jitter=True)
    t_c1 = time.perf_counter() - tc
    log("cpu oracle, config 1 chain (32^3, 20 x 10): %.1f s" % t_c1)
    # config 2: five gradients at 128^3, extrapolated to its 200 x 50 chain
    m2 = mocks.single_chain_128()
    p2 = model.Problem(**m2.problem_kwargs())
    dh2 = hmc.symmetrise(128, m2.dhat_true)
    tc = time.perf_counter()
    for _ in range(5):
        model.logpost_grad(p2, dh2, m2.d_true, 1.5)
    t_c2 = (time.perf_counter() - tc) / 5
    log("cpu oracle, config 2 (128^3): %.2f s per gradient" % t_c2)
    single = {"value": round(1.0 / t1, 5), "cores": 1, "s_per_grad": round(t1, 2)}
    use = all_cores if all_cores and "value" in all_cores else single
    cpu = {"value": use["value"], "unit": "grad evals/s", "cores": use["cores"], "kind": "oracle",
           "sample": "oracle log-posterior-and-gradient evaluations of the timed workload's state (%d^3, %d points; "
                     "numpy FP64, own radix-2 FFT): %s" % (
                         mock.n_grid, mock.n_gal,
                         "%d at once in %d single-thread processes" % (use["cores"], use["cores"])
                         if use is all_cores else "one on one thread"),
           "cpu_model": cpu_name, "usable_cores": usable,
           "single_thread": single, "all_cores": all_cores,
           "config1_chain": {"workload": "32^3, box 400, 1000 points, 20 HMC iterations x 10 leapfrog steps (201 "
                                         "gradients), one thread", "seconds": round(t_c1, 2),
                             "grad_evals_per_s": round(201 / t_c1, 3)},
           "config2_gradients": {"workload": "128^3, box 500, 10 000 points, 5 gradients, one thread",
                                 "s_per_grad": round(t_c2, 3),
                                 "chain_200x50_extrapolated_s": round(t_c2 * (200 * 50 + 1), 1)}}
    return cpu, ref


def schedule_info(hamlet, grids, precisions=("fp32", "fp64")):
    """The kernel schedule the library runs at each grid size, and where it
    comes from (the autotuner's JSON cache when it has the grid)."""
    path = os.path.join(os.path.dirname(os.path.abspath(hamlet.__file__)), "tuned_schedules.json")
    tuned = {}
    if os.path.exists(path):
        with open(path) as f:
            tuned = json.load(f).get("schedules", {})
    out = {}
    for prec in precisions:
        for n in grids:
            src = "autotuned" if str(n) in tuned.get(prec, {}) else "default"
            out.setdefault(prec, {})[str(n)] = dict(hamlet.schedule(n, prec), source=src)
    return out


def rel_err(x, ref):
    import numpy as np
    x = np.asarray(x)
    ref = np.asarray(ref)
    den = float(np.abs(ref).max())
    return float(np.abs(x - ref).max() / (den if den > 0 else 1.0))


def main():
    args = parse()
    if args.oracle_worker:
        return oracle_worker(args.oracle_worker)
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(independent chains shard across GPUs with no exchange; see the design notes)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2203_02369_amd import hamlet, mocks

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.workload == "batched":
        return run_batched(args, dev)
    if args.workload == "served":
        return run_served(args, dev)
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read + 1 GiB written")
        del src, dst
    t0 = time.time()
    if args.n_grid > 256:
        # the benchmark's universe and catalogue on the finer grid
        mock = mocks.refine(mocks.paper_scale_256(n_gal=args.n_gal), args.n_grid)
    else:
        mock = mocks.paper_scale_256(n_gal=args.n_gal, n_grid=args.n_grid)
    log("mock %d^3, %d points in %.1fs" % (mock.n_grid, mock.n_gal, time.time() - t0))
    n = mock.n_grid
    # start at a posterior-typical point: the mock field, Hermitian on kz = 0
    dhat0 = mock.dhat_true[:, :, : n // 2]
    d0 = mock.d_true.copy()
    ft = touched_pencil_fraction(mock, d0)
    s0 = 1.5
    L = args.leapfrog
    seed = mocks.config_seed(3) + 3

    def state(plan):
        q = torch.from_numpy(np.ascontiguousarray(dhat0)).to(dev)
        qd = torch.from_numpy(d0.copy()).to(dev)
        return q, qd, plan.scalar(s0)

    # ---- the oracle's state, on both GPU paths (their error is reported) -----
    gpu_at_oracle_state = {}

    def grad_at_start(plan):
        q, qd, qs = state(plan)
        g, gd, gs, psi = plan.zeros_modes(), plan.zeros_dist(), plan.scalar(), plan.scalar()
        hamlet.logpost_grad([plan], [q], [qd], [qs], [g], [gd], [gs], [psi])
        torch.cuda.synchronize()
        gpu_at_oracle_state[plan.precision] = (psi.item(), g.cpu().numpy(), gd.cpu().numpy(), gs.item())

    # ---- adaptation: dual averaging of the step on the FP32 path (untimed) ----
    # The step is set by its own untimed phase, whatever --warmup says; then
    # --warmup iterations run at that step, untimed, and both paths start from
    # where they end.
    plan = hamlet.Plan.from_mock(mock, precision="fp32", device=dev)
    grad_at_start(plan)
    q, qd, qs = state(plan)
    eps = 0.002
    adapt = max(args.adapt, 1)
    acc_a = torch.zeros(adapt, dtype=torch.int32, device=dev)
    eps = hamlet.hmc_run([plan], [q], [qd], [qs], n_iter=adapt, n_leapfrog=L, eps0=eps, seed=seed, warmup=adapt,
                         jitter=True, accepted=[acc_a])[0]
    log("adaptation: %d iterations, eps = %.4g (acceptance during adaptation %.2f)"
        % (adapt, eps, acc_a.float().mean().item()))
    if args.warmup > 0:
        hamlet.hmc_run([plan], [q], [qd], [qs], n_iter=args.warmup, n_leapfrog=L, eps0=eps, seed=seed + 2,
                       jitter=True, want_eps=False)
    torch.cuda.synchronize()
    log("warm-up: %d iterations at eps = %.4g" % (args.warmup, eps))
    start = (q.clone(), qd.clone(), qs.clone())     # both paths start here

    # ---- timed: FP32 fields + FP64 Hamiltonian --------------------------------
    acc = torch.zeros(args.steps, dtype=torch.int32, device=dev)
    dh32 = torch.zeros(args.steps, dtype=torch.float64, device=dev)
    q, qd, qs = (t.clone() for t in start)
    prof = hamlet.KernelTimer(plan, hamlet.PROFILE_KERNELS["fwd_x"])
    torch.cuda.synchronize()
    prof.start()
    t1 = time.perf_counter()
    hamlet.hmc_run([plan], [q], [qd], [qs], n_iter=args.steps, n_leapfrog=L, eps0=eps, seed=seed + 1,
                   jitter=True, accepted=[acc], dh=[dh32], want_eps=False)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    kern_ms, kern_launches = prof.stop()
    dt = t2 - t1
    grads = args.steps * L + 1
    value = grads / dt
    acc32 = acc.cpu().numpy()
    log("fp32: %d iterations x %d steps in %.3fs: %.1f grad/s, acceptance %.2f"
        % (args.steps, L, dt, value, acc32.mean()))

    # ---- the other passes, each timed over two more iterations -----------------
    # algorithmic bytes per launch in c (the z passes also move the points'
    # records, a few MB); the y and z passes move only the rows of pencils in
    # reach of a point (fraction ft, taken at the start positions); the galaxy
    # kernels are latency-bound (time only)
    passes = {"touched_pencil_fraction": round(ft, 4)}
    c_bytes = 8 * n * n * (n // 2)
    for kind, name, cs in (("inv_y", "k_inv_y", 2 + 3 * ft), ("inv_z_gather", "k_inv_z_gather", 3 * ft),
                           ("fwd_z_scatter", "k_fwd_z_scatter", 3 * ft), ("fwd_y", "k_fwd_y", 3 * ft + 2),
                           ("like", "k_like", None), ("bin", "binning (3 kernels)", None)):
        timer = hamlet.KernelTimer(plan, hamlet.PROFILE_KERNELS[kind])
        q2, qd2, qs2 = (t.clone() for t in start)
        torch.cuda.synchronize()
        timer.start()
        hamlet.hmc_run([plan], [q2], [qd2], [qs2], n_iter=2, n_leapfrog=L, eps0=eps, seed=seed + 1, jitter=True,
                       want_eps=False)
        ms, launches = timer.stop()
        entry = {"avg_launch_ms": round(ms / launches, 4), "launches": launches}
        if cs is not None:
            gbs = cs * c_bytes / (ms / launches * 1e-3) / 1e9
            entry.update({"bytes_per_launch": int(cs * c_bytes), "achieved": round(gbs, 1), "unit": "GB/s",
                          "frac": round(gbs / HBM_PEAK_GBS, 4)})
        passes[name] = entry
        del q2, qd2, qs2
    log("passes: " + ", ".join("%s %.4f ms" % (k, v["avg_launch_ms"]) for k, v in passes.items()
                               if isinstance(v, dict)))

    # ---- the No-U-Turn sampler on the same chain (trees of at most 2^6 - 1 steps) ----
    nuts = None
    if args.nuts_iters > 0:
        q2, qd2, qs2 = (t.clone() for t in start)
        hamlet.nuts_run([plan], [q2], [qd2], [qs2], n_iter=1, eps0=eps, seed=seed + 5, max_depth=2)
        q2, qd2, qs2 = (t.clone() for t in start)
        torch.cuda.synchronize()
        tn = time.perf_counter()
        res = hamlet.nuts_run([plan], [q2], [qd2], [qs2], n_iter=args.nuts_iters, eps0=eps, seed=seed + 5,
                              max_depth=args.nuts_depth)[0]
        torch.cuda.synchronize()
        dtn = time.perf_counter() - tn
        leaves = int(res["leaves"].sum())
        nuts = {"value": round(leaves / dtn, 2), "unit": "grad evals/s", "iterations": args.nuts_iters,
                "max_depth": args.nuts_depth, "eps": round(eps, 8), "mean_depth": float(res["depth"].mean()),
                "leapfrog_steps": leaves, "mean_accept_stat": round(float(res["alpha"].mean()), 4),
                "moved": int((res["where"][:, 0] >= 0).sum()),
                "vs_hmc_grad_evals": round(leaves / dtn / value, 3)}
        log("nuts: %d iterations, %d leapfrog steps in %.3fs: %.1f grad/s, mean depth %.1f"
            % (args.nuts_iters, leaves, dtn, leaves / dtn, res["depth"].mean()))
        del q2, qd2, qs2

    # ---- analysis of a state ----------------------------------------------------
    analysis = run_analysis(hamlet, plan, q, mock, c_bytes)
    plan.close()
    del q, qd, qs

    # ---- plain FP64 path, same start, step and seed ------------------------------
    fp64 = None
    acc64 = None
    if not args.no_fp64 and args.fp64_steps > 0:
        plan = hamlet.Plan.from_mock(mock, precision="fp64", device=dev)
        grad_at_start(plan)
        acc64_t = torch.zeros(args.fp64_steps, dtype=torch.int32, device=dev)
        q, qd, qs = (t.clone() for t in start)
        hamlet.hmc_run([plan], [q], [qd], [qs], n_iter=1, n_leapfrog=2, eps0=eps, seed=seed, want_eps=False)
        q, qd, qs = (t.clone() for t in start)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        hamlet.hmc_run([plan], [q], [qd], [qs], n_iter=args.fp64_steps, n_leapfrog=L, eps0=eps, seed=seed + 1,
                       jitter=True, accepted=[acc64_t], want_eps=False)
        torch.cuda.synchronize()
        dt64 = time.perf_counter() - t3
        v64 = (args.fp64_steps * L + 1) / dt64
        acc64 = acc64_t.cpu().numpy()
        m = min(len(acc64), len(acc32))
        fp64 = {"value": round(v64, 2), "unit": "grad evals/s", "ms_per_step": round(1e3 * dt64 / args.fp64_steps, 3),
                "steps": args.fp64_steps, "acceptance": float(acc64.mean()),
                "same_decisions_as_fp32": "%d of %d" % (int((acc64[:m] == acc32[:m]).sum()), m),
                "speedup_fp32_vs_fp64": round(value / v64, 3)}
        log("fp64: %.1f grad/s, acceptance %.2f" % (v64, acc64.mean()))
        plan.close()
        del q, qd, qs

    # ---- a short served stream: latency of continuous batching ----------------
    served = None
    if not args.no_served and args.served_jobs > 0 and n == 256:
        served = run_served_short(args, hamlet, mocks, mock, dev)

    # ---- roofline of the dominant kernel ------------------------------------
    # k_x_pass: the x pass of every evaluation, fused with the leapfrog update
    # and the next inverse pass 1.  Algorithmic bytes in units of one complex64
    # spectral array c (8 N^2 N/2 bytes; the FP64 per-mode prior variance
    # sigma_k^2 counts 1c).  The FP32 path's chain keeps its modes q, momenta
    # p and cached gradient G (and the start point q0, G0) in complex64, 1c
    # each:
    #   plain gradient (1 per run):        S1, S2, q, var in; G out           = 5c
    #   first step of a chain's trajectory (momenta drawn in the pass):
    #                                       G, q, var in; p, q, A, B and the
    #                                       kept start q0, G0 out           = 9c
    #   middle steps (L - 1 per traj.):    S1, S2, p, q, var in; p, q, A, B   = 9c
    #   last step:                         S1, S2, p, q, var in; p, G out     = 7c
    nm = n * n * (n // 2)
    c32 = 8 * nm
    x_bytes = c32 * (5 + args.steps * (9 + 9 * (L - 1) + 7))
    x_launches = 1 + args.steps * (L + 1)
    assert kern_launches == x_launches, (kern_launches, x_launches)
    avg_ms = kern_ms / kern_launches
    per_launch = x_bytes / x_launches
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    traffic = None
    if n == 256 and kernel_sources_sha1(hamlet.schedule(n, "fp32")) == X_TRAFFIC_SOURCES_SHA1:
        t = X_TRAFFIC
        tot = sum(t["grad"]) + args.steps * (sum(t["first"]) + (L - 1) * sum(t["mid"]) + sum(t["last"]))
        traffic = int(tot / x_launches)
    roofline = {"bound": "hbm", "kernel": "k_x_pass (x FFT + gradient + leapfrog update + next inverse x FFT)",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "bytes_per_launch": int(per_launch), "avg_launch_ms": round(avg_ms, 4), "launches": kern_launches}

    # ---- CPU baseline: the oracle on the host cores --------------------------
    cpu = None
    oracle_err = None
    if not args.no_cpu_baseline and n <= 256:   # the oracle takes minutes per evaluation above 256^3
        from oracle import hmc
        dh_full = hmc.symmetrise(n, mock.dhat_true)
        cpu, ref = cpu_baseline(args, mock, dh_full, d0, s0)
        # the GPU paths' error against this same oracle evaluation (relative,
        # max-norm per array; the modes compared on the stored kz < N/2)
        oracle_err = {}
        for prec, (psi, g, gd, gs) in gpu_at_oracle_state.items():
            oracle_err[prec] = {"psi": abs(psi - ref[0]) / abs(ref[0]),
                                "grad_modes": rel_err(g, ref[1][:, :, : n // 2]),
                                "grad_dist": rel_err(gd, ref[2]),
                                "grad_s": abs(gs - ref[3]) / abs(ref[3])}
        log("error against the oracle: " + json.dumps(oracle_err))

    out = {
        "metric": "grad evals/s (fwd+adjoint) at %d³, N=3e4 vs plain FP64; p50/p99 job latency" % n,
        "value": round(value, 2),
        "unit": "grad evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 fields, f64 Hamiltonian",
        "data": "synthetic",
        "config": {"workload": "paper-scale single chain: %d^3 grid, box 500 Mpc/h, %d points, "
                               "HMC iteration of %d leapfrog steps" % (n, mock.n_gal, L),
                   "n_grid": n, "n_gal": mock.n_gal, "leapfrog_steps": L, "eps": round(eps, 8),
                   "adaptation_iterations": adapt,
                   "acceptance": float(acc32.mean()), "grad_evals_timed": grads},
        "fp64_path": fp64,
        "nuts": nuts,
        "served": served,
        "oracle_err": oracle_err,
        "schedule": schedule_info(hamlet, [n]),
        "roofline": roofline,
        "passes": passes,
        "analysis": analysis,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    low = [name for name, a in (("fp32", acc32), ("fp64", acc64)) if a is not None and a.mean() < MIN_ACCEPTANCE]
    if low:
        log("acceptance below %.2f on %s: the paths were not compared while sampling" % (MIN_ACCEPTANCE, low))
        sys.exit(3)


def run_analysis(hamlet, plan, q, mock, c_bytes):
    """Timings of the on-device analysis of a state (sphere moments, velocity
    and density fields, running sums of the maps, shell statistics)."""
    import torch
    n = mock.n_grid
    # monopole and dipole in 16 spheres, four passes over the FP64 modes; the
    # FP64 window per mode and radius bounds it, not the mode reads
    radii = [5.0 + 15.0 * j for j in range(16)]
    hamlet.sphere_moments(plan, q, radii)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(plan.stream)
    for _ in range(5):
        hamlet.sphere_moments(plan, q, radii)
    ev1.record(plan.stream)
    ev1.synchronize()
    mom_ms = ev0.elapsed_time(ev1) / 5
    mom_passes = 2   # 8 radii per pass over the FP64 modes
    mom_bytes = mom_passes * 16 * n * n * (n // 2)
    analysis = {"sphere_moments": {"radii": len(radii), "avg_call_ms": round(mom_ms, 4), "mode_passes": mom_passes,
                                   "mode_bytes_per_call": mom_bytes,
                                   "mode_read_GBs": round(mom_bytes / (mom_ms * 1e-3) / 1e9, 1)}}
    log("sphere moments (16 radii): %.3f ms per call" % mom_ms)
    # the whole velocity field of the state (three grids of N^3 reals): the
    # inverse x pass (modes, sigma^2 in: 3c; A, B out: 2c), the y pass with
    # every row (2c in, 3c out) and the z pass writing the field (3c in, 3c out)
    vf = hamlet.velocity_field(plan, q)
    ev0.record(plan.stream)
    for _ in range(5):
        hamlet.velocity_field(plan, q, out=vf)
    ev1.record(plan.stream)
    ev1.synchronize()
    vf_ms = ev0.elapsed_time(ev1) / 5
    vf_bytes = 16 * c_bytes
    analysis["velocity_field"] = {"avg_call_ms": round(vf_ms, 4), "bytes_per_call": vf_bytes,
                                  "achieved": round(vf_bytes / (vf_ms * 1e-3) / 1e9, 1), "unit": "GB/s"}
    log("velocity field: %.3f ms per call" % vf_ms)
    del vf
    # the density contrast of the state: the velocity field's passes with one
    # grid out move 14c; a density-only chain of passes would move 7c
    dg = hamlet.density_field(plan, q)
    ev0.record(plan.stream)
    for _ in range(5):
        hamlet.density_field(plan, q, out=dg)
    ev1.record(plan.stream)
    ev1.synchronize()
    dg_ms = ev0.elapsed_time(ev1) / 5
    analysis["density_field"] = {"avg_call_ms": round(dg_ms, 4), "bytes_per_call": 14 * c_bytes,
                                 "density_only_minimum_bytes": 7 * c_bytes,
                                 "achieved": round(14 * c_bytes / (dg_ms * 1e-3) / 1e9, 1), "unit": "GB/s"}
    log("density field: %.3f ms per call" % dg_ms)
    del dg
    # a state added to the running sums of delta, v_r and their squares:
    # both chains of passes, the sums read and written in FP64 (42c)
    acc = hamlet.field_stats_accumulate(plan, q)
    ev0.record(plan.stream)
    for _ in range(3):
        hamlet.field_stats_accumulate(plan, q, acc)
    ev1.record(plan.stream)
    ev1.synchronize()
    fs_ms = ev0.elapsed_time(ev1) / 3
    analysis["field_stats_accumulate"] = {"avg_call_ms": round(fs_ms, 4), "bytes_per_call": 42 * c_bytes,
                                          "achieved": round(42 * c_bytes / (fs_ms * 1e-3) / 1e9, 1), "unit": "GB/s"}
    log("field statistics: %.3f ms per state" % fs_ms)
    # shells of 10 Mpc/h out past the box corner, over two FP64 grids: 4c
    # algorithmic (each grid once); the two sweeps read them twice
    n_sh = int(math.ceil(math.sqrt(3.0) * 0.5 * mock.box / 10.0)) + 1
    hamlet.shell_stats(plan, acc[0], acc[2], 10.0, n_sh)
    ev0.record(plan.stream)
    for _ in range(3):
        hamlet.shell_stats(plan, acc[0], acc[2], 10.0, n_sh)
    ev1.record(plan.stream)
    ev1.synchronize()
    sh_ms = ev0.elapsed_time(ev1) / 3
    analysis["shell_stats"] = {"shells": n_sh, "width": 10.0, "avg_call_ms": round(sh_ms, 4),
                               "bytes_per_call": 4 * c_bytes, "sweeps": 2,
                               "achieved": round(4 * c_bytes / (sh_ms * 1e-3) / 1e9, 1), "unit": "GB/s"}
    log("shell statistics: %.3f ms per call" % sh_ms)
    del acc
    return analysis


def run_served_short(args, hamlet, mocks, mock, dev):
    """p50 / p99 latency of a short seeded Poisson stream of requests (grids
    64^3, 128^3, 256^3; 1000-30 000 points; 100 iterations of 20 leapfrog
    steps each), served by continuous batching in FP32 and, for comparison,
    one job at a time by the plain FP64 path."""
    import numpy as np

    class A:
        jobs = args.served_jobs
        rate = args.rate
    trace = served_trace(A, mocks, np, pools=1)
    universes = {(256, 0): mock}
    for ng in (64, 128):
        universes[(ng, 0)] = mocks.paper_scale_256(n_gal=30000, n_grid=ng, seed=mocks.config_seed(5) + ng)
    L, n_iter = 20, 100
    budget = 96 << 30
    grads = sum(1 + n_iter * L for _ in trace)
    lat32, span32 = serve_trace(hamlet, trace, universes, "fp32", 0, L, n_iter, budget, dev, "served fp32")
    out = {"requests": len(trace), "rate_per_s": A.rate, "iterations": n_iter, "leapfrog_steps": L,
           "latency_p50_s": round(float(np.percentile(lat32, 50)), 3),
           "latency_p99_s": round(float(np.percentile(lat32, 99)), 3),
           "grad_evals_per_s": round(grads / span32, 1), "makespan_s": round(span32, 2)}
    log("served fp32: %d jobs, p50 %.2fs, p99 %.2fs" % (len(trace), out["latency_p50_s"], out["latency_p99_s"]))
    if not args.no_fp64:
        lat64, span64 = serve_trace(hamlet, trace, universes, "fp64", 1, L, n_iter, budget, dev, "fp64 one at a time")
        out["fp64_one_job_at_a_time"] = {"latency_p50_s": round(float(np.percentile(lat64, 50)), 3),
                                         "latency_p99_s": round(float(np.percentile(lat64, 99)), 3),
                                         "grad_evals_per_s": round(grads / span64, 1),
                                         "makespan_s": round(span64, 2)}
        log("fp64 one at a time: p50 %.2fs, p99 %.2fs" % (float(np.percentile(lat64, 50)),
                                                          float(np.percentile(lat64, 99))))
    return out


def run_batched(args, dev):
    import numpy as np
    import torch

    from paper_2203_02369_amd import hamlet, mocks

    L = args.leapfrog
    t0 = time.time()
    ms = []
    for j, (ng, n) in enumerate(mocks.batched_16_sizes()):
        ms.append(mocks.make_mock(ng, 500.0, n, 200.0, "inv_r", (0.20, 0.25), seed=mocks.config_seed(4) + j))
        log("mock %d: %d^3, %d points (%.0fs)" % (j, ng, n, time.time() - t0))
    plans = [hamlet.Plan.from_mock(m, precision="fp32", device=dev) for m in ms]
    qm = [torch.from_numpy(np.ascontiguousarray(m.dhat_true[:, :, : m.n_grid // 2])).to(dev) for m in ms]
    qd = [torch.from_numpy(m.d_true.copy()).to(dev) for m in ms]
    qs = [p.scalar(1.5) for p in plans]
    seeds = [mocks.config_seed(4) + 100 + j for j in range(len(plans))]

    # warm-up: every chain adapts its own step (dual averaging), all together
    eps = hamlet.hmc_run(plans, qm, qd, qs, n_iter=args.warmup, n_leapfrog=L, eps0=0.002, seed=0, seeds=seeds,
                         warmup=args.warmup, jitter=True)
    log("warm-up: %d iterations, eps %s" % (args.warmup, " ".join("%.3g" % e for e in eps)))

    # timed: shared launches, every chain continuing from its warm-up
    lead = plans[[p.n_grid for p in plans].index(256)]
    prof = hamlet.KernelTimer(lead, hamlet.PROFILE_KERNELS["fwd_x"])
    acc = [torch.zeros(args.warmup + 2 * args.steps, dtype=torch.int32, device=dev) for _ in plans]
    torch.cuda.synchronize()
    prof.start()
    t1 = time.perf_counter()
    hamlet.hmc_run(plans, qm, qd, qs, n_iter=args.steps, n_leapfrog=L, eps0=0.002, seed=0, seeds=seeds,
                   jitter=True, accepted=acc, resume=True, want_eps=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    kern_ms, kern_launches = prof.stop()
    grads = len(plans) * args.steps * L
    value = grads / dt
    log("batched: %d chains x %d iterations x %d steps in %.3fs: %.1f grad/s" % (len(plans), args.steps, L, dt, value))

    # the same chains one at a time
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for j, p in enumerate(plans):
        hamlet.hmc_run([p], [qm[j]], [qd[j]], [qs[j]], n_iter=args.steps, n_leapfrog=L, eps0=0.002, seed=0,
                       seeds=[seeds[j]], jitter=True, accepted=[acc[j]], resume=True, want_eps=False)
        torch.cuda.synchronize()   # one chain after the other, whatever the streams
    dt_seq = time.perf_counter() - t2
    v_seq = grads / dt_seq
    log("one at a time: %.3fs: %.1f grad/s" % (dt_seq, v_seq))
    rate = float(np.mean([a.cpu().numpy()[args.warmup:].mean() for a in acc]))

    # roofline of the x pass of the 256^3 group (5 chains per launch, chain
    # states in complex64): per chain and iteration first 9c, L - 1 middle 9c,
    # last 7c.
    n256 = [p for p in plans if p.n_grid == 256]
    c32 = 8 * 256 * 256 * 128
    per_iter = len(n256) * c32 * (9 + 9 * (L - 1) + 7)
    assert kern_launches == args.steps * (L + 1), (kern_launches, args.steps * (L + 1))
    avg_ms = kern_ms / kern_launches
    per_launch = per_iter * args.steps / kern_launches
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    out = {
        "metric": "grad evals/s summed over 16 independent chains (64^3/128^3/256^3, 2000-30000 points)",
        "value": round(value, 2),
        "unit": "grad evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * dt / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 fields, f64 Hamiltonian",
        "data": "synthetic",
        "config": {"workload": "batched: 16 chains, grids 64^3/128^3/256^3 in turn, n_j = 2000 + 28000 j / 15, "
                               "box 500 Mpc/h, HMC iterations of %d leapfrog steps; chains of one grid size "
                               "share every launch, the grid sizes run side by side" % L,
                   "chains": [[p.n_grid, p.n_gal] for p in plans], "leapfrog_steps": L,
                   "acceptance": round(rate, 3), "grad_evals_timed": grads},
        "schedule": schedule_info(hamlet, sorted({p.n_grid for p in plans}), ("fp32",)),
        "one_at_a_time": {"value": round(v_seq, 2), "unit": "grad evals/s",
                          "speedup_shared_vs_one_at_a_time": round(value / v_seq, 3)},
        "roofline": {"bound": "hbm", "kernel": "k_x_pass<float, 256> over the five 256^3 chains of one launch",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_launch": int(per_launch), "avg_launch_ms": round(avg_ms, 4),
                     "launches": kern_launches},
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)
    for p in plans:
        p.close()


def served_trace(args, mocks, np, pools=2):
    """Seeded request stream: arrival time, grid, pool universe, catalogue size, seed."""
    rng = np.random.default_rng(mocks.config_seed(5))
    t = np.cumsum(rng.exponential(1.0 / args.rate, args.jobs))
    grids = rng.choice([64, 128, 256], args.jobs)
    pool = rng.integers(0, pools, args.jobs)
    sizes = rng.integers(1000, 30001, args.jobs)
    return [dict(t=float(t[k]), n_grid=int(grids[k]), pool=int(pool[k]), n_gal=int(sizes[k]),
                 seed=mocks.config_seed(5) + 1000 + k) for k in range(args.jobs)]


def serve_trace(hamlet, trace, universes, precision, max_running, L, n_iter, budget, dev, label):
    """Replays the request stream in real time through a server; returns per-job latencies (s) and the makespan."""
    import numpy as np
    sv = hamlet.Server(budget, max_running=max_running, ticks_ahead=2, device=dev)
    t0 = time.perf_counter()
    pending = list(range(len(trace)))
    live = {}
    lat = {}
    last_log = t0
    while len(lat) < len(trace):
        now = time.perf_counter() - t0
        while pending and trace[pending[0]]["t"] <= now:
            k = pending.pop(0)
            r = trace[k]
            u = universes[(r["n_grid"], r["pool"])]
            n = r["n_gal"]
            prob = u.problem_kwargs()
            for key in ("rhat", "mu", "sigma_mu", "cz", "sigma_cz"):
                prob[key] = prob[key][:n]
            live[sv.submit(n_iter=n_iter, n_leapfrog=L, eps0=2e-3, warmup=n_iter // 5, jitter=True,
                           seed=r["seed"], precision=precision, **prob)] = k
        if live:
            sv.tick()
            for j in list(live):
                if sv.state(j) == "finished":
                    k = live.pop(j)
                    sv.take(j, outputs=("dh", "accepted"))
                    lat[k] = time.perf_counter() - t0 - trace[k]["t"]
        elif pending:
            time.sleep(max(0.0, min(0.05, trace[pending[0]]["t"] - now)))
        if time.perf_counter() - last_log > 5.0:
            last_log = time.perf_counter()
            log("%s: %.0fs, %d done, %d running or queued" % (label, last_log - t0, len(lat), len(live)))
    makespan = time.perf_counter() - t0 - trace[0]["t"]
    sv.close()
    return np.array([lat[k] for k in range(len(trace))]), makespan


def run_served(args, dev):
    import numpy as np

    from paper_2203_02369_amd import hamlet, mocks

    L = args.leapfrog
    n_iter = args.iters
    trace = served_trace(args, mocks, np)
    t0 = time.time()
    universes = {}
    for ng in (64, 128, 256):
        for p in range(2):
            universes[(ng, p)] = mocks.paper_scale_256(n_gal=30000, n_grid=ng, seed=mocks.config_seed(5) + 10 * p + ng)
            log("universe %d^3 #%d (%.0fs)" % (ng, p, time.time() - t0))
    budget = 96 << 30
    grads = sum(1 + n_iter * L for _ in trace)
    lat32, span32 = serve_trace(hamlet, trace, universes, "fp32", args.max_running, L, n_iter, budget, dev,
                                "served fp32")
    log("served fp32: %d jobs in %.1fs, p50 %.2fs, p99 %.2fs" % (len(trace), span32, np.percentile(lat32, 50),
                                                                 np.percentile(lat32, 99)))
    fp64 = None
    if not args.no_fp64:
        lat64, span64 = serve_trace(hamlet, trace, universes, "fp64", 1, L, n_iter, budget, dev, "fp64 one at a time")
        log("fp64 one job at a time: %.1fs, p50 %.2fs, p99 %.2fs" % (span64, np.percentile(lat64, 50),
                                                                     np.percentile(lat64, 99)))
        fp64 = {"value": round(grads / span64, 2), "unit": "grad evals/s", "jobs_per_s": round(len(trace) / span64, 3),
                "latency_p50_s": round(float(np.percentile(lat64, 50)), 3),
                "latency_p99_s": round(float(np.percentile(lat64, 99)), 3), "makespan_s": round(span64, 2)}
    value = grads / span32
    out = {
        "metric": "grad evals/s serving a Poisson stream of reconstructions (64^3/128^3/256^3, 1000-30000 points)",
        "value": round(value, 2),
        "unit": "grad evals/s",
        "n_gpus": 1,
        "steps": len(trace),
        "warmup": 0,
        "ms_per_step": round(1e3 * span32 / len(trace), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 fields, f64 Hamiltonian",
        "data": "synthetic",
        "config": {"workload": "served: %d requests, Poisson arrivals at %.2f/s, grid uniform in 64^3/128^3/256^3, "
                               "1000-30000 points (paper-scale catalogue generator), %d HMC iterations of %d "
                               "leapfrog steps each, continuous batching, admission by device footprint%s"
                               % (len(trace), args.rate, n_iter, L,
                                  ", at most %d jobs advanced together" % args.max_running if args.max_running else ""),
                   "jobs_per_s": round(len(trace) / span32, 3), "latency_p50_s": round(float(np.percentile(lat32, 50)), 3),
                   "latency_p99_s": round(float(np.percentile(lat32, 99)), 3), "makespan_s": round(span32, 2),
                   "grad_evals": grads},
        "fp64_one_job_at_a_time": fp64,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

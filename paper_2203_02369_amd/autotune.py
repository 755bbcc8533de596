"""Autotuner of the kernel schedule (csrc/schedule.hpp).

Per grid size and precision it picks the threads per block of each pass
kind, the tile width of the x and y passes, the pencils per z tile of the
gather and of the scatter, and the radix plan of the LDS transforms.

Candidates move one parameter away from the hand-picked defaults.  Each is a
library built for one grid size (-DHAMLET_ONLY_N, -DHAMLET_SCHED_DEFAULTS and
the parameter's -D) and timed in a process of its own (HAMLET_LIB names the
library) on the benchmark's synthetic problem at that grid size: the HIP
events of hamlet_profile_* give each kernel kind's time per gradient inside
HMC trajectories.  A candidate whose gradient at the start point differs
from the default's by more than rounding is discarded.  A parameter takes
the value that minimises the time of the kernels it shapes when that beats
the default by more than the noise margin; the choices go into
tuned_schedules.json (beside this file) and are compiled in through
csrc/tuned.hpp.  Parameters are chosen one at a time, so the combined
schedule is timed again against the default before it is trusted.

    python -m paper_2203_02369_amd.autotune build [--grids 64 128 256 512]  # CPU: candidates
    python -m paper_2203_02369_amd.autotune time --out FILE [--grids ...]   # GPU: time them
    python -m paper_2203_02369_amd.autotune select FILE [FILE ...]          # CPU: JSON + tuned.hpp
    python -m paper_2203_02369_amd.autotune time --out V --only default --current   # GPU: combined
    python -m paper_2203_02369_amd.autotune verify V                        # CPU: record it
    python -m paper_2203_02369_amd.autotune build --refine --grids ...      # CPU: moves from the tuned
    python -m paper_2203_02369_amd.autotune select --refine FILE            # CPU: merge them
    python -m paper_2203_02369_amd.autotune header                          # CPU: tuned.hpp from JSON
"""
import argparse
import concurrent.futures
import json
import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
TUNE_DIR = os.path.join(ROOT, "_build", "tune")
MANIFEST = os.path.join(TUNE_DIR, "manifest.json")
TUNED_JSON = os.path.join(PKG, "tuned_schedules.json")
TUNED_HPP = os.path.join(PKG, "csrc", "tuned.hpp")

GRIDS = (64, 128, 256, 512, 1024)
PRECISIONS = ("fp32", "fp64")
KINDS = ("bin", "inv_y", "inv_z_gather", "like", "fwd_z_scatter", "fwd_y", "fwd_x")
FFT_KINDS = ("inv_y", "inv_z_gather", "fwd_z_scatter", "fwd_y", "fwd_x")
# parameter: (macro, candidate values, schedule field it sets, kernel kinds whose time decides)
PARAMS = {
    "XY": ("HAMLET_SCHED_XY", (128, 256, 512, 1024), "threads_xy", ("inv_y", "fwd_y")),
    "X": ("HAMLET_SCHED_X", (256, 512, 1024), "threads_x", ("fwd_x",)),
    "ZG": ("HAMLET_SCHED_ZG", (128, 256, 512), "threads_gather", ("inv_z_gather",)),
    "ZS": ("HAMLET_SCHED_ZS", (128, 256, 512), "threads_scatter", ("fwd_z_scatter",)),
    "W": ("HAMLET_SCHED_W_SHIFT", (-1, 1, 2), "tile_width", ("inv_y", "fwd_y", "fwd_x")),
    "PZ": ("HAMLET_SCHED_PZ_SHIFT", (-1, 1), "pencils_scatter", ("fwd_z_scatter",)),
    "PG": ("HAMLET_SCHED_PG_SHIFT", (-1, 1), "pencils_gather", ("inv_z_gather",)),
    "RADIX": ("HAMLET_SCHED_RADIX", None, "radix_plan", FFT_KINDS),
}
# the tuned.hpp member each schedule field sets
FIELD_MEMBER = {"threads_xy": "XY", "threads_x": "X", "threads_gather": "ZG", "threads_scatter": "ZS",
                "tile_width": "W", "pencils_scatter": "PZ", "pencils_gather": "PG", "radix_plan": "RADIX"}
MARGIN = 0.03          # a change must gain at least this fraction of the deciding kernels' time
EPS = 0.001            # leapfrog step of the timed trajectories (well inside the stable range)
ITER, LEAP, REPS = 3, 10, 2


def trajectory(n):
    """(iterations, leapfrog steps) of each timed run: shorter at 1024^3,
    where one gradient takes tens of milliseconds."""
    return (1, 5) if n >= 1024 else (ITER, LEAP)
SEED = 20220304


def radix_plans(n):
    # the number of radix plans csrc/schedule.hpp holds for a transform length
    return {16: 2, 32: 3, 64: 3, 128: 3, 256: 4, 512: 3}.get(n, 1)


def candidates(grids, refine=False):
    """One-parameter moves from the defaults, or (refine) from the schedule
    the committed tuned.hpp holds: a second sweep catches parameters whose
    best value moved once the others were chosen."""
    out = []
    for n in grids:
        base = ["HAMLET_ONLY_N=%d" % n] + ([] if refine else ["HAMLET_SCHED_DEFAULTS"])
        pre = "n%d_%s" % (n, "r" if refine else "")
        out.append({"name": pre + ("tuned" if refine else "default"), "n": n, "param": None, "value": None,
                    "defines": base})
        for param, (macro, values, _field, _kinds) in PARAMS.items():
            if values is None:
                values = range(0 if refine else 1, radix_plans(n))
            for v in values:
                if not refine and param in ("XY", "X", "ZG", "ZS") and v == default_threads(param, n):
                    continue
                tag = ("m%d" % -v) if v < 0 else str(v)
                out.append({"name": pre + "%s%s" % (param, tag), "n": n, "param": param, "value": v,
                            "defines": base + ["%s=%d" % (macro, v)]})
    for c in out:
        c["lib"] = os.path.join("_build", "tune", c["name"] + ".so")
    return out


def default_threads(param, n):
    return {"XY": 512 if n >= 512 else 256, "X": 512, "ZG": 256, "ZS": 256}[param]


# -- build (CPU) ---------------------------------------------------------------

def cmd_build(args):
    from . import build
    os.makedirs(TUNE_DIR, exist_ok=True)
    cands = [c for c in candidates(args.grids, args.refine) if c["param"] is None or not args.params
             or c["param"] in args.params]

    def one(c):
        t = time.time()
        try:
            build.build(out=os.path.join(ROOT, c["lib"]), defines=c["defines"], quiet=True)
            return c, None, time.time() - t
        except RuntimeError as e:
            return c, str(e), time.time() - t

    built = []
    with concurrent.futures.ThreadPoolExecutor(max_workers=args.jobs) as ex:
        for c, err, dt in ex.map(one, cands):
            if err:
                print("%-22s does not build (%.0fs): %s" % (c["name"], dt, err.splitlines()[-1][:200]), flush=True)
            else:
                print("%-22s built (%.0fs)" % (c["name"], dt), flush=True)
                built.append(c)
    with open(MANIFEST, "w") as f:
        json.dump(built, f, indent=1)
    print("%d of %d candidates built; manifest %s" % (len(built), len(cands), MANIFEST))


# -- timing (GPU, one process per library) ---------------------------------------

def tune_mock(n):
    from . import mocks
    if n > 256:
        return mocks.refine(mocks.paper_scale_256(), n)
    return mocks.paper_scale_256(n_grid=n)


def measure(n, ref_path, save_ref, precisions):
    """Times the loaded library's kernels at grid size n; prints one JSON line."""
    import numpy as np
    import torch

    from . import hamlet
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    mock = tune_mock(n)
    dhat0 = np.ascontiguousarray(mock.dhat_true[:, :, : n // 2])
    res = {"n": n, "n_gal": int(mock.n_gal), "precisions": {}}
    refs = dict(np.load(ref_path)) if (ref_path and not save_ref and os.path.exists(ref_path)) else {}
    saved = {}
    for prec in precisions:
        plan = hamlet.Plan.from_mock(mock, precision=prec, device=dev)

        def start():
            return (torch.from_numpy(dhat0).to(dev), torch.from_numpy(mock.d_true.copy()).to(dev),
                    plan.scalar(1.5))

        q, qd, qs = start()
        g, gd, gs, psi = plan.zeros_modes(), plan.zeros_dist(), plan.scalar(), plan.scalar()
        hamlet.logpost_grad([plan], [q], [qd], [qs], [g], [gd], [gs], [psi])
        # the mode gradient on a fixed strided sample of at most 4M entries
        flat = g.reshape(-1)
        gn = flat[:: max(1, flat.numel() >> 22)].cpu().numpy()
        del flat
        gdn = gd.cpu().numpy()
        psin = float(psi.item())
        entry = {"schedule": hamlet.schedule(n, prec)}
        if save_ref:
            saved.update({prec + "_g": gn, prec + "_gd": gdn, prec + "_psi": np.array([psin])})
            entry["check"] = "reference"
        elif refs:
            rg, rgd, rpsi = refs[prec + "_g"], refs[prec + "_gd"], float(refs[prec + "_psi"][0])
            err = {"g": float(np.abs(gn - rg).max() / max(np.abs(rg).max(), 1e-300)),
                   "gd": float(np.abs(gdn - rgd).max() / max(np.abs(rgd).max(), 1e-300)),
                   "psi": abs(psin - rpsi) / max(abs(rpsi), 1e-300)}
            # rounding only: FP32 transforms in another order of operations,
            # FP64 sums in another order
            tol = {"g": 1e-4, "gd": 1e-4, "psi": 1e-5} if prec == "fp32" else {"g": 1e-10, "gd": 1e-10, "psi": 1e-11}
            entry["check"] = err
            entry["ok"] = all(err[k] <= tol[k] for k in err)
        # warm-up trajectory, then each kernel kind timed over ITER
        # trajectories of LEAP steps, REPS times (the fastest is kept)
        n_it, n_lf = trajectory(n)
        q, qd, qs = start()
        hamlet.hmc_run([plan], [q], [qd], [qs], n_iter=1, n_leapfrog=n_lf, eps0=EPS, seed=SEED, want_eps=False)
        kinds = {}
        for _ in range(REPS):
            for kind in KINDS:
                q, qd, qs = start()
                timer = hamlet.KernelTimer(plan, hamlet.PROFILE_KERNELS[kind])
                torch.cuda.synchronize()
                timer.start()
                hamlet.hmc_run([plan], [q], [qd], [qs], n_iter=n_it, n_leapfrog=n_lf, eps0=EPS, seed=SEED,
                               want_eps=False)
                ms, launches = timer.stop()
                per = ms / (n_it * n_lf)
                kinds[kind] = min(kinds.get(kind, float("inf")), per)
        # the whole gradient, wall clock (no events armed)
        q, qd, qs = start()
        torch.cuda.synchronize()
        t = time.perf_counter()
        hamlet.hmc_run([plan], [q], [qd], [qs], n_iter=n_it, n_leapfrog=n_lf, eps0=EPS, seed=SEED, want_eps=False)
        torch.cuda.synchronize()
        entry["wall_ms_per_grad"] = round((time.perf_counter() - t) * 1e3 / (n_it * n_lf), 5)
        entry["kinds_ms_per_grad"] = {k: round(v, 5) for k, v in kinds.items()}
        entry["kernel_ms_per_grad"] = round(sum(kinds.values()), 5)
        res["precisions"][prec] = entry
        plan.close()
        del q, qd, qs, g, gd, gs, psi
        torch.cuda.empty_cache()
    if save_ref:
        np.savez(ref_path, **saved)
    print("RESULT " + json.dumps(res), flush=True)


def cmd_time(args):
    with open(MANIFEST) as f:
        cands = [c for c in json.load(f) if c["n"] in args.grids]
    if args.only:
        cands = [c for c in cands if c["name"] in args.only or (c["param"] is None and "default" in args.only)]
    if args.current:
        # the library as built in the package (tuned), beside the defaults
        for n in args.grids:
            cands.append({"name": "n%d_current" % n, "n": n, "param": "current", "value": None, "lib": None})
    cands.sort(key=lambda c: (c["n"], c["param"] is not None))
    import torch
    device = torch.cuda.get_device_name(0) if torch.cuda.device_count() else "unknown"
    out = {"device": device, "eps": EPS, "iterations": ITER, "leapfrog": LEAP, "reps": REPS, "results": []}
    ref_dir = os.path.join(TUNE_DIR, "refs")
    os.makedirs(ref_dir, exist_ok=True)
    t0 = time.time()
    for i, c in enumerate(cands):
        env = dict(os.environ)
        if c.get("lib"):
            env["HAMLET_LIB"] = os.path.join(ROOT, c["lib"])
        else:
            env.pop("HAMLET_LIB", None)
        ref = os.path.join(ref_dir, "n%d.npz" % c["n"])
        cmd = [sys.executable, "-u", "-m", "paper_2203_02369_amd.autotune", "measure", "--n", str(c["n"]),
               "--ref", ref] + (["--save-ref"] if c["param"] is None else [])
        print("[%4.0fs] %d/%d %s" % (time.time() - t0, i + 1, len(cands), c["name"]), flush=True)
        try:
            p = subprocess.run(cmd, env=env, cwd=ROOT, capture_output=True, text=True, timeout=args.timeout)
        except subprocess.TimeoutExpired:
            print("  timed out: stopping the sweep", flush=True)
            out["stopped"] = c["name"] + ": timed out"
            break
        line = [ln for ln in p.stdout.splitlines() if ln.startswith("RESULT ")]
        if p.returncode != 0 or not line:
            print("  exit %d: stopping the sweep\n%s" % (p.returncode, (p.stdout + p.stderr)[-3000:]), flush=True)
            out["stopped"] = "%s: exit %d" % (c["name"], p.returncode)
            break
        r = json.loads(line[-1][len("RESULT "):])
        r.update({"name": c["name"], "param": c["param"], "value": c["value"]})
        out["results"].append(r)
        print("  " + ", ".join("%s %.4f ms/grad%s" % (k, v["kernel_ms_per_grad"],
                                                       "" if v.get("ok", True) else " (MISMATCH)")
                               for k, v in r["precisions"].items()), flush=True)
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1)
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    if "stopped" in out:
        sys.exit(1)


# -- selection (CPU) -------------------------------------------------------------

def select(results, margin=MARGIN):
    """Per (precision, grid): the base schedule (the defaults, or the tuned
    one in a refinement sweep) with the one-parameter changes that gain more
    than `margin` on the kernels they shape.  Changes are taken in order of
    their gain, and one that shapes a kernel an earlier change shaped is left
    out: each was timed against the base alone, so only changes to disjoint
    kernels are known to add up."""
    chosen, gains = {}, {}
    by_n = {}
    for r in results:
        by_n.setdefault(r["n"], []).append(r)
    for n, rs in sorted(by_n.items()):
        base = [r for r in rs if r["param"] is None]
        if not base:
            continue
        base = base[0]
        for prec in PRECISIONS:
            if prec not in base["precisions"]:
                continue
            b = base["precisions"][prec]
            sched = {k: v for k, v in b["schedule"].items() if k != "radix"}
            moves = []
            for param, (_macro, _values, field, kinds) in PARAMS.items():
                def cost(e):
                    return sum(e["kinds_ms_per_grad"][k] for k in kinds)
                best, best_cost = None, cost(b)
                for r in rs:
                    e = r["precisions"].get(prec)
                    if r["param"] != param or e is None or not e.get("ok", False):
                        continue
                    if e["schedule"][field] == b["schedule"][field]:
                        continue   # clamped back to the base value
                    if cost(e) < best_cost:
                        best, best_cost = e, cost(e)
                if best is not None and best_cost < (1.0 - margin) * cost(b):
                    moves.append((cost(b) - best_cost, param, field, kinds, best, best_cost, cost(b)))
            g, shaped = {}, set()
            for gain, param, field, kinds, best, best_cost, base_cost in sorted(moves, key=lambda m: -m[0]):
                if shaped & set(kinds):
                    continue
                shaped |= set(kinds)
                sched[field] = best["schedule"][field]
                g[param] = {"value": best["schedule"][field], "default": b["schedule"][field],
                            "kernels": list(kinds), "ms_per_grad": round(best_cost, 5),
                            "default_ms_per_grad": round(base_cost, 5)}
            chosen.setdefault(prec, {})[str(n)] = sched
            gains.setdefault(prec, {})[str(n)] = g
    return chosen, gains


def write_header(chosen, defaults):
    lines = ["// Kernel schedules chosen by the autotuner (paper_2203_02369_amd/autotune.py)",
             "// from tuned_schedules.json; grids and types not listed keep DefaultSched.",
             "// Generated: do not edit by hand.",
             "#pragma once", "", "namespace hamlet {", ""]
    for prec, typ in (("fp32", "float"), ("fp64", "double")):
        for n, sched in sorted(chosen.get(prec, {}).items(), key=lambda kv: int(kv[0])):
            d = defaults[prec][n]
            diff = {f: v for f, v in sched.items() if d.get(f) != v}
            if not diff:
                continue
            lines.append("template <> struct Tuned<%s, %s> : DefaultSched<%s, %s> {" % (typ, n, typ, n))
            for f, v in sorted(diff.items()):
                lines.append("  static constexpr int %s = %d;" % (FIELD_MEMBER[f], v))
            lines.append("};")
            lines.append("")
    lines.append("}  // namespace hamlet")
    with open(TUNED_HPP, "w") as f:
        f.write("\n".join(lines) + "\n")


def cmd_select(args):
    results, meta = [], {}
    for path in args.files:
        with open(path) as f:
            d = json.load(f)
        results += [r for r in d["results"] if r["param"] != "current"]
        meta = {k: d[k] for k in ("device", "eps", "iterations", "leapfrog", "reps")}
    chosen, gains = select(results)
    defaults = {}
    if args.refine:
        # a sweep from the tuned schedules: merge into the committed choice,
        # whose defaults stay the hand-picked schedules
        with open(TUNED_JSON) as f:
            old = json.load(f)
        defaults = old["defaults"]
        for prec, per_n in chosen.items():
            for n, sched in per_n.items():
                old["schedules"].setdefault(prec, {})[n] = sched
                old.setdefault("refined", {}).setdefault(prec, {})[n] = gains[prec][n]
        old["timings"] += [{"name": r["name"], **{p: {"kernel_ms_per_grad": e["kernel_ms_per_grad"],
                                                      "kinds_ms_per_grad": e["kinds_ms_per_grad"]}
                                                  for p, e in r["precisions"].items()}} for r in results]
        with open(TUNED_JSON, "w") as f:
            json.dump(old, f, indent=1)
        write_header(old["schedules"], defaults)
        for prec in PRECISIONS:
            for n, g in sorted(gains.get(prec, {}).items(), key=lambda kv: int(kv[0])):
                print(prec, n, "refined:", {k: (v["default"], "->", v["value"]) for k, v in g.items()})
        print("merged into", TUNED_JSON, "and wrote", TUNED_HPP)
        return
    for r in results:
        if r["param"] is None:
            for prec, e in r["precisions"].items():
                defaults.setdefault(prec, {})[str(r["n"])] = {k: v for k, v in e["schedule"].items() if k != "radix"}
    rejected = [{"name": r["name"], "precision": p, "check": e["check"]} for r in results
                for p, e in r["precisions"].items() if e.get("ok") is False]
    doc = {"what": "kernel schedule per precision and grid size, chosen by autotune.py from per-kernel HIP-event "
                   "times on the benchmark's synthetic problem at each grid size",
           "measured_on": meta, "margin": MARGIN, "schedules": chosen, "defaults": defaults, "gains": gains,
           "rejected": rejected,
           "timings": [{"name": r["name"], **{p: {"kernel_ms_per_grad": e["kernel_ms_per_grad"],
                                                  "kinds_ms_per_grad": e["kinds_ms_per_grad"]}
                                              for p, e in r["precisions"].items()}} for r in results]}
    with open(TUNED_JSON, "w") as f:
        json.dump(doc, f, indent=1)
    write_header(chosen, defaults)
    for prec in PRECISIONS:
        for n, g in sorted(gains.get(prec, {}).items(), key=lambda kv: int(kv[0])):
            print(prec, n, {k: (v["default"], "->", v["value"], "%.4f->%.4f ms" % (v["default_ms_per_grad"],
                                                                                    v["ms_per_grad"]))
                            for k, v in g.items()})
    print("wrote", TUNED_JSON, "and", TUNED_HPP)


def cmd_verify(args):
    """Records, from a `time --only default --current` run, the combined
    schedule's kernel time per gradient beside the default's."""
    with open(args.file) as f:
        d = json.load(f)
    by_n = {}
    for r in d["results"]:
        by_n.setdefault(r["n"], {})["default" if r["param"] is None else r["param"]] = r
    with open(TUNED_JSON) as f:
        doc = json.load(f)
    ver = {}
    for n, rs in sorted(by_n.items()):
        if "default" not in rs or "current" not in rs:
            continue
        for prec in PRECISIONS:
            a, b = rs["default"]["precisions"].get(prec), rs["current"]["precisions"].get(prec)
            if a is None or b is None:
                continue
            ver.setdefault(prec, {})[str(n)] = {
                "default_ms_per_grad": a["kernel_ms_per_grad"], "tuned_ms_per_grad": b["kernel_ms_per_grad"],
                "change": round(b["kernel_ms_per_grad"] / a["kernel_ms_per_grad"] - 1.0, 4),
                "gradient_check": b.get("check"), "ok": b.get("ok")}
            print(prec, n, ver[prec][str(n)])
    doc["verified"] = ver
    with open(TUNED_JSON, "w") as f:
        json.dump(doc, f, indent=1)


def cmd_header(args):
    with open(TUNED_JSON) as f:
        doc = json.load(f)
    write_header(doc["schedules"], doc["defaults"])
    print("wrote", TUNED_HPP)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    b = sub.add_parser("build")
    b.add_argument("--grids", type=int, nargs="+", default=list(GRIDS))
    b.add_argument("--jobs", type=int, default=4)
    b.add_argument("--refine", action="store_true", help="moves from the tuned schedules, not the defaults")
    b.add_argument("--params", nargs="+", default=None, help="only these parameters (%s)" % ", ".join(PARAMS))
    t = sub.add_parser("time")
    t.add_argument("--out", required=True)
    t.add_argument("--grids", type=int, nargs="+", default=list(GRIDS))
    t.add_argument("--only", nargs="+", default=None, help="candidate names (or 'default')")
    t.add_argument("--current", action="store_true", help="also time the package's library")
    t.add_argument("--timeout", type=float, default=150.0)
    m = sub.add_parser("measure")
    m.add_argument("--n", type=int, required=True)
    m.add_argument("--ref", default=None)
    m.add_argument("--save-ref", action="store_true")
    m.add_argument("--precisions", nargs="+", default=list(PRECISIONS))
    s = sub.add_parser("select")
    s.add_argument("files", nargs="+")
    s.add_argument("--refine", action="store_true", help="merge a sweep from the tuned schedules")
    v = sub.add_parser("verify")
    v.add_argument("file")
    sub.add_parser("header")
    args = ap.parse_args(argv)
    if args.cmd == "build":
        return cmd_build(args)
    if args.cmd == "time":
        return cmd_time(args)
    if args.cmd == "measure":
        return measure(args.n, args.ref, args.save_ref, args.precisions)
    if args.cmd == "select":
        return cmd_select(args)
    if args.cmd == "verify":
        return cmd_verify(args)
    return cmd_header(args)


if __name__ == "__main__":
    main()

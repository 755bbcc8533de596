"""The kernel schedule: the library's query, the autotuner's committed cache
and the selection rule (host only, no GPU)."""
import json
import os

import pytest

from paper_2203_02369_amd import autotune, hamlet

GRIDS = (16, 32, 64, 128, 256, 512, 1024)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("n", GRIDS)
def test_schedule_query_is_consistent(n, prec):
    s = hamlet.schedule(n, prec)
    radices = [int(r) for r in s["radix"].split("x")]
    prod = 1
    for r in radices:
        assert r in (2, 4, 8, 16)
        prod *= r
    assert prod == n
    assert 0 <= s["radix_plan"] < autotune.radix_plans(n)
    for k in ("threads_xy", "threads_x", "threads_gather", "threads_scatter"):
        assert s[k] % 64 == 0 and 64 <= s[k] <= 1024
    # FP32 moves the strided tiles two columns at a time
    assert (n // 2) % s["tile_width"] == 0 and s["tile_width"] >= (2 if prec == "fp32" else 1)
    assert s["pencils_scatter"] % 2 == 0 and 2 <= s["pencils_scatter"] <= 8
    assert s["pencils_gather"] % 2 == 0 and 2 <= s["pencils_gather"] <= 16


def test_schedule_query_rejects_bad_arguments():
    from paper_2203_02369_amd import _capi
    lib = _capi.load()
    out = _capi.Schedule()
    import ctypes
    assert lib.hamlet_schedule_get(1, 48, ctypes.byref(out)) == -4
    assert lib.hamlet_schedule_get(7, 64, ctypes.byref(out)) == -1
    assert lib.hamlet_schedule_get(1, 64, None) == -1


def test_library_runs_the_committed_schedules():
    """The built library holds what tuned_schedules.json chose."""
    if not os.path.exists(autotune.TUNED_JSON):
        pytest.skip("no autotuned schedules committed")
    with open(autotune.TUNED_JSON) as f:
        doc = json.load(f)
    for prec, per_n in doc["schedules"].items():
        for n, sched in per_n.items():
            got = hamlet.schedule(int(n), prec)
            for field, value in sched.items():
                assert got[field] == value, (prec, n, field)


def _result(name, n, param, value, scheds, kinds, ok=True):
    prec = {}
    for p, (sched, times) in scheds.items():
        prec[p] = {"schedule": dict(sched), "kinds_ms_per_grad": dict(zip(kinds, times)),
                   "kernel_ms_per_grad": sum(times)}
        if param is not None:
            prec[p]["ok"] = ok
    return {"name": name, "n": n, "param": param, "value": value, "precisions": prec}


BASE = {"threads_xy": 256, "threads_x": 512, "threads_gather": 256, "threads_scatter": 256, "tile_width": 16,
        "pencils_scatter": 8, "pencils_gather": 8, "radix_plan": 0, "radix": "16x16"}


def test_selection_takes_gains_above_the_margin_only():
    kinds = autotune.KINDS
    t0 = [0.05, 0.10, 0.20, 0.05, 0.30, 0.10, 0.30]   # bin, inv_y, gather, like, scatter, fwd_y, x

    def with_(**kw):
        s = dict(BASE)
        s.update(kw)
        return s

    def times(**kw):
        t = dict(zip(kinds, t0))
        t.update(kw)
        return [t[k] for k in kinds]

    res = [
        _result("d", 256, None, None, {"fp32": (BASE, t0)}, kinds),
        # the x pass 10% faster with 1024 threads: taken
        _result("x", 256, "X", 1024, {"fp32": (with_(threads_x=1024), times(fwd_x=0.27))}, kinds),
        # the scatter 1% faster: inside the margin, not taken
        _result("zs", 256, "ZS", 512, {"fp32": (with_(threads_scatter=512), times(fwd_z_scatter=0.297))}, kinds),
        # the scatter 10% faster with 4-pencil tiles (kernels disjoint from the x pass): taken
        _result("pz", 256, "PZ", -1, {"fp32": (with_(pencils_scatter=4), times(fwd_z_scatter=0.27))}, kinds),
        # the gather much faster but the gradient differs: rejected
        _result("pg", 256, "PG", 1, {"fp32": (with_(pencils_gather=16), times(inv_z_gather=0.1))}, kinds, ok=False),
        # a shift clamped back to the default schedule: ignored
        _result("w", 256, "W", 1, {"fp32": (BASE, times(inv_y=0.05))}, kinds),
        # a narrower tile: faster y passes and x pass (5% on them), but it
        # shapes the x pass, which the larger gain above already changed
        _result("w2", 256, "W", -1, {"fp32": (with_(tile_width=8), times(inv_y=0.095, fwd_y=0.095, fwd_x=0.285))},
                kinds),
    ]
    chosen, gains = autotune.select(res)
    s = chosen["fp32"]["256"]
    assert s["threads_x"] == 1024
    assert s["threads_scatter"] == 256
    assert s["pencils_scatter"] == 4
    assert s["pencils_gather"] == 8
    assert s["tile_width"] == 16
    assert set(gains["fp32"]["256"]) == {"X", "PZ"}
    # a radix plan faster over the transforms as a whole shapes every
    # transform kernel: with the larger gain it is taken alone
    res.append(_result("r", 256, "RADIX", 2, {"fp32": (with_(radix_plan=2, radix="16x4x4"),
                                                       times(inv_y=0.08, fwd_y=0.08, fwd_x=0.26))}, kinds))
    chosen, gains = autotune.select(res)
    s = chosen["fp32"]["256"]
    assert s["radix_plan"] == 2 and s["threads_x"] == 512 and s["pencils_scatter"] == 8
    assert set(gains["fp32"]["256"]) == {"RADIX"}


def test_header_lists_only_changed_fields(tmp_path, monkeypatch):
    hpp = tmp_path / "tuned.hpp"
    monkeypatch.setattr(autotune, "TUNED_HPP", str(hpp))
    base = {k: v for k, v in BASE.items() if k != "radix"}
    chosen = {"fp32": {"256": dict(base, threads_x=1024)}, "fp64": {"256": dict(base)}}
    autotune.write_header(chosen, {"fp32": {"256": base}, "fp64": {"256": base}})
    text = hpp.read_text()
    assert "struct Tuned<float, 256> : DefaultSched<float, 256>" in text
    assert "static constexpr int X = 1024;" in text
    assert "Tuned<double" not in text

"""Autotuner for the subdivision parameters (g, r, B), beside the cost model.

The paper searches {g, r, B} by measurement (Sec. 6.2) and predicts the best
values with its cost model (Sec. 4.3). This module does both for a window on
the GPU:

* ``sweep`` renders the window once per candidate (the kernel's own device
  time, best of ``reps``) and records the counters of the render;
* ``fit_model`` fits the two unknowns of the time model to the measurements:
  the split cost lambda (S = lambda A) and the seconds per model time unit,
  with P the measured split probability and q = CUs, c = 64 lanes;
* ``tune`` returns the measured optimum and the model optimum, and caches the
  measured choice in a JSON file keyed by the workload class;
* ``fit_model_v2`` and ``guided_search``: the model with measured GPU
  overheads (a split probability per level, read as a function of the
  region side, and a per-region scheduling cost sigma) fitted to a few
  pilot renders, then used as a prior: only the parameters it ranks best
  are measured;
* ``compare_schemes`` measures one region per wave for leaf work (SBR, Sec.
  4.3.1) against leaves shared by several waves as row bands (MBR, Sec.
  4.3.2) at several band sizes, beside the model's T_MBR / T_SBR.

Run ``python -m paper_2206_02255_amd.autotune --size 16384 --dwell 2048`` for
the sweep of the paper's window.
"""
import argparse
import json
import math
import os
import sys

import numpy as np

from . import ask, costmodel

PAPER_OPTIMA = {
    "abstract (cost model)": "g in [2, 16], r in {2, 4}, B ~ 32",
    "conclusions (cost model)": "g in [2, 64], r ~ 2, B ~ 32",
    "experiments, ASK-SBR": "{g, r, B} = {32 or 64, 4, 16}",
    "experiments, ASK-MBR": "{g, r, B} = {32 or 64, 2, 32}",
}


def default_grid(n):
    """(g, r, B) candidates for an n-pixel side: g and B powers of two,
    r in {2, 4, 8}, keeping at least one split level."""
    out = []
    for g in (2, 4, 8, 16, 32, 64, 128, 256):
        for r in (2, 4, 8):
            for B in (16, 32, 64, 128):
                if g <= n and n // g > B:
                    out.append((g, r, B))
    return out


def sweep(ctx, win, grid, form="persistent", reps=3, out=None):
    """Measure every (g, r, B) of ``grid`` on window ``win`` (an ask_window).
    Returns one dict per candidate: g, r, B, ms (kernel device time, best of
    reps), iterations, P (measured split probability) and the counters."""
    import torch
    stream = torch.cuda.current_stream().cuda_stream
    if out is None:
        out = torch.empty(win.W * win.H, dtype=torch.int32, device="cuda")
    ask.ask_enable_timing(ctx, True)
    rows = []
    try:
        for g, r, B in grid:
            prm = ask.params(g, r, B, form)
            st = ask.ask_dwell_subdiv(ctx, win, prm, out.data_ptr(), stream, want_stats=True)
            best = math.inf
            for _ in range(reps):
                ask.ask_dwell_subdiv(ctx, win, prm, out.data_ptr(), stream)
                best = min(best, ask.ask_last_kernel_ms(ctx))
            rows.append({"g": g, "r": r, "B": B, "ms": best,
                         "iterations": st["iters_ring"] + st["iters_leaf"],
                         "P": costmodel.split_probability(st),
                         "P_levels": costmodel.split_probabilities(st),
                         "regions": sum(st["regions"]), "levels": st["levels"]})
    finally:
        ask.ask_enable_timing(ctx, False)
        ask.ask_synchronize(ctx, stream)
    return rows


def compare_schemes(ctx, win, g, r, B, bands=(ask.BAND_NONE, 4096, 1024, 256), reps=5, q=256,
                    c=64, lam=1.0, form="persistent"):
    """Render of ``win`` in ``form`` with (g, r, B) for every leaf band size of
    ``bands`` (ask.BAND_NONE: SBR, each leaf on the wave that decides it;
    others: MBR, leaves above that many pixels shared out as row bands). Returns
    the measured kernel times (best and median of ``reps``) and the cost
    model's T_SBR and T_MBR for the same parameters, with P measured here."""
    import torch
    stream = torch.cuda.current_stream().cuda_stream
    out = torch.empty(win.W * win.H, dtype=torch.int32, device="cuda")
    ask.ask_enable_timing(ctx, True)
    rows = []
    P = None
    try:
        for band in bands:
            prm = ask.params(g, r, B, form, band)
            st = ask.ask_dwell_subdiv(ctx, win, prm, out.data_ptr(), stream, want_stats=True)
            P = costmodel.split_probability(st)
            ms = []
            for _ in range(reps):
                ask.ask_dwell_subdiv(ctx, win, prm, out.data_ptr(), stream)
                ms.append(ask.ask_last_kernel_ms(ctx))
            ms.sort()
            rows.append({"band": "none (SBR)" if band == ask.BAND_NONE else int(band),
                         "best_ms": ms[0], "median_ms": ms[len(ms) // 2]})
    finally:
        ask.ask_enable_timing(ctx, False)
        ask.ask_synchronize(ctx, stream)
    n, A = float(max(win.W, win.H)), float(win.D)
    t_sbr = float(costmodel.time_sbr(n, g, r, B, A, P, lam, q, c))
    t_mbr = float(costmodel.time_mbr(n, g, r, B, A, P, lam, q, c))
    sbr = rows[0]["best_ms"] if bands[0] == ask.BAND_NONE else None
    best_mbr = min((row["best_ms"] for row in rows if row["band"] != "none (SBR)"), default=None)
    return {"g": g, "r": r, "B": B, "form": form, "P": P, "lambda": lam, "rows": rows,
            "model": {"T_SBR": t_sbr, "T_MBR": t_mbr, "T_MBR/T_SBR": t_mbr / t_sbr},
            "measured": {"best_MBR/SBR": (best_mbr / sbr) if sbr and best_mbr else None}}


def fit_model(rows, n, A, q, c=64, lambdas=None):
    """Fit lambda and the seconds per model unit so that kappa * T_SBR(g, r, B)
    matches the measured times in the least-squares sense of log time. P is
    the median of the measured split probabilities (the SSD assumption of one
    P for the problem). Returns (lambda, kappa, P, relative rms error)."""
    if lambdas is None:
        lambdas = [0.0] + list(np.logspace(-1, 5, 25))
    P = float(np.median([row["P"] for row in rows]))
    g = np.array([row["g"] for row in rows], dtype=np.float64)
    r = np.array([row["r"] for row in rows], dtype=np.float64)
    B = np.array([row["B"] for row in rows], dtype=np.float64)
    t = np.log(np.array([row["ms"] for row in rows]))
    best = None
    for lam in lambdas:
        m = np.log(costmodel.time_sbr(n, g, r, B, A, P, lam, q, c))
        k = float(np.mean(t - m))
        err = float(np.sqrt(np.mean((t - m - k) ** 2)))
        if best is None or err < best[3]:
            best = (float(lam), math.exp(k), P, err)
    return best


def fit_model_v2(rows, n, A, q, c=64, lambdas=None, sigmas=None):
    """Fit lambda, sigma and the seconds per model unit (kappa) to measured
    rows (each with its own per-level P_levels, over the levels the render
    has), least squares in log time.
    Returns (lambda, sigma, kappa, relative rms error)."""
    lambdas = np.geomspace(0.01, 1e5, 36) if lambdas is None else lambdas
    sigmas = np.concatenate(([0.0], np.geomspace(1.0, 1e8, 33))) if sigmas is None else sigmas
    y = np.log([row["ms"] for row in rows])
    levels = [costmodel.rendered_levels(n, row["g"], row["r"], row["B"]) for row in rows]
    best = None
    for lam in lambdas:
        for sig in sigmas:
            m = np.log([costmodel.time_sbr_levels(n, row["g"], row["r"], row["B"], A,
                                                  row["P_levels"] or [0.0], lam, q, c, sig, L)
                        for row, L in zip(rows, levels)])
            k = float(np.mean(y - m))
            err = float(np.sqrt(np.mean((y - m - k) ** 2)))
            if best is None or err < best[3]:
                best = (float(lam), float(sig), math.exp(k), err)
    return best


def guided_search(measure, grid, n, A, q, c=64, pilot=8, top=8):
    """The model as a prior for the search over ``grid``: measure ``pilot``
    evenly spaced candidates (measure(list of (g, r, B)) -> rows as ``sweep``
    returns), fit P(side) from their per-level split probabilities and
    lambda, sigma, kappa from their times, predict every candidate, and
    measure the ``top`` best predicted ones not yet measured. Returns the
    measured rows, the best of them, the fit and the predicted order."""
    grid = [tuple(p) for p in grid]
    step = max(1, len(grid) // max(1, pilot))
    first = grid[::step][:pilot]
    rows = list(measure(first))
    points = [(s, p) for row in rows
              for s, p in zip(costmodel.level_sides(
                  n, row["g"], row["r"], row["B"],
                  costmodel.rendered_levels(n, row["g"], row["r"], row["B"])), row["P_levels"])]
    curve = costmodel.split_curve(points) if points else (lambda s: 0.0)
    lam, sig, kappa, err = fit_model_v2(rows, n, A, q, c)
    pred = {p: kappa * costmodel.predict_sbr(n, *p, A, curve, lam, q, c, sig) for p in grid}
    order = sorted(grid, key=lambda p: pred[p])
    seen = {(row["g"], row["r"], row["B"]) for row in rows}
    more = [p for p in order if p not in seen][:top]
    rows += list(measure(more))
    best = min(rows, key=lambda row: row["ms"])
    return {"rows": rows, "measured": len(rows), "best": {k: best[k] for k in ("g", "r", "B", "ms")},
            "fit": {"lambda": lam, "sigma": sig, "seconds_per_unit": kappa * 1e-3,
                    "log_rms": err},
            "predicted_order": [list(p) for p in order[:top + pilot]],
            "predicted_ms": {"%d,%d,%d" % p: pred[p] for p in order[:top + pilot]}}


def model_optimum(grid, n, A, P, lam, q, c=64, scheme="sbr"):
    """The (g, r, B) of ``grid`` that the time model ranks fastest."""
    g, r, B = (np.array([p[i] for p in grid], dtype=np.float64) for i in range(3))
    f = costmodel.time_sbr if scheme == "sbr" else costmodel.time_mbr
    t = f(n, g, r, B, A, P, lam, q, c)
    i = int(np.argmin(t))
    return tuple(int(v) for v in grid[i]), float(t[i])


# The measured choices of the workload classes tuned so far, kept beside the
# package so that every run of the benchmark reads the same choices.
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")

TILES = [(4, 16), (8, 8), (16, 4), (32, 2), (64, 1)]


def cache_path():
    return os.environ.get("ASK_TUNE_CACHE", DEFAULT_CACHE)


def load_cache(path=None):
    path = path or cache_path()
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def store(key, entry, path=None):
    """Record the measured choice of one workload class in the cache."""
    path = path or cache_path()
    cache = load_cache(path)
    cache[key] = entry
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)


def lookup(key, path=None):
    """The cached choice of a workload class, or None."""
    return load_cache(path).get(key)


def workload_key(win, form):
    width = max(win.x1 - win.x0, win.y1 - win.y0)
    return "%dx%d-D%d-w1e%d-%s" % (win.W, win.H, win.D, int(math.floor(math.log10(width))), form)


def _median_ms(ctx, render, reps):
    import torch
    stream = torch.cuda.current_stream().cuda_stream
    render()
    ask.ask_synchronize(ctx, stream)
    ask.ask_enable_timing(ctx, True)
    try:
        for _ in range(reps):
            render()
        ms = sorted(ask.ask_kernel_times(ctx))
    finally:
        ask.ask_enable_timing(ctx, False)
        ask.ask_synchronize(ctx, stream)
    return ms[len(ms) // 2]


def tile_sweep(ctx, win, g, r, B, form="persistent", tiles=None, reps=5, out=None):
    """Kernel time (median of reps) of the subdivision render of ``win`` with
    (g, r, B) for each wave tile (the block-size study of Sec. 6.2): (0, 0),
    the default row order of leaf pixels, then every tile of ``tiles``."""
    import torch
    stream = torch.cuda.current_stream().cuda_stream
    if out is None:
        out = torch.empty(win.W * win.H, dtype=torch.int32, device="cuda")
    rows = []
    for tile in [(0, 0)] + list(tiles or TILES):
        prm = ask.params(g, r, B, form, 0, tile)
        ms = _median_ms(ctx, lambda: ask.ask_dwell_subdiv(ctx, win, prm, out.data_ptr(), stream),
                        reps)
        rows.append({"tile": list(tile), "ms": ms})
    return rows


def exhaustive_tile_sweep(ctx, win, tiles=None, reps=3, out=None):
    """Kernel time (median of reps) of the exhaustive image of ``win`` for each
    wave tile."""
    import torch
    stream = torch.cuda.current_stream().cuda_stream
    if out is None:
        out = torch.empty(win.W * win.H, dtype=torch.int32, device="cuda")
    rows = []
    for tile in list(tiles or TILES):
        ms = _median_ms(ctx, lambda: ask.ask_dwell_exhaustive(ctx, win, out.data_ptr(), stream,
                                                              tile=tile), reps)
        rows.append({"tile": list(tile), "ms": ms})
    return rows


def batch_rule_sweep(ctx, images, rules, reps=1):
    """Kernel time of the batch of ``images`` (workloads.Window) in one
    persistent launch for each per-image parameter rule of ``rules``: dicts
    with s0 (level-0 region side: g = side // s0, clamped to [1, 256]), r, B
    and tile. Returns the rules with their times, fastest first."""
    import numpy as np
    import torch
    import workloads
    stream = torch.cuda.current_stream().cuda_stream
    sizes = [w.pixels for w in images]
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    out = torch.empty(int(sum(sizes)), dtype=torch.int32, device="cuda")
    ptrs = [out.data_ptr() + 4 * int(o) for o in offs]
    wins = [ask.window(w) for w in images]
    rows = []
    for rule in rules:
        prms = []
        for w in images:
            p = workloads.rule_params(w.W, rule["s0"], rule["r"], rule["B"])
            prms.append(ask.params(p.g, p.r, p.B, "persistent", 0, rule.get("tile", (0, 0))))
        ms = _median_ms(ctx, lambda: ask.ask_dwell_batch(ctx, wins, prms, ptrs, stream), reps)
        rows.append(dict(rule, ms=ms))
    del out
    return sorted(rows, key=lambda row: row["ms"])


def tune(ctx, win, grid=None, form="persistent", reps=3, q=256, use_cache=True):
    """Measured optimum (g, r, B) for window ``win``, from the cache when it
    holds this workload class, else from a sweep (then cached). Returns a
    dict with the measured optimum, the model optimum and the sweep rows."""
    key = workload_key(win, form)
    if use_cache:
        hit = lookup(key)
        if hit is not None and "rows" in hit:
            return hit
    grid = grid or default_grid(min(win.W, win.H))
    rows = sweep(ctx, win, grid, form, reps)
    n = min(win.W, win.H)
    lam, kappa, P, err = fit_model(rows, n, float(win.D), q)
    best = min(rows, key=lambda row: row["ms"])
    (mg, mr, mB), _ = model_optimum(grid, n, float(win.D), P, lam, q)
    measured_at_model = next(row["ms"] for row in rows if (row["g"], row["r"], row["B"]) == (mg, mr, mB))
    result = {"key": key, "form": form,
              "measured_optimum": {"g": best["g"], "r": best["r"], "B": best["B"], "ms": best["ms"]},
              "model_optimum": {"g": mg, "r": mr, "B": mB, "ms_measured": measured_at_model},
              "model_fit": {"lambda": lam, "seconds_per_unit": kappa * 1e-3, "P": P,
                            "log_rms_error": err, "q": q, "c": 64},
              "rows": rows}
    if use_cache:
        store(key, result)
    return result


BATCH_KEY = "batch-256-seed4-persistent"


def tune_class(ctx, name, log=print):
    """Measure the choices of one workload class of the benchmark and store
    them in the cache: ``large`` (the paper's window at 16384^2, D = 2048) and
    ``deep`` (the deep zoom at 32768^2, D = 8192): (g, r, B), then the wave
    tile of the subdivision's leaves and of the exhaustive kernel; ``batch``
    (256 boundary images): the per-image rule (level-0 region side, r, B),
    then its wave tile."""
    import torch
    import workloads
    if name == "batch":
        ims = workloads.batch_images()
        rules = [{"s0": s0, "r": r, "B": B, "tile": [0, 0]}
                 for s0 in (128, 256, 512) for r in (2, 4) for B in (32, 64, 128)]
        rows = batch_rule_sweep(ctx, ims, rules)
        for row in rows[:5]:
            log("batch rule %s" % row)
        best = dict(rows[0])
        trows = batch_rule_sweep(ctx, ims, [dict(best, tile=list(t)) for t in TILES])
        for row in trows:
            log("batch tile %s" % row)
        if trows[0]["ms"] < best["ms"]:
            best = dict(trows[0])
        entry = {"rule": {k: best[k] for k in ("s0", "r", "B", "tile")}, "ms": best["ms"],
                 "rows": rows, "tile_rows": trows}
        store(BATCH_KEY, entry)
        return BATCH_KEY, entry
    if name == "large":
        w, reps = workloads.LARGE, 5
        grid = [(g, r, B) for g in (16, 32, 64, 128) for r in (2, 4) for B in (16, 32, 64)]
    elif name == "deep":
        w, reps = workloads.deep_window(), 1
        grid = [(g, r, B) for g in (32, 64, 128) for r in (2, 4) for B in (32, 64, 128)]
    else:
        raise ValueError(name)
    win = ask.window(w)
    out = torch.empty(w.W * w.H, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    rows = []
    for g, r, B in grid:
        prm = ask.params(g, r, B, "persistent")
        ms = _median_ms(ctx, lambda: ask.ask_dwell_subdiv(ctx, win, prm, out.data_ptr(), stream),
                        reps)
        rows.append({"g": g, "r": r, "B": B, "ms": ms})
        log("%s g=%d r=%d B=%d %.3f ms" % (name, g, r, B, ms))
    rows.sort(key=lambda row: row["ms"])
    best = rows[0]
    trows = tile_sweep(ctx, win, best["g"], best["r"], best["B"], "persistent", reps=reps, out=out)
    for row in trows:
        log("%s leaf tile %s %.3f ms" % (name, row["tile"], row["ms"]))
    tbest = min(trows, key=lambda row: row["ms"])
    erows = exhaustive_tile_sweep(ctx, win, reps=max(1, min(3, reps)), out=out)
    for row in erows:
        log("%s exhaustive tile %s %.3f ms" % (name, row["tile"], row["ms"]))
    ebest = min(erows, key=lambda row: row["ms"])
    key = workload_key(win, "persistent")
    entry = {"g": best["g"], "r": best["r"], "B": best["B"], "tile": tbest["tile"],
             "ms": tbest["ms"], "exhaustive_tile": ebest["tile"], "exhaustive_ms": ebest["ms"],
             "rows": rows, "tile_rows": trows, "exhaustive_tile_rows": erows}
    store(key, entry)
    del out
    return key, entry


VOLUME_GRID = [(32, 2, 8), (32, 2, 16), (16, 2, 16), (64, 2, 8), (16, 4, 8), (64, 2, 4),
               (16, 2, 8), (32, 4, 4), (8, 2, 16), (64, 2, 16)]


def volume_sweep(v, grid=VOLUME_GRID, curve="morton", reps=7, log=print):
    """Kernel time (median of reps renders, HIP events on the stream) of the
    3-D subdivision volume for each (g, r, B) of grid, and of the exhaustive
    volume, with the voxels where each subdivision volume differs from the
    exhaustive one."""
    import torch
    vol = ask.volume(v)
    sp = torch.cuda.current_stream().cuda_stream
    out = torch.empty(v.voxels, dtype=torch.int32, device="cuda")
    ex = torch.empty(v.voxels, dtype=torch.int32, device="cuda")
    wk = torch.empty(ask.EXHAUSTIVE3_WORK_BYTES, dtype=torch.uint8, device="cuda")

    def timed(fn):
        ms = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            ms.append(a.elapsed_time(b))
        return sorted(ms)[len(ms) // 2]

    def exf():
        ask.ask3_dwell_exhaustive(vol, ex.data_ptr(), wk.data_ptr(), stream=sp)
    exf()
    res = {"exhaustive_ms": timed(exf), "rows": []}
    log("exhaustive %.3f ms" % res["exhaustive_ms"])
    for g, r, B in grid:
        prm = ask.params3(g, r, B, curve)
        nb = ask.ask3_workspace_bytes(vol, prm)
        work = torch.empty(nb, dtype=torch.uint8, device="cuda")
        st = ask.ask3_dwell_subdiv(vol, prm, out.data_ptr(), work.data_ptr(), nb, sp,
                                   want_stats=True)

        def fn():
            ask.ask3_dwell_subdiv(vol, prm, out.data_ptr(), work.data_ptr(), nb, sp)
        row = {"g": g, "r": r, "B": B, "ms": timed(fn), "regions": st["regions"],
               "differ": int((out != ex).sum().item())}
        res["rows"].append(row)
        log("(%d, %d, %d) %.3f ms, regions %s, voxels differing %d"
            % (g, r, B, row["ms"], row["regions"], row["differ"]))
        del work
    return res


def main(argv=None):
    import torch
    ap = argparse.ArgumentParser(description="(g, r, B) sweep on the paper's window")
    ap.add_argument("--tune", default=None, nargs="+", choices=["large", "deep", "batch"],
                    help="measure the benchmark's workload classes and store their choices in "
                         "the cache (ASK_TUNE_CACHE, default tuned.json beside the package)")
    ap.add_argument("--size", type=int, default=16384)
    ap.add_argument("--dwell", type=int, default=2048)
    ap.add_argument("--form", default="persistent", choices=["levels", "persistent"])
    ap.add_argument("--grid", default="paper", choices=["paper", "wide"])
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--json", default=None, help="write the result here")
    ap.add_argument("--schemes", default=None, metavar="G,R,B",
                    help="compare SBR and MBR leaf work for these parameters instead")
    ap.add_argument("--prior", default=None, nargs="+", metavar="PILOT,TOP",
                    help="also run the model-guided search (PILOT pilot renders, then the TOP "
                         "best predicted) against the full sweep's measurements, for each pair")
    ap.add_argument("--volume", action="store_true",
                    help="sweep (g, r, B) of the 3-D subdivision of the benchmark's volume")
    ap.add_argument("--window", default="paper", choices=["paper", "deep", "julia"],
                    help="--schemes: the paper's window (--size, --dwell), the deep zoom "
                         "or the Julia-set workload")
    args = ap.parse_args(argv)
    import workloads
    from workloads import LARGE_SWEEP, paper_window
    if args.volume:
        res = volume_sweep(workloads.VOLUME, log=lambda m: print(m, flush=True))
        if args.json:
            with open(args.json, "w") as f:
                json.dump(res, f, indent=1)
        return
    if args.tune:
        ctx = ask.ask_create(0)
        try:
            for name in args.tune:
                key, entry = tune_class(ctx, name, log=lambda m: print(m, flush=True))
                print(json.dumps({key: {k: v for k, v in entry.items() if not k.endswith("rows")}}),
                      flush=True)
        finally:
            ask.ask_destroy(ctx)
        return
    w = {"paper": lambda: paper_window(args.size, args.dwell), "deep": workloads.deep_window,
         "julia": lambda: workloads.JULIA}[args.window]()
    if args.schemes:
        g, r, B = (int(x) for x in args.schemes.split(","))
        ctx = ask.ask_create(0)
        try:
            props = torch.cuda.get_device_properties(0)
            res = compare_schemes(ctx, ask.window(w), g, r, B, reps=args.reps,
                                  q=props.multi_processor_count, form=args.form)
        finally:
            ask.ask_destroy(ctx)
        for row in res["rows"]:
            print("band %-12s best %8.3f ms  median %8.3f ms" %
                  (row["band"], row["best_ms"], row["median_ms"]), flush=True)
        print(json.dumps({k: res[k] for k in ("g", "r", "B", "P", "model", "measured")}))
        if args.json:
            with open(args.json, "w") as f:
                json.dump(res, f, indent=1)
        return
    grid = ([(p.g, p.r, p.B) for p in LARGE_SWEEP] if args.grid == "paper"
            else default_grid(args.size))
    ctx = ask.ask_create(0)
    try:
        props = torch.cuda.get_device_properties(0)
        res = tune(ctx, ask.window(w), grid, args.form, args.reps,
                   q=props.multi_processor_count, use_cache=False)
    finally:
        ask.ask_destroy(ctx)
    res["paper_optima"] = PAPER_OPTIMA
    if args.prior:
        n, A = float(max(w.W, w.H)), float(w.D)
        q = torch.cuda.get_device_properties(0).multi_processor_count
        by_p = {(row["g"], row["r"], row["B"]): row for row in res["rows"]}
        full_best = min(res["rows"], key=lambda row: row["ms"])
        res["guided"] = []
        for pair in args.prior:
            pilot, top = (int(x) for x in pair.split(","))
            g_res = guided_search(lambda ps: [by_p[tuple(p)] for p in ps], grid, n, A, q,
                                  pilot=pilot, top=top)
            res["guided"].append({"pilot": pilot, "top": top, "measured": g_res["measured"],
                                  "best": g_res["best"], "fit": g_res["fit"],
                                  "best_over_full_sweep_best": g_res["best"]["ms"] / full_best["ms"],
                                  "predicted_order": g_res["predicted_order"]})
        lam2, sig2, kap2, err2 = fit_model_v2(res["rows"], n, A, q)
        res["full_sweep"] = {"size": len(res["rows"]),
                             "best": {k: full_best[k] for k in ("g", "r", "B", "ms")}}
        res["model_v2_fit_all"] = {"lambda": lam2, "sigma": sig2,
                                   "seconds_per_unit": kap2 * 1e-3, "log_rms": err2}
        print(json.dumps({k: res[k] for k in ("guided", "full_sweep", "model_v2_fit_all")}))
    for row in sorted(res["rows"], key=lambda row: row["ms"])[:10]:
        print("g=%3d r=%d B=%3d  %8.3f ms  P=%.3f  iterations=%d" %
              (row["g"], row["r"], row["B"], row["ms"], row["P"], row["iterations"]), flush=True)
    print(json.dumps({k: res[k] for k in ("measured_optimum", "model_optimum", "model_fit")}))
    if args.json:
        with open(args.json, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    main()

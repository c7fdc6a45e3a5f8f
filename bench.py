#!/usr/bin/env python3
"""Benchmark on one MI355X: Mandelbrot dwell image of the paper's window
[-1.5, 0.5] x [-1, 1] at 16384 x 16384 pixels, maximum dwell 2048, binary64.

One step renders the whole image by Mariani-Silver subdivision in the chosen
form (persistent queue kernel by default): level-0 seeding, border queries,
fills, splits and per-pixel leaves. Inputs (the window) are on the device
before the timed region starts; the image stays in HBM.

Printed as one JSON line:
  value      effective Mpix/s of the subdivision render (W*H / wall time)
  roofline   the dominant kernel against the FP64 vector peak: 8 flops per
             dwell iteration actually computed, over the kernel's own device
             time (HIP events recorded by the library on the render's stream)
  forms      the exhaustive kernel and the per-level (ASK) form on the same
             image, for the speedups; the batched workload (256 images of
             uneven size and zoom centred on boundary points, one
             persistent launch) against the same images rendered one by
             one; the served workload (Poisson arrivals into the server
             kernel) with p50/p99 latency, against sequential per-level
             renders of the same requests
  cpu_baseline  the CPU oracle rendering the same full image on the host
             cores; its image is compared with the GPU image bit for bit
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpix/s + % FP64 vector peak; exhaustive vs ASK vs batched; bit-exact dwell"
PEAK_FP64_TFLOPS = 78.6      # MI355X vector FP64, FMA counted as 2 flops
FLOPS_PER_ITERATION = 8      # 3 multiplies + 5 adds of z <- z^2 + c and |z|^2


PROFILE = os.path.join(ROOT, "profiles", "persistent_kernel_mandelbrot16384_D2048.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2206_02255_amd", "csrc", f)
                  for f in ("ask_kernels.hip", "ask_internal.hpp")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled(key):
    """A per-launch figure of the persistent kernel from the committed counter
    runs (HBM traffic, FP64 instructions), or None when the kernel sources
    have changed since they were taken."""
    try:
        fields = dict(line.split(": ", 1) for line in open(PROFILE).read().splitlines()
                      if line.startswith((key + ":", "kernel_source_sha256:")))
    except (OSError, ValueError):
        return None
    if fields.get("kernel_source_sha256", "").strip() != kernel_source_hash() or key not in fields:
        return None
    return int(fields[key])


def log(msg):
    """Progress on stderr (the JSON result is the only stdout line)."""
    print("bench: " + msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--form", default=None, choices=["levels", "levels_readback", "persistent"])
    ap.add_argument("--g", type=int, default=None)
    ap.add_argument("--r", type=int, default=None)
    ap.add_argument("--B", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-count", type=int, default=256,
                    help="images of the batched workload (0: skip it)")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--no-deep", action="store_true", help="skip the deep-zoom image")
    ap.add_argument("--no-julia", action="store_true", help="skip the Julia-set image")
    ap.add_argument("--no-volume", action="store_true", help="skip the 3-D volume")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="first copy BYTES of device memory once (a plain copy kernel of known "
                         "size, to scale the memory-traffic counters of a profile)")
    ap.add_argument("--serve-seconds", type=float, default=2.0,
                    help="seconds of Poisson arrivals (200/s) for the served workload (0: skip it)")
    return ap.parse_args()


def batched_leg(ctx, torch, ask, autotune, workloads, sp, count, steps):
    """The batched workload (256 boundary images) captured whole into a HIP
    graph and replayed, one persistent launch per replay, with the per-image
    (g, r, B) rule and wave tile the autotuner chose for it; against the same
    images rendered one at a time (persistent, then per-level form)."""
    import numpy as np
    ims = workloads.batch_images(count=count)
    hit = autotune.lookup(autotune.BATCH_KEY) if count == 256 else None
    rule = hit["rule"] if hit else {"s0": 256, "r": 2, "B": 128, "tile": [0, 0]}
    prms = [workloads.rule_params(w.W, rule["s0"], rule["r"], rule["B"]) for w in ims]
    tile = tuple(rule["tile"])
    sizes = [w.pixels for w in ims]
    total = sum(sizes)
    offs = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    ptrs = [out.data_ptr() + 4 * int(o) for o in offs]
    wins = [ask.window(w) for w in ims]
    pers = [ask.params(p.g, p.r, p.B, "persistent", 0, tile) for p in prms]
    log("batched: %d images, %.2f Gpix, rule %s; counting pass" % (count, total / 1e9, rule))
    st = ask.ask_dwell_batch(ctx, wins, pers, ptrs, sp, want_stats=True)
    iters = st["iters_ring"] + st["iters_leaf"]
    eager_img = out.clone()
    # The whole batch as one graph: image table, counter reset, queue clear,
    # seeding and the persistent kernel.
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        ask.ask_dwell_batch(ctx, wins, pers, ptrs, torch.cuda.current_stream().cuda_stream)
    log("batched: captured")
    replay_stream = torch.cuda.current_stream()
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    out.zero_()
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks[0].record(replay_stream)
    for k in range(steps):
        graph.replay()
        marks[k + 1].record(replay_stream)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    replay_ms = sorted(marks[k].elapsed_time(marks[k + 1]) for k in range(steps))
    kms = replay_ms[len(replay_ms) // 2]
    replay_same = bool(torch.equal(out, eager_img))
    log("batched: %d replays done" % steps)
    ask.ask_synchronize(ctx, sp)
    del graph

    def one_by_one(form, params, tile_=(0, 0)):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for w, p, ptr in zip(wins, params, ptrs):
            ask.ask_dwell_subdiv(ctx, w, ask.params(p.g, p.r, p.B, form, 0, tile_), ptr, sp)
        torch.cuda.synchronize()
        ask.ask_synchronize(ctx, sp)
        return 1e3 * (time.perf_counter() - t)

    # The same images and parameters one at a time must give the batch's images.
    seq_pers_ms = one_by_one("persistent", prms, tile)
    log("batched: one by one (persistent) done")
    same = bool(torch.equal(out, eager_img))
    seq_lv_same_ms = one_by_one("levels", prms, tile)
    log("batched: one by one (levels, same parameters) done")
    same = same and bool(torch.equal(out, eager_img))
    # The per-level form also with smaller leaves (B = 32); its baseline is the
    # faster of the two.
    lv_prms = [workloads.batch_params_levels(w.W) for w in ims]
    seq_lv_small_ms = one_by_one("levels", lv_prms)
    log("batched: one by one (levels, B = 32) done")
    seq_lv_ms = min(seq_lv_same_ms, seq_lv_small_ms)
    del out, eager_img
    return {"workload": "batch-%d-boundary-images" % count, "images": count, "pixels": total,
            "rule": rule, "params_source": "autotuner cache" if hit else "default",
            "graph_replay": True,
            "ms": round(ms, 3), "mpix_s": round(total / (ms * 1e-3) / 1e6, 1),
            "replay_ms_median": round(kms, 3), "dwell_iterations": iters,
            "fp64_frac": round(FLOPS_PER_ITERATION * iters / (kms * 1e-3) / 1e12
                               / PEAK_FP64_TFLOPS, 4),
            "replays_equal_eager_batch": replay_same,
            "one_by_one_persistent_ms": round(seq_pers_ms, 3),
            "one_by_one_levels_ms": round(seq_lv_ms, 3),
            "one_by_one_levels_same_params_ms": round(seq_lv_same_ms, 3),
            "one_by_one_levels_b32_ms": round(seq_lv_small_ms, 3),
            "speedup_vs_one_by_one_levels": round(seq_lv_ms / ms, 2),
            "equals_one_by_one": same}


def deep_leg(ctx, torch, ask, autotune, workloads, sp):
    """The deep-zoom image (32768^2, width 1e-6 around a boundary point,
    D = 8192) with the autotuner's choice for its class: exhaustive kernel,
    persistent and per-level subdivision."""
    w = workloads.deep_window()
    win = ask.window(w)
    hit = autotune.lookup(autotune.workload_key(win, "persistent"))
    if hit and "tile" in hit:
        g, r, B, tile, ex_tile = hit["g"], hit["r"], hit["B"], tuple(hit["tile"]), tuple(
            hit["exhaustive_tile"])
    else:
        p = workloads.DEEP_PARAMS
        g, r, B, tile, ex_tile = p.g, p.r, p.B, (0, 0), (16, 4)
    out = torch.empty(w.W * w.H, dtype=torch.int32, device="cuda")

    def timed(fn, reps):
        ask.ask_enable_timing(ctx, True)
        for _ in range(reps):
            fn()
        ms = sorted(ask.ask_kernel_times(ctx, cap=reps))
        ask.ask_enable_timing(ctx, False)
        return ms[len(ms) // 2]

    log("deep: %s, exhaustive" % (w,))
    ex_ms = timed(lambda: ask.ask_dwell_exhaustive(ctx, win, out.data_ptr(), sp, tile=ex_tile), 1)
    ex_iters = int(out.to(torch.int64).sum().item())
    ex = out.clone()
    res = {"workload": "mandelbrot-deep-32768x32768-D8192-width1e-6", "g": g, "r": r, "B": B,
           "tile": list(tile), "params_source": "autotuner cache" if hit else "default",
           "exhaustive": {"kernel_ms": round(ex_ms, 2), "tile": list(ex_tile),
                          "dwell_iterations": ex_iters,
                          "fp64_frac": round(FLOPS_PER_ITERATION * ex_iters / (ex_ms * 1e-3) / 1e12
                                             / PEAK_FP64_TFLOPS, 4)}}
    for form in ("persistent", "levels"):
        log("deep: %s" % form)
        prm = ask.params(g, r, B, form, 0, tile)
        st = ask.ask_dwell_subdiv(ctx, win, prm, out.data_ptr(), sp, want_stats=True)
        iters = st["iters_ring"] + st["iters_leaf"]
        ms = timed(lambda: ask.ask_dwell_subdiv(ctx, win, prm, out.data_ptr(), sp), 3)
        res[form] = {"kernel_ms": round(ms, 2), "dwell_iterations": iters,
                     "mpix_s": round(w.pixels / (ms * 1e-3) / 1e6, 1),
                     "fp64_frac": round(FLOPS_PER_ITERATION * iters / (ms * 1e-3) / 1e12
                                        / PEAK_FP64_TFLOPS, 4),
                     "speedup_vs_exhaustive": round(ex_ms / ms, 3),
                     "pixels_differing_from_exhaustive": int((out != ex).sum().item())}
    ask.ask_synchronize(ctx, sp)
    del out, ex
    return res


def julia_leg(ctx, torch, ask, workloads, sp, steps):
    """The filled Julia set of c = -1 at 16384^2, D = 2048 (the second
    escape-time workload of the class): exhaustive kernel, persistent and
    per-level subdivision with the single-image parameters."""
    w, p = workloads.JULIA, workloads.JULIA_PARAMS
    win = ask.window(w)
    out = torch.empty(w.W * w.H, dtype=torch.int32, device="cuda")
    log("julia: %s, exhaustive" % (w,))
    ask.ask_enable_timing(ctx, True)
    ask.ask_dwell_exhaustive(ctx, win, out.data_ptr(), sp)
    ex_ms = []
    for _ in range(3):
        ask.ask_dwell_exhaustive(ctx, win, out.data_ptr(), sp)
        ex_ms.append(ask.ask_last_kernel_ms(ctx))
    ex_ms = min(ex_ms)
    ex_iters = int(out.to(torch.int64).sum().item())
    ex = out.clone()
    res = {"workload": "julia-basilica-16384x16384-D2048", "c": list(w.julia),
           "window": [w.x0, w.x1, w.y0, w.y1], "g": p.g, "r": p.r, "B": p.B,
           "exhaustive": {"kernel_ms": round(ex_ms, 3), "dwell_iterations": ex_iters,
                          "fp64_frac": round(FLOPS_PER_ITERATION * ex_iters / (ex_ms * 1e-3) / 1e12
                                             / PEAK_FP64_TFLOPS, 4)}}
    images = {}
    for form in ("persistent", "levels"):
        log("julia: %s" % form)
        prm = ask.params(p.g, p.r, p.B, form)
        st = ask.ask_dwell_subdiv(ctx, win, prm, out.data_ptr(), sp, want_stats=True)
        iters = st["iters_ring"] + st["iters_leaf"]
        ms = []
        for _ in range(max(3, steps)):
            ask.ask_dwell_subdiv(ctx, win, prm, out.data_ptr(), sp)
            ms.append(ask.ask_last_kernel_ms(ctx))
        ms.sort()
        med = ms[len(ms) // 2]
        res[form] = {"kernel_ms": round(med, 3), "dwell_iterations": iters,
                     "mpix_s": round(w.pixels / (med * 1e-3) / 1e6, 1),
                     "fp64_frac": round(FLOPS_PER_ITERATION * iters / (med * 1e-3) / 1e12
                                        / PEAK_FP64_TFLOPS, 4),
                     "speedup_vs_exhaustive": round(ex_ms / med, 2),
                     "work_reduction": round(ex_iters / iters, 2),
                     "pixels_differing_from_exhaustive": int((out != ex).sum().item())}
        images[form] = out.clone()
    res["levels_equals_persistent"] = bool(torch.equal(images["levels"], images["persistent"]))
    ask.ask_enable_timing(ctx, False)
    ask.ask_synchronize(ctx, sp)
    del out, ex, images
    return res


# binary64 operations of one quaternion Julia iteration: 5 products (three
# squares, two cross terms), 7 sums for the new parts, 2 sums for the squared
# modulus (its squares are the next iteration's).
FLOPS_PER_QUAT_ITERATION = 14


def volume_leg(torch, ask, workloads, sp, steps):
    """The 3-D extension: the quaternion Julia volume of c = -0.2 + 0.6i at
    512^3 voxels, D = 256, exhaustive and level-by-level subdivision with
    both curves."""
    v, p = workloads.VOLUME, workloads.VOLUME_PARAMS
    vol = ask.volume(v)
    out = torch.empty(v.voxels, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    def timed(fn, n):
        ms = []
        for _ in range(n):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            b.synchronize()
            ms.append(a.elapsed_time(b))
        ms.sort()
        return ms[len(ms) // 2]

    log("volume: %s, exhaustive" % (v,))
    ex_work = torch.empty(ask.EXHAUSTIVE3_WORK_BYTES, dtype=torch.uint8, device="cuda")
    ex_fn = lambda: ask.ask3_dwell_exhaustive(vol, out.data_ptr(), ex_work.data_ptr(),  # noqa: E731
                                              stream=sp)
    ex_fn()
    ex_ms = timed(ex_fn, max(3, steps))
    ex_iters = int(out.to(torch.int64).sum().item())
    ex = out.clone()
    res = {"workload": "quaternion-julia-512^3-D256", "c": list(v.c),
           "box": [v.x0, v.x1, v.y0, v.y1, v.z0, v.z1], "g": p.g, "r": p.r, "B": p.B,
           "exhaustive": {"ms": round(ex_ms, 3), "dwell_iterations": ex_iters,
                          "mvox_s": round(v.voxels / (ex_ms * 1e-3) / 1e6, 1),
                          "fp64_frac": round(FLOPS_PER_QUAT_ITERATION * ex_iters / (ex_ms * 1e-3)
                                             / 1e12 / PEAK_FP64_TFLOPS, 4)}}
    for curve in ("canonical", "morton"):
        log("volume: subdivision, %s curve" % curve)
        prm = ask.params3(p.g, p.r, p.B, curve)
        nbytes = ask.ask3_workspace_bytes(vol, prm)
        work = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        st = ask.ask3_dwell_subdiv(vol, prm, out.data_ptr(), work.data_ptr(), nbytes, sp,
                                   want_stats=True)
        fn = lambda: ask.ask3_dwell_subdiv(vol, prm, out.data_ptr(), work.data_ptr(),  # noqa: E731
                                           nbytes, sp)
        ms = timed(fn, max(3, steps))
        res[curve] = {"ms": round(ms, 3), "mvox_s": round(v.voxels / (ms * 1e-3) / 1e6, 1),
                      "speedup_vs_exhaustive": round(ex_ms / ms, 2),
                      "levels": st["levels"], "regions": st["regions"],
                      "voxels_differing_from_exhaustive": int((out != ex).sum().item())}
        del work
    del out, ex
    return res


def served_leg(ctx, ask, workloads, seconds):
    """Poisson arrivals at 200/s into the server kernel, and the same requests
    rendered back to back by the per-level form."""
    from paper_2206_02255_amd import serve
    sched = workloads.serving_requests(seconds=seconds)
    params_of = lambda w: workloads.batch_params(w.W)  # noqa: E731
    log("served: %d requests over %.1f s" % (len(sched), seconds))
    res = serve.serve(ctx, sched, params_of, slots=64, log=log)
    res.pop("images")
    res.pop("probes")
    log("served: done; sequential per-level renders of the same requests")
    # The per-level form back to back, with the serving parameters and with
    # smaller leaves (B = 32); the baseline is the faster of the two.
    seq = {}
    for name, rule in (("same_params", params_of),
                       ("b32", lambda w: workloads.batch_params_levels(w.W))):
        seq[name] = serve.sequential(ctx, [w for _, w in sched], rule, "levels")
        log("served: sequential per-level (%s) done" % name)
    res["sequential_levels_mpix_s"] = round(res["pixels"] / min(seq.values()) / 1e6, 1)
    for name, sec in seq.items():
        res["sequential_levels_%s_mpix_s" % name] = round(res["pixels"] / sec / 1e6, 1)
    res["arrival_seconds"] = seconds
    for k in ("offered_mpix_s", "achieved_mpix_s", "makespan_s", "latency_p50_ms",
              "latency_p99_ms", "latency_max_ms"):
        res[k] = round(res[k], 3)
    return res


def tuned_large(workloads, ask, autotune):
    """(form, g, r, B, tile, exhaustive tile, source) of the main image: the
    autotuner's cached choice for its workload class, else the defaults."""
    p = workloads.LARGE_DEFAULT
    hit = autotune.lookup(autotune.workload_key(ask.window(workloads.LARGE), "persistent"))
    if hit and "tile" in hit:
        return ("persistent", hit["g"], hit["r"], hit["B"], tuple(hit["tile"]),
                tuple(hit["exhaustive_tile"]), "autotuner cache")
    return (workloads.LARGE_DEFAULT_FORM, p.g, p.r, p.B, (0, 0), (16, 4), "default")


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the method needs no cross-GPU exchange, and "
              "the benchmark runs and reports a single MI355X (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2206_02255_amd import ask, autotune
    import workloads

    w = workloads.LARGE
    form, g, r, B, tile, ex_tile, source = tuned_large(workloads, ask, autotune)
    if args.form or args.g or args.r or args.B:
        form, g, r, B = args.form or form, args.g or g, args.r or r, args.B or B
        source = "command line"
    win = ask.window(w)
    prm = ask.params(g, r, B, form, 0, tile)
    pixels = w.W * w.H

    if args.copy_calibration:
        src = torch.ones(args.copy_calibration // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: %d bytes read and written" % (src.numel() * 4))
        del src, dst

    ctx = ask.ask_create(0)
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    out = torch.empty(pixels, dtype=torch.int32, device="cuda")

    def render(prm_=prm):
        ask.ask_dwell_subdiv(ctx, win, prm_, out.data_ptr(), sp)

    # Work counters of this render (untimed): dwell iterations computed.
    st = ask.ask_dwell_subdiv(ctx, win, prm, out.data_ptr(), sp, want_stats=True)
    iters = st["iters_ring"] + st["iters_leaf"]

    log("main: %s, form %s, (g, r, B) = (%d, %d, %d), tile %s (%s)"
        % (w, form, g, r, B, tile, source))
    for _ in range(args.warmup):
        render()
    ask.ask_synchronize(ctx, sp)
    # The timed steps: the library records HIP events around the dominant
    # kernel of every render on its stream, and torch events between the
    # steps give each step's span on the same stream.
    ask.ask_enable_timing(ctx, True)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks[0].record(stream)
    for k in range(args.steps):
        render()
        marks[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = sorted(ask.ask_kernel_times(ctx, cap=args.steps))
    ask.ask_enable_timing(ctx, False)
    ask.ask_synchronize(ctx, sp)
    ms_step = 1e3 * wall / args.steps
    step_ms = sorted(marks[k].elapsed_time(marks[k + 1]) for k in range(args.steps))
    kernel_ms = kms[len(kms) // 2]
    step_median = step_ms[len(step_ms) // 2]

    # The same image by the exhaustive kernel and by the per-level form.
    def timed(fn, reps):
        fn()
        ask.ask_enable_timing(ctx, True)
        for _ in range(reps):
            fn()
        ms = sorted(ask.ask_kernel_times(ctx, cap=reps))
        ask.ask_enable_timing(ctx, False)
        return ms[len(ms) // 2]

    gpu_img = out.clone()
    ex_ms = timed(lambda: ask.ask_dwell_exhaustive(ctx, win, out.data_ptr(), sp, tile=ex_tile), 3)
    ex_iters = int(out.to(torch.int64).sum().item())
    mismatch = int((out != gpu_img).sum().item())
    lv_prm = ask.params(g, r, B, "levels", 0, tile)
    lv_ms = timed(lambda: render(lv_prm), 5)
    same_forms = bool(torch.equal(out, gpu_img))
    ask.ask_synchronize(ctx, sp)

    result = {
        "metric": METRIC,
        "value": round(pixels / (ms_step * 1e-3) / 1e6, 1),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "mandelbrot-dwell-16384x16384-D2048",
                   "window": [w.x0, w.x1, w.y0, w.y1], "W": w.W, "H": w.H, "D": w.D,
                   "form": form, "g": g, "r": r, "B": B, "tile": list(tile),
                   "params_source": source},
        "roofline": {"bound": "alu", "kernel": "persistent_kernel" if form == "persistent"
                     else "level_kernel",
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "traffic": profiled("traffic_bytes_per_launch")
                     if (form, g, r, B, tile) == ("persistent", 64, 4, 16, (0, 0)) else None,
                     "fp64_wave_instructions": profiled("fp64_wave_instructions_per_launch")
                     if (form, g, r, B, tile) == ("persistent", 64, 4, 16, (0, 0)) else None,
                     "kernel_ms": round(kernel_ms, 4),
                     "kernel_ms_timed_steps": [round(x, 4) for x in kms],
                     "step_ms_median": round(step_median, 4),
                     "iterations_executed": iters},
        "mismatch_vs_exhaustive": mismatch,
        "forms": {
            "subdivision": {"form": form, "ms": round(ms_step, 4),
                            "mpix_s": round(pixels / (ms_step * 1e-3) / 1e6, 1)},
            "levels": {"kernel_ms": round(lv_ms, 4),
                       "mpix_s": round(pixels / (lv_ms * 1e-3) / 1e6, 1)},
            "exhaustive": {"kernel_ms": round(ex_ms, 4), "tile": list(ex_tile),
                           "mpix_s": round(pixels / (ex_ms * 1e-3) / 1e6, 1),
                           "dwell_iterations": ex_iters,
                           "fp64_frac": round(FLOPS_PER_ITERATION * ex_iters / (ex_ms * 1e-3)
                                              / 1e12 / PEAK_FP64_TFLOPS, 4)},
            "speedup_vs_exhaustive": round(ex_ms / ms_step, 2),
            "work_reduction": round(ex_iters / iters, 2),
            "levels_equals_chosen_form": same_forms,
        },
        "cpu_baseline": None,
    }

    def roofline(i_count, which):
        ach = FLOPS_PER_ITERATION * i_count / (kernel_ms * 1e-3) / 1e12
        result["roofline"].update({"achieved": round(ach, 2), "frac": round(ach / PEAK_FP64_TFLOPS, 4),
                                   "iterations_counted": which, "iterations": i_count})

    # Until the oracle's algorithmic count is known, the kernel's own count.
    roofline(iters, "executed by the kernel")
    log("main: done (%.3f ms per step)" % ms_step)
    if args.batch_count > 0:
        result["forms"]["batched"] = batched_leg(ctx, torch, ask, autotune, workloads, sp,
                                                 args.batch_count, args.batch_steps)
    if args.serve_seconds > 0:
        result["forms"]["served"] = served_leg(ctx, ask, workloads, args.serve_seconds)
    if not args.no_deep:
        result["forms"]["deep"] = deep_leg(ctx, torch, ask, autotune, workloads, sp)
    if not args.no_julia:
        result["forms"]["julia"] = julia_leg(ctx, torch, ask, workloads, sp, args.steps)
    if not args.no_volume:
        result["forms"]["volume"] = volume_leg(torch, ask, workloads, sp, args.steps)

    if not args.no_cpu_baseline:
        import numpy as np
        from oracle import askref
        log("cpu baseline: the oracle on the full image")
        threads = os.cpu_count() or 1
        t0 = time.perf_counter()
        ref_img, ref_st = askref.subdiv(w, g, r, B, threads=threads)
        cpu_s = time.perf_counter() - t0
        gpu_np = gpu_img.cpu().numpy().view(np.uint32).reshape(w.H, w.W)
        result["cpu_baseline"] = {
            "value": round(pixels / cpu_s / 1e6, 2), "unit": "Mpix/s", "cores": threads,
            "kind": "oracle",
            "sample": "the full 16384x16384 image, same window, D and (g, r, B)",
            "seconds": round(cpu_s, 2)}
        result["bit_exact_vs_oracle"] = bool(np.array_equal(gpu_np, ref_img))
        # The method's algorithmic work (every scanned ring's dwells and every
        # leaf's), from the oracle: the roofline counts it.
        roofline(int(ref_st["iters_alg"]), "algorithmic (oracle)")
        result["roofline"]["frac_executed"] = round(
            FLOPS_PER_ITERATION * iters / (kernel_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4)

    ask.ask_destroy(ctx)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

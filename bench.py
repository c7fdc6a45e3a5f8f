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
             image, for the speedups
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
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the method needs no cross-GPU exchange, and "
              "this build runs and reports a single MI355X (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2206_02255_amd import ask
    import workloads

    w = workloads.LARGE
    p = workloads.LARGE_DEFAULT
    form = args.form or workloads.LARGE_DEFAULT_FORM
    g, r, B = args.g or p.g, args.r or p.r, args.B or p.B
    win = ask.window(w)
    prm = ask.params(g, r, B, form)
    pixels = w.W * w.H

    ctx = ask.ask_create(0)
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    out = torch.empty(pixels, dtype=torch.int32, device="cuda")

    def render(prm_=prm):
        ask.ask_dwell_subdiv(ctx, win, prm_, out.data_ptr(), sp)

    # Work counters of this render (untimed): dwell iterations computed.
    st = ask.ask_dwell_subdiv(ctx, win, prm, out.data_ptr(), sp, want_stats=True)
    iters = st["iters_ring"] + st["iters_leaf"]

    for _ in range(args.warmup):
        render()
    ask.ask_synchronize(ctx, sp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        render()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ask.ask_synchronize(ctx, sp)
    ms_step = 1e3 * wall / args.steps

    # Device time of the dominant kernel, per launch.
    ask.ask_enable_timing(ctx, True)
    kms = []
    for _ in range(args.steps):
        render()
        kms.append(ask.ask_last_kernel_ms(ctx))
    kernel_ms = sum(kms) / len(kms)
    achieved = FLOPS_PER_ITERATION * iters / (kernel_ms * 1e-3) / 1e12

    # The same image by the exhaustive kernel and by the per-level form.
    def timed(fn, reps):
        fn()
        ms = []
        for _ in range(reps):
            fn()
            ms.append(ask.ask_last_kernel_ms(ctx))
        return min(ms)

    gpu_img = out.clone()
    ex_ms = timed(lambda: ask.ask_dwell_exhaustive(ctx, win, out.data_ptr(), sp), 2)
    ex_iters = int(out.to(torch.int64).sum().item())
    lv_prm = ask.params(g, r, B, "levels")
    lv_ms = timed(lambda: render(lv_prm), 5)
    same_forms = bool(torch.equal(out, gpu_img))
    ask.ask_enable_timing(ctx, False)
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
                   "form": form, "g": g, "r": r, "B": B},
        "roofline": {"bound": "alu", "kernel": "persistent_kernel" if form == "persistent"
                     else "level_kernel", "achieved": round(achieved, 2),
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": None,
                     "kernel_ms": round(kernel_ms, 4), "dwell_iterations": iters},
        "forms": {
            "subdivision": {"form": form, "ms": round(ms_step, 4),
                            "mpix_s": round(pixels / (ms_step * 1e-3) / 1e6, 1)},
            "levels": {"kernel_ms": round(lv_ms, 4),
                       "mpix_s": round(pixels / (lv_ms * 1e-3) / 1e6, 1)},
            "exhaustive": {"kernel_ms": round(ex_ms, 4),
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

    if not args.no_cpu_baseline:
        import numpy as np
        from oracle import askref
        threads = os.cpu_count() or 1
        t0 = time.perf_counter()
        ref_img, _ = askref.subdiv(w, g, r, B, threads=threads)
        cpu_s = time.perf_counter() - t0
        gpu_np = gpu_img.cpu().numpy().view(np.uint32).reshape(w.H, w.W)
        result["cpu_baseline"] = {
            "value": round(pixels / cpu_s / 1e6, 2), "unit": "Mpix/s", "cores": threads,
            "kind": "oracle",
            "sample": "the full 16384x16384 image, same window, D and (g, r, B)",
            "seconds": round(cpu_s, 2)}
        result["bit_exact_vs_oracle"] = bool(np.array_equal(gpu_np, ref_img))

    ask.ask_destroy(ctx)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

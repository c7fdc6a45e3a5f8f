"""Serving loop over the server kernel (include/ask.h, serving).

Replays a schedule of render requests in real time: each request arrives at
its time, waits in a first-come first-served backlog until its output fits
the output arena (device memory set aside for results: admission by free
HBM) and the server accepts it (a free slot and room for its region queue in
the server's pool), then runs on the device together with every other
admitted request. Latency is measured from arrival to the host seeing the
request finished; throughput over the whole run.

The output arena is allocated once before the server starts, so nothing
allocates or frees device memory while the server kernel runs (a free
would wait for every kernel on the device, the server's included).
"""
import collections
import time

import numpy as np

from . import ask


class FirstFit:
    """First-fit allocation of ranges of [0, size), merging freed neighbours."""

    def __init__(self, size):
        self.free = [(0, size)] if size else []

    def alloc(self, n):
        for k, (off, size) in enumerate(self.free):
            if size >= n:
                if size == n:
                    self.free.pop(k)
                else:
                    self.free[k] = (off + n, size - n)
                return off
        return None

    def release(self, off, n):
        self.free.append((off, n))
        self.free.sort()
        merged = []
        for o, s in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((o, s))
        self.free = merged


class Arena(FirstFit):
    """FirstFit over the uint32 words of one device tensor."""

    def __init__(self, torch, words):
        super().__init__(words)
        self.t = torch.empty(words, dtype=torch.int32, device="cuda")

    def ptr(self, off):
        return self.t.data_ptr() + 4 * off


def serve(ctx, schedule, params_of, slots=64, arena_bytes=16 << 30, pool_bytes=1 << 30,
          keep=None, log=None, limit_s=120.0, probe=None):
    """Run `schedule` [(arrival_s, window)] through a server on ctx.

    params_of(window) -> workloads.Params. keep(i) -> True to copy request
    i's image to the host (returned in 'images'). probe(i, image) is called
    with request i's finished image (a flat device tensor view, valid only
    during the call); its results are returned in 'probes'. Raises
    TimeoutError when the run lasts limit_s beyond the last arrival. Returns
    a dict of the run's measurements."""
    import torch
    arena = Arena(torch, arena_bytes // 4)
    torch.cuda.current_stream().synchronize()
    sv = ask.ask_server_create(ctx, slots=slots, pool_bytes=pool_bytes)
    backlog = collections.deque()
    inflight = {}
    lat, peak, images, failed, probes = [], 0, {}, 0, {}
    done_px = 0
    n = len(schedule)
    i = 0
    t0 = time.perf_counter()
    last_log = t0
    try:
        deadline = (schedule[-1][0] if n else 0.0) + limit_s
        while i < n or backlog or inflight:
            now = time.perf_counter() - t0
            if now > deadline:
                raise TimeoutError("serving did not finish: %d of %d done, %d in flight"
                                   % (len(lat), n, len(inflight)))
            while i < n and schedule[i][0] <= now:
                backlog.append(i)
                i += 1
            while backlog:  # first come, first served
                j = backlog[0]
                w = schedule[j][1]
                off = arena.alloc(w.pixels)
                if off is None:
                    break
                p = params_of(w)
                t = ask.ask_server_submit(sv, ask.window(w), ask.params(p.g, p.r, p.B), arena.ptr(off))
                if t is None:
                    arena.release(off, w.pixels)
                    break
                inflight[t] = (j, off)
                backlog.popleft()
            peak = max(peak, len(inflight))
            for t, st in ask.ask_server_reap(sv):
                j, off = inflight.pop(t)
                w = schedule[j][1]
                lat.append(time.perf_counter() - t0 - schedule[j][0])
                done_px += w.pixels
                failed += st != 0
                if keep is not None and keep(j):
                    images[j] = arena.t[off:off + w.pixels].cpu().numpy().view(np.uint32).reshape(w.H, w.W)
                if probe is not None:
                    probes[j] = probe(j, arena.t[off:off + w.pixels])
                arena.release(off, w.pixels)
            if log and time.perf_counter() - last_log > 5.0:
                last_log = time.perf_counter()
                log("serve: %.0f s, %d of %d arrived, %d done, %d in flight, %d waiting"
                    % (last_log - t0, i, n, len(lat), len(inflight), len(backlog)))
            if not inflight and not backlog and i < n:
                time.sleep(max(0.0, min(schedule[i][0] - (time.perf_counter() - t0), 0.001)))
            else:
                time.sleep(20e-6)
        makespan = time.perf_counter() - t0
    finally:
        ask.ask_server_destroy(sv)
    lat = np.array(lat) if lat else np.zeros(1)
    total_px = sum(w.pixels for _, w in schedule)
    span = schedule[-1][0] if schedule else 0.0
    return {"requests": n, "failed": int(failed), "pixels": int(total_px),
            "offered_mpix_s": total_px / max(span, 1e-9) / 1e6,
            "achieved_mpix_s": total_px / makespan / 1e6, "makespan_s": makespan,
            "latency_p50_ms": float(np.percentile(lat, 50) * 1e3),
            "latency_p99_ms": float(np.percentile(lat, 99) * 1e3),
            "latency_max_ms": float(lat.max() * 1e3),
            "peak_in_flight": peak, "slots": slots, "images": images, "probes": probes}


def sequential(ctx, windows, params_of, form="levels"):
    """Render the windows one after another (each alone, on the current
    stream), as a plain per-level ASK service would; returns the device
    time in seconds, from the first render's start to the last one's end."""
    import torch
    s = torch.cuda.current_stream()
    biggest = max(w.pixels for w in windows)
    out = torch.empty(biggest, dtype=torch.int32, device="cuda")
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(s)
    for w in windows:
        p = params_of(w)
        ask.ask_dwell_subdiv(ctx, ask.window(w), ask.params(p.g, p.r, p.B, form), out.data_ptr(),
                             s.cuda_stream)
    b.record(s)
    b.synchronize()
    ask.ask_synchronize(ctx, s.cuda_stream)
    return a.elapsed_time(b) / 1e3

"""Tuning and load helpers of the batched decoder and the request server.

The block length D changes which bits the decoder returns (Sec. III-A: a PB
sees only L stages beyond its decoded range), so the tuners only choose among
the candidate D values given to them, with L fixed by the caller (about 6K
keeps the error rate at the full-frame level, Sec. V); results are compared
with the oracle run with the chosen D and L.  D at least the longest frame
decodes every frame as one block (full-frame Viterbi).

Throughput tuning times pbvd_batch_decode on the device; latency tuning
drives a pbvd_server with Poisson arrivals and takes the 99th percentile."""
from __future__ import annotations

import time

import numpy as np

from . import datagen, pbvd


def time_batch(torch, codes, frames, syms_dev, out_dev, reps: int = 5, warmup: int = 2):
    """Median seconds of one pbvd_batch_decode of `frames` with `codes`,
    and the batch's work-list statistics."""
    with pbvd.Batch(codes) as b:
        b.set_frames(frames, syms_dev.numel(), out_dev.numel())
        for _ in range(warmup):
            b.decode(syms_dev, out_dev)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            b.decode(syms_dev, out_dev)
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        ts.sort()
        return ts[len(ts) // 2], b.info()


def lanes_allowed(code, lanes: int) -> bool:
    """Lane-group widths the library supports for a code (16-bit metrics,
    at least 16 packed registers per lane; 64 lanes, the state-parallel
    mapping, takes any code)."""
    if lanes in (1, 64):
        return True
    return (code.get("pm_bits", 16) == 16 and lanes in (2, 4, 8)
            and (1 << (code["K"] - 2)) // lanes >= 16)


# Layouts the batch tuner tries: (name, lanes_per_pb, mapping).  "lanes1"
# and "lanes2": the register kernel with one or two lanes per PB (codes that
# do not take two keep one), one tile launch per code; "wave": the
# state-parallel kernel, one persistent launch per K over all its codes;
# "group": the paper's group mapping, 2^R lanes per PB.
BATCH_LAYOUTS = (("lanes1", 1, 1), ("lanes2", 2, 1), ("wave", 64, 2), ("group", 0, 3))


def layout_codes(codes, d, layout):
    """codes with block length d and one of BATCH_LAYOUTS."""
    name, lanes, mapping = layout
    out = []
    for c in codes:
        l = lanes if mapping != 1 or lanes_allowed(c, lanes) else 1
        out.append(dict(c, D=int(d), lanes_per_pb=l, mapping=mapping))
    return out


def tune_batch_d(torch, codes, frames, syms_dev, out_dev,
                 d_candidates=(48, 64, 96, 128, 160, 192, 224, 256, 320, 512),
                 layouts=BATCH_LAYOUTS, reps: int = 5, refine: int = 2):
    """One D for all codes and one layout per run (block length, and how a
    PB maps to lanes: the survivor layout follows from it), the fastest
    batched decode of `frames`: a coarse grid of D for every layout, then D
    in steps of 8 within 24 of the `refine` best (D, layout) pairs (the time
    is not smooth in D: the number of tiles against the number of SIMDs and
    each PB's trip alignment both change with it).  Returns (codes with D,
    lanes_per_pb and mapping filled in, [((D, layout name), seconds,
    info)])."""
    table = []
    seen = set()

    def run(d, layout):
        if (d, layout[0]) in seen or d < 8:
            return
        seen.add((d, layout[0]))
        t, info = time_batch(torch, layout_codes(codes, d, layout), frames, syms_dev, out_dev, reps=reps)
        table.append(((int(d), layout[0]), t, info))
    for layout in layouts:
        for d in d_candidates:
            run(int(d), layout)
    for (d, name), _, _ in sorted(table, key=lambda r: r[1])[:refine]:
        layout = next(l for l in layouts if l[0] == name)
        for dd in range(d - 24, d + 25, 8):
            run(dd, layout)
    (best_d, best_l) = min(table, key=lambda r: r[1])[0]
    layout = next(l for l in layouts if l[0] == best_l)
    return layout_codes(codes, best_d, layout), table


def tune_plan_lanes(torch, K, gens, D, L, syms_dev, n_bits, out_dev, reps: int = 5, **plan_kw):
    """The fastest lane-group width for decoding one stream with pbvd_decode.
    Returns (lanes, {lanes: seconds})."""
    res = {}
    for lanes in (1, 2, 4, 8):
        if not lanes_allowed(dict(K=K, **plan_kw), lanes):
            continue
        with pbvd.Plan(K, gens, D, L, lanes_per_pb=lanes, **plan_kw) as p:
            for _ in range(2):
                p.decode(syms_dev, n_bits, out=out_dev)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                p.decode(syms_dev, n_bits, out=out_dev)
            e1.record()
            e1.synchronize()
            res[lanes] = e0.elapsed_time(e1) * 1e-3 / reps
    return min(res, key=res.get), res


def serve_load(srv, pool, rate: float, seconds: float, seed: int = 1):
    """Submit requests drawn from `pool` ((code, stream) pairs) to a
    pbvd.Server at Poisson arrival times of the given rate for `seconds`,
    wait for all, and return latency percentiles (ms), decoded Mbps over
    the span from the first submission to the last completion, and the mean
    batch size."""
    rng = np.random.default_rng(seed)
    n = max(1, int(rate * seconds))
    arrivals = datagen.poisson_arrivals(rng, n, rate)
    pick = rng.integers(0, len(pool), size=n)
    tickets = []
    bits = 0
    start = time.perf_counter()
    for k in range(n):
        target = start + arrivals[k]
        while time.perf_counter() < target:
            pass
        ci, st = pool[pick[k]]
        tickets.append(srv.submit(ci, st["syms"], st["n"]))
        bits += st["n"]
    submitted = time.perf_counter()
    infos = [srv.wait(t)[1] for t in tickets]
    lat = np.array([i["latency_ns"] for i in infos], dtype=np.float64) / 1e6
    # queue wait: submission to the launch of the batch carrying the
    # request; service: that launch to the bits in the caller's buffer
    wait = np.array([i["start_ns"] - i["submit_ns"] for i in infos], dtype=np.float64) / 1e6
    service = np.array([i["done_ns"] - i["start_ns"] for i in infos], dtype=np.float64) / 1e6
    span = (max(i["done_ns"] for i in infos) - min(i["submit_ns"] for i in infos)) / 1e9
    return {"rate": rate, "requests": n, "offered_rate": round(n / (submitted - start), 1),
            "p50_ms": round(float(np.percentile(lat, 50)), 4),
            "p99_ms": round(float(np.percentile(lat, 99)), 4),
            "max_ms": round(float(lat.max()), 4),
            "queue_wait_p50_ms": round(float(np.percentile(wait, 50)), 4),
            "queue_wait_p99_ms": round(float(np.percentile(wait, 99)), 4),
            "service_p50_ms": round(float(np.percentile(service, 50)), 4),
            "service_p99_ms": round(float(np.percentile(service, 99)), 4),
            "mbps": round(bits / span / 1e6, 2),
            "mean_batch": round(float(np.mean([i["batch_frames"] for i in infos])), 2)}


def tune_server_d(codes, pool_for, rate: float, seconds: float = 0.5, d_candidates=(16, 32, 64),
                  **server_kw):
    """One D for all codes, the lowest p99 latency at `rate`.  pool_for(codes)
    returns the request pool for codes with D set.  Returns (codes with D
    filled in, [(D, load result)])."""
    table = []
    for d in d_candidates:
        cs = [dict(c, D=int(d)) for c in codes]
        with pbvd.Server(cs, **server_kw) as srv:
            pool = pool_for(cs)
            serve_load(srv, pool, rate, 0.1, seed=0)
            table.append((int(d), serve_load(srv, pool, rate, seconds, seed=1)))
    best = min(table, key=lambda r: r[1]["p99_ms"])[0]
    return [dict(c, D=best) for c in codes], table

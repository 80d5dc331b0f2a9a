#!/usr/bin/env python3
"""Throughput benchmark of the MI355X parallel block-based Viterbi decoder.

Workload (the plain-decoder throughput run): K=7 rate-1/2 code (171,133),
a stream of 2^27 random information bits, BPSK/AWGN at Eb/N0 = 3 dB, int8
soft inputs, D = 512, L = 42 (= 6K), int16 path metrics, zero-terminated.
One step = one pbvd_decode of the whole stream with inputs and outputs
resident in HBM.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("decoded Mbps, K=7 r1/2 soft, 1 MI355X (batched vs plain); serving p99 latency")
PEAK_ALU_OPS = {16: 78.6e12, 32: 39.3e12}  # 256 CU x 64 lanes x 2.4 GHz (x2 for packed 16-bit)
KERNEL_SOURCES = ["paper_1608_00066_amd/csrc/pbvd_kernel.hpp",
                  "paper_1608_00066_amd/csrc/pbvd_code_inst.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "decode_kernel_k7_d512_2p27_traffic.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def forward_stage_sum(plan, n_bits: int) -> int:
    geo = plan.block_geometry(n_bits)
    return int((geo[:, 1] - geo[:, 0]).sum())


def settle_clocks(torch, plan, syms, n_bits, out, seconds: float = 0.08) -> int:
    """Decode back to back for `seconds` of wall time, untimed.  The MI355X
    raises its clock over the first ~40 ms of sustained load (a 2^27-bit
    decode takes 1.1 ms at first, 0.83 ms from about the 40th on, and ramps
    again after 200 ms idle), so a short warm-up would time the ramp instead
    of the steady state.  Returns the number of decodes run."""
    stream = torch.cuda.current_stream()
    count = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(8):
            plan.decode(syms, n_bits, out=out, stream=stream)
        count += 8
        torch.cuda.synchronize()
    return count


def time_decode_graph(torch, plan, syms, n_bits, out, steps):
    """ms per decode when `steps` decodes are captured in one HIP graph and
    replayed (no host launch cost per decode: a short stream's decode is
    shorter than the Python call that launches it)."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    plan.decode(syms, n_bits, out=out)  # workspace allocated outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            for _ in range(steps):
                plan.decode(syms, n_bits, out=out, stream=side)
    torch.cuda.current_stream().wait_stream(side)
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.replay()
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / steps
    del g
    return ms


def time_decode(torch, plan, syms, n_bits, out, steps, warmup):
    """Warm-up, then `steps` timed decodes.  Returns (ms per step from the
    host clock between synchronizations, mean kernel ms from HIP events on
    the stream the decode kernel runs on)."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.decode(syms, n_bits, out=out, stream=stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, e in ev:
        s.record(stream)
        plan.decode(syms, n_bits, out=out, stream=stream)
        e.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kernel_ms = sum(s.elapsed_time(e) for s, e in ev) / steps
    return (t1 - t0) * 1e3 / steps, kernel_ms


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """Threads the oracle may use: the CPUs this process may run on."""
    try:
        return len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        return os.cpu_count() or 1


def cpu_baseline(st, K, gens, D, L, target_s: float, gpu_bits, batch_check=None):
    """The CPU oracle on a contiguous sample of the same stream's blocks
    (the whole stream when it fits about target_s), using every host core,
    plus a single-threaded leg on a smaller sample.  The multi-threaded
    leg's bits are compared with the GPU's output of the same blocks, and
    every frame of the batched decode (batch_check) with the oracle."""
    import numpy as np

    import oracle
    n = st["n"]
    threads = host_threads()
    nb_total = oracle.num_blocks(n, D)

    def calibrated(nthreads, budget_s, probe):
        probe = min(nb_total, probe)
        t0 = time.perf_counter()
        oracle.decode(K, gens, D, L, st["syms"], n, pb_first=0, pb_count=probe, nthreads=nthreads)
        dt = time.perf_counter() - t0
        return int(min(nb_total, max(probe, probe * budget_s / max(dt, 1e-3))))

    count = calibrated(threads, target_s, max(64, 8 * threads))
    t0 = time.perf_counter()
    res = oracle.decode(K, gens, D, L, st["syms"], n, pb_first=0, pb_count=count,
                        nthreads=threads)
    dt = time.perf_counter() - t0
    bits = res["bits"].size
    same = bool(np.array_equal(res["bits"], gpu_bits[:bits]))
    count1 = calibrated(1, target_s / 2, 64)
    t0 = time.perf_counter()
    r1 = oracle.decode(K, gens, D, L, st["syms"], n, pb_first=0, pb_count=count1, nthreads=1)
    dt1 = time.perf_counter() - t0
    bits1 = r1["bits"].size
    same = same and bool(np.array_equal(r1["bits"], gpu_bits[:bits1]))
    cpu = {"value": round(bits / dt / 1e6, 3), "unit": "Mbps", "cores": threads,
           "kind": "oracle",
           "sample": "first %d of %d parallel blocks (%d decoded bits) of the same stream, "
                     "%.1f s on %d threads" % (count, nb_total, bits, dt, threads),
           "single_thread": {"value": round(bits1 / dt1 / 1e6, 3), "unit": "Mbps", "cores": 1,
                             "sample": "first %d parallel blocks (%d decoded bits), %.1f s"
                                       % (count1, bits1, dt1)},
           "cpu_model": cpu_model()}
    parity = {"equal": same, "bits_compared": bits,
              "scope": "GPU output of the timed decode against the oracle, bit for bit, over "
                       "the first %d of %d parallel blocks" % (count, nb_total)}
    if batch_check is not None:
        parity["batched_equal"] = batch_matches_oracle(*batch_check)
        parity["batched_scope"] = "every frame of the batched decode (%d frames)" % len(batch_check[1])
    return cpu, parity


def plain_per_frame(torch, pbvd, codes, frames, syms, out, reps: int = 1):
    """Seconds of decoding every frame with its own pbvd_decode call (one
    launch per frame, one plan per code), median of `reps` passes."""
    import ctypes
    L = pbvd.lib()
    plans = [pbvd.Plan(c["K"], c["gens"], c["D"], c["L"]) for c in codes]
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    bs, bo = syms.data_ptr(), out.data_ptr()
    calls = [(ctypes.c_void_p(plans[ci].handle), ctypes.c_void_p(bs + so), n, ctypes.c_void_p(bo + oo))
             for (so, n, oo, ci) in frames]

    def one_pass():
        for h, sp, n, op in calls:
            if L.pbvd_decode(h, sp, n, op, stream) != 0:
                raise RuntimeError("pbvd_decode failed: " + pbvd.pbvd_last_error())
    one_pass()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        one_pass()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    for p in plans:
        p.close()
    return sorted(ts)[len(ts) // 2]


def bench_pipeline(torch, plan, st, n, kernel_mbps, reps: int = 3):
    """Host-buffer decoding of the same stream (pinned host memory) with
    N_s chunks on N_s streams, against the Eq. 7 estimate
    T/P = D N_t N_s / (T_H2D + N_s T_k + T_D2H) for chunks of N_t PBs."""
    from paper_1608_00066_amd import pbvd
    R, D, L = plan.R, plan.D, plan.L
    h_syms = torch.from_numpy(st["syms"]).pin_memory()
    h_out = torch.zeros((n + 7) // 8, dtype=torch.uint8).pin_memory()
    # PCIe rates of this machine (pinned, one large copy each way)
    d_buf = torch.empty(h_syms.numel(), dtype=torch.uint8, device="cuda")

    def rate(fn, nbytes):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return nbytes * reps / (time.perf_counter() - t0)
    b_h2d = rate(lambda: d_buf.copy_(h_syms, non_blocking=True), h_syms.numel())
    b_d2h = rate(lambda: h_out.copy_(d_buf[:h_out.numel()], non_blocking=True), h_out.numel())
    del d_buf
    nb = plan.num_blocks(n)
    res = {"h2d_GBps": round(b_h2d / 1e9, 2), "d2h_GBps": round(b_d2h / 1e9, 2), "runs": []}
    ref = None
    for ns in (1, 2, 3, 4, 8):
        chunk = -(-nb // ns)
        chunk += (-chunk) % 8
        plan.decode_host(h_syms, n, out=h_out, n_streams=ns, chunk_pbs=chunk, pinned=True)
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.decode_host(h_syms, n, out=h_out, n_streams=ns, chunk_pbs=chunk, pinned=True)
        t = (time.perf_counter() - t0) / reps
        if ref is None:
            ref = h_out.clone()
        same = bool(torch.equal(h_out, ref))
        nt = chunk
        t_h2d = (D + 2 * L) * nt * R / b_h2d
        t_d2h = D * nt / 8 / b_d2h
        t_k = D * nt / (kernel_mbps * 1e6)
        model = D * nt * ns / (t_h2d + ns * t_k + t_d2h) / 1e6
        res["runs"].append({"n_streams": ns, "chunk_pbs": chunk, "tp_mbps": round(n / t / 1e6, 1),
                            "eq7_mbps": round(model, 1), "same_bits": same})
    return res


def bench_ber_vs_l(torch, log2_bits: int = 24, ebn0s=(2.0, 3.0, 4.0),
                   ls=(0, 7, 14, 21, 28, 35, 42, 56, 84, 210)):
    """Bit error rate of K=7 (171,133), D=512 against the overlap L at a few
    Eb/N0 (the experiment of Sec. V, Fig. 4, whose curve is not printed)."""
    import numpy as np
    from paper_1608_00066_amd import datagen, pbvd
    n = 1 << log2_bits
    res = {"n_bits": n, "D": 512, "by_ebn0": {}}
    for e in ebn0s:
        st = datagen.make_stream(7, (0o171, 0o133), n, e, datagen.config_seed(5, e, 0))
        d_syms = torch.from_numpy(st["syms"]).cuda()
        row = {}
        for L in ls:
            with pbvd.Plan(7, (0o171, 0o133), 512, L) as plan:
                bits = np.unpackbits(plan.decode(d_syms, n).cpu().numpy(), bitorder="little")[:n]
            row[str(L)] = float(np.mean(bits != st["info"]))
        res["by_ebn0"][str(e)] = row
        del d_syms
    return res


def batch_matches_oracle(codes, frames, streams, host_out) -> bool:
    """Every frame of a batched decode against the CPU oracle with the same
    D and L (frames on all host threads; the oracle releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle

    def ok(f):
        so, n, oo, ci = frames[f]
        c = codes[ci]
        ref = oracle.decode(c["K"], c["gens"], c["D"], c["L"], streams[f]["syms"], n)["bits"]
        got = np.unpackbits(host_out[oo:oo + (n + 7) // 8], bitorder="little")[:n]
        return bool(np.array_equal(got, ref))
    with ThreadPoolExecutor(max_workers=host_threads()) as ex:
        return all(ex.map(ok, range(len(frames))))


def bench_batched(torch, steps: int, fixed=None):
    """Batched decode of 4096 frames (lengths U[40, 6144], K=7 r1/2 and r1/3
    50/50, Eb/N0 U[1, 5] dB): D and layout tuned (or `fixed` = (D, layout name)),
    HIP-graph replay timed, against one plain launch per frame."""
    from paper_1608_00066_amd import autotune, datagen, pbvd
    base = [dict(K=7, gens=(0o171, 0o133), L=42), dict(K=7, gens=(0o133, 0o171, 0o165), L=42)]
    frames, streams, syms_h, out_bytes = datagen.make_frames(
        [dict(c, D=512) for c in base], 4096, 40, 6144, seed=datagen.config_seed(3, 0, 0))
    n_bits = sum(f[1] for f in frames)
    syms = torch.from_numpy(syms_h).cuda()
    out = torch.zeros(out_bytes, dtype=torch.uint8, device="cuda")
    if fixed:
        layout = next(l for l in autotune.BATCH_LAYOUTS if l[0] == fixed[1])
        codes, table = autotune.layout_codes(base, fixed[0], layout), []
    else:
        codes, table = autotune.tune_batch_d(torch, base, frames, syms, out)
    D = codes[0]["D"]
    layout_name = next(l[0] for l in autotune.BATCH_LAYOUTS
                       if autotune.layout_codes(base, D, l) == codes)
    log("batched: tuned D=%d layout=%s" % (D, layout_name))
    with pbvd.Batch(codes) as b:
        b.set_frames(frames, syms.numel(), out.numel())
        info = b.info()
        b.decode(syms, out)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                b.decode(syms, out)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        for _ in range(3):
            g.replay()
        torch.cuda.synchronize()
        # the steps back to back, as a stream of batches runs: one pair of
        # events around all of them (events between replays would add their
        # own gaps)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(steps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        dev = e0.elapsed_time(e1) / steps * 1e-3
        del g
        # the same decode, 20 captured in one graph (no graph launch between
        # them, as a loop that replays a captured sequence of batches runs)
        per_graph = 20
        gm = torch.cuda.CUDAGraph()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with torch.cuda.graph(gm, stream=side):
                for _ in range(per_graph):
                    b.decode(syms, out)
        torch.cuda.current_stream().wait_stream(side)
        gm.replay()
        torch.cuda.synchronize()
        reps = max(1, steps // per_graph)
        e0.record()
        for _ in range(reps):
            gm.replay()
        e1.record()
        torch.cuda.synchronize()
        multi = e0.elapsed_time(e1) / (reps * per_graph) * 1e-3
        del gm
    batched = out.clone()
    log("batched: plain per-frame launches")
    t_plain_512 = plain_per_frame(torch, pbvd, [dict(c, D=512) for c in base], frames, syms, out)
    t_plain_d = plain_per_frame(torch, pbvd, codes, frames, syms, out)
    same = bool(torch.equal(out, batched))
    ops = 4.0 * info["forward_stages"] * 64
    return {
        "workload": "4096 zero-terminated frames, info bits U[40,6144], K=7 r1/2 (171,133) and "
                    "r1/3 (133,171,165) 50/50, int8 soft at Eb/N0 U[1,5] dB, L=42",
        "n_bits": n_bits, "D": D, "tiles": info["tiles"],
        "batched_graph_ms": round(wall * 1e3, 4), "batched_event_ms": round(dev * 1e3, 4),
        "batched_mbps": round(n_bits / wall / 1e6, 1),
        "batched_alu_frac": round(ops / dev / PEAK_ALU_OPS[16], 4),
        "batched_alu_tops": round(ops / dev / 1e12, 3),
        "batched_multi_graph": {"decodes_per_graph": per_graph, "ms_per_decode": round(multi * 1e3, 4),
                                "mbps": round(n_bits / multi / 1e6, 1),
                                "alu_frac": round(ops / multi / PEAK_ALU_OPS[16], 4)},
        "plain_per_frame_d512_mbps": round(n_bits / t_plain_512 / 1e6, 2),
        "plain_per_frame_same_d_mbps": round(n_bits / t_plain_d / 1e6, 2),
        "speedup_vs_plain_d512": round(t_plain_512 / wall, 1),
        "batched_equals_plain_same_d": same,
        # for the oracle comparison of the CPU-baseline leg (not printed)
        "_check": (codes, frames, streams, batched.cpu().numpy()),
        "layout": layout_name,
        "tuning_ms": {"D%d_%s" % dl: round(t * 1e3, 4) for dl, t, _ in table},
        # the fastest D of each layout (wave: one persistent launch per K)
        "best_by_layout": {name: {"D": dl[0], "mbps": round(n_bits / t / 1e6, 1)}
                           for name in {dl[1] for dl, _, _ in table}
                           for dl, t, _ in [min((r for r in table if r[0][1] == name), key=lambda r: r[1])]},
    }


def bench_serving(seconds: float, rates=(2000, 5000, 10000, 20000, 50000)):
    """Request server under Poisson arrivals: lengths log-normal (median
    1500, sigma 1, clipped to [40, 65536]), codes K=7 r1/2, K=7 r1/3 and
    K=9 r1/3 uniform, Eb/N0 U[1, 5] dB; D tuned for p99 at 10k requests/s."""
    from paper_1608_00066_amd import autotune, datagen, pbvd
    base = [dict(K=7, gens=(0o171, 0o133), L=42), dict(K=7, gens=(0o133, 0o171, 0o165), L=42),
            dict(K=9, gens=(0o557, 0o663, 0o711), L=54)]
    pools = {}

    def pool_for(cs):
        # the symbols do not depend on D: one pool serves every candidate
        if "p" not in pools:
            pools["p"] = datagen.make_requests(cs, 1500, seed=datagen.config_seed(4, 0, 0))
        return pools["p"]
    kw = dict(device_bytes=1 << 30, max_inflight=4, max_batch_frames=4096)
    codes, table = autotune.tune_server_d(base, pool_for, 10000, seconds=0.5, **kw)
    res = {"workload": "Poisson arrivals, 1500-request pool, info bits log-normal(median 1500, "
                       "sigma 1) clipped to [40,65536], K=7 r1/2, K=7 r1/3, K=9 r1/3 uniform, "
                       "Eb/N0 U[1,5] dB, L=6K; %.1f s per rate" % seconds,
           "D": codes[0]["D"], "max_inflight": kw["max_inflight"],
           "device_bytes": kw["device_bytes"],
           "tuning_p99_ms": {str(d): r["p99_ms"] for d, r in table}, "rates": []}
    with pbvd.Server(codes, **kw) as srv:
        pool = pool_for(codes)
        autotune.serve_load(srv, pool, rates[0], 0.2, seed=0)
        for r in rates:
            log("serving: %d requests/s" % r)
            res["rates"].append(autotune.serve_load(srv, pool, r, seconds, seed=r))
    return res


def batched_summary(b):
    """The batched leg of the metric next to the plain value: decoded Mbps of
    the graph-replayed batch, its ALU roofline, and the plain per-frame
    launches it replaces."""
    if not b:
        return None
    return {"value": b["batched_mbps"], "unit": "Mbps", "ms_per_step": b["batched_graph_ms"],
            "workload": b["workload"], "D": b["D"], "layout": b["layout"],
            "best_by_layout": b.get("best_by_layout"),
            "roofline": {"bound": "alu", "achieved": b["batched_alu_tops"], "peak": PEAK_ALU_OPS[16] / 1e12,
                         "unit": "Tops/s", "frac": b["batched_alu_frac"]},
            "plain_per_frame_mbps": b["plain_per_frame_d512_mbps"],
            "multi_decode_graph": b.get("batched_multi_graph")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--log2-bits", type=int, default=27)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the secondary K=9 and 2^20-bit measurements")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--serve-seconds", type=float, default=1.0,
                    help="seconds of Poisson load per arrival rate in the serving measurement")
    ap.add_argument("--only-batched", nargs=2, default=None, metavar=("D", "LAYOUT"),
                    help="only run the batched measurement at block length D and layout LAYOUT "
                         "(lanes1, lanes2, wave, group; no tuning), print its JSON and exit "
                         "(for profiling)")
    ap.add_argument("--only-stream", nargs=4, default=None, metavar=("K", "LOG2_BITS", "D", "MAPPING"),
                    help="only time pbvd_decode of one 3 dB stream (K=7 r1/2 (171,133) or K=9 r1/3 "
                         "(557,663,711), L=6K) of 2^LOG2_BITS bits at block length D on MAPPING "
                         "(auto, lanes, wave, group), print its JSON and exit (for profiling)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (to scale the "
                         "FETCH_SIZE/WRITE_SIZE counters of rocprofv3) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the decoder has no multi-GPU path in this "
              "build (PBs shard without communication; see the design notes). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1608_00066_amd import datagen, pbvd

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.only_batched:
        res = bench_batched(torch, args.steps, (int(args.only_batched[0]), args.only_batched[1]))
        res.pop("_check", None)
        print(json.dumps(res), flush=True)
        return
    if args.only_stream:
        k_s, lb_s, d_s = (int(x) for x in args.only_stream[:3])
        mapping = {"auto": 0, "lanes": 1, "wave": 2, "group": 3}[args.only_stream[3]]
        g_s = {7: (0o171, 0o133), 9: (0o557, 0o663, 0o711)}[k_s]
        n_s = 1 << lb_s
        st_s = datagen.make_stream(k_s, g_s, n_s, 3.0, datagen.config_seed(2, 3.0, 0 if k_s == 7 else 1))
        d_sy = torch.from_numpy(st_s["syms"]).cuda()
        o_s = torch.empty((n_s + 7) // 8, dtype=torch.uint8, device="cuda")
        with pbvd.Plan(k_s, g_s, d_s, 6 * k_s, mapping=mapping) as p_s:
            settle_clocks(torch, p_s, d_sy, n_s, o_s)
            ms_s, kms_s = time_decode(torch, p_s, d_sy, n_s, o_s, args.steps, args.warmup)
            msg_s = time_decode_graph(torch, p_s, d_sy, n_s, o_s, args.steps)
            lanes_s = p_s.call_lanes(n_s)
        print(json.dumps({"K": k_s, "n_bits": n_s, "D": d_s, "mapping": args.only_stream[3],
                          "lanes_per_pb": lanes_s, "ms_per_step": round(ms_s, 4),
                          "kernel_ms": round(kms_s, 4), "mbps": round(n_s / (ms_s * 1e-3) / 1e6, 1),
                          "graph_ms_per_step": round(msg_s, 4),
                          "graph_mbps": round(n_s / (msg_s * 1e-3) / 1e6, 1)}),
              flush=True)
        return
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": nbytes}), flush=True)
        return
    pbvd.lib()
    K, gens, D, L, ebn0 = 7, (0o171, 0o133), 512, 42, 3.0
    n = 1 << args.log2_bits
    log("generating %d-bit stream" % n)
    st = datagen.make_stream(K, gens, n, ebn0, datagen.config_seed(2, ebn0, 0))
    syms = torch.from_numpy(st["syms"]).cuda()
    out = torch.empty((n + 7) // 8, dtype=torch.uint8, device="cuda")
    plan = pbvd.Plan(K, gens, D, L, True, datagen.SOFT_I8, 16)
    settle = settle_clocks(torch, plan, syms, n, out)
    log("timing %d steps after %d warm-up (clock settling: %d decodes)" % (args.steps, args.warmup, settle))
    ms, kernel_ms = time_decode(torch, plan, syms, n, out, args.steps, args.warmup)
    bits = np.unpackbits(out.cpu().numpy(), bitorder="little")[:n]
    ber = float(np.mean(bits != st["info"]))
    acs = forward_stage_sum(plan, n) * (1 << (K - 1))
    ops = 4.0 * acs  # add, add, compare, select per add-compare-select
    achieved = ops / (kernel_ms * 1e-3)
    peak = PEAK_ALU_OPS[16]
    value = n / (ms * 1e-3) / 1e6

    extras = {"ber": ber, "kernel_ms": round(kernel_ms, 4),
              "kernel_decoded_mbps": round(n / (kernel_ms * 1e-3) / 1e6, 1),
              "acs_per_bit": round(acs / n, 2)}
    if not args.no_extras:
        for tag, (k2, g2, d2, l2, lb) in {
                "k9_r3_d512_2p27": (9, (0o557, 0o663, 0o711), 512, 54, args.log2_bits),
                "k7_r2_d512_2p20": (7, (0o171, 0o133), 512, 42, 20)}.items():
            n2 = 1 << lb
            s2 = datagen.make_stream(k2, g2, n2, ebn0, datagen.config_seed(2, ebn0, 1))
            d_s2 = torch.from_numpy(s2["syms"]).cuda()
            o2 = torch.empty((n2 + 7) // 8, dtype=torch.uint8, device="cuda")
            with pbvd.Plan(k2, g2, d2, l2, True, datagen.SOFT_I8, 16) as p2:
                # the short stream decodes in tens of microseconds: time
                # enough of them, on settled clocks
                short = lb <= 22
                if short:
                    settle_clocks(torch, p2, d_s2, n2, o2)
                ms2, kms2 = time_decode(torch, p2, d_s2, n2, o2,
                                        200 if short else max(3, args.steps // 4), 50 if short else 20)
                if short:
                    msg = time_decode_graph(torch, p2, d_s2, n2, o2, 200)
            extras[tag + "_mbps"] = round(n2 / (ms2 * 1e-3) / 1e6, 1)
            extras[tag + "_kernel_ms"] = round(kms2, 4)
            if short:
                # 200 decodes replayed from one captured graph
                extras[tag + "_graph_mbps"] = round(n2 / (msg * 1e-3) / 1e6, 1)
            del d_s2, o2, s2
        sweep = {}
        for d2 in (256, 1024, 2048):
            with pbvd.Plan(K, gens, d2, L, True, datagen.SOFT_I8, 16) as p2:
                ms2, _ = time_decode(torch, p2, syms, n, out, max(3, args.steps // 4), 20)
            sweep[str(d2)] = round(n / (ms2 * 1e-3) / 1e6, 1)
        extras["k7_r2_2p%d_mbps_by_d" % args.log2_bits] = sweep
        log("host pipeline")
        extras["host_pipeline"] = bench_pipeline(torch, plan, st, n, n / (kernel_ms * 1e-3) / 1e6)
        extras["host_pipeline"]["workload"] = ("the same 2^%d-bit stream in pinned host memory, "
                                               "N_s chunks on N_s streams" % args.log2_bits)
        log("BER against L")
        extras["ber_vs_L"] = bench_ber_vs_l(torch)
        log("batched decoding")
        extras["batched"] = bench_batched(torch, args.steps)
        log("serving")
        extras["serving"] = bench_serving(args.serve_seconds)

    cpu, parity = None, None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        cpu, parity = cpu_baseline(st, K, gens, D, L, args.cpu_seconds, bits,
                                   extras.get("batched", {}).get("_check"))
    if "batched" in extras:
        extras["batched"].pop("_check", None)

    rec = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "Mbps",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        # untimed decodes before the warm-up steps (80 ms of load) that
        # bring the clocks to their steady state
        "clock_settle_decodes": settle,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int16",
        "data": "synthetic",
        "config": {
            "workload": "plain PBVD throughput run: K=7 r1/2 (171,133), 2^%d info bits, "
                        "int8 soft at Eb/N0=3 dB, D=512, L=42, int16 path metrics, "
                        "zero-terminated" % args.log2_bits,
            "n_bits": n, "K": K, "R": 2, "D": D, "L": L, "parallel_blocks": plan.num_blocks(n),
            "lanes_per_pb": plan.call_lanes(n),
        },
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved / 1e12, 3),
            "peak": peak / 1e12,
            "unit": "Tops/s",
            "frac": round(achieved / peak, 4),
            "traffic": measured_traffic(),
        },
        "cpu_baseline": cpu,
        "parity": parity,
        "batched": batched_summary(extras.get("batched")),
        "extras": extras,
    }
    plan.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()

"""Autotuner of the batched decoder: picks the block length D of each code
for a given set of frames by timing pbvd_batch_decode on the device.

D changes which bits the decoder returns (Sec. III-A: a PB sees only L
stages beyond its decoded range), so the tuner only chooses among the
candidate D values given to it, with L fixed by the caller (6K keeps the
error rate at the full-frame level, Sec. V); results are compared with the
oracle run with the chosen D and L.  D >= the longest frame decodes every
frame as one block (full-frame Viterbi)."""
from __future__ import annotations

import itertools
import time

from . import pbvd


def time_batch(torch, codes, frames, syms_dev, out_dev, reps: int = 5, warmup: int = 2):
    """Median seconds of one pbvd_batch_decode of `frames` with `codes`."""
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


def tune(torch, codes, frames, syms_dev, out_dev, d_candidates=(128, 256, 512, 1024, 2048),
         reps: int = 5, joint: bool = False):
    """Returns (best code list with D filled in, table of (D tuple, seconds))."""
    table = []
    if joint:
        combos = list(itertools.product(d_candidates, repeat=len(codes)))
    else:
        combos = [tuple([d] * len(codes)) for d in d_candidates]
    for ds in combos:
        cs = [dict(c, D=int(d)) for c, d in zip(codes, ds)]
        t, info = time_batch(torch, cs, frames, syms_dev, out_dev, reps=reps)
        table.append((ds, t, info))
    best = min(table, key=lambda r: r[1])
    return [dict(c, D=int(d)) for c, d in zip(codes, best[0])], table


def wall_seconds(fn, torch):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0

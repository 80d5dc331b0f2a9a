"""Batched decoding (many frames, several codes: one tile launch per
register-kernel code, one persistent launch per constraint length for the
state-parallel codes) against the CPU oracle frame by frame, against
per-frame stream decoding, and under HIP-graph capture and replay."""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_1608_00066_amd import datagen

pytestmark = pytest.mark.gpu

NTHREADS = min(16, os.cpu_count() or 4)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a ROCm device"
    return t


@pytest.fixture(scope="module")
def pbvd():
    from paper_1608_00066_amd import pbvd as mod
    mod.lib()
    return mod


def make_batch(codes, n_frames, lo, hi, seed, gap=1):
    """Frames with random lengths/codes/Eb-N0 packed back to back; output
    ranges separated by `gap` bytes that must stay untouched."""
    return datagen.make_frames(codes, n_frames, lo, hi, seed, gap=gap)


def check_batch(torch, pbvd, codes, n_frames, lo, hi, seed):
    frames, streams, syms, out_bytes = make_batch(codes, n_frames, lo, hi, seed)
    d_syms = torch.from_numpy(syms).cuda()
    out = torch.full((out_bytes,), 0xA5, dtype=torch.uint8, device="cuda")
    with pbvd.Batch(codes) as b:
        b.set_frames(frames, syms.size, out_bytes)
        info = b.info()
        b.decode(d_syms, out)
        torch.cuda.synchronize()
    host = out.cpu().numpy()
    covered = np.zeros(out_bytes, dtype=bool)
    for (so, n, oo, ci), st in zip(frames, streams):
        c = {**dict(terminated=True, input_kind=0), **codes[ci]}
        nbytes = (n + 7) // 8
        got = np.unpackbits(host[oo:oo + nbytes], bitorder="little")[:n]
        ref = oracle.decode(c["K"], c["gens"], c["D"], c["L"], st["syms"], n,
                            terminated=c["terminated"], input_kind=c["input_kind"])
        bad = np.flatnonzero(got != ref["bits"])
        assert bad.size == 0, "frame at %d (n=%d code %d): bits differ at %s" % (so, n, ci, bad[:8])
        # pad bits of the last byte are zero
        assert np.all(np.unpackbits(host[oo:oo + nbytes], bitorder="little")[n:] == 0)
        covered[oo:oo + nbytes] = True
    assert np.all(host[~covered] == 0xA5), "bytes outside the frames were written"
    return frames, streams, syms, out_bytes, info


def test_batch_mixed_k7_codes(torch, pbvd):
    codes = [dict(K=7, gens=(0o171, 0o133), D=512, L=42),
             dict(K=7, gens=(0o133, 0o171, 0o165), D=512, L=42)]
    log("batch: 300 frames K=7 r1/2 + r1/3, lengths 40..3000")
    _, _, _, _, info = check_batch(torch, pbvd, codes, 300, 40, 3000, seed=7)
    assert info["tiles"] >= 2 and info["blocks"] >= 300


def test_batch_matches_stream_decoder(torch, pbvd):
    """Every frame of a batch equals decoding that frame alone."""
    codes = [dict(K=7, gens=(0o171, 0o133), D=256, L=42)]
    frames, streams, syms, out_bytes, _ = check_batch(torch, pbvd, codes, 64, 40, 5000, seed=11)
    d_syms = torch.from_numpy(syms).cuda()
    out = torch.zeros(out_bytes, dtype=torch.uint8, device="cuda")
    with pbvd.Batch(codes) as b:
        b.set_frames(frames, syms.size, out_bytes)
        b.decode(d_syms, out)
    with pbvd.Plan(7, (0o171, 0o133), 256, 42) as plan:
        for (so, n, oo, ci), st in zip(frames[:16], streams[:16]):
            alone = plan.decode(torch.from_numpy(st["syms"]).cuda(), n)
            torch.cuda.synchronize()
            assert np.array_equal(alone.cpu().numpy(), out[oo:oo + (n + 7) // 8].cpu().numpy())


def test_batch_unterminated_hard_int32_and_small_trellis(torch, pbvd):
    codes = [dict(K=3, gens=(0o7, 0o5), D=64, L=16, terminated=False, input_kind=1, pm_bits=32),
             dict(K=5, gens=(0o23, 0o35), D=256, L=30),
             dict(K=9, gens=(0o557, 0o663, 0o711), D=96, L=54, terminated=False)]
    log("batch: K=3 hard/int32/unterminated + K=5 + K=9 unterminated, lengths 1..700")
    check_batch(torch, pbvd, codes, 120, 1, 700, seed=21)


@pytest.mark.parametrize("lanes", [1, 2])
def test_batch_equal_frames_uniform_tiles(torch, pbvd, lanes):
    """Frames of one length: whole tiles of PBs with one geometry (interior
    PBs, and the best-state-start end PBs of unterminated frames), which run
    the kernel's uniform-wave path, next to the mixed tiles of the frame
    starts; every frame equals the oracle."""
    codes = [dict(K=7, gens=(0o171, 0o133), D=64, L=42, terminated=False, lanes_per_pb=lanes),
             dict(K=9, gens=(0o557, 0o663, 0o711), D=64, L=54, terminated=False, lanes_per_pb=lanes),
             dict(K=7, gens=(0o133, 0o171, 0o165), D=64, L=42, lanes_per_pb=lanes)]
    log("batch lanes %d: 150 frames of 1000 bits, K=7 + K=9 unterminated, K=7 r1/3" % lanes)
    check_batch(torch, pbvd, codes, 150, 1000, 1000, seed=31)


@pytest.mark.parametrize("lanes,kind", [(1, 1), (2, 0)], ids=["lanes1-hard", "lanes2-soft"])
def test_batch_code_pair_one_launch(torch, pbvd, lanes, kind):
    """The registered pair K=7 r1/2 (171,133) + r1/3 (133,171,165) decodes in
    one tile launch (each tile names its code): listed in the other order,
    with different D and L, another code between them, hard and soft input;
    every frame against the oracle."""
    codes = [dict(K=7, gens=(0o133, 0o171, 0o165), D=96, L=42, input_kind=kind, lanes_per_pb=lanes),
             dict(K=5, gens=(0o23, 0o35), D=128, L=30, input_kind=kind),
             dict(K=7, gens=(0o171, 0o133), D=64, L=30, input_kind=kind, lanes_per_pb=lanes)]
    log("batch pair lanes %d kind %d: 200 frames, lengths 1..2500" % (lanes, kind))
    check_batch(torch, pbvd, codes, 200, 1, 2500, seed=61 + lanes)


def test_batch_pair_auto_lanes_counts_both_codes(torch, pbvd):
    """Codes of a registered pair that leave the lanes per PB open share one
    launch, so the library sizes their lane groups by the PBs of both: each
    code alone has fewer than 1,024 waves of PBs (two lanes per PB would be
    chosen), together more (one lane per PB, 64 PBs per tile).  Every frame
    against the oracle."""
    codes = [dict(K=7, gens=(0o171, 0o133), D=64, L=42), dict(K=7, gens=(0o133, 0o171, 0o165), D=64, L=42)]
    log("batch pair, auto lanes: 800 frames of 6400 bits")
    _, _, _, _, info = check_batch(torch, pbvd, codes, 800, 6400, 6400, seed=71)
    assert info["blocks"] == 800 * 100
    assert info["tiles"] <= info["blocks"] // 64 + 8, "expected one lane per PB: %s" % info


@pytest.mark.parametrize("mapping", [0, 2], ids=["auto", "wave"])
def test_batch_graph_capture_replays(torch, pbvd, mapping):
    """The decode call only launches kernels (the persistent launch's work
    counter is reset by a fill kernel): capture it in a HIP graph and replay
    it several times with eager work in between."""
    codes = [dict(K=7, gens=(0o171, 0o133), D=512, L=42, mapping=mapping),
             dict(K=7, gens=(0o133, 0o171, 0o165), D=512, L=42, mapping=mapping)]
    frames, streams, syms, out_bytes = make_batch(codes, 100, 40, 2000, seed=31, gap=0)
    d_syms = torch.from_numpy(syms).cuda()
    out = torch.zeros(out_bytes, dtype=torch.uint8, device="cuda")
    with pbvd.Batch(codes) as b:
        b.set_frames(frames, syms.size, out_bytes)
        b.decode(d_syms, out)
        torch.cuda.synchronize()
        eager = out.clone()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                b.decode(d_syms, out)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        for _ in range(3):
            out.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(out, eager)
        del g


def test_batch_full_size_tuned(torch, pbvd):
    """The full 4096-frame mixed-code workload at the block length the tuner
    picks: every frame against the oracle with that D and L and against its
    own plain decode."""
    from paper_1608_00066_amd import autotune
    base = [dict(K=7, gens=(0o171, 0o133), L=42), dict(K=7, gens=(0o133, 0o171, 0o165), L=42)]
    frames, streams, syms, out_bytes = make_batch([dict(c, D=512) for c in base], 4096, 40, 6144,
                                                  seed=datagen.config_seed(3, 0, 0), gap=0)
    d_syms = torch.from_numpy(syms).cuda()
    out = torch.zeros(out_bytes, dtype=torch.uint8, device="cuda")
    codes, _ = autotune.tune_batch_d(torch, base, frames, d_syms, out, d_candidates=(64, 96, 128), reps=3)
    log("batch full size: tuned D=%d" % codes[0]["D"])
    out.fill_(0xA5)
    with pbvd.Batch(codes) as b:
        b.set_frames(frames, syms.size, out_bytes)
        b.decode(d_syms, out)
        torch.cuda.synchronize()
    host = out.cpu().numpy()
    # every frame against the oracle with the tuned D and L (frames in
    # parallel: the oracle call releases the interpreter lock)
    def frame_ok(f):
        so, n, oo, ci = frames[f]
        c = codes[ci]
        ref = oracle.decode(c["K"], c["gens"], c["D"], c["L"], streams[f]["syms"], n)["bits"]
        got = np.unpackbits(host[oo:oo + (n + 7) // 8], bitorder="little")[:n]
        return np.array_equal(got, ref)
    with ThreadPoolExecutor(max_workers=NTHREADS) as ex:
        ok = list(ex.map(frame_ok, range(len(frames))))
    bad = [f for f, v in enumerate(ok) if not v]
    assert not bad, "%d frames differ from the oracle, first %s" % (len(bad), bad[:8])
    alone = torch.full((out_bytes,), 0xA5, dtype=torch.uint8, device="cuda")
    plans = [pbvd.Plan(c["K"], c["gens"], c["D"], c["L"]) for c in codes]
    for (so, n, oo, ci) in frames:
        plans[ci].decode(d_syms[so:], n, out=alone[oo:oo + (n + 7) // 8])
    torch.cuda.synchronize()
    for p in plans:
        p.close()
    assert torch.equal(alone, out)


@pytest.mark.parametrize("lanes", [1, 2, 4, 8])
def test_batch_lane_groups(torch, pbvd, lanes):
    """Batches with 2^lb lanes per PB (K=7 takes at most 2): same bits as the
    oracle and as one lane per PB."""
    l7 = min(lanes, 2)
    codes = [dict(K=7, gens=(0o171, 0o133), D=96, L=42, lanes_per_pb=l7),
             dict(K=9, gens=(0o557, 0o663, 0o711), D=64, L=54, lanes_per_pb=lanes),
             dict(K=9, gens=(0o557, 0o663, 0o711), D=128, L=54, terminated=False, lanes_per_pb=lanes)]
    log("batch lanes %d: K=7 + K=9 + K=9 unterminated, lengths 1..3000" % lanes)
    check_batch(torch, pbvd, codes, 90, 1, 3000, seed=41 + lanes)


def test_batch_failed_set_frames_leaves_empty_batch(torch, pbvd, monkeypatch):
    """A pbvd_batch_set_frames that fails after it has started replacing the
    work list (an injected allocation failure) leaves a batch without
    frames: the next decode writes nothing, and setting the frames again
    restores normal decoding."""
    codes = [dict(K=7, gens=(0o171, 0o133), D=64, L=42)]
    frames, streams, syms, out_bytes = make_batch(codes, 40, 40, 2000, seed=61, gap=0)
    frames2, streams2, syms2, out_bytes2 = make_batch(codes, 70, 40, 3000, seed=62, gap=0)
    d_syms = torch.from_numpy(syms).cuda()
    d_syms2 = torch.from_numpy(syms2).cuda()
    with pbvd.Batch(codes) as b:
        b.set_frames(frames, syms.size, out_bytes)
        out = torch.zeros(out_bytes, dtype=torch.uint8, device="cuda")
        b.decode(d_syms, out)
        monkeypatch.setenv("PBVD_FAULT_INJECT", "batch_alloc")
        with pytest.raises(pbvd.PbvdError) as ei:
            b.set_frames(frames2, syms2.size, out_bytes2)
        assert ei.value.status == pbvd.PBVD_ENOMEM
        monkeypatch.delenv("PBVD_FAULT_INJECT")
        assert b.info()["tiles"] == 0
        out2 = torch.full((out_bytes2,), 0xA5, dtype=torch.uint8, device="cuda")
        b.decode(d_syms2, out2)
        torch.cuda.synchronize()
        assert bool((out2 == 0xA5).all()), "a batch left empty by a failed call wrote output"
        b.set_frames(frames2, syms2.size, out_bytes2)
        b.decode(d_syms2, out2)
        torch.cuda.synchronize()
    host = out2.cpu().numpy()
    for (so, n, oo, ci), st in zip(frames2, streams2):
        c = codes[ci]
        ref = oracle.decode(c["K"], c["gens"], c["D"], c["L"], st["syms"], n)["bits"]
        assert np.array_equal(np.unpackbits(host[oo:oo + (n + 7) // 8], bitorder="little")[:n], ref)


@pytest.mark.parametrize("mapping", [1, 2], ids=["lanes", "wave"])
def test_batch_mapping_per_code(torch, pbvd, mapping):
    """The same frames with every code on the register kernel or on the
    state-parallel kernel: each frame equals the oracle."""
    codes = [dict(K=7, gens=(0o171, 0o133), D=64, L=42, mapping=mapping),
             dict(K=7, gens=(0o133, 0o171, 0o165), D=96, L=42, mapping=mapping),
             dict(K=9, gens=(0o557, 0o663, 0o711), D=64, L=54, terminated=False, mapping=mapping),
             dict(K=3, gens=(0o7, 0o5), D=32, L=16, input_kind=1, mapping=mapping)]
    log("batch mapping %d: 160 frames of four codes, lengths 1..3000" % mapping)
    check_batch(torch, pbvd, codes, 160, 1, 3000, seed=71 + mapping)


def test_batch_codes_outside_the_registry(torch, pbvd):
    """Codes without a register kernel batch on the state-parallel kernel
    (persistent launches, one per K) next to registered ones on tiles and on
    the group mapping, in one batch; the decode replays from a captured HIP
    graph with the same bytes."""
    codes = [dict(K=7, gens=(0o171, 0o133), D=128, L=42),
             dict(K=6, gens=(0o53, 0o56, 0o76, 0o64), D=64, L=30),       # not registered
             dict(K=8, gens=(0o237, 0o350, 0o222), D=96, L=48, terminated=False),  # not registered
             dict(K=5, gens=(0o31, 0o6), D=40, L=25, input_kind=1),      # not registered
             dict(K=8, gens=(0o247, 0o371), D=64, L=48, mapping=2),      # same K, one launch
             dict(K=7, gens=(0o133, 0o171, 0o165), D=72, L=42, mapping=3)]
    log("batch: registered + unregistered codes, three layouts, 200 frames")
    frames, streams, syms, out_bytes, _ = check_batch(torch, pbvd, codes, 200, 1, 2500, seed=81)
    d_syms = torch.from_numpy(syms).cuda()
    out = torch.zeros(out_bytes, dtype=torch.uint8, device="cuda")
    with pbvd.Batch(codes) as b:
        b.set_frames(frames, syms.size, out_bytes)
        b.decode(d_syms, out)
        torch.cuda.synchronize()
        eager = out.clone()
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                b.decode(d_syms, out)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        for _ in range(3):
            out.zero_()
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(out, eager)
        del g


@pytest.mark.parametrize("waves", [1, 5, 64])
def test_batch_persistent_waves_take_many_blocks(torch, pbvd, monkeypatch, waves):
    """A persistent launch with few waves: each wave takes many PBs of both
    K=7 codes (and of the K=9 code in its own launch) from the work counter,
    longest first; every frame equals the oracle."""
    monkeypatch.setenv("PBVD_PERSISTENT_WAVES", str(waves))
    codes = [dict(K=7, gens=(0o171, 0o133), D=64, L=42, mapping=2),
             dict(K=7, gens=(0o133, 0o171, 0o165), D=96, L=42, mapping=2),
             dict(K=9, gens=(0o557, 0o663, 0o711), D=48, L=54, terminated=False, mapping=2),
             dict(K=7, gens=(0o171, 0o133), D=128, L=42, terminated=False, input_kind=1, mapping=2)]
    log("batch persistent, %d waves per launch: 120 frames, lengths 1..2500" % waves)
    check_batch(torch, pbvd, codes, 120, 1, 2500, seed=91 + waves)


def test_batch_persistent_full_size(torch, pbvd):
    """The full 4096-frame mixed-code workload (K=7 r1/2 and r1/3, lengths
    40..6144, both codes in one persistent launch): every frame against the
    oracle, twice in a row (the work counter starts again at zero)."""
    codes = [dict(K=7, gens=(0o171, 0o133), D=128, L=42, mapping=2),
             dict(K=7, gens=(0o133, 0o171, 0o165), D=128, L=42, mapping=2)]
    frames, streams, syms, out_bytes = make_batch(codes, 4096, 40, 6144,
                                                  seed=datagen.config_seed(3, 0, 0), gap=0)
    d_syms = torch.from_numpy(syms).cuda()
    out = torch.full((out_bytes,), 0xA5, dtype=torch.uint8, device="cuda")
    with pbvd.Batch(codes) as b:
        b.set_frames(frames, syms.size, out_bytes)
        b.decode(d_syms, out)
        torch.cuda.synchronize()
        first = out.clone()
        out.fill_(0xA5)
        b.decode(d_syms, out)
        torch.cuda.synchronize()
    assert torch.equal(first, out)
    host = out.cpu().numpy()

    def frame_ok(f):
        so, n, oo, ci = frames[f]
        c = codes[ci]
        ref = oracle.decode(c["K"], c["gens"], c["D"], c["L"], streams[f]["syms"], n)["bits"]
        got = np.unpackbits(host[oo:oo + (n + 7) // 8], bitorder="little")[:n]
        return np.array_equal(got, ref)
    with ThreadPoolExecutor(max_workers=NTHREADS) as ex:
        ok = list(ex.map(frame_ok, range(len(frames))))
    bad = [f for f, v in enumerate(ok) if not v]
    assert not bad, "%d frames differ from the oracle, first %s" % (len(bad), bad[:8])

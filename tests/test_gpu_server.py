"""Request server (continuous batching): every request's bits equal the
oracle's and decoding the same request alone; admission by the device
budget; several submitting threads."""
import sys
import threading

import numpy as np
import pytest

import oracle
from paper_1608_00066_amd import datagen

pytestmark = pytest.mark.gpu

CODES = [dict(K=7, gens=(0o171, 0o133), D=64, L=42),
         dict(K=7, gens=(0o133, 0o171, 0o165), D=64, L=42),
         dict(K=9, gens=(0o557, 0o663, 0o711), D=64, L=54)]


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pbvd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_1608_00066_amd import pbvd as mod
    mod.lib()
    return mod


def oracle_bits(c, st):
    c = {**dict(terminated=True, input_kind=0), **c}
    return oracle.decode(c["K"], c["gens"], c["D"], c["L"], st["syms"], st["n"],
                         terminated=c["terminated"], input_kind=c["input_kind"])["bits"]


def unpack(out, n):
    return np.unpackbits(out, bitorder="little")[:n]


def test_server_mix_equals_alone_and_oracle(pbvd):
    reqs = datagen.make_requests(CODES, 150, seed=501, median=400, hi=5000)
    log("server: 150 requests, 3 codes, median 400 bits")
    with pbvd.Server(CODES, device_bytes=128 << 20, max_inflight=3, max_batch_frames=64) as srv:
        tickets = [srv.submit(ci, st["syms"], st["n"]) for ci, st in reqs]
        mixed = [srv.wait(t) for t in tickets]
        cnt = srv.counters()
        log("counters %s" % cnt)
        assert cnt["requests_done"] == len(reqs)
        alone = []
        for ci, st in reqs:
            alone.append(srv.wait(srv.submit(ci, st["syms"], st["n"])))
    for (ci, st), (m, mi), (a, ai) in zip(reqs, mixed, alone):
        assert ai["batch_frames"] == 1
        assert np.array_equal(m, a), "request differs alone and in the mix"
        bits = unpack(m, st["n"])
        ref = oracle_bits(CODES[ci], st)
        assert np.array_equal(bits, ref), "request of %d bits (code %d) differs from the oracle" % (st["n"], ci)
        assert np.all(np.unpackbits(m, bitorder="little")[st["n"]:] == 0)
    assert max(i["batch_frames"] for _, i in mixed) > 1


def test_server_small_budget_many_batches(pbvd):
    reqs = datagen.make_requests(CODES[:1], 60, seed=502, median=2000, hi=6000)
    log("server: 1 MiB per batch, 60 requests")
    with pbvd.Server(CODES[:1], device_bytes=2 << 20, max_inflight=2, max_batch_frames=1000) as srv:
        with pytest.raises(pbvd.PbvdError) as ei:  # alone exceeds a batch's budget
            big = datagen.make_stream(7, (0o171, 0o133), 60000, 3.0, seed=1)
            srv.submit(0, big["syms"], big["n"])
        assert ei.value.status == pbvd.PBVD_EINVAL
        tickets = [srv.submit(ci, st["syms"], st["n"]) for ci, st in reqs]
        res = [srv.wait(t) for t in tickets]
        cnt = srv.counters()
        log("counters %s" % cnt)
        assert cnt["batches"] > 2
    for (ci, st), (out, _) in zip(reqs, res):
        assert np.array_equal(unpack(out, st["n"]), oracle_bits(CODES[ci], st))


def test_server_concurrent_submitters(pbvd):
    reqs = datagen.make_requests(CODES[:2], 200, seed=503, median=300, hi=3000)
    results = [None] * len(reqs)
    errors = []
    with pbvd.Server(CODES[:2], device_bytes=64 << 20, max_inflight=4, max_batch_frames=32) as srv:
        def run(k):
            try:
                for i in range(k, len(reqs), 4):
                    ci, st = reqs[i]
                    results[i] = srv.wait(srv.submit(ci, st["syms"], st["n"]))[0]
            except Exception as e:  # reported below
                errors.append(e)
        th = [threading.Thread(target=run, args=(k,)) for k in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join(timeout=120)
        assert not any(t.is_alive() for t in th)
    assert not errors, errors
    for (ci, st), out in zip(reqs, results):
        assert np.array_equal(unpack(out, st["n"]), oracle_bits(CODES[ci], st))


def test_server_unterminated_hard_int32_mix(pbvd):
    """Codes whose last block starts its traceback from the best state, hard
    input with 32-bit metrics, and explicit lane widths, in one server."""
    codes = [dict(K=3, gens=(0o7, 0o5), D=64, L=16, terminated=False, input_kind=1, pm_bits=32),
             dict(K=9, gens=(0o557, 0o663, 0o711), D=96, L=54, terminated=False),
             dict(K=7, gens=(0o133, 0o171, 0o165), D=64, L=42, lanes_per_pb=1)]
    reqs = datagen.make_requests(codes, 90, seed=504, median=300, hi=4000)
    log("server: unterminated / hard / int32 / lanes mix, 90 requests")
    with pbvd.Server(codes, device_bytes=64 << 20, max_inflight=2, max_batch_frames=16) as srv:
        tickets = [srv.submit(ci, st["syms"], st["n"]) for ci, st in reqs]
        res = [srv.wait(t) for t in tickets]
    for (ci, st), (out, _) in zip(reqs, res):
        assert np.array_equal(unpack(out, st["n"]), oracle_bits(codes[ci], st)), \
            "request of %d bits (code %d) differs from the oracle" % (st["n"], ci)


def test_server_admission_counts_every_best_state_block(pbvd):
    """Unterminated frames with L > D end in several PBs that start their
    traceback from the best state (each a tile of its own unless another
    frame's PB has its length).  A slot budget that fits a few dozen such
    frames: admission must count those tiles, so every request decodes
    (none fails with its batch for want of survivor memory) and equals the
    oracle."""
    codes = [dict(K=9, gens=(0o557, 0o663, 0o711), D=16, L=54, terminated=False)]
    rng = np.random.default_rng(505)
    reqs = []
    for i in range(200):
        n = int(rng.integers(150, 450))
        reqs.append((0, datagen.make_stream(9, codes[0]["gens"], n, float(rng.uniform(1, 5)),
                                            seed=6000 + i, terminated=False)))
    # one slot: the requests submitted while a batch runs all wait for the
    # next one, so batches grow to what the budget admits
    log("server: 200 unterminated K=9 frames, D=16 L=54, 3 MiB per batch, one slot")
    with pbvd.Server(codes, device_bytes=3 << 20, max_inflight=1, max_batch_frames=4096) as srv:
        tickets = [srv.submit(ci, st["syms"], st["n"]) for ci, st in reqs]
        res = [srv.wait(t) for t in tickets]
        cnt = srv.counters()
        log("counters %s" % cnt)
    assert max(i["batch_frames"] for _, i in res) > 8
    for (ci, st), (out, _) in zip(reqs, res):
        assert np.array_equal(unpack(out, st["n"]), oracle_bits(codes[ci], st))


def test_server_admission_counts_register_tiles(pbvd):
    """The same on the register kernel (one lane per PB, 64 PBs per tile):
    unterminated K=7 frames with D < L, whose PBs start their traceback at
    four different stages (0, 16, 32, L = 42; a tile holds PBs of one first
    traced stage) and end in four best-state-start PBs each.  Admission must
    count every such tile, so no batch fails for want of survivor memory."""
    codes = [dict(K=7, gens=(0o171, 0o133), D=16, L=42, terminated=False, mapping=1, lanes_per_pb=1)]
    rng = np.random.default_rng(506)
    reqs = []
    for i in range(160):
        n = int(rng.integers(100, 400))
        reqs.append((0, datagen.make_stream(7, codes[0]["gens"], n, float(rng.uniform(1, 5)),
                                            seed=6500 + i, terminated=False)))
    log("server: 160 unterminated K=7 frames on the register kernel, D=16 L=42, 2 MiB per batch")
    with pbvd.Server(codes, device_bytes=2 << 20, max_inflight=1, max_batch_frames=4096) as srv:
        tickets = [srv.submit(ci, st["syms"], st["n"]) for ci, st in reqs]
        res = [srv.wait(t) for t in tickets]
        log("counters %s" % srv.counters())
    assert max(i["batch_frames"] for _, i in res) > 1
    for (ci, st), (out, _) in zip(reqs, res):
        assert np.array_equal(unpack(out, st["n"]), oracle_bits(codes[ci], st))


def test_server_wave_mapping_and_unregistered_code(pbvd):
    """A server whose codes run on the state-parallel kernel (one explicitly,
    one because it has no register kernel) next to a register-kernel code:
    every request equals the oracle and decoding it alone."""
    codes = [dict(K=7, gens=(0o171, 0o133), D=64, L=42, mapping=pbvd.PBVD_MAP_WAVE),
             dict(K=8, gens=(0o237, 0o350, 0o222), D=64, L=48),
             dict(K=9, gens=(0o557, 0o663, 0o711), D=64, L=54)]
    reqs = datagen.make_requests(codes, 90, seed=506, median=500, hi=5000)
    log("server: wave mapping + unregistered code, 90 requests")
    with pbvd.Server(codes, device_bytes=128 << 20, max_inflight=3, max_batch_frames=32) as srv:
        tickets = [srv.submit(ci, st["syms"], st["n"]) for ci, st in reqs]
        mixed = [srv.wait(t) for t in tickets]
        alone = [srv.wait(srv.submit(ci, st["syms"], st["n"])) for ci, st in reqs[:20]]
    for (ci, st), (out, _) in zip(reqs, mixed):
        assert np.array_equal(unpack(out, st["n"]), oracle_bits(codes[ci], st)), \
            "request of %d bits (code %d) differs from the oracle" % (st["n"], ci)
    for (m, _), (a, _) in zip(mixed[:20], alone):
        assert np.array_equal(m, a)

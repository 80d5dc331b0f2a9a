"""pbvd_decode_ex_noalloc (the entry point for callers that cannot allocate
device memory) against pbvd_decode_ex, through the C ABI: the same bits and
final metrics on two calls in a row, the second smaller, on both kernels and
on the output-staging path; calls whose staging exceeds the static scratch
are refused."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1608_00066_amd import datagen

pytestmark = pytest.mark.gpu


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


def noalloc(torch, pbvd, plan, dsyms, n, pb_first, pb_count, out, fpm):
    st = pbvd.lib().pbvd_decode_ex_noalloc(
        ctypes.c_void_p(plan.handle), ctypes.c_void_p(dsyms.data_ptr()), n, pb_first, pb_count,
        ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(fpm.data_ptr()) if fpm is not None else None,
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st


@pytest.mark.parametrize("mapping,D,offset", [(1, 512, 0), (2, 512, 0), (2, 100, 1), (1, 96, 0), (3, 512, 0),
                                               (3, 100, 1)],
                         ids=["lanes", "wave", "wave-staging", "lanes-staging", "group", "group-staging"])
def test_noalloc_equals_decode_ex_twice(torch, pbvd, mapping, D, offset):
    K, gens, L = 7, (0o171, 0o133), 42
    print("noalloc mapping %d D=%d" % (mapping, D), flush=True)
    with pbvd.Plan(K, gens, D, L, mapping=mapping) as plan:
        for n, pb_first, count in [(300000, 0, None), (20000, 3, 17)]:
            st = datagen.make_stream(K, gens, n, 2.5, seed=n + D + mapping)
            dsyms = torch.from_numpy(st["syms"]).cuda()
            nb = plan.num_blocks(n)
            count = nb - pb_first if count is None else count
            ref_out, ref_pm = plan.decode_ex(dsyms, n, pb_first, count, want_pm=True)
            nbytes = (plan.out_bits(n, pb_first, count) + 7) // 8
            buf = torch.full((nbytes + 8,), 0xA5, dtype=torch.uint8, device="cuda")
            out = buf[offset:offset + nbytes]
            fpm = torch.full((count, 64), -7, dtype=torch.int32, device="cuda")
            assert noalloc(torch, pbvd, plan, dsyms, n, pb_first, count, out, fpm) == 0, \
                pbvd.pbvd_last_error()
            torch.cuda.synchronize()
            assert torch.equal(out, ref_out[:nbytes])
            assert torch.equal(fpm, ref_pm[:count])
            assert bool((buf[:offset] == 0xA5).all()) and bool((buf[offset + nbytes:] == 0xA5).all())
            ref = oracle.decode(K, gens, D, L, st["syms"], n, pb_first=pb_first, pb_count=count,
                                want_pm=True, nthreads=8)
            bits = np.unpackbits(out.cpu().numpy(), bitorder="little")[:ref["bits"].size]
            assert np.array_equal(bits, ref["bits"])
            assert np.array_equal(fpm.cpu().numpy(), ref["final_pm"])


def test_noalloc_refuses_staging_beyond_scratch(torch, pbvd):
    """D % 32 != 0 needs 4 bytes of staging per 32 decoded bits: 2^29 bits
    need 64 MiB, more than the static scratch (nothing is decoded)."""
    with pbvd.Plan(7, (0o171, 0o133), 100, 42) as plan:
        n = 1 << 29
        dsyms = torch.zeros(16, dtype=torch.uint8, device="cuda")  # never read
        out = torch.zeros(16, dtype=torch.uint8, device="cuda")
        st = noalloc(torch, pbvd, plan, dsyms, n, 0, plan.num_blocks(n), out, None)
        assert st == pbvd.PBVD_EINVAL
        assert "static scratch" in pbvd.pbvd_last_error()

"""ctypes binding of ``libpbvd.so`` (declared in ``include/pbvd.h``).

Argument marshalling only: every step of the decode runs in the HIP kernels
of the library.  Device buffers are torch tensors on a ROCm device; the
stream is torch's current stream unless one is given.  The module raises
when the library is not built -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# PBVD_LIBRARY may name another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("PBVD_LIBRARY") or os.path.join(_PKG, "libpbvd.so")

PBVD_OK = 0
PBVD_EINVAL = -1
PBVD_ENOTSUP = -2
PBVD_ENOMEM = -3
PBVD_EHIP = -4
PBVD_EAGAIN = -5
PBVD_SOFT_I8 = 0
PBVD_HARD_U8 = 1
PBVD_HOST_PINNED = 1
PBVD_MAP_AUTO = 0
PBVD_MAP_LANES = 1
PBVD_MAP_WAVE = 2
PBVD_MAP_GROUP = 3


class pbvd_code(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("R", ctypes.c_int32), ("gen", ctypes.c_uint32 * 4),
                ("D", ctypes.c_int32), ("L", ctypes.c_int32), ("terminated", ctypes.c_int32),
                ("input_kind", ctypes.c_int32), ("pm_bits", ctypes.c_int32),
                ("lanes_per_pb", ctypes.c_int32), ("mapping", ctypes.c_int32)]


class pbvd_frame(ctypes.Structure):
    _fields_ = [("sym_offset", ctypes.c_int64), ("n_bits", ctypes.c_int64),
                ("out_offset", ctypes.c_int64), ("code", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class pbvd_server_config(ctypes.Structure):
    _fields_ = [("device_bytes", ctypes.c_int64), ("max_inflight", ctypes.c_int32),
                ("max_batch_frames", ctypes.c_int32), ("max_queued", ctypes.c_int64)]


class pbvd_request_info(ctypes.Structure):
    _fields_ = [("submit_ns", ctypes.c_int64), ("start_ns", ctypes.c_int64),
                ("done_ns", ctypes.c_int64), ("batch_frames", ctypes.c_int32),
                ("status", ctypes.c_int32)]


class PbvdError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s failed: %s (%d): %s" % (where, pbvd_strerror(status), status,
                                                   pbvd_last_error()))


_lib = None

# exported entry points of include/pbvd.h: name -> (restype, argtypes)
_P, _I64, _I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
SIGNATURES = {
    "pbvd_create": (_I32, [ctypes.POINTER(pbvd_code), ctypes.POINTER(_P)]),
    "pbvd_decode": (_I32, [_P, _P, _I64, _P, _P]),
    "pbvd_decode_ex": (_I32, [_P, _P, _I64, _I64, _I64, _P, _P, _P]),
    "pbvd_decode_ex_noalloc": (_I32, [_P, _P, _I64, _I64, _I64, _P, _P, _P]),
    "pbvd_decode_host": (_I32, [_P, _P, _I64, _P, _I32, _I64, ctypes.c_uint32]),
    "pbvd_num_blocks": (_I64, [_P, _I64]),
    "pbvd_call_lanes": (_I32, [_P, _I64, _I64, _I64]),
    "pbvd_block_geometry": (_I32, [_P, _I64, _I64, _I64, _P]),
    "pbvd_debug_survivors": (_I32, [_P, _P, _I64, _I64, _I64, _P, _P, _P]),
    "pbvd_debug_branch_metrics": (_I32, [_P, _P, _I64, _P, _P]),
    "pbvd_debug_group_table": (_I32, [ctypes.POINTER(pbvd_code), _P, _P]),
    "pbvd_destroy": (None, [_P]),
    "pbvd_batch_create": (_I32, [_P, _I32, ctypes.POINTER(_P)]),
    "pbvd_batch_set_frames": (_I32, [_P, _P, _I64, _I64, _I64]),
    "pbvd_batch_decode": (_I32, [_P, _P, _P, _P]),
    "pbvd_batch_info": (_I32, [_P, _P, _P, _P, _P]),
    "pbvd_batch_destroy": (None, [_P]),
    "pbvd_server_create": (_I32, [_P, _I32, _P, ctypes.POINTER(_P)]),
    "pbvd_server_submit": (_I32, [_P, _I32, _P, _I64, _P, ctypes.POINTER(_I64)]),
    "pbvd_server_wait": (_I32, [_P, _I64, _I64, _P]),
    "pbvd_server_counters": (_I32, [_P, _P, _P, _P]),
    "pbvd_server_destroy": (None, [_P]),
    "pbvd_strerror": (ctypes.c_char_p, [_I32]),
    "pbvd_last_error": (ctypes.c_char_p, []),
}


def lib():
    """Load ``libpbvd.so``; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpbvd.so is not built (%s); run "
                               "`python -m paper_1608_00066_amd.build`" % LIB_PATH)
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


def pbvd_strerror(status: int) -> str:
    return lib().pbvd_strerror(status).decode()


def pbvd_last_error() -> str:
    return lib().pbvd_last_error().decode()


def _check(status: int, where: str):
    if status != PBVD_OK:
        raise PbvdError(status, where)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, what, min_bytes, dtypes):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % what)
    if t.dtype not in dtypes:
        raise TypeError("%s has dtype %s, expected one of %s" % (what, t.dtype, dtypes))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    if t.numel() * t.element_size() < min_bytes:
        raise ValueError("%s has %d bytes, needs %d" % (what, t.numel() * t.element_size(),
                                                        min_bytes))
    return ctypes.c_void_p(t.data_ptr())


def pbvd_create(K: int, gens, D: int, L: int, terminated: bool = True,
                input_kind: int = PBVD_SOFT_I8, pm_bits: int = 16, lanes_per_pb: int = 0,
                mapping: int = PBVD_MAP_AUTO) -> int:
    """Returns an opaque plan handle (int)."""
    c = _code_struct(K, gens, D, L, terminated, input_kind, pm_bits, lanes_per_pb, mapping)
    h = ctypes.c_void_p()
    _check(lib().pbvd_create(ctypes.byref(c), ctypes.byref(h)), "pbvd_create")
    return h.value


def pbvd_destroy(plan: int):
    lib().pbvd_destroy(ctypes.c_void_p(plan))


def pbvd_num_blocks(plan: int, n_bits: int) -> int:
    return int(lib().pbvd_num_blocks(ctypes.c_void_p(plan), n_bits))


def pbvd_block_geometry(plan: int, n_bits: int, pb_first: int, pb_count: int) -> np.ndarray:
    out = np.zeros((max(pb_count, 0), 4), dtype=np.int64)
    _check(lib().pbvd_block_geometry(ctypes.c_void_p(plan), n_bits, pb_first, pb_count,
                                     out.ctypes.data_as(ctypes.c_void_p)), "pbvd_block_geometry")
    return out


class Plan:
    """One decoder plan (code + block parameters + its device workspace)."""

    def __init__(self, K: int, gens, D: int, L: int, terminated: bool = True,
                 input_kind: int = PBVD_SOFT_I8, pm_bits: int = 16, lanes_per_pb: int = 0,
                 mapping: int = PBVD_MAP_AUTO):
        self.K, self.gens, self.R = K, tuple(int(g) for g in gens), len(gens)
        self.D, self.L, self.terminated = D, L, bool(terminated)
        self.input_kind, self.pm_bits, self.lanes_per_pb = input_kind, pm_bits, lanes_per_pb
        self.mapping = mapping
        self.N = 1 << (K - 1)
        self.handle = pbvd_create(K, gens, D, L, terminated, input_kind, pm_bits, lanes_per_pb,
                                  mapping)

    def close(self):
        if self.handle:
            pbvd_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # sizes -----------------------------------------------------------------
    def stages(self, n_bits: int) -> int:
        return n_bits + (self.K - 1 if self.terminated else 0)

    def num_blocks(self, n_bits: int) -> int:
        return pbvd_num_blocks(self.handle, n_bits)

    def call_lanes(self, n_bits: int, pb_first: int = 0, pb_count: int | None = None) -> int:
        """Lanes per PB a decode of these PBs uses (pbvd_call_lanes)."""
        if pb_count is None:
            pb_count = self.num_blocks(n_bits) - pb_first
        return int(lib().pbvd_call_lanes(ctypes.c_void_p(self.handle), n_bits, pb_first, pb_count))

    def block_geometry(self, n_bits: int, pb_first: int = 0, pb_count: int | None = None):
        if pb_count is None:
            pb_count = self.num_blocks(n_bits) - pb_first
        return pbvd_block_geometry(self.handle, n_bits, pb_first, pb_count)

    def out_bits(self, n_bits: int, pb_first: int, pb_count: int) -> int:
        if pb_count <= 0:
            return 0
        return min(n_bits, (pb_first + pb_count) * self.D) - pb_first * self.D

    # decoding --------------------------------------------------------------
    def _syms_ptr(self, syms, n_bits):
        import torch
        return _dev_ptr(syms, "syms", self.stages(n_bits) * self.R, (torch.uint8, torch.int8))

    def decode(self, syms, n_bits: int, out=None, stream=None):
        """pbvd_decode: returns the packed decoded bits (uint8 device tensor)."""
        import torch
        nbytes = (n_bits + 7) // 8
        if out is None:
            out = torch.empty(nbytes, dtype=torch.uint8, device=syms.device)
        st = lib().pbvd_decode(ctypes.c_void_p(self.handle), self._syms_ptr(syms, n_bits), n_bits,
                               _dev_ptr(out, "out", nbytes, (torch.uint8,)), _stream_handle(stream))
        _check(st, "pbvd_decode")
        return out

    def decode_ex(self, syms, n_bits: int, pb_first: int, pb_count: int, out=None,
                  final_pm=None, want_pm: bool = False, stream=None):
        """pbvd_decode_ex: returns (packed bits, final_pm or None)."""
        import torch
        nbytes = (self.out_bits(n_bits, pb_first, pb_count) + 7) // 8
        if out is None:
            out = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=syms.device)
        if want_pm and final_pm is None:
            final_pm = torch.empty((max(pb_count, 1), self.N), dtype=torch.int32,
                                   device=syms.device)
        pm_ptr = (_dev_ptr(final_pm, "final_pm", pb_count * self.N * 4, (torch.int32,))
                  if final_pm is not None else None)
        st = lib().pbvd_decode_ex(ctypes.c_void_p(self.handle), self._syms_ptr(syms, n_bits),
                                  n_bits, pb_first, pb_count,
                                  _dev_ptr(out, "out", nbytes, (torch.uint8,)), pm_ptr,
                                  _stream_handle(stream))
        _check(st, "pbvd_decode_ex")
        return out, final_pm

    def decode_host(self, syms, n_bits: int, out=None, n_streams: int = 3, chunk_pbs: int = 0,
                    pinned: bool = False):
        """pbvd_decode_host: host symbols (numpy array or pinned CPU tensor) to
        host packed bits; returns `out` (a new numpy array if None)."""
        def ptr(a):
            if hasattr(a, "data_ptr"):
                if a.is_cuda or not a.is_contiguous():
                    raise ValueError("host buffers must be contiguous CPU memory")
                return ctypes.c_void_p(a.data_ptr()), a.numel() * a.element_size()
            if not (isinstance(a, np.ndarray) and a.flags["C_CONTIGUOUS"]):
                raise ValueError("host buffers must be contiguous numpy arrays or CPU tensors")
            return ctypes.c_void_p(a.ctypes.data), a.nbytes
        nbytes = (n_bits + 7) // 8
        if out is None:
            out = np.zeros(nbytes, dtype=np.uint8)
        sp, sb = ptr(syms)
        op, ob = ptr(out)
        if sb < self.stages(n_bits) * self.R or ob < nbytes:
            raise ValueError("host buffer too small")
        st = lib().pbvd_decode_host(ctypes.c_void_p(self.handle), sp, n_bits, op, n_streams,
                                    chunk_pbs, PBVD_HOST_PINNED if pinned else 0)
        _check(st, "pbvd_decode_host")
        return out

    def debug_survivors(self, syms, n_bits: int, pb_first: int, pb_count: int, stream=None):
        """pbvd_debug_survivors: returns (packed bits, dec[pb_count][D+L][N])."""
        import torch
        nbytes = (self.out_bits(n_bits, pb_first, pb_count) + 7) // 8
        out = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=syms.device)
        dec = torch.empty((max(pb_count, 1), self.D + self.L, self.N), dtype=torch.uint8,
                          device=syms.device)
        st = lib().pbvd_debug_survivors(ctypes.c_void_p(self.handle),
                                        self._syms_ptr(syms, n_bits), n_bits, pb_first,
                                        pb_count, ctypes.c_void_p(out.data_ptr()),
                                        ctypes.c_void_p(dec.data_ptr()), _stream_handle(stream))
        _check(st, "pbvd_debug_survivors")
        return out, dec

    def debug_branch_metrics(self, syms, n_stages: int, stream=None):
        """pbvd_debug_branch_metrics: int32 [n_stages][2^R] device tensor."""
        import torch
        bm = torch.empty((max(n_stages, 1), 1 << self.R), dtype=torch.int32, device=syms.device)
        st = lib().pbvd_debug_branch_metrics(
            ctypes.c_void_p(self.handle),
            _dev_ptr(syms, "syms", n_stages * self.R, (torch.uint8, torch.int8)), n_stages,
            ctypes.c_void_p(bm.data_ptr()), _stream_handle(stream))
        _check(st, "pbvd_debug_branch_metrics")
        return bm


def unpack_bits(packed: np.ndarray, n_bits: int) -> np.ndarray:
    """Packed output (bit i = bit i&7 of byte i>>3) to one uint8 per bit."""
    return np.unpackbits(np.asarray(packed, dtype=np.uint8), bitorder="little")[:n_bits]


def _code_struct(K, gens, D, L, terminated=True, input_kind=PBVD_SOFT_I8, pm_bits=16,
                 lanes_per_pb=0, mapping=PBVD_MAP_AUTO):
    c = pbvd_code()
    c.K, c.R = K, len(gens)
    for i, g in enumerate(gens[:4]):
        c.gen[i] = int(g)
    c.D, c.L, c.terminated, c.input_kind, c.pm_bits = D, L, int(terminated), input_kind, pm_bits
    c.lanes_per_pb = lanes_per_pb
    c.mapping = mapping
    return c


def group_table(K, gens):
    """pbvd_debug_group_table: (alpha of each butterfly [N/2], code words of
    each group's alpha, beta, gamma, theta [2^R][4]) as numpy arrays, c^(1)
    the most significant bit."""
    import numpy as np
    c = _code_struct(K, gens, 64, 0, mapping=PBVD_MAP_GROUP)
    alpha = np.zeros(1 << (K - 2), dtype=np.int32)
    masks = np.zeros((1 << len(gens), 4), dtype=np.int32)
    _check(lib().pbvd_debug_group_table(ctypes.byref(c), alpha.ctypes.data, masks.ctypes.data),
           "pbvd_debug_group_table")
    return alpha, masks


class Batch:
    """pbvd_batch_*: many frames, several codes, one launch per code.

    ``codes`` is a list of dicts with keys K, gens, D, L and optionally
    terminated, input_kind, pm_bits, lanes_per_pb, mapping."""

    def __init__(self, codes):
        defaults = dict(terminated=True, input_kind=PBVD_SOFT_I8, pm_bits=16, lanes_per_pb=0,
                        mapping=PBVD_MAP_AUTO)
        self.codes = [{**defaults, **c} for c in codes]
        arr = (pbvd_code * len(codes))(*[_code_struct(**c) for c in self.codes])
        h = ctypes.c_void_p()
        _check(lib().pbvd_batch_create(ctypes.cast(arr, ctypes.c_void_p), len(codes),
                                       ctypes.byref(h)), "pbvd_batch_create")
        self.handle = h.value
        self.n_frames = 0

    def close(self):
        if self.handle:
            lib().pbvd_batch_destroy(ctypes.c_void_p(self.handle))
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_frames(self, frames, sym_bytes: int, out_bytes: int):
        """frames: iterable of (sym_offset, n_bits, out_offset, code)."""
        frames = list(frames)
        arr = (pbvd_frame * max(len(frames), 1))()
        for i, (so, nb, oo, code) in enumerate(frames):
            arr[i].sym_offset, arr[i].n_bits, arr[i].out_offset = int(so), int(nb), int(oo)
            arr[i].code, arr[i].reserved = int(code), 0
        _check(lib().pbvd_batch_set_frames(ctypes.c_void_p(self.handle),
                                           ctypes.cast(arr, ctypes.c_void_p), len(frames),
                                           int(sym_bytes), int(out_bytes)),
               "pbvd_batch_set_frames")
        self.n_frames = len(frames)

    def decode(self, syms, out, stream=None):
        import torch
        st = lib().pbvd_batch_decode(ctypes.c_void_p(self.handle),
                                     _dev_ptr(syms, "syms", 0, (torch.uint8, torch.int8)),
                                     _dev_ptr(out, "out", 0, (torch.uint8,)),
                                     _stream_handle(stream))
        _check(st, "pbvd_batch_decode")
        return out

    def info(self):
        v = [ctypes.c_int64() for _ in range(4)]
        _check(lib().pbvd_batch_info(ctypes.c_void_p(self.handle), *[ctypes.byref(x) for x in v]),
               "pbvd_batch_info")
        return dict(zip(("tiles", "blocks", "forward_stages", "workspace_bytes"),
                        (x.value for x in v)))


class Server:
    """pbvd_server_*: continuous batching of decode requests (host in/out).

    ``codes`` as for :class:`Batch`.  ``submit`` copies the symbols and
    returns a ticket; ``wait`` returns (packed bits, timing dict)."""

    def __init__(self, codes, device_bytes: int = 256 << 20, max_inflight: int = 4,
                 max_batch_frames: int = 1024, max_queued: int = 1 << 20):
        defaults = dict(terminated=True, input_kind=PBVD_SOFT_I8, pm_bits=16, lanes_per_pb=0,
                        mapping=PBVD_MAP_AUTO)
        self.codes = [{**defaults, **c} for c in codes]
        arr = (pbvd_code * len(codes))(*[_code_struct(**c) for c in self.codes])
        cfg = pbvd_server_config(int(device_bytes), int(max_inflight), int(max_batch_frames),
                                 int(max_queued))
        h = ctypes.c_void_p()
        _check(lib().pbvd_server_create(ctypes.cast(arr, ctypes.c_void_p), len(codes),
                                        ctypes.byref(cfg), ctypes.byref(h)), "pbvd_server_create")
        self.handle = h.value
        self._pending = {}   # ticket -> (out array, n_bits, symbols kept alive)

    def close(self):
        if self.handle:
            lib().pbvd_server_destroy(ctypes.c_void_p(self.handle))
            self.handle = None
            self._pending.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, code: int, syms: np.ndarray, n_bits: int) -> int:
        syms = np.ascontiguousarray(syms, dtype=np.uint8)
        c = self.codes[code]
        need = (n_bits + (c["K"] - 1 if c["terminated"] else 0)) * len(c["gens"])
        if syms.size < need:
            raise ValueError("syms has %d bytes, needs %d" % (syms.size, need))
        out = np.zeros((n_bits + 7) // 8, dtype=np.uint8)
        t = ctypes.c_int64()
        _check(lib().pbvd_server_submit(ctypes.c_void_p(self.handle), int(code),
                                        syms.ctypes.data_as(ctypes.c_void_p), int(n_bits),
                                        out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(t)),
               "pbvd_server_submit")
        self._pending[t.value] = (out, n_bits)
        return t.value

    def wait(self, ticket: int, timeout_us: int = -1):
        info = pbvd_request_info()
        st = lib().pbvd_server_wait(ctypes.c_void_p(self.handle), int(ticket), int(timeout_us),
                                    ctypes.byref(info))
        if st == PBVD_EAGAIN:
            return None
        out, _ = self._pending.pop(ticket, (None, 0))
        _check(st, "pbvd_server_wait")
        return out, dict(submit_ns=info.submit_ns, start_ns=info.start_ns, done_ns=info.done_ns,
                         batch_frames=info.batch_frames, latency_ns=info.done_ns - info.submit_ns)

    def counters(self):
        v = [ctypes.c_int64() for _ in range(3)]
        _check(lib().pbvd_server_counters(ctypes.c_void_p(self.handle),
                                          *[ctypes.byref(x) for x in v]), "pbvd_server_counters")
        return dict(zip(("batches", "requests_done", "peak_inflight"), (x.value for x in v)))

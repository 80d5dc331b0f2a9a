"""CPU oracle for the parallel block-based Viterbi decoder (arXiv 1608.00066).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of ``bench.py`` may import this package; the product library never does.

The arithmetic lives in ``pbvd_oracle.c`` (plain C, int64 path metrics, one
byte per decision).  This module only compiles it with gcc and marshals numpy
arrays through ctypes.  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pbvd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

SOFT_I8 = 0
HARD_U8 = 1


def build(force: bool = False) -> str:
    """Compile ``pbvd_oracle.c`` into ``liboracle.so`` (gcc -O2, pthreads)."""
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=200809L", "-fPIC", "-shared",
           "-pthread", "-Wall", "-Wextra", "-o", tmp, _SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            i32, i64, p = ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
            lib.oracle_trellis.argtypes = [i32, i32, p, p, p]
            lib.oracle_trellis.restype = i32
            lib.oracle_branch_metrics.argtypes = [i32, i32, p, i64, p]
            lib.oracle_branch_metrics.restype = i32
            lib.oracle_num_blocks.argtypes = [i64, i64]
            lib.oracle_num_blocks.restype = i64
            lib.oracle_pb_geometry.argtypes = [i64, i64, i64, i64, i64, p]
            lib.oracle_pb_geometry.restype = None
            lib.oracle_decode.argtypes = [i32, i32, p, i32, i32, i32, i32, p, i64, i64, i64,
                                          p, p, p, i32]
            lib.oracle_decode.restype = i32
            _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _gens(gens) -> np.ndarray:
    g = np.zeros(8, dtype=np.uint32)
    g[: len(gens)] = np.asarray(gens, dtype=np.uint32)
    return g


def trellis(K: int, gens):
    """Return (next[N][2], label[N][2]) of the rate-1/R code (Eq. 2, Sec. III-B)."""
    lib = _load()
    N = 1 << (K - 1)
    nxt = np.zeros((N, 2), dtype=np.int32)
    lab = np.zeros((N, 2), dtype=np.int32)
    g = _gens(gens)
    if lib.oracle_trellis(K, len(gens), _ptr(g), _ptr(nxt), _ptr(lab)):
        raise ValueError("invalid code")
    return nxt, lab


def branch_metrics(R: int, syms: np.ndarray, input_kind: int = SOFT_I8) -> np.ndarray:
    """bm[s][c] for every stage s and code word c (Sec. II distance)."""
    lib = _load()
    syms = np.ascontiguousarray(syms).view(np.uint8).reshape(-1)
    n_stages = syms.size // R
    bm = np.zeros((n_stages, 1 << R), dtype=np.int64)
    if lib.oracle_branch_metrics(R, input_kind, _ptr(syms), n_stages, _ptr(bm)):
        raise ValueError("invalid arguments")
    return bm


def num_blocks(n: int, D: int) -> int:
    return int(_load().oracle_num_blocks(n, D))


def pb_geometry(n: int, T: int, D: int, L: int, b: int):
    """(f0, f1, d0, d1) of parallel block b (Sec. III-A, M = L)."""
    out = np.zeros(4, dtype=np.int64)
    _load().oracle_pb_geometry(n, T, D, L, b, _ptr(out))
    return tuple(int(v) for v in out)


def decode(K: int, gens, D: int, L: int, syms: np.ndarray, n: int, *, terminated: bool = True,
           input_kind: int = SOFT_I8, pb_first: int = 0, pb_count: int | None = None,
           want_pm: bool = False, want_dec: bool = False, nthreads: int = 1):
    """Block-based decode (Sec. III-A).  Returns a dict with ``bits`` (uint8
    0/1 per decoded bit of blocks [pb_first, pb_first+pb_count)), and
    optionally ``final_pm`` [pb_count][N] (int64, minus the block minimum)
    and ``dec`` [pb_count][D+L][N] (decisions of stages [b*D, f1))."""
    lib = _load()
    R = len(gens)
    N = 1 << (K - 1)
    T = n + (K - 1 if terminated else 0)
    syms = np.ascontiguousarray(syms).view(np.uint8).reshape(-1)
    if syms.size < T * R:
        raise ValueError("need %d symbols, got %d" % (T * R, syms.size))
    nb = num_blocks(n, D)
    if pb_count is None:
        pb_count = nb - pb_first
    d_lo = pb_first * D
    d_hi = min(n, (pb_first + pb_count) * D)
    bits = np.zeros(max(0, d_hi - d_lo), dtype=np.uint8)
    fpm = np.zeros((pb_count, N), dtype=np.int64) if want_pm else None
    dec = np.zeros((pb_count, D + L, N), dtype=np.uint8) if want_dec else None
    g = _gens(gens)
    rc = lib.oracle_decode(K, R, _ptr(g), D, L, 1 if terminated else 0, input_kind, _ptr(syms),
                           n, pb_first, pb_count, _ptr(bits),
                           _ptr(fpm) if want_pm else None, _ptr(dec) if want_dec else None,
                           nthreads)
    if rc:
        raise ValueError("oracle_decode failed (invalid arguments)")
    out = {"bits": bits}
    if want_pm:
        out["final_pm"] = fpm
    if want_dec:
        out["dec"] = dec
    return out


def viterbi_full(K: int, gens, syms: np.ndarray, n: int, *, terminated: bool = True,
                 input_kind: int = SOFT_I8, want_pm: bool = False):
    """Full-frame Viterbi (Sec. II): one block whose forward range is the
    whole trellis [0, T) and whose decoded range is every information bit."""
    return decode(K, gens, max(n, 1), K - 1, syms, n, terminated=terminated,
                  input_kind=input_kind, want_pm=want_pm)

"""Seeded synthetic inputs for the decoder: information bits, a rate-1/R
convolutional encoder, BPSK over AWGN, and the 8-bit soft / 1-bit hard
quantizers.

This module holds the channel model only.  It contains none of the decoder's
arithmetic (no branch metrics, path metrics or traceback) and imports neither
the GPU library nor the CPU oracle, so both can be fed the same inputs.

Conventions (the same ones the decoder and its oracle read from the paper):
  * generator integer ``g`` has bit k equal to g_k of Eq. 2 (octal 171 is
    1111001, bit K-1 taps the current input bit);
  * the register cell D_{K-2} holds the newest past input (the butterfly of
    Sec. III-B moves S_d to S_{(x << (K-2)) | (d >> 1)});
  * the R code bits of one stage are emitted in generator order, c^(1) first;
  * BPSK maps bit 0 to +1 and bit 1 to -1; a soft value q >= 0 reads as bit 0.
"""
from __future__ import annotations

import math

import numpy as np

# Codes of the workloads, generators in octal as they are usually written.
CODES = {
    "k3_r2": (3, (0o7, 0o5)),
    "k7_r2": (7, (0o171, 0o133)),
    "k7_r3": (7, (0o133, 0o171, 0o165)),
    "k9_r3": (9, (0o557, 0o663, 0o711)),
}

SOFT_I8 = 0
HARD_U8 = 1
SOFT_SCALE = 16.0  # q = clip(rint(SOFT_SCALE * y / sigma^2), -127, 127)


def config_seed(config_index: int, ebn0_db: float, code_index: int = 0) -> int:
    """Seed of one workload: 1000*config + 10*Eb/N0 + code index."""
    return int(1000 * config_index + round(10 * ebn0_db) + code_index)


def noise_variance(R: int, ebn0_db: float) -> float:
    """sigma^2 = N0/2 for unit-energy BPSK symbols at rate 1/R: each
    information bit carries R symbols, so Eb = R and N0 = R / 10^(Eb/N0 / 10)."""
    return R / (2.0 * 10.0 ** (ebn0_db / 10.0))


def encode(K: int, gens, info: np.ndarray, terminated: bool = True) -> np.ndarray:
    """Encode information bits: code bit r at time t is the GF(2)
    convolution sum_m g^(r)_{K-1-m} * u_{t-m} (Eq. 2 with D_k = u_{t-(K-1-k)}).
    With ``terminated`` the input is followed by K-1 zero bits.
    Returns uint8 code bits of shape [T][R]."""
    u = np.asarray(info, dtype=np.uint8) & 1
    if terminated:
        u = np.concatenate([u, np.zeros(K - 1, dtype=np.uint8)])
    T = u.size
    out = np.zeros((T, len(gens)), dtype=np.uint8)
    for r, g in enumerate(gens):
        acc = np.zeros(T, dtype=np.uint8)
        for m in range(K):
            if (int(g) >> (K - 1 - m)) & 1:
                if m == 0:
                    acc ^= u
                else:
                    acc[m:] ^= u[:-m]
        out[:, r] = acc
    return out


def quantize_soft(y: np.ndarray, sigma2: float) -> np.ndarray:
    """8-bit soft values: clip(rint(16 * y / sigma^2), -127, 127), round half to even."""
    q = np.rint(SOFT_SCALE * np.asarray(y, dtype=np.float64) / sigma2)
    return np.clip(q, -127, 127).astype(np.int8)


def quantize_hard(y: np.ndarray) -> np.ndarray:
    """Hard decisions: bit 1 where the received value is negative."""
    return (np.asarray(y) < 0).astype(np.uint8)


def channel(code_bits: np.ndarray, ebn0_db: float | None, rng: np.random.Generator,
            kind: int = SOFT_I8, chunk: int = 1 << 22) -> np.ndarray:
    """BPSK over AWGN and quantization of a [T][R] code-bit array, returned
    as a flat uint8 array of T*R symbols (soft values are int8 bit patterns).
    ``ebn0_db=None`` is the noiseless channel (soft values are +-127)."""
    R = code_bits.shape[1]
    flat = code_bits.reshape(-1)
    out = np.empty(flat.size, dtype=np.uint8)
    if ebn0_db is None:
        if kind == HARD_U8:
            out[:] = flat & 1
        else:
            out[:] = np.where(flat & 1, -127, 127).astype(np.int8).view(np.uint8)
        return out
    sigma2 = noise_variance(R, ebn0_db)
    sigma = math.sqrt(sigma2)
    for lo in range(0, flat.size, chunk):
        hi = min(flat.size, lo + chunk)
        x = 1.0 - 2.0 * flat[lo:hi].astype(np.float64)
        y = x + sigma * rng.standard_normal(hi - lo)
        if kind == HARD_U8:
            out[lo:hi] = quantize_hard(y)
        else:
            out[lo:hi] = quantize_soft(y, sigma2).view(np.uint8)
    return out


def make_stream(K: int, gens, n: int, ebn0_db: float | None, seed: int, kind: int = SOFT_I8,
                terminated: bool = True):
    """One seeded stream: ``info`` (uint8 0/1, n bits), ``syms`` (uint8, T*R
    received symbols, stage-major), ``T`` and ``R``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    info = rng.integers(0, 2, size=n, dtype=np.uint8)
    code_bits = encode(K, gens, info, terminated)
    syms = channel(code_bits, ebn0_db, rng, kind)
    return {"info": info, "syms": syms, "T": code_bits.shape[0], "R": len(gens),
            "K": K, "gens": tuple(int(g) for g in gens), "n": n, "terminated": terminated,
            "kind": kind}


def uncoded_ber(ebn0_db: float) -> float:
    """Bit error rate of uncoded BPSK, Q(sqrt(2 Eb/N0))."""
    return 0.5 * math.erfc(math.sqrt(10.0 ** (ebn0_db / 10.0)))


def make_frames(codes, n_frames: int, len_lo: int, len_hi: int, seed: int, ebn0_lo: float = 1.0,
                ebn0_hi: float = 5.0, gap: int = 0, lengths=None, code_ids=None):
    """Many independent frames packed back to back: random code (uniform over
    `codes`, each a dict with K, gens and optionally terminated / input_kind),
    info length uniform in [len_lo, len_hi] (or `lengths`), Eb/N0 uniform in
    [ebn0_lo, ebn0_hi].  Returns (frames, streams, syms, out_bytes) where
    frames are (sym_offset, n_bits, out_offset, code) tuples and outputs are
    byte aligned, `gap` bytes apart."""
    rng = np.random.default_rng(seed)
    frames, streams = [], []
    sym_off = out_off = 0
    for f in range(n_frames):
        ci = int(code_ids[f]) if code_ids is not None else int(rng.integers(0, len(codes)))
        c = codes[ci]
        n = int(lengths[f]) if lengths is not None else int(rng.integers(len_lo, len_hi + 1))
        ebn0 = float(rng.uniform(ebn0_lo, ebn0_hi))
        st = make_stream(c["K"], c["gens"], n, ebn0, seed=seed * 1000003 + f,
                         kind=c.get("input_kind", SOFT_I8), terminated=c.get("terminated", True))
        frames.append((sym_off, n, out_off, ci))
        streams.append(st)
        sym_off += st["syms"].size
        out_off += (n + 7) // 8 + gap
    syms = np.concatenate([s["syms"] for s in streams]) if streams else np.zeros(0, np.uint8)
    return frames, streams, syms, out_off


def lognormal_lengths(rng: np.random.Generator, n: int, median: float = 1500.0, sigma: float = 1.0,
                      lo: int = 40, hi: int = 65536) -> np.ndarray:
    """Request lengths: log-normal with the given median and sigma (of the
    log), rounded and clipped to [lo, hi]."""
    x = rng.lognormal(mean=math.log(median), sigma=sigma, size=n)
    return np.clip(np.rint(x), lo, hi).astype(np.int64)


def poisson_arrivals(rng: np.random.Generator, n: int, rate: float) -> np.ndarray:
    """Arrival times in seconds of a Poisson process of the given rate."""
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def make_requests(codes, n: int, seed: int, median: float = 1500.0, sigma: float = 1.0,
                  lo: int = 40, hi: int = 65536, ebn0_lo: float = 1.0, ebn0_hi: float = 5.0):
    """Serving requests: code uniform over `codes`, log-normal length,
    Eb/N0 uniform in [ebn0_lo, ebn0_hi].  Returns a list of
    (code index, stream dict)."""
    rng = np.random.default_rng(seed)
    lengths = lognormal_lengths(rng, n, median, sigma, lo, hi)
    out = []
    for i in range(n):
        ci = int(rng.integers(0, len(codes)))
        c = codes[ci]
        ebn0 = float(rng.uniform(ebn0_lo, ebn0_hi))
        st = make_stream(c["K"], c["gens"], int(lengths[i]), ebn0, seed=seed * 1000003 + i,
                         kind=c.get("input_kind", SOFT_I8), terminated=c.get("terminated", True))
        out.append((ci, st))
    return out

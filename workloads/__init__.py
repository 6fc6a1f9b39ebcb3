"""Seeded synthetic inputs for the five PACO semiring-MM workloads.

This module only draws random numbers and lays them out; it holds none of
the multiplication arithmetic.  Both the CPU oracle's tests and the GPU
library's tests and benchmark draw their inputs from it, so both sides see
bit-identical operands.

Generator: counter-based splitmix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): the i-th 64-bit word of stream
s under seed S is  mix(key(S, s) + (i + 1) * 0x9E3779B97F4A7C15)  with
mix(z) = z ^= z>>30; z *= 0xBF58476D1CE4E5B9; z ^= z>>27;
z *= 0x94D049BB133111EB; z ^= z>>31.  key(S, s) = mix(S * 2^20 + s).

Recipes (seed 0 everywhere; each matrix is drawn row-major):
  minplus   : entries uniform in [0, 2^20), each replaced by INF = 2^30 with
              independent probability 0.05
  ring      : float32 N(0,1) by Box-Muller in float64, rounded to nearest
  maxplus   : entries uniform in [-2^15, 2^15)
  boolean   : independent Bernoulli(density) bits, rows packed LSB-first into
              uint32 words with zero padding bits
  strassen  : float32 uniform on the grid {j/2^23 - 1}, i.e. U[-1, 1)
  server    : exponential inter-arrival times, n, m, k log-uniform integers
              in [32, 4096], 70% ring / 30% (min,+) requests
"""
import math

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
INF = 1 << 30

_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z):
    z = z.copy() if isinstance(z, np.ndarray) else np.uint64(z)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def _key(seed, stream):
    return _mix(np.array([(int(seed) << 20) + int(stream)], np.uint64))[0]


def words(seed, stream, count, offset=0):
    """`count` 64-bit words of stream `stream`, starting at counter `offset`."""
    idx = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = _key(seed, stream) + idx * GOLDEN
    return _mix(z)


_CHUNK = 1 << 22   # even, so Box-Muller pairs never straddle two chunks


def _parallel(job, count, chunk=_CHUNK):
    """Run job(start, length) over [0, count) in chunks, on a few threads
    (numpy releases the interpreter lock in its array loops).  Chunks are
    independent: the generator is counter-based."""
    starts = list(range(0, count, chunk))
    if len(starts) <= 1:
        for s in starts:
            job(s, min(chunk, count - s))
        return
    import concurrent.futures as cf
    import os
    workers = max(1, min(16, len(os.sched_getaffinity(0)), len(starts)))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(lambda s: job(s, min(chunk, count - s)), starts))


def _chunked(fn, seed, stream, count, dtype):
    out = np.empty(count, dtype)

    def job(s, c):
        out[s:s + c] = fn(words(seed, stream, c, s))

    _parallel(job, count)
    return out


def uniform01(w):
    """float64 in [0, 1) from the top 53 bits."""
    return (w >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def randint_pow2(seed, stream, shape, lo, log2_range):
    """Integers uniform in [lo, lo + 2^log2_range), exact (top bits)."""
    count = int(np.prod(shape))
    sh = np.uint64(64 - log2_range)
    v = _chunked(lambda w: (w >> sh).astype(np.int64), seed, stream, count, np.int64)
    return (v + lo).reshape(shape)


def bernoulli(seed, stream, shape, p):
    count = int(np.prod(shape))
    return _chunked(lambda w: uniform01(w) < p, seed, stream, count, np.bool_).reshape(shape)


def normal_f32(seed, stream, shape):
    """float32 N(0,1): Box-Muller on pairs of words, rounded to nearest."""
    count = int(np.prod(shape))

    def fn(w):
        half = (w.size + 1) // 2
        w = np.concatenate([w, w[:1]]) if w.size % 2 else w
        u1 = 1.0 - uniform01(w[0::2])          # (0, 1]
        u2 = uniform01(w[1::2])
        r = np.sqrt(-2.0 * np.log(u1))
        z = np.empty(2 * half, np.float64)
        z[0::2] = r * np.cos(2.0 * np.pi * u2)
        z[1::2] = r * np.sin(2.0 * np.pi * u2)
        return z[: w.size].astype(np.float32)

    out = np.empty(count, np.float32)

    def job(s, c):
        out[s:s + c] = fn(words(seed, stream, c + (c % 2), s))[:c]

    _parallel(job, count)
    return out.reshape(shape)


def uniform_pm1_f32(seed, stream, shape):
    """float32 on the grid {j / 2^23 - 1 : 0 <= j < 2^24}, i.e. U[-1, 1)."""
    count = int(np.prod(shape))
    sh = np.uint64(40)
    return _chunked(lambda w: ((w >> sh).astype(np.float64) * (1.0 / (1 << 23)) - 1.0)
                    .astype(np.float32), seed, stream, count, np.float32).reshape(shape)


def pack_bits(bits):
    """Pack a 0/1 (rows, cols) array into (rows, ceil(cols/32)) uint32, LSB first."""
    bits = np.ascontiguousarray(bits, np.uint8)
    rows, cols = bits.shape
    w = (cols + 31) // 32
    padded = np.zeros((rows, w * 32), np.uint8)
    padded[:, :cols] = bits
    by = np.packbits(padded, axis=1, bitorder="little")
    return np.ascontiguousarray(by).view("<u4").reshape(rows, w).astype(np.uint32)


# ----------------------------------------------------------------- recipes

def minplus_matrix(seed, stream, shape, inf_prob=0.05):
    v = randint_pow2(seed, 2 * stream, shape, 0, 20)
    mask = bernoulli(seed, 2 * stream + 1, shape, inf_prob)
    v[mask] = INF
    return v.astype(np.int32)


def minplus_operands(n, m, k, seed=0, inf_prob=0.05):
    return (minplus_matrix(seed, 0, (n, k), inf_prob),
            minplus_matrix(seed, 1, (k, m), inf_prob))


def maxplus_operands(n, m, k, seed=0):
    return (randint_pow2(seed, 10, (n, k), -(1 << 15), 16).astype(np.int32),
            randint_pow2(seed, 11, (k, m), -(1 << 15), 16).astype(np.int32))


def ring_operands(n, m, k, seed=0):
    return normal_f32(seed, 20, (n, k)), normal_f32(seed, 21, (k, m))


def strassen_operands(n, seed=0):
    return uniform_pm1_f32(seed, 30, (n, n)), uniform_pm1_f32(seed, 31, (n, n))


def small_int_operands(n, m, k, seed=0, lo=-2, hi=2):
    """float32 entries in {lo..hi}: every partial sum is an exact integer."""
    span = hi - lo + 1
    a = (words(seed, 40, n * k) % np.uint64(span)).astype(np.int64) + lo
    b = (words(seed, 41, k * m) % np.uint64(span)).astype(np.int64) + lo
    return (a.reshape(n, k).astype(np.float32), b.reshape(k, m).astype(np.float32))


def bool_operands(n, m, k, density=0.05, seed=0):
    """Returns (A_bits, B_bits, A_packed, B_packed)."""
    a = bernoulli(seed, 50, (n, k), density).astype(np.uint8)
    b = bernoulli(seed, 51, (k, m), density).astype(np.uint8)
    return a, b, pack_bits(a), pack_bits(b)


def bool_operands_packed(n, m, k, density=0.05, seed=0):
    _, _, ap, bp = bool_operands(n, m, k, density, seed)
    return ap, bp


def server_stream(count=4096, rate=2000.0, seed=0, dim_lo=32, dim_hi=4096,
                  ring_frac=0.7):
    """Request list: dicts with arrival time (s), kind, n, m, k, seed."""
    w = words(seed, 60, 5 * count).reshape(count, 5)
    u = uniform01(w)
    inter = -np.log(1.0 - u[:, 0]) / rate
    t = np.cumsum(inter) - inter[0]
    lo, hi = math.log(dim_lo), math.log(dim_hi)
    dims = np.clip(np.floor(np.exp(lo + u[:, 1:4] * (hi - lo))), dim_lo, dim_hi).astype(np.int64)
    kinds = np.where(u[:, 4] < ring_frac, "ring", "minplus")
    return [dict(t=float(t[i]), kind=str(kinds[i]), n=int(dims[i, 0]), m=int(dims[i, 1]),
                 k=int(dims[i, 2]), seed=1000 + i) for i in range(count)]


def server_request_operands(req):
    n, m, k, s = req["n"], req["m"], req["k"], req["seed"]
    if req["kind"] == "ring":
        return ring_operands(n, m, k, seed=s)
    return minplus_operands(n, m, k, seed=s)

"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws numbers; it holds none of the sorting method's
arithmetic, and it is the one module that both the oracle-side tests and the
device path take their inputs from.

The paper sorts random permutations of {1..n} of machine integers
(Experiments section); the workloads here widen that to the shapes the
benchmarks use: uniform 32-bit keys, nearly sorted and reverse-sorted keys,
duplicate-heavy Zipf keys with an index payload, float keys (normal and
uniform), and log-uniform segment lengths for batched and served sorting.

Generator: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014) used counter-based: value i of stream
(seed, stream) is the SplitMix64 output mix of  base + (i + 1) * gamma,
where base is itself the mix of seed and stream.  Everything is vectorised
uint64 numpy arithmetic (wrap-around), so a value depends only on
(seed, stream, i).
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    """Values start .. start+count-1 of the counter-based stream (uint64)."""
    with np.errstate(over="ignore"):
        base = _mix(np.array([seed & (2**64 - 1)], dtype=np.uint64) * _GAMMA
                    + np.uint64(stream & (2**64 - 1)))[0]
        idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        return _mix(base + idx * _GAMMA)


def _chunks(n: int, chunk: int = 1 << 24):
    for s in range(0, n, chunk):
        yield s, min(chunk, n - s)


def uniform_u32(n: int, seed: int, stream: int = 0) -> np.ndarray:
    """i.i.d. uniform keys on [0, 2^32): the top 32 bits of each draw."""
    out = np.empty(n, dtype=np.uint32)
    for s, c in _chunks(n):
        out[s:s + c] = (splitmix64(seed, stream, s, c) >> np.uint64(32)).astype(np.uint32)
    return out


def unit_f64(n: int, seed: int, stream: int) -> np.ndarray:
    """i.i.d. uniform doubles on [0, 1) with 53 random bits."""
    out = np.empty(n, dtype=np.float64)
    for s, c in _chunks(n):
        out[s:s + c] = (splitmix64(seed, stream, s, c) >> np.uint64(11)).astype(np.float64) * 2.0**-53
    return out


def sorted_u32(n: int) -> np.ndarray:
    """a[i] = 16 i: sorted, distinct (n <= 2^28)."""
    return (np.arange(n, dtype=np.uint64) * np.uint64(16)).astype(np.uint32)


def reverse_u32(n: int) -> np.ndarray:
    """a[i] = 16 (n - 1 - i): reverse-sorted, distinct."""
    return sorted_u32(n)[::-1].copy()


def sorted_with_swaps_u32(n: int, seed: int, frac: float = 0.01) -> np.ndarray:
    """Sorted keys after floor(frac n) transpositions of uniformly random
    position pairs, applied one after the other."""
    a = sorted_u32(n)
    k = int(frac * n)
    if n < 2 or k == 0:
        return a
    pos = (splitmix64(seed, 1, 0, 2 * k) % np.uint64(n)).astype(np.int64)
    ii, jj = pos[0::2], pos[1::2]
    # transpositions applied in order; conflict-free runs are applied in bulk
    start = 0
    while start < k:
        seen: set[int] = set()
        end = start
        while end < k:
            x, y = int(ii[end]), int(jj[end])
            if x in seen or y in seen:
                break
            seen.add(x)
            seen.add(y)
            end += 1
            if end - start >= 65536:
                break
        xi, yi = ii[start:end], jj[start:end]
        a[xi], a[yi] = a[yi].copy(), a[xi].copy()
        start = end
    return a


def zipf_table(s: float = 1.1, nvals: int = 1024) -> np.ndarray:
    """Cumulative distribution of P(key = r) ~ (r + 1)^-s, r = 0..nvals-1 (fp64)."""
    w = np.arange(1, nvals + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    return cdf / cdf[-1]


def zipf_u32(n: int, seed: int, s: float = 1.1, nvals: int = 1024) -> np.ndarray:
    """Duplicate-heavy keys: Zipf(s) over {0 .. nvals-1} by inverse CDF."""
    cdf = zipf_table(s, nvals)
    out = np.empty(n, dtype=np.uint32)
    for st, c in _chunks(n):
        u = (splitmix64(seed, 2, st, c) >> np.uint64(11)).astype(np.float64) * 2.0**-53
        out[st:st + c] = np.minimum(np.searchsorted(cdf, u, side="right"), nvals - 1)
    return out


def normal_f32(n: int, seed: int, stream: int = 3) -> np.ndarray:
    """N(0,1) floats by Box-Muller in fp64, rounded to binary32.  Never NaN;
    a zero comes out as +0.0."""
    out = np.empty(n, dtype=np.float32)
    for st, c in _chunks(n):
        r = splitmix64(seed, stream, st, c)
        u1 = ((r >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0**-53  # (0, 1]
        u2 = (r & np.uint64((1 << 32) - 1)).astype(np.float64) * 2.0**-32
        z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
        z32 = z.astype(np.float32)
        z32[z32 == 0] = np.float32(0.0)
        out[st:st + c] = z32
    return out


def uniform_f32(n: int, seed: int, stream: int = 4) -> np.ndarray:
    """Uniform floats on [0, 1): (u32 >> 8) * 2^-24, exact in binary32."""
    u = uniform_u32(n, seed, stream)
    return ((u >> np.uint32(8)).astype(np.float32) * np.float32(2.0**-24)).astype(np.float32)


def permutation_u32(n: int, seed: int, stream: int = 7) -> np.ndarray:
    """A random order of 1..n (the paper's inputs: random permutations of
    {1..n}).  Position i holds 1 + P(i) for a bijection P of [0, n): a
    four-round balanced Feistel network on 2h-bit words (2^(2h) >= n) whose
    round functions are SplitMix64 mixes of the other half, the round and
    the (seed, stream) base; values that land at n or above are mapped again
    until they fall inside [0, n) (cycle walking keeps it a bijection)."""
    if n <= 0:
        return np.zeros(0, dtype=np.uint32)
    bits = max(2, int(n - 1).bit_length())
    h = (bits + 1) // 2
    mask = np.uint64((1 << h) - 1)
    base = _mix(np.array([(seed * 0x100000001B3 + stream) % (1 << 64)], dtype=np.uint64))
    rk = [_mix(base + np.full(1, r + 1, dtype=np.uint64) * _GAMMA)[0] for r in range(4)]

    def feistel(x: np.ndarray) -> np.ndarray:
        left, right = x >> np.uint64(h), x & mask
        for r in range(4):
            f = _mix(right ^ rk[r]) & mask
            left, right = right, left ^ f
        return (left << np.uint64(h)) | right

    out = np.empty(n, dtype=np.uint32)
    for a, c in _chunks(n):
        b = a + c
        v = feistel(np.arange(a, b, dtype=np.uint64))
        bad = v >= np.uint64(n)
        while bad.any():
            v[bad] = feistel(v[bad])
            bad = v >= np.uint64(n)
        out[a:b] = (v + np.uint64(1)).astype(np.uint32)
    return out


def log_uniform_lengths(count: int, seed: int, lo_exp: int = 6,
                        hi_exp: int = 20, stream: int = 5) -> np.ndarray:
    """floor(2^(lo + (hi-lo) u)) clamped to [2^lo, 2^hi], u uniform in [0,1)."""
    u = unit_f64(count, seed, stream)
    L = np.floor(2.0 ** (lo_exp + (hi_exp - lo_exp) * u)).astype(np.int64)
    return np.clip(L, 2**lo_exp, 2**hi_exp)


def offsets_from_lengths(lengths: np.ndarray) -> np.ndarray:
    off = np.zeros(len(lengths) + 1, dtype=np.uint64)
    np.cumsum(np.asarray(lengths, dtype=np.uint64), out=off[1:])
    return off


def poisson_arrivals(count: int, rate: float, seed: int, stream: int = 6) -> np.ndarray:
    """Arrival times (s) of an open-loop Poisson stream: gaps -ln(1-u)/rate."""
    u = unit_f64(count, seed, stream)
    return np.cumsum(-np.log1p(-u) / rate)


# Named workloads (sizes, distributions and seeds of the benchmark configs).
WORKLOADS = {
    "uniform_u32_2^20": dict(n=1 << 20, kind="uniform", seed=1),
    "uniform_u32_2^28": dict(n=1 << 28, kind="uniform", seed=2),
    "nearly_sorted_u32_2^28": dict(n=1 << 28, kind="sorted_swaps", seed=3),
    "reverse_u32_2^28": dict(n=1 << 28, kind="reverse", seed=0),
    "zipf_pairs_2^26": dict(n=1 << 26, kind="zipf", seed=4),
}


def make_keys(kind: str, n: int, seed: int) -> np.ndarray:
    if kind == "uniform":
        return uniform_u32(n, seed)
    if kind == "sorted_swaps":
        return sorted_with_swaps_u32(n, seed)
    if kind == "reverse":
        return reverse_u32(n)
    if kind == "sorted":
        return sorted_u32(n)
    if kind == "zipf":
        return zipf_u32(n, seed)
    if kind == "normal_f32":
        return normal_f32(n, seed)
    if kind == "uniform_f32":
        return uniform_f32(n, seed)
    if kind == "equal":
        return np.full(n, 12345, dtype=np.uint32)
    raise ValueError(f"unknown input kind {kind!r}")

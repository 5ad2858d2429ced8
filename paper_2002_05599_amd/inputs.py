"""Seeded synthetic workloads shared by the tests, the bench and the serving demo.

This module generates inputs only; it contains none of the sorting method's
arithmetic, and both the GPU path and the CPU oracle consume what it makes.

Random keys come from SplitMix64 (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used counter-style: value i of
stream ``seed`` is the SplitMix64 output mix(seed*G + (i+1)*G) with
G = 0x9E3779B97F4A7C15.  Sizes (uniform, geometric, Zipf) come from numpy's
PCG64 generator seeded with the same seed.  The paper drew 31-bit keys from
minstd_rand (Section 4.1); a 64-bit generator is used instead so that keys
cover the full range of every key type.

Workload shapes (all seeded):
  * ``fixed_keys``      -- count arrays of n keys at stride n, one of four
                           distributions: uniform, few (values in [0,4)),
                           sorted, reverse.
  * ``csr_sizes``       -- segment sizes uniform in [lo, hi], int32 CSR offsets.
  * ``geometric_sizes`` -- truncated geometric sizes (mean ~24, range 1..256).
  * ``zipf_keys``       -- int32 ranks r >= 1 with P(r) ~ r^-s, r < 2^31.
  * ``distinct_u64``    -- distinct uint64 keys (bijective mix of a counter).
"""
import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

DISTRIBUTIONS = ("uniform", "few", "sorted", "reverse")


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (a bijection on 64-bit words)."""
    z = z.copy()
    z ^= z >> np.uint64(30)
    z *= _M1
    z ^= z >> np.uint64(27)
    z *= _M2
    z ^= z >> np.uint64(31)
    return z


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """``count`` 64-bit words of stream ``seed`` beginning at index ``start``."""
    with np.errstate(over="ignore"):
        base = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) * GOLDEN
        ctr = np.arange(start + 1, start + count + 1, dtype=np.uint64) * GOLDEN + base
        return _mix64(ctr)


def random_keys(dtype, count: int, seed: int) -> np.ndarray:
    """Uniform keys over the full range of ``dtype`` (u32/i32/u64/i64); for
    float32/float64, uniformly random bit patterns (every class of value:
    normal, subnormal, zeros, infinities and NaNs of both signs)."""
    dt = np.dtype(dtype)
    w = splitmix64(seed, count)
    if dt.itemsize == 4:
        return (w >> np.uint64(32)).astype(np.uint32).view(dt)
    return w.view(dt)


def float_keys(dtype, count: int, seed: int) -> np.ndarray:
    """Float keys for the tests: 60% values spread over many magnitudes (a
    sign, a 53-bit fraction and a power of two in [2^-40, 2^40]), 35% random
    bit patterns (every class of value), 5% special values (+-0, +-inf,
    +-NaN, +-1), which also makes duplicates."""
    dt = np.dtype(dtype)
    w = splitmix64(seed, 3 * count).reshape(3, count) if count else np.zeros((3, 0), np.uint64)
    frac = (w[0] >> np.uint64(11)).astype(np.float64) / float(1 << 53)
    mag = np.ldexp(0.5 + frac / 2, ((w[1] >> np.uint64(58)).astype(np.int64) - 32) * 5 // 4)
    vals = np.where((w[1] & np.uint64(1)) == 1, -mag, mag).astype(dt)
    if dt.itemsize == 4:
        bits = (w[2] >> np.uint64(32)).astype(np.uint32).view(dt)
    else:
        bits = w[2].view(dt)
    pick = (w[2] % np.uint64(100)).astype(np.int64)
    specials = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, -np.nan, 1.0, -1.0], dtype=dt)
    specials[5] = np.copysign(specials[4], -1.0)
    out = np.where(pick < 60, vals, bits)
    sp = pick >= 95
    out[sp] = specials[(w[0][sp] % np.uint64(8)).astype(np.int64)]
    return np.ascontiguousarray(out.astype(dt))


def fixed_keys(dtype, n: int, count: int, dist: str, seed: int) -> np.ndarray:
    """``count`` arrays of ``n`` keys packed at stride n, flattened."""
    dt = np.dtype(dtype)
    total = n * count
    if dist == "uniform":
        return random_keys(dt, total, seed)
    if dist == "few":
        w = splitmix64(seed, total) >> np.uint64(62)  # uniform in [0, 4)
        return w.astype(dt)
    if dist in ("sorted", "reverse"):
        a = random_keys(dt, total, seed).reshape(count, n) if n else np.zeros((count, 0), dt)
        a = np.sort(a, axis=1)
        if dist == "reverse":
            a = a[:, ::-1]
        return np.ascontiguousarray(a).reshape(-1)
    raise ValueError(f"unknown distribution {dist!r}")


def offsets_from_sizes(sizes: np.ndarray) -> np.ndarray:
    off = np.zeros(sizes.size + 1, dtype=np.int64)
    np.cumsum(sizes, out=off[1:])
    if off[-1] >= 2**31:
        raise ValueError("total size exceeds int32 offsets")
    return off.astype(np.int32)


def csr_sizes(nseg: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Segment sizes uniform in [lo, hi] (inclusive)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(lo, hi + 1, size=nseg, dtype=np.int64)


def geometric_sizes(nseg: int, seed: int, mean: float = 24.0, cap: int = 256) -> np.ndarray:
    """Sizes ~ Geometric(p=1/mean) on {1, 2, ...}, redrawing values above ``cap``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = rng.geometric(1.0 / mean, size=nseg).astype(np.int64)
    bad = s > cap
    while bad.any():
        s[bad] = rng.geometric(1.0 / mean, size=int(bad.sum()))
        bad = s > cap
    return s


def zipf_keys(count: int, seed: int, s: float = 1.1) -> np.ndarray:
    """int32 ranks r >= 1 with P(r) proportional to r^-s, redrawing r >= 2^31."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r = rng.zipf(s, size=count)
    bad = r >= 2**31
    while bad.any():
        r[bad] = rng.zipf(s, size=int(bad.sum()))
        bad = r >= 2**31
    return r.astype(np.int32)


def distinct_u64(count: int, seed: int) -> np.ndarray:
    """Distinct uint64 keys: the SplitMix64 mix (a bijection) of distinct counters."""
    with np.errstate(over="ignore"):
        ctr = np.arange(count, dtype=np.uint64) + np.uint64((seed & 0xFFFF) << 40)
        return _mix64(ctr)


def segment_index_payload(offsets: np.ndarray) -> np.ndarray:
    """uint32 payload = each item's index within its segment."""
    off = offsets.astype(np.int64)
    total = int(off[-1] - off[0])
    sizes = np.diff(off)
    seg_start = np.repeat(off[:-1] - off[0], sizes)
    return (np.arange(total, dtype=np.int64) - seg_start).astype(np.uint32)


# --- the five workload recipes -------------------------------------------

def config1(seed: int = 1):
    """100,000 arrays of n=8 uint32 keys, uniform, stride 8."""
    return fixed_keys(np.uint32, 8, 100_000, "uniform", seed)


def config3(nseg: int = 1 << 20, dist: str = "uniform", seed: int = 3):
    """CSR int32 segments, sizes uniform in [17, 256]; uniform or Zipf(1.1) keys."""
    off = offsets_from_sizes(csr_sizes(nseg, 17, 256, seed))
    total = int(off[-1])
    if dist == "uniform":
        keys = random_keys(np.int32, total, seed)
    elif dist == "zipf":
        keys = zipf_keys(total, seed)
    else:
        raise ValueError(dist)
    return keys, off


def config4(nseg: int = 10_000_000, seed: int = 4):
    """Ragged batch: geometric sizes (mean 24, 1..256), distinct u64 keys, u32 payload."""
    off = offsets_from_sizes(geometric_sizes(nseg, seed))
    total = int(off[-1])
    keys = distinct_u64(total, seed)
    vals = segment_index_payload(off)
    return keys, vals, off


def serving_request(rid: int, seed: int = 5, max_segments: int = 100_000):
    """One serving request: 1..max_segments segments, sizes U{2..256}, u32 uniform keys."""
    rng = np.random.Generator(np.random.PCG64([seed, rid]))
    nseg = int(rng.integers(1, max_segments + 1))
    sizes = rng.integers(2, 257, size=nseg, dtype=np.int64)
    off = offsets_from_sizes(sizes)
    keys = random_keys(np.uint32, int(off[-1]), (seed << 32) ^ (rid + 1))
    return keys, off

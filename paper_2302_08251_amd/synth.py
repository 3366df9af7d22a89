"""Seeded synthetic inputs (numpy PCG64) for tests and the benchmark.

This module only draws random numbers; it holds none of the mappings' or
codecs' arithmetic.  Every generator returns per-field planes (one numpy
array per leaf field), which is exactly the content of a SoA multi-blob
view, so no layout code is needed to turn them into blobs.

Recipes (the paper has no datasets; these stand in for its particle and
integer workloads):
  particles        pos ~ U[-1, 1], vel ~ N(0, 0.1), mass ~ U[0.5, 1], drawn
                   field by field (all pos.x, then pos.y, ... then mass).
  random_bit_planes  uniform 32-bit patterns (every NaN payload, denormal and
                   infinity appears), for bit-exact copy checks.
  float_specials   f32 N(0, 1); each element independently becomes +-Inf with
                   probability 1%, NaN (random sign, mantissa uniform in
                   [1, 2^23), so quiet and signalling) with 1%, a denormal
                   (random sign, mantissa uniform in [1, 2^23)) with 1%.
  int_values       signed int32 uniform over [-2^(B-1), 2^(B-1)).
  changetype_values  particle distribution in f64, the same special mix as
                   float_specials (in f64 form), plus 0.1% values with
                   |x| > FLT_MAX and 0.1% with |x| < 2^-150.
  batch_views      2000 record counts rint(exp(U(ln 1e3, ln 4e6))), then 2000
                   mapping-pair indices integers(0, 30) from the same generator.
"""
import numpy as np

FIELDS = ("pos.x", "pos.y", "pos.z", "vel.x", "vel.y", "vel.z", "mass")


def particles(n, seed=0, dtype=np.float64):
    rng = np.random.default_rng(seed)
    planes = [rng.uniform(-1.0, 1.0, n) for _ in range(3)]
    planes += [rng.normal(0.0, 0.1, n) for _ in range(3)]
    planes.append(rng.uniform(0.5, 1.0, n))
    return [np.ascontiguousarray(p.astype(dtype)) for p in planes]


def random_bit_planes(n, n_fields=7, seed=0, bits=32):
    rng = np.random.default_rng(seed)
    dt = {8: np.uint8, 16: np.uint16, 32: np.uint32, 64: np.uint64}[bits]
    return [rng.integers(0, np.iinfo(dt).max, n, dtype=dt, endpoint=True) for _ in range(n_fields)]


def _special_mix_f32_bits(rng, n, base_bits):
    """Overwrites ~1% each of base_bits (uint32 f32 patterns) with Inf, NaN, denormals."""
    u = rng.random(n)
    sign = rng.integers(0, 2, n, dtype=np.uint32) << np.uint32(31)
    mant = rng.integers(1, 1 << 23, n, dtype=np.uint32)
    out = base_bits.copy()
    inf = u < 0.01
    nan = (u >= 0.01) & (u < 0.02)
    den = (u >= 0.02) & (u < 0.03)
    out[inf] = sign[inf] | np.uint32(0x7F800000)
    out[nan] = sign[nan] | np.uint32(0x7F800000) | mant[nan]
    out[den] = sign[den] | mant[den]
    return out


def float_specials(n, seed=0):
    """One f32 plane (as uint32 bit patterns) with the special-value mix."""
    rng = np.random.default_rng(seed)
    base = rng.standard_normal(n, dtype=np.float32).view(np.uint32)
    return _special_mix_f32_bits(rng, n, base)


def int_values(n, bits, seed=0):
    rng = np.random.default_rng(seed)
    return rng.integers(-(1 << (bits - 1)), 1 << (bits - 1), n, dtype=np.int64).astype(np.int32)


def uint_values(n, bits, seed=0):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 1 << bits, n, dtype=np.uint64).astype(np.uint32)


def changetype_values(n, seed=0, n_fields=7):
    """f64 planes: particle values, special mix, out-of-f32-range magnitudes."""
    rng = np.random.default_rng(seed)
    planes = particles(n, seed=seed, dtype=np.float64)[:n_fields]
    out = []
    for p in planes:
        bits = p.view(np.uint64).copy()
        u = rng.random(n)
        sign = rng.integers(0, 2, n, dtype=np.uint64) << np.uint64(63)
        mant = rng.integers(1, 1 << 52, n, dtype=np.uint64)
        inf = u < 0.01
        nan = (u >= 0.01) & (u < 0.02)
        den = (u >= 0.02) & (u < 0.03)
        big = (u >= 0.03) & (u < 0.031)
        tiny = (u >= 0.031) & (u < 0.032)
        bits[inf] = sign[inf] | np.uint64(0x7FF0000000000000)
        bits[nan] = sign[nan] | np.uint64(0x7FF0000000000000) | mant[nan]
        # f32 denormal magnitudes expressed in f64: U(0, 2^-126)
        dv = rng.uniform(0.0, 2.0 ** -126, n)
        bits[den] = sign[den] | dv.view(np.uint64)[den]
        bv = np.exp(rng.uniform(np.log(3.5e38), np.log(1e300), n))
        bits[big] = sign[big] | bv.view(np.uint64)[big]
        tv = np.exp(rng.uniform(np.log(1e-300), np.log(2.0 ** -150), n))
        bits[tiny] = sign[tiny] | tv.view(np.uint64)[tiny]
        out.append(bits.view(np.float64))
    return out


def batch_views(count=2000, seed=0, lo=1e3, hi=4e6, n_pairs=30):
    rng = np.random.default_rng(seed)
    n = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), count))).astype(np.int64)
    pairs = rng.integers(0, n_pairs, count)
    return n, pairs


def narrow_range_values(n, seed=0, dtype=np.float32):
    """One plane (as unsigned bit patterns) of values around the f16 / bf16
    ranges: log-uniform magnitudes over 2^-30 .. 2^20 with random signs; a
    quarter of them with the mantissa bits below a 10- or 7-bit mantissa set
    to exactly half a unit (rounding ties); then the special-value mix."""
    rng = np.random.default_rng(seed)
    mag = np.exp2(rng.uniform(-30.0, 20.0, n)).astype(dtype)
    vals = np.where(rng.integers(0, 2, n) == 1, -mag, mag).astype(dtype)
    if dtype == np.float32:
        bits = vals.view(np.uint32).copy()
        drop = np.where(rng.integers(0, 2, n) == 1, 13, 16).astype(np.uint32)
        one = np.uint32(1)
    else:
        bits = vals.view(np.uint64).copy()
        drop = np.where(rng.integers(0, 2, n) == 1, 42, 45).astype(np.uint64)
        one = np.uint64(1)
    tie = rng.random(n) < 0.25
    low = (one << drop) - one
    bits[tie] = (bits[tie] & ~low[tie]) | (one << (drop[tie] - one))
    if dtype == np.float32:
        return _special_mix_f32_bits(rng, n, bits)
    # f64: ~1 % each of infinities, NaNs with random payloads, denormals
    u = rng.random(n)
    sign = rng.integers(0, 2, n, dtype=np.uint64) << np.uint64(63)
    mant = rng.integers(1, 1 << 52, n, dtype=np.uint64)
    inf, nan, den = u < 0.01, (u >= 0.01) & (u < 0.02), (u >= 0.02) & (u < 0.03)
    bits[inf] = sign[inf] | np.uint64(0x7FF0000000000000)
    bits[nan] = sign[nan] | np.uint64(0x7FF0000000000000) | mant[nan]
    bits[den] = sign[den] | mant[den]
    return bits

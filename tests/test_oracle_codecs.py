"""Pins of the oracle's computed mappings (CPU only).

BitPackedIntSoA   - Python big-int stream closed form; B = 8/16/32 equal numpy casts.
BitPackedFloatSoA - exact-rational brute force over every (E, M) for float32 (the code
                    is the largest-magnitude representable value <= |x|, overflow to
                    Inf), E = 8 closed form (bits >> (23 - M)), e5m10 against numpy
                    float16, decode of every code of small formats, pack(unpack(c)) = c.
ChangeType        - numpy astype (float64 <-> float32, float16), torch bfloat16, all with
                    round to nearest even; NaN rule from hand-worked payload examples.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def golden(kind):
    with open(os.path.join(GOLD, "codec_examples.jsonl")) as f:
        for line in f:
            d = json.loads(line)
            if d.get("codec") == kind:
                yield d


# ---------------------------------------------------------------- golden examples

@pytest.mark.parametrize("d", list(golden("float")), ids=lambda d: d["cite"][:40])
def test_float_encode_examples(d):
    assert oracle.float_encode(int(d["in"], 16), d["type"], d["E"], d["M"]) == int(d["code"], 16)


@pytest.mark.parametrize("d", list(golden("float_decode")), ids=lambda d: d["cite"][:40])
def test_float_decode_examples(d):
    assert oracle.float_decode(int(d["code"], 16), d["type"], d["E"], d["M"]) == int(d["out"], 16)


@pytest.mark.parametrize("d", list(golden("convert")), ids=lambda d: d["cite"][:40])
def test_convert_examples(d):
    assert oracle.convert(int(d["in"], 16), d["from"], d["to"]) == int(d["out"], 16)


@pytest.mark.parametrize("d", list(golden("int_stream")), ids=lambda d: d["cite"][:30])
def test_int_stream_examples(d):
    t = "i32" if d["signed"] else "u32"
    vals = np.array(d["values"], dtype=np.int64).astype(np.int32 if d["signed"] else np.uint32)
    blobs = oracle.store_planes([t], {"kind": "bitpack_int", "bits": d["bits"]}, [vals])
    assert blobs[0].tobytes().hex() == d["bytes_hex"]
    back = oracle.load_planes([t], {"kind": "bitpack_int", "bits": d["bits"]}, blobs, len(vals))
    assert np.array_equal(back[0], vals)


# ---------------------------------------------------------------- BitPackedInt

@pytest.mark.parametrize("B", [1, 2, 3, 5, 7, 8, 11, 12, 13, 16, 17, 24, 31, 32])
@pytest.mark.parametrize("signed", [False, True])
def test_bitpack_int_big_int_closed_form(B, signed):
    rng = np.random.default_rng(B)
    n = 203
    t = "i32" if signed else "u32"
    vals = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    vals = vals.view(np.int32) if signed else vals
    blobs = oracle.store_planes([t, t], {"kind": "bitpack_int", "bits": B}, [vals, vals[::-1].copy()])
    nbytes = 4 * ((n * B + 31) // 32)
    for f, v in enumerate([vals, vals[::-1]]):
        big = sum((int(x) % (1 << B)) << (i * B) for i, x in enumerate(v.tolist()))
        assert blobs[f].tobytes() == big.to_bytes(nbytes, "little")
    back = oracle.load_planes([t, t], {"kind": "bitpack_int", "bits": B}, blobs, n)
    low = vals.astype(np.int64) % (1 << B)
    if signed:
        exp = np.where(low >= (1 << (B - 1)), low - (1 << B), low)
    else:
        exp = low
    assert np.array_equal(back[0].astype(np.int64), exp)


@pytest.mark.parametrize("B,dt", [(8, np.uint8), (16, np.uint16), (32, np.uint32)])
def test_bitpack_int_byte_widths_equal_numpy_cast(B, dt):
    rng = np.random.default_rng(0)
    vals = rng.integers(0, 2 ** 32, 1000, dtype=np.uint64).astype(np.uint32)
    blob = oracle.store_planes(["u32"], {"kind": "bitpack_int", "bits": B}, [vals])[0]
    exp = vals.astype(dt).view(np.uint8)
    assert np.array_equal(blob[: len(exp)], exp)
    assert not blob[len(exp):].any()


def test_bitpack_int_64bit_fields():
    rng = np.random.default_rng(1)
    vals = rng.integers(-2 ** 63, 2 ** 63, 99, dtype=np.int64)
    for B in (1, 33, 40, 63, 64):
        blobs = oracle.store_planes(["i64"], {"kind": "bitpack_int", "bits": B}, [vals])
        back = oracle.load_planes(["i64"], {"kind": "bitpack_int", "bits": B}, blobs, 99)[0]
        for a, b in zip(vals.tolist(), back.tolist()):
            low = a % (1 << B)
            exp = low - (1 << B) if low >= (1 << (B - 1)) else low
            assert b == exp


# ---------------------------------------------------------------- BitPackedFloat brute force

def decode_exact(code, E, M):
    """Exact value of a [sign|E|M] code (independent definition), None for NaN."""
    s = (code >> (E + M)) & 1
    e = (code >> M) & ((1 << E) - 1)
    m = code & ((1 << M) - 1)
    bias = (1 << (E - 1)) - 1
    if e == (1 << E) - 1:
        if m:
            return None
        return float("-inf") if s else float("inf")
    if e == 0:
        v = Fraction(m, 1 << M) * Fraction(2) ** (1 - bias)
    else:
        v = (1 + Fraction(m, 1 << M)) * Fraction(2) ** (e - bias)
    return -v if s else v


def encode_reference(x32, E, M):
    """Largest-magnitude representable value <= |x| (truncation), Inf when the exponent
    exceeds the bias; found by bisection over the monotone positive codes."""
    bits = int(np.float32(x32).view(np.uint32))
    sign = bits >> 31
    ax = abs(Fraction(float(np.float32(x32))))
    bias = (1 << (E - 1)) - 1
    inf_code = ((1 << E) - 1) << M
    if ax >= Fraction(2) ** (bias + 1):
        c = inf_code
    else:
        lo, hi = 0, inf_code - 1  # decode(lo) = 0 <= ax
        while lo < hi:
            mid = (lo + hi + 1) // 2
            if decode_exact(mid, E, M) <= ax:
                lo = mid
            else:
                hi = mid - 1
        c = lo
    return c | (sign << (E + M))


def probe_values(E, M, rng):
    bias = (1 << (E - 1)) - 1
    vals = [0.0, -0.0, 1.0, -1.0, 3.0, 0.1, -2.5e-3, 1e30, -1e-30, 3.4e38, 1e-40, -1e-45]
    # edges of the target format: max finite, overflow threshold, min normal, min subnormal
    maxfin = float((2 - Fraction(1, 1 << M)) * Fraction(2) ** bias)
    minnorm = float(Fraction(2) ** (1 - bias))
    minsub = float(Fraction(2) ** (1 - bias - M))
    for v in (maxfin, 2.0 ** (bias + 1), minnorm, minsub, minsub / 2, minsub * 1.5, minnorm * 0.75):
        if v < 3.4e38:
            f = np.float32(v)
            vals += [float(f), float(np.nextafter(f, np.float32(0))), float(np.nextafter(f, np.float32(np.inf)))]
    rb = rng.integers(0, 2 ** 32, 60, dtype=np.uint64).astype(np.uint32)
    rb = rb[(rb & 0x7F800000) != 0x7F800000]
    vals += [float(x) for x in rb.view(np.float32)]
    # values near 1 in magnitude exercise mantissa truncation
    vals += [float(x) for x in rng.standard_normal(20).astype(np.float32)]
    return [v for v in vals if np.isfinite(np.float32(v))]


@pytest.mark.parametrize("E", list(range(2, 9)))
def test_float_encode_brute_force_all_formats(E):
    rng = np.random.default_rng(E)
    for M in range(0, 24):
        for v in probe_values(E, M, rng):
            bits = int(np.float32(v).view(np.uint32))
            got = oracle.float_encode(bits, "f32", E, M)
            assert got == encode_reference(v, E, M), (E, M, hex(bits))
        # infinities
        inf_code = ((1 << E) - 1) << M
        assert oracle.float_encode(0x7F800000, "f32", E, M) == inf_code
        assert oracle.float_encode(0xFF800000, "f32", E, M) == inf_code | (1 << (E + M))


@pytest.mark.parametrize("E,M", [(E, M) for E in range(2, 9) for M in range(0, 24) if 1 + E + M <= 12])
def test_float_decode_all_codes_small_formats(E, M):
    width = 1 + E + M
    for code in range(1 << width):
        got = oracle.float_decode(code, "f32", E, M)
        v = decode_exact(code, E, M)
        if v is None:
            e_all = ((1 << E) - 1) << M
            m = code & ((1 << M) - 1)
            exp = ((code >> (E + M)) << 31) | 0x7F800000 | (m << (23 - M))
            assert got == exp
            continue
        f = np.float32(float(v))
        assert float(f) == v  # representable
        exp = int(f.view(np.uint32))
        if v == 0 and (code >> (E + M)):
            exp = 0x80000000
        assert got == exp, (E, M, code)


@pytest.mark.parametrize("E,M", [(5, 10), (8, 7), (8, 15), (3, 4), (6, 13), (8, 23), (4, 0)])
def test_float_pack_unpack_roundtrip(E, M):
    width = 1 + E + M
    if width <= 20:
        codes = np.arange(1 << width, dtype=np.uint64)
    else:
        rng = np.random.default_rng(width)
        codes = rng.integers(0, 1 << width, 1 << 20, dtype=np.uint64)
    dec = oracle.float_decode_array(codes, "f32", E, M)
    enc = oracle.float_encode_array(dec, "f32", E, M)
    e = (codes >> np.uint64(M)) & np.uint64((1 << E) - 1)
    m = codes & np.uint64((1 << M) - 1)
    isnan = (e == np.uint64((1 << E) - 1)) & (m != 0)
    if M > 0:
        quiet = (m >> np.uint64(M - 1)) & np.uint64(1)
        keep = ~isnan | (quiet == 1)
    else:
        keep = ~isnan
    assert np.array_equal(enc[keep], codes[keep])
    if M > 0:  # signalling NaN codes come back quiet
        q = codes[isnan] | np.uint64(1 << (M - 1))
        assert np.array_equal(enc[isnan], q)


def strided_f32(stride=257, offset=0):
    return (np.arange(offset, 1 << 32, stride, dtype=np.uint64)).astype(np.uint32)


def closed_form_e8(bits, M):
    sh = np.uint32(23 - M)
    code = bits >> sh
    isnan = (bits & np.uint32(0x7F800000)) == np.uint32(0x7F800000)
    isnan &= (bits & np.uint32(0x7FFFFF)) != 0
    if M > 0:
        code = np.where(isnan, code | np.uint32(1 << (M - 1)), code)
    else:
        code = np.where(isnan, (bits >> np.uint32(31) << np.uint32(8)) | np.uint32(0xFF), code)
    return code.astype(np.uint64)


def closed_form_e5m10(bits):
    x = bits.view(np.float32)
    with np.errstate(over="ignore", invalid="ignore"):
        r = x.astype(np.float16)  # round to nearest even
        away = np.abs(r.astype(np.float32)) > np.abs(x)
    t = np.where(away, np.nextafter(r, np.float16(0)), r).astype(np.float16)
    code = t.view(np.uint16).astype(np.uint64)
    sign = (bits >> np.uint32(31)).astype(np.uint64) << np.uint64(15)
    with np.errstate(invalid="ignore"):
        big = np.abs(x) >= np.float32(65536.0)
    code = np.where(big, sign | np.uint64(0x7C00), code)
    isnan = np.isnan(x)
    m = (bits >> np.uint32(13)) & np.uint32(0x3FF)
    nan_code = ((bits >> np.uint32(31)).astype(np.uint64) << np.uint64(15)) | np.uint64(0x7C00) | \
        m.astype(np.uint64) | np.uint64(0x200)
    return np.where(isnan, nan_code, code)


@pytest.mark.parametrize("E,M", [(8, 7), (8, 15), (8, 0), (8, 23), (5, 10)])
def test_float_encode_strided_closed_forms(E, M):
    bits = strided_f32(stride=255 if (E, M) != (5, 10) else 1021)
    got = oracle.float_encode_array(bits, "f32", E, M)
    exp = closed_form_e8(bits, M) if E == 8 else closed_form_e5m10(bits)
    bad = np.nonzero(got != exp)[0]
    assert len(bad) == 0, [hex(int(b)) for b in bits[bad[:5]]]


def test_e5m10_decode_equals_numpy_float16():
    codes = np.arange(1 << 16, dtype=np.uint64)
    dec = oracle.float_decode_array(codes, "f32", 5, 10)
    ref = codes.astype(np.uint16).view(np.float16).astype(np.float32)
    ok = ~np.isnan(ref)
    assert np.array_equal(dec.view(np.uint32)[ok], ref.view(np.uint32)[ok])


def test_float_monotone_and_not_larger():
    rng = np.random.default_rng(7)
    x = np.sort(rng.standard_normal(20000).astype(np.float32) * np.float32(1e3))
    for E, M in [(5, 10), (8, 7), (8, 15), (3, 2), (6, 9)]:
        enc = oracle.float_encode_array(x, "f32", E, M)
        dec = oracle.float_decode_array(enc, "f32", E, M)
        fin = np.isfinite(dec)
        assert np.all(np.abs(dec[fin]) <= np.abs(x[fin]))
        d = dec[fin].astype(np.float64)
        assert np.all(np.diff(d) >= 0)


def test_float_encode_from_f64_matches_f32_path_for_e8m15():
    """For double user values the e8m15 code equals (f32 truncation of x) >> 8 whenever the
    double is inside float range (truncation composes)."""
    rng = np.random.default_rng(11)
    x = rng.standard_normal(5000) * 10.0 ** rng.integers(-30, 30, 5000)
    c64 = oracle.float_encode_array(x, "f64", 8, 15)
    # truncate double -> float32 toward zero via the e8m23 code of the double
    t32 = oracle.float_encode_array(x, "f64", 8, 23).astype(np.uint32)
    c32 = oracle.float_encode_array(t32.view(np.float32), "f32", 8, 15)
    assert np.array_equal(c64, c32)


# ---------------------------------------------------------------- ChangeType

def test_changetype_f64_to_f32_equals_numpy():
    rng = np.random.default_rng(3)
    x = np.concatenate([
        rng.standard_normal(200000),
        rng.standard_normal(20000) * 1e-40, rng.standard_normal(20000) * 1e-44,
        rng.standard_normal(20000) * 3.4e38, np.array([3.4028235677973366e38, 3.4028235677973367e38,
                                                        3.40282357e38, 1e-300, -1e-300, 0.0, -0.0,
                                                        np.inf, -np.inf, 2.0 ** -150, 2.0 ** -149 * 1.5]),
        rng.integers(0, 2 ** 63, 100000, dtype=np.uint64).view(np.float64)])
    x = x[~np.isnan(x)]
    got = oracle.convert_array(x, "f64", "f32")
    with np.errstate(over="ignore"):
        ref = x.astype(np.float32)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_changetype_f32_to_f64_equals_numpy():
    bits = strided_f32(stride=1009)
    x = bits.view(np.float32)
    ok = ~np.isnan(x)
    got = oracle.convert_array(x, "f32", "f64")
    assert np.array_equal(got.view(np.uint64)[ok], x[ok].astype(np.float64).view(np.uint64))
    nanb = bits[~ok]
    exp = ((nanb.astype(np.uint64) >> np.uint64(31)) << np.uint64(63)) | np.uint64(0x7FF8000000000000) | \
        ((nanb.astype(np.uint64) & np.uint64(0x7FFFFF)) << np.uint64(29))
    assert np.array_equal(got.view(np.uint64)[~ok], exp)


def test_changetype_f32_to_f16_equals_numpy():
    bits = strided_f32(stride=263)
    x = bits.view(np.float32)
    ok = ~np.isnan(x)
    got = oracle.convert_array(x[ok], "f32", "f16")
    with np.errstate(over="ignore"):
        ref = x[ok].astype(np.float16)
    assert np.array_equal(got.view(np.uint16), ref.view(np.uint16))


def test_changetype_f64_to_f16_equals_numpy():
    rng = np.random.default_rng(9)
    x = rng.standard_normal(300000) * 10.0 ** rng.integers(-9, 6, 300000)
    got = oracle.convert_array(x, "f64", "f16")
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16)
    assert np.array_equal(got.view(np.uint16), ref.view(np.uint16))


def test_changetype_f32_to_bf16_equals_torch():
    torch = pytest.importorskip("torch")
    bits = strided_f32(stride=269)
    x = bits.view(np.float32)
    ok = ~np.isnan(x)
    got = oracle.convert_array(x[ok], "f32", "bf16")
    ref = torch.from_numpy(x[ok].copy()).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(got.view(np.uint16), ref)


def test_changetype_integer_conversions():
    rng = np.random.default_rng(2)
    v = rng.integers(-2 ** 63, 2 ** 63, 1000, dtype=np.int64)
    assert np.array_equal(oracle.convert_array(v, "i64", "i32"), v.astype(np.int32))
    assert np.array_equal(oracle.convert_array(v.astype(np.int16), "i16", "i64"), v.astype(np.int16).astype(np.int64))
    assert np.array_equal(oracle.convert_array(v.astype(np.uint16), "u16", "i64"), v.astype(np.uint16).astype(np.int64))


def test_changetype_view_roundtrip():
    rec = ["f64"] * 3
    rng = np.random.default_rng(4)
    planes = [rng.standard_normal(50) for _ in range(3)]
    spec = {"kind": "changetype", "stored": ["f32"] * 3, "inner": {"kind": "aosoa", "lanes": 8}}
    blobs = oracle.store_planes(rec, spec, planes)
    back = oracle.load_planes(rec, spec, blobs, 50)
    for p, q in zip(planes, back):
        assert np.array_equal(q, p.astype(np.float32).astype(np.float64))


@pytest.mark.exhaustive
@pytest.mark.parametrize("E,M", [(8, 7), (8, 15), (5, 10)])
def test_float_encode_all_2_32(E, M):
    for off in range(0, 1 << 32, 1 << 28):
        bits = np.arange(off, off + (1 << 28), dtype=np.uint64).astype(np.uint32)
        got = oracle.float_encode_array(bits, "f32", E, M)
        exp = closed_form_e8(bits, M) if E == 8 else closed_form_e5m10(bits)
        assert np.array_equal(got, exp)


# ---------------------------------------------------------------- BitPackedFloat, round to nearest even
# Sec. 3 only asks that the mantissa be "preserved as best as possible"; the
# mapping truncates by default and rounds to nearest, ties to even, when its
# round flag asks for it.  Ties compare the significand's last bit, which for
# M = 0 is the (always set) hidden bit: there a tie rounds away from zero.

def encode_rne_reference(x, E, M):
    """Nearest representable value (independent exact-rational definition)."""
    f = float(x)
    sign = 1 if np.signbit(f) else 0
    ax = abs(Fraction(f))
    bias = (1 << (E - 1)) - 1
    inf_code = ((1 << E) - 1) << M
    top = Fraction(2) ** (bias + 1)  # the next value after the largest finite one
    if ax >= top:
        return inf_code | (sign << (E + M))
    lo, hi = 0, inf_code - 1
    while lo < hi:  # largest code whose value is <= ax
        mid = (lo + hi + 1) // 2
        if decode_exact(mid, E, M) <= ax:
            lo = mid
        else:
            hi = mid - 1
    lo_v = decode_exact(lo, E, M)
    hi_v = decode_exact(lo + 1, E, M) if lo + 1 < inf_code else top
    if ax - lo_v < hi_v - ax:
        c = lo
    elif ax - lo_v > hi_v - ax:
        c = lo + 1
    else:
        even = (lo & 1) == 0 if M >= 1 else lo == 0
        c = lo if even else lo + 1
    return c | (sign << (E + M))


def tie_values(E, M, rng, k=40):
    """f32 values exactly halfway between two neighbouring codes."""
    bias = (1 << (E - 1)) - 1
    out = []
    for c in rng.integers(0, ((1 << E) - 1) << M, k):
        c = int(c)
        a = decode_exact(c, E, M)
        b = decode_exact(c + 1, E, M) if c + 1 < ((1 << E) - 1) << M else Fraction(2) ** (bias + 1)
        mid = (a + b) / 2
        f = np.float32(float(mid))
        if np.isfinite(f) and Fraction(float(f)) == mid:
            out += [float(f), -float(f)]
    return out


@pytest.mark.parametrize("E", list(range(2, 9)))
def test_float_encode_rne_brute_force(E):
    rng = np.random.default_rng(100 + E)
    for M in (0, 1, 2, 3, 7, 10, 15, 23):
        for v in probe_values(E, M, rng) + tie_values(E, M, rng):
            bits = int(np.float32(v).view(np.uint32))
            got = int(oracle.float_encode_array(np.array([bits], np.uint32).view(np.float32), "f32", E, M, rne=True)[0])
            assert got == encode_rne_reference(np.float32(v), E, M), (E, M, hex(bits))


def test_float_encode_rne_e5m10_equals_numpy_float16():
    x = strided_f32(stride=263).view(np.float32)
    x = x[~np.isnan(x)]
    got = oracle.float_encode_array(x, "f32", 5, 10, rne=True)
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16).view(np.uint16)
    assert np.array_equal(got.astype(np.uint16), ref)


def test_float_encode_rne_e8m7_equals_torch_bfloat16():
    torch = pytest.importorskip("torch")
    x = strided_f32(stride=271).view(np.float32)
    x = x[~np.isnan(x)]
    got = oracle.float_encode_array(x, "f32", 8, 7, rne=True)
    ref = torch.from_numpy(x.copy()).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(got.astype(np.uint16), ref)


def test_float_encode_rne_from_f64_e8m23_equals_numpy_float32():
    rng = np.random.default_rng(5)
    bits = rng.integers(0, 2 ** 64, 400000, dtype=np.uint64, endpoint=False)
    x = bits.view(np.float64)
    x = np.concatenate([x[~np.isnan(x)], rng.standard_normal(100000) * 10.0 ** rng.integers(-45, 39, 100000)])
    got = oracle.float_encode_array(x, "f64", 8, 23, rne=True)
    with np.errstate(over="ignore"):
        ref = x.astype(np.float32).view(np.uint32)
    assert np.array_equal(got.astype(np.uint32), ref)


def test_float_encode_rne_nan_rule_equals_truncation():
    rng = np.random.default_rng(6)
    nan = (rng.integers(0, 2, 5000, dtype=np.uint32) << np.uint32(31)) | np.uint32(0x7F800000) | \
        rng.integers(1, 1 << 23, 5000, dtype=np.uint32)
    x = nan.view(np.float32)
    for E, M in ((5, 10), (8, 7), (3, 0), (6, 12)):
        assert np.array_equal(oracle.float_encode_array(x, "f32", E, M, rne=True),
                              oracle.float_encode_array(x, "f32", E, M))


def test_float_rne_view_copy_uses_the_flag():
    rng = np.random.default_rng(7)
    n = 3000
    x = rng.standard_normal(n).astype(np.float32) * np.float32(1000)
    spec = {"kind": "bitpack_float", "exp": 5, "man": 10, "round": "rne"}
    blobs = oracle.store_planes(["f32"], {"kind": "soa_mb"}, [x])
    packed = oracle.copy(["f32"], {"kind": "soa_mb"}, blobs, spec, n)
    codes = oracle.float_encode_array(x, "f32", 5, 10, rne=True)
    stream = np.zeros(4 * ((n * 16 + 31) // 32), np.uint8)
    stream[: 2 * n] = codes.astype(np.uint16).view(np.uint8)
    assert np.array_equal(packed[0], stream)
    trunc = oracle.copy(["f32"], {"kind": "soa_mb"}, blobs, {"kind": "bitpack_float", "exp": 5, "man": 10}, n)
    assert not np.array_equal(packed[0], trunc[0])


# ---------------------------------------------------------------- BitPackedFloat from f64 sources

def encode_trunc_reference(x, E, M):
    """Truncation from any binary64 value: the largest-magnitude code whose exact value is
    <= |x|, Inf when the exponent exceeds the bias (exact rationals, bisection over the
    monotone positive codes)."""
    f = float(x)
    sign = 1 if np.signbit(f) else 0
    ax = abs(Fraction(f))
    bias = (1 << (E - 1)) - 1
    inf_code = ((1 << E) - 1) << M
    if ax >= Fraction(2) ** (bias + 1):
        return inf_code | (sign << (E + M))
    lo, hi = 0, inf_code - 1
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if decode_exact(mid, E, M) <= ax:
            lo = mid
        else:
            hi = mid - 1
    return lo | (sign << (E + M))


def probe_values64(E, M, rng):
    """binary64 probes: target-format edges and their f64 neighbours, f64 subnormals,
    random finite bit patterns and values near 1 in magnitude."""
    bias = (1 << (E - 1)) - 1
    vals = [0.0, -0.0, 1.0, -1.0, 0.1, -2.5e-3, 1e300, -1e-300, 5e-324, -2.2250738585072014e-308]
    maxfin = (2 - Fraction(1, 1 << M)) * Fraction(2) ** bias
    edges = [maxfin, Fraction(2) ** (bias + 1), Fraction(2) ** (1 - bias), Fraction(2) ** (1 - bias - M)]
    edges += [edges[3] / 2, edges[3] * 3 / 2, edges[2] * 3 / 4]
    for e in edges:
        v = float(e) if e < Fraction(2) ** 1024 else None
        if v is None or v == 0.0:
            continue
        vals += [v, float(np.nextafter(v, 0.0)), float(np.nextafter(v, np.inf))]
        # halfway between two neighbouring codes near the edge (RNE ties)
    for c in rng.integers(0, ((1 << E) - 1) << M, 30):
        c = int(c)
        a = decode_exact(c, E, M)
        b = decode_exact(c + 1, E, M) if c + 1 < ((1 << E) - 1) << M else Fraction(2) ** (bias + 1)
        mid = (a + b) / 2
        if Fraction(float(mid)) == mid:
            vals += [float(mid), -float(mid), float(a), float(np.nextafter(float(mid), 0.0))]
    rb = rng.integers(0, 2 ** 63, 60, dtype=np.uint64) | (rng.integers(0, 2, 60, dtype=np.uint64) << np.uint64(63))
    rb = rb[(rb & np.uint64(0x7FF0000000000000)) != np.uint64(0x7FF0000000000000)]
    vals += [float(x) for x in rb.view(np.float64)]
    vals += [float(x) for x in rng.standard_normal(20)]
    subn = rng.integers(1, 1 << 52, 10, dtype=np.uint64)
    vals += [float(x) for x in subn.view(np.float64)]
    return vals


F64_FORMATS = [(11, 20), (11, 0), (9, 22), (2, 29), (8, 15), (5, 10)]


@pytest.mark.parametrize("E,M", F64_FORMATS)
def test_float_encode_from_f64_brute_force_both_roundings(E, M):
    rng = np.random.default_rng(1000 + 31 * E + M)
    vals = np.array(probe_values64(E, M, rng), dtype=np.float64)
    got_t = oracle.float_encode_array(vals, "f64", E, M).astype(np.int64).tolist()
    got_r = oracle.float_encode_array(vals, "f64", E, M, rne=True).astype(np.int64).tolist()
    for v, gt, gr in zip(vals.tolist(), got_t, got_r):
        assert gt == encode_trunc_reference(v, E, M), ("trunc", E, M, v.hex())
        assert gr == encode_rne_reference(v, E, M), ("rne", E, M, v.hex())


@pytest.mark.parametrize("E,M", F64_FORMATS)
def test_float_encode_from_f64_specials(E, M):
    """Inf keeps its sign; a NaN keeps its sign and top M payload bits with the quiet
    bit forced (M = 0: Inf); both roundings agree on them."""
    inf_code = ((1 << E) - 1) << M
    sgn = 1 << (E + M)
    payloads = [1, 1 << 51, (1 << 52) - 1, 0x5555555555555, 0x0000000ABCDEF]
    bits = [0x7FF0000000000000, 0xFFF0000000000000]
    bits += [0x7FF0000000000000 | p for p in payloads] + [0xFFF0000000000000 | p for p in payloads]
    x = np.array(bits, dtype=np.uint64).view(np.float64)
    for rne in (False, True):
        got = oracle.float_encode_array(x, "f64", E, M, rne=rne).astype(np.int64).tolist()
        assert got[0] == inf_code and got[1] == inf_code | sgn
        for k, p in enumerate(payloads):
            quiet = (1 << (M - 1)) if M else 0
            want = inf_code | quiet | ((p >> (52 - M)) & ((1 << M) - 1))
            assert got[2 + k] == want and got[2 + len(payloads) + k] == want | sgn, (rne, hex(p))


def decoded_reference(codes, t, E, M):
    """Field-type bits of every finite code, from the code's exact value (Sec. 3
    BitPackedFloatSoA: a code stands for one value, which decoding reproduces in
    the field type).  float64 holds every value exactly (M <= 52, |exponent| well
    inside its range); float16 / float32 conversion of a representable value is
    exact too, which the round trip checks.  NaN and Inf codes are left out."""
    s = (codes >> np.uint64(E + M)) & np.uint64(1)
    e = ((codes >> np.uint64(M)) & np.uint64((1 << E) - 1)).astype(np.int64)
    m = codes & np.uint64((1 << M) - 1)
    bias = (1 << (E - 1)) - 1
    finite = e != (1 << E) - 1
    s, e, m = s[finite], e[finite], m[finite]
    sig = np.where(e > 0, m + np.uint64(1 << M), m).astype(np.float64)
    ex = np.where(e > 0, e - bias - M, 1 - bias - M)
    val = np.ldexp(sig, ex) * np.where(s == 1, -1.0, 1.0)
    if t == "f64":
        return finite, val.view(np.uint64)
    narrow = val.astype(np.float16 if t == "f16" else np.float32)
    assert np.array_equal(narrow.astype(np.float64), val)  # representable
    if t == "f16":
        return finite, narrow.view(np.uint16).astype(np.uint64)
    b = narrow.view(np.uint32).astype(np.uint64)
    assert not np.any(b & np.uint64(0xFFFF))  # a bfloat16 value
    return finite, b >> np.uint64(16)


def decode_formats():
    out = []
    for t, (Et, Mt) in (("f16", (5, 10)), ("bf16", (8, 7)), ("f64", (11, 52))):
        for E in range(2, Et + 1):
            for M in sorted({0, 1, 2, Mt // 2, Mt - 2, Mt - 1, Mt} - {-1}):
                if M >= 0 and (t != "f64" or E in (2, 3, 4, 5, 8, 10, 11)):
                    out.append((t, E, M))
    return out


@pytest.mark.parametrize("t,E,M", decode_formats(), ids=lambda x: str(x))
def test_float_decode_into_f16_bf16_f64(t, E, M):
    """Decoding into field types other than float32.  Subnormal codes whose value
    is still subnormal in a field type with more exponent bits (E = 4, M >= 9
    into float16) are the case that a shift by the mantissa difference alone
    gets wrong."""
    width = 1 + E + M
    if width <= 16:
        codes = np.arange(1 << width, dtype=np.uint64)
    else:
        rng = np.random.default_rng(width)
        top = (1 << width) - 1
        codes = np.concatenate([rng.integers(0, top, 1 << 15, dtype=np.uint64, endpoint=True),
                                rng.integers(0, 1 << M, 1 << 12, dtype=np.uint64, endpoint=True),  # subnormals
                                np.arange(0, 64, dtype=np.uint64),
                                np.uint64(1 << (E + M)) + np.arange(0, 64, dtype=np.uint64)])
    finite, exp = decoded_reference(codes, t, E, M)
    got = np.array([oracle.float_decode(int(c), t, E, M) for c in codes[finite]], dtype=np.uint64)
    bad = np.nonzero(got != exp)[0]
    assert len(bad) == 0, (t, E, M, hex(int(codes[finite][bad[0]])), hex(int(got[bad[0]])), hex(int(exp[bad[0]])))

"""GPU parity of the value-level copy against the oracle, whole blobs bit for
bit: pairs where both sides are computed (Sec. 3: bit-packed to bit-packed,
ChangeType to ChangeType with a conversion on each side), integer ChangeType,
bit-packed codes of 33 to 64 bits, bit-packed floats of float16 / bfloat16
leaves, SPLIT trees with computed parts against a partner of another form,
the two linearisation orders (Sec. 2) and instrumented computed views
(Sec. 4).  Destinations start filled with a sentinel; a bit-packed stream's
bits past the last code are 0 on both sides."""
import numpy as np
import pytest

import oracle
from gpu_helpers import F32x7, assert_blobs_equal, bits_planes, download, gpu_view, say, upload

import paper_2302_08251_amd as lm

pytestmark = pytest.mark.gpu

AOS, SB, MB = {"kind": "aos"}, {"kind": "soa_sb"}, {"kind": "soa_mb"}
AO3, AO16 = {"kind": "aosoa", "lanes": 3}, {"kind": "aosoa", "lanes": 16}
BS = {"kind": "bytesplit", "inner": {"kind": "soa_sb"}}
SIZES = [1, 31, 33, 1000, 4097]


def bpi(bits):
    return {"kind": "bitpack_int", "bits": bits}


def bpf(E, M, rne=False):
    d = {"kind": "bitpack_float", "exp": E, "man": M}
    if rne:
        d["round"] = "rne"
    return d


def ct(stored, inner=AOS):
    return {"kind": "changetype", "stored": stored, "inner": inner}


def run(rec, a, b, n, planes, what=""):
    src_host = oracle.store_planes(rec, a, planes, fill=0x5A) if a["kind"] != "null" else []
    sv = gpu_view(rec, a, n, src_host)
    dv = gpu_view(rec, b, n, fill=0xA5)
    lm.llama_copy(sv, dv)
    exp = oracle.copy(rec, a, src_host, b, n, fill=0xA5)
    assert_blobs_equal(download(dv), exp, "%s %s -> %s n=%d" % (what, a, b, n))
    sv.close()
    dv.close()


@pytest.mark.parametrize("n", SIZES)
def test_bitpacked_int_to_bitpacked_int(n):
    rec = ["i32", "u32", "i64"]
    planes = bits_planes(n, rec, seed=n)
    for b1, b2 in ((7, 13), (13, 7), (32, 5), (1, 32), (20, 20)):
        say("bpi", b1, b2, n)
        run(rec, bpi(b1), bpi(b2), n, planes)


@pytest.mark.parametrize("n", SIZES)
def test_bitpacked_int_codes_over_32_bits(n):
    rec = ["i64", "u64"]
    planes = bits_planes(n, rec, seed=n + 1)
    for B in (33, 40, 63, 64):
        for a, b in ((AOS, bpi(B)), (bpi(B), SB), (bpi(B), bpi(17)), (bpi(9), bpi(B)), (AO3, bpi(B))):
            say("bpi64", a, b, n)
            run(rec, a, b, n, planes)


@pytest.mark.parametrize("n", SIZES)
def test_bitpacked_float_to_bitpacked_float(n):
    """Re-encoding between two float codes, truncating and rounding to nearest
    even; NaN payloads, infinities, subnormals of both formats."""
    rec = ["f32", "f64", "f32"]
    planes = bits_planes(n, rec, seed=n + 2)
    for (e1, m1), (e2, m2) in (((8, 15), (5, 10)), ((5, 10), (8, 15)), ((8, 23), (6, 3)), ((4, 2), (8, 23))):
        for rne in (False, True):
            say("bpf", e1, m1, e2, m2, rne, n)
            run(rec, bpf(e1, m1), bpf(e2, m2, rne), n, planes)


@pytest.mark.parametrize("n", SIZES)
def test_bitpacked_float_codes_over_32_bits(n):
    rec = ["f64", "f64"]
    planes = bits_planes(n, rec, seed=n + 3)
    for E, M in ((11, 40), (11, 52), (10, 30)):
        for rne in (False, True):
            for a in (AOS, BS):
                say("bpf64", a, E, M, rne, n)
                run(rec, a, bpf(E, M, rne), n, planes)
        say("bpf64 decode", E, M, n)
        run(rec, bpf(E, M), MB, n, planes)
        run(rec, bpf(E, M), bpf(5, 10, True), n, planes)


@pytest.mark.parametrize("n", SIZES)
def test_bitpacked_float_of_half_leaves(n):
    """float16 / bfloat16 leaves: E = 4, M >= 9 codes of float16 decode to values
    that are still subnormal in float16."""
    for rec, fmts in ((["f16", "bf16", "f16"], ((5, 7), (3, 2), (2, 0), (4, 6))),
                      (["f16", "f16"], ((4, 9), (5, 10), (4, 10)))):
        planes = bits_planes(n, rec, seed=n + 4)
        for E, M in fmts:
            for rne in (False, True):
                say("bpf16", rec, E, M, rne, n)
                run(rec, AOS, bpf(E, M, rne), n, planes)
            run(rec, bpf(E, M), AO3, n, planes)
            run(rec, bpf(E, M), ct(["f32"] * len(rec)), n, planes)


@pytest.mark.parametrize("n", SIZES)
def test_changetype_on_both_sides_and_integer_changetype(n):
    rec = ["f32", "i32", "u16", "f64", "i8"]
    planes = bits_planes(n, rec, seed=n + 5)
    st1 = ["f16", "i16", "u8", "f32", "i64"]
    st2 = ["f64", "u8", "i64", "bf16", "i8"]
    for a, b in ((ct(st1), ct(st2, SB)), (ct(st2, AO3), ct(st1, BS)), (ct(st1, MB), AOS), (SB, ct(st2, AO3)),
                 ({"kind": "null"}, ct(st1))):
        say("ct", a, b, n)
        run(rec, a, b, n, planes)
    rec = ["i32", "u16", "i64", "u8"]
    planes = bits_planes(n, rec, seed=n + 6)
    for a, b in ((AOS, ct(["i16", "u8", "i32", "u64"])), (ct(["i8", "i64", "u16", "i16"], SB), BS),
                 (ct(["i8", "i64", "u16", "i16"], SB), bpi(5)), (bpi(8), ct(["u8", "u8", "u8", "u8"], AO3))):
        say("int ct", a, b, n)
        run(rec, a, b, n, planes)


SPLIT_A = {"kind": "split", "at": 3, "parts": [AOS, bpf(5, 10)]}
SPLIT_B = {"kind": "split", "at": 2, "parts": [SB, ct(["f16", "bf16", "f64", "f32", "f16"])]}
SPLIT_N = {"kind": "split", "at": 5, "parts": [{"kind": "split", "at": 2, "parts": [bpf(8, 7, True), BS]},
                                               {"kind": "null"}]}


@pytest.mark.parametrize("n", [1, 1000, 4097])
def test_split_with_computed_parts_against_any_partner(n):
    planes = bits_planes(n, F32x7, seed=n)
    for a, b in ((AOS, SPLIT_A), (SPLIT_A, AOS), (SPLIT_A, SPLIT_B), (SPLIT_B, SPLIT_A), (SPLIT_N, AO16),
                 (AO16, SPLIT_N), (SPLIT_B, BS), (BS, SPLIT_N), (SPLIT_A, SPLIT_N), (bpf(6, 9), SPLIT_A),
                 (SPLIT_A, bpf(6, 9))):
        say("split computed", a, b, n)
        run(F32x7, a, b, n, planes)
    rec = ["u8", "f64", "i16", "f32"]
    planes = bits_planes(n, rec, seed=n + 9)
    s1 = {"kind": "split", "at": 2, "parts": [ct(["u8", "f32"]), AO3]}
    s2 = {"kind": "split", "at": 1, "parts": [bpi(5), {"kind": "split", "at": 1, "parts": [
        bpf(11, 30), ct(["i64", "f16"], SB)]}]}
    for a, b in ((s1, {"kind": "aos", "packed": True}), (AOS, s1), (s1, s2), (s2, s1), (s2, BS), (BS, s2)):
        say("split computed mixed", a, b, n)
        run(rec, a, b, n, planes)


def test_large_aosoa_lane_count():
    """AoSoA with 4096 lanes: a tile of the tile kernels would not fit in LDS,
    the value-level copy moves it."""
    n = 10000
    planes = bits_planes(n, F32x7, seed=12)
    big = {"kind": "aosoa", "lanes": 4096}
    for a, b in ((AOS, big), (big, SB), (big, bpf(8, 10))):
        say("aosoa4096", a, b)
        run(F32x7, a, b, n, planes)


@pytest.mark.parametrize("ext", [(37, 45), (3, 4, 5, 6)])
def test_computed_sides_in_both_orders(ext):
    n = int(np.prod(ext))
    rec = ["i32", "u32", "i64"]
    planes = bits_planes(n, rec, seed=2)
    pairs = [(bpi(13), AOS), (SB, bpi(7)), (bpi(9), bpi(21)), (ct(["i8", "i16", "u32"]), bpi(30))]
    for a, b in pairs:
        for sc, dc in ((False, True), (True, False), (True, True)):
            sa, sb = dict(a, col_major=sc), dict(b, col_major=dc)
            say("order", ext, sa, sb)
            src_host = oracle.store_planes(rec, sa, planes, fill=0x5A)
            exp = oracle.copy_nd(rec, sa, src_host, sb, list(ext), fill=0xA5)
            sv = lm.View(rec, sa, list(ext), blobs=upload(src_host))
            dv = lm.View(rec, sb, list(ext), fill=0xA5)
            lm.llama_copy(sv, dv)
            assert_blobs_equal(download(dv), exp, "%s -> %s ext=%s" % (sa, sb, ext))
    sa, sb = dict(SPLIT_A, col_major=True), dict(AOS, col_major=False)
    planes = bits_planes(n, F32x7, seed=3)
    say("order split", ext)
    src_host = oracle.store_planes(F32x7, sa, planes, fill=0x5A)
    exp = oracle.copy_nd(F32x7, sa, src_host, sb, list(ext), fill=0xA5)
    sv = lm.View(F32x7, sa, list(ext), blobs=upload(src_host))
    dv = lm.View(F32x7, sb, list(ext), fill=0xA5)
    lm.llama_copy(sv, dv)
    assert_blobs_equal(download(dv), exp, "split col-major -> aos")


def test_instrumented_computed_views():
    """FieldAccessCount around computed mappings on both sides of a value-level
    copy: the data and every counter match the oracle's."""
    n = 3001
    rec = ["i32", "u16", "i64", "u8"]
    planes = bits_planes(n, rec, seed=13)
    fac = {"kind": "field_access_count", "inner": bpi(7)}
    dst = {"kind": "field_access_count", "inner": ct(["i8", "i64", "u16", "i16"], SB)}
    say("instrumented value-level")
    src_host = oracle.store_planes(rec, fac, planes, fill=0)
    dst_host = oracle.alloc_blobs(rec, dst, n, fill=0)
    sv, dv = gpu_view(rec, fac, n, src_host), gpu_view(rec, dst, n, dst_host)
    lm.llama_copy(sv, dv)
    oracle.copy(rec, fac, src_host, dst, n, dst_blobs=dst_host)
    assert_blobs_equal(download(sv), src_host, "source counters")
    assert_blobs_equal(download(dv), dst_host, "destination data and counters")
    s = {"kind": "split", "at": 2, "parts": [{"kind": "field_access_count", "inner": bpi(11)}, AO3]}
    say("instrumented split part")
    src_host = oracle.store_planes(rec, s, planes, fill=0)
    sv, dv = gpu_view(rec, s, n, src_host), gpu_view(rec, AOS, n, fill=0xA5)
    lm.llama_copy(sv, dv)
    exp = oracle.copy(rec, s, src_host, AOS, n, fill=0xA5)
    assert_blobs_equal(download(dv), exp, "data")
    assert_blobs_equal(download(sv), src_host, "split part counters")

"""GPU parity of the per-leaf copy against the oracle, whole blobs bit for bit:
records whose leaves differ in size (Sec. 1 record dimension: a C struct
{u8; f64; i16; f32} with its alignment padding, its packed form, SoA,
AoSoA, Bytesplit), and SPLIT views (Sec. 3) copied to or from a partner of
any other form.  Destinations start filled with a sentinel, so padding bytes
and AoSoA padding lanes that a copy must not write are checked too."""
import numpy as np
import pytest

import oracle
from gpu_helpers import F32x7, assert_blobs_equal, bits_planes, download, gpu_view, say, upload

import paper_2302_08251_amd as lm

pytestmark = pytest.mark.gpu

RECS = {
    "cstruct": ["u8", "f64", "i16", "f32"],   # aligned AoS: 24-byte records, 9 bytes of padding
    "i16u8": ["i16", "u8"],
    "wide": ["u16", "i8", "u64", "f32", "u8", "f64"],
}
LAYOUTS = {
    "aos": {"kind": "aos"},
    "aos_packed": {"kind": "aos", "packed": True},
    "soa_sb": {"kind": "soa_sb"},
    "soa_mb": {"kind": "soa_mb"},
    "aosoa8": {"kind": "aosoa", "lanes": 8},
    "aosoa3": {"kind": "aosoa", "lanes": 3},
    "bs_sb": {"kind": "bytesplit", "inner": {"kind": "soa_sb"}},
    "bs_aos": {"kind": "bytesplit", "inner": {"kind": "aos"}},
    "bs_aosoa4": {"kind": "bytesplit", "inner": {"kind": "aosoa", "lanes": 4}},
    "bs_mb": {"kind": "bytesplit", "inner": {"kind": "soa_mb"}},
}


def run(rec, a, b, n, planes, what=""):
    src_host = oracle.store_planes(rec, a, planes, fill=0x5A)
    sv = gpu_view(rec, a, n, src_host)
    dv = gpu_view(rec, b, n, fill=0xA5)
    lm.llama_copy(sv, dv)
    exp = oracle.copy(rec, a, src_host, b, n, fill=0xA5)
    assert_blobs_equal(download(dv), exp, "%s %s -> %s n=%d" % (what, a, b, n))
    sv.close()
    dv.close()


@pytest.mark.parametrize("n", [1, 4099])
@pytest.mark.parametrize("recname", sorted(RECS))
def test_mixed_leaf_sizes_all_pairs(recname, n):
    rec = RECS[recname]
    planes = bits_planes(n, rec, seed=n + len(rec))
    for a in LAYOUTS:
        for b in LAYOUTS:
            say("mixed", recname, a, b, n)
            run(rec, LAYOUTS[a], LAYOUTS[b], n, planes, recname)


@pytest.mark.parametrize("n", [1000, 33, 100003])
def test_mixed_awkward_sizes(n):
    rec = RECS["cstruct"]
    planes = bits_planes(n, rec, seed=7)
    for a, b in (("aos", "soa_sb"), ("soa_mb", "aos"), ("aos_packed", "aosoa3"), ("bs_sb", "aos"),
                 ("aosoa8", "bs_aosoa4"), ("aos", "aos_packed")):
        say("mixed awkward", a, b, n)
        run(rec, LAYOUTS[a], LAYOUTS[b], n, planes)


def test_mixed_null_and_instrumented():
    """A NULL source writes zeros into every mapped byte of a mixed record (padding
    untouched); a NULL destination drops the values; FieldAccessCount and Heatmap
    around a mixed record count every access."""
    rec = RECS["cstruct"]
    n = 2001
    planes = bits_planes(n, rec, seed=3)
    for b in ("aos", "aosoa3", "bs_sb"):
        say("mixed null ->", b)
        run(rec, {"kind": "null"}, LAYOUTS[b], n, planes)
    sv = gpu_view(rec, LAYOUTS["aos"], n, oracle.store_planes(rec, LAYOUTS["aos"], planes))
    lm.llama_copy(sv, gpu_view(rec, {"kind": "null"}, n))
    fac = {"kind": "field_access_count", "inner": {"kind": "aos"}}
    heat = {"kind": "heatmap", "granularity": 8, "inner": {"kind": "soa_sb"}}
    say("mixed instrumented")
    src_host = oracle.store_planes(rec, fac, planes, fill=0)
    dst_host = oracle.alloc_blobs(rec, heat, n, fill=0)
    sv, dv = gpu_view(rec, fac, n, src_host), gpu_view(rec, heat, n, dst_host)
    lm.llama_copy(sv, dv)
    oracle.copy(rec, fac, src_host, heat, n, dst_blobs=dst_host)
    assert_blobs_equal(download(sv), src_host, "source counters")
    assert_blobs_equal(download(dv), dst_host, "destination data and counters")


SPLIT_A = {"kind": "split", "at": 3, "parts": [{"kind": "aos"}, {"kind": "soa_mb"}]}
SPLIT_B = {"kind": "split", "at": 2, "parts": [{"kind": "soa_sb"}, {"kind": "aosoa", "lanes": 32}]}
SPLIT_N = {"kind": "split", "at": 5, "parts": [
    {"kind": "split", "at": 2, "parts": [{"kind": "bytesplit", "inner": {"kind": "soa_sb"}}, {"kind": "aos"}]},
    {"kind": "null"}]}


@pytest.mark.parametrize("n", [1, 1000, 4097])
def test_split_with_any_partner(n):
    """SPLIT against a partner that cannot be divided at the same field: AoS, AoSoA,
    Bytesplit, another split point, nested SPLITs with a NULL part."""
    planes = bits_planes(n, F32x7, seed=n)
    aos, aosoa, bs = {"kind": "aos"}, {"kind": "aosoa", "lanes": 16}, {"kind": "bytesplit", "inner": {"kind": "soa_sb"}}
    for a, b in ((aos, SPLIT_A), (SPLIT_A, aos), (SPLIT_A, SPLIT_B), (SPLIT_B, SPLIT_A), (SPLIT_N, aosoa),
                 (aosoa, SPLIT_N), (SPLIT_B, bs), (bs, SPLIT_N)):
        say("split partner", a, b, n)
        run(F32x7, a, b, n, planes)


def test_split_mixed_record_and_instrumented_part():
    rec = RECS["cstruct"]
    n = 3001
    planes = bits_planes(n, rec, seed=11)
    s = {"kind": "split", "at": 2, "parts": [{"kind": "field_access_count", "inner": {"kind": "aos"}},
                                             {"kind": "aosoa", "lanes": 3}]}
    d = {"kind": "aos", "packed": True}
    say("split mixed instrumented")
    src_host = oracle.store_planes(rec, s, planes, fill=0)
    sv, dv = gpu_view(rec, s, n, src_host), gpu_view(rec, d, n, fill=0xA5)
    lm.llama_copy(sv, dv)
    exp = oracle.copy(rec, s, src_host, d, n, fill=0xA5)
    assert_blobs_equal(download(dv), exp, "data")
    assert_blobs_equal(download(sv), src_host, "source counters")
    run(rec, d, s, n, planes, "into split")


@pytest.mark.parametrize("ext", [(37, 45), (3, 4, 5, 6)])
def test_mixed_column_major(ext):
    rec = RECS["cstruct"]
    n = int(np.prod(ext))
    planes = bits_planes(n, rec, seed=2)
    for a, b in (("aos", "soa_sb"), ("bs_sb", "aosoa3"), ("aos_packed", "aos")):
        for sc, dc in ((False, True), (True, False)):
            say("mixed order", ext, a, sc, b, dc)
            sa, sb = dict(LAYOUTS[a], col_major=sc), dict(LAYOUTS[b], col_major=dc)
            src_host = oracle.store_planes(rec, sa, planes, fill=0x5A)
            exp = oracle.copy_nd(rec, sa, src_host, sb, list(ext), fill=0xA5)
            sv = lm.View(rec, sa, list(ext), blobs=upload(src_host))
            dv = lm.View(rec, sb, list(ext), fill=0xA5)
            lm.llama_copy(sv, dv)
            assert_blobs_equal(download(dv), exp, "%s -> %s ext=%s" % (sa, sb, ext))


def test_per_leaf_copy_limits():
    """A SPLIT with a computed part against AoS moves value by value; a Bytesplit
    side of more than 64 byte columns is rejected before any launch."""
    n = 100
    ct = {"kind": "split", "at": 3, "parts": [{"kind": "aos"},
                                              {"kind": "changetype", "stored": ["f16"] * 4, "inner": {"kind": "aos"}}]}
    run(F32x7, ct, {"kind": "aos"}, n, bits_planes(n, F32x7, seed=1), "computed part")
    big = ["u8"] * 40 + ["f64"] * 4  # a Bytesplit of 72 bytes: more than 64 byte columns
    with pytest.raises(lm.LlamaError) as e:
        lm.llama_copy(gpu_view(big, {"kind": "aos"}, n, fill=0),
                      gpu_view(big, {"kind": "bytesplit", "inner": {"kind": "soa_sb"}}, n))
    assert e.value.name == "UNSUPPORTED"

"""GPU parity of the meta-mappings (Sec. 3 Split and Null) against the oracle,
bit for bit: Split copies run one copy per part, a Null source writes zero to
every mapped byte (padding untouched), a Null destination drops the values."""
import numpy as np
import pytest

import oracle
from gpu_helpers import F32x7, assert_blobs_equal, bits_planes, download, gpu_view, say

import paper_2302_08251_amd as lm

pytestmark = pytest.mark.gpu

SPLIT_A = {"kind": "split", "at": 3, "parts": [{"kind": "aos"}, {"kind": "soa_mb"}]}
SPLIT_B = {"kind": "split", "at": 3, "parts": [{"kind": "soa_sb"}, {"kind": "aosoa", "lanes": 32}]}
SPLIT_C = {"kind": "split", "at": 3,
           "parts": [{"kind": "bytesplit", "inner": {"kind": "soa_sb"}}, {"kind": "null"}]}


def run(rec, a, b, n, planes):
    src_host = oracle.store_planes(rec, a, planes, fill=0x5A)
    sv = gpu_view(rec, a, n, src_host)
    dv = gpu_view(rec, b, n, fill=0xA5)
    lm.llama_copy(sv, dv)
    exp = oracle.copy(rec, a, src_host, b, n, fill=0xA5)
    assert_blobs_equal(download(dv), exp, "%s -> %s n=%d" % (a, b, n))


@pytest.mark.parametrize("n", [1, 1000, 4097])
def test_split_copies(n):
    planes = bits_planes(n, F32x7, seed=n)
    mb = {"kind": "soa_mb"}
    for a, b in ((SPLIT_A, mb), (mb, SPLIT_A), (SPLIT_A, SPLIT_B), (SPLIT_B, SPLIT_A), (SPLIT_B, SPLIT_C),
                 (SPLIT_C, SPLIT_A), (mb, SPLIT_C)):
        say("split", a, b, n)
        run(F32x7, a, b, n, planes)


@pytest.mark.parametrize("n", [1, 777, 4097])
def test_null_source_writes_zero(n):
    rec = ["f32"] * 3
    null = {"kind": "null"}
    for dst in ({"kind": "aos"}, {"kind": "soa_sb"}, {"kind": "aosoa", "lanes": 32}, {"kind": "aosoa", "lanes": 3},
                {"kind": "bytesplit", "inner": {"kind": "soa_sb"}},
                {"kind": "bitpack_float", "exp": 5, "man": 10},
                {"kind": "changetype", "stored": ["f16"] * 3, "inner": {"kind": "aos"}}):
        say("null ->", dst, n)
        sv = gpu_view(rec, null, n)
        dv = gpu_view(rec, dst, n, fill=0xA5)
        lm.llama_copy(sv, dv)
        exp = oracle.copy(rec, null, [], dst, n, fill=0xA5)
        assert_blobs_equal(download(dv), exp, "null -> %s n=%d" % (dst, n))
    ints = ["u16"] * 2
    dv = gpu_view(ints, {"kind": "bitpack_int", "bits": 7}, n, fill=0xA5)
    lm.llama_copy(gpu_view(ints, null, n), dv)
    assert_blobs_equal(download(dv), oracle.copy(ints, null, [], {"kind": "bitpack_int", "bits": 7}, n, fill=0xA5))


def tree(lo, hi):
    """A SPLIT tree with one AoS part per field in [lo, hi)."""
    if hi - lo == 1:
        return {"kind": "aos"}
    mid = (lo + hi) // 2
    return {"kind": "split", "at": mid - lo, "parts": [tree(lo, mid), tree(mid, hi)]}


def test_null_destination_and_unsupported_pairs():
    n = 500
    planes = bits_planes(n, F32x7, seed=5)
    src_host = oracle.store_planes(F32x7, {"kind": "aos"}, planes)
    sv = gpu_view(F32x7, {"kind": "aos"}, n, src_host)
    lm.llama_copy(sv, gpu_view(F32x7, {"kind": "null"}, n))  # values dropped, nothing to write
    # a SPLIT tree of more than 8 physical parts against a partner of another form
    r10 = ["f32"] * 10
    with pytest.raises(lm.LlamaError) as e:
        lm.llama_copy(gpu_view(r10, {"kind": "aos"}, n, fill=0), gpu_view(r10, tree(0, 10), n))
    assert e.value.name == "UNSUPPORTED"


def test_unsupported_split_part_launches_nothing():
    """Part 0 (AoS -> SoA-SB) is supported, part 1 (a SPLIT tree of ten parts
    against AoS) is not: the copy is planned whole first, so the destination
    stays untouched."""
    n = 1000
    rec = ["f32"] * 12
    a = {"kind": "split", "at": 2, "parts": [{"kind": "aos"}, tree(0, 10)]}
    b = {"kind": "split", "at": 2, "parts": [{"kind": "soa_sb"}, {"kind": "aos"}]}
    sv = gpu_view(rec, a, n, fill=0x11)
    dv = gpu_view(rec, b, n, fill=0xA5)
    with pytest.raises(lm.LlamaError) as e:
        lm.llama_copy(sv, dv)
    assert e.value.name == "UNSUPPORTED"
    for blob in download(dv):
        assert np.all(blob == 0xA5)

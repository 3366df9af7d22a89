"""GPU parity of layout-aware copies (Sec. 1 layout-aware copy; mappings of
Sec. 3 and Sec. 5) against the oracle, bit for bit, on whole blobs.

Destination blobs start filled with a sentinel (0xA5) on both sides, so the
comparison also checks that AoSoA padding lanes are never written."""
import itertools

import numpy as np
import pytest

import oracle
from gpu_helpers import (CFG2, F32x7, F64x7, assert_blobs_equal, bits_planes, download, gpu_view,
                         say)

import paper_2302_08251_amd as lm
from paper_2302_08251_amd import synth

pytestmark = pytest.mark.gpu


def run_pair(rec, src_spec, dst_spec, n, planes, tile=0, grid=0):
    src_host = oracle.store_planes(rec, src_spec, planes, fill=0x5A)
    sv = gpu_view(rec, src_spec, n, src_host)
    dv = gpu_view(rec, dst_spec, n, fill=0xA5)
    if tile or grid:
        lm.llama_copy_ex(sv, dv, tile_records=tile, grid=grid)
    else:
        lm.llama_copy(sv, dv)
    got = download(dv)
    exp = oracle.copy(rec, src_spec, src_host, dst_spec, n, fill=0xA5)
    assert_blobs_equal(got, exp, "%s -> %s n=%d" % (src_spec, dst_spec, n))


@pytest.mark.parametrize("n", [1, 3, 31, 33, 127, 1000, 4097])
def test_cfg2_all_ordered_pairs_small(n):
    planes = bits_planes(n, F32x7, seed=n)
    for a, b in itertools.product(CFG2, CFG2):
        say("pair", a, b, n)
        run_pair(F32x7, CFG2[a], CFG2[b], n, planes)


@pytest.mark.parametrize("n", [4096, 1000])
def test_cfg1_f64_records(n):
    planes = synth.particles(n, 0)
    specs = [{"kind": "aos"}, {"kind": "soa_sb"}, {"kind": "soa_mb"}, {"kind": "aosoa", "lanes": 8}]
    for a, b in itertools.permutations(specs, 2):
        say("f64", a, b, n)
        run_pair(F64x7, a, b, n, planes)


MIXED = [
    {"kind": "aos", "packed": True}, {"kind": "aosoa", "lanes": 3}, {"kind": "aosoa", "lanes": 48},
    {"kind": "aosoa", "lanes": 1}, {"kind": "bytesplit", "inner": {"kind": "aos"}},
    {"kind": "bytesplit", "inner": {"kind": "soa_mb"}}, {"kind": "bytesplit", "inner": {"kind": "soa_sb"}},
    {"kind": "bytesplit", "inner": {"kind": "aosoa", "lanes": 8}},
    {"kind": "bytesplit", "inner": {"kind": "aosoa", "lanes": 32}},
    {"kind": "soa_sb"}, {"kind": "aos"},
]


@pytest.mark.parametrize("rec", [["u8"] * 5, ["i16", "u16", "i16"], ["f64", "i64", "u64"], ["f32", "i32", "u32"]], ids=str)
@pytest.mark.parametrize("n", [7, 130, 777])
def test_other_records_and_mappings(rec, n):
    planes = bits_planes(n, rec, seed=n + len(rec))
    for a, b in itertools.product(MIXED, MIXED):
        if a == b:
            continue
        say(rec, a, b, n)
        run_pair(rec, a, b, n, planes)


@pytest.mark.parametrize("tile,grid", [(128, 0), (256, 0), (1024, 0), (2048, 0), (512, 7), (128, 1), (384, 3)])
def test_launch_parameters(tile, grid):
    n = 5003
    planes = bits_planes(n, F32x7, seed=9)
    for a, b in [("aos", "soa_sb"), ("aosoa64", "bytesplit"), ("bytesplit", "aosoa32"), ("soa_mb", "aos")]:
        say("tile", tile, grid, a, b)
        try:
            run_pair(F32x7, CFG2[a], CFG2[b], n, planes, tile=tile, grid=grid)
        except lm.LlamaError as e:
            # a relayout through a canonical image holds two tile images in LDS (a
            # Bytesplit side, or single-blob planes off the line grid as here with
            # n = 5003): 2048 records exceed 64 KiB and the tile is rejected
            assert tile >= 2048 and ("bytesplit" in (a, b) or b == "soa_sb") and e.name == "INVALID_ARG", e


def test_empty_view_is_a_no_op():
    sv = gpu_view(F32x7, CFG2["aos"], 0, fill=0)
    dv = gpu_view(F32x7, CFG2["soa_sb"], 0, fill=0)
    lm.llama_copy(sv, dv)
    download(dv)


def test_index_types_give_same_result():
    n = 3000
    planes = bits_planes(n, F32x7, seed=4)
    src_host = oracle.store_planes(F32x7, CFG2["aos"], planes)
    exp = oracle.copy(F32x7, CFG2["aos"], src_host, CFG2["aosoa32"], n, fill=0xA5)
    for idx in ("i32", "u32", "i64", "u64"):
        sv = gpu_view(F32x7, CFG2["aos"], n, src_host, index=idx)
        dv = gpu_view(F32x7, CFG2["aosoa32"], n, fill=0xA5, index=idx)
        lm.llama_copy(sv, dv)
        assert_blobs_equal(download(dv), exp, idx)


# 16-bit index types (Sec. 2): the largest ragged record counts whose every
# blob still fits the type.  7 x f32 records are 28 bytes; an AoSoA-64 blob
# of ceil(n / 64) * 64 records must stay below 2^15 (I16) or 2^16 (U16) bytes.
IDX16 = {"i16": 1150, "u16": 2303}


@pytest.mark.parametrize("idx", sorted(IDX16))
def test_index16_all_pairs(idx):
    n = IDX16[idx]
    limit = 0x7FFF if idx == "i16" else 0xFFFF
    assert -(-n // 64) * 64 * 28 - 1 <= limit
    planes = bits_planes(n, F32x7, seed=5)
    for a, sa in CFG2.items():
        src_host = oracle.store_planes(F32x7, sa, planes)
        sv = gpu_view(F32x7, sa, n, src_host, index=idx)
        for b, sb in CFG2.items():
            say("index", idx, a, b, n)
            exp = oracle.copy(F32x7, sa, src_host, sb, n, fill=0xA5)
            dv = gpu_view(F32x7, sb, n, fill=0xA5, index=idx)
            lm.llama_copy(sv, dv)
            assert_blobs_equal(download(dv), exp, "%s %s -> %s" % (idx, a, b))


def test_index16_rejects_what_does_not_fit():
    with pytest.raises(lm.LlamaError) as e:
        lm.View(F32x7, CFG2["aos"], [1171], index_type="i16")
    assert e.value.name == "INDEX_OVERFLOW"
    with pytest.raises(lm.LlamaError) as e:
        lm.View(F32x7, CFG2["aosoa64"], [2305], index_type="u16")
    assert e.value.name == "INDEX_OVERFLOW"

"""Pins of the oracle's physical mappings (CPU only).

The oracle is checked against things other than itself: hand-worked offsets
(tests/golden/layout_offsets.jsonl), numpy reshapes/transposes that express
each layout independently, brute-force injectivity and coverage, and the
closed-form reductions between mappings (AoSoA-1 = AoS, AoSoA-N = SoA single
blob, concatenated SoA multi-blob = SoA single blob, Bytesplit(AoS) = AoS,
ChangeType(T -> T) = inner).
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def rec_of(s):
    if "x" in s and "," not in s:
        cnt, t = s.split("x")
        return [t] * int(cnt)
    return s.split(",")


def golden_lines(name):
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            d = json.loads(line)
            if "_doc" not in d:
                yield d


@pytest.mark.parametrize("case", list(golden_lines("layout_offsets.jsonl")), ids=lambda d: d["cite"][:40])
def test_hand_worked_offsets(case):
    rec = rec_of(case["rec"])
    assert oracle.locate(rec, case["map"], case["n"], case["i"], case["f"], case["k"]) == (
        case["blob"], case["off"])
    assert oracle.blob_sizes(rec, case["map"], case["n"]) == case["sizes"]


PHYS = [
    {"kind": "aos"}, {"kind": "aos", "packed": True}, {"kind": "soa_sb"}, {"kind": "soa_mb"},
    {"kind": "aosoa", "lanes": 1}, {"kind": "aosoa", "lanes": 3}, {"kind": "aosoa", "lanes": 8},
    {"kind": "bytesplit", "inner": {"kind": "aos"}}, {"kind": "bytesplit", "inner": {"kind": "soa_sb"}},
    {"kind": "bytesplit", "inner": {"kind": "soa_mb"}},
    {"kind": "bytesplit", "inner": {"kind": "aosoa", "lanes": 4}},
]
RECS = [["f32"] * 7, ["f64"] * 7, ["u8", "f64", "i16", "f32"], ["i16", "u8"]]


@pytest.mark.parametrize("spec", PHYS, ids=lambda s: json.dumps(s))
@pytest.mark.parametrize("rec", RECS, ids=lambda r: ",".join(r))
@pytest.mark.parametrize("n", [1, 5, 17])
def test_injective_and_covering(spec, rec, n):
    """Every (i, f, k) maps to a distinct byte; the mapped bytes are the whole blobs except
    AoS alignment padding and AoSoA tail-block padding."""
    sizes = oracle.blob_sizes(rec, spec, n)
    seen = set()
    for i in range(n):
        for f, t in enumerate(rec):
            for k in range(oracle.TYPE_SIZE[t]):
                b, o = oracle.locate(rec, spec, n, i, f, k)
                assert 0 <= o < sizes[b]
                assert (b, o) not in seen
                seen.add((b, o))
    S = sum(oracle.TYPE_SIZE[t] for t in rec)
    assert len(seen) == n * S
    inner = spec.get("inner", spec)
    padded = inner["kind"] == "aosoa" or (spec["kind"] == "aos" and not spec.get("packed"))
    if not padded:
        assert sum(sizes) == n * S


def planes_for(rec, n, seed=1):
    rng = np.random.default_rng(seed)
    return [rng.integers(0, 256, n * oracle.TYPE_SIZE[t], dtype=np.uint8).view(oracle._NP[t])
            for t in rec]


def bytes_matrix(planes):
    """(n, S) matrix of the packed record bytes, built with numpy only."""
    return np.concatenate([p.view(np.uint8).reshape(len(p), -1) for p in planes], axis=1)


@pytest.mark.parametrize("rec", [["f32"] * 7, ["f64"] * 7, ["u8", "f64", "i16", "f32"]],
                         ids=lambda r: ",".join(r))
@pytest.mark.parametrize("n", [1, 8, 13, 64])
def test_layouts_equal_numpy_closed_forms(rec, n):
    planes = planes_for(rec, n)
    M = bytes_matrix(planes)  # (n, S)
    S = M.shape[1]
    sizes = [oracle.TYPE_SIZE[t] for t in rec]
    offs = np.cumsum([0] + sizes)
    # packed AoS: the byte matrix row by row
    aos = oracle.store_planes(rec, {"kind": "aos", "packed": True}, planes)
    assert np.array_equal(aos[0], M.reshape(-1))
    # SoA single blob: the planes back to back
    sb = oracle.store_planes(rec, {"kind": "soa_sb"}, planes)
    assert np.array_equal(sb[0], np.concatenate([p.view(np.uint8) for p in planes]))
    # SoA multi blob: each plane
    mb = oracle.store_planes(rec, {"kind": "soa_mb"}, planes)
    for b, p in zip(mb, planes):
        assert np.array_equal(b, p.view(np.uint8))
    # AoSoA-L: pad to whole blocks, then (block, field, lane, byte)
    for L in (1, 4, 8):
        nb = -(-n // L)
        blob = oracle.store_planes(rec, {"kind": "aosoa", "lanes": L}, planes, fill=0xA5)[0]
        parts = []
        for blk in range(nb):
            for f in range(len(rec)):
                lo, hi = blk * L, min(n, blk * L + L)
                seg = np.full((L, sizes[f]), 0xA5, np.uint8)
                seg[: hi - lo] = M[lo:hi, offs[f]:offs[f + 1]]
                parts.append(seg.reshape(-1))
        assert np.array_equal(blob, np.concatenate(parts)), L
    # Bytesplit(SoA single blob): the byte matrix transposed (byte planes)
    bs = oracle.store_planes(rec, {"kind": "bytesplit", "inner": {"kind": "soa_sb"}}, planes)
    assert np.array_equal(bs[0], np.ascontiguousarray(M.T).reshape(-1))
    # Bytesplit(AoS) is the packed AoS byte image
    ba = oracle.store_planes(rec, {"kind": "bytesplit", "inner": {"kind": "aos"}}, planes)
    assert np.array_equal(ba[0], M.reshape(-1))
    # C-struct AoS via a numpy structured dtype with aligned layout
    dt = np.dtype([("f%d" % f, oracle._NP[t]) for f, t in enumerate(rec)], align=True)
    arr = np.zeros(n, dtype=dt)
    for f in range(len(rec)):
        arr["f%d" % f] = planes[f]
    got = oracle.store_planes(rec, {"kind": "aos"}, planes)[0]
    raw = arr.view(np.uint8)
    pad_mask = np.zeros(dt.itemsize, bool)
    for f in range(len(rec)):
        o = dt.fields["f%d" % f][1]
        pad_mask[o:o + sizes[f]] = True
    mask = np.tile(pad_mask, n)
    assert dt.itemsize * n == len(got)
    assert np.array_equal(got[mask], raw[mask])


@pytest.mark.parametrize("rec", [["f32"] * 7, ["u8", "f64", "i16", "f32"]], ids=lambda r: ",".join(r))
def test_special_case_reductions(rec):
    n = 24
    planes = planes_for(rec, n, seed=3)
    aosp = oracle.store_planes(rec, {"kind": "aos", "packed": True}, planes)
    assert np.array_equal(oracle.store_planes(rec, {"kind": "aosoa", "lanes": 1}, planes)[0], aosp[0])
    sb = oracle.store_planes(rec, {"kind": "soa_sb"}, planes)
    assert np.array_equal(oracle.store_planes(rec, {"kind": "aosoa", "lanes": n}, planes)[0], sb[0])
    mb = oracle.store_planes(rec, {"kind": "soa_mb"}, planes)
    assert np.array_equal(np.concatenate(mb), sb[0])
    bsa = oracle.store_planes(rec, {"kind": "bytesplit", "inner": {"kind": "aos"}}, planes)
    assert np.array_equal(bsa[0], aosp[0])
    for inner in ({"kind": "aos"}, {"kind": "soa_mb"}, {"kind": "aosoa", "lanes": 4}):
        ct = oracle.store_planes(rec, {"kind": "changetype", "stored": rec, "inner": inner}, planes)
        ref = oracle.store_planes(rec, inner, planes)
        assert all(np.array_equal(a, b) for a, b in zip(ct, ref))


def test_copy_roundtrip_and_composition():
    rec = ["f32"] * 3 + ["f64"] * 2 + ["i16"]
    n = 37
    planes = planes_for(rec, n, seed=5)
    specs = [{"kind": "aos"}, {"kind": "aos", "packed": True}, {"kind": "soa_sb"},
             {"kind": "soa_mb"}, {"kind": "aosoa", "lanes": 4},
             {"kind": "bytesplit", "inner": {"kind": "soa_sb"}},
             {"kind": "bytesplit", "inner": {"kind": "aosoa", "lanes": 8}}]
    blobs = {json.dumps(s): oracle.store_planes(rec, s, planes) for s in specs}
    for a, b in itertools.permutations(specs, 2):
        ab = oracle.copy(rec, a, blobs[json.dumps(a)], b, n)
        back = oracle.load_planes(rec, b, ab, n)
        for p, q in zip(planes, back):
            assert np.array_equal(p.view(np.uint8), q.view(np.uint8))
    for a, b, c in itertools.islice(itertools.permutations(specs, 3), 0, None, 7):
        ab = oracle.copy(rec, a, blobs[json.dumps(a)], b, n)
        abc = oracle.copy(rec, b, ab, c, n, fill=0)
        ac = oracle.copy(rec, a, blobs[json.dumps(a)], c, n, fill=0)
        assert all(np.array_equal(x, y) for x, y in zip(abc, ac))


def test_aosoa_padding_untouched():
    rec = ["f32"] * 7
    n = 10
    planes = planes_for(rec, n)
    src = oracle.store_planes(rec, {"kind": "soa_mb"}, planes)
    dst = oracle.copy(rec, {"kind": "soa_mb"}, src, {"kind": "aosoa", "lanes": 4}, n, fill=0xA5)
    blob = dst[0]
    # block 2 holds records 8, 9 in lanes 0, 1; lanes 2, 3 are padding
    for f in range(7):
        base = 2 * 112 + f * 16
        assert np.all(blob[base + 8: base + 16] == 0xA5)


# ---------------------------------------------------------------- Split and Null (Sec. 3)

def test_split_blobs_equal_numpy_parts():
    """Split(3, AoS, SoA-MB) over 7 x f32: blob 0 is the packed AoS of fields 0..2,
    blobs 1..4 are the raw planes of fields 3..6 (numpy closed forms)."""
    rng = np.random.default_rng(21)
    n = 53
    rec = ["f32"] * 7
    planes = [rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32) for _ in range(7)]
    spec = {"kind": "split", "at": 3, "parts": [{"kind": "aos"}, {"kind": "soa_mb"}]}
    assert oracle.blob_count(rec, spec) == 5
    blobs = oracle.store_planes(rec, spec, [p.view(np.float32) for p in planes])
    aos = np.stack(planes[:3], axis=1).astype("<u4").view(np.uint8).reshape(-1)
    assert np.array_equal(blobs[0], aos)
    for f in range(3, 7):
        assert np.array_equal(blobs[f - 2], planes[f].astype("<u4").view(np.uint8))


def test_split_with_null_part_and_nesting():
    rng = np.random.default_rng(22)
    n = 40
    rec = ["f64", "f64", "i32", "i32", "u8"]
    planes = [rng.integers(0, 2 ** 63, n, dtype=np.uint64).view(np.float64) for _ in range(2)] + \
             [rng.integers(-2 ** 31, 2 ** 31, n, dtype=np.int64).astype(np.int32) for _ in range(2)] + \
             [rng.integers(0, 256, n, dtype=np.uint64).astype(np.uint8)]
    inner = {"kind": "split", "at": 2, "parts": [{"kind": "soa_sb"}, {"kind": "null"}]}
    spec = {"kind": "split", "at": 2, "parts": [{"kind": "aos"}, inner]}
    # blobs: AoS of the two f64, SoA-SB of the two i32; the u8 field is dropped
    assert oracle.blob_sizes(rec, spec, n) == [16 * n, 8 * n]
    blobs = oracle.store_planes(rec, spec, planes)
    assert np.array_equal(blobs[0], np.stack([p.view(np.uint64) for p in planes[:2]], 1).view(np.uint8).reshape(-1))
    assert np.array_equal(blobs[1], np.concatenate([planes[2].view(np.uint8), planes[3].view(np.uint8)]))
    back = oracle.copy(rec, spec, blobs, {"kind": "soa_mb"}, n, fill=0x77)
    for f in range(4):
        assert np.array_equal(back[f], np.ascontiguousarray(planes[f]).view(np.uint8))
    assert not back[4].any()  # a Null field reads as zero


def test_null_source_and_destination():
    rec = ["f32"] * 3
    n = 77
    assert oracle.blob_count(rec, {"kind": "null"}) == 0
    for dst in ({"kind": "aos"}, {"kind": "aosoa", "lanes": 8}, {"kind": "soa_sb"}):
        out = oracle.copy(rec, {"kind": "null"}, [], dst, n, fill=0xA5)
        mapped = oracle.copy(rec, {"kind": "soa_mb"}, [np.full(4 * n, 0xFF, np.uint8)] * 3, dst, n, fill=0xA5)
        for o, m in zip(out, mapped):
            # every mapped byte becomes 0; bytes no field maps (AoSoA padding) keep the fill
            assert np.array_equal(o, np.where(m == 0xFF, 0, 0xA5).astype(np.uint8))
    src = oracle.store_planes(rec, {"kind": "aos"}, [np.arange(n, dtype=np.float32)] * 3)
    assert oracle.copy(rec, {"kind": "aos"}, src, {"kind": "null"}, n) == []


# ---------------------------------------------------------------- array extents: linearisation

def test_linearize_matches_numpy_both_orders():
    """Sec. 2 array extents: row-major = numpy order 'C', column-major = order 'F'."""
    rng = np.random.default_rng(7)
    for rank in range(1, 6):
        for _ in range(10):
            ext = [int(x) for x in rng.integers(1, 6, rank)]
            a = [int(rng.integers(0, e)) for e in ext]
            assert oracle.linearize(ext, a) == np.ravel_multi_index(a, ext, order="C")
            assert oracle.linearize(ext, a, col_major=True) == np.ravel_multi_index(a, ext, order="F")


@pytest.mark.parametrize("ext", [(3, 5), (4, 3, 5), (2, 3, 2, 3), (7, 1, 4)])
@pytest.mark.parametrize("dst", [{"kind": "soa_mb"}, {"kind": "aos"}, {"kind": "aosoa", "lanes": 4},
                                 {"kind": "bytesplit", "inner": {"kind": "soa_sb"}}])
def test_copy_nd_row_to_column_major_is_numpy_order_f(ext, dst):
    """Each record holds its own row-major index; after a copy into a column-major
    view, linear position j holds the row-major index of the multi-index whose
    column-major index is j: numpy's C-to-F reordering of arange."""
    rec = ["i32", "f32", "u32"]
    n = int(np.prod(ext))
    idx = np.arange(n, dtype=np.int32)
    planes = [idx, (idx * 0.5).astype(np.float32), (idx ^ 0x5A5A).astype(np.uint32)]
    src = oracle.store_planes(rec, {"kind": "aos"}, planes)
    got = oracle.copy_nd(rec, {"kind": "aos"}, src, dict(dst, col_major=True), list(ext))
    back = oracle.load_planes(rec, dst, got, n)
    perm = np.arange(n).reshape(ext, order="C").ravel(order="F")
    for f in range(3):
        assert np.array_equal(back[f], planes[f][perm]), f
    # and back to row-major restores the records
    again = oracle.copy_nd(rec, dict(dst, col_major=True), got, {"kind": "soa_sb"}, list(ext))
    assert all(np.array_equal(a, b) for a, b in zip(oracle.load_planes(rec, {"kind": "soa_sb"}, again, n), planes))


def test_copy_nd_same_order_is_the_linear_copy():
    """Two views in the same order (either one) place every record at the same
    linear position, so the copy is the plain linear copy; so is any copy whose
    extents have a single non-unit dimension."""
    rec = ["f32"] * 4
    rng = np.random.default_rng(3)
    for ext in ([4, 6], [2, 3, 5], [1, 9, 1], [11]):
        n = int(np.prod(ext))
        planes = [rng.standard_normal(n).astype(np.float32) for _ in range(4)]
        src = oracle.store_planes(rec, {"kind": "aosoa", "lanes": 8}, planes)
        lin = oracle.copy(rec, {"kind": "aosoa", "lanes": 8}, src, {"kind": "soa_sb"}, n)
        for so, do in ((False, False), (True, True)):
            got = oracle.copy_nd(rec, {"kind": "aosoa", "lanes": 8, "col_major": so}, src,
                                 {"kind": "soa_sb", "col_major": do}, ext)
            assert all(np.array_equal(a, b) for a, b in zip(got, lin))
        if sum(e > 1 for e in ext) <= 1:
            got = oracle.copy_nd(rec, {"kind": "aosoa", "lanes": 8}, src, {"kind": "soa_sb", "col_major": True}, ext)
            assert all(np.array_equal(a, b) for a, b in zip(got, lin))

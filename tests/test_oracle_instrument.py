"""Pins of the oracle's instrumentation mappings (Sec. 4), CPU only.

FieldAccessCount keeps two counters per leaf field (loads, stores); Heatmap
keeps one counter per G bytes of every inner blob and adds one to each counter
an access touches.  The counts are checked against closed forms: a copy loads
every field of every record once from the source and stores it once into the
destination.  Byte positions come from ctypes C structs and numpy reshapes,
not from the oracle.  Counting must not change the copied data.
"""
import ctypes as C

import numpy as np
import pytest

import oracle

REC = ["u8", "f64", "i16", "f32"]  # C struct: 1 + 7 pad + 8 + 2 + 2 pad + 4 = 24 bytes
F7 = ["f32"] * 7
_CT = {"u8": C.c_uint8, "f64": C.c_double, "i16": C.c_int16, "f32": C.c_float}


def fac(inner):
    return {"kind": "field_access_count", "inner": inner}


def heat(inner, g):
    return {"kind": "heatmap", "granularity": g, "inner": inner}


def seeded_blobs(rec, spec, n, seed):
    rng = np.random.default_rng(seed)
    return [rng.integers(0, 256, s, dtype=np.uint8) for s in oracle.blob_sizes(rec, spec, n)]


def counters(blobs, first):
    return [b.view(np.uint64) for b in blobs[first:]]


def c_struct_mapped_bytes(rec):
    """Mask of the bytes of one C struct that belong to a field (ctypes layout)."""
    class S(C.Structure):
        _fields_ = [("f%d" % i, _CT[t]) for i, t in enumerate(rec)]
    mask = np.zeros(C.sizeof(S), bool)
    for i, t in enumerate(rec):
        off = getattr(S, "f%d" % i).offset
        mask[off:off + C.sizeof(_CT[t])] = True
    return mask


@pytest.mark.parametrize("inner", [{"kind": "aos"}, {"kind": "soa_sb"}, {"kind": "soa_mb"},
                                   {"kind": "aosoa", "lanes": 4},
                                   {"kind": "bitpack_int", "bits": 5}])
def test_field_access_count_closed_form(inner):
    rec = ["i16", "u8", "i32"] if inner["kind"] == "bitpack_int" else REC
    n = 37
    src = seeded_blobs(rec, {"kind": "soa_mb"}, n, 1)
    dspec = fac(inner)
    sizes = oracle.blob_sizes(rec, dspec, n)
    assert sizes[-1] == 16 * len(rec)  # 2 x fields counters of 8 bytes (Sec. 4)
    dst = oracle.copy(rec, {"kind": "soa_mb"}, src, dspec, n)
    cnt = counters(dst, len(sizes) - 1)[0]
    assert cnt[0::2].tolist() == [0] * len(rec)  # loads
    assert cnt[1::2].tolist() == [n] * len(rec)  # stores
    # reading back through the instrumented view counts loads and leaves stores
    back = oracle.copy(rec, dspec, dst, {"kind": "soa_mb"}, n)
    assert cnt[0::2].tolist() == [n] * len(rec)
    assert cnt[1::2].tolist() == [n] * len(rec)
    for a, b in zip(back, src):
        if inner["kind"] != "bitpack_int":
            assert np.array_equal(a, b)
    # the inner blobs equal those of an uninstrumented copy
    plain = oracle.copy(rec, {"kind": "soa_mb"}, src, inner, n)
    for a, b in zip(dst[:len(plain)], plain):
        assert np.array_equal(a, b)


def test_field_access_count_accumulates_and_both_sides():
    n = 50
    sspec, dspec = fac({"kind": "aos"}), fac({"kind": "aosoa", "lanes": 8})
    src = seeded_blobs(REC, sspec, n, 2)
    src[-1][:] = 0
    dst = oracle.alloc_blobs(REC, dspec, n)
    for _ in range(3):
        oracle.copy(REC, sspec, src, dspec, n, dst_blobs=dst)
    s, d = src[-1].view(np.uint64), dst[-1].view(np.uint64)
    assert s.tolist() == [3 * n, 0] * 4
    assert d.tolist() == [0, 3 * n] * 4


def test_heatmap_bytes_aos_padding_is_zero():
    """Granularity 1 over C-struct AoS: every field byte is hit once, padding never."""
    n = 9
    spec = heat({"kind": "aos"}, 1)
    dst = oracle.copy(REC, {"kind": "soa_mb"}, seeded_blobs(REC, {"kind": "soa_mb"}, n, 3), spec, n)
    sizes = oracle.blob_sizes(REC, spec, n)
    assert sizes == [24 * n, 8 * 24 * n]  # 8x memory for 64-bit byte counters (Sec. 4)
    hm = counters(dst, 1)[0]
    assert np.array_equal(hm, np.tile(c_struct_mapped_bytes(REC), n).astype(np.uint64))


@pytest.mark.parametrize("inner", [{"kind": "soa_sb"}, {"kind": "soa_mb"}, {"kind": "aos", "packed": True}])
def test_heatmap_bytes_dense_layouts_all_ones(inner):
    n = 13
    spec = heat(inner, 1)
    nb = oracle.blob_count(REC, inner)
    dst = oracle.copy(REC, {"kind": "soa_mb"}, seeded_blobs(REC, {"kind": "soa_mb"}, n, 4), spec, n)
    for c in counters(dst, nb):
        assert c.size > 0 and np.all(c == 1)


@pytest.mark.parametrize("L", [1, 4, 5])
def test_heatmap_aosoa_tail_lanes_untouched(L):
    n = 11
    spec = heat({"kind": "aosoa", "lanes": L}, 1)
    dst = oracle.copy(F7, {"kind": "soa_mb"}, seeded_blobs(F7, {"kind": "soa_mb"}, n, 5), spec, n)
    hm = counters(dst, 1)[0].reshape(-1, 7, L, 4)  # blocks, fields, lanes, bytes
    lane = np.arange(hm.shape[0])[:, None] * L + np.arange(L)[None, :]
    want = (lane < n).astype(np.uint64)[:, None, :, None] * np.ones((1, 7, 1, 4), np.uint64)
    assert np.array_equal(hm, want)


@pytest.mark.parametrize("g", [2, 4, 8, 16, 64, 4096])
def test_heatmap_soa_mb_granules(g):
    """Blob f of SoA-MB holds n elements of s_f bytes; a counter of G bytes sees
    ceil-overlap many of them: elements i with [i s, i s + s) meeting [kG, kG + G)."""
    n = 1000
    spec = heat({"kind": "soa_mb"}, g)
    dst = oracle.copy(REC, {"kind": "soa_mb"}, seeded_blobs(REC, {"kind": "soa_mb"}, n, 6), spec, n)
    for f, c in enumerate(counters(dst, len(REC))):
        s = oracle.TYPE_SIZE[REC[f]]
        k = np.arange(c.size, dtype=np.int64)
        first = (k * g) // s
        last = np.minimum((k * g + g - 1) // s, n - 1)
        assert np.array_equal(c, (last - first + 1).astype(np.uint64))


def test_heatmap_record_granules_packed_aos():
    """Granularity = record size over packed AoS: every counter sees every field of one record."""
    n = 21
    S = sum(oracle.TYPE_SIZE[t] for t in REC)
    spec = heat({"kind": "aos", "packed": True}, S)
    dst = oracle.copy(REC, {"kind": "soa_mb"}, seeded_blobs(REC, {"kind": "soa_mb"}, n, 7), spec, n)
    assert counters(dst, 1)[0].tolist() == [len(REC)] * n


def test_heatmap_cache_lines_brute_force():
    """128-byte counters over AoS of 7 f32 (28-byte records) against a direct count
    from C-struct offsets; loads and stores both count."""
    n, g = 100, 128
    spec = heat({"kind": "aos"}, g)
    src = seeded_blobs(F7, {"kind": "soa_mb"}, n, 8)
    dst = oracle.copy(F7, {"kind": "soa_mb"}, src, spec, n)
    want = np.zeros(-(-28 * n // g), np.uint64)
    for i in range(n):
        for f in range(7):
            o = 28 * i + 4 * f
            want[o // g:(o + 3) // g + 1] += 1
    assert np.array_equal(counters(dst, 1)[0], want)
    oracle.copy(F7, spec, dst, {"kind": "soa_mb"}, n)  # loads double every counter
    assert np.array_equal(counters(dst, 1)[0], 2 * want)


def test_heatmap_total_is_granules_touched():
    """Sum of all counters = sum over accesses of the counters each touches."""
    n, g = 333, 8
    spec = heat({"kind": "soa_sb"}, g)
    dst = oracle.copy(REC, {"kind": "soa_mb"}, seeded_blobs(REC, {"kind": "soa_mb"}, n, 9), spec, n)
    total = 0
    base = 0
    for t in REC:
        s = oracle.TYPE_SIZE[t]
        o = base + s * np.arange(n)
        total += int(np.sum((o + s - 1) // g - o // g + 1))
        base += n * s
    assert int(counters(dst, 1)[0].sum()) == total


def test_instrumented_copy_moves_the_same_bytes():
    n = 64
    for inner in ({"kind": "aos"}, {"kind": "aosoa", "lanes": 8}, {"kind": "soa_sb"}):
        src = seeded_blobs(REC, {"kind": "soa_mb"}, n, 10)
        plain = oracle.copy(REC, {"kind": "soa_mb"}, src, inner, n)
        for spec in (fac(inner), heat(inner, 1), heat(inner, 64)):
            inst = oracle.copy(REC, {"kind": "soa_mb"}, src, spec, n)
            for a, b in zip(inst, plain):
                assert np.array_equal(a, b)

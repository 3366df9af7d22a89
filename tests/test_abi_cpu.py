"""C ABI checks that need no GPU: the library loads, exports every entry point
include/llama_mi.h declares, sizes blobs like the oracle, and rejects bad
descriptors, extents, index types and blobs before any GPU work."""
import os
import re

import pytest

import oracle
import paper_2302_08251_amd as lm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

F32x7 = ["f32"] * 7
FAKE = 1 << 40  # 16-byte aligned fake device address; validation never dereferences it


def header_functions():
    src = open(os.path.join(ROOT, "include", "llama_mi.h")).read()
    return re.findall(r"^(?:llama_status|const char\*)\s+(\w+)\(", src, re.M)


def test_library_exports_every_declared_function():
    names = header_functions()
    assert len(names) >= 18
    L = lm.lib()
    for n in names:
        assert hasattr(L, n), n
    assert "gfx950" in lm.llama_version()


SPECS = [
    {"kind": "aos"}, {"kind": "aos", "packed": True}, {"kind": "soa_sb"}, {"kind": "soa_mb"},
    {"kind": "aosoa", "lanes": 32}, {"kind": "aosoa", "lanes": 3},
    {"kind": "bytesplit", "inner": {"kind": "soa_sb"}},
    {"kind": "bytesplit", "inner": {"kind": "aosoa", "lanes": 8}},
    {"kind": "bytesplit", "inner": {"kind": "soa_mb"}},
]


@pytest.mark.parametrize("rec", [F32x7, ["f64"] * 7, ["u8", "f64", "i16", "f32"]], ids=str)
@pytest.mark.parametrize("n", [0, 1, 10, 4097])
def test_blob_sizes_match_oracle(rec, n):
    specs = list(SPECS)
    specs.append({"kind": "changetype", "stored": rec, "inner": {"kind": "aosoa", "lanes": 4}})
    if all(t.startswith("f") for t in rec):
        specs.append({"kind": "changetype", "stored": ["f32"] * len(rec), "inner": {"kind": "soa_mb"}})
        specs.append({"kind": "bitpack_float", "exp": 5, "man": 10})
    specs.append({"kind": "field_access_count", "inner": {"kind": "aosoa", "lanes": 3}})
    specs.append({"kind": "field_access_count", "inner": {"kind": "bytesplit", "inner": {"kind": "soa_mb"}}})
    for g in (1, 8, 128, 1 << 20):
        specs.append({"kind": "heatmap", "granularity": g, "inner": {"kind": "aos"}})
        specs.append({"kind": "heatmap", "granularity": g, "inner": {"kind": "soa_mb"}})
    specs.append({"kind": "heatmap", "granularity": 64, "inner": {"kind": "aosoa", "lanes": 3}})
    for s in specs:
        assert lm.blob_sizes(rec, s, [n]) == oracle.blob_sizes(rec, s, n), s
    ints = ["i32", "u16", "i64"]
    for B in (1, 12, 16):
        s = {"kind": "bitpack_int", "bits": B}
        assert lm.blob_sizes(ints, s, [n]) == oracle.blob_sizes(ints, s, n)


def test_rank_and_extents():
    assert lm.llama_mapping_blob_size(F32x7, {"kind": "aos"}, [3, 4, 5], 0) == 60 * 28
    assert lm.llama_mapping_blob_size(F32x7, {"kind": "aos"}, [3, 0, 5], 0) == 0


def err(fn, *a, **k):
    with pytest.raises(lm.LlamaError) as e:
        fn(*a, **k)
    return e.value.name


def test_descriptor_errors():
    c = lm.llama_mapping_blob_count
    assert err(c, F32x7, {"kind": "aosoa", "lanes": 0}) == "INVALID_ARG"
    assert err(c, ["i32"], {"kind": "bitpack_int", "bits": 0}) == "INVALID_ARG"
    assert err(c, ["i32"], {"kind": "bitpack_int", "bits": 33}) == "INVALID_ARG"
    assert err(c, ["f32"], {"kind": "bitpack_int", "bits": 8}) == "INVALID_ARG"
    assert err(c, ["f32"], {"kind": "bitpack_float", "exp": 1, "man": 5}) == "INVALID_ARG"
    assert err(c, ["f32"], {"kind": "bitpack_float", "exp": 9, "man": 5}) == "INVALID_ARG"
    assert err(c, ["f32"], {"kind": "bitpack_float", "exp": 8, "man": 24}) == "INVALID_ARG"
    assert c(["f64"], {"kind": "bitpack_float", "exp": 11, "man": 52}) == 1
    assert err(c, ["i32"], {"kind": "bitpack_float", "exp": 5, "man": 5}) == "INVALID_ARG"
    assert err(c, F32x7, {"kind": "changetype", "stored": ["i32"] * 7, "inner": {"kind": "aos"}}) == "INVALID_ARG"
    assert err(c, ["f16"], {"kind": "changetype", "stored": ["bf16"], "inner": {"kind": "aos"}}) == "INVALID_ARG"
    assert err(c, F32x7, {"kind": "bytesplit", "inner": {"kind": "bytesplit", "inner": {"kind": "aos"}}}) == "INVALID_ARG"
    # Split needs 1 <= at < fields and two parts; Null has no blobs
    assert err(c, F32x7, {"kind": "split", "at": 0, "parts": [{"kind": "aos"}, {"kind": "aos"}]}) == "INVALID_ARG"
    assert err(c, F32x7, {"kind": "split", "at": 7, "parts": [{"kind": "aos"}, {"kind": "aos"}]}) == "INVALID_ARG"
    assert c(F32x7, {"kind": "split", "at": 3, "parts": [{"kind": "aos"}, {"kind": "soa_mb"}]}) == 5
    assert c(F32x7, {"kind": "split", "at": 2, "parts": [{"kind": "null"}, {"kind": "soa_sb"}]}) == 1
    assert c(F32x7, {"kind": "null"}) == 0
    # the rounding flag belongs to BitPackedFloatSoA only
    assert err(c, F32x7, {"kind": "aos", "round": "rne"}) == "INVALID_ARG"
    assert err(c, ["i32"], {"kind": "bitpack_int", "bits": 5, "round": "rne"}) == "INVALID_ARG"
    assert c(["f32"], {"kind": "bitpack_float", "exp": 5, "man": 10, "round": "rne"}) == 1
    # instrumentation (Sec. 4): FieldAccessCount over kinds 0-7, Heatmap over
    # physical layouts with a power-of-two granularity up to 2^20
    fac = lambda inner: {"kind": "field_access_count", "inner": inner}
    heat = lambda g, inner: {"kind": "heatmap", "granularity": g, "inner": inner}
    assert c(F32x7, fac({"kind": "soa_mb"})) == 8
    assert c(F32x7, fac({"kind": "bitpack_float", "exp": 5, "man": 10})) == 8
    assert err(c, F32x7, fac({"kind": "null"})) == "INVALID_ARG"
    assert err(c, F32x7, fac(fac({"kind": "aos"}))) == "INVALID_ARG"
    assert err(c, F32x7, {"kind": "field_access_count"}) == "INVALID_ARG"
    assert c(F32x7, heat(1, {"kind": "soa_mb"})) == 14
    assert c(F32x7, heat(1 << 20, {"kind": "aos"})) == 2
    for g in (0, 3, 96, 1 << 21):
        assert err(c, F32x7, heat(g, {"kind": "aos"})) == "INVALID_ARG", g
    assert err(c, F32x7, heat(1, {"kind": "bytesplit", "inner": {"kind": "aos"}})) == "INVALID_ARG"
    assert err(c, F32x7, heat(1, {"kind": "bitpack_float", "exp": 5, "man": 10})) == "INVALID_ARG"
    assert err(c, [], {"kind": "aos"}) == "INVALID_ARG"
    assert err(c, ["f32"] * 65, {"kind": "aos"}) == "INVALID_ARG"


def view(rec, spec, n, index="i64", ptrs=None, caps=None):
    sizes = lm.blob_sizes(rec, spec, [n])
    ptrs = ptrs if ptrs is not None else [FAKE + (b << 36) for b in range(len(sizes))]
    caps = caps if caps is not None else sizes
    return lm.llama_view_create(rec, spec, [n], index, ptrs, caps)


def test_view_errors():
    # 64 Mi f64 AoS records need 3.76 GB: too large for I32, fine for U32 / I64
    n = 64 << 20
    assert err(view, ["f64"] * 7, {"kind": "aos"}, n, "i32") == "INDEX_OVERFLOW"
    lm.llama_view_destroy(view(["f64"] * 7, {"kind": "aos"}, n, "u32"))
    lm.llama_view_destroy(view(F32x7, {"kind": "aos"}, n, "i32"))
    assert err(view, F32x7, {"kind": "aos"}, 40000, "i16") == "INDEX_OVERFLOW"
    assert err(view, F32x7, {"kind": "aos"}, 10, ptrs=[FAKE + 4]) == "ALIGNMENT"
    assert err(view, F32x7, {"kind": "aos"}, 10, caps=[279]) == "NO_MEMORY"
    assert err(view, F32x7, {"kind": "aos"}, 10, ptrs=[0]) == "INVALID_ARG"
    assert err(view, F32x7, {"kind": "soa_mb"}, 10, ptrs=[FAKE], caps=[40]) == "INVALID_ARG"


def test_copy_errors_before_gpu_work():
    a = view(F32x7, {"kind": "aos"}, 100)
    b = view(["f32"] * 6, {"kind": "aos"}, 100)
    c = view(F32x7, {"kind": "soa_sb"}, 99)
    d = view(F32x7, {"kind": "bitpack_float", "exp": 8, "man": 15}, 100)
    e = view(F32x7, {"kind": "bitpack_float", "exp": 5, "man": 10}, 100)
    assert err(lm.llama_copy, a, b) == "RECORD_MISMATCH"
    assert err(lm.llama_copy, a, c) == "RECORD_MISMATCH"
    assert err(lm.llama_pack, d, a) == "UNSUPPORTED"
    assert err(lm.llama_unpack, a, d) == "UNSUPPORTED"
    assert err(lm.llama_copy_ex, a, view(F32x7, {"kind": "soa_sb"}, 100), 100) == "INVALID_ARG"
    # every valid pair copies, within two limits: at most 8 physical parts in
    # one SPLIT tree against a partner of another form, at most 64 storage
    # columns (blobs, byte columns, bit streams) on one side

    def tree(lo, hi):
        if hi - lo == 1:
            return {"kind": "aos"}
        mid = (lo + hi) // 2
        return {"kind": "split", "at": mid - lo, "parts": [tree(lo, mid), tree(mid, hi)]}

    r16 = ["f32"] * 16
    sp, sa = view(r16, tree(0, 16), 100), view(r16, {"kind": "aos"}, 100)
    assert err(lm.llama_copy, sp, sa) == "UNSUPPORTED"
    assert err(lm.llama_copy, sa, sp) == "UNSUPPORTED"
    big = ["u8"] * 40 + ["f64"] * 4
    g1, g2 = view(big, {"kind": "aos"}, 100), view(big, {"kind": "bytesplit", "inner": {"kind": "soa_sb"}}, 100)
    assert err(lm.llama_copy, g1, g2) == "UNSUPPORTED"
    for v in (a, b, c, d, e, sp, sa, g1, g2):
        lm.llama_view_destroy(v)


def test_column_major_flag_outermost_only():
    import ctypes as C
    rec = ["f32"] * 3
    n = lm.llama_mapping_blob_count(rec, {"kind": "aos", "col_major": True})
    assert n == 1
    with pytest.raises(lm.LlamaError) as e:
        lm.llama_mapping_blob_count(rec, {"kind": "bytesplit", "inner": {"kind": "aos", "col_major": True}})
    assert e.value.name == "INVALID_ARG"
    # the order does not change blob sizes
    assert lm.llama_mapping_blob_size(rec, {"kind": "aosoa", "lanes": 8, "col_major": True}, [3, 5], 0) == \
        lm.llama_mapping_blob_size(rec, {"kind": "aosoa", "lanes": 8}, [3, 5], 0)

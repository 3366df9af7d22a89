"""GPU parity of the instrumentation mappings (Sec. 4 FieldAccessCount and
Heatmap) against the oracle, bit for bit: the copied bytes and every 64-bit
counter, after one copy and after a second copy back that adds loads."""
import numpy as np
import pytest

import oracle
from gpu_helpers import F32x7, assert_blobs_equal, bits_planes, download, say, upload

import paper_2302_08251_amd as lm
from paper_2302_08251_amd import synth

pytestmark = pytest.mark.gpu

# the tile engine takes records whose leaves have one size
I16x3 = ["i16", "u16", "i16"]
W8x3 = ["f64", "i64", "u64"]
PHYS = [{"kind": "aos"}, {"kind": "aos", "packed": True}, {"kind": "soa_sb"}, {"kind": "soa_mb"},
        {"kind": "aosoa", "lanes": 32}, {"kind": "aosoa", "lanes": 3}]


def fac(inner):
    return {"kind": "field_access_count", "inner": inner}


def heat(inner, g):
    return {"kind": "heatmap", "granularity": g, "inner": inner}


def host_blobs(rec, spec, n, planes=None, fill=0xA5):
    """Blobs of `spec` with zeroed counters; the inner blobs hold `planes` (or `fill`)."""
    sizes = oracle.blob_sizes(rec, spec, n)
    inner = spec.get("inner", spec) if spec["kind"] in ("field_access_count", "heatmap") else spec
    nin = oracle.blob_count(rec, inner)
    if planes is not None:
        data = oracle.store_planes(rec, inner, planes, fill=0x5A)
    else:
        data = oracle.alloc_blobs(rec, inner, n, fill)
    return data + [np.zeros(s, np.uint8) for s in sizes[nin:]]


def view(rec, spec, n, blobs):
    return lm.View(rec, spec, [n], blobs=upload(blobs))


def round_trip(rec, a, b, n, seed):
    """Copies a -> b, then b -> a into fresh data blobs whose counters are a's;
    checks both views' blobs against the oracle after each copy."""
    planes = bits_planes(n, rec, seed)
    sh, dh = host_blobs(rec, a, n, planes), host_blobs(rec, b, n)
    sv, dv = view(rec, a, n, sh), view(rec, b, n, dh)
    lm.llama_copy(sv, dv)
    oracle.copy(rec, a, sh, b, n, dst_blobs=dh)
    assert_blobs_equal(download(sv), sh, "src %s -> %s n=%d" % (a, b, n))
    assert_blobs_equal(download(dv), dh, "dst %s -> %s n=%d" % (a, b, n))
    lm.llama_copy(dv, sv)
    oracle.copy(rec, b, dh, a, n, dst_blobs=sh)
    assert_blobs_equal(download(sv), sh, "back src %s <- %s n=%d" % (a, b, n))
    assert_blobs_equal(download(dv), dh, "back dst %s <- %s n=%d" % (a, b, n))


@pytest.mark.parametrize("n", [1, 1000, 40961])
@pytest.mark.parametrize("rec", [F32x7, W8x3], ids=["f32x7", "w8x3"])
def test_field_access_count(rec, n):
    for a, b in ((fac({"kind": "aos"}), fac({"kind": "soa_sb"})), ({"kind": "soa_mb"}, fac({"kind": "aosoa", "lanes": 32})),
                 (fac({"kind": "bytesplit", "inner": {"kind": "soa_sb"}}), {"kind": "aos"})):
        say("fac", a, b, n)
        round_trip(rec, a, b, n, seed=n)


@pytest.mark.parametrize("n", [1, 1000, 40961])
def test_field_access_count_computed(n):
    rec = ["f32"] * 3
    for a, b in (({"kind": "aos"}, fac({"kind": "bitpack_float", "exp": 6, "man": 9})),
                 (fac({"kind": "soa_sb"}), fac({"kind": "changetype", "stored": ["f16"] * 3, "inner": {"kind": "aos"}}))):
        say("fac computed", a, b, n)
        planes = bits_planes(n, rec, seed=n + 1)
        sh, dh = host_blobs(rec, a, n, planes), host_blobs(rec, b, n)
        sv, dv = view(rec, a, n, sh), view(rec, b, n, dh)
        lm.llama_copy(sv, dv)
        oracle.copy(rec, a, sh, b, n, dst_blobs=dh)
        assert_blobs_equal(download(sv), sh)
        assert_blobs_equal(download(dv), dh)


@pytest.mark.parametrize("g", [1, 4, 64, 128, 4096])
@pytest.mark.parametrize("rec", [F32x7, I16x3], ids=["f32x7", "i16x3"])
def test_heatmap_every_layout(rec, g):
    for n in (1, 777, 40961):
        for i, inner in enumerate(PHYS):
            other = PHYS[(i + 2) % len(PHYS)]
            say("heatmap", g, inner, other, n)
            round_trip(rec, heat(inner, g), heat(other, max(1, g // 2)), n, seed=n + i)


def test_heatmap_and_fac_together_and_empty():
    n = 5000
    round_trip(W8x3, heat({"kind": "aosoa", "lanes": 8}, 16), fac({"kind": "aos"}), n, seed=3)
    sv, dv = lm.View(F32x7, fac({"kind": "aos"}), [0]), lm.View(F32x7, heat({"kind": "soa_sb"}, 1), [0])
    sv.blobs[-1].zero_()
    lm.llama_copy(sv, dv)
    assert download(sv)[-1].view(np.uint64).tolist() == [0] * 14


def test_full_size_heatmap_cache_lines():
    """16 Mi records of 7 f32 (the copy benchmark's size), 128-byte counters on
    both sides, against the oracle."""
    n = 1 << 24
    a, b = heat({"kind": "aos"}, 128), heat({"kind": "soa_sb"}, 128)
    say("full-size heatmap", n)
    planes = bits_planes(n, F32x7, seed=11)
    sh, dh = host_blobs(F32x7, a, n, planes), host_blobs(F32x7, b, n)
    sv, dv = view(F32x7, a, n, sh), view(F32x7, b, n, dh)
    lm.llama_copy(sv, dv)
    oracle.copy(F32x7, a, sh, b, n, dst_blobs=dh)
    got_s, got_d = download(sv), download(dv)
    assert_blobs_equal(got_s[1:], sh[1:], "source counters")
    assert_blobs_equal(got_d, dh, "destination")


def test_rejected_uses():
    n = 100
    with pytest.raises(lm.LlamaError) as e:
        lm.View(F32x7, heat({"kind": "bytesplit", "inner": {"kind": "aos"}}, 1), [n])
    assert e.value.name == "INVALID_ARG"
    with pytest.raises(lm.LlamaError) as e:
        lm.View(F32x7, heat({"kind": "aos"}, 3), [n])
    assert e.value.name == "INVALID_ARG"
    with pytest.raises(lm.LlamaError) as e:
        lm.View(F32x7, fac({"kind": "split", "at": 2, "parts": [{"kind": "aos"}, {"kind": "aos"}]}), [n])
    assert e.value.name == "INVALID_ARG"
    sv, dv = lm.View(F32x7, fac({"kind": "aos"}), [n], fill=0), lm.View(F32x7, {"kind": "soa_sb"}, [n])
    with pytest.raises(lm.LlamaError) as e:
        lm.Batch([sv], [dv])
    assert e.value.name == "UNSUPPORTED"


def test_heatmap_soa_blob_beyond_4_gib():
    """One SoA-SB period of 160 Mi + 3 records x 28 bytes (4.7 GB) takes the 64-bit
    arithmetic.  SoA-SB of 4-byte leaves is dense and 4-byte aligned, so a counter of
    G bytes sees (its bytes inside the blob) / 4 accesses; this closed form is the
    one the oracle is pinned on for SoA granules."""
    n, g = (160 << 20) + 3, 4096
    say("heatmap beyond 4 GiB", n)
    sv = lm.View(F32x7, {"kind": "aos"}, [n], fill=0)
    dv = lm.View(F32x7, heat({"kind": "soa_sb"}, g), [n], fill=0)
    lm.llama_copy(sv, dv)
    got = download(dv)[1].view(np.uint64)
    size = 28 * n
    q = np.arange(got.size, dtype=np.int64)
    want = (np.minimum(q * g + g, size) - q * g) // 4
    assert np.array_equal(got, want.astype(np.uint64))
    sv.close()
    dv.close()


@pytest.mark.parametrize("n", [1, 3001])
def test_instrumented_parts_and_null(n):
    """Instrumentation composes with the meta-mappings: counted parts inside Splits,
    loads counted when the destination is Null, stores counted when the source is."""
    a = {"kind": "split", "at": 3, "parts": [fac({"kind": "aos"}), heat({"kind": "soa_mb"}, 4)]}
    b = {"kind": "split", "at": 3, "parts": [{"kind": "soa_sb"}, fac({"kind": "aosoa", "lanes": 32})]}
    say("split parts", n)
    planes = bits_planes(n, F32x7, seed=n)
    sh = oracle.store_planes(F32x7, a, planes, fill=0)
    # blobs: AoS data, 2 x 3 counters | 4 SoA-MB planes, 4 counter blobs
    for i in (1, 6, 7, 8, 9):
        sh[i][:] = 0
    dh = oracle.alloc_blobs(F32x7, b, n, 0xA5)
    dh[-1][:] = 0
    sv, dv = view(F32x7, a, n, sh), view(F32x7, b, n, dh)
    lm.llama_copy(sv, dv)
    oracle.copy(F32x7, a, sh, b, n, dst_blobs=dh)
    assert_blobs_equal(download(sv), sh, "split source")
    assert_blobs_equal(download(dv), dh, "split destination")
    say("null ends", n)
    null = {"kind": "null"}
    fs = fac({"kind": "soa_sb"})
    s2 = host_blobs(F32x7, fs, n, planes)
    v2 = view(F32x7, fs, n, s2)
    lm.llama_copy(v2, lm.View(F32x7, null, [n]))
    oracle.copy(F32x7, fs, s2, null, n, dst_blobs=[])
    assert_blobs_equal(download(v2), s2, "loads into null")
    # a Split source with instrumented parts counts its loads into Null too
    s4 = oracle.store_planes(F32x7, a, planes, fill=0)
    for i in (1, 6, 7, 8, 9):
        s4[i][:] = 0
    v4 = view(F32x7, a, n, s4)
    lm.llama_copy(v4, lm.View(F32x7, null, [n]))
    oracle.copy(F32x7, a, s4, null, n, dst_blobs=[])
    assert any(b.any() for b in (s4[1], s4[6])), "the oracle counts the loads"
    assert_blobs_equal(download(v4), s4, "split loads into null")
    hd = heat({"kind": "aosoa", "lanes": 3}, 8)
    d3 = host_blobs(F32x7, hd, n)
    v3 = view(F32x7, hd, n, d3)
    lm.llama_copy(lm.View(F32x7, null, [n]), v3)
    oracle.copy(F32x7, null, [], hd, n, dst_blobs=d3)
    assert_blobs_equal(download(v3), d3, "stores from null")


@pytest.mark.parametrize("n", [3001, 256])
@pytest.mark.parametrize("spec", [fac({"kind": "soa_mb"}), fac({"kind": "bitpack_float", "exp": 8, "man": 15}),
                                  heat({"kind": "soa_mb"}, 128), heat({"kind": "aos"}, 4),
                                  heat({"kind": "aosoa", "lanes": 32}, 1)],
                         ids=["fac_soa_mb", "fac_e8m15", "heat128_soa_mb", "heat4_aos", "heat1_aosoa32"])
def test_instrumented_nbody_counts_every_access(spec, n):
    """The n-body consumer through an instrumented view (Sec. 4): every load and
    store its kernels make adds to the counters; bit-exact against the oracle's
    n-body through the same mapping with the same access pattern (a particle's
    position once per update, every j-particle's position and mass once per
    256-particle i-block, the move's loads and stores), over two steps and one
    energy check."""
    rec = F32x7
    inner = spec["inner"]
    planes = [p.astype(np.float32) for p in synth.particles(n, 4)]
    host = host_blobs(rec, spec, n, planes)
    say("instrumented nbody", spec, n)
    v = view(rec, spec, n, host)
    lm.nbody_step(v, 2, 1e-4, 0.01)
    lm.nbody_energy(v, 0.01)
    got = download(v)
    oracle.nbody_view(rec, spec, host, n, 2, 1e-4, 0.01, tile=256)
    oracle.energy_view(rec, spec, host, n, 0.01)
    nin = oracle.blob_count(rec, inner)
    assert_blobs_equal(got[nin:], host[nin:], "counters")
    v.close()

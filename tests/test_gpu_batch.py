"""Batched copy: many views of uneven sizes with mixed mapping pairs moved by
one persistent, hipGraph-captured launch; every destination must equal the
oracle's copy, on every graph replay, and equal the per-view launches."""
import numpy as np
import pytest

import oracle
from gpu_helpers import CFG2, F32x7, assert_blobs_equal, bits_planes, download, gpu_view, say

import paper_2302_08251_amd as lm
from paper_2302_08251_amd import synth

pytestmark = pytest.mark.gpu

NAMES = list(CFG2)
OFFDIAG = [(a, b) for a in NAMES for b in NAMES if a != b]


def make_batch(count, lo, hi, seed):
    ns, pairs = synth.batch_views(count, seed, lo, hi)
    views = []
    for k, (n, p) in enumerate(zip(ns.tolist(), pairs.tolist())):
        a, b = OFFDIAG[p]
        planes = bits_planes(n, F32x7, seed=seed * 1000 + k)
        src_host = oracle.store_planes(F32x7, CFG2[a], planes, fill=0x5A)
        exp = oracle.copy(F32x7, CFG2[a], src_host, CFG2[b], n, fill=0xA5)
        views.append((gpu_view(F32x7, CFG2[a], n, src_host), gpu_view(F32x7, CFG2[b], n, fill=0xA5), exp, (a, b, n)))
    return views


def check(views, what):
    for sv, dv, exp, tag in views:
        assert_blobs_equal(download(dv), exp, "%s %s" % (what, tag))


def reset(views):
    for _, dv, _, _ in views:
        for t in dv.blobs:
            t.fill_(0xA5)


def test_batch_graph_replays_match_oracle():
    torch = pytest.importorskip("torch")
    views = make_batch(120, 1, 30000, seed=1)
    batch = lm.Batch([v[0] for v in views], [v[1] for v in views])
    info = batch.info()
    say("batch info", info)
    # tile code: 0 = each view's default tile, 1 = the same capped to 16 KiB of LDS,
    # 2 = grown to the largest default tile's LDS; else records per tile
    assert info["n_views"] == 120 and (info["tile_records"] in (0, 1, 2) or info["tile_records"] % 128 == 0)
    reset(views)
    for rep in range(3):
        batch.launch()
        torch.cuda.synchronize()
        check(views, "graph replay %d" % rep)
        reset(views)  # eager work between replays
        x = torch.ones(1 << 20, device="cuda").sum()
        assert float(x) == float(1 << 20)
        torch.cuda.synchronize()
    batch.launch_per_view()
    check(views, "per-view")
    batch.close()


def test_batch_tune_cache_roundtrip(tmp_path):
    torch = pytest.importorskip("torch")
    views = make_batch(40, 100, 5000, seed=2)
    path = str(tmp_path / "tune.json")
    b1 = lm.Batch([v[0] for v in views], [v[1] for v in views], tune_cache=path)
    i1 = b1.info()
    assert i1["tune_seconds"] > 0
    b2 = lm.Batch([v[0] for v in views], [v[1] for v in views], tune_cache=path)
    i2 = b2.info()
    assert i2["tune_seconds"] == 0 and (i2["tile_records"], i2["grid"]) == (i1["tile_records"], i1["grid"])
    reset(views)
    b2.launch()
    torch.cuda.synchronize()
    check(views, "cached batch")
    b1.close()
    b2.close()


@pytest.mark.parametrize("code,grid", [(0, 256), (1, 2048), (2, 97), (2, 0), (512, 1000)])
def test_batch_every_tile_choice_matches_oracle(tmp_path, code, grid):
    """Every tile choice the autotuner can make, forced through the tune cache
    (the cached entry is used as is), with a persistent grid smaller than, and
    one workgroup per, tile."""
    torch = pytest.importorskip("torch")
    views = make_batch(50, 1, 20000, seed=3)
    path = tmp_path / "tune.json"
    b0 = lm.Batch([v[0] for v in views], [v[1] for v in views], tune_cache=str(path))
    total = b0.info()["total_tiles"]
    b0.close()
    text = path.read_text()
    import re
    g = grid if grid else 1 << 30  # 0: one workgroup per tile (clamped below)
    text = re.sub(r'"tile_records": \d+, "grid": \d+', '"tile_records": %d, "grid": %d' % (code, min(g, 1 << 20)), text)
    path.write_text(text)
    b = lm.Batch([v[0] for v in views], [v[1] for v in views], tune_cache=str(path))
    info = b.info()
    say("forced", code, grid, info, "code-0 tiles", total)
    assert info["tune_seconds"] == 0 and info["tile_records"] == code
    reset(views)
    b.launch()
    torch.cuda.synchronize()
    check(views, "tile code %d grid %d" % (code, grid))
    b.close()


@pytest.mark.parametrize("tile_map", [0, 1])
def test_batch_xcd_tile_map_matches_oracle(tmp_path, tile_map):
    """One workgroup per tile, with and without each XCD taking a contiguous
    run of tiles (forced through the tune cache), over mixed mapping pairs."""
    torch = pytest.importorskip("torch")
    views = make_batch(40, 1, 30000, seed=8)
    path = tmp_path / "tune.json"
    b0 = lm.Batch([v[0] for v in views], [v[1] for v in views], tune_cache=str(path))
    b0.close()
    import re
    text = re.sub(r'"grid": \d+', '"grid": %d' % (1 << 30), path.read_text())
    text = re.sub(r'"tile_map": \d+', '"tile_map": %d' % tile_map, text)
    path.write_text(text)
    b = lm.Batch([v[0] for v in views], [v[1] for v in views], tune_cache=str(path))
    info = b.info()
    say("tile map", tile_map, info)
    assert info["tile_map"] == tile_map and info["grid"] == info["total_tiles"]
    reset(views)
    b.launch()
    torch.cuda.synchronize()
    check(views, "tile map %d" % tile_map)
    b.close()


def test_batch_mixed_record_types_matches_oracle():
    """One launch over views of different leaf sizes (f64, f32, i16, u8 records)
    and mappings, Bytesplit included; every view equals the oracle's copy."""
    torch = pytest.importorskip("torch")
    recs = [["f64"] * 3, ["f32"] * 7, ["i16", "u16", "i16"], ["u8"] * 5]
    maps = [{"kind": "aos"}, {"kind": "soa_sb"}, {"kind": "soa_mb"}, {"kind": "aosoa", "lanes": 32},
            {"kind": "bytesplit", "inner": {"kind": "soa_sb"}}, {"kind": "bytesplit", "inner": {"kind": "aos"}}]
    rng = np.random.default_rng(11)
    views = []
    for k in range(48):
        rec = recs[k % len(recs)]
        a, b = rng.choice(len(maps), 2, replace=False)
        n = int(rng.integers(1, 9000))
        planes = bits_planes(n, rec, seed=500 + k)
        src_host = oracle.store_planes(rec, maps[a], planes, fill=0x5A)
        exp = oracle.copy(rec, maps[a], src_host, maps[b], n, fill=0xA5)
        views.append((gpu_view(rec, maps[a], n, src_host), gpu_view(rec, maps[b], n, fill=0xA5), exp,
                      (str(rec[0]), maps[a]["kind"], maps[b]["kind"], n)))
    batch = lm.Batch([v[0] for v in views], [v[1] for v in views])
    reset(views)
    batch.launch()
    torch.cuda.synchronize()
    check(views, "mixed records")
    batch.launch_per_view()
    check(views, "mixed records, per view")
    batch.close()

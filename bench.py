"""Benchmark of the gfx950 layout-copy / pack library on one MI355X.

One step = one pass of the layout-copy hot path over the single-view workload:
64 Mi particle records {pos.x,pos.y,pos.z,vel.x,vel.y,vel.z,mass} of float32,
copied once along each of the 36 ordered pairs of AoS, SoA single-blob, SoA
multi-blob, AoSoA-32, AoSoA-64 and Bytesplit(SoA single-blob), 32-bit index
type.  `value` is the step's algorithmic bytes (mapped bytes read + mapped
bytes written) divided by its time, inputs resident in HBM.

The same JSON line carries the other rows of the hot path measured at their
own workloads (float/int bit packing and ChangeType on 256 Mi / 64 Mi
elements, the 2000-view batched copy against per-view launches, and the
all-pairs n-body step), the roofline of the dominant kernel and the CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3        # vector FP32 peak
FP32_LANE_OPS = FP32_PEAK_TFLOPS * 1e12 / 2   # FMA lane operations per second at that peak
METRIC = "layout-copy & pack GB/s (% of HBM peak), batched vs per-view, bit-exact"
F32x7 = ["f32"] * 7
LAYOUTS = {
    "AoS": {"kind": "aos"},
    "SoA-SB": {"kind": "soa_sb"},
    "SoA-MB": {"kind": "soa_mb"},
    "AoSoA-32": {"kind": "aosoa", "lanes": 32},
    "AoSoA-64": {"kind": "aosoa", "lanes": 64},
    "Bytesplit": {"kind": "bytesplit", "inner": {"kind": "soa_sb"}},
}
PAIR_ORDER = list(LAYOUTS)  # pair index p -> (src, dst) over the 30 off-diagonal pairs
OFFDIAG = [(a, b) for a in PAIR_ORDER for b in PAIR_ORDER if a != b]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class Timer:
    """HIP events on the current torch stream (the stream the library launches on)."""

    def __init__(self, torch):
        self.torch = torch

    def warm(self, fn, seconds=0.2):
        """Runs fn until `seconds` of GPU work have passed: after CPU-side input
        generation the GPU needs that long to return to its steady clocks."""
        t = self.torch
        t.cuda.synchronize()
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            fn()
            t.cuda.synchronize()

    def time(self, fn, reps, warm=True):
        t = self.torch
        if warm:
            self.warm(fn)
        evs = [(t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in evs:
            a.record()
            fn()
            b.record()
        t.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in evs]  # ms


def kernel_hash(files=("tile_engine.hpp", "kernels.hpp", "k_raw.hip", "k_raw4.hip", "internal.hpp")):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2302_08251_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


NB_FILES = ("nbody.hip", "static_view.hpp", "tile_engine.hpp", "internal.hpp")


def nbody_valu_per_interaction():
    """VALU wave instructions x 64 lanes per interaction of the n-body update kernel,
    from the committed SQ counter run when it was taken on the current sources."""
    try:
        with open(os.path.join(ROOT, "profiles", "nbody_update_sq.json")) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    return d.get("valu_per_interaction") if d.get("kernel_hash") == kernel_hash(NB_FILES) else None


def measured_traffic(alg_bytes):
    """HBM bytes per launch from committed rocprofv3 counter runs, when they were taken
    on the current kernel sources; otherwise None."""
    p = os.path.join(ROOT, "profiles", "traffic_copy_cfg2.json")
    try:
        with open(p) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d.get("hbm_bytes_per_launch")


# ------------------------------------------------------------------ in-run parity gates
# Every row checks its results before it is timed; a row whose check fails
# raises RowFailed and reports the failure instead of a number.

class RowFailed(Exception):
    pass


def gate(ok, what):
    if not ok:
        raise RowFailed("parity gate failed: " + what)


def gate_equal_floats(torch, got, want, what):
    """Bitwise equality, except that a NaN only has to stay a NaN."""
    nan_w = torch.isnan(want)
    gate(torch.equal(torch.isnan(got), nan_w), what + ": NaN positions differ")
    ib = {torch.float32: torch.int32, torch.float64: torch.int64}[got.dtype]
    diff = (got.view(ib) != want.view(ib)) & ~nan_w
    bad = int(diff.sum())
    gate(bad == 0, "%s: %d of %d values differ" % (what, bad, got.numel()))


def gate_float_codes(lm, torch, src, c, back, E, M, n):
    """BitPackedFloat (Sec. 3) with truncation: (1) decoding then re-encoding gives
    the same packed stream (the decoded values are representable); (2) for E = 8
    the format keeps the f32 exponent, so a decoded non-NaN value is the input
    with its 23 - M low mantissa bits cleared; otherwise every decoded value keeps
    the sign, never grows in magnitude, and is infinite only when the input's
    magnitude reaches 2^(2^(E-1)) (the first power of two above the largest
    finite value) or is infinite."""
    code = c.blobs[0].clone()
    again = lm.View(["f32"], {"kind": "bitpack_float", "exp": E, "man": M}, [n], index_type="u32")
    lm.llama_pack(back, again)
    nbytes = (n * (1 + E + M) + 7) // 8
    gate(torch.equal(again.blobs[0][:nbytes], code[:nbytes]), "e%dm%d: re-encoding the decoded values "
         "changes the stream" % (E, M))
    again.close()
    x = src.blobs[0][: 4 * n].view(torch.int32)
    y = back.blobs[0][: 4 * n].view(torch.int32)
    xf, yf = x.view(torch.float32), y.view(torch.float32)
    gate(torch.equal(torch.isnan(xf), torch.isnan(yf)), "e%dm%d: NaN positions differ" % (E, M))
    ok = ~torch.isnan(xf)
    if E == 8:
        mask = -(1 << (23 - M))
        gate(torch.equal((x & mask)[ok], y[ok]), "e8m%d: decoded != input with low bits cleared" % M)
    else:
        gate(torch.equal((x < 0)[ok], (y < 0)[ok]), "e%dm%d: sign changed" % (E, M))
        ax, ay = xf.abs(), yf.abs()
        fin = ok & torch.isfinite(yf)
        gate(bool((ay[fin] <= ax[fin]).all()), "e%dm%d: truncation grew a value" % (E, M))
        inf = ok & torch.isinf(yf)
        gate(bool((ax[inf] >= 2.0 ** (1 << (E - 1))).all()), "e%dm%d: finite input became Inf" % (E, M))
        del ax, ay, fin, inf
    del code, ok


# ------------------------------------------------------------------ cfg2: single view, 36 pairs

def bench_cfg2(lm, torch, steps, warmup, n):
    from paper_2302_08251_amd import synth
    T = Timer(torch)
    log("cfg2: generating %d records" % n)
    planes = synth.particles(n, 0, dtype=np.float32)
    mb = lm.View(F32x7, LAYOUTS["SoA-MB"], [n], index_type="i32",
                 blobs=[torch.from_numpy(p.view(np.uint8)).cuda() for p in planes])
    del planes
    src = {k: lm.View(F32x7, s, [n], index_type="i32") for k, s in LAYOUTS.items()}
    dst = {k: lm.View(F32x7, s, [n], index_type="i32") for k, s in LAYOUTS.items()}
    for k in LAYOUTS:
        lm.llama_copy(mb, src[k])
    torch.cuda.synchronize()
    # property check before timing: X -> Y -> SoA-MB reproduces the planes bit for bit
    back = lm.View(F32x7, LAYOUTS["SoA-MB"], [n], index_type="i32")
    for a in PAIR_ORDER:
        for b in PAIR_ORDER:
            lm.llama_copy(src[a], dst[b])
            lm.llama_copy(dst[b], back)
            torch.cuda.synchronize()
            for f in range(7):
                if not torch.equal(back.blobs[f][: 4 * n], mb.blobs[f][: 4 * n]):
                    raise RowFailed("cfg2 round trip %s -> %s -> SoA-MB is not bit-exact" % (a, b))
    alg = 2 * n * 28
    pairs = [(a, b) for a in PAIR_ORDER for b in PAIR_ORDER]

    def step():
        for a, b in pairs:
            lm.llama_copy(src[a], dst[b])

    for _ in range(warmup):
        step()
    T.warm(step)
    per_pair = {f"{a}->{b}": [] for a, b in pairs}
    step_ms = []
    for _ in range(steps):
        ts = []
        for a, b in pairs:
            ms = T.time(lambda: lm.llama_copy(src[a], dst[b]), 1, warm=False)[0]
            per_pair[f"{a}->{b}"].append(ms)
            ts.append(ms)
        step_ms.append(sum(ts))
    med = {k: float(np.median(v)) for k, v in per_pair.items()}
    step_med = float(np.median(step_ms))
    # also the end-to-end step time without per-launch events
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3 / steps
    # device-to-device memcpy of one side's bytes: practical copy ceiling
    a = torch.empty(n * 28, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    cp = T.time(lambda: b.copy_(a), 5)
    memcpy_gbs = 2 * n * 28 / (np.median(cp) * 1e-3) / 1e9
    del a, b
    for v in list(src.values()) + list(dst.values()) + [mb, back]:
        v.close()
    torch.cuda.empty_cache()
    pair_gbs = {k: alg / (v * 1e-3) / 1e9 for k, v in med.items()}
    off = [pair_gbs[f"{a}->{b}"] for a, b in OFFDIAG]
    return {
        "records": n, "alg_bytes_per_pair": alg, "step_ms": step_med, "step_wall_ms": wall_ms,
        "step_ms_min": float(np.min(step_ms)), "step_ms_max": float(np.max(step_ms)), "timed_steps": len(step_ms),
        "gbs_step": 36 * alg / (step_med * 1e-3) / 1e9,
        "records_per_s": 36 * n / (step_med * 1e-3),
        "pair_gbs": {k: round(v, 1) for k, v in pair_gbs.items()},
        "pair_ms": {k: round(v, 4) for k, v in med.items()},
        "offdiag_min_gbs": min(off), "offdiag_max_gbs": max(off),
        "memcpy_dtod_gbs": memcpy_gbs,
    }


# ------------------------------------------------------------------ cfg3: computed mappings

def bench_cfg3(lm, torch, reps, n_vals, n_rec):
    from paper_2302_08251_amd import synth
    T = Timer(torch)
    out = {}
    log("cfg3: float pack/unpack on %d values" % n_vals)
    bits = torch.from_numpy(synth.float_specials(n_vals, 0).view(np.uint8)).cuda()
    src = lm.View(["f32"], {"kind": "soa_mb"}, [n_vals], blobs=[bits], index_type="u32")
    back = lm.View(["f32"], {"kind": "soa_mb"}, [n_vals], index_type="u32")
    x = src.blobs[0][: 4 * n_vals].view(torch.int32)
    xf = x.view(torch.float32)
    for E, M in ((8, 7), (5, 10), (8, 15)):
        c = lm.View(["f32"], {"kind": "bitpack_float", "exp": E, "man": M}, [n_vals], index_type="u32")
        lm.llama_pack(src, c)
        lm.llama_unpack(c, back)
        gate_float_codes(lm, torch, src, c, back, E, M, n_vals)
        alg = 4 * n_vals + (n_vals * (1 + E + M) + 7) // 8
        tp = float(np.median(T.time(lambda: lm.llama_pack(src, c), reps)))
        tu = float(np.median(T.time(lambda: lm.llama_unpack(c, back), reps)))
        out[f"float_e{E}m{M}"] = {"pack_gbs": alg / tp / 1e6, "unpack_gbs": alg / tu / 1e6,
                                  "pack_ms": tp, "unpack_ms": tu, "alg_bytes": alg}
        c.close()
    # ChangeType into half formats on the same values (narrowing RNE / exact widening)
    for stored in ("f16", "bf16"):
        c = lm.View(["f32"], {"kind": "changetype", "stored": [stored], "inner": {"kind": "soa_mb"}}, [n_vals],
                    index_type="u32")
        lm.llama_pack(src, c)
        lm.llama_unpack(c, back)
        ht = torch.float16 if stored == "f16" else torch.bfloat16
        gate_equal_floats(torch, back.blobs[0][: 4 * n_vals].view(torch.float32),
                          xf.to(ht).to(torch.float32), "ChangeType f32->%s->f32 (RNE narrowing)" % stored)
        alg = 6 * n_vals
        tp = float(np.median(T.time(lambda: lm.llama_pack(src, c), reps)))
        tu = float(np.median(T.time(lambda: lm.llama_unpack(c, back), reps)))
        out[f"changetype_f32_{stored}"] = {"pack_gbs": alg / tp / 1e6, "unpack_gbs": alg / tu / 1e6,
                                           "pack_ms": tp, "unpack_ms": tu, "alg_bytes": alg}
        c.close()
    log("cfg3: int pack/unpack B=3..31")
    g = torch.Generator(device="cuda").manual_seed(0)
    u = torch.randint(0, 2 ** 31, (n_vals,), generator=g, device="cuda", dtype=torch.int64).to(torch.int32)
    ints = {}
    iback = lm.View(["i32"], {"kind": "soa_mb"}, [n_vals], index_type="u32")
    for B in range(3, 32):
        # uniform over [-2^(B-1), 2^(B-1)): top B bits of a uniform 31-bit draw, recentred
        vals = (u >> (31 - B)) - (1 << (B - 1))
        s = lm.View(["i32"], {"kind": "soa_mb"}, [n_vals], blobs=[vals.view(torch.uint8)], index_type="u32")
        c = lm.View(["i32"], {"kind": "bitpack_int", "bits": B}, [n_vals], index_type="u32")
        lm.llama_pack(s, c)
        lm.llama_unpack(c, iback)
        torch.cuda.synchronize()
        if not torch.equal(iback.blobs[0][: 4 * n_vals], s.blobs[0][: 4 * n_vals]):
            raise RowFailed("int B=%d round trip is not exact" % B)
        alg = 4 * n_vals + (n_vals * B + 7) // 8
        tp = float(np.median(T.time(lambda: lm.llama_pack(s, c), reps)))
        tu = float(np.median(T.time(lambda: lm.llama_unpack(c, iback), reps)))
        ints[B] = (alg / tp / 1e6, alg / tu / 1e6)
        s.close()
        c.close()
        del vals
    out["int"] = {"pack_gbs": {B: round(v[0], 1) for B, v in ints.items()},
                  "unpack_gbs": {B: round(v[1], 1) for B, v in ints.items()},
                  "pack_min_gbs": min(v[0] for v in ints.values()),
                  "unpack_min_gbs": min(v[1] for v in ints.values())}
    del u, bits, x, xf
    src.close()
    back.close()
    iback.close()
    torch.cuda.empty_cache()
    log("cfg3: ChangeType f64->f32 on %d records" % n_rec)
    planes = synth.changetype_values(n_rec, 0)
    mb = lm.View(["f64"] * 7, {"kind": "soa_mb"}, [n_rec], index_type="u32",
                 blobs=[torch.from_numpy(p.view(np.uint8)).cuda() for p in planes])
    del planes
    aos = lm.View(["f64"] * 7, {"kind": "aos"}, [n_rec], index_type="u32")
    lm.llama_copy(mb, aos)
    ct = lm.View(["f64"] * 7, {"kind": "changetype", "stored": ["f32"] * 7, "inner": {"kind": "soa_mb"}},
                 [n_rec], index_type="u32")
    aos2 = lm.View(["f64"] * 7, {"kind": "aos"}, [n_rec], index_type="u32")
    lm.llama_pack(aos, ct)
    lm.llama_unpack(ct, aos2)
    mb2 = lm.View(["f64"] * 7, {"kind": "soa_mb"}, [n_rec], index_type="u32")
    lm.llama_copy(aos2, mb2)
    for f in range(7):
        a = mb.blobs[f][: 8 * n_rec].view(torch.float64)
        gate_equal_floats(torch, mb2.blobs[f][: 8 * n_rec].view(torch.float64),
                          a.to(torch.float32).to(torch.float64), "ChangeType f64->f32->f64 field %d" % f)
    mb2.close()
    alg = n_rec * 56 + n_rec * 28
    tp = float(np.median(T.time(lambda: lm.llama_pack(aos, ct), reps)))
    tu = float(np.median(T.time(lambda: lm.llama_unpack(ct, aos2), reps)))
    out["changetype_f64_f32"] = {"pack_gbs": alg / tp / 1e6, "unpack_gbs": alg / tu / 1e6,
                                 "pack_ms": tp, "unpack_ms": tu, "alg_bytes": alg, "records": n_rec}
    for v in (mb, aos, ct, aos2):
        v.close()
    torch.cuda.empty_cache()
    return out


# ------------------------------------------------------------------ instrumentation

def fac(m):
    return {"kind": "field_access_count", "inner": m}


def heat(m, g):
    return {"kind": "heatmap", "granularity": g, "inner": m}


def counters(torch, v, first):
    """The 64-bit counters of an instrumented view (blobs from index `first` on)."""
    return [t[: sz].view(torch.int64) for t, sz in zip(v.blobs[first:], v.sizes[first:])]


def bench_instr(lm, torch, reps, n):
    """Sec. 4 instrumentation: the AoS -> SoA-SB copy of 7 x f32 records, plain and
    with FieldAccessCount or Heatmap (G = 128 and G = 1) on both views; the
    slowdown over the plain copy and the counter memory per view.  I64 index
    everywhere: a G = 1 heatmap of these views holds 15 GB of counters.
    Gate: the destination records equal the plain copy's; FieldAccessCount reads
    n loads per field on the source and n stores per field on the destination;
    every field access of these 4-byte aligned fields touches one G = 128
    counter or four G = 1 counters, so each view's heatmap sums to 7n or 28n."""
    T = Timer(torch)
    log("instr: AoS -> SoA-SB on %d records, plain and instrumented" % n)
    rec = ["f32"] * 7
    base = lm.View(rec, {"kind": "aos"}, [n], index_type="i64", fill=1)
    base.blobs[0].copy_(torch.randint(0, 256, base.blobs[0].shape, device="cuda", dtype=torch.uint8))
    out = {"records": n}
    cases = [("plain", None), ("field_access_count", fac),
             ("heatmap_g128", lambda m: heat(m, 128)), ("heatmap_g1", lambda m: heat(m, 1))]
    t_plain = None
    want = None
    for name, wrap in cases:
        sm, dm = {"kind": "aos"}, {"kind": "soa_sb"}
        if wrap:
            sm, dm = wrap(sm), wrap(dm)
        if wrap:  # counters start at zero; the data blob holds the same records
            sv = lm.View(rec, sm, [n], index_type="i64", fill=0)
            sv.blobs[0].copy_(base.blobs[0][: sv.sizes[0]])
        else:
            sv = lm.View(rec, sm, [n], index_type="i64", blobs=[base.blobs[0]])
        dv = lm.View(rec, dm, [n], index_type="i64", fill=0)
        lm.llama_copy(sv, dv)
        torch.cuda.synchronize()
        if want is None:
            want = dv.blobs[0][: 28 * n].clone()
        else:
            gate(torch.equal(dv.blobs[0][: 28 * n], want), "instr %s: records differ from the plain copy" % name)
            cs, cd = counters(torch, sv, 1), counters(torch, dv, 1)
            if name == "field_access_count":
                ls, ld = cs[0].view(7, 2), cd[0].view(7, 2)
                gate(bool((ls[:, 0] == n).all() and (ls[:, 1] == 0).all()), "instr fac: source counts")
                gate(bool((ld[:, 0] == 0).all() and (ld[:, 1] == n).all()), "instr fac: destination counts")
            else:
                per = 7 * n * (4 if name == "heatmap_g1" else 1)
                for c, side in ((cs, "source"), (cd, "destination")):
                    gate(sum(int(t.sum()) for t in c) == per, "instr %s: %s heatmap total" % (name, side))
        t = float(np.median(T.time(lambda: lm.llama_copy(sv, dv), reps)))
        row = {"ms": round(t, 4), "gbs": round(2 * 28 * n / t / 1e6, 1)}
        counter_bytes = sum(sv.sizes[1:]) if wrap else 0
        if wrap:
            row["counter_bytes_per_view"] = counter_bytes
            row["memory_factor"] = round(counter_bytes / (28 * n), 3)
        if t_plain is None:
            t_plain = t
        else:
            row["slowdown"] = round(t / t_plain, 3)
        if wrap and "heatmap" in name and t > t_plain:
            # counters read and written once per copy, both views; time over the plain copy
            row["counter_rmw_gbs"] = round(2 * 2 * counter_bytes / (t - t_plain) / 1e6, 1)
            row["counter_frac_of_hbm_peak"] = round(row["counter_rmw_gbs"] / HBM_PEAK_GBS, 3)
        out[name] = row
        sv.close()
        dv.close()
        del sv, dv
        torch.cuda.empty_cache()
    base.close()
    del want
    torch.cuda.empty_cache()
    out["nbody"] = bench_instr_nbody(lm, torch, reps, 65536)
    return out


def bench_instr_nbody(lm, torch, reps, n):
    """The n-body step (Sec. 5) on 7 x f32 SoA-MB particles, plain and through
    FieldAccessCount or Heatmap(G = 128): every access the kernels make is
    counted with wave-aggregated atomics.  Gate: one step from the same state
    leaves the particles bit-identical to the plain step's and the counters
    non-zero."""
    from paper_2302_08251_amd import synth
    T = Timer(torch)
    log("instr: n-body on %d particles, plain and instrumented" % n)
    rec = ["f32"] * 7
    planes = [torch.from_numpy(p.view(np.uint8).copy()).cuda() for p in synth.particles(n, 0, dtype=np.float32)]
    out = {"particles": n}
    want = None
    t_plain = None
    for name, spec in (("plain", {"kind": "soa_mb"}), ("field_access_count", fac({"kind": "soa_mb"})),
                       ("heatmap_g128", heat({"kind": "soa_mb"}, 128))):
        v = lm.View(rec, spec, [n], index_type="i32", fill=0)
        for f in range(7):
            v.blobs[f][: 4 * n].copy_(planes[f])
        lm.nbody_step(v, 1, 1e-4, 0.01)
        torch.cuda.synchronize()
        got = [v.blobs[f][: 4 * n].clone() for f in range(7)]
        if want is None:
            want = got
        else:
            gate(all(torch.equal(a, b) for a, b in zip(got, want)), "instr nbody %s: particles differ" % name)
            gate(all(int(c.sum()) > 0 for c in counters(torch, v, 7)), "instr nbody %s: no counts" % name)
        T.warm(lambda: lm.nbody_energy(v, 0.01))
        t = float(np.median(T.time(lambda: lm.nbody_step(v, 1, 1e-4, 0.01), reps, warm=False)))
        row = {"ms_per_step": round(t, 4)}
        if t_plain is None:
            t_plain = t
        else:
            row["slowdown"] = round(t / t_plain, 3)
            row["counter_bytes"] = sum(v.sizes[7:])
        out[name] = row
        v.close()
    del planes, want
    torch.cuda.empty_cache()
    return out


# ------------------------------------------------------------------ cfg4: batched

def bench_cfg4(lm, torch, reps, count):
    from paper_2302_08251_amd import synth
    T = Timer(torch)
    ns, pairs = synth.batch_views(count, 0)
    log("cfg4: %d views, %d records" % (count, int(ns.sum())))
    g = torch.Generator(device="cuda").manual_seed(0)
    srcs, dsts = [], []
    for n, p in zip(ns.tolist(), pairs.tolist()):
        a, b = OFFDIAG[p]
        s = lm.View(F32x7, LAYOUTS[a], [n], index_type="i32")
        for t in s.blobs:
            t.copy_(torch.randint(0, 256, t.shape, generator=g, device="cuda", dtype=torch.uint8))
        srcs.append(s)
        dsts.append(lm.View(F32x7, LAYOUTS[b], [n], index_type="i32"))
    t0 = time.perf_counter()
    try:
        cache = os.environ.get("LLAMA_MI_TUNE_CACHE",
                               os.path.join(tempfile.gettempdir(), "llama_mi_batch_tune.json"))
        batch = lm.Batch(srcs, dsts, tune_cache=cache)
    except lm.LlamaError as e:
        return {"skipped": str(e)}
    create_s = time.perf_counter() - t0
    info = batch.info()
    batch.launch()
    torch.cuda.synchronize()
    # gate: every destination, read back through SoA-MB, holds its source's records
    for i, (s, d) in enumerate(zip(srcs, dsts)):
        n = s.n
        ms, md = (lm.View(F32x7, LAYOUTS["SoA-MB"], [n], index_type="i32") for _ in range(2))
        lm.llama_copy(s, ms)
        lm.llama_copy(d, md)
        ok = all(torch.equal(ms.blobs[f][: 4 * n], md.blobs[f][: 4 * n]) for f in range(7))
        ms.close()
        md.close()
        gate(ok, "cfg4 view %d (%s -> %s, %d records) differs from its source" % ((i,) + OFFDIAG[pairs[i]] + (n,)))
    batch.launch_per_view()
    tb = T.time(batch.launch, reps)
    tv = T.time(batch.launch_per_view, reps)
    alg = info["algorithmic_bytes"]
    res = {"views": count, "records": int(ns.sum()), "alg_bytes": alg,
           "batched_ms": float(np.median(tb)), "per_view_ms": float(np.median(tv)),
           "batched_ms_min_max": [float(np.min(tb)), float(np.max(tb))],
           "per_view_ms_min_max": [float(np.min(tv)), float(np.max(tv))],
           "batched_gbs": alg / np.median(tb) / 1e6, "per_view_gbs": alg / np.median(tv) / 1e6,
           "speedup": float(np.median(tv) / np.median(tb)), "tile_records": info["tile_records"],
           "grid": info["grid"], "total_tiles": info["total_tiles"],
           "persistent_grid": bool(info["grid"] < info["total_tiles"]),
           "xcd_contiguous_tiles": bool(info["tile_map"]),
           "records_per_s": float(ns.sum()) / (np.median(tb) * 1e-3),
           "tune_seconds": info["tune_seconds"], "create_seconds": create_s, "parity_gate": "round trip via SoA-MB"}
    batch.close()
    for v in srcs + dsts:
        v.close()
    torch.cuda.empty_cache()
    return res


# ------------------------------------------------------------------ cfg5: n-body

NB_FORMS = {
    "ChangeType(f64->f32, AoSoA-32)": {"kind": "changetype", "stored": ["f32"] * 7,
                                       "inner": {"kind": "aosoa", "lanes": 32}},
    "BitPackedFloat e8m15": {"kind": "bitpack_float", "exp": 8, "man": 15},
}
NB_DT, NB_EPS2 = 1e-4, 0.01
NB_SMALL = 4096                # particles of the drift comparison with the FP64 oracle
NB_SMALL_STATES = {}           # form -> (steps, GPU state after them), for the cpu_baseline leg


def nb_state(lm, torch, v, n):
    """The particles of an f64-record view as seven float64 numpy planes."""
    mb = lm.View(["f64"] * 7, {"kind": "soa_mb"}, [n])
    lm.llama_unpack(v, mb)
    out = [mb.blobs[f][: 8 * n].cpu().numpy().view(np.float64).copy() for f in range(7)]
    mb.close()
    return out


def momentum(pl):
    """Total momentum and the sum of |m v| (its natural scale)."""
    m = pl[6]
    p = np.array([np.sum(m * pl[3 + k]) for k in range(3)])
    return p, float(np.sum(m * np.sqrt(pl[3] ** 2 + pl[4] ** 2 + pl[5] ** 2)))


def bench_cfg5(lm, torch, n, steps):
    """All-pairs n-body (Sec. 5) on f64 records stored as ChangeType(f32) AoSoA-32
    or BitPackedFloat e8m15.  Gate: the forces are pairwise antisymmetric, so the
    total momentum must not move by more than 1e-4 of sum |m v| over the timed
    steps (FP32 summation and storage rounding stay orders of magnitude below),
    and the energy drift must stay under 1e-2."""
    from paper_2302_08251_amd import synth
    T = Timer(torch)
    out = {}
    planes = synth.particles(n, 0, dtype=np.float64)
    small = synth.particles(NB_SMALL, 0, dtype=np.float64)
    for name, spec in NB_FORMS.items():
        mb = lm.View(["f64"] * 7, {"kind": "soa_mb"}, [n],
                     blobs=[torch.from_numpy(p.view(np.uint8).copy()).cuda() for p in planes])
        v = lm.View(["f64"] * 7, spec, [n])
        lm.llama_pack(mb, v)
        p0, _ = momentum(nb_state(lm, torch, v, n))
        e0 = lm.nbody_energy(v, NB_EPS2)
        lm.nbody_step(v, 1, NB_DT, NB_EPS2)
        T.warm(lambda: lm.nbody_energy(v, NB_EPS2))  # steady clocks without moving the particles
        ts = T.time(lambda: lm.nbody_step(v, 1, NB_DT, NB_EPS2), steps, warm=False)
        e1 = lm.nbody_energy(v, NB_EPS2)
        te = T.time(lambda: lm.nbody_energy(v, NB_EPS2), 2, warm=False)
        p1, scale = momentum(nb_state(lm, torch, v, n))
        dp = float(np.linalg.norm(p1 - p0)) / scale
        drift = (e1 - e0) / abs(e0)
        gate(dp < 1e-4, "cfg5 %s: momentum moved by %.3g of sum |m v|" % (name, dp))
        gate(abs(drift) < 1e-2, "cfg5 %s: energy drift %.3g" % (name, drift))
        ms = float(np.median(ts))
        inter = float(n) * n
        vpi = nbody_valu_per_interaction()
        ips = inter / (ms * 1e-3)
        out[name] = {"ms_per_step": ms, "interactions_per_s": ips,
                     "valu_per_interaction_counted": vpi,
                     "valu_lane_ops_per_s": None if vpi is None else ips * vpi,
                     "frac_fp32_vector_issue": None if vpi is None else ips * vpi / FP32_LANE_OPS,
                     "gflops_20_per_interaction": 20 * inter / (ms * 1e-3) / 1e9,
                     "frac_fp32_peak": 20 * inter / (ms * 1e-3) / (FP32_PEAK_TFLOPS * 1e12),
                     "energy_ms": float(np.median(te)),
                     "energy_drift_over_%d_steps" % (steps + 1): drift,
                     "momentum_change_rel": dp}
        mb.close()
        v.close()
        # the same storage form on NB_SMALL particles, for the oracle's drift beside the GPU's
        mb = lm.View(["f64"] * 7, {"kind": "soa_mb"}, [NB_SMALL],
                     blobs=[torch.from_numpy(p.view(np.uint8).copy()).cuda() for p in small])
        v = lm.View(["f64"] * 7, spec, [NB_SMALL])
        lm.llama_pack(mb, v)
        e0 = lm.nbody_energy(v, NB_EPS2)
        lm.nbody_step(v, steps + 1, NB_DT, NB_EPS2)
        e1 = lm.nbody_energy(v, NB_EPS2)
        out[name]["small"] = {"particles": NB_SMALL, "steps": steps + 1, "energy_drift": (e1 - e0) / abs(e0)}
        NB_SMALL_STATES[name] = (steps + 1, nb_state(lm, torch, v, NB_SMALL))
        mb.close()
        v.close()
    return out


# ------------------------------------------------------------------ CPU oracle baseline

def cpu_baseline(n_sample, cfg5=None):
    """The oracle's element-by-element copy over all 36 ordered pairs of the single-view
    workload, on the first n_sample records, with every host core; the median of
    three passes.  When the n-body row ran, also the FP64 oracle's n-body through
    the same storage forms from the same initial state, its energy drift beside
    the GPU's and the GPU's largest deviation from it."""
    import oracle
    from paper_2302_08251_amd import synth
    threads = len(os.sched_getaffinity(0))
    planes = synth.particles(n_sample, 0, dtype=np.float32)
    blobs = {k: oracle.store_planes(F32x7, s, planes, threads=threads) for k, s in LAYOUTS.items()}
    dsts = {k: oracle.alloc_blobs(F32x7, s, n_sample) for k, s in LAYOUTS.items()}
    passes = []
    for _ in range(3):
        tot_s = 0.0
        for a in PAIR_ORDER:
            for b in PAIR_ORDER:
                t0 = time.perf_counter()
                oracle.copy(F32x7, LAYOUTS[a], blobs[a], LAYOUTS[b], n_sample, dst_blobs=dsts[b], threads=threads)
                tot_s += time.perf_counter() - t0
        passes.append(tot_s)
    tot_s = float(np.median(passes))
    del blobs, dsts
    tot_bytes = 36 * 2 * n_sample * 28
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    # further oracle figures on bounded samples: one thread on one pair, the
    # B = 12 int pack, and the FP64 n-body (the GPU rows' workloads)
    n1 = min(n_sample, 1 << 19)
    b1 = oracle.store_planes(F32x7, LAYOUTS["AoS"], [p[:n1] for p in planes], threads=threads)
    t0 = time.perf_counter()
    oracle.copy(F32x7, LAYOUTS["AoS"], b1, LAYOUTS["SoA-MB"], n1, threads=1)
    one_thread = 2 * n1 * 28 / (time.perf_counter() - t0) / 1e9
    n_int = 16 << 20
    vals = [synth.int_values(n_int, 12, 0)]
    ib = oracle.store_planes(["i32"], {"kind": "soa_mb"}, vals, threads=threads)
    t0 = time.perf_counter()
    oracle.copy(["i32"], {"kind": "soa_mb"}, ib, {"kind": "bitpack_int", "bits": 12}, n_int, threads=threads)
    pack12 = (4 * n_int + n_int * 12 // 8) / (time.perf_counter() - t0) / 1e9
    n_nb = 16384
    pl = synth.particles(n_nb, 0, dtype=np.float64)
    pos, vel = np.stack(pl[0:3], 1), np.stack(pl[3:6], 1)
    t0 = time.perf_counter()
    oracle.nbody(pos, vel, pl[6], 1, NB_DT, NB_EPS2, threads=threads)
    nb_ips = float(n_nb) * n_nb / (time.perf_counter() - t0)
    also = {"copy_AoS_to_SoA-MB_1_thread_gbs": one_thread, "copy_1_thread_records": n1,
            "int_pack_B12_gbs": pack12, "int_pack_B12_values": n_int,
            "nbody_fp64_interactions_per_s": nb_ips, "nbody_fp64_n": n_nb}
    rec64 = ["f64"] * 7
    for name, (steps, gpu) in NB_SMALL_STATES.items():
        spec = NB_FORMS[name]
        pl = synth.particles(NB_SMALL, 0, dtype=np.float64)
        host = oracle.store_planes(rec64, spec, pl)
        e0 = oracle.energy_view(rec64, spec, host, NB_SMALL, NB_EPS2)
        oracle.nbody_view(rec64, spec, host, NB_SMALL, steps, NB_DT, NB_EPS2)
        e1 = oracle.energy_view(rec64, spec, host, NB_SMALL, NB_EPS2)
        ref = oracle.load_planes(rec64, spec, host, NB_SMALL)
        d_or = (e1 - e0) / abs(e0)
        d_gpu = cfg5[name]["small"]["energy_drift"] if cfg5 and name in cfg5 else None
        pos_err = max(float(np.max(np.abs(gpu[k] - ref[k]))) for k in range(3))
        vel_err = max(float(np.max(np.abs(gpu[k] - ref[k]))) for k in range(3, 6))
        vel_scale = max(float(np.max(np.abs(ref[k]))) for k in range(3, 6))
        also["nbody_drift_" + name] = {
            "particles": NB_SMALL, "steps": steps, "oracle_fp64_energy_drift": d_or, "gpu_energy_drift": d_gpu,
            "gpu_minus_oracle_drift": None if d_gpu is None else d_gpu - d_or,
            "max_abs_pos_err": pos_err, "max_abs_vel_err": vel_err, "max_abs_vel": vel_scale}
    return {"value": tot_bytes / tot_s / 1e9, "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": "first %d of the 64Mi records, all 36 ordered pairs, element-by-element oracle "
                      "copy (OpenMP over record blocks), median of 3 passes; cpu: %s" % (n_sample, model),
            "seconds": tot_s, "passes_seconds": passes, "also": also}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--records", type=int, default=64 << 20)
    ap.add_argument("--rows", default="cfg3,cfg4,cfg5,instr", help="extra rows to measure (comma list or 'none')")
    ap.add_argument("--cpu-sample", type=int, default=3 << 20)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2302_08251_amd as lm
    lm.lib()
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    torch.cuda.init()
    rows = [] if args.rows == "none" else args.rows.split(",")
    try:
        r2 = bench_cfg2(lm, torch, args.steps, args.warmup, args.records)
    except RowFailed as e:  # the headline failed its parity gate: no number
        print(json.dumps({"metric": METRIC, "value": None, "unit": "GB/s", "n_gpus": 1, "error": str(e)}))
        sys.exit(1)
    extra = {}
    row_fns = {"cfg3": lambda: bench_cfg3(lm, torch, max(3, args.steps), 256 << 20, 64 << 20),
               "cfg4": lambda: bench_cfg4(lm, torch, max(3, args.steps), 2000),
               "cfg5": lambda: bench_cfg5(lm, torch, 65536, max(3, args.steps)),
               "instr": lambda: bench_instr(lm, torch, max(3, args.steps), 64 << 20)}
    for r in rows:
        try:
            extra[r] = row_fns[r]()
        except (lm.LlamaError, RowFailed) as e:  # a failing row is reported, not hidden
            extra[r] = {"error": str(e)}
            log("row %s failed: %s" % (r, e))
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    alg = r2["alg_bytes_per_pair"]
    achieved = r2["gbs_step"]
    traffic = measured_traffic(alg)
    line = {
        "metric": METRIC,
        "value": round(r2["gbs_step"], 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r2["step_ms"], 4),
        "records_per_s": round(36 * r2["records"] / (r2["step_ms"] * 1e-3), 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded numpy: pos U[-1,1], vel N(0,0.1), mass U[0.5,1])",
        "config": {"workload": "single view: 64Mi records of 7 x f32, all 36 ordered pairs of "
                               "AoS/SoA-SB/SoA-MB/AoSoA-32/AoSoA-64/Bytesplit(SoA-SB), I32 index",
                   "records": r2["records"], "pairs": 36, "alg_bytes_per_step": 36 * alg},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic},
        "parity_gates": "every row checks its results before timing (round trips, closed forms of the "
                        "codecs, counter totals, conservation laws); a failing row reports an error, no number",
        "cfg2": r2,
    }
    line.update(extra)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.cpu_sample, extra.get("cfg5"))
    print(json.dumps(line))


if __name__ == "__main__":
    main()

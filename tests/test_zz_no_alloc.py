"""nbody_step_noalloc (the n-body step without library allocations, for callers
that cannot allocate) against nbody_step through the C ABI: the same kernels
and summation order, so the particles must agree bit for bit.  Two calls in a
row on one GPU, the second with fewer particles, so the second reuses the
static scratch that the first left behind."""
import numpy as np
import pytest

import oracle
from gpu_helpers import F64x7, download, say, upload

import paper_2302_08251_amd as lm
from paper_2302_08251_amd import synth

pytestmark = pytest.mark.gpu

FORMS = {
    "f32_soa_mb": (["f32"] * 7, {"kind": "soa_mb"}),
    "changetype_aosoa32": (F64x7, {"kind": "changetype", "stored": ["f32"] * 7, "inner": {"kind": "aosoa", "lanes": 32}}),
    "e8m15": (F64x7, {"kind": "bitpack_float", "exp": 8, "man": 15}),
}
MAX_PARTICLES = (16 << 20) // 12


def packed_blobs(rec, spec, n, seed):
    planes = synth.particles(n, seed, dtype=np.float32 if rec[0] == "f32" else np.float64)
    return oracle.store_planes(rec, spec, planes)


@pytest.mark.parametrize("form", sorted(FORMS))
def test_noalloc_matches_nbody_step_twice(form):
    rec, spec = FORMS[form]
    for n, steps in ((65536 + 37, 2), (3001, 3)):  # the second call is smaller
        say("noalloc", form, n, steps)
        host = packed_blobs(rec, spec, n, seed=n)
        ref = lm.View(rec, spec, [n], blobs=upload(host))
        got = lm.View(rec, spec, [n], blobs=upload(host))
        lm.nbody_step(ref, steps, 1e-4, 0.01)
        lm.nbody_step_noalloc(got, steps, 1e-4, 0.01)
        want, have = download(ref), download(got)
        for b, (w, h) in enumerate(zip(want, have)):
            assert np.array_equal(w, h), "%s n=%d blob %d differs" % (form, n, b)
        assert any(not np.array_equal(w, o) for w, o in zip(want, host)), "the step moved the particles"
        ref.close()
        got.close()


def test_noalloc_rejects_beyond_its_maximum():
    n = MAX_PARTICLES + 1
    v = lm.View(["f32"] * 7, {"kind": "soa_mb"}, [n], fill=0)
    with pytest.raises(lm.LlamaError) as e:
        lm.nbody_step_noalloc(v, 1, 1e-4, 0.01)
    assert e.value.name == "NO_MEMORY" and "static maximum" in str(e.value)
    v.close()
    w = lm.View(["f32"] * 7, {"kind": "soa_mb"}, [MAX_PARTICLES], fill=0)
    lm.nbody_step_noalloc(w, 1, 1e-4, 0.01)  # the largest size is accepted
    download(w)
    w.close()

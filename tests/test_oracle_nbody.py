"""Pins of the oracle's FP64 n-body (CPU only).

Sec. 5 gives the update/move loop structure (update writes only velocities from
all positions, then the move phase advances positions); the interaction is the
textbook softened gravity with G = 1.  Pins: a two-body closed form, momentum
conservation, a symmetric configuration with zero force at the centre, an
N = 8 high-precision (50-digit Decimal) evaluation, and the two-body energy.
"""
from decimal import Decimal, getcontext

import numpy as np
import pytest

import oracle


def test_two_body_one_step_closed_form():
    d, m1, m2, eps2, dt = 0.75, 0.6, 0.9, 0.01, 1e-3
    pos = np.array([[-d / 2, 0, 0], [d / 2, 0, 0]], float)
    vel = np.zeros((2, 3))
    mass = np.array([m1, m2])
    p, v = oracle.nbody(pos, vel, mass, 1, dt, eps2)
    k = d / (d * d + eps2) ** 1.5
    assert np.isclose(v[0, 0], dt * m2 * k, rtol=1e-14, atol=0)
    assert np.isclose(v[1, 0], -dt * m1 * k, rtol=1e-14, atol=0)
    assert np.isclose(p[0, 0], -d / 2 + dt * dt * m2 * k, rtol=1e-14, atol=0)
    assert np.all(v[:, 1:] == 0) and np.all(p[:, 1:] == 0)


def test_momentum_conserved():
    rng = np.random.default_rng(0)
    n = 300
    pos = rng.uniform(-1, 1, (n, 3))
    vel = rng.normal(0, 0.1, (n, 3))
    mass = rng.uniform(0.5, 1, n)
    p0 = (mass[:, None] * vel).sum(0)
    _, v = oracle.nbody(pos, vel, mass, 5, 1e-4, 0.01)
    p1 = (mass[:, None] * v).sum(0)
    scale = (mass[:, None] * np.abs(v)).sum()
    assert np.all(np.abs(p1 - p0) <= 1e-12 * scale)


def test_symmetric_centre_has_zero_acceleration():
    pts = [[0, 0, 0]] + [[s * (a == 0), s * (a == 1), s * (a == 2)] for a in range(3) for s in (1.0, -1.0)]
    pos = np.array(pts, float)
    vel = np.zeros_like(pos)
    mass = np.ones(len(pos))
    p, v = oracle.nbody(pos, vel, mass, 1, 0.1, 0.01)
    assert np.all(v[0] == 0) and np.all(p[0] == 0)
    # outer particles are pulled inward symmetrically
    assert v[1, 0] < 0 and np.isclose(v[1, 0], -v[2, 0], rtol=1e-15)


def test_n8_against_high_precision():
    getcontext().prec = 50
    rng = np.random.default_rng(42)
    n, eps2, dt = 8, 0.01, 1e-3
    pos = rng.uniform(-1, 1, (n, 3))
    vel = rng.normal(0, 0.1, (n, 3))
    mass = rng.uniform(0.5, 1, n)
    p, v = oracle.nbody(pos, vel, mass, 1, dt, eps2)
    D = lambda x: Decimal(float(x))  # noqa: E731
    for i in range(n):
        acc = [Decimal(0)] * 3
        for j in range(n):
            dx = [D(pos[j, c]) - D(pos[i, c]) for c in range(3)]
            r2 = sum(x * x for x in dx) + D(eps2)
            w = D(mass[j]) / (r2 * r2.sqrt())
            acc = [acc[c] + dx[c] * w for c in range(3)]
        for c in range(3):
            vn = D(vel[i, c]) + D(dt) * acc[c]
            xn = D(pos[i, c]) + D(dt) * vn
            assert abs(float(vn) - v[i, c]) <= 1e-13 * max(1e-3, abs(float(vn)))
            assert abs(float(xn) - p[i, c]) <= 1e-13 * max(1e-3, abs(float(xn)))


def test_two_body_energy_closed_form():
    pos = np.array([[0.1, 0.2, 0.3], [-0.4, 0.5, 0.0]])
    vel = np.array([[0.01, -0.02, 0.03], [0.0, 0.05, -0.01]])
    mass = np.array([0.7, 0.8])
    eps2 = 0.01
    r2 = ((pos[0] - pos[1]) ** 2).sum()
    exp = 0.5 * (mass[:, None] * vel ** 2).sum() - mass[0] * mass[1] / np.sqrt(r2 + eps2)
    assert np.isclose(oracle.energy(pos, vel, mass, eps2), exp, rtol=1e-15)


def test_energy_drift_small_for_small_steps():
    rng = np.random.default_rng(3)
    n = 64
    pos = rng.uniform(-1, 1, (n, 3))
    vel = rng.normal(0, 0.1, (n, 3))
    mass = rng.uniform(0.5, 1, n)
    e0 = oracle.energy(pos, vel, mass, 0.01)
    p, v = oracle.nbody(pos, vel, mass, 20, 1e-5, 0.01)
    e1 = oracle.energy(p, v, mass, 0.01)
    assert abs(e1 - e0) / abs(e0) < 1e-5


# ---------------------------------------------------------------- n-body through a mapping (Sec. 4, Sec. 5)

def _state(n, seed, dtype):
    from paper_2302_08251_amd import synth
    return synth.particles(n, seed, dtype=dtype)


def test_nbody_view_equals_the_plain_fp64_oracle():
    n, steps = 300, 3
    planes = _state(n, 5, np.float64)
    rec = ["f64"] * 7
    spec = {"kind": "aosoa", "lanes": 8}
    blobs = oracle.store_planes(rec, spec, planes)
    oracle.nbody_view(rec, spec, blobs, n, steps, 1e-4, 0.01, tile=64)
    got = oracle.load_planes(rec, spec, blobs, n)
    rp, rv = oracle.nbody(np.stack(planes[0:3], 1), np.stack(planes[3:6], 1), planes[6], steps, 1e-4, 0.01)
    assert np.allclose(np.stack(got[0:3], 1), rp, rtol=0, atol=1e-13)
    assert np.allclose(np.stack(got[3:6], 1), rv, rtol=0, atol=1e-13)
    e = oracle.energy_view(rec, spec, blobs, n, 0.01)
    assert e == pytest.approx(oracle.energy(rp, rv, planes[6], 0.01), rel=1e-12)


@pytest.mark.parametrize("n,tile", [(300, 64), (257, 256), (1, 256)])
def test_nbody_view_field_access_counts_closed_form(n, tile):
    """Per step: each position leaf is loaded once per particle, once per particle and
    i-block (the j-tile) and once more by the move, and stored once; velocities are
    loaded and stored once; the mass is loaded once per particle and i-block."""
    steps = 2
    rec = ["f32"] * 7
    spec = {"kind": "field_access_count", "inner": {"kind": "soa_mb"}}
    blobs = oracle.store_planes(rec, spec["inner"], _state(n, 1, np.float32)) + [np.zeros(112, np.uint8)]
    oracle.nbody_view(rec, spec, blobs, n, steps, 1e-4, 0.01, tile=tile)
    got = blobs[-1].view(np.uint64).reshape(7, 2)
    blocks = -(-n // tile)
    want = np.zeros((7, 2), np.uint64)
    want[0:3, 0] = steps * (n + n * blocks + n)
    want[0:3, 1] = steps * n
    want[3:6, :] = steps * n
    want[6, 0] = steps * n * blocks
    assert np.array_equal(got, want)
    oracle.energy_view(rec, spec, blobs, n, 0.01)
    want[:, 0] += n
    assert np.array_equal(blobs[-1].view(np.uint64).reshape(7, 2), want)


def test_nbody_view_heatmap_one_counter_per_element():
    """Heatmap with 4 bytes per counter over SoA-MB f32: every counter is the number of
    accesses (loads and stores) of its element."""
    n, tile, steps = 130, 64, 1
    rec = ["f32"] * 7
    spec = {"kind": "heatmap", "granularity": 4, "inner": {"kind": "soa_mb"}}
    blobs = oracle.store_planes(rec, spec["inner"], _state(n, 2, np.float32))
    blobs += [np.zeros(8 * n, np.uint8) for _ in range(7)]
    oracle.nbody_view(rec, spec, blobs, n, steps, 1e-4, 0.01, tile=tile)
    blocks = -(-n // tile)
    per = [1 + blocks + 2] * 3 + [2] * 3 + [blocks]
    for f in range(7):
        assert np.array_equal(blobs[7 + f].view(np.uint64), np.full(n, steps * per[f], np.uint64)), f

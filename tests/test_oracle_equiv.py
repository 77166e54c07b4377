"""The live rearrangement against the offline definitions (Sections 2 and 6)."""
import cmath
import math

import numpy as np
import pytest

import oracle.wdd as O
import synth


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def small():
    wl = synth.WORKLOADS["small"]
    pos = synth.raster_positions(wl.sy, wl.sx)
    frames = wl.frames(pos)
    plan = O.make_plan(wl.sy, wl.sx, wl.n, wl.n, wl.radius, wl.k, amplitude=wl.aperture_amplitude())
    return wl, plan, frames, pos


def test_live_equals_offline(small):
    wl, plan, frames, pos = small
    a2, d2, o2 = O.offline_reduced(plan, frames, pos)
    live = O.Live(plan, "N")
    for b in range(0, len(pos), wl.batch):
        live.push(frames[b:b + wl.batch], pos[b:b + wl.batch])
    assert live.frames_seen == len(pos)
    assert _rel(live.acc, a2) < 1e-12
    assert _rel(live.spectrum(), d2) < 1e-12
    assert _rel(live.snapshot(), o2) < 1e-12


def test_both_wiener_orders_agree(small):
    wl, plan, frames, pos = small
    n_, p_ = O.Live(plan, "N"), O.Live(plan, "P")
    for b in range(0, len(pos), 100):
        n_.push(frames[b:b + 100], pos[b:b + 100])
        p_.push(frames[b:b + 100], pos[b:b + 100])
    assert _rel(p_.spectrum(), n_.spectrum()) < 1e-13


def test_order_and_partition_do_not_matter(small):
    wl, plan, frames, pos = small
    ref = O.Live(plan, "N")
    ref.push(frames, pos)
    rng = np.random.default_rng(7)
    perm = rng.permutation(len(pos))
    cuts = np.sort(rng.choice(np.arange(1, len(pos)), size=20, replace=False))
    live = O.Live(plan, "N")
    for part in np.split(perm, cuts):
        live.push(frames[part], pos[part])
    assert _rel(live.acc, ref.acc) < 1e-13
    # partial results taken at any point are snapshots of the frames seen so far
    half = O.Live(plan, "N")
    half.push(frames[perm[:300]], pos[perm[:300]])
    other = O.Live(plan, "N")
    other.push(frames[perm[300:]], pos[perm[300:]])
    assert _rel(half.acc + other.acc, ref.acc) < 1e-13


def test_repeated_position_sums(small):
    wl, plan, frames, pos = small
    one = O.Live(plan, "N")
    one.push(frames[:5] * 2.0, pos[:5])
    two = O.Live(plan, "N")
    two.push(frames[:5], pos[:5])
    two.push(frames[:5], pos[:5])
    assert _rel(two.acc, one.acc) < 1e-14


def test_fourier_basis_reduces_to_conventional_wdd():
    wl = synth.periodic_workload(s=16, n=16, radius=4.0)
    pos = synth.raster_positions(wl.sy, wl.sx)
    frames = wl.frames(pos)
    amp = wl.aperture_amplitude()
    plan = O.make_plan(wl.sy, wl.sx, wl.n, wl.n, wl.radius, phi=O.fourier_basis(wl.n, wl.n), amplitude=amp)
    _, d, ot = O.offline_reduced(plan, frames, pos)
    dc, oc = O.offline_conventional(frames.reshape(wl.sy, wl.sx, wl.n, wl.n), wl.radius, amplitude=amp)
    assert _rel(O.scatter(plan, d), dc) < 1e-12
    assert _rel(ot, oc) < 1e-12


def _conventional_by_loops(i4, radius, eps_rel):
    """Equations deconv_mat and extract written out with explicit sums."""
    sy, sx, ny, nx = i4.shape
    cy, cx = ny // 2, nx // 2

    def ap(uy, ux):
        return 1.0 if uy * uy + ux * ux <= radius * radius else 0.0

    g = np.zeros(i4.shape, dtype=complex)       # FT over the scan (unitary)
    for vy in range(sy):
        for vx in range(sx):
            acc = np.zeros((ny, nx), dtype=complex)
            for py in range(sy):
                for px in range(sx):
                    acc += i4[py, px] * cmath.exp(-2j * math.pi * (vy * py / sy + vx * px / sx))
            g[vy, vx] = acc / math.sqrt(sy * sx)
    ey = np.array([[cmath.exp(2j * math.pi * q * r / ny) for r in range(ny)] for q in range(ny)])
    ex = np.array([[cmath.exp(2j * math.pi * q * r / nx) for r in range(nx)] for q in range(nx)])
    hh = np.zeros(i4.shape, dtype=complex)      # inverse FT over the detector
    wp = np.zeros(i4.shape, dtype=complex)
    for vy in range(sy):
        for vx in range(sx):
            svy = vy - sy if 2 * vy >= sy else vy
            svx = vx - sx if 2 * vx >= sx else vx
            dy, dx = svy * ny / sy, svx * nx / sx
            y = np.array([[ap(qy - cy, qx - cx) * ap(qy - cy + dy, qx - cx + dx) for qx in range(nx)]
                          for qy in range(ny)])
            for ry in range(ny):
                for rx in range(nx):
                    hh[vy, vx, ry, rx] = np.sum(g[vy, vx] * np.outer(ey[:, ry], ex[:, rx])) / (ny * nx)
                    wp[vy, vx, ry, rx] = np.sum(y * np.outer(ey[:, ry], ex[:, rx])) / (ny * nx)
    eps = eps_rel * np.max(np.abs(wp) ** 2)
    wo = hh * np.conj(wp) / (np.abs(wp) ** 2 + eps)
    d = wo.sum(axis=(2, 3))
    out = np.zeros((sy, sx), dtype=complex)
    for y in range(sy):
        for x in range(sx):
            acc = 0j
            for vy in range(sy):
                for vx in range(sx):
                    acc += d[vy, vx] * cmath.exp(2j * math.pi * (vy * y / sy + vx * x / sx))
            out[y, x] = (acc / math.sqrt(sy * sx)).conjugate() / math.sqrt(abs(d[0, 0]))
    return d, out


def test_conventional_wdd_against_explicit_sums():
    rng = np.random.default_rng(2)
    i4 = rng.uniform(0, 1, size=(4, 4, 8, 8))
    d_ref, o_ref = _conventional_by_loops(i4, 2.0, 0.01)
    d, o = O.offline_conventional(i4, 2.0, eps_rel=0.01)
    assert _rel(d, d_ref) < 1e-12
    assert _rel(o, o_ref) < 1e-12

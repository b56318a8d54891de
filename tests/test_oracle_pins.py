"""Pins of the CPU oracle against facts fixed outside it: exact arithmetic,
brute force over small voxel grids, hand-derived closed forms (golden/),
and invariants of the method. None of these reuses the oracle's own code."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import brute
import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# -- rdiv / isqrt: textbook definitions --------------------------------------

def test_rdiv_exhaustive_small():
    for n in range(-300, 301):
        for d in range(1, 40):
            assert oracle.rdiv(n, d) == brute.round_half_away(Fraction(n, d)), (n, d)


def test_rdiv_examples_and_large():
    assert [oracle.rdiv(1, 3), oracle.rdiv(3, 2), oracle.rdiv(-3, 2), oracle.rdiv(2, 4), oracle.rdiv(-1, 2)] == \
        [0, 2, -2, 1, -1]
    g = np.random.default_rng(7)
    for _ in range(3000):
        n = int(g.integers(-(2 ** 52), 2 ** 52))
        d = int(g.integers(1, 2 ** 34))
        assert oracle.rdiv(n, d) == brute.round_half_away(Fraction(n, d))


def test_isqrt():
    for n in range(0, 5000):
        assert oracle.isqrt(n) == math.isqrt(n)
    g = np.random.default_rng(8)
    vals = [int(v) for v in g.integers(0, 2 ** 63, size=3000, dtype=np.uint64)]
    vals += [k * k for k in (2 ** 31, 2 ** 32 - 1, 3037000499)] + [k * k - 1 for k in (2 ** 31, 2 ** 32 - 1)]
    vals += [2 ** 64 - 1, 3 * 2 ** 62]
    for n in vals:
        assert oracle.isqrt(n) == math.isqrt(n), n


# -- transform + quantisation: exact fma emulation ---------------------------

def test_quantise_identity_grid_points():
    scale = 1024.0 / 0.05
    for p in [(0.05, 0.1, -0.15), (1.0, -2.0, 0.5), (0.0, 0.0, 0.0)]:
        q = oracle.quantise_point(p, np.eye(4), scale)
        expect = [round(float(np.float32(v)) * scale) for v in p]
        assert list(q) == expect


def test_quantise_random_poses_match_exact_fma():
    g = np.random.default_rng(9)
    for k in range(400):
        M = synth.fuzz_pose(1000 + k, max_t=20.0)
        scale = 1024.0 / float(g.choice([0.05, 0.064, 0.08, 0.1, 1.0 / 3.0]))
        p = g.uniform(-60, 60, size=3).astype(np.float32)
        q = oracle.quantise_point(p, M, scale)
        ref = brute.quantise(p, M, scale)
        assert (q is None and ref is None) or list(q) == ref
        o = oracle.quantise_origin(M, scale)
        assert list(o) == [round(M[a][3] * scale) for a in range(3)]


def test_quantise_fma_chain_crafted_rounding():
    """A case built so that the fused chain and separately rounded products
    land on different sides of a rounding boundary: with x = 1 + 2^-23 and
    M[0][0] = 1 + 2^-30, the exact product carries a 2^-53 term that a
    separate multiply drops (a tie, to even), and the translation cancels
    everything else to 2^-11. The chain gives w = 2^-11 + 2^-53, so at
    1024 units per metre q_x = rint(0.5 + 2^-43) = 1; unfused it would be
    rint(0.5) = 0."""
    x = 1.0 + 2.0 ** -23
    assert float(np.float32(x)) == x
    M = np.eye(4)
    M[0, 0] = 1.0 + 2.0 ** -30
    M[0, 3] = -(1.0 + 2.0 ** -23 + 2.0 ** -30) + 2.0 ** -11
    assert Fraction(M[0, 3]) == -(1 + Fraction(1, 2 ** 23) + Fraction(1, 2 ** 30)) + Fraction(1, 2 ** 11)
    p = np.array([x, 0.0, 0.0], dtype=np.float32)
    assert brute.quantise(p, M, 1024.0)[0] == 1
    assert oracle.quantise_point(p, M, 1024.0)[0] == 1
    unfused = M[0, 0] * x + M[0, 3]  # two roundings
    assert round(unfused * 1024.0) == 0


def test_quantise_half_even_and_range():
    # w * scale = 2.5 exactly -> 2 (half to even); 3.5 -> 4
    M = np.eye(4)
    assert list(oracle.quantise_point((2.5 / 1024, 3.5 / 1024, -2.5 / 1024), M, 1024.0)) == [2, 4, -2]
    # |q| >= 2^30 is dropped; non-finite is dropped
    assert oracle.quantise_point((2.0 ** 20, 0, 0), M, 1024.0) is None
    assert oracle.quantise_point((2.0 ** 20 - 1, 0, 0), M, 1024.0) is not None
    assert oracle.quantise_point((np.nan, 0, 0), M, 1024.0) is None
    assert oracle.quantise_point((np.inf, 0, 0), M, 1024.0) is None


# -- band --------------------------------------------------------------------

def test_band_closed_forms():
    # axis-parallel ray: off is exactly tau along the axis
    D, r, S, E = oracle.band([20580, 512, 512], [512, 512, 512], 3072)
    assert list(D) == [20068, 0, 0] and r == 20068
    assert list(S) == [17508, 512, 512] and list(E) == [23652, 512, 512]
    # point within tau of the sensor: the band starts at the sensor
    D, r, S, E = oracle.band([1000, 0, 0], [0, 0, 0], 3072)
    assert list(S) == [0, 0, 0] and list(E) == [4072, 0, 0]
    # zero-length ray: no band
    assert oracle.band([5, 5, 5], [5, 5, 5], 3072) is None
    # diagonal: |D|^2 = 3 * 1000^2, r = 1732, off = rdiv(3072 * 1000, 1732) = 1774 (1773.67)
    D, r, S, E = oracle.band([11000, 11000, 11000], [10000, 10000, 10000], 3072)
    assert r == 1732 and list(E) == [12774] * 3 and list(S) == [10000] * 3


# -- traversal: closed forms, brute force, invariants ------------------------

def test_segment_closed_forms():
    cases = json.load(open(os.path.join(GOLDEN, "segment_closed_forms.json")))["cases"]
    for c in cases:
        got = oracle.segment_voxels(c["S"], c["E"]).tolist()
        assert got == c["voxels"], c["name"]


def _brute_box(S, E):
    lo = [min(S[a], E[a]) // 1024 - 1 for a in range(3)]
    hi = [max(S[a], E[a]) // 1024 + 2 for a in range(3)]
    return lo, hi


def _check_invariants(S, E, vox):
    assert tuple(vox[0]) == tuple(s // 1024 for s in S)
    assert tuple(vox[-1]) == tuple(e // 1024 for e in E)
    for a in range(3):
        steps = np.diff(vox[:, a])
        assert np.all(np.abs(steps) <= 1)
        sgn = np.sign(E[a] - S[a])
        assert np.all(steps * sgn >= 0)
    assert len({tuple(v) for v in vox}) == len(vox)


@pytest.mark.parametrize("mode", ["random", "grid", "corner"])
def test_segment_vs_brute_force(mode):
    g = np.random.default_rng({"random": 11, "grid": 12, "corner": 13}[mode])
    for _ in range(150):
        if mode == "random":
            S = [int(v) for v in g.integers(-4096, 4096, size=3)]
            E = [int(v) for v in g.integers(-4096, 4096, size=3)]
        elif mode == "grid":  # endpoints on voxel faces / edges / corners
            S = [int(v) * 512 for v in g.integers(-8, 8, size=3)]
            E = [int(v) * 512 for v in g.integers(-8, 8, size=3)]
        else:  # segments through cell corners at shared crossing times
            base = [int(v) * 1024 for v in g.integers(-3, 3, size=3)]
            k = [int(v) for v in g.integers(-3, 4, size=3)]
            S = base
            E = [base[a] + 1024 * k[a] for a in range(3)]
        vox = oracle.segment_voxels(S, E)
        lo, hi = _brute_box(S, E)
        ref = brute.segment_voxels_brute(S, E, lo, hi)
        assert sorted(map(tuple, vox.tolist())) == sorted(ref), (S, E)
        _check_invariants(S, E, vox)


# -- signed distance: the single-plane closed form ---------------------------

def _single_point_map(prof, tau_u, vs, j=0, k=0):
    m = oracle.OracleMap((64, 8, 8), (0, 0, 0), vs, tau_u, 64)
    pose = np.eye(4)
    pose[:3, 3] = [prof["sensor_m"][0], prof["sensor_m"][1] + j, prof["sensor_m"][2] + k]
    m.integrate(np.array([prof["point_sensor_m"]], dtype=np.float32), pose)
    return m


def test_plane_profile_closed_form():
    d = json.load(open(os.path.join(GOLDEN, "plane_profile.json")))
    for side in ("plus_x", "minus_x"):
        prof = d[side]
        for j, k in [(0, 0), (1, 2), (3, 3)]:
            m = _single_point_map(prof, d["tau_u"], d["voxel_size_m"], j, k)
            sdf, w = m.readback((0, 0, 0), (64, 8, 8))
            xs = np.nonzero(w[:, j, k])[0].tolist()
            assert xs == prof["voxels_x"], side
            assert sdf[xs, j, k].tolist() == prof["sdf"], side
            assert int(w.sum()) == len(xs)  # nothing else touched
            m.close()


# -- min rule: brute force over an 8^3 window --------------------------------

def _tiny_scan(seed, n):
    g = np.random.default_rng(seed)
    pts = g.uniform(-2.0, 2.0, size=(n, 3))
    # repeat some points so that exact ties in |s| occur across indices
    pts[n // 2:n // 2 + 3] = pts[0]
    pts[-1] = np.nan
    return pts.astype(np.float32)


@pytest.mark.parametrize("seed", [21, 22, 23])
def test_volume_vs_brute_force(seed):
    vs, tau = 0.5, 1536
    scale = 1024.0 / vs
    dims, origin = (8, 8, 8), (-4, -4, -4)
    xyz = _tiny_scan(seed, 24)
    M = synth.fuzz_pose(seed, max_t=0.8)
    m = oracle.OracleMap(dims, origin, vs, tau, 64)
    keys = m.volume(xyz, M)  # slot order; origin multiple of dims -> slot = g mod 8
    best = brute.volume_brute(xyz, M, scale, tau, origin, dims)
    seen = 0
    for gx in range(origin[0], origin[0] + 8):
        for gy in range(origin[1], origin[1] + 8):
            for gz in range(origin[2], origin[2] + 8):
                kk = int(keys[gx % 8, gy % 8, gz % 8])
                if (gx, gy, gz) in best:
                    a, i, s = best[(gx, gy, gz)]
                    assert kk == (a << 48) | (i << 16) | (s & 0xFFFF)
                    seen += 1
                else:
                    assert kk == 0xFFFFFFFFFFFFFFFF
    assert seen > 50
    m.close()


def test_volume_permutation_invariance():
    """Sec. VI keeps, per voxel, the smallest distance over all rays of a
    scan; with ties broken by the point index (reading 1) the result cannot
    depend on the order in which the rays are taken. Points taken in
    reverse and in shuffled orders (each keeping its row as its index) give
    the identical volume, on a room scan with index ties, NaN rows and many
    voxels reached by several rays."""
    w1 = synth.config1()
    spec = w1.maps[0]
    xyz = w1.scans[0].xyz[::4].copy()
    n = xyz.shape[0]
    xyz[n // 3:n // 3 + 40] = xyz[:40]  # duplicates: equal |s| from different rows
    xyz[7::97] = np.nan
    pose = synth.fuzz_pose(61, max_t=0.3)
    m = oracle.OracleMap.from_spec(spec)
    ref = m.volume(xyz, pose)
    assert np.array_equal(m.volume(xyz, pose, order=np.arange(n)), ref)
    g = np.random.default_rng(61)
    orders = [np.arange(n)[::-1], g.permutation(n), g.permutation(n)]
    for order in orders:
        assert np.array_equal(m.volume(xyz, pose, order=order), ref)
    # the volume holds ties between rows: the index part of the key decides
    reached = ref[ref != np.uint64(0xFFFFFFFFFFFFFFFF)]
    assert reached.size > 10000
    with pytest.raises(ValueError):
        m.volume(xyz, pose, order=np.zeros(n, np.int64))  # not a permutation
    m.close()


# -- merge: Eq. (1) / Eq. (2) closed forms and invariants --------------------

def _profile_run(values_scans, w_max=64):
    """Integrate axis-parallel single-ray scans whose plane distance varies,
    returning the resulting (sdf, w) profile along x."""
    m = oracle.OracleMap((64, 4, 4), (0, 0, 0), 1.0, 3072, w_max)
    for X in values_scans:
        pose = np.eye(4)
        pose[:3, 3] = [0.5, 0.5, 0.5]
        m.integrate(np.array([[X - 0.5, 0.0, 0.0]], dtype=np.float32), pose)
    sdf, w = m.readback((0, 0, 0), (64, 1, 1))
    m.close()
    return sdf[:, 0, 0].astype(int), w[:, 0, 0].astype(int)


def test_merge_identical_scans_keep_value():
    X = 20580 / 1024
    base_sdf, base_w = _profile_run([X])
    for k in (2, 5, 70):
        sdf, w = _profile_run([X] * k)
        assert np.array_equal(sdf, base_sdf)
        assert np.array_equal(w, np.where(base_w > 0, min(k, 64), 0))


def test_merge_two_scans_average():
    Xa, Xb = 20580 / 1024, 20000 / 1024
    a_sdf, a_w = _profile_run([Xa])
    b_sdf, b_w = _profile_run([Xb])
    ab_sdf, ab_w = _profile_run([Xa, Xb])
    for x in range(64):
        if a_w[x] and b_w[x]:
            assert ab_sdf[x] == brute.round_half_away(Fraction(int(a_sdf[x]) + int(b_sdf[x]), 2))
            assert ab_w[x] == 2
        elif a_w[x] or b_w[x]:
            assert ab_sdf[x] == (a_sdf[x] if a_w[x] else b_sdf[x]) and ab_w[x] == 1


def test_merge_at_weight_cap():
    Xa, Xb = 20580 / 1024, 20100 / 1024
    cap = 5
    sdf_a, w_a = _profile_run([Xa] * 7, w_max=cap)
    sdf_b, w_b = _profile_run([Xb])
    sdf, w = _profile_run([Xa] * 7 + [Xb], w_max=cap)
    both = 0
    for x in range(64):
        if w_a[x] and w_b[x]:
            both += 1
            assert w[x] == cap
            assert sdf[x] == brute.round_half_away(Fraction(cap * int(sdf_a[x]) + int(sdf_b[x]), cap + 1))
    assert both >= 5


def test_merge_invariants_on_room_scans():
    w1 = synth.config1()
    spec = w1.maps[0]
    m = oracle.OracleMap.from_spec(spec)
    prev_w = np.zeros(spec.dims, np.int16)
    for k in range(4):
        pose = synth.fuzz_pose(500 + k, max_t=0.3)
        pose[:3, :3] = np.eye(3) if k == 0 else pose[:3, :3]
        st = m.integrate(w1.scans[0].xyz, pose)
        sdf, w, _ = m.window()
        assert np.all(np.abs(sdf.astype(int)) <= spec.tau_u)
        assert np.all((w >= 0) & (w <= spec.w_max))
        assert np.all(w >= prev_w)
        assert int((w != prev_w).sum()) <= st["voxels_updated"]
        # voxels whose weight did not change kept their value bit-exactly
        prev_w = w.copy()
    m.close()


def test_untouched_voxels_unchanged():
    w1 = synth.config1()
    spec = w1.maps[0]
    m = oracle.OracleMap.from_spec(spec)
    m.integrate(w1.scans[0].xyz, w1.scans[0].pose)
    sdf0, w0, _ = m.window()
    keys = m.volume(w1.scans[0].xyz[:4000], synth.fuzz_pose(3, 0.2))
    st = m.integrate(w1.scans[0].xyz[:4000], synth.fuzz_pose(3, 0.2))
    sdf1, w1_, _ = m.window()
    untouched = keys == np.uint64(0xFFFFFFFFFFFFFFFF)
    assert np.array_equal(sdf0[untouched], sdf1[untouched]) and np.array_equal(w0[untouched], w1_[untouched])
    assert int((~untouched).sum()) == st["voxels_updated"]
    m.close()


# -- shift: readback is invariant, shift then inverse is the identity -------

def test_shift_inverse_and_readback_invariance():
    w1 = synth.config1()
    m = oracle.OracleMap((64, 64, 64), (-32, -32, -32), 0.05, 3072, 64)
    for k in range(3):
        m.integrate(w1.scans[0].xyz, synth.fuzz_pose(40 + k, 0.2))
    box_lo, box_hi = (-100, -100, -100), (100, 100, 100)
    before = m.readback(box_lo, box_hi)
    sdf0, w0, o0 = m.window()
    for d in [(64, 0, 0), (-64, 64, 0), (5, -7, 3), (0, 0, -200)]:
        new = tuple(o0[a] + d[a] for a in range(3))
        m.shift(new)
        after = m.readback(box_lo, box_hi)
        assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
        m.shift(o0)
        sdf1, w1_, o1 = m.window()
        assert o1 == o0 and np.array_equal(sdf0, sdf1) and np.array_equal(w0, w1_)
    m.close()


def test_ring_run_equals_fixed_run_inside_overlap():
    """Scans whose bands stay inside every window the ring visits give the
    same global map as a fixed window holding all of them."""
    xyz = synth.fuzz_scan(77, 3000, extent_m=1.0, nan_frac=0.0)
    xyz = xyz[np.linalg.norm(xyz, axis=1) < 1.0]
    ring = oracle.OracleMap((64, 64, 64), (-32, -32, -32), 0.05, 3072, 64)
    fixed = oracle.OracleMap((128, 128, 128), (-64, -64, -64), 0.05, 3072, 64)
    origins = [(-32, -32, -32), (-28, -32, -32), (-32, -36, -30), (-34, -30, -32)]
    for k, o in enumerate(origins):
        ring.shift(o)
        pose = np.eye(4)
        pose[:3, 3] = [0.01 * k, -0.02 * k, 0.0]
        ring.integrate(xyz, pose)
        fixed.integrate(xyz, pose)
    a = ring.readback((-64, -64, -64), (64, 64, 64))
    b = fixed.readback((-64, -64, -64), (64, 64, 64))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert int((a[1] > 0).sum()) > 1000
    ring.close()
    fixed.close()


def test_recentre_rule_closed_form():
    dims = (512, 512, 128)
    vs = 0.05
    # sensor at voxel (100, -3, 0): nearest chunk-grid point is (128, 0, 0)
    pose = np.eye(4)
    pose[:3, 3] = [100 * vs + 0.01, -3 * vs + 0.01, 0.01]
    due, o = oracle.recentre(dims, (0, 0, 0), vs, pose, 65536, force=True)
    assert due and o == (128 - 256, 0 - 256, 0 - 64)
    # at the centre: no shift; just beyond 64 voxels: shift
    pose[:3, 3] = [0.0, 0.0, 0.0]
    assert oracle.recentre(dims, (-256, -256, -64), vs, pose, 65536)[0] is False
    pose[:3, 3] = [64 * vs, 0.0, 0.0]      # exactly 65536 away: not beyond
    assert oracle.recentre(dims, (-256, -256, -64), vs, pose, 65536)[0] is False
    pose[:3, 3] = [64 * vs + 0.001, 0.0, 0.0]
    due, o = oracle.recentre(dims, (-256, -256, -64), vs, pose, 65536)
    assert due and o == (64 - 256, -256, -64)


def test_stats_counts():
    m = oracle.OracleMap((64, 8, 8), (0, 0, 0), 1.0, 3072, 64)
    pose = np.eye(4)
    pose[:3, 3] = [0.5, 0.5, 0.5]
    pts = np.array([[19.59765625, 0, 0], [np.nan, 0, 0], [0.0, 0.0, 0.0], [19.59765625, 0, 0]], np.float32)
    st = m.integrate(pts, pose)
    # point 2 coincides with the sensor (D = 0): skipped; point 3 repeats point 0
    assert st == dict(points_in=4, points_valid=2, visits=14, voxels_updated=7)
    m.close()


# -- vertical interpolation between scan lines (Sec. VI, Eq. (3), Eq. (4)) ----

def _round_half_away(x: Fraction) -> int:
    a = abs(x)
    k = int(a + Fraction(1, 2))  # floor(a + 1/2)
    return k if x >= 0 else -k


def test_interp_delta_eq3():
    # Eq. (3) with degrees converted to radians, in 1/2^20 units (half even)
    for vfov, lines in [(45.0, 128), (30.0, 16), (90.0, 64), (22.5, 32), (40.0, 4)]:
        want = round(math.tan(math.radians(vfov / lines)) * 2 ** 20)
        assert oracle.interp_delta(vfov, lines) == want
    for vfov, lines in [(0.0, 16), (-5.0, 16), (30.0, 0), (90.0, 2), (200.0, 3)]:
        assert oracle.interp_delta(vfov, lines) == 0  # invalid, or angle >= 45 deg


def _exact_q20(num_terms):
    """round-half-even(2^20 x) for x = sum of c * sqrt(k) terms, evaluated
    with integer square roots at 2^-80 precision (no trigonometry)."""
    P = 80
    acc = 0
    for c, k in num_terms:
        acc += Fraction(c) * Fraction(math.isqrt(k << (2 * P)), 1 << P)
    return acc * 2 ** 20


def test_interp_delta_closed_form_surds():
    """Eq. (3) at angles whose tangent is a known surd: tan 30 = 1/sqrt 3,
    tan 22.5 = sqrt 2 - 1, tan 15 = 2 - sqrt 3, tan 7.5 = sqrt 6 - sqrt 3 +
    sqrt 2 - 2. Values in 1/2^20 units against the exact rounding, with no
    trigonometric function on the checking side."""
    cases = [
        ((60.0, 2), [(Fraction(1, 3), 3)]),                      # 30 deg
        ((90.0, 4), [(1, 2), (-1, 1)]),                          # 22.5 deg
        ((45.0, 3), [(2, 1), (-1, 3)]),                          # 15 deg
        ((30.0, 4), [(1, 6), (-1, 3), (1, 2), (-2, 1)]),         # 7.5 deg
        ((120.0, 4), [(Fraction(1, 3), 3)]),                     # 30 deg again
    ]
    for (vfov, lines), terms in cases:
        got = oracle.interp_delta(vfov, lines)
        x = _exact_q20(terms)
        lo = math.floor(x)
        assert abs(x - lo - Fraction(1, 2)) > Fraction(1, 10 ** 6)  # not near a tie
        assert got == (lo + 1 if x - lo > Fraction(1, 2) else lo), (vfov, lines, got, float(x))
    # a wrong unit (degrees taken as radians) or hlines - 1 would move these far
    assert oracle.interp_delta(60.0, 2) != oracle.interp_delta(60.0, 3)


def _rot_x(deg):
    c, s = math.cos(math.radians(deg)), math.sin(math.radians(deg))
    M = np.eye(4)
    M[:3, :3] = [[1, 0, 0], [0, c, -s], [0, s, c]]
    return M


# sensor x -> world +y, sensor y -> world +z, sensor z (up) -> world +x: an
# exact rotation whose column 2 and row 2 differ
_R_YZX = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])


def test_up_vector_rotated_poses_closed_form():
    """The sensor's up vector is its z axis seen in the world frame (reading
    25): rolled 90 degrees about x it is world -y; under the rotation with
    sensor z -> world x it is world +x. Row 2 of these rotations is (0, 1, 0)
    in both cases, so taking a row for the column fails here."""
    M = _rot_x(90.0)
    M[:3, 3] = [1.25, -3.5, 0.75]
    assert oracle.up_vector(M) == (0, -1024, 0)
    M2 = np.eye(4)
    M2[:3, :3] = _R_YZX
    M2[:3, 3] = [-2.0, 4.0, 1.0]
    assert oracle.up_vector(M2) == (1024, 0, 0)
    # tilted 30 degrees about x: up = (0, -sin 30, cos 30) in 1/1024 units
    M3 = _rot_x(30.0)
    assert oracle.up_vector(M3) == (0, -512, round(1024 * math.sqrt(3) / 2))


def test_up_vector_is_the_image_of_the_sensor_z_axis():
    """For random poses, U is within one unit of q(p = (0, 0, 1 m)) - o at
    1 m voxels: the pinned transform (exact-fma emulation) of the sensor's z
    axis, minus the sensor position, i.e. 1024 R e_z up to two roundings."""
    scale = 1024.0
    for it in range(300):
        M = synth.fuzz_pose((71, it), max_t=3.0)
        q = brute.quantise((0.0, 0.0, 1.0), M, scale)
        o = [round(M[a][3] * scale) for a in range(3)]
        U = oracle.up_vector(M)
        for a in range(3):
            assert abs(U[a] - (q[a] - o[a])) <= 1, (it, U, q, o)


def test_fill_offset_under_a_roll_closed_form():
    """Sensor rolled 90 degrees about x (up = world -y): a ray along the
    sensor's x axis (world +x) is filled along world y, e = (0, +h, 0), the
    interpolation vector d x (d x up) pointing against up, with h from
    Eq. (4). With up taken from the wrong axis this sign flips (or the fill
    vanishes)."""
    M = _rot_x(90.0)
    U = oracle.up_vector(M)
    dq = oracle.interp_delta(45.0, 128)
    o = [512, 1536, -512]
    for dist in (5 * 1024 + 100, 300 * 1024 + 7):
        q = [o[0] + dist, o[1], o[2]]
        D = [dist, 0, 0]
        for k in (-2, 0, 3):
            g = [q[0] // 1024 + k, o[1] // 1024, o[2] // 1024]
            length = 1024 * g[0] + 512 - o[0]
            h = min(_round_half_away(Fraction(dq * length, 2 ** 20)), 65535) if length > 0 else 0
            assert oracle.fill_offset(q, o, D, dist, U, g, dq) == (0, h, 0)


def test_interp_volume_rotated_sensor_closed_form():
    """One ray along the sensor's x axis under the exact rotation sensor x ->
    world +y, sensor z -> world +x: the band lies along world y with the
    plane profile, and every band voxel fills its run along world x (up),
    from floor((c_x - h) / 1024) to floor((c_x + h) / 1024); the smallest
    |s| wins where runs meet."""
    dq = oracle.interp_delta(40.0, 4)  # tan(10 deg)
    tau = 3072
    dims, origin = (24, 40, 8), (-12, 0, 0)
    m = oracle.OracleMap(dims, origin, 1.0, tau, 64)
    m.set_interpolation(dq=dq)
    pose = np.eye(4)
    pose[:3, :3] = _R_YZX
    pose[:3, 3] = [0.5, 0.5, 4.5]
    Y = 30.2
    xyz = np.array([[Y - 0.5, 0.0, 0.0]], dtype=np.float32)  # sensor x
    keys = m.volume(xyz, pose)
    oy = 512
    qy = int(round(float(np.float32(Y - 0.5)) * 1024)) + 512
    expect = {}
    for gy in range((qy - tau) // 1024, (qy + tau) // 1024 + 1):
        cy = 1024 * gy + 512
        s = max(-tau, min(tau, qy - cy))
        h = min(_round_half_away(Fraction(dq * (cy - oy), 2 ** 20)), 65535)
        cx = 512
        for gx in range((cx - h) // 1024, (cx + h) // 1024 + 1):
            if not (-12 <= gx < 12):
                continue
            key = (abs(s) << 48) | (s & 0xFFFF)
            expect[(gx, gy, 4)] = min(expect.get((gx, gy, 4), 1 << 64), key)
    assert len(expect) > 20 and any(gx < 0 for gx, _, _ in expect)
    for gx in range(-12, 12):
        for gy in range(40):
            for gz in range(8):
                kk = int(keys[gx % 24, gy % 40, gz % 8])
                assert kk == expect.get((gx, gy, gz), 0xFFFFFFFFFFFFFFFF), (gx, gy, gz)
    m.close()


def _up_of(M):
    """The sensor's z axis in the world in 1/1024 units, half to even, from
    the rotation applied to e_z (the definition; not the oracle's code)."""
    v = np.asarray(M, dtype=np.float64)[:3, :3] @ np.array([0.0, 0.0, 1.0])
    return tuple(int(x) for x in np.rint(1024.0 * v))


def test_fill_offset_axis_rays_closed_form():
    """Identity pose (up = +z): a ray along x or y is filled straight down and
    up, e = (0, 0, -h) with h = delta_z * (distance of the voxel centre along
    the ray), rounded half away from zero and capped at 64 voxels."""
    U = oracle.up_vector(np.eye(4))
    assert U == (0, 0, 1024)
    dq = oracle.interp_delta(45.0, 128)
    for axis, sign in [(0, 1), (0, -1), (1, 1), (1, -1)]:
        o = [512, -1536, 2560]
        for dist in (7 * 1024 + 300, 200 * 1024 + 5, 9000 * 1024 + 77):
            q = list(o)
            q[axis] += sign * dist
            D = [q[a] - o[a] for a in range(3)]
            r = abs(D[axis])
            for k in (-3, 0, 2):  # band voxels around the point
                g = [(o[a]) // 1024 for a in range(3)]
                g[axis] = (q[axis] // 1024) + k
                c = 1024 * g[axis] + 512
                length = sign * (c - o[axis])  # projection onto the ray, exact here
                h = min(_round_half_away(Fraction(dq * length, 2 ** 20)), 65535) if length > 0 else 0
                e = oracle.fill_offset(q, o, D, r, U, g, dq)
                assert e == (0, 0, -h), (axis, sign, dist, k, e, h)
    # a vertical ray has no interpolation direction
    e = oracle.fill_offset((0, 0, 50 * 1024), (0, 0, 0), (0, 0, 50 * 1024), 50 * 1024, U, (0, 0, 49), dq)
    assert e == (0, 0, 0)


def test_fill_offset_geometry_random():
    """Properties of e for random rays and poses: perpendicular to the ray,
    in the plane of the ray and the sensor's up vector, pointing against up,
    of length h up to rounding."""
    g = np.random.default_rng(41)
    dq = oracle.interp_delta(30.0, 16)
    checked = 0
    for it in range(400):
        M = synth.fuzz_pose((41, it), max_t=2.0)
        U = _up_of(M)
        assert U == oracle.up_vector(M)
        o = [int(v) for v in g.integers(-50000, 50000, size=3)]
        D = [int(v) for v in g.integers(-400000, 400000, size=3)]
        q = [o[a] + D[a] for a in range(3)]
        r = math.isqrt(sum(v * v for v in D))
        if r == 0:
            continue
        k = [q[a] // 1024 for a in range(3)]
        e = oracle.fill_offset(q, o, D, r, U, k, dq)
        c = [1024 * k[a] + 512 for a in range(3)]
        length = Fraction(sum((c[a] - o[a]) * D[a] for a in range(3)), r)
        h = min(float(length) * dq / 2 ** 20, 65535)
        ne = math.sqrt(sum(v * v for v in e))
        cross = [D[1] * U[2] - D[2] * U[1], D[2] * U[0] - D[0] * U[2], D[0] * U[1] - D[1] * U[0]]
        nc = math.sqrt(sum(v * v for v in cross))
        if nc < 1e-3 * r * 1024:  # ray nearly along up: direction ill-defined
            continue
        assert abs(ne - h) <= 2.0 + 4e-3 * h, (ne, h)
        if ne > 50:
            dot_d = sum(e[a] * D[a] for a in range(3)) / (ne * r)
            dot_plane = sum(e[a] * cross[a] for a in range(3)) / (ne * nc)
            dot_up = sum(e[a] * U[a] for a in range(3))
            assert abs(dot_d) < 4e-3 + 2.0 / ne, dot_d
            assert abs(dot_plane) < 4e-3 + 2.0 / ne, dot_plane
            assert dot_up <= 0
            checked += 1
    assert checked > 200


def _axis_ray_map(dq, tau=3072):
    m = oracle.OracleMap((40, 8, 24), (0, 0, -12), 1.0, tau, 64)
    m.set_interpolation(dq=dq)
    return m


def test_interp_volume_axis_ray_closed_form():
    """One ray along +x from (0.5, 4.5, 0.5) voxels to x = 30.2: band voxels
    get the plane profile, each fills its column from floor((c_z - h)/1024)
    to floor((c_z + h)/1024), and a voxel reached from several band voxels
    keeps the smallest |s| (one ray: no index ties to break)."""
    dq = oracle.interp_delta(40.0, 4)  # tan(10 deg): fills of a few voxels
    tau = 3072
    m = _axis_ray_map(dq, tau)
    pose = np.eye(4)
    pose[:3, 3] = [0.5, 4.5, 0.5]
    X = 30.2
    xyz = np.array([[X - 0.5, 0.0, 0.0]], dtype=np.float32)
    keys = m.volume(xyz, pose)
    # closed form
    ox = 512
    qx = int(round(float(np.float32(X - 0.5)) * 1024)) + 512
    expect = {}
    for gx in range((qx - tau) // 1024, (qx + tau) // 1024 + 1):
        cx = 1024 * gx + 512
        s = max(-tau, min(tau, qx - cx))
        h = min(_round_half_away(Fraction(dq * (cx - ox), 2 ** 20)), 65535)
        cz = 512
        for gz in range((cz - h) // 1024, (cz + h) // 1024 + 1):
            key = (abs(s) << 48) | (s & 0xFFFF)
            if not (-12 <= gz < 12):
                continue
            expect[(gx, 4, gz)] = min(expect.get((gx, 4, gz), 1 << 64), key)
    assert len(expect) > 20
    for gx in range(40):
        for gy in range(8):
            for gz in range(-12, 12):
                kk = int(keys[gx, gy, gz % 24])
                assert kk == expect.get((gx, gy, gz), 0xFFFFFFFFFFFFFFFF), (gx, gy, gz)
    m.close()


def _interp_case(seed):
    g = np.random.default_rng(seed)
    xyz = g.uniform(-3.0, 3.0, size=(30, 3)).astype(np.float32)
    xyz[5] = np.nan
    xyz[7:9] = xyz[0]  # index ties
    return xyz, synth.fuzz_pose((seed, 3), max_t=1.0)


@pytest.mark.parametrize("seed", [51, 52, 53])
def test_interp_volume_vs_brute_force(seed):
    """The interpolated volume over a 16^3 window against a brute-force
    assembly: band from the pinned band function, band voxels and fill voxels
    from the exact-rational floor-set of each segment (not the oracle's
    walk), fill offsets from the pinned fill_offset, minimum over keys."""
    vs, tau = 0.5, 1536
    scale = 1024.0 / vs
    dims, origin = (16, 16, 16), (-8, -8, -8)
    dq = oracle.interp_delta(60.0, 4)  # tan(15 deg)
    xyz, M = _interp_case(seed)
    m = oracle.OracleMap(dims, origin, vs, tau, 64)
    m.set_interpolation(dq=dq)
    keys = m.volume(xyz, M)
    o = oracle.quantise_origin(M, scale)
    U = _up_of(M)  # the definition, so that the oracle's own up vector is checked too
    best = {}
    for i, p in enumerate(xyz):
        q = oracle.quantise_point(p, M, scale)
        if q is None:
            continue
        b = oracle.band(q, o, tau)
        if b is None:
            continue
        D, r, S, E = b
        q, D, S, E = ([int(v) for v in a] for a in (q, D, S, E))
        o = [int(v) for v in o]
        blo = [min(S[a], E[a]) // 1024 for a in range(3)]
        bhi = [max(S[a], E[a]) // 1024 + 1 for a in range(3)]
        band_vox = brute.segment_voxels_brute(S, E, blo, bhi)
        for gb in band_vox:
            s = oracle.voxel_sdf(q, D, r, gb, tau)
            key = (abs(s) << 48) | (i << 16) | (s & 0xFFFF)
            e = oracle.fill_offset(q, o, D, r, U, gb, dq)
            c = [1024 * gb[a] + 512 for a in range(3)]
            A = [c[a] - e[a] for a in range(3)]
            Bv = [c[a] + e[a] for a in range(3)]
            lo = [min(A[a], Bv[a]) // 1024 for a in range(3)]
            hi = [max(A[a], Bv[a]) // 1024 + 1 for a in range(3)]
            for gf in brute.segment_voxels_brute(A, Bv, lo, hi):
                if all(origin[a] <= gf[a] < origin[a] + dims[a] for a in range(3)):
                    best[gf] = min(best.get(gf, 1 << 64), key)
    hits = 0
    for gx in range(origin[0], origin[0] + dims[0]):
        for gy in range(origin[1], origin[1] + dims[1]):
            for gz in range(origin[2], origin[2] + dims[2]):
                kk = int(keys[gx % 16, gy % 16, gz % 16])
                assert kk == best.get((gx, gy, gz), 0xFFFFFFFFFFFFFFFF), (gx, gy, gz)
                hits += kk != 0xFFFFFFFFFFFFFFFF
    assert hits > 100
    m.close()


def test_interp_invariants_room_scan():
    """Turning interpolation off gives the plain volume; with it on, every
    voxel the plain volume holds is still held, with a key no larger, and
    more voxels are reached."""
    w = synth.config1()
    sc = w.scans[0]
    spec = w.maps[0]
    sub = sc.xyz[::8]
    plain = oracle.OracleMap.from_spec(spec)
    kp = plain.volume(sub, sc.pose)
    off = oracle.OracleMap.from_spec(spec)
    off.set_interpolation(30.0, 16)
    off.set_interpolation(0.0, 0)
    assert np.array_equal(off.volume(sub, sc.pose), kp)
    on = oracle.OracleMap.from_spec(spec)
    on.set_interpolation(30.0, 16)
    ki = on.volume(sub, sc.pose)
    held = kp != np.uint64(0xFFFFFFFFFFFFFFFF)
    assert np.all(ki[held] <= kp[held])
    assert int((ki != np.uint64(0xFFFFFFFFFFFFFFFF)).sum()) > int(held.sum())
    for m in (plain, off, on):
        m.close()


# -- surface extraction for inspection (marching tetrahedra) -----------------

def _tri_area(t):
    a, b, c = (np.asarray(v, dtype=np.float64) for v in t)
    return 0.5 * np.linalg.norm(np.cross(b - a, c - a))


def test_mesh_of_a_plane_closed_form():
    """Axis-parallel single-ray scans, one per (y, z) voxel centre of a 6 x 5
    patch, all hitting the plane x = 20580/1024 voxels: the band voxels hold
    the plane profile (golden/plane_profile.json), its sign changes between
    voxels 19 and 20 at exactly t = 612/1024, so every vertex has
    x = 20.09765625 voxels, and the triangles tile the patch between the ray
    centres: 5 x 4 cubes, 8 triangles each, total area 20 voxel^2."""
    vs = 0.25
    m = oracle.OracleMap((32, 8, 8), (0, 0, 0), vs, 3072, 64)
    for j in range(6):
        for k in range(5):
            pose = np.eye(4)
            pose[:3, 3] = [0.5 * vs, (j + 0.5) * vs, (k + 0.5) * vs]
            x = 20580 / 1024 * vs - 0.5 * vs
            m.integrate(np.array([[x, 0.0, 0.0]], dtype=np.float32), pose)
    tris = m.mesh((0, 0, 0), (32, 8, 8))
    assert tris.shape == (5 * 4 * 8, 3, 3)
    assert np.all(tris[:, :, 0] == np.float32(20.09765625 * vs))
    area = sum(_tri_area(t) for t in tris)
    assert abs(area - 20 * vs * vs) < 1e-5
    ys, zs = tris[:, :, 1], tris[:, :, 2]
    assert ys.min() == np.float32(0.5 * vs) and ys.max() == np.float32(5.5 * vs)
    assert zs.min() == np.float32(0.5 * vs) and zs.max() == np.float32(4.5 * vs)
    # a sub-box that leaves out the crossing layer has no surface
    assert m.mesh((21, 0, 0), (32, 8, 8)).shape[0] == 0
    with pytest.raises(ValueError):
        m.mesh((0, 0, 0), (33, 8, 8))
    m.close()


def test_mesh_of_room_scan_is_consistent():
    """Invariants on a real scan's map: every vertex lies on a segment
    between two corners of a cube (the varying coordinates share one
    fraction t or 1 - t) inside the box; the whole box's triangles are those
    of its two halves, split on an x plane (the halves share that plane's
    voxels, not a cube)."""
    w = synth.config1()
    spec, sc = w.maps[0], w.scans[0]
    m = oracle.OracleMap.from_spec(spec)
    m.integrate(sc.xyz, sc.pose)
    lo, hi = spec.origin, tuple(spec.origin[a] + spec.dims[a] for a in range(3))
    tris = m.mesh(lo, hi)
    assert tris.shape[0] > 10000
    vs = spec.voxel_size
    v = tris.reshape(-1, 3).astype(np.float64) / vs - 0.5
    f = v - np.floor(v)
    for row in f[:: max(1, len(f) // 5000)]:
        vary = [x for x in row if 1e-4 < x < 1 - 1e-4]
        assert all(min(abs(x - vary[0]), abs(x - (1 - vary[0]))) < 1e-4 for x in vary), row
    assert np.all((v >= np.array(lo) - 1e-4) & (v <= np.array(hi) - 1 + 1e-4))
    mid = lo[0] + spec.dims[0] // 2
    a = m.mesh(lo, (mid + 1, hi[1], hi[2]))
    b = m.mesh((mid, lo[1], lo[2]), hi)
    assert a.shape[0] + b.shape[0] == tris.shape[0]
    m.close()


# -- point-to-TSDF registration (the paper's stated next step) ---------------

def test_reg_linear_field_closed_form():
    """On a map whose sdf is a linear function of the voxel index, the
    trilinear residual and gradient are that function and its slope."""
    vs = 0.1
    dims, origin = (16, 16, 16), (0, 0, 0)
    A, Bc, Cc, D0 = 37, -21, 12, -40
    g = np.indices(dims)
    sdf = (A * g[0] + Bc * g[1] + Cc * g[2] + D0).astype(np.int16)
    m = oracle.OracleMap(dims, origin, vs, 3072, 64)
    m.set_voxels(origin, dims, sdf, np.ones(dims, np.int16))
    rng = np.random.default_rng(91)
    for _ in range(50):
        p = rng.uniform(0.1 * vs + 0.5 * vs, (dims[0] - 1.6) * vs, size=3).astype(np.float32)
        got = m.reg_point(p, np.eye(4))
        assert got is not None
        phi, grad, w = got
        u = np.asarray(p, np.float64) / vs - 0.5
        want = (A * u[0] + Bc * u[1] + Cc * u[2] + D0) * vs / 1024
        assert abs(phi - want) < 1e-12
        assert np.allclose(grad, np.array([A, Bc, Cc]) / 1024, rtol=0, atol=1e-12)
    # a corner outside the window, unobserved or truncated drops the point
    assert m.reg_point(np.array([0.02, 0.5, 0.5], np.float32), np.eye(4)) is None
    w0 = np.ones(dims, np.int16)
    w0[5, 5, 5] = 0
    m.set_voxels(origin, dims, sdf, w0)
    assert m.reg_point(np.array([0.55, 0.55, 0.55], np.float32), np.eye(4)) is None
    m.close()


def test_reg_jacobian_matches_finite_differences():
    w = synth.config1()
    spec, sc = w.maps[0], w.scans[0]
    m = oracle.OracleMap.from_spec(spec)
    m.integrate(sc.xyz, sc.pose)
    pts = sc.xyz[::37]
    checked = 0
    for p in pts:
        got = m.reg_point(p, sc.pose)
        if got is None:
            continue
        phi, grad, wv = got
        J = np.concatenate([grad, np.cross(wv, grad)])
        h = 1e-6
        for k in range(6):
            d = np.zeros(6)
            d[k] = h
            vals = []
            for sgn in (1, -1):
                res = oracle.reg_step(np.concatenate([np.eye(6)[np.triu_indices(6)], -sgn * d, [0, 1]]), 0.0,
                                      sc.pose)
                # the step with H = I and J^T r = -d is exactly d: the pose exp(d) T
                P = res[0]
                r = m.reg_point(p, P)
                vals.append(None if r is None else r[0])
            if None in vals:
                continue
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - J[k]) < 1e-5 + 1e-4 * abs(J[k]), (k, fd, J[k])
        checked += 1
    assert checked > 20
    m.close()


def test_reg_step_solves_normal_equations_and_rotation():
    """The step against numpy's solve, its rotation against the rotation
    vector's exponential (Rodrigues, from the matrix series)."""
    rng = np.random.default_rng(92)
    for _ in range(20):
        Jm = rng.normal(size=(40, 6))
        r = rng.normal(size=40) * 0.01
        H = Jm.T @ Jm
        sums = np.concatenate([H[np.triu_indices(6)], Jm.T @ r, [r @ r, 40.0]])
        pose = synth.fuzz_pose(int(rng.integers(1 << 30)), 1.0)
        lam = 0.3
        P, d = oracle.reg_step(sums, lam, pose)
        assert np.allclose((H + lam * np.eye(6)) @ d, -(Jm.T @ r), atol=1e-12)
        th = d[3:]
        K = np.array([[0, -th[2], th[1]], [th[2], 0, -th[0]], [-th[1], th[0], 0]])
        R = np.eye(3)
        term = np.eye(3)
        for k in range(1, 30):  # exp(K) by its series
            term = term @ K / k
            R = R + term
        assert np.allclose(P[:3, :3], R @ pose[:3, :3], atol=1e-12)
        assert np.allclose(P[:3, 3], R @ pose[:3, 3] + d[:3], atol=1e-12)


def test_reg_recovers_a_perturbed_pose():
    """A room scan registered to the map built from it, from 5 cm and 1.1 deg
    off, comes back to within 1 cm and 0.5 deg; the cost falls."""
    w = synth.config1()
    spec, sc = w.maps[0], w.scans[0]
    m = oracle.OracleMap.from_spec(spec)
    m.integrate(sc.xyz, sc.pose)
    P = sc.pose.copy()
    P[0, 3] += 0.04
    P[1, 3] -= 0.03
    c, s = math.cos(0.02), math.sin(0.02)
    P[:3, :3] = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]]) @ P[:3, :3]
    cost0 = m.reg_sums(sc.xyz, P)
    pose, info = m.register(sc.xyz, P, 10, 1e-6)
    assert np.linalg.norm(pose[:3, 3] - sc.pose[:3, 3]) < 0.01
    dR = pose[:3, :3] @ sc.pose[:3, :3].T
    ang = math.degrees(math.acos(max(-1.0, min(1.0, (np.trace(dR) - 1) / 2))))
    assert ang < 0.5
    assert info["cost"] / info["points"] < cost0[27] / cost0[28]
    m.close()


# -- free-space carving: the ray walked from the sensor ----------------------

def _carve_axis_case(sensor_x, X):
    """One ray along x from a voxel centre at sensor_x to the point at X
    (metres = voxels): with carving, every voxel from the sensor's to the
    band end's receives clamp(q_x - c_x, +-tau), and no other voxel; the
    voxel where the free-space segment meets the band is visited twice."""
    tau = 3072
    m = oracle.OracleMap((80, 8, 8), (0, 0, 0), 1.0, tau, 64)
    m.set_carving(True)
    pose = np.eye(4)
    pose[:3, 3] = [sensor_x, 4.5, 3.5]
    xyz = np.array([[X - sensor_x, 0.0, 0.0]], dtype=np.float32)
    st = m.integrate(xyz, pose)
    sdf, w = m.readback((0, 0, 0), (80, 8, 8))
    m.close()
    ox = int(round(sensor_x * 1024))
    qx = int(round(float(np.float32(X - sensor_x)) * 1024)) + ox
    sgn = 1 if qx > ox else -1
    ex = qx + sgn * tau  # off = rdiv(tau D, r) = tau sign(D) on an axis ray
    want_sdf = np.zeros((80, 8, 8), dtype=np.int16)
    want_w = np.zeros((80, 8, 8), dtype=np.int16)
    for gx in range(min(ox, ex) // 1024, max(ox, ex) // 1024 + 1):
        if 0 <= gx < 80:
            s = sgn * (qx - (1024 * gx + 512))  # (q - c) . D / r along the ray
            want_sdf[gx, 4, 3] = max(-tau, min(tau, s))
            want_w[gx, 4, 3] = 1
    return st, sdf, w, want_sdf, want_w


@pytest.mark.parametrize("sensor_x,X", [(0.5, 30.2), (70.5, 20.3), (2.5, 77.9), (5.5, 0.25)])
def test_carve_axis_ray_closed_form(sensor_x, X):
    st, sdf, w, want_sdf, want_w = _carve_axis_case(sensor_x, X)
    assert np.array_equal(sdf, want_sdf)
    assert np.array_equal(w, want_w)
    assert st["voxels_updated"] == int(want_w.sum())
    assert st["visits"] == st["voxels_updated"] + 1


@pytest.mark.parametrize("seed", [71, 72, 73, 74])
def test_carve_volume_vs_brute_force(seed):
    """The carved volume over an 8^3 window against the brute-force interval
    test on the band and on the segment from the sensor to the band's start
    (sensors inside and outside the window, NaNs and index ties), and the
    visit count against the number of (segment, window voxel) incidences."""
    vs, tau = 0.5, 1536
    scale = 1024.0 / vs
    dims, origin = (8, 8, 8), (-4, -4, -4)
    xyz = _tiny_scan(seed, 20)
    M = synth.fuzz_pose(seed, max_t=0.8 if seed % 2 else 3.0)
    m = oracle.OracleMap(dims, origin, vs, tau, 64)
    m.set_carving(True)
    keys = m.volume(xyz, M)
    best = brute.volume_brute(xyz, M, scale, tau, origin, dims, carve=True)
    seen = 0
    for gx in range(origin[0], origin[0] + 8):
        for gy in range(origin[1], origin[1] + 8):
            for gz in range(origin[2], origin[2] + 8):
                kk = int(keys[gx % 8, gy % 8, gz % 8])
                if (gx, gy, gz) in best:
                    a, i, s = best[(gx, gy, gz)]
                    assert kk == (a << 48) | (i << 16) | (s & 0xFFFF)
                    seen += 1
                else:
                    assert kk == 0xFFFFFFFFFFFFFFFF
    assert seen > 10
    # visits: every (ray, window voxel) pair the segment from the sensor touches
    o = [round(M[a][3] * scale) for a in range(3)]
    lo, hi = tuple(origin), tuple(origin[a] + dims[a] for a in range(3))
    visits = 0
    for p in xyz:
        q = brute.quantise(p, M, scale)
        if q is None or q == o:
            continue
        D = [q[a] - o[a] for a in range(3)]
        r = brute.isqrt_floor(sum(d * d for d in D))
        off = [brute.round_half_away(Fraction(tau * D[a], r)) for a in range(3)]
        E = [q[a] + off[a] for a in range(3)]
        S = o if r <= tau else [q[a] - off[a] for a in range(3)]
        visits += len(brute.segment_voxels_brute(S, E, lo, hi))
        if r > tau:
            visits += len(brute.segment_voxels_brute(o, S, lo, hi))
    st = m.integrate(xyz, M)
    assert st["visits"] == visits
    m.close()


def test_carve_equals_band_for_short_rays():
    """Rays no longer than tau already start at the sensor: carving changes
    nothing."""
    tau = 3072  # 3 voxels at 0.1 m: points within 0.3 m
    g = np.random.default_rng(75)
    d = g.normal(size=(300, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    xyz = (d * g.uniform(0.02, 0.29, size=(300, 1))).astype(np.float32)
    pose = synth.fuzz_pose(76, 0.5)
    a = oracle.OracleMap((16, 16, 16), (-8, -8, -8), 0.1, tau, 64)
    b = oracle.OracleMap((16, 16, 16), (-8, -8, -8), 0.1, tau, 64)
    b.set_carving(True)
    assert np.array_equal(a.volume(xyz, pose), b.volume(xyz, pose))
    a.close()
    b.close()


def test_carve_superset_of_band_room_scan():
    """Carving adds candidates and removes none: every voxel's key is at most
    its band-only key, every band voxel is still visited, and the carved-only
    voxels hold what the free space in front of the surfaces gives."""
    w = synth.config1()
    spec, sc = w.maps[0], w.scans[0]
    xyz = sc.xyz[::7]
    a = oracle.OracleMap.from_spec(spec)
    b = oracle.OracleMap.from_spec(spec)
    b.set_carving(True)
    ka = a.volume(xyz, sc.pose)
    kb = b.volume(xyz, sc.pose)
    E = np.uint64(0xFFFFFFFFFFFFFFFF)
    assert np.all(kb <= ka)
    assert np.all(kb[ka != E] != E)
    extra = (kb != E) & (ka == E)
    assert extra.sum() > 5 * (ka != E).sum()
    s = (kb[extra] & np.uint64(0xFFFF)).astype(np.uint16).view(np.int16)
    assert np.mean(s == spec.tau_u) > 0.9  # mostly truncated free space
    assert np.all(s > -spec.tau_u)
    a.close()
    b.close()


def test_voxel_sdf_wide_numerators():
    """The distance numerator (q - c) . D of a voxel near the sensor of a
    long ray exceeds 64 bits; the result is still the exact rounded,
    clamped quotient (Python integers)."""
    g = np.random.default_rng(77)
    for _ in range(300):
        o = [int(v) for v in g.integers(-2 ** 30 + 1, -2 ** 29, size=3)]
        q = [int(v) for v in g.integers(2 ** 29, 2 ** 30, size=3)]
        D = [q[a] - o[a] for a in range(3)]
        r = brute.isqrt_floor(sum(d * d for d in D))
        tau = int(g.integers(1, 32768))
        # voxels near the sensor, near the point and at a random place
        t = float(g.uniform(0, 1))
        for base in (o, q, [int(o[a] + t * D[a]) for a in range(3)]):
            gv = [(base[a] >> 10) + int(g.integers(-2, 3)) for a in range(3)]
            dot = sum((q[a] - (1024 * gv[a] + 512)) * D[a] for a in range(3))
            want = max(-tau, min(tau, brute.round_half_away(Fraction(dot, r))))
            assert oracle.voxel_sdf(q, D, r, gv, tau) == want
    # the sign of a huge numerator decides the clamp
    assert oracle.voxel_sdf(q, D, r, [v >> 10 for v in o], 5) == 5


def test_carve_and_interpolation_exclusive():
    m = oracle.OracleMap((8, 8, 8), (0, 0, 0), 0.1, 3072, 64)
    m.set_carving(True)
    with pytest.raises(ValueError):
        m.set_interpolation(30.0, 16)
    m.set_carving(False)
    m.set_interpolation(30.0, 16)
    with pytest.raises(ValueError):
        m.set_carving(True)
    m.close()

"""GPU parity of free-space carving (each ray longer than tau also walked
from the sensor to the start of its band): maps, per-scan counts and the
routing of carving maps in batches, bit-exact with the oracle; rays as long
as the fixed point allows, sensors outside the window."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_map(dims, origin, vs, tau, wmax):
    from paper_2310_05766_amd.tsdf import TsdfMap
    return TsdfMap(dims, origin, vs, tau, wmax)


def same(gm, om, dims):
    o = gm.origin
    hi = tuple(o[a] + dims[a] for a in range(3))
    g = gm.readback(o, hi)
    r = om.readback(o, hi)
    return np.array_equal(g[0], r[0]) and np.array_equal(g[1], r[1])


def test_config1_carved_bit_exact():
    w = synth.config1()
    spec, sc = w.maps[0], w.scans[0]
    say("config1 with carving")
    om = oracle.OracleMap.from_spec(spec)
    gm = gpu_map(spec.dims, spec.origin, spec.voxel_size, spec.tau_u, spec.w_max)
    om.set_carving(True)
    assert gm.set_carving(True) is True
    poses = [sc.pose] + [synth.fuzz_pose((91, k), 0.5) for k in range(3)]
    for k, p in enumerate(poses):
        gst = gm.integrate(sc.xyz, p, stats=True)
        ost = om.integrate(sc.xyz, p)
        assert gst == ost, (k, gst, ost)
    assert same(gm, om, spec.dims)
    gm.close()
    om.close()


def test_config2_scans_carved_bit_exact():
    """Sensors outside the window (x = -24.5 m, +24.5 m) and inside it."""
    w = synth.config2(50)
    spec = w.maps[0]
    om = oracle.OracleMap.from_spec(spec)
    gm = gpu_map(spec.dims, spec.origin, spec.voxel_size, spec.tau_u, spec.w_max)
    om.set_carving(True)
    gm.set_carving(True)
    for k in (0, 25, 49):
        sc = w.scans[k]
        say("config2 scan", k, "with carving")
        gst = gm.integrate(sc.xyz, sc.pose, stats=True)
        ost = om.integrate(sc.xyz, sc.pose)
        assert gst == ost, (k, gst, ost)
    assert same(gm, om, spec.dims)
    gm.close()
    om.close()


FUZZ = [((24, 24, 24), (-12, -12, -12), 0.1, 3072, 64, 0.5),
        ((33, 17, 29), (-16, -9, -14), 0.07, 2048, 5, 2.5),
        ((16, 40, 12), (-7, -21, -5), 0.12, 5120, 64, 4.0),
        ((64, 8, 8), (3, -4, -4), 0.05, 1, 3, 1.0)]


@pytest.mark.parametrize("case", range(len(FUZZ)))
def test_fuzz_carving(case):
    """Odd window shapes and ring offsets, sensors inside and well outside
    the window, NaN slots, index ties, grid-snapped points, tau of 1."""
    dims, origin, vs, tau, wmax, reach = FUZZ[case]
    om = oracle.OracleMap(dims, origin, vs, tau, wmax)
    gm = gpu_map(dims, origin, vs, tau, wmax)
    om.set_carving(True)
    gm.set_carving(True)
    for k in range(5):
        xyz = synth.fuzz_scan((case, k, 92), 2500, extent_m=1.5, nan_frac=0.05,
                              grid_snap=vs if k == 1 else None)
        xyz[10:14] = xyz[3]
        pose = synth.fuzz_pose((case, k, 93), reach)
        say("carving fuzz", case, k)
        assert gm.integrate(xyz, pose, stats=True) == om.integrate(xyz, pose), k
    assert same(gm, om, dims)
    gm.close()
    om.close()


def test_carving_after_shift():
    dims, vs, tau = (128, 64, 64), 0.05, 3072
    om = oracle.OracleMap(dims, (-64, -32, -32), vs, tau, 64)
    gm = gpu_map(dims, (-64, -32, -32), vs, tau, 64)
    om.set_carving(True)
    gm.set_carving(True)
    for k in range(4):
        if k == 2:
            om.shift((0, -32, -32))
            gm.shift((0, -32, -32))
        xyz = synth.fuzz_scan((94, k), 3000, extent_m=2.5, nan_frac=0.02)
        pose = synth.fuzz_pose((95, k), 1.0)
        say("carving around a shift, scan", k)
        assert gm.integrate(xyz, pose, stats=True) == om.integrate(xyz, pose), k
    assert same(gm, om, dims)
    gm.close()
    om.close()


def test_carving_rays_at_the_fixed_point_limit():
    """Sensors about 2^20 voxels from the points on every axis (distance
    numerators near 3 * 2^62), with the window next to the sensor (the long
    walk set down at once and left early) or next to the points (entered
    after about 2^21 crossings)."""
    vs = 0.05
    lim = 1 << 20
    far = np.array([lim - 40, lim - 40, lim - 40], dtype=np.float64)
    for case, near_sensor in enumerate((True, False)):
        sensor_v = -far if case == 0 else far
        points_v = -sensor_v
        centre_v = sensor_v if near_sensor else points_v
        dims = (24, 20, 16)
        origin = tuple(int(centre_v[a]) - dims[a] // 2 for a in range(3))
        om = oracle.OracleMap(dims, origin, vs, 3072, 64)
        gm = gpu_map(dims, origin, vs, 3072, 64)
        om.set_carving(True)
        gm.set_carving(True)
        pose = np.eye(4)
        pose[:3, 3] = (sensor_v + 0.5) * vs
        g = np.random.default_rng((96, case))
        xyz = ((points_v - sensor_v) * vs + g.uniform(-0.5, 0.5, size=(6, 3))).astype(np.float32)
        if near_sensor:
            # and rays that pass the window obliquely
            xyz = np.concatenate([xyz, (g.uniform(-1.0, 1.0, size=(4, 3)) * 3.0).astype(np.float32)])
        say("carving at the limit, window near the sensor" if near_sensor else "... near the points")
        gst = gm.integrate(xyz, pose, stats=True)
        ost = om.integrate(xyz, pose)
        assert gst == ost, (case, gst, ost)
        assert ost["voxels_updated"] > 0
        assert same(gm, om, dims)
        gm.close()
        om.close()


def test_carving_in_batches_and_switching():
    """A carving map and a plain map sharing batches; carving off and on
    again; device points; per-scan counts in submission order."""
    import torch
    from paper_2310_05766_amd.tsdf import integrate_batch
    spec = ((32, 32, 32), (-16, -16, -16), 0.08, 3072, 64)
    g1, g2 = gpu_map(*spec), gpu_map(*spec)
    o1, o2 = oracle.OracleMap(*spec), oracle.OracleMap(*spec)
    for step, on in enumerate((True, False, True)):
        g1.set_carving(on)
        o1.set_carving(on)
        items, refs = [], []
        for k in range(5):
            xyz = synth.fuzz_scan((97, step, k), 1800, extent_m=1.2, nan_frac=0.03)
            pose = synth.fuzz_pose((98, step, k), 0.6)
            gm, om = (g1, o1) if k % 2 == 0 else (g2, o2)
            items.append((gm, torch.from_numpy(xyz).to("cuda"), pose))
            refs.append(om.integrate(xyz, pose))
        say("batch, carving", on)
        assert integrate_batch(items, stats=True) == refs
        assert same(g1, o1, spec[0]) and same(g2, o2, spec[0])
    for m in (g1, g2, o1, o2):
        m.close()


def test_carving_arguments():
    from paper_2310_05766_amd import TsdfError
    gm = gpu_map((16, 16, 16), (-8, -8, -8), 0.1, 3072, 64)
    assert gm.get_carving() is False
    gm.set_interpolation(30.0, 16)
    with pytest.raises(TsdfError):
        gm.set_carving(True)
    gm.set_interpolation(0.0, 0)
    assert gm.set_carving(True) is True
    with pytest.raises(TsdfError):
        gm.set_interpolation(30.0, 16)
    assert gm.get_interpolation() == 0
    assert gm.set_carving(False) is False
    gm.close()


def test_atomic_probe():
    """The benchmark's measurement aid behind the key-volume roofline (its
    own library, not the TSDF library): it applies atomicMins inside the
    buffer (pattern 1 only to its first 2^19 keys) and checks its
    arguments."""
    import torch
    from paper_2310_05766_amd.probe import atomic_probe
    keys = torch.full((1 << 20,), -1, dtype=torch.int64, device="cuda")
    assert atomic_probe(keys, 64, 8, 1) > 0
    torch.cuda.synchronize()
    assert int((keys[: 1 << 19] != -1).sum()) > 0 and int((keys[1 << 19:] != -1).sum()) == 0
    assert atomic_probe(keys, 64, 8, 0) > 0
    torch.cuda.synchronize()
    assert int((keys[1 << 19:] != -1).sum()) > 0
    for args in [(keys[:1000], 64, 8, 1), (keys, 63, 8, 0), (keys, 64, 0, 0), (keys, 64, 8, 2)]:
        with pytest.raises(ValueError):
            atomic_probe(*args)


def test_carving_degenerate_cases():
    """Empty and all-NaN scans, points at the sensor, rays no longer than
    tau, axis-aligned rays from a sensor on a voxel corner (flat axes, ties
    at t = 0), and a window one voxel thick."""
    cases = [((16, 16, 16), (-8, -8, -8)), ((24, 1, 20), (-12, 0, -10)), ((1, 1, 40), (0, 0, -20))]
    vs, tau = 0.1, 3072
    for case, (dims, origin) in enumerate(cases):
        om = oracle.OracleMap(dims, origin, vs, tau, 64)
        gm = gpu_map(dims, origin, vs, tau, 64)
        om.set_carving(True)
        gm.set_carving(True)
        corner = np.eye(4)  # sensor on a voxel corner of the grid
        centre = np.eye(4)
        centre[:3, 3] = [0.05, 0.05, 0.05]  # sensor on a voxel centre
        axis = np.array([[d * s, 0, 0] for d in (0.35, 1.0, 2.2) for s in (1, -1)] +
                        [[0, d * s, 0] for d in (0.35, 1.0, 2.2) for s in (1, -1)] +
                        [[0, 0, d * s] for d in (0.35, 1.0, 2.2) for s in (1, -1)] +
                        [[0.5, 0.5, 0.0], [-0.7, 0.7, 0.7], [0.3, 0.0, -0.9]], dtype=np.float32)
        scans = [
            (np.zeros((0, 3), np.float32), corner),
            (np.full((50, 3), np.nan, np.float32), corner),
            (np.zeros((20, 3), np.float32), centre),  # every point at the sensor
            (synth.fuzz_scan((99, case), 400, extent_m=0.25, nan_frac=0.1), centre),  # r <= tau mostly
            (axis, corner),
            (axis, centre),
            (synth.fuzz_scan((98, case), 600, extent_m=2.0, nan_frac=0.05, grid_snap=0.1), corner),
        ]
        for k, (xyz, pose) in enumerate(scans):
            say("carving degenerate case", case, "scan", k)
            assert gm.integrate(xyz, pose, stats=True) == om.integrate(xyz, pose), (case, k)
        assert same(gm, om, dims)
        gm.close()
        om.close()

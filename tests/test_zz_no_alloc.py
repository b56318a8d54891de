"""The allocation-free entry point, tsdf_integrate_scan_noalloc, through the C
ABI: on two calls in a row (the second with a smaller input, on another map
shape) it gives exactly the map and counts of tsdf_integrate_scan on the same
scans; sizes beyond its fixed device array are rejected without touching the
map; maps on the key-volume paths are rejected."""
import ctypes as C
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _entry():
    from paper_2310_05766_amd import _abi
    return _abi.lib().tsdf_integrate_scan_noalloc


def _noalloc(m, xyz_dev, pose, want_stats=True):
    from paper_2310_05766_amd import _abi
    M = np.ascontiguousarray(np.asarray(pose, dtype=np.float64).reshape(16))
    st = _abi.ScanStats()
    rc = _entry()(m.handle, C.c_void_p(xyz_dev.data_ptr()), xyz_dev.shape[0], M.ctypes.data_as(C.POINTER(C.c_double)),
                  C.byref(st) if want_stats else None)
    stats = dict(points_in=st.points_in, points_valid=st.points_valid, visits=st.visits,
                 voxels_updated=st.voxels_updated)
    return rc, stats


def _window(m):
    o = m.origin
    return m.readback(o, tuple(o[a] + m.dims[a] for a in range(3)))


def test_noalloc_matches_integrate_scan_two_calls():
    import torch
    from paper_2310_05766_amd.tsdf import TsdfMap
    torch.cuda.set_device(0)
    w2 = synth.config2(2)
    spec2 = w2.maps[0]
    w1 = synth.config1()
    spec1 = w1.maps[0]
    st = torch.cuda.current_stream()
    cases = [
        # (map spec, points, pose): a full OS1-128 scan, then a smaller one on another window
        (spec2, w2.scans[1].xyz, w2.scans[1].pose),
        (spec1, w1.scans[0].xyz[: 9000], w1.scans[0].pose),
    ]
    for k, (spec, xyz, pose) in enumerate(cases):
        say("no-alloc call", k, "points", xyz.shape[0], "window", spec.dims)
        dev = torch.from_numpy(np.ascontiguousarray(xyz)).to("cuda")
        torch.cuda.synchronize()
        a = TsdfMap.from_spec(spec, stream=st)
        b = TsdfMap.from_spec(spec, stream=st)
        rc, sa = _noalloc(a, dev, pose)
        assert rc == 0, rc
        sb = b.integrate(dev, pose, stats=True)
        assert sa == sb, (sa, sb)
        assert sa["voxels_updated"] > 1000
        # a second scan on the same maps: the state the first left behind
        rc, sa2 = _noalloc(a, dev, synth.fuzz_pose((91, k), 0.2) @ pose)
        assert rc == 0, rc
        sb2 = b.integrate(dev, synth.fuzz_pose((91, k), 0.2) @ pose, stats=True)
        assert sa2 == sb2
        ga, gb = _window(a), _window(b)
        assert np.array_equal(ga[0], gb[0]) and np.array_equal(ga[1], gb[1])
        a.close()
        b.close()
        del dev


def test_noalloc_small_case_matches_oracle_and_no_stats():
    import torch

    import oracle
    from paper_2310_05766_amd.tsdf import TsdfMap
    w1 = synth.config1()
    spec, sc = w1.maps[0], w1.scans[0]
    dev = torch.from_numpy(sc.xyz).to("cuda")
    torch.cuda.synchronize()
    m = TsdfMap.from_spec(spec, stream=torch.cuda.current_stream())
    rc, _ = _noalloc(m, dev, sc.pose, want_stats=False)  # returns without waiting
    assert rc == 0
    om = oracle.OracleMap.from_spec(spec)
    om.integrate(sc.xyz, sc.pose)
    o = spec.origin
    ref = om.readback(o, tuple(o[a] + spec.dims[a] for a in range(3)))
    got = _window(m)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    om.close()
    m.close()


def test_noalloc_rejects_what_it_cannot_hold():
    import torch
    from paper_2310_05766_amd import _abi
    from paper_2310_05766_amd.tsdf import TsdfMap
    w2 = synth.config2(1)
    spec, sc = w2.maps[0], w2.scans[0]
    big = torch.from_numpy(np.tile(sc.xyz, (4, 1))).to("cuda")  # 524,288 points: beyond the array
    torch.cuda.synchronize()
    m = TsdfMap.from_spec(spec, stream=torch.cuda.current_stream())
    rc, _ = _noalloc(m, big, sc.pose)
    assert rc == -4  # TSDF_ERANGE
    sdf, w = _window(m)
    assert not w.any() and not sdf.any()  # untouched
    m.set_carving(True)
    rc, _ = _noalloc(m, big[:1000], sc.pose)
    assert rc == -1  # key-volume maps take their own (allocating) path
    m.set_carving(False)
    rc, _ = _noalloc(m, big[:1000], np.full((4, 4), np.nan))
    assert rc == -1
    m.close()

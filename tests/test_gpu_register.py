"""GPU parity of point-to-TSDF registration: the normal equations at a pose
against the oracle's (same points used; sums equal up to the summation
order), and whole Gauss-Newton runs ending at the oracle's pose."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _perturbed(pose, dx, dy, yaw):
    P = pose.copy()
    P[0, 3] += dx
    P[1, 3] += dy
    c, s = math.cos(yaw), math.sin(yaw)
    P[:3, :3] = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]]) @ P[:3, :3]
    return P


def _maps(n_scans=3):
    from paper_2310_05766_amd.tsdf import TsdfMap
    w = synth.config1()
    spec, sc = w.maps[0], w.scans[0]
    gm = TsdfMap.from_spec(spec)
    om = oracle.OracleMap.from_spec(spec)
    poses = [sc.pose] + [synth.fuzz_pose((95, k), 0.1) for k in range(n_scans - 1)]
    for p in poses:
        gm.integrate(sc.xyz, p)
        om.integrate(sc.xyz, p)
    return spec, sc, gm, om


def test_normal_equations_match_oracle():
    import torch
    spec, sc, gm, om = _maps()
    dev = torch.from_numpy(sc.xyz).to("cuda")
    torch.cuda.synchronize()
    for k, P in enumerate([sc.pose, _perturbed(sc.pose, 0.03, -0.02, 0.01), _perturbed(sc.pose, -0.1, 0.05, -0.03)]):
        g = gm.register_sums(sc.xyz, P)
        gd = gm.register_sums(dev, P)
        o = om.reg_sums(sc.xyz, P)
        say("pose", k, "points", o[28])
        assert o[28] > 1000 and g[28] == o[28]
        assert np.array_equal(g, gd)  # host and device points, same order of sums
        assert np.allclose(g, o, rtol=1e-11, atol=1e-14 * np.abs(o).max())
    gm.close()
    om.close()


def test_registration_runs_match_oracle():
    spec, sc, gm, om = _maps()
    for k, (dx, dy, yaw) in enumerate([(0.04, -0.03, 0.02), (-0.06, 0.02, -0.015)]):
        P0 = _perturbed(sc.pose, dx, dy, yaw)
        gp, gi = gm.register(sc.xyz, P0, 8, 1e-6)
        op, oi = om.register(sc.xyz, P0, 8, 1e-6)
        say("run", k, gi, oi)
        assert gi["steps"] == oi["steps"]
        assert abs(gi["points"] - oi["points"]) <= 2
        assert np.allclose(gp, op, rtol=0, atol=1e-7)
        assert np.linalg.norm(gp[:3, 3] - sc.pose[:3, 3]) < 0.01
    gm.close()
    om.close()


def test_registration_arguments():
    from paper_2310_05766_amd import TsdfError
    spec, sc, gm, om = _maps(1)
    with pytest.raises(TsdfError):
        gm.register(sc.xyz, sc.pose, -1)
    bad = sc.pose.copy()
    bad[0, 0] = np.nan
    with pytest.raises(TsdfError):
        gm.register(sc.xyz, bad)
    p, info = gm.register(np.zeros((0, 3), np.float32), sc.pose, 5)
    assert info["points"] == 0 and info["steps"] == 0 and np.array_equal(p, sc.pose)
    gm.close()
    om.close()

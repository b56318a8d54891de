"""GPU parity of the batched forms: ordered multi-scan batches on one map,
interleaved batches over several maps, batches longer than one chunk, and
every candidate tiling -- each bit-exact with the oracle applied scan by
scan in submission order."""
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


def test_config2_ordered_batch():
    from paper_2310_05766_amd.tsdf import integrate_batch
    w = synth.config2(20)
    spec = w.maps[0]
    say("config2: 20 scans, one batch")
    om = oracle.OracleMap.from_spec(spec)
    ost = [om.integrate(s.xyz, s.pose) for s in w.scans]
    gm = gpu_map(spec.dims, spec.origin, spec.voxel_size, spec.tau_u, spec.w_max)
    gst = integrate_batch([(gm, s.xyz, s.pose) for s in w.scans], stats=True)
    assert gst == ost
    assert same(gm, om, spec.dims)
    gm.close()
    om.close()


def test_config2_full_batch_as_benchmarked():
    """The benchmark's launch shape: all 50 OS1-128 scans of the sequence as
    one ordered batch, points already in device memory, on a stream of its
    own, graph launch on; the second batch replays the captured graph."""
    import torch
    from paper_2310_05766_amd.tsdf import TsdfMap, integrate_batch, set_graph_launch
    w = synth.config2()
    spec = w.maps[0]
    set_graph_launch(True)
    st = torch.cuda.Stream()
    dev = [torch.from_numpy(s.xyz).to("cuda") for s in w.scans]
    torch.cuda.synchronize()
    gm = TsdfMap.from_spec(spec, stream=st)
    om = oracle.OracleMap.from_spec(spec)
    for rep in range(2):
        say("config2: batch of 50, pass", rep)
        integrate_batch([(gm, x, s.pose) for x, s in zip(dev, w.scans)], stream=st)
        for s in w.scans:
            om.integrate(s.xyz, s.pose)
        gm.synchronize()
        assert same(gm, om, spec.dims), rep
    gm.close()
    om.close()


def test_interleaved_maps_and_long_batches():
    """Three maps, scans interleaved in random order; one map gets 70 scans
    (more than one chunk of 64)."""
    from paper_2310_05766_amd.tsdf import integrate_batch
    specs = [((48, 40, 24), (-24, -20, -12), 0.05, 3072, 5),
             ((33, 65, 17), (-16, -30, -8), 0.08, 5120, 64),
             ((64, 64, 64), (-32, -32, -32), 0.064, 5120, 64)]
    g = np.random.default_rng(5)
    order = [0] * 70 + [1] * 12 + [2] * 9
    g.shuffle(order)
    items, refs = [], []
    gms = [gpu_map(*s) for s in specs]
    oms = [oracle.OracleMap(*s) for s in specs]
    for k, m in enumerate(order):
        xyz = synth.fuzz_scan((77, k), 1500 + 97 * (k % 5), extent_m=1.5, nan_frac=0.05,
                              grid_snap=0.05 if k % 7 == 0 else None)
        pose = synth.fuzz_pose((78, k), max_t=0.3)
        items.append((gms[m], xyz, pose))
        refs.append(oms[m].integrate(xyz, pose))
    say("interleaved batch of", len(items), "scans")
    st = integrate_batch(items, stats=True)
    assert st == refs
    for k, s in enumerate(specs):
        assert same(gms[k], oms[k], s[0]), k
        gms[k].close()
        oms[k].close()


TILINGS = [(3, 3, 3), (2, 3, 4), (3, 4, 5), (4, 4, 4), (2, 2, 5), (4, 3, 3), (3, 3, 6), (4, 4, 3)]


@pytest.mark.parametrize("lt", TILINGS)
def test_every_tiling_gives_the_same_map(lt):
    from paper_2310_05766_amd.tsdf import integrate_batch
    w = synth.config1()
    spec, sc = w.maps[0], w.scans[0]
    om = oracle.OracleMap.from_spec(spec)
    gm = gpu_map(spec.dims, spec.origin, spec.voxel_size, spec.tau_u, spec.w_max)
    gm.set_tiling(lt)
    assert gm.get_tiling()[0] == tuple(lt)
    poses = [sc.pose] + [synth.fuzz_pose((lt, k), 0.4) for k in range(5)]
    for p in poses[:2]:
        assert gm.integrate(sc.xyz, p, stats=True) == om.integrate(sc.xyz, p)
    st = integrate_batch([(gm, sc.xyz, p) for p in poses[2:]], stats=True)
    assert st == [om.integrate(sc.xyz, p) for p in poses[2:]]
    assert same(gm, om, spec.dims)
    gm.close()
    om.close()


@pytest.mark.parametrize("workgroups", [1, 3, 7, 8, 9])
def test_few_tile_workgroups_drain_every_queue(workgroups):
    """Grids smaller than the number of work queues (one per XCD): every busy
    tile is still processed, over two batches in a row (the second starts
    from the per-tile counts the first left), bit-exact with the oracle."""
    from paper_2310_05766_amd.tsdf import integrate_batch
    w = synth.config1()
    spec, sc = w.maps[0], w.scans[0]
    om = oracle.OracleMap.from_spec(spec)
    gm = gpu_map(spec.dims, spec.origin, spec.voxel_size, spec.tau_u, spec.w_max)
    gm.set_tiling((3, 3, 3), workgroups)
    assert gm.get_tiling() == ((3, 3, 3), workgroups)
    for b in range(2):
        poses = [synth.fuzz_pose((workgroups, b, k), 0.4) for k in range(3)]
        st = integrate_batch([(gm, sc.xyz, p) for p in poses], stats=True)
        assert st == [om.integrate(sc.xyz, p) for p in poses], (workgroups, b)
        assert gm.integrate(sc.xyz, sc.pose, stats=True) == om.integrate(sc.xyz, sc.pose)
    assert same(gm, om, spec.dims)
    gm.close()
    om.close()


@pytest.mark.parametrize("blocks", [(128, 256), (512, 256), (256, 512), (512, 512), (128, 512)])
def test_every_block_size_gives_the_same_map(blocks):
    """Binning blocks of 128, 256 and 512 points and tile workgroups of 256
    and 512 threads: the same map and counts as the oracle, for single
    scans and for a batch of several scans of one map."""
    from paper_2310_05766_amd import TsdfError
    from paper_2310_05766_amd.tsdf import integrate_batch
    w = synth.config1()
    spec, sc = w.maps[0], w.scans[0]
    om = oracle.OracleMap.from_spec(spec)
    gm = gpu_map(spec.dims, spec.origin, spec.voxel_size, spec.tau_u, spec.w_max)
    gm.set_blocks(*blocks)
    assert gm.get_blocks() == tuple(blocks)
    poses = [sc.pose] + [synth.fuzz_pose((blocks, k), 0.4) for k in range(9)]
    for p in poses[:2]:
        assert gm.integrate(sc.xyz, p, stats=True) == om.integrate(sc.xyz, p)
    st = integrate_batch([(gm, sc.xyz, p) for p in poses[2:]], stats=True)
    assert st == [om.integrate(sc.xyz, p) for p in poses[2:]]
    assert same(gm, om, spec.dims)
    for bad in [(64, 256), (256, 128), (300, 256), (-1, 0)]:
        with pytest.raises(TsdfError):
            gm.set_blocks(*bad)
    gm.set_blocks(0, 0)
    assert gm.get_blocks() == (256, 256)
    gm.close()
    om.close()


def test_invalid_tilings_rejected():
    from paper_2310_05766_amd import TsdfError
    gm = gpu_map((32, 32, 32), (-16, -16, -16), 0.05, 3072, 64)
    assert gm.get_tiling()[0] == (0, 0, 0)  # chosen per call until set
    for lt in [(1, 4, 4), (3, 3, 2), (7, 3, 3), (2, 2, 3), (5, 5, 5), (0, 3, 3)]:
        with pytest.raises(TsdfError):
            gm.set_tiling(lt)
    gm.set_tiling((4, 4, 4))
    gm.set_tiling((0, 0, 0))
    assert gm.get_tiling()[0] == (0, 0, 0)
    gm.close()


def test_batch_of_nothing_and_empty_scans():
    from paper_2310_05766_amd.tsdf import integrate_batch
    gm = gpu_map((16, 16, 16), (-8, -8, -8), 0.1, 3072, 64)
    om = oracle.OracleMap((16, 16, 16), (-8, -8, -8), 0.1, 3072, 64)
    assert integrate_batch([]) is None
    xyz = synth.fuzz_scan(91, 300, extent_m=0.7)
    items = [(gm, np.zeros((0, 3), np.float32), np.eye(4)), (gm, xyz, np.eye(4)),
             (gm, np.full((5, 3), np.nan, np.float32), np.eye(4))]
    st = integrate_batch(items, stats=True)
    ref = [om.integrate(x, p) for _, x, p in items]
    assert st == ref
    assert same(gm, om, (16, 16, 16))
    gm.close()
    om.close()


def test_graph_replays_match_direct_launches():
    """Captured graphs replayed many times, with eager work and syncs in
    between, give the same maps as direct launches and as the oracle."""
    from paper_2310_05766_amd.tsdf import integrate_batch, set_graph_launch
    w = synth.config1()
    spec, sc = w.maps[0], w.scans[0]
    om = oracle.OracleMap.from_spec(spec)
    maps = {}
    try:
        for mode in (True, False):
            set_graph_launch(mode)
            gm = gpu_map(spec.dims, spec.origin, spec.voxel_size, spec.tau_u, spec.w_max)
            snaps = []
            for k in range(6):
                poses = [synth.fuzz_pose((k, j, 5), 0.4) for j in range(1 + k % 3)]
                if k % 2:
                    integrate_batch([(gm, sc.xyz[: 4000 + 1000 * j], p) for j, p in enumerate(poses)])
                else:
                    for j, p in enumerate(poses):
                        gm.integrate(sc.xyz[: 4000 + 1000 * j], p)
                gm.synchronize()
                snaps.append(gm.readback_window())
                if mode:
                    for j, p in enumerate(poses):
                        om.integrate(sc.xyz[: 4000 + 1000 * j], p)
                    ref = om.readback(spec.origin, tuple(spec.origin[a] + spec.dims[a] for a in range(3)))
                    assert np.array_equal(snaps[-1][0], ref[0]) and np.array_equal(snaps[-1][1], ref[1]), k
            maps[mode] = snaps
            gm.close()
    finally:
        set_graph_launch(True)
    for a, b in zip(maps[True], maps[False]):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    om.close()


def test_autotuner_candidates_agree(tmp_path, monkeypatch):
    import torch
    from paper_2310_05766_amd.autotune import autotune
    monkeypatch.setenv("XDG_CACHE_HOME", str(tmp_path))
    w = synth.config1()
    spec, sc = w.maps[0], w.scans[0]
    sample = [(torch.from_numpy(sc.xyz).to("cuda"), synth.fuzz_pose((3, k), 0.3)) for k in range(4)]
    torch.cuda.synchronize()
    best = autotune(spec, sample, mode="batch", reps=1)
    assert tuple(best["lt"]) in [tuple(c["lt"]) for c in best["candidates"]]
    # all three knobs were searched and are recorded: tiling, workgroups, block sizes
    seen = {(c["bin_block"], c["tile_block"]) for c in best["candidates"]}
    assert {(256, 256), (128, 256), (512, 256), (256, 512), (512, 512)} <= seen
    again = autotune(spec, sample, mode="batch", reps=1)
    assert again["cached"] and tuple(again["lt"]) == tuple(best["lt"])
    assert (again["bin_block"], again["tile_block"]) == (best["bin_block"], best["tile_block"])


@pytest.mark.parametrize("lt", [(2, 2, 5), (3, 3, 6), (4, 4, 4), (0, 0, 0)])
def test_longest_bands_resume_at_tile_entries(lt):
    """tau = 32767 (a band of 64 voxels) on rays along z that enter a tile
    after 64 or more voxel crossings on z: the resume counts of the tile
    pass reach their largest values (up to 66 per axis)."""
    from paper_2310_05766_amd.tsdf import integrate_batch
    vs, tau = 1.0, 32767
    dims, origin = (8, 8, 256), (-4, -4, 0)
    om = oracle.OracleMap(dims, origin, vs, tau, 64)
    gm = gpu_map(dims, origin, vs, tau, 64)
    gm.set_tiling(lt)
    pose = np.eye(4)
    pose[:3, 3] = [0.5, 0.5, 0.5]  # sensor on a voxel centre
    pts = []
    for k, zk in enumerate((1, 2, 3, 4, 5)):
        for dz in (2, 10, 500, 1000, 1023):
            # band start S_z = 1024 * 32 * zk + dz (fixed point): 64 crossings
            qz = 1024 * 32 * zk + dz + tau
            pts.append([0.0, 0.0, (qz - 512) / 1024.0])
            pts.append([0.25 * (k - 2) / 1024.0, 0.0, (qz - 512 + 1) / 1024.0])  # nearly vertical
    xyz = np.array(pts, dtype=np.float32)
    assert gm.integrate(xyz, pose, stats=True) == om.integrate(xyz, pose)
    poses = [pose.copy() for _ in range(3)]
    for j, p in enumerate(poses):
        p[:3, 3] = [0.5 - j, 0.5 + j, 0.5 + 7 * j]
    st = integrate_batch([(gm, xyz, p) for p in poses], stats=True)
    assert st == [om.integrate(xyz, p) for p in poses]
    assert same(gm, om, dims)
    gm.close()
    om.close()


@pytest.mark.parametrize("bin_block", [128, 256, 512])
def test_full_binning_table_sends_entries_straight_to_runs(bin_block):
    """Points scattered over a wide window with the longest band (tau =
    32767): each ray crosses about ten tiles, so a binning block meets far
    more (sequence slot, tile) keys than its hash table holds (two slots per
    point) and more tiles per point than it lists in LDS; those entries go
    straight to their runs. Bit-exact with the oracle, one scan and a batch."""
    from paper_2310_05766_amd.tsdf import integrate_batch
    vs, tau = 0.1, 32767
    dims, origin = (256, 256, 64), (-128, -128, -32)
    rng = np.random.default_rng(bin_block)
    xyz = rng.uniform([-12.0, -12.0, -3.0], [12.0, 12.0, 3.0], size=(3000, 3)).astype(np.float32)
    poses = []
    for j in range(3):
        p = np.eye(4)
        p[:3, 3] = [0.03 + 0.4 * j, -0.02 - 0.3 * j, 0.01 + 0.1 * j]
        poses.append(p)
    om = oracle.OracleMap(dims, origin, vs, tau, 64)
    gm = gpu_map(dims, origin, vs, tau, 64)
    gm.set_blocks(bin_block, 0)
    say(f"bin block {bin_block}: one scan")
    assert gm.integrate(xyz, poses[0], stats=True) == om.integrate(xyz, poses[0])
    say(f"bin block {bin_block}: batch of two")
    st = integrate_batch([(gm, xyz, p) for p in poses[1:]], stats=True)
    assert st == [om.integrate(xyz, p) for p in poses[1:]]
    assert same(gm, om, dims)
    gm.close()
    om.close()


@pytest.mark.parametrize("graphs", [True, False])
def test_one_scan_and_multi_scan_batches_interleaved_on_one_stream(graphs):
    """One-scan batches (their descriptors handed to the first kernel, in a
    table of their own) and batches of several scans (descriptor tables
    copied on the engine's copy stream, two device copies used in turn)
    interleaved on one stream, device points, with graph replays and with
    direct launches: the map equals the oracle's scan by scan."""
    torch = pytest.importorskip("torch")
    from paper_2310_05766_amd.tsdf import integrate_batch, set_graph_launch
    w = synth.config2(12)
    spec = w.maps[0]
    say("one-scan and multi-scan batches interleaved, graphs", graphs)
    om = oracle.OracleMap.from_spec(spec)
    for s in w.scans:
        om.integrate(s.xyz, s.pose)
    dev = [torch.from_numpy(s.xyz).to("cuda") for s in w.scans]
    st = torch.cuda.Stream()
    set_graph_launch(graphs)
    try:
        from paper_2310_05766_amd.tsdf import TsdfMap
        gm = TsdfMap.from_spec(spec, stream=st)
        # sizes 1, 3, 1, 2, 1, 4: every batch kind follows every other
        k = 0
        for n in (1, 3, 1, 2, 1, 4):
            integrate_batch([(gm, dev[j], w.scans[j].pose) for j in range(k, k + n)], stream=st)
            k += n
        assert k == len(w.scans)
        assert same(gm, om, spec.dims)
        gm.close()
    finally:
        set_graph_launch(True)

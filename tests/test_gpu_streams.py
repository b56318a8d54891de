"""Device points written on torch's stream just before a call: the library's
stream must wait for them (a torch event, skipped only when torch's stream
has nothing left to do). The points are produced after a long device-side
delay on torch's current stream, so a call that did not wait would read
memory that is not written yet; the result must equal the same scan given
as host points."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _late_points(torch, xyz):
    """A device copy of xyz that torch's current stream writes only after
    about 20 ms of spinning (torch.cuda._sleep)."""
    src = torch.from_numpy(np.ascontiguousarray(xyz, dtype=np.float32)).to("cuda")
    torch.cuda.synchronize()
    torch.cuda._sleep(50_000_000)
    out = torch.empty_like(src)
    out.copy_(src)  # queued behind the spin on the same stream
    return out


def _host_reference(spec, scans):
    from paper_2310_05766_amd.tsdf import TsdfMap

    m = TsdfMap.from_spec(spec)
    for sc in scans:
        m.integrate(sc.xyz, sc.pose)
    sdf, w = m.readback_window()
    m.close()
    return sdf, w


def test_plain_call_waits_for_points_written_on_torch_stream():
    torch = pytest.importorskip("torch")
    from paper_2310_05766_amd.tsdf import TsdfMap

    w = synth.config1()
    spec, sc = w.maps[0], w.scans[0]
    say("plain call, late points", spec.dims)
    want_sdf, want_w = _host_reference(spec, [sc])
    m = TsdfMap.from_spec(spec)  # the library's own stream, not torch's
    x = _late_points(torch, sc.xyz)
    assert not torch.cuda.current_stream().query()  # still spinning: the call must order itself
    m.integrate(x, sc.pose)
    del x  # the map keeps the points alive until its stream has read them
    sdf, ww = m.readback_window()
    m.close()
    assert (ww > 0).sum() > 10000
    assert np.array_equal(sdf, want_sdf) and np.array_equal(ww, want_w)


def test_batch_waits_for_points_written_on_torch_stream():
    torch = pytest.importorskip("torch")
    from paper_2310_05766_amd.tsdf import TsdfMap, integrate_batch

    w = synth.config1()
    spec = w.maps[0]
    base = w.scans[0]
    # the same points from three poses: the batch merges them in order
    scans = [base] + [synth.Scan(xyz=base.xyz, pose=synth.fuzz_pose(s, max_t=0.2), rings=base.rings, cols=base.cols)
                      for s in (3, 4)]
    say("batch, late points", len(scans))
    want_sdf, want_w = _host_reference(spec, scans)
    st = torch.cuda.Stream()
    m = TsdfMap.from_spec(spec, stream=st)
    xs = [_late_points(torch, s.xyz) for s in scans]
    assert not torch.cuda.current_stream().query()
    integrate_batch([(m, x, s.pose) for x, s in zip(xs, scans)], stream=st)
    del xs  # recorded on the batch's stream: kept until it has read them
    sdf, ww = m.readback_window()
    m.close()
    assert (ww > 0).sum() > 10000
    assert np.array_equal(sdf, want_sdf) and np.array_equal(ww, want_w)

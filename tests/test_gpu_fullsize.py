"""GPU parity at the full sizes the benchmark times, against the oracle's
digests of the same workloads (tests/golden/oracle_digests.json, written by
tests/golden/make_oracle_digests.py, which calls only the oracle):

* free-space carving over all 50 OS1-128-shaped config-2 scans;
* vertical interpolation (45 deg over 128 lines) over the first 10;
* config 5 at its stated scale: all 48 sessions over the full 60 s Poisson
  trace (about 28,800 distinct 16x1024 scans), served by continuous batching
  (the trace compressed 1000 times), every session's final map compared.

Each final window is compared by its sha256 (sdf bytes, then w bytes), and
the per-scan counts (or, for config 5, their sums per session) exactly; the
inputs are checked by their own digest first, so that a change of the inputs
is told apart from a parity failure."""
import sys

import numpy as np
import pytest

import oracle_runs
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def golden():
    return oracle_runs.load_digests()


def _config2_run(golden_entry, n, option):
    import torch
    from paper_2310_05766_amd.tsdf import TsdfMap
    w = synth.config2(n)
    spec = w.maps[0]
    assert oracle_runs.input_digest([(s.xyz, s.pose) for s in w.scans]) == golden_entry["inputs_sha256"]
    dev = [torch.from_numpy(s.xyz).to("cuda") for s in w.scans]
    st = torch.cuda.Stream()
    torch.cuda.synchronize()
    m = TsdfMap.from_spec(spec, stream=st)
    if option == "carving":
        m.set_carving(True)
    else:
        m.set_interpolation(45.0, 128)
    per = []
    for k, (x, s) in enumerate(zip(dev, w.scans)):
        r = m.integrate(x, s.pose, stats=True)
        per.append([r["points_valid"], r["visits"], r["voxels_updated"]])
    o = spec.origin
    sdf, wt = m.readback(o, tuple(o[a] + spec.dims[a] for a in range(3)))
    m.close()
    for k, (g, e) in enumerate(zip(per, golden_entry["per_scan_valid_visits_updated"])):
        assert g == e, (option, k, g, e)
    assert oracle_runs.window_digest(sdf, wt) == golden_entry["window_sha256"], option


def test_carving_all_50_config2_scans(golden):
    say("carving: 50 config-2 scans")
    _config2_run(golden["carve50"], 50, "carving")


def test_interpolation_10_config2_scans(golden):
    say("interpolation: 10 config-2 scans")
    _config2_run(golden["interp10"], 10, "interpolation")


def test_config5_full_trace_served(golden):
    from paper_2310_05766_amd.serve import GpuExecutor, Server, replay
    ref = golden["config5"]
    sessions = synth.config5(n_sessions=48, duration_s=60.0)
    say("config 5: generating the scans of 48 sessions x 60 s")
    data = oracle_runs.all_session_scans(48, 60.0)
    for s in sessions:
        x, p = data[s.sid]
        assert x.shape[0] == ref[str(s.sid)]["scans"] == len(s.arrivals)
        assert oracle_runs.input_digest(zip(x, p)) == ref[str(s.sid)]["inputs_sha256"], s.sid

    def scans_of(sid, k):
        x, p = data[sid]
        return x[k], p[k]

    say("config 5: replaying", sum(len(s.arrivals) for s in sessions), "scans")
    ex = GpuExecutor(lanes=2, stats=True)
    srv = Server(ex, budget_bytes=200 * 10 ** 9, lanes=2, max_batch=64)
    recs = replay(srv, [(s.sid, s.spec, s.arrivals) for s in sessions], scans_of, speedup=1000.0,
                  close_at_end=False)
    for st in ex.streams:
        st.synchronize()
    assert len(recs) == sum(len(s.arrivals) for s in sessions)
    assert srv.batches < len(recs)
    tot = {s.sid: {"points_valid": 0, "visits": 0, "voxels_updated": 0} for s in sessions}
    order = {s.sid: [] for s in sessions}
    for r in recs:
        for k in tot[r.sid]:
            tot[r.sid][k] += r.stats[k]
        order[r.sid].append(r.k)
    bad = []
    for s in sessions:
        m = srv.sessions[s.sid].map
        o = s.spec.origin
        sdf, w = m.readback(o, tuple(o[a] + s.spec.dims[a] for a in range(3)))
        if oracle_runs.window_digest(sdf, w) != ref[str(s.sid)]["window_sha256"] or \
                tot[s.sid] != ref[str(s.sid)]["totals"]:
            bad.append(s.sid)
        assert order[s.sid] == sorted(order[s.sid])
        srv.close_session(s.sid)
    ex.close()
    say("config 5: sessions differing from the oracle:", bad)
    assert not bad

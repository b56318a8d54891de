"""Serving on the GPU: config-5-shaped sessions (map sizes 256^3, 384^3,
512x512x256 at 6.4 cm, 16x1024 scans, Poisson arrivals), continuously
batched over two lanes; every session's map bit-exact with the oracle, the
same alone and in the mix, also when a small memory budget makes sessions
wait for admission."""
import sys

import numpy as np
import pytest

import oracle_runs
import synth

pytestmark = pytest.mark.gpu

N_SESSIONS, DURATION = 8, 2.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run(sessions, budget, speedup, options=None):
    from paper_2310_05766_amd.serve import GpuExecutor, Server, latency_summary, replay
    ex = GpuExecutor(lanes=2)
    maps = {}

    def keep(sid, m):
        o = m.origin
        maps[sid] = m.readback(o, tuple(o[a] + m.dims[a] for a in range(3)))

    srv = Server(ex, budget_bytes=budget, lanes=2, max_batch=32, on_release=keep)
    cache = {}

    def scans_of(sid, k):
        if (sid, k) not in cache:
            sc = sessions[sid].scan(k)
            cache[(sid, k)] = (sc.xyz, sc.pose)
        return cache[(sid, k)]

    # scans are generated ahead, so that generation never stalls the replay
    for s in sessions:
        for k in range(len(s.arrivals)):
            scans_of(s.sid, k)
    options = options or {}
    recs = replay(srv, [(s.sid, s.spec, s.arrivals, options.get(s.sid)) for s in sessions], scans_of,
                  speedup=speedup)
    ex.close()
    return recs, maps, srv, latency_summary(recs)


@pytest.fixture(scope="module")
def reference():
    say("oracle for", N_SESSIONS, "sessions")
    return oracle_runs.sessions_oracle(list(range(N_SESSIONS)), 10 ** 6, N_SESSIONS, DURATION)


def test_sessions_bit_exact_in_the_mix(reference):
    sessions = synth.config5(n_sessions=N_SESSIONS, duration_s=DURATION)
    recs, maps, srv, lat = run(sessions, budget=200 * 10 ** 9, speedup=4.0)
    say("mix:", lat, "batches", srv.batches)
    assert len(recs) == sum(len(s.arrivals) for s in sessions)
    assert srv.batches < len(recs)  # scans were batched
    for s in sessions:
        ref = reference[s.sid]
        assert np.array_equal(maps[s.sid][0], ref[0]) and np.array_equal(maps[s.sid][1], ref[1]), s.sid
        ks = [r.k for r in recs if r.sid == s.sid]
        assert ks == sorted(ks)


def test_session_alone_equals_mix(reference):
    sessions = synth.config5(n_sessions=N_SESSIONS, duration_s=DURATION)
    recs, maps, srv, lat = run([sessions[0]], budget=200 * 10 ** 9, speedup=4.0)
    ref = reference[0]
    assert np.array_equal(maps[0][0], ref[0]) and np.array_equal(maps[0][1], ref[1])


def test_small_budget_admission(reference):
    sessions = synth.config5(n_sessions=N_SESSIONS, duration_s=DURATION)
    budget = 1 << 30  # 1 GiB: a few maps at a time
    recs, maps, srv, lat = run(sessions, budget=budget, speedup=8.0)
    say("1 GiB budget:", lat, "admissions", len(srv.admit_log))
    assert len(srv.admit_log) == N_SESSIONS
    assert max(t for t, _ in srv.admit_log) > 0.0  # someone waited for memory
    for s in sessions:
        ref = reference[s.sid]
        assert np.array_equal(maps[s.sid][0], ref[0]) and np.array_equal(maps[s.sid][1], ref[1]), s.sid


def test_sessions_with_map_options():
    """A carving session and an interpolating session served beside a plain
    one: each map bit-exact with the oracle integrating that session's scans
    in order with the same option."""
    import oracle
    sessions = synth.config5(n_sessions=3, duration_s=1.0)
    opts = {0: {"carving": True}, 1: {"interpolation": (30.0, 16)}, 2: None}
    recs, maps, srv, lat = run(sessions, budget=200 * 10 ** 9, speedup=4.0, options=opts)
    say("options mix:", lat, "batches", srv.batches)
    for s in sessions:
        m = oracle.OracleMap.from_spec(s.spec)
        if s.sid == 0:
            m.set_carving(True)
        if s.sid == 1:
            m.set_interpolation(30.0, 16)
        for k in range(len(s.arrivals)):
            sc = s.scan(k)
            m.integrate(sc.xyz, sc.pose)
        o = s.spec.origin
        ref = m.readback(o, tuple(o[a] + s.spec.dims[a] for a in range(3)))
        m.close()
        assert np.array_equal(maps[s.sid][0], ref[0]) and np.array_equal(maps[s.sid][1], ref[1]), s.sid

"""The continuous-batching request server on the GPU.

* a cold request served in a mix equals the oracle (FP64 mode, 1e-9) and the same request solved
  through the problem API;
* MPC sessions: every warm-started request equals the oracle's session solver (shifted warm
  start, FP64, 1e-9);
* alone vs in the mix: every request of a session gives bit-identical results when its session
  runs alone on a fresh server and when it is interleaved with other sessions, request types and
  horizons (FP32);
* the same holds when the only difference is the kernel instantiation of the launches (a
  companion with more obstacles, or of the other model, shares every launch);
* backpressure: under a small HBM budget every request still completes, the resident footprint
  never exceeds the budget, and idle warm states are evicted.
"""
import math

import numpy as np
import pytest

import oracle
import scpgen
from _parity import oracle_scp, rel_err

pytestmark = pytest.mark.gpu

TOL64 = 1e-9


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def B(lib):
    from paper_2603_10711_amd import binding
    return binding


def _server(B, prec="f32", scp=2, admm=30, block=None, **kw):
    prm = B.scp_params(scp, admm)
    return B.Server(prm, precision=prec, block=block or (256 if prec == "f32" else 128), max_nodes=1 << 15,
                    max_traj=512, max_wg=512, max_span=64, max_requests=64, **kw)


def test_cold_request_fp64_matches_oracle_and_problem_api(B):
    req = scpgen.config4_request(11, S=16, N=30)
    other = [scpgen.quad_instance(4, 700 + i, N=25 + 7 * i, K=4) for i in range(3)]
    srv = _server(B, "f64")
    ids = [srv.submit([d]) for d in other[:2]]
    rid = srv.submit(req, session=-1)
    ids.append(srv.submit([other[2]]))
    res = srv.drain(ids + [rid])
    got = res[rid]
    trajs, oinfo = oracle_scp(req, 2, 30)
    worst = max(max(rel_err(x, t.xbar), rel_err(u, t.ubar)) for x, u, t in zip(got["x"], got["u"], trajs))
    _say("served vs oracle", worst, srv.stats())
    assert worst < TOL64
    prob = B.Problem(req, precision="f64", block=128)
    prob.solve(B.scp_params(2, 30))
    x, u, info = (a.cpu().numpy() for a in prob.result())
    for m in range(16):
        np.testing.assert_array_equal(prob.split(x, m, 6), got["x"][m])
        np.testing.assert_array_equal(prob.split(u, m, 3, True), got["u"][m])
    for i, o in zip(got["info"], oinfo):
        assert i["admm_iters"] == o["admm_iters"] and i["n_accept"] == o["n_accept"]
    prob.close()
    srv.close()


def _session_reqs(session, n, S=3, N=12):
    return [scpgen.config4_request(session, S=S, N=N) for _ in range(n)]


def test_session_warm_starts_fp64_match_oracle(B):
    reqs = _session_reqs(21, 3)
    prm = oracle.default_params(scp_iters=2, admm_iters=30)
    ref = oracle.mpc_session(reqs, prm)
    srv = _server(B, "f64")
    got = []
    for r in reqs:                      # the MPC loop: the next request follows the previous result
        rid = srv.submit(r, session=21)
        got.append(srv.drain([rid])[rid])
    assert srv.stats()["warm_starts"] == 2
    for k, ((trajs, _), g) in enumerate(zip(ref, got)):
        worst = max(max(rel_err(x, t.xbar), rel_err(u, t.ubar)) for x, u, t in zip(g["x"], g["u"], trajs))
        _say("session request", k, worst)
        assert worst < TOL64
    srv.close()


def _mixed_stream(seed=0):
    """Interleaved submissions: three MPC sessions (16 and 4 scenarios, different horizons),
    single quadrotors and powered-descent instances."""
    rng = np.random.default_rng(seed)
    events = []
    for k in range(3):
        events.append(("s", 31, scpgen.config4_request(31, S=16, N=40)))
        events.append(("s", 32, scpgen.config4_request(32, S=4, N=70)))
        events.append(("s", 33, scpgen.config4_request(33, S=16, N=80)))
        events.append(("q", -1, [scpgen.quad_instance(3, 40 + k, N=int(rng.integers(20, 121)), K=8, T=5.0)]))
        events.append(("m", -1, [scpgen.mars_instance(3, 50 + k, N=int(rng.integers(20, 121)), tf=50.0)]))
    return events


def _run_stream(B, srv, events, steps_between=1):
    ids = []
    for kind, sess, req in events:
        ids.append((kind, sess, srv.submit(req, session=sess)))
        for _ in range(steps_between):
            srv.step()
    res = srv.drain([i for _, _, i in ids])
    return [(kind, sess, res[i]) for kind, sess, i in ids]


def test_alone_equals_in_mix_fp32(B):
    events = _mixed_stream()
    srv = _server(B, "f32", scp=3, admm=40)
    mixed = _run_stream(B, srv, events)
    st = srv.stats()
    _say("mix stats", st)
    assert st["warm_starts"] == 6 and st["completed"] == len(events)
    srv.close()
    for sess in (31, 32, 33):
        alone_srv = _server(B, "f32", scp=3, admm=40)
        alone = _run_stream(B, alone_srv, [e for e in events if e[1] == sess])
        alone_srv.close()
        mine = [r for k, s, r in mixed if s == sess]
        assert len(alone) == len(mine) == 3
        for (_, _, a), m in zip(alone, mine):
            for xa, xm in zip(a["x"], m["x"]):
                np.testing.assert_array_equal(xa, xm)
            for ua, um in zip(a["u"], m["u"]):
                np.testing.assert_array_equal(ua, um)
            assert [i["admm_iters"] for i in a["info"]] == [i["admm_iters"] for i in m["info"]]
    # the independent requests: alone through the problem API
    for kind, sess, r in mixed:
        if sess >= 0:
            continue
    singles = [e for e in events if e[1] < 0]
    for (kind, _, req), (_, _, m) in zip(singles, [x for x in mixed if x[1] < 0]):
        prob = B.Problem(req, precision="f32", block=256)
        prob.solve(B.scp_params(3, 40))
        x, u, info = (a.cpu().numpy() for a in prob.result())
        nx, nu = req[0]["nx"], req[0]["nu"]
        np.testing.assert_array_equal(prob.split(x, 0, nx), m["x"][0])
        np.testing.assert_array_equal(prob.split(u, 0, nu, True), m["u"][0])
        prob.close()


def _session_with_companions(B, sess, S, N, companions):
    """Three requests of one MPC session; with companions, every request shares its launches with
    an 8-obstacle quadrotor and a powered-descent instance (another kernel instantiation)."""
    srv = _server(B, "f32", scp=3, admm=40)
    req = scpgen.config4_request(sess, S=S, N=N)
    outs = []
    for k in range(3):
        ids = [srv.submit(req, session=sess)]
        if companions:
            ids.append(srv.submit([scpgen.quad_instance(3, 40 + k, N=90, K=8, T=5.0)]))
            ids.append(srv.submit([scpgen.mars_instance(3, 50 + k, N=60, tf=50.0)]))
        outs.append(srv.drain(ids)[ids[0]])
    srv.close()
    return outs


@pytest.mark.parametrize("sess,S,N", [(34, 4, 50), (35, 8, 60), (37, 4, 30)])
def test_result_independent_of_kernel_instantiation_fp32(B, sess, S, N):
    """The kernel instantiation a launch uses (obstacle capacity, model mix) must not change any
    bit of a request's result."""
    alone = _session_with_companions(B, sess, S, N, False)
    mixed = _session_with_companions(B, sess, S, N, True)
    for k, (a, m) in enumerate(zip(alone, mixed)):
        _say("request", k, [int((xa != xm).sum()) for xa, xm in zip(a["x"], m["x"])])
        for xa, xm in zip(a["x"], m["x"]):
            np.testing.assert_array_equal(xa, xm)
        for ua, um in zip(a["u"], m["u"]):
            np.testing.assert_array_equal(ua, um)


def test_backpressure_small_budget(B):
    reqs = [scpgen.config4_request(60 + k, S=16, N=30) for k in range(8)]
    probe = _server(B, "f32")
    one = probe.request_bytes(reqs[0])
    probe.close()
    srv = _server(B, "f32", budget_bytes=int(2.5 * one))
    ids = [srv.submit(r, session=60 + k) for k, r in enumerate(reqs)]
    res = srv.drain(ids)
    st = srv.stats()
    _say("backpressure", one, st)
    assert len(res) == 8 and st["completed"] == 8
    assert st["peak_resident_bytes"] <= 2.5 * one
    assert st["evictions"] >= 6
    # a request larger than the whole budget is refused at submission
    tiny = _server(B, "f32", budget_bytes=one // 2)
    with pytest.raises(B.ScpError):
        tiny.submit(reqs[0])
    tiny.close()
    srv.close()


def test_cancel_timeout_done_list_and_stats(B):
    """Cancellation (queued and running), the configured timeout, the done list and the library's
    latency quantiles on the device path; the neighbours of a cancelled request are unaffected."""
    reqs = [scpgen.config4_request(40 + k, S=4, N=30) for k in range(6)]
    srv = _server(B, scp=4, admm=30, max_inflight=1)
    ids = [srv.submit(r) for r in reqs]
    srv.cancel(ids[5])                       # queued: ends at once
    srv.step(wait=True)                      # the others are admitted and run one SCP iteration
    srv.cancel(ids[1])                       # running: leaves at the next step
    res = srv.drain(ids, timeout_s=120)
    states = [res[i]["state"] for i in ids]
    _say(states, srv.stats())
    assert states == ["done", "cancelled", "done", "done", "done", "cancelled"]
    st = srv.stats()
    assert st["cancelled"] == 2 and st["completed"] == 4 and st["resident"] == 0
    assert 0 < st["latency_ms_p50"] <= st["latency_ms_p99"] <= st["latency_ms_p999"] and st["solves_per_s"] > 0
    assert srv.take_done() == []
    # the completed ones equal the same requests served without the cancellations
    ref = _server(B, scp=4, admm=30, max_inflight=1)
    rids = [ref.submit(reqs[k]) for k in (0, 2, 3, 4)]
    rres = ref.drain(rids)
    for k, rid in zip((0, 2, 3, 4), rids):
        for a, b in zip(res[ids[k]]["x"], rres[rid]["x"]):
            np.testing.assert_array_equal(a, b)
    ref.close()
    with pytest.raises(B.ScpError):
        srv.cancel(ids[0])                   # already ended
    srv.close()
    # a timeout shorter than one request's solve: every request ends without a result
    slow = _server(B, scp=10, admm=200, max_inflight=1, timeout_ms=0.5)
    tids = [slow.submit(r) for r in reqs[:3]]
    tres = slow.drain(tids, timeout_s=120)
    _say([tres[i]["state"] for i in tids], slow.stats())
    assert all(tres[i]["state"] == "timeout" for i in tids)
    st = slow.stats()
    assert st["timed_out"] == 3 and st["resident"] == 0
    slow.close()


def test_served_trace_writes_one_record_per_request(B, tmp_path):
    """The load generator's per-request JSON lines: one per served request of a short Poisson
    trace, with the fields the summary is computed from."""
    import json
    from paper_2603_10711_amd import serve_load as SL
    n_sess = 6
    reqs = [scpgen.config4_request(90 + k, S=4, N=20) for k in range(n_sess)]
    srv = _server(B, "f32")
    prepared = [srv.prepare(r) for r in reqs]
    times, sess = SL.arrivals(400.0, 0.05, n_sess)
    path = tmp_path / "served.jsonl"
    with open(path, "w") as log:
        out = SL.run_served(srv, prepared, times, sess, progress=0.0, log=log)
    srv.close()
    recs = [json.loads(line) for line in open(path)]
    _say(out, recs[:2])
    assert out["completed"] == len(times) == len(recs) and out["unfinished"] == 0
    assert len({r["id"] for r in recs}) == len(recs)
    for r in recs:
        assert r["latency_ms"] > 0 and r["done_s"] >= r["arrival_s"] and 0 <= r["session"] < n_sess
        assert r["status"] & (1 | 2 | 4 | 16) == 0
    lat = sorted(r["latency_ms"] for r in recs)
    assert abs(np.median(lat) - out["latency_ms"]["p50"]) <= 1e-2 * max(1.0, out["latency_ms"]["p50"])


def test_served_blowup_detection_changes_no_result(B):
    """The server with residual blow-up detection (the kernel variants that carry the tracking, a
    warm-started session and a spanning request) returns the same bits as without it, and no
    healthy request is flagged."""
    reqs = [scpgen.config4_request(13, S=16, N=40), _session_reqs(5, 2)[0], _session_reqs(5, 2)[1],
            [scpgen.quad_instance(4, 720, N=30, K=4)]]
    out = []
    for detect in (False, True):
        prm = B.scp_params(2, 30, detect_blowup=detect)
        srv = B.Server(prm, precision="f32", block=256, max_nodes=1 << 15, max_traj=512, max_wg=512, max_span=64,
                       max_requests=64)
        ids = [srv.submit(reqs[0], session=-1), srv.submit(reqs[1], session=5), srv.submit(reqs[2], session=5),
               srv.submit(reqs[3])]
        res = srv.drain(ids)
        out.append([res[i] for i in ids])
        srv.close()
    for a, b in zip(*out):
        for m in range(len(a["x"])):
            np.testing.assert_array_equal(a["x"][m], b["x"][m])
            np.testing.assert_array_equal(a["u"][m], b["u"][m])
        assert all(not (int(i["status"]) & B.ST_DIVERGED) for i in b["info"])


def test_served_failure_is_flagged_and_contained(B):
    """Requests with a NaN initial state and with an empty hard box, served among healthy ones (a
    spanning 16-scenario request, a warm-started session, single trajectories): each bad request
    carries its status bit, and every healthy request returns the same bits as on a server
    without the bad ones."""
    good = [scpgen.config4_request(14, S=16, N=40), _session_reqs(6, 2)[0], _session_reqs(6, 2)[1],
            [scpgen.quad_instance(4, 730, N=30, K=4)], [scpgen.mars_instance(3, 731, N=50)]]
    nan = dict(scpgen.quad_instance(4, 732, N=25, K=3))
    nan["x_init"] = nan["x_init"].copy()
    nan["x_init"][2] = math.nan
    box = dict(scpgen.quad_instance(4, 733, N=35, K=2))
    box["x_lo"], box["x_hi"] = box["x_lo"].copy(), box["x_hi"].copy()
    box["x_lo"][3], box["x_hi"][3] = 2.0, -2.0

    def serve(with_bad):
        srv = _server(B, "f32", scp=2, admm=30)
        ids = [srv.submit(good[0]), srv.submit(good[1], session=6)]
        bad_ids = [srv.submit([nan]), srv.submit([box])] if with_bad else []
        ids += [srv.submit(good[2], session=6), srv.submit(good[3]), srv.submit(good[4])]
        res = srv.drain(ids + bad_ids)
        srv.close()
        return [res[i] for i in ids], [res[i] for i in bad_ids]

    with_bad, bad = serve(True)
    without, _ = serve(False)
    assert int(bad[0]["info"][0]["status"]) & B.ST_NONFINITE
    assert int(bad[1]["info"][0]["status"]) & B.ST_EMPTYSET
    for a, b in zip(with_bad, without):
        fail = B.ST_NONFINITE | B.ST_BADPIVOT | B.ST_EMPTYSET | B.ST_SYNC
        assert all((int(i["status"]) & fail) == 0 for i in a["info"])
        for m in range(len(a["x"])):
            np.testing.assert_array_equal(a["x"][m], b["x"][m])
            np.testing.assert_array_equal(a["u"][m], b["u"][m])

"""Open-loop Poisson load of robust-MPC planning requests against the request server.

Workload (the paper's scenario-robust MPC, Sec. IV-A.4, served): sessions are MPC streams, each a
quadrotor with N ~ U{30..80} and S scenarios (drag and mass scale drawn per scenario) sharing the
first control; requests arrive as a Poisson process and go to seeded-uniform sessions.  A
session's next request is warm-started on the device from its previous solution.

Two serving policies over the same arrival trace:
  * served: the library's continuous-batching server (persistent kernel, iteration-level
    admission, device-resident warm state);
  * static plain: whenever the device is idle, everything queued is solved as one batch by the
    plain form (host-enqueued kernels per ADMM iteration) to completion; arrivals wait for the
    next batch; every request starts from its initial guess.
Latency = completion observed by the client minus arrival time.
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np

import scpgen


def session_requests(n_sessions: int, S: int = 16) -> list[list[dict]]:
    """The request of every session (its data is fixed; only x_init moves on warm starts)."""
    return [scpgen.config4_request(s, S=S) for s in range(n_sessions)]


def arrivals(rate: float, duration: float, n_sessions: int, seed: int = 4000):
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(rate * duration * 1.2) + 16
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    t = t[t < duration]
    sess = rng.integers(0, n_sessions, size=t.size)
    return t, sess


def _pcts(lat: list[float]) -> dict:
    a = np.asarray(lat, dtype=float)
    if a.size == 0:
        return dict(p50=None, p99=None, mean=None, max=None)
    return dict(p50=round(float(np.percentile(a, 50)), 3), p99=round(float(np.percentile(a, 99)), 3),
                mean=round(float(a.mean()), 3), max=round(float(a.max()), 3))


def run_served(srv, prepared: list, times, sess, progress: float = 5.0, drain_s: float = 30.0, log=None) -> dict:
    """Drive the server with the arrival trace.  prepared[s] = srv.prepare(request of session s).
    log: a text file that receives one JSON record per ended request (id, session, arrival and
    observed completion in seconds from the start, latency, worst defect over the request's
    trajectories, the OR of their status bits, whether all converged)."""
    n = len(times)
    lat, defect, conv, failed = [], [], 0, 0
    outstanding = {}
    t0 = time.perf_counter()
    i = 0
    last_print = 0.0
    end_deadline = (times[-1] if n else 0.0) + drain_s
    while i < n or outstanding:
        now = time.perf_counter() - t0
        if now > end_deadline:
            break
        while i < n and times[i] <= now:
            rid = srv.submit(prepared[int(sess[i])], session=int(sess[i]))
            outstanding[rid] = (times[i], int(sess[i]))
            i += 1
        srv.step(wait=False)
        ended = srv.take_done()
        if ended:
            t_obs = time.perf_counter() - t0
            for rid in ended:
                r = srv.poll(rid)
                arr, ses = outstanding.pop(rid)
                lat.append((t_obs - arr) * 1e3)
                info = r[1]
                defect.append(float(info[:, 6].max()))
                st = info[:, 5].astype(np.int64)
                conv += int(np.all(st & 8))
                failed += int(np.any(st & (1 | 2 | 4 | 16)))   # non-finite, pivot, empty set, group barrier
                if log is not None:
                    log.write(json.dumps(dict(id=int(rid), session=ses, arrival_s=round(float(arr), 6),
                                              done_s=round(t_obs, 6), latency_ms=round(lat[-1], 3),
                                              max_defect=defect[-1], status=int(np.bitwise_or.reduce(st)),
                                              converged=bool(np.all(st & 8)))) + "\n")
        if progress and now - last_print > progress:
            last_print = now
            print(f"[serve] t={now:.1f}s submitted={i}/{n} outstanding={len(outstanding)} done={len(lat)}",
                  file=sys.stderr, flush=True)
        if i < n and not outstanding and srv.stats()["queued"] == 0:
            time.sleep(max(0.0, min(times[i] - (time.perf_counter() - t0), 0.001)))
    wall = time.perf_counter() - t0
    st = srv.stats()
    return dict(offered=n, completed=len(lat), wall_s=round(wall, 3), latency_ms=_pcts(lat),
                solves_per_s=round(len(lat) / max(wall, 1e-9), 1), unfinished=len(outstanding),
                failure_status=failed,
                defect_p50=float(np.median(defect)) if defect else None, steps=st["steps"],
                warm_starts=st["warm_starts"], evictions=st["evictions"],
                peak_resident_mb=round(st["peak_resident_bytes"] / 2**20, 2))


def run_static_plain(B, parts: list[dict], times, sess, prm, precision: str = "f32", progress: float = 5.0,
                     stream=None, max_wall: float | None = None) -> dict:
    """Static batching with the plain form: take every queued request, solve, repeat."""
    import torch
    n = len(times)
    lat = []
    t0 = time.perf_counter()
    i = 0
    queue = []
    batches = 0
    last_print = 0.0
    while i < n or queue:
        now = time.perf_counter() - t0
        if max_wall is not None and now > max_wall:
            break
        while i < n and times[i] <= now:
            queue.append((times[i], int(sess[i])))
            i += 1
        if not queue:
            time.sleep(max(0.0, min(times[i] - now, 0.001)))
            continue
        batch, queue = queue, []
        prob = B.Problem(None, precision=precision, device="cuda", stream=stream, parts=[parts[s] for _, s in batch])
        prob.solve(prm)
        torch.cuda.synchronize()
        prob.close()
        t_done = time.perf_counter() - t0
        lat.extend((t_done - a) * 1e3 for a, _ in batch)
        batches += 1
        if progress and t_done - last_print > progress:
            last_print = t_done
            print(f"[plain] t={t_done:.1f}s arrived={i}/{n} done={len(lat)} batch={len(batch)}", file=sys.stderr,
                  flush=True)
    wall = time.perf_counter() - t0
    return dict(offered=n, completed=len(lat), wall_s=round(wall, 3), latency_ms=_pcts(lat),
                solves_per_s=round(len(lat) / max(wall, 1e-9), 1), batches=batches, unfinished=n - len(lat))

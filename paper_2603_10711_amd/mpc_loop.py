"""Closed-loop scenario-robust MPC served by the library (Sec. IV-A.4).

The controller loop around the request server: every MPC step submits the S scenario problems
of the measured state as one request of a session; from the second step on the server warm-starts
it in place from the session's resident solution while keeping the measured initial state
(SUBMIT_MEASURED).  The shared first control of scenario 0 goes to the plant, and a linear
disturbance observer updates the estimate carried by the next request:

    d_{k+1} = d_k + K_OBS (v_meas - v_pred) / h,

with v_pred scenario 0's predicted velocity at node 1.  The plant, the wind and the noise come
from the world module passed in (the simulated environment); every solve runs on the GPU.
"""
from __future__ import annotations

import time

import numpy as np

K_OBS = 0.5


def closed_loop_served(srv, world, template: dict, steps: int, draws: dict, session: int = 0) -> dict:
    """Run ``steps`` MPC steps through the server ``srv``.  Returns the plant states
    (steps + 1, 6), the applied controls (steps, 3), the disturbance estimates (steps + 1, 3),
    the per-step wall time of the solve as the controller sees it (ms) and the server's
    per-request latency (ms)."""
    x = np.concatenate([world.START, np.zeros(3)])
    d_hat = np.zeros(3)
    xs, us, ds, wall, lat, infos = [x.copy()], [], [d_hat.copy()], [], [], []
    h = template["h"]
    for k in range(steps):
        req = world.request(template, x, d_hat, draws["xi"][k])
        t0 = time.perf_counter()
        rid = srv.submit(req, session=session, measured=k > 0)
        res = srv.drain([rid])[rid]
        wall.append((time.perf_counter() - t0) * 1e3)
        lat.append(res["latency_ms"])
        infos.append(res["info"])
        u0 = np.array(res["u"][0][0], dtype=float)
        v_pred = np.array(res["x"][0][1, 3:6], dtype=float)
        w = world.wind(x[:3], draws["wind"][k])
        x = world.plant_step(x, u0, h, w)
        d_hat = d_hat + K_OBS * (x[3:6] - v_pred) / h
        xs.append(x.copy())
        us.append(u0)
        ds.append(d_hat.copy())
    return dict(x=np.array(xs), u=np.array(us), d_hat=np.array(ds), wall_ms=np.array(wall),
                latency_ms=np.array(lat), info=infos)

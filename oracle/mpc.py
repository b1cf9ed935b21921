"""Closed-loop scenario-robust MPC around the oracle solver (Sec. IV-A.4).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Per MPC step k (the paper's loop, with the readings stated here):
  1. the S scenario problems start at the measured plant state and carry the disturbance
     estimate d_k plus their scaled draws (the world module builds them);
  2. the first step is solved from the template's guess; every later one is warm-started by
     shifting the previous solution while keeping the measured initial state
     (``shift_warm_start(..., measured=True)``);
  3. the controller applies the shared first control of scenario 0 to the plant for one
     interval;
  4. a linear disturbance observer updates the estimate from the velocity mismatch between
     the measurement and scenario 0's predicted node-1 state:
        d_{k+1} = d_k + K_OBS (v_meas - v_pred) / h.
"""
from __future__ import annotations

import numpy as np

from .scp import init_traj, scp_group, shift_warm_start

K_OBS = 0.5


def closed_loop(world, template: dict, steps: int, draws: dict, params: dict) -> dict:
    """Run ``steps`` MPC steps; ``world`` is the environment module (scene, plant, wind).
    Returns the plant states (steps + 1, 6), applied controls (steps, 3), disturbance
    estimates (steps + 1, 3) and the per-step solver info of scenario 0."""
    x = np.concatenate([world.START, np.zeros(3)])
    d_hat = np.zeros(3)
    xs, us, ds, infos = [x.copy()], [], [d_hat.copy()], []
    prev = None
    h = template["h"]
    for k in range(steps):
        req = world.request(template, x, d_hat, draws["xi"][k])
        trajs = [init_traj(d) for d in req] if prev is None else shift_warm_start(prev, req, measured=True)
        info = scp_group(trajs, params)
        u0 = np.array(trajs[0].ubar[0], dtype=float)
        v_pred = np.array(trajs[0].xbar[1, 3:6], dtype=float)
        w = world.wind(x[:3], draws["wind"][k])
        x = world.plant_step(x, u0, h, w)
        d_hat = d_hat + K_OBS * (x[3:6] - v_pred) / h
        xs.append(x.copy())
        us.append(u0)
        ds.append(d_hat.copy())
        infos.append(info)
        prev = trajs
    return dict(x=np.array(xs), u=np.array(us), d_hat=np.array(ds), info=infos)

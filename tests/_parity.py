"""Helpers shared by the GPU parity tests: run the oracle step by step and compare node fields."""
from __future__ import annotations

import numpy as np

from oracle.admm import admm_run
from oracle.scp import _prepare, default_params, init_traj, scp_group

RHO1 = (1.0, 1.0, 1.0)


def rel_err(gpu, ref) -> float:
    """||gpu - ref||_inf / max(1, ||ref||_inf)."""
    gpu = np.asarray(gpu, dtype=float)
    ref = np.asarray(ref, dtype=float)
    if ref.size == 0:
        return 0.0
    return float(np.max(np.abs(gpu - ref)) / max(1.0, float(np.max(np.abs(ref)))))


def oracle_scp(insts, scp_iters, admm_iters, **kw):
    """Solve each group of instances with the oracle; returns the Traj objects (state included)."""
    p = default_params(scp_iters=scp_iters, admm_iters=admm_iters, **kw)
    trajs = [init_traj(d) for d in insts]
    i = 0
    infos = [None] * len(insts)
    while i < len(insts):
        j = i + 1
        if insts[i]["group"] >= 0:
            while j < len(insts) and insts[j]["group"] == insts[i]["group"]:
                j += 1
        info = scp_group(trajs[i:j], p)
        for k in range(i, j):
            infos[k] = info
        i = j
    return trajs, infos


def oracle_linearize_admm(inst, admm_iters, rho=RHO1):
    t = init_traj(inst)
    packs = _prepare([t], inst["delta"], rho)
    admm_run(packs, rho, admm_iters)
    return t


FIELDS = ("x", "u", "z", "lam", "mu", "copy", "dual", "xbar", "ubar")


def gpu_fields(prob, names=FIELDS):
    return {k: prob.field(k).cpu().numpy() for k in names}


def compare(prob, f, insts, trajs, idx=None):
    """Worst relative error per block over the given trajectories (idx: positions in prob)."""
    idx = list(range(len(insts))) if idx is None else idx
    worst = {}
    for ti, d, t in zip(idx, insts, trajs):
        nx, nu = d["nx"], d["nu"]
        st = t.state
        cp = np.concatenate(st.copy, axis=1)
        du = np.concatenate(st.dual, axis=1)
        C = cp.shape[1]
        pairs = dict(x=(prob.split(f["x"], ti, nx), st.x), u=(prob.split(f["u"], ti, nu, True), st.u),
                     z=(prob.split(f["z"], ti, nx), st.z), lam=(prob.split(f["lam"], ti, nx), st.lam),
                     mu=(prob.split(f["mu"], ti, nx), st.mu), copy=(prob.split(f["copy"], ti, C), cp),
                     dual=(prob.split(f["dual"], ti, C), du), xbar=(prob.split(f["xbar"], ti, nx), t.xbar),
                     ubar=(prob.split(f["ubar"], ti, nu, True), t.ubar))
        for k, (g, o) in pairs.items():
            if k in f:
                worst[k] = max(worst.get(k, 0.0), rel_err(g, o))
    return worst

"""The converged-solution bar on the 6-DOF quadrotor batch at its goodput setting.

Workload: the 1000 6-DOF quadrotor instances of the scalability batch (Sec. IV-A.3: N = 40, three
obstacles, noise-initialized), solved in FP32 exactly as the benchmark times them: resident ADMM,
50 SCP x 300 ADMM iterations, rho 10 -> 3e4 geometric over the SCP iterations (Sec. IV-A.2), and
the trust-region ratio test of the SCP step (accept when the actual/predicted merit ratio is
positive, radius halved below 0.25, doubled above 0.75 up to 4).  Expected values: the FP64
oracle's final cost and max dynamics defect of the first 256 instances
(tests/golden/quad6_1000_converged.json, written by tests/golden/make_converged.py --workload
quad6_1000, which calls only the oracle).

An instance passes when the oracle and the GPU both reach max defect <= 1e-5 and the GPU's cost is
within 1e-3 relative of the oracle's.  The FP32 pass rate is reported and held to a floor; every
FP32 miss among the oracle-converged instances is re-run in FP64 mode, where the cost must agree to
COST_TOL64 and the defect bound must hold.
"""
import json
import os

import numpy as np
import pytest

import scpgen

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
DEFECT = 1e-5
COST_TOL = 1e-3
COST_TOL64 = 1e-10       # FP64 mode against the FP64 oracle: measured 2.5e-12 on the FP32 misses
FP32_MIN_PASS = 0.88     # measured 177 of 197


@pytest.fixture(scope="module")
def B(lib):
    from paper_2603_10711_amd import binding
    return binding


@pytest.fixture(scope="module")
def golden():
    with open(os.path.join(HERE, "golden", "quad6_1000_converged.json")) as fh:
        g = json.load(fh)
    s = g["setting"]
    cost = np.array([r["cost"] for r in g["instances"]])
    defect = np.array([r["defect"] for r in g["instances"]])
    return s, cost, defect


def _solve(B, insts, prec, s):
    s = dict(s)
    k, j, rho = s.pop("scp_iters"), s.pop("admm_iters"), s.pop("rho")
    prob = B.Problem(insts, precision=prec)
    prob.solve(B.scp_params(k, j, rho=rho, form="persistent", **s))
    info = prob.result()[2].cpu().numpy()
    prob.close()
    return info


def _passes(info, cost_o, def_o, tol):
    rel = np.abs(info[:, 7] - cost_o) / np.abs(cost_o)
    ok = (def_o <= DEFECT) & (info[:, 6] <= DEFECT) & (rel <= tol)
    return ok, rel


def test_quad6_fp32_converged_cost_and_defect(B, golden):
    s, cost_o, def_o = golden
    n = len(cost_o)
    insts = scpgen.config5(1000)
    conv_o = def_o <= DEFECT
    print(f"setting {s}; oracle defect <= 1e-5 on {int(np.sum(conv_o))}/{n}", flush=True)
    info = _solve(B, insts, "f32", s)
    print(f"GPU FP32 defect <= 1e-5 on {int(np.sum(info[:, 6] <= DEFECT))}/1000", flush=True)
    ok, rel = _passes(info[:n], cost_o, def_o, COST_TOL)
    rate = float(np.sum(ok)) / float(np.sum(conv_o))
    print(f"FP32 pass rate {int(np.sum(ok))}/{int(np.sum(conv_o))} = {rate:.4f}; cost rel diff over the "
          f"oracle-converged p50 {np.median(rel[conv_o]):.2e} max {rel[conv_o].max():.2e}", flush=True)
    miss = [i for i in range(n) if conv_o[i] and not ok[i]]
    print("FP32 misses (instance, cost rel diff, GPU defect, oracle defect): "
          f"{[(i, float(rel[i]), float(info[i, 6]), float(def_o[i])) for i in miss]}", flush=True)
    if miss:
        info64 = _solve(B, [insts[i] for i in miss], "f64", s)
        ok64, rel64 = _passes(info64, cost_o[miss], def_o[miss], COST_TOL64)
        print(f"FP64 re-run of the misses: cost rel diff max {rel64.max():.2e}, defects "
              f"{[float(v) for v in info64[:, 6]]}", flush=True)
        assert np.all(ok64), [(miss[k], rel64[k], info64[k, 6]) for k in range(len(miss)) if not ok64[k]]
    assert rate >= FP32_MIN_PASS

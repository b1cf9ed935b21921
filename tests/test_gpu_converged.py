"""The converged-solution bar: GPU solutions of the full quadrotor batch against the oracle's.

Workload: the 1024 point-mass quadrotor instances (N = 50, 8 obstacles), solved with the
geometric penalty schedule of the paper's parameter study (Sec. IV-A.2) from 5 to 1e4 over 20 SCP
iterations of 300 ADMM iterations, in the persistent form, exactly as the benchmark times it.
Expected values: the FP64 oracle's final cost and max dynamics defect of every instance
(tests/golden/quad1024_converged.json, written by tests/golden/make_converged.py, which calls only
the oracle).

An instance passes when the oracle and the GPU both reach max defect <= 1e-5 and the GPU's cost is
within 1e-3 relative of the oracle's.  The FP32 pass rate over the batch is reported and held to a
floor; every FP32 miss among the oracle-converged instances is re-run in FP64 mode, where the cost
must agree to COST_TOL64 (rounding order only) and the defect bound must hold.  The FP64 mode is
also checked over the whole batch.
"""
import json
import os

import numpy as np
import pytest

import scpgen

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
DEFECT = 1e-5
COST_TOL = 1e-3          # converged cost, relative
COST_TOL64 = 1e-10       # FP64 mode against the FP64 oracle: rounding-order differences only (measured 4e-15)
FP32_MIN_PASS = 0.99     # measured 1019 of 1019


@pytest.fixture(scope="module")
def B(lib):
    from paper_2603_10711_amd import binding
    return binding


@pytest.fixture(scope="module")
def golden():
    with open(os.path.join(HERE, "golden", "quad1024_converged.json")) as fh:
        g = json.load(fh)
    s = g["setting"]
    cost = np.array([r["cost"] for r in g["instances"]])
    defect = np.array([r["defect"] for r in g["instances"]])
    return s, cost, defect


def _solve(B, insts, prec, s):
    prob = B.Problem(insts, precision=prec)
    prob.solve(B.scp_params(s["scp_iters"], s["admm_iters"], rho=s["rho"], rho_final=s["rho_final"]))
    info = prob.result()[2].cpu().numpy()
    prob.close()
    return info


def _passes(info, cost_o, def_o, tol):
    rel = np.abs(info[:, 7] - cost_o) / np.abs(cost_o)
    ok = (def_o <= DEFECT) & (info[:, 6] <= DEFECT) & (rel <= tol)
    return ok, rel


def test_fp32_converged_cost_and_defect(B, golden):
    s, cost_o, def_o = golden
    insts = scpgen.config1(1024)
    print(f"setting {s}; oracle defect <= 1e-5 on {int(np.sum(def_o <= DEFECT))}/1024", flush=True)
    info = _solve(B, insts, "f32", s)
    ok, rel = _passes(info, cost_o, def_o, COST_TOL)
    conv_o = def_o <= DEFECT
    rate = float(np.sum(ok)) / float(np.sum(conv_o))
    print(f"FP32 pass rate {int(np.sum(ok))}/{int(np.sum(conv_o))} = {rate:.4f}; cost rel diff p50 "
          f"{np.median(rel):.2e} max {rel.max():.2e}; GPU defect <= 1e-5 on {int(np.sum(info[:, 6] <= DEFECT))}/1024",
          flush=True)
    assert rate >= FP32_MIN_PASS
    # FP32 misses among the instances the oracle converges: FP64 mode must reproduce the oracle
    miss = [i for i in range(1024) if conv_o[i] and not ok[i]]
    print(f"FP32 misses: {miss}", flush=True)
    if miss:
        info64 = _solve(B, [insts[i] for i in miss], "f64", s)
        ok64, rel64 = _passes(info64, cost_o[miss], def_o[miss], COST_TOL64)
        print(f"FP64 re-run of the misses: cost rel diff max {rel64.max():.2e}", flush=True)
        assert np.all(ok64), [(miss[k], rel64[k], info64[k, 6]) for k in range(len(miss)) if not ok64[k]]


def test_fp64_converged_cost_whole_batch(B, golden):
    s, cost_o, def_o = golden
    insts = scpgen.config1(1024)
    info = _solve(B, insts, "f64", s)
    rel = np.abs(info[:, 7] - cost_o) / np.abs(cost_o)
    dd = np.abs(info[:, 6] - def_o)
    print(f"FP64: cost rel diff p50 {np.median(rel):.2e} max {rel.max():.2e} (argmax {int(rel.argmax())}); "
          f"defect abs diff max {dd.max():.2e}", flush=True)
    assert np.all(rel <= COST_TOL64)
    # same verdict on the defect bound wherever the oracle is not within 5 % of it
    clear = np.abs(def_o - DEFECT) > 0.05 * DEFECT
    assert np.array_equal((info[:, 6] <= DEFECT)[clear], (def_o <= DEFECT)[clear])

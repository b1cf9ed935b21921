"""Lanes per node in the persistent form: lane groups of four for the point-mass quadrotor and the
3-DOF powered descent (scp_params.lanes_per_node = 4).

The four lanes of a DPP quad share one node: each owns some state and control components, their
rows of the factor and their columns of A and B; the triangular solves broadcast within the quad
and the ADMM iterations of an SCP iteration stay resident in one workgroup per trajectory.  The
sums run in another order than with one lane per node, so the bar is the oracle's (FP64 1e-9,
FP32 1e-4 where the iteration is well conditioned) and, at the full budget, the converged-solution
bar of the batch (cost within 1e-3 of the oracle's, defect <= 1e-5).
"""
import json
import os

import numpy as np
import pytest

import scpgen
from _parity import compare, gpu_fields, oracle_scp

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def B(lib):
    from paper_2603_10711_amd import binding
    return binding


def _ragged():
    out = [scpgen.quad_instance(14, i, N=5 + (11 * i) % 59, K=i % 9) for i in range(7)]
    out += [scpgen.mars_instance(14, i, N=8 + 17 * i) for i in range(4)]      # N up to 59
    out += [scpgen.quad_instance(14, 50, N=1, K=0), scpgen.quad_instance(14, 51, N=63, K=8)]
    return out


@pytest.mark.parametrize("prec,tol", [("f64", 1e-9), ("f32", 1e-4)])
def test_lane_groups_match_oracle(B, prec, tol):
    insts = _ragged()
    _say(prec, [d["N"] for d in insts])
    prob = B.Problem(insts, precision=prec)
    prob.solve(B.scp_params(2, 30, rho=2.0, lanes_per_node=4))
    f = gpu_fields(prob)
    trajs, _ = oracle_scp(insts, 2, 30, rho_eq=2.0, rho_dyn=2.0, rho_geo=2.0)
    worst = compare(prob, f, insts, trajs)
    _say(worst)
    assert max(worst.values()) < tol
    prob.close()


def test_lane_groups_schedule_fp64(B):
    """Penalty schedule and several SCP iterations on the powered descent and the quadrotor."""
    insts = [scpgen.quad_instance(15, 0, N=50, K=8), scpgen.mars_instance(15, 2, N=60)]
    prob = B.Problem(insts, precision="f64")
    prob.solve(B.scp_params(5, 60, rho=5.0, rho_final=1e3, lanes_per_node=4))
    f = gpu_fields(prob)
    info = prob.result()[2].cpu().numpy()
    trajs, oinfo = oracle_scp(insts, 5, 60, rho_eq=5.0, rho_dyn=5.0, rho_geo=5.0, rho_final=1e3)
    worst = compare(prob, f, insts, trajs)
    _say(worst)
    assert max(worst.values()) < 1e-9
    assert np.all(info[:, 0] == 300) and np.all(info[:, 3] == 5)
    prob.close()


def test_lane_groups_full_batch_converged(B):
    """The quadrotor batch at the benchmark's setting with lane groups of four, against the oracle's
    converged solutions (cost within 1e-3, defect <= 1e-5 on both)."""
    with open(os.path.join(HERE, "golden", "quad1024_converged.json")) as fh:
        g = json.load(fh)
    s = g["setting"]
    cost_o = np.array([r["cost"] for r in g["instances"]])
    def_o = np.array([r["defect"] for r in g["instances"]])
    insts = scpgen.config1(1024)
    prob = B.Problem(insts, precision="f32")
    prob.solve(B.scp_params(s["scp_iters"], s["admm_iters"], rho=s["rho"], rho_final=s["rho_final"],
                            lanes_per_node=4))
    info = prob.result()[2].cpu().numpy()
    prob.close()
    rel = np.abs(info[:, 7] - cost_o) / np.abs(cost_o)
    ok = (def_o <= 1e-5) & (info[:, 6] <= 1e-5) & (rel <= 1e-3)
    rate = float(ok.sum()) / float((def_o <= 1e-5).sum())
    _say(f"lanes 4: FP32 pass rate {int(ok.sum())}/{int((def_o <= 1e-5).sum())} = {rate:.4f}")
    assert rate >= 0.97
    assert np.all(info[:, 0] == s["scp_iters"] * s["admm_iters"])


def test_lane_group_refusals(B):
    short = [scpgen.quad_instance(16, 0, N=20, K=2)]
    prob = B.Problem(short, precision="f32")
    with pytest.raises(B.ScpError, match="fixed ADMM budgets"):
        prob.solve(B.scp_params(1, 10, check_every=5, eps=1e-4, lanes_per_node=4))
    with pytest.raises(B.ScpError, match="lanes_per_node"):
        prob.solve(B.scp_params(1, 10, lanes_per_node=3))
    prob.close()
    long = [scpgen.quad_instance(16, 1, N=64, K=2)]
    prob = B.Problem(long, precision="f32")
    with pytest.raises(B.ScpError, match="at most 64 nodes"):
        prob.solve(B.scp_params(1, 10, lanes_per_node=4))
    prob.solve(B.scp_params(1, 10, lanes_per_node=1))
    prob.close()
    grp = scpgen.config4_request(3, S=3, N=20)
    prob = B.Problem(grp, precision="f32")
    with pytest.raises(B.ScpError, match="consensus groups"):
        prob.solve(B.scp_params(1, 10, lanes_per_node=4))
    prob.close()
    six = [scpgen.quad6_benchmark_instance(0, N=10)]
    prob = B.Problem(six, precision="f32")
    with pytest.raises(B.ScpError, match="one lane per node"):
        prob.solve(B.scp_params(1, 10, rho=100.0, lanes_per_node=1))
    prob.solve(B.scp_params(1, 10, rho=100.0, lanes_per_node=4))     # the 6-DOF default
    prob.close()


def test_autotune_sweeps_lanes_per_node(B):
    insts = [scpgen.quad_instance(17, i, N=30 + i, K=8) for i in range(24)]
    prm = B.scp_params(2, 40, rho=5.0)
    best, table = B.autotune(insts, prm, cadences=(0,), reps=1)
    _say(best, table)
    four = [e for e in table if e["lanes_per_node"] == 4]
    one = [e for e in table if e["lanes_per_node"] == 1]
    assert len(four) == 1 and four[0]["valid"] and four[0]["block"] == 256
    assert len(one) == 5 and all(e["valid"] for e in one)
    assert best["ms"] == min(e["ms"] for e in table if e["valid"])

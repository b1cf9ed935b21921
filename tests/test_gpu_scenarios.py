"""Scenario consensus groups in the persistent kernel, inside one workgroup and spanning several
(16-scenario robust-MPC requests with N up to 80, and the largest group, 64 members).

A spanning group exchanges its member values through HBM with a group barrier, summing over
members in member order exactly as a group held by one workgroup does, so the two placements
are compared bit for bit; both are compared with the FP64 oracle in FP64 mode (1e-9) and with
FP32 mode at a short budget (1e-4).
"""
import numpy as np
import pytest

import scpgen
from _parity import compare, gpu_fields, oracle_scp

pytestmark = pytest.mark.gpu

TOL64 = 1e-9
TOL32 = 1e-4


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def B(lib):
    from paper_2603_10711_amd import binding
    return binding


def _batch():
    """A 4-scenario group of 41-node quadrotors between independent trajectories."""
    req = scpgen.config4_request(7, S=4, N=40)
    other = [scpgen.quad_instance(4, 500 + i, N=15 + 4 * i, K=4) for i in range(3)]
    return other[:1] + req + other[1:]


def test_spanning_group_equals_single_workgroup_fp32(B):
    insts = _batch()
    prm = B.scp_params(3, 40, check_every=5, eps=1e-4, rho=3.0)
    out = {}
    for block in (256, 128, 64):
        pl = B.plan(insts, block=block)
        _say("block", block, pl)
        assert pl["spanning"] == (0 if block == 256 else 1)
        prob = B.Problem(insts, precision="f32", block=block)
        prob.solve(prm)
        out[block] = [a.cpu().numpy() for a in prob.result()]
        info = out[block][2]
        assert not np.any(info[:, 5].astype(np.int64) & B.ST_SYNC)
        prob.close()
    for block in (128, 64):
        for a, b in zip(out[block], out[256]):
            np.testing.assert_array_equal(a, b)


def test_spanning_group_fp64_matches_oracle(B):
    insts = _batch()
    kw = dict(check_every=5, eps_p=1e-4, eps_d=1e-4, rho_eq=3.0, rho_dyn=3.0, rho_geo=3.0)
    trajs, oinfo = oracle_scp(insts, 3, 40, **kw)
    res = []
    for block in (128, 64):
        _say("fp64 spanning, block", block)
        prob = B.Problem(insts, precision="f64", block=block)
        prob.solve(B.scp_params(3, 40, check_every=5, eps=1e-4, rho=3.0))
        f = gpu_fields(prob)
        worst = compare(prob, f, insts, trajs)
        _say(worst)
        assert max(worst.values()) < TOL64
        _, _, info = prob.result()
        inf = prob.info_dicts(info.cpu().numpy())
        assert [i["admm_iters"] for i in inf] == [o["admm_iters"] for o in oinfo]
        res.append(f)
        prob.close()
    for k in res[0]:
        np.testing.assert_array_equal(res[0][k], res[1][k])


def test_sixteen_scenario_request_fp64(B):
    """A robust-MPC request as served: 16 scenarios, N = 30, first control shared."""
    req = scpgen.config4_request(2, S=16, N=30)
    trajs, _ = oracle_scp(req, 2, 30)
    prob = B.Problem(req, precision="f64")
    pl = B.plan(req, precision="f64")
    _say("16 scenarios fp64", pl)
    assert pl["spanning"] == 1
    prob.solve(B.scp_params(2, 30))
    f = gpu_fields(prob)
    worst = compare(prob, f, req, trajs)
    _say(worst)
    assert max(worst.values()) < TOL64
    u0 = [f["copy"][prob.offsets[m], 6:12] for m in range(16)]
    for v in u0[1:]:
        np.testing.assert_array_equal(v, u0[0])
    prob.close()


@pytest.mark.parametrize("N", [50, 80])
def test_sixteen_scenario_request_fp32(B, N):
    req = scpgen.config4_request(3, S=16, N=N)
    trajs, _ = oracle_scp(req, 1, 100)
    got = {}
    for form in ("persistent", "plain"):
        prob = B.Problem(req, precision="f32")
        prob.solve(B.scp_params(1, 100, form=form))
        got[form] = gpu_fields(prob)
        worst = compare(prob, got[form], req, trajs)
        _say("16 scenarios fp32", N, form, B.plan(req), worst)
        assert max(worst.values()) < TOL32
        _, _, info = prob.result()
        assert not np.any(info.cpu().numpy()[:, 5].astype(np.int64) & B.ST_SYNC)
        prob.close()


def test_largest_spanning_group_fp64_matches_oracle(B):
    """The largest group the persistent form takes, 64 members, spread over 13 workgroups of 64
    lanes (five 11-node members per wavefront): every barrier exchanges all 64 member rows
    (scenario mean of the nominal, first-control copies, residual test, merit), FP64 against the
    oracle to 1e-9 with the residual test on, and the ADMM iteration counts exactly."""
    req = scpgen.config4_request(21, S=64, N=10)
    insts = [scpgen.quad_instance(4, 600, N=12, K=2)] + req
    pl = B.plan(insts, block=64)
    _say("64-member group", pl)
    assert pl["spanning"] == 1
    kw = dict(check_every=5, eps_p=1e-4, eps_d=1e-4, rho_eq=3.0, rho_dyn=3.0, rho_geo=3.0)
    trajs, oinfo = oracle_scp(insts, 2, 30, **kw)
    prob = B.Problem(insts, precision="f64", block=64)
    prob.solve(B.scp_params(2, 30, check_every=5, eps=1e-4, rho=3.0))
    f = gpu_fields(prob)
    worst = compare(prob, f, insts, trajs)
    _say(worst)
    assert max(worst.values()) < TOL64
    _, _, info = prob.result()
    inf = prob.info_dicts(info.cpu().numpy())
    assert [i["admm_iters"] for i in inf] == [o["admm_iters"] for o in oinfo]
    assert not np.any(info.cpu().numpy()[:, 5].astype(np.int64) & B.ST_SYNC)
    prob.close()

"""GPU parity of the adaptive penalty (residual balancing between SCP iterations) against the
FP64 oracle, through the C ABI: every node block at 1e-9 in FP64 mode (plain form, persistent
form in one launch and split into one launch per SCP iteration, the 6-DOF resident ADMM), at
1e-4 in FP32 mode on short budgets; the cases are chosen so the oracle's factor moves (the
penalty starts far too small or too large).  Arguments the rule does not support are errors."""
import numpy as np
import pytest

import scpgen
from _parity import compare, gpu_fields, oracle_scp
from test_gpu_quad6 import _fields as quad6_fields

pytestmark = pytest.mark.gpu

TOL64 = 1e-9
TOL32 = 1e-4


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def B(lib):
    from paper_2603_10711_amd import binding
    return binding


def _mixed(seed):
    out = []
    for i in range(5):
        N = 6 + (5 * i) % 17
        out.append(scpgen.quad_instance(9, seed + i, N=N, K=i % 5, T=0.1 * N + 1.0))
    return out + [scpgen.mars_instance(2, seed, N=14), scpgen.mars_instance(2, seed + 1, N=9)]


def _moved(oinfo):
    return sum(1 for i in oinfo if i["rho_scale"] != 1.0)


CASES = [
    ("small", dict(rho=1e-2), dict(rho_eq=1e-2, rho_dyn=1e-2, rho_geo=1e-2), 10.0, 2.0),
    ("schedule", dict(rho=100.0, rho_final=1e4), dict(rho_eq=100.0, rho_dyn=100.0, rho_geo=100.0, rho_final=1e4),
     5.0, 1.5),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("form,per_launch", [("plain", 0), ("persistent", 0), ("persistent", 1)])
def test_adaptive_penalty_fp64(B, case, form, per_launch):
    name, gkw, okw, mu, tau = case
    insts = _mixed(70)
    K, J = 5, 40
    trajs, oinfo = oracle_scp(insts, K, J, adapt_mu=mu, adapt_tau=tau, **okw)
    assert _moved(oinfo) >= len(insts) // 2, [i["rho_scale"] for i in oinfo]
    _say("adapt", name, form, per_launch, [i["rho_scale"] for i in oinfo])
    prob = B.Problem(insts, precision="f64")
    prob.solve(B.scp_params(K, J, form=form, scp_per_launch=per_launch, adapt_mu=mu, adapt_tau=tau, **gkw))
    worst = compare(prob, gpu_fields(prob), insts, trajs)
    _say(worst)
    assert max(worst.values()) < TOL64
    _, _, info = (t.cpu().numpy() for t in prob.result())
    for t, o in enumerate(oinfo):
        assert abs(info[t, 1] - o["r_p"]) <= TOL64 * max(1.0, abs(o["r_p"]))
        assert abs(info[t, 2] - o["r_d"]) <= TOL64 * max(1.0, abs(o["r_d"]))
    prob.close()


@pytest.mark.parametrize("form", ["plain", "persistent"])
def test_adaptive_penalty_fp32_short_budget(B, form):
    insts = scpgen.config1(4) + [scpgen.mars_instance(2, 5, N=60)]
    K, J = 3, 50
    trajs, oinfo = oracle_scp(insts, K, J, rho_eq=1e-2, rho_dyn=1e-2, rho_geo=1e-2, adapt_mu=10.0)
    assert _moved(oinfo) == len(insts)
    _say("adapt fp32", form)
    prob = B.Problem(insts, precision="f32")
    prob.solve(B.scp_params(K, J, rho=1e-2, form=form, adapt_mu=10.0))
    worst = compare(prob, gpu_fields(prob), insts, trajs)
    _say(worst)
    assert max(worst.values()) < TOL32
    prob.close()


@pytest.mark.parametrize("model", ["quad6", "lander6"])
@pytest.mark.parametrize("form", ["plain", "persistent"])
def test_adaptive_penalty_6dof_fp64(B, model, form):
    if model == "quad6":
        insts = [scpgen.quad6_benchmark_instance(i, N=8 + 3 * i) for i in range(3)]
        rho = 1e-2
    else:
        insts = [scpgen.lander6_perturbed(i) for i in range(3)]
        rho = 1e4
    K, J = 3, 30
    trajs, oinfo = oracle_scp(insts, K, J, rho_eq=rho, rho_dyn=rho, rho_geo=rho, adapt_mu=10.0)
    assert _moved(oinfo) >= 2, [i["rho_scale"] for i in oinfo]
    _say("adapt 6dof", model, form, [i["rho_scale"] for i in oinfo])
    prob = B.Problem(insts, precision="f64")
    prob.solve(B.scp_params(K, J, rho=rho, form=form, adapt_mu=10.0))
    # the 6-DOF quadrotor keeps the point mass's (empty) ball slots, which the oracle does not have
    f = quad6_fields(prob) if model == "quad6" else gpu_fields(prob)
    worst = compare(prob, f, insts, trajs)
    _say(worst)
    assert max(worst.values()) < TOL64
    prob.close()


def test_adaptive_penalty_refusals(B):
    insts = scpgen.config1(2)
    prob = B.Problem(insts, precision="f32")
    for kw in (dict(adapt_mu=0.5), dict(adapt_mu=10.0, adapt_tau=1.0), dict(adapt_mu=float("inf"))):
        with pytest.raises(RuntimeError, match="adapt"):
            prob.solve(B.scp_params(2, 10, **kw))
    with pytest.raises(RuntimeError, match="fixed budgets"):
        prob.solve(B.scp_params(2, 10, check_every=5, eps=1e-4, adapt_mu=10.0))
    prob.solve(B.scp_params(2, 10, adapt_mu=10.0))   # still usable
    prob.close()
    one = scpgen.config1(1)[0]
    grp = [dict(one, group=0) for _ in range(2)]
    gp = B.Problem(grp, precision="f32")
    with pytest.raises(RuntimeError, match="consensus groups"):
        gp.solve(B.scp_params(2, 10, adapt_mu=10.0))
    gp.close()


def test_solve_after_adaptive_solve_starts_from_factor_one(B):
    """Each scp_solve starts from factor 1: an adaptive solve leaves no trace in a later one."""
    insts = _mixed(90)
    fresh = B.Problem(insts, precision="f64")
    fresh.solve(B.scp_params(3, 30, rho=1e-2, form="plain", adapt_mu=10.0))
    want = gpu_fields(fresh)
    fresh.close()
    prob = B.Problem(insts, precision="f64")
    prob.solve(B.scp_params(4, 30, rho=1e-2, form="plain", adapt_mu=10.0))
    prob.reset()
    prob.solve(B.scp_params(3, 30, rho=1e-2, form="plain", adapt_mu=10.0))
    got = gpu_fields(prob)
    for k in want:
        np.testing.assert_array_equal(got[k], want[k])
    prob.close()

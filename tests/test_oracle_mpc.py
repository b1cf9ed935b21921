"""Pins of the oracle's MPC warm start (receding-horizon shift of a session's previous solution).

The shift has no formula in the paper; what pins it:
  * alignment: shifting a dynamically feasible rollout keeps intervals 0..N-2 exactly feasible
    (a state/control index offset would break every interval);
  * receding horizon: the new x_init is the previous scenario-0 state at node 1, so the shifted
    scenario-0 nominal meets the new boundary condition exactly;
  * duals stay consistent with the constraint groups of the next problem (zero where a group
    does not exist, no dynamic-coupling duals at node 0), and a shifted steady state is a steady
    state;
  * a warm-started session request ends closer to its solution than a cold start of the same
    problem at the same small budget.
"""
import numpy as np
import pytest

import oracle
import scpgen
from oracle.scp import _prepare, scp_group, shift_warm_start, mpc_session, init_traj

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _rollout(inst, rng):
    """A dynamically feasible trajectory from x_init under random bounded controls."""
    N, nu = inst["N"], inst["nu"]
    u = rng.uniform(-3.0, 3.0, size=(N, nu))
    if inst["model"] == scpgen.MARS:
        u[:, 3] = np.linalg.norm(u[:, :3], axis=1) + 0.3
    x = np.zeros((N + 1, inst["nx"]))
    x[0] = inst["x_init"]
    for i in range(N):
        x[i + 1] = oracle.rk4(inst, x[i], u[i])
    return x, u


@pytest.mark.parametrize("model", ["quad", "mars"])
def test_shift_keeps_rollout_feasible(model):
    rng = np.random.default_rng(5)
    inst = scpgen.quad_instance(4, 3, N=12, K=4) if model == "quad" else scpgen.mars_instance(2, 3, N=12)
    t = init_traj(inst)
    t.xbar, t.ubar = _rollout(inst, rng)
    (nt,) = shift_warm_start([t])
    for i in range(inst["N"] - 1):
        np.testing.assert_array_equal(oracle.rk4(inst, nt.xbar[i], nt.ubar[i]), nt.xbar[i + 1])
    # the receding horizon: the new start is the old node 1, and the nominal starts there
    np.testing.assert_array_equal(nt.inst["x_init"], t.xbar[1])
    np.testing.assert_array_equal(nt.xbar[0], nt.inst["x_init"])
    # the previous instance is untouched
    np.testing.assert_array_equal(inst["x_init"], scpgen.quad_instance(4, 3, N=12, K=4)["x_init"]
                                  if model == "quad" else scpgen.mars_instance(2, 3, N=12)["x_init"])


def test_all_scenarios_take_scenario0_start():
    req = scpgen.config4_request(5, S=3, N=8)
    rng = np.random.default_rng(1)
    trajs = []
    for d in req:
        t = init_traj(d)
        t.xbar, t.ubar = _rollout(d, rng)
        trajs.append(t)
    new = shift_warm_start(trajs)
    for nt in new:
        np.testing.assert_array_equal(nt.inst["x_init"], trajs[0].xbar[1])


def _solved(inst, scp_iters=2, admm_iters=40):
    t = init_traj(inst)
    scp_group([t], oracle.default_params(scp_iters=scp_iters, admm_iters=admm_iters))
    return t


def test_shifted_duals_fit_the_next_problem():
    inst = scpgen.quad_instance(4, 11, N=10, K=3)
    t = _solved(inst)
    assert any(np.any(d != 0) for d in t.state.dual)
    (nt,) = shift_warm_start([t])
    st = nt.state
    assert np.all(st.lam[0] == 0) and np.all(st.mu[0] == 0)
    for g, d in zip(nt.groups, st.dual):
        assert np.all(d[~g.active] == 0.0)
        assert d.shape == (inst["N"] + 1, len(g.comps))
    # the next problem accepts the state as is (same group layout, finite everything)
    packs = _prepare([nt], inst["delta"], (1.0, 1.0, 1.0))
    assert len(packs) == 1 and all(np.all(np.isfinite(d)) for d in nt.state.dual)


def test_steady_state_is_a_fixed_point():
    """Constant rows stay constant: shifting a trajectory whose every row is equal changes
    nothing but the zeroed node-0 coupling duals."""
    inst = scpgen.quad_instance(4, 12, N=6, K=0)
    t = _solved(inst, 1, 5)
    N = inst["N"]
    c = np.arange(1, inst["nx"] + 1, dtype=float)
    t.xbar = np.tile(c, (N + 1, 1))
    t.ubar = np.tile(c[:3], (N, 1))
    t.state.lam = np.tile(c, (N + 1, 1))
    for g, d in zip(t.groups, t.state.dual):
        d[:] = 0.0
        d[g.active] = 2.0
    (nt,) = shift_warm_start([t])
    np.testing.assert_array_equal(nt.xbar, t.xbar)
    np.testing.assert_array_equal(nt.ubar, t.ubar)
    np.testing.assert_array_equal(nt.state.lam[1:], t.state.lam[1:])
    for d0, d1 in zip(t.state.dual, nt.state.dual):
        np.testing.assert_array_equal(d0, d1)


@pytest.mark.parametrize("session", [6, 7, 8])
def test_session_warm_start_beats_cold_start(session):
    """Second request of a session: warm start from the shifted solution against a cold start
    of the same problem (same x_init) at the same small budget (2 SCP x 50 ADMM): the warm
    start ends with a lower merit (cost + 1e3 x l1 dynamics defect), and both are finite."""
    from oracle.scp import _merit_terms
    reqs = [scpgen.config4_request(session, S=2, N=12) for _ in range(2)]
    (t0, _), = mpc_session(reqs[:1], oracle.default_params(scp_iters=5, admm_iters=100))
    x1 = t0[0].xbar[1]
    warm = shift_warm_start(t0, reqs[1])
    cold = [init_traj(dict(d, x_init=x1.copy())) for d in reqs[1]]
    p = oracle.default_params(scp_iters=2, admm_iters=50)
    scp_group(warm, p)
    scp_group(cold, p)

    def merit(ts):
        return sum(J + 1e3 * pen for J, pen in (_merit_terms(t.inst, t.xbar, t.ubar) for t in ts))

    assert np.isfinite(merit(warm)) and np.isfinite(merit(cold))
    assert merit(warm) < merit(cold)
    for t in warm:
        np.testing.assert_array_equal(t.inst["x_init"], x1)

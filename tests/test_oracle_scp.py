"""Pins for the oracle's SCP layer (Sec. III-A) and the reported metrics.

* the cost encoding reproduces the workloads' stated objectives;
* defect / violation / boundary error on constructed trajectories with known values;
* the linearized obstacle half-space is tangent to the sphere and excludes its interior;
* with affine (drag-free) dynamics one SCP step solves the convex subproblem: the ADMM
  output satisfies the subproblem's KKT conditions, checked set by set;
* nonlinear behaviour: defect and step shrink on a converging instance; the ratio test
  never accepts a merit increase; scenario groups of identical copies equal one instance;
* failure detection: the residual blow-up bit follows its rule (first positive residual of the
  solve as the reference, strictly above 1e6 times it) and is set when an indefinite cost makes
  ADMM diverge.
"""
import math

import numpy as np
import pytest

import scpgen
import oracle
from oracle import rk4
from oracle.scp import _prepare, init_traj, convexify, _merit_terms, scp_group
from oracle.admm import admm_run


def test_cost_encodings_match_workload_objectives():
    rng = np.random.default_rng(0)
    q = scpgen.quad_instance(0, 0, N=10)
    x = rng.normal(size=(11, 6))
    u = rng.normal(size=(10, 3)) * 4
    goal = q["x_target"]
    direct = float(np.sum(u ** 2) + 100.0 * np.sum((x[-1] - goal) ** 2))
    assert abs(oracle.cost(q, x, u) - direct) < 1e-9 * abs(direct)
    m = scpgen.mars_instance(2, 0, N=10)
    xm = rng.normal(size=(11, 7))
    um = rng.normal(size=(10, 4))
    assert oracle.cost(m, xm, um) == pytest.approx(-xm[-1, 6], abs=1e-15)


def test_defect_violation_boundary_on_constructed_trajectory():
    inst = scpgen.quad_instance(0, 1, N=8, K=2)
    rng = np.random.default_rng(1)
    u = rng.uniform(-3, 3, (8, 3)) + np.array([0, 0, 9.81])
    x = np.zeros((9, 6))
    x[0] = inst["x_init"]
    errs = np.zeros(8)
    for i in range(8):
        e = np.zeros(6)
        e[i % 6] = (-1) ** i * 1e-3 * (i + 1)
        errs[i] = abs(e[i % 6])
        x[i + 1] = rk4(inst, x[i], u[i]) + e
    assert oracle.defect(inst, x, u) == pytest.approx(errs.max(), rel=1e-12)
    assert oracle.boundary_error(inst, x) == 0.0
    x2 = x.copy()
    x2[0, 1] += 0.25
    assert oracle.boundary_error(inst, x2) == pytest.approx(0.25)
    # obstacle penetration: put node 3 at distance r/2 from an obstacle centre
    c, r = inst["obstacles"][0, :3], inst["obstacles"][0, 3]
    x3 = x.copy()
    x3[3, :3] = c + np.array([0.5 * r, 0, 0])
    u3 = np.zeros_like(u)
    assert oracle.violation(inst, x3, u3) >= 0.5 * r - 1e-12
    # control bound and ball: u = (16, 0, 0) violates |u| <= 15 by 1; u = (12,12,12) ball by sqrt(432)-20
    u4 = u3.copy()
    u4[2] = [16.0, 0, 0]
    x4 = x.copy()
    x4[1:, :3] = c + 10.0
    assert oracle.violation(inst, x4, u4) == pytest.approx(1.0)
    u4[2] = [12.0, 12.0, 12.0]
    assert oracle.violation(inst, x4, u4) == pytest.approx(math.sqrt(432.0) - 20.0)


def test_mars_terminal_and_cone_metrics():
    m = scpgen.mars_instance(2, 3, N=6)
    x = np.zeros((7, 7))
    x[0] = m["x_init"]
    x[:, 6] = 1.0
    x[1:6, 2] = 0.5
    x[-1, 3] = 0.02          # terminal velocity error
    assert oracle.boundary_error(m, x) == pytest.approx(0.02)
    x[2, 0] = 20.0           # ||r_xy|| = 20 > tan(86 deg) * 0.5
    u = np.zeros((6, 4))
    u[:, 3] = 0.3
    assert oracle.violation(m, x, u) == pytest.approx(20.0 - m["glide_tan"] * 0.5)


def test_obstacle_halfspace_is_tangent_and_safe():
    inst = scpgen.quad_instance(1, 5, N=20, K=8)
    rng = np.random.default_rng(2)
    xbar = inst["x_guess"] + 0.3 * rng.normal(size=inst["x_guess"].shape)
    groups = convexify(inst, xbar, inst["u_guess"], 1.0)
    hs = [g for g in groups if g.kind == "halfspace"]
    assert len(hs) == 8
    for j, g in enumerate(hs):
        c, r = inst["obstacles"][j, :3], inst["obstacles"][j, 3]
        assert not g.active[0] and np.all(g.active[1:])
        for i in range(1, inst["N"] + 1):
            a, b = g.a[i], g.b[i]
            assert abs(np.linalg.norm(a) - 1.0) < 1e-14
            tangent = c + r * a
            assert abs(a @ tangent - b) < 1e-12
            pts = c + rng.normal(size=(50, 3)) * 2
            inside = pts[a @ pts.T >= b]
            assert np.all(np.linalg.norm(inside - c, axis=1) >= r - 1e-12)


def test_convexify_boundary_boxes_and_trust_region():
    inst = scpgen.mars_instance(2, 1, N=10)
    xbar, ubar = inst["x_guess"], inst["u_guess"]
    groups = convexify(inst, xbar, ubar, 0.05)
    xb, ub = groups[0], groups[1]
    np.testing.assert_array_equal(xb.lo[0], inst["x_init"])
    np.testing.assert_array_equal(xb.hi[0], inst["x_init"])
    np.testing.assert_array_equal(xb.lo[-1, :6], 0.0)
    np.testing.assert_array_equal(xb.hi[-1, :6], 0.0)
    np.testing.assert_allclose(xb.hi[3] - xb.lo[3], 0.1)
    # Gamma trust box clipped by the hard thrust bounds
    assert np.all(ub.lo[:-1, 3] >= inst["u_lo"][3]) and np.all(ub.hi[:-1, 3] <= inst["u_hi"][3])
    assert [g.kind for g in groups] == ["box", "box", "cone", "soc"]
    # an empty trust/hard intersection collapses onto the nearest hard point
    ubar2 = ubar.copy()
    ubar2[4, 3] = 2.0
    g2 = convexify(inst, xbar, ubar2, 0.05)[1]
    assert g2.lo[4, 3] == g2.hi[4, 3] == inst["u_hi"][3]


def _kkt_check(traj, rho, tol):
    """KKT conditions of the convex subproblem at the ADMM output, using mu as the dynamics
    multipliers and each group's dual as its normal-cone element."""
    qp, groups, st = traj.qp, traj.groups, traj.state
    N = qp.N
    # primal feasibility
    np.testing.assert_allclose(st.x[1:], np.einsum("kij,kj->ki", qp.A, st.x[:N]) + np.einsum("kij,kj->ki", qp.B, st.u) + qp.d, atol=tol)
    gx = np.einsum("kij,kj->ki", qp.Q, st.x) + qp.q
    gx[:N] += np.einsum("kij,kj->ki", qp.M, st.u)
    gu = np.einsum("kij,kj->ki", qp.R, st.u) + qp.r + np.einsum("kij,ki->kj", qp.M, st.x[:N])
    gx[1:] += st.mu[1:]
    gx[:N] -= np.einsum("kij,ki->kj", qp.A, st.mu[1:])
    gu -= np.einsum("kij,ki->kj", qp.B, st.mu[1:])
    for gi, g in enumerate(groups):
        for i in np.nonzero(g.active)[0]:
            nu = st.dual[gi][i]
            y = (st.x[i] if g.var == "x" else st.u[i])[list(g.comps)]
            tgt = gx if g.var == "x" else gu
            tgt[i, list(g.comps)] += nu
            if g.kind == "box":
                assert np.all(y >= g.lo[i] - tol) and np.all(y <= g.hi[i] + tol)
                eqc = np.isclose(g.lo[i], g.hi[i])
                assert np.all((nu <= tol) | eqc | (np.abs(y - g.hi[i]) <= tol))
                assert np.all((nu >= -tol) | eqc | (np.abs(y - g.lo[i]) <= tol))
            elif g.kind == "halfspace":
                s = -(nu @ g.a[i])
                assert np.allclose(nu, -s * g.a[i], atol=tol) and s >= -tol
                assert g.a[i] @ y >= g.b[i] - tol
                assert s <= tol or abs(g.a[i] @ y - g.b[i]) <= tol
            elif g.kind == "ball":
                ny = np.linalg.norm(y)
                assert ny <= g.radius + tol
                t = (nu @ y) / max(ny * ny, 1e-30)
                assert np.allclose(nu, t * y, atol=tol) and t >= -tol
                assert t <= tol or abs(ny - g.radius) <= tol
    np.testing.assert_allclose(gx, 0.0, atol=tol)
    np.testing.assert_allclose(gu, 0.0, atol=tol)


def test_affine_scp_step_solves_convex_subproblem():
    inst = scpgen.quad_instance(0, 0, N=6, K=0, T=3.0, drag=0.0, delta=3.0)
    inst["x_init"] = np.zeros(6)
    inst["x_target"] = np.array([1.2, 0.5, 0.3, 0, 0, 0])
    inst["qn"] = -200.0 * inst["x_target"]
    inst["obstacles"] = np.array([[0.6, 0.25, 0.2, 0.3]])
    s = np.linspace(0, 1, 7)[:, None]
    inst["x_guess"] = np.hstack([s * inst["x_target"][:3], np.tile(inst["x_target"][:3] / 3.0, (7, 1))])
    inst["u_ball"] = 10.3
    rho = (1.0, 1.0, 1.0)
    t = init_traj(inst)
    packs = _prepare([t], inst["delta"], rho)
    it, rp, rd = admm_run(packs, rho, 30000, check_every=50, eps_p=1e-11, eps_d=1e-11)
    assert rp < 1e-9 and rd < 1e-9, (rp, rd)
    _kkt_check(t, rho, 1e-7)
    # the instance must exercise at least one inequality (obstacle, ball or trust box)
    hs = t.groups[3]
    act_h = np.any(np.abs(np.einsum("ij,ij->i", hs.a[1:], t.state.x[1:, :3]) - hs.b[1:]) < 1e-6)
    act_b = np.any(np.abs(np.linalg.norm(t.state.u, axis=1) - 10.3) < 1e-6)
    xb = t.groups[0]
    act_t = np.any(np.isclose(t.state.x[1:], xb.hi[1:], atol=1e-7) | np.isclose(t.state.x[1:], xb.lo[1:], atol=1e-7))
    assert act_h or act_b or act_t


def test_nonlinear_scp_converges_on_quadrotor():
    inst = scpgen.config0()[0]
    p = oracle.default_params(scp_iters=15, admm_iters=200, rho_eq=100.0, rho_dyn=100.0, rho_geo=100.0)
    sols, infos = oracle.scp_solve([inst], p)
    inf = infos[0]
    assert inf["defect"] < 1e-4 and inf["viol"] < 1e-4 and inf["bnd_err"] < 1e-4
    assert inf["n_accept"] == 15 and inf["status"] == 0


def test_ratio_test_never_accepts_a_merit_increase():
    inst = scpgen.quad_instance(1, 7, N=20, K=4)
    p = oracle.default_params(scp_iters=8, admm_iters=60, eta0=0.05, shrink=0.5, grow=2.0, delta_max=2.0)
    t = init_traj(inst)
    merits = []
    w = p["merit_w"]
    for k in range(p["scp_iters"]):
        J, pen = _merit_terms(inst, t.xbar, t.ubar)
        merits.append(J + w * pen)
        oracle.scp.scp_group([t], dict(p, scp_iters=1), delta=None)
    J, pen = _merit_terms(inst, t.xbar, t.ubar)
    merits.append(J + w * pen)
    assert all(b <= a + 1e-9 * abs(a) for a, b in zip(merits, merits[1:]))


def test_scenario_group_of_identical_copies_equals_single_instance():
    base = scpgen.quad_instance(4, 0, N=12, K=2)
    p = oracle.default_params(scp_iters=3, admm_iters=40)
    single, _ = oracle.scp_solve([dict(base, group=-1)], p)
    copies = [dict(base, group=7) for _ in range(3)]
    grouped, _ = oracle.scp_solve(copies, p)
    for xs, us in grouped:
        np.testing.assert_allclose(xs, single[0][0], atol=1e-11)
        np.testing.assert_allclose(us, single[0][1], atol=1e-11)
    one, _ = oracle.scp_solve([dict(base, group=3)], p)
    np.testing.assert_array_equal(one[0][0], single[0][0])


def test_scenario_group_shares_first_control_set():
    reqs = scpgen.config4_request(0, S=4, N=10)
    p = oracle.default_params(scp_iters=2, admm_iters=30)
    trajs = [init_traj(r) for r in reqs]
    for t in trajs:
        t.ubar[0] += np.random.default_rng(len(trajs)).normal(size=3) * 0.1
    _prepare(trajs, 1.0, (1.0, 1.0, 1.0))
    lo0 = [t.groups[1].lo[0] for t in trajs]
    for lo in lo0[1:]:
        np.testing.assert_array_equal(lo, lo0[0])


def test_penalty_schedule_factors():
    """Geometric schedule (parameter study of Sec. IV-A.2): factor 1 at the first SCP iteration,
    rho_final / rho at the last, constant ratio; no schedule gives ones."""
    from oracle.scp import penalty_factors
    f = penalty_factors(dict(scp_iters=20, rho_eq=100.0, rho_final=1e4))
    assert f[0] == 1.0 and abs(f[-1] - 100.0) < 1e-10
    r = np.array(f[1:]) / np.array(f[:-1])
    assert np.allclose(r, r[0], rtol=1e-13)
    assert penalty_factors(dict(scp_iters=5, rho_eq=3.0, rho_final=0.0)) == [1.0] * 5
    assert penalty_factors(dict(scp_iters=1, rho_eq=3.0, rho_final=50.0)) == [1.0]
    # rho_final equal to rho: exactly the fixed-penalty solver
    inst = scpgen.quad_instance(1, 3, N=8, K=2)
    a = init_traj(inst)
    b = init_traj(inst)
    scp_group([a], oracle.default_params(scp_iters=3, admm_iters=20, rho_eq=2.0, rho_dyn=2.0, rho_geo=2.0))
    scp_group([b], oracle.default_params(scp_iters=3, admm_iters=20, rho_eq=2.0, rho_dyn=2.0, rho_geo=2.0,
                                         rho_final=2.0))
    np.testing.assert_array_equal(a.xbar, b.xbar)
    np.testing.assert_array_equal(a.state.dual[3], b.state.dual[3])


def test_penalty_schedule_reaches_the_subproblem_kkt_point():
    """Affine dynamics, four SCP iterations with the penalties growing 1 -> 8: each subproblem's
    optimum does not depend on rho, so the last ADMM output (converged at rho = 8, with the duals
    carried from the smaller penalties and the factor rebuilt) satisfies the KKT conditions of
    the last subproblem.  A stale factor or duals rescaled with rho would leave a residual."""
    inst = scpgen.quad_instance(0, 0, N=6, K=0, T=3.0, drag=0.0, delta=3.0)
    inst["x_init"] = np.zeros(6)
    inst["x_target"] = np.array([1.2, 0.5, 0.3, 0, 0, 0])
    inst["qn"] = -200.0 * inst["x_target"]
    inst["obstacles"] = np.array([[0.6, 0.25, 0.2, 0.3]])
    s = np.linspace(0, 1, 7)[:, None]
    inst["x_guess"] = np.hstack([s * inst["x_target"][:3], np.tile(inst["x_target"][:3] / 3.0, (7, 1))])
    inst["u_ball"] = 10.3
    t = init_traj(inst)
    p = oracle.default_params(scp_iters=4, admm_iters=30000, check_every=50, eps_p=1e-11, eps_d=1e-11,
                              rho_final=8.0)
    info = scp_group([t], p)
    assert info["r_p"] < 1e-9 and info["r_d"] < 1e-9, info
    # the last subproblem was built at the nominal before the last acceptance
    _kkt_check(t, (8.0, 8.0, 8.0), 1e-7)


def test_penalty_schedule_improves_the_nonlinear_defect():
    """The paper's schedule (1e2 -> 1e3) against a fixed rho = 1 at the batch budget (15 x 200):
    measured 0.17 -> 4.8e-5."""
    inst = scpgen.config1(1)[0]
    fixed = oracle.scp_solve([inst], oracle.default_params(scp_iters=15, admm_iters=200))[1][0]
    sched = oracle.scp_solve([inst], oracle.default_params(scp_iters=15, admm_iters=200, rho_eq=100.0,
                                                           rho_dyn=100.0, rho_geo=100.0, rho_final=1e3))[1][0]
    assert sched["defect"] < 1e-3 * fixed["defect"]


@pytest.mark.parametrize("seq,flagged", [
    ([1e-3, 2e3], True),            # 2e6 times the reference
    ([1e-3, 1e3], False),           # exactly 1e6 times: not above it
    ([0.0, 1e-3, 9e2], False),      # a zero residual is no reference; 9e5 times the first positive one
    ([0.0, 1e-3, 1.5e3], True),
    ([5.0, 1e-9, 4e6], False),      # the reference is the first positive residual, not the smallest
])
def test_residual_blowup_rule(monkeypatch, seq, flagged):
    """The blow-up bit compares each SCP iteration's primal residual with the first positive one of
    the solve (fed here through a stand-in for the ADMM run, so only the rule is exercised)."""
    import oracle.scp as S
    vals = iter(seq)
    monkeypatch.setattr(S, "admm_run", lambda *a, **k: (1, next(vals), 0.0))
    t = init_traj(scpgen.quad_instance(1, 5, N=6, K=1))
    info = scp_group([t], oracle.default_params(scp_iters=len(seq), admm_iters=1, detect_blowup=True))
    assert bool(info["status"] & S.ST_DIVERGED) == flagged
    vals = iter(seq)
    off = scp_group([init_traj(scpgen.quad_instance(1, 5, N=6, K=1))],
                    oracle.default_params(scp_iters=len(seq), admm_iters=1))
    assert not off["status"] & S.ST_DIVERGED     # detection off: never set


def test_indefinite_cost_diverges_and_is_flagged():
    """A negative control weight makes the Step-1 Hessian indefinite: ADMM diverges and the blow-up
    bit is set; the same instance with its own cost converges unflagged."""
    import oracle.scp as S
    d = scpgen.quad_instance(1, 3, N=10, K=2)
    with np.errstate(all="ignore"):
        t = init_traj(dict(d, R=np.full(3, -2.0)))
        bad = scp_group([t], oracle.default_params(scp_iters=4, admm_iters=50, detect_blowup=True))
    t = init_traj(d)
    good = scp_group([t], oracle.default_params(scp_iters=4, admm_iters=50, detect_blowup=True))
    assert bad["status"] & S.ST_DIVERGED
    assert good["status"] == 0

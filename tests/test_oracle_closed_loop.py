"""Pins of the oracle pieces added for closed-loop robust MPC (Sec. IV-A.4).

* Constant disturbance acceleration in the quadrotor model: for the drag-free model RK4 is exact
  for constant acceleration, so one step equals the double-integrator closed form with the
  disturbance added; the Jacobians of the disturbed map agree with complex-step derivatives
  (and, without drag, do not depend on the disturbance).
* Vertical cylinder obstacles: the linearized half-space has a horizontal unit normal, its
  boundary touches the cylinder at the closest point, and the whole cylinder (at any height)
  lies on its excluded side; the violation metric uses the horizontal distance.
* Measured warm start: identical to the receding-horizon shift except that the initial state
  is the request's own.
* The closed loop: under a constant wind everywhere the linear observer's estimate converges to
  the wind; without wind the loop steers around the obstacle to the target.
"""
import types

import numpy as np
import pytest

import oracle
import scpgen
from oracle.mpc import closed_loop
from oracle.scp import init_traj, scp_group, shift_warm_start
from scpgen import closed_loop as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def test_disturbance_enters_as_constant_acceleration():
    inst = scpgen.quad_instance(0, 0, N=10, K=0, drag=0.0)
    d = np.array([0.3, -1.2, 0.7])
    inst["dist"] = d
    rng = np.random.default_rng(3)
    x, u = rng.normal(size=6), rng.normal(size=3) * 4.0
    h = inst["h"]
    a = u / inst["mscale"] - np.array([0.0, 0.0, inst["grav"]]) + d
    exact = np.concatenate([x[:3] + h * x[3:] + 0.5 * h * h * a, x[3:] + h * a])
    np.testing.assert_allclose(oracle.rk4(inst, x, u), exact, rtol=0, atol=1e-13)


def test_jacobians_with_a_disturbance():
    # drag-free: the map is affine in (x, u) and the disturbance only shifts it
    inst = scpgen.quad_instance(0, 1, N=10, K=0, drag=0.0)
    rng = np.random.default_rng(4)
    x, u = rng.normal(size=6), rng.normal(size=3)
    _, A0, B0, _ = oracle.rk4_jac(inst, x, u)
    inst["dist"] = np.array([1.0, 2.0, -3.0])
    _, A1, B1, _ = oracle.rk4_jac(inst, x, u)
    np.testing.assert_allclose(A1, A0, rtol=0, atol=1e-14)
    np.testing.assert_allclose(B1, B0, rtol=0, atol=1e-14)
    # with drag the stage points move with the disturbance: complex step through the map
    inst = scpgen.quad_instance(0, 1, N=10, K=0)
    inst["dist"] = np.array([1.0, 2.0, -3.0])
    F1, A1, B1, d1 = oracle.rk4_jac(inst, x, u)
    eps = 1e-30
    for j in range(6):
        xc = x.astype(complex)
        xc[j] += 1j * eps
        np.testing.assert_allclose(np.imag(oracle.rk4(inst, xc, u.astype(complex))) / eps, A1[:, j], atol=1e-12)
    # the residual carries the disturbance: d = F - A x - B u
    np.testing.assert_allclose(d1, F1 - A1 @ x - B1 @ u, atol=1e-12)


def _cyl_inst(N=6):
    inst = scpgen.quad_instance(0, 2, N=N, K=1)
    inst["obstacles"] = np.array([[1.0, -2.0, 5.0, 1.5]])
    inst["cyl"] = np.array([True])
    return inst


def test_cylinder_halfspace_is_tangent_and_excludes_the_cylinder():
    inst = _cyl_inst()
    N = inst["N"]
    rng = np.random.default_rng(7)
    xbar = np.zeros((N + 1, 6))
    xbar[:, :3] = rng.uniform(-6.0, 6.0, size=(N + 1, 3))
    xbar[:, 2] += 40.0  # far above the centre's z: a sphere's normal would point up
    groups = oracle.convexify(inst, xbar, np.zeros((N, 3)), 1.0)
    hs = [g for g in groups if g.kind == "halfspace"][0]
    c, r = inst["obstacles"][0, :3], inst["obstacles"][0, 3]
    for i in range(1, N + 1):
        a, b = hs.a[i], hs.b[i]
        assert a[2] == 0.0 and abs(np.linalg.norm(a) - 1.0) < 1e-14
        dxy = xbar[i, :2] - c[:2]
        np.testing.assert_allclose(a[:2], dxy / np.linalg.norm(dxy), atol=1e-14)
        touch = np.array([*(c[:2] + r * a[:2]), 123.0])
        assert abs(a @ touch - b) < 1e-12
        for th in np.linspace(0.0, 2.0 * np.pi, 24, endpoint=False):
            for z in (-50.0, 0.0, 70.0):
                y = np.array([c[0] + r * np.cos(th), c[1] + r * np.sin(th), z])
                assert a @ y <= b + 1e-12


def test_cylinder_violation_uses_horizontal_distance():
    inst = _cyl_inst(N=2)
    c, r = inst["obstacles"][0, :3], inst["obstacles"][0, 3]
    x = np.zeros((3, 6))
    x[:, :3] = [c[0] + 0.5, c[1], c[2] + 30.0]   # inside the cylinder, far from its centre point
    u = np.zeros((2, 3))
    assert abs(oracle.violation(inst, x, u) - (r - 0.5)) < 1e-12
    inst["cyl"] = np.array([False])               # the same point as a sphere: far outside
    assert oracle.violation(inst, x, u) == 0.0


def test_measured_warm_start_keeps_the_request_state():
    req = scpgen.config4_request(7, S=3, N=12)
    prm = oracle.default_params(scp_iters=2, admm_iters=20)
    trajs = [init_traj(d) for d in req]
    scp_group(trajs, prm)
    nxt = [dict(d) for d in req]
    meas = np.array([0.1, 0.2, 0.3, -0.4, 0.5, -0.6])
    for d in nxt:
        d["x_init"] = meas.copy()
    a = shift_warm_start(trajs, nxt)
    b = shift_warm_start(trajs, nxt, measured=True)
    for ta, tb in zip(a, b):
        np.testing.assert_array_equal(tb.inst["x_init"], meas)
        np.testing.assert_array_equal(ta.inst["x_init"], trajs[0].xbar[1])
        np.testing.assert_array_equal(ta.xbar, tb.xbar)
        np.testing.assert_array_equal(ta.ubar, tb.ubar)
        for da, db in zip(ta.state.dual, tb.state.dual):
            np.testing.assert_array_equal(da, db)


def _world(wind_fn, scen_sigma):
    return types.SimpleNamespace(
        START=W.START,
        request=lambda tpl, x, d, xi: W.request(tpl, x, d, scen_sigma * xi),
        wind=wind_fn,
        plant_step=W.plant_step,
    )


def test_observer_converges_to_a_constant_wind():
    world = _world(lambda p, n: W.WIND_BASE.copy(), 0.0)
    tpl = W.scene_instance(N=15)
    steps = 12
    out = closed_loop(world, tpl, steps, W.draws(1, steps, 2), oracle.default_params(scp_iters=3, admm_iters=40))
    err = np.linalg.norm(out["d_hat"][-1] - W.WIND_BASE)
    assert err < 0.2 * np.linalg.norm(W.WIND_BASE), (out["d_hat"][-1], err)


def test_loop_without_wind_reaches_the_target_around_the_obstacle():
    world = _world(lambda p, n: np.zeros(3), 0.0)
    tpl = W.scene_instance(N=15)
    steps = 30
    out = closed_loop(world, tpl, steps, W.draws(2, steps, 1), oracle.default_params(scp_iters=3, admm_iters=40))
    d0 = np.linalg.norm(out["x"][0, :3] - W.TARGET)
    d1 = np.linalg.norm(out["x"][-1, :3] - W.TARGET)
    assert d1 < d0 / 5.0, (d0, d1)
    assert min(W.clearance(x) for x in out["x"]) > 0.0
    # once the plan has converged (the cold first step at this small budget has not), the
    # estimate only sees the solver's residual defect
    assert np.max(np.abs(out["d_hat"][5:])) < 0.5

"""Pins of the oracle's 6-DOF quadrotor model (Sec. IV-A.1: Newton-Euler rigid body with a unit
quaternion, thrust and body torques), against closed forms that do not reuse its formulas:

* hover is an equilibrium of the continuous and the RK4 map (thrust m g, level, at rest);
* a level vehicle under constant thrust is a double integrator, which RK4 integrates exactly;
* attitude convention: rotating the body about x by theta tilts the thrust to (0, -sin, cos),
  about y to (sin, 0, cos); the thrust direction does not depend on the quaternion's scale;
* body-rate kinematics: at a constant rate about a principal axis (no torque) the exact
  attitude is q0 (x) (cos(|w| t / 2), sin(|w| t / 2) w/|w|) (right multiplication: body-frame
  rates); RK4 from a generic q0 matches it with fourth-order convergence (error ratio ~16
  per halving of the step over a fixed time);
* Euler's equations: an axisymmetric body (J_x = J_y) precesses, w_x + i w_y turning at
  lambda = (J_z - J_x) w_z / J_x with w_z constant; this fixes the sign of the gyroscopic term;
* Jacobians of f and of the RK4 map agree with complex-step derivatives;
* the convexified sets: no control ball, one position half-space per obstacle.
"""
import math

import numpy as np
import pytest

import oracle
import scpgen
from oracle.dynamics import f_cont, jac_cont, rk4, rk4_jac

M, G = scpgen.Q6_MASS, scpgen.G_EARTH


def _inst(h=0.12, inertia=None):
    d = scpgen.quad6_scene()
    d["h"] = h
    if inertia is not None:
        d["inertia"] = np.asarray(inertia, dtype=float)
    return d


def _state(p=(0.0, 0.0, 0.0), v=(0.0, 0.0, 0.0), q=(1.0, 0.0, 0.0, 0.0), w=(0.0, 0.0, 0.0)):
    return np.concatenate([p, v, q, w]).astype(float)


def _hamilton(a, b):
    # written out component by component (independent of the oracle's vector form)
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return np.array([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw])


def test_hover_is_an_equilibrium():
    d = _inst()
    x = _state(p=(1.0, -2.0, 3.0))
    u = np.array([M * G, 0.0, 0.0, 0.0])
    np.testing.assert_array_equal(f_cont(d, x, u), np.zeros(13))
    np.testing.assert_allclose(rk4(d, x, u), x, rtol=0, atol=1e-15)


def test_level_constant_thrust_is_a_double_integrator():
    d = _inst(h=0.2)
    x = _state(p=(0.5, 0.1, -0.3), v=(1.0, -2.0, 0.5))
    f = 14.0
    a = np.array([0.0, 0.0, f / M - G])
    y = rk4(d, x, np.array([f, 0.0, 0.0, 0.0]))
    h = d["h"]
    np.testing.assert_allclose(y[:3], x[:3] + h * x[3:6] + 0.5 * h * h * a, rtol=0, atol=1e-14)
    np.testing.assert_allclose(y[3:6], x[3:6] + h * a, rtol=0, atol=1e-14)
    np.testing.assert_array_equal(y[6:], x[6:])


@pytest.mark.parametrize("theta", [0.3, -1.1, 2.5])
def test_attitude_tilts_the_thrust(theta):
    d = _inst()
    f = 7.0
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    for q, direction in (((c, s, 0.0, 0.0), (0.0, -math.sin(theta), math.cos(theta))),
                         ((c, 0.0, s, 0.0), (math.sin(theta), 0.0, math.cos(theta)))):
        for scale in (1.0, 1.7):
            acc = f_cont(d, _state(q=scale * np.array(q)), np.array([f, 0.0, 0.0, 0.0]))[3:6]
            np.testing.assert_allclose(acc, f / M * np.array(direction) - np.array([0.0, 0.0, G]), atol=1e-13)


def test_constant_rate_rotation_matches_the_exponential_map():
    J = np.array([0.02, 0.03, 0.04])
    q0 = np.array([0.8, -0.2, 0.5, 0.26])
    q0 /= np.linalg.norm(q0)
    wz = 1.3
    T_total = 0.8
    phi = wz * T_total / 2
    exact = _hamilton(q0, np.array([math.cos(phi), 0.0, 0.0, math.sin(phi)]))
    left = _hamilton(np.array([math.cos(phi), 0.0, 0.0, math.sin(phi)]), q0)
    assert np.max(np.abs(exact - left)) > 0.05   # the convention is observable from this q0
    errs = []
    for n in (8, 16, 32):
        d = _inst(h=T_total / n, inertia=J)
        x = _state(q=q0, w=(0.0, 0.0, wz))
        for _ in range(n):
            x = rk4(d, x, np.array([M * G, 0.0, 0.0, 0.0]))
        np.testing.assert_allclose(x[10:13], [0.0, 0.0, wz], atol=1e-15)
        errs.append(np.max(np.abs(x[6:10] - exact)))
    assert errs[-1] < 1e-8
    assert 12.0 < errs[0] / errs[1] < 20.0 and 12.0 < errs[1] / errs[2] < 20.0


def test_axisymmetric_body_precesses_at_the_euler_rate():
    J = np.array([0.02, 0.02, 0.05])
    w0 = np.array([0.7, -0.4, 2.0])
    lam = (J[2] - J[0]) * w0[2] / J[0]
    T_total, n = 1.0, 400
    d = _inst(h=T_total / n, inertia=J)
    x = _state(w=w0)
    for _ in range(n):
        x = rk4(d, x, np.array([M * G, 0.0, 0.0, 0.0]))
    z = (w0[0] + 1j * w0[1]) * np.exp(1j * lam * T_total)
    np.testing.assert_allclose(x[10:13], [z.real, z.imag, w0[2]], atol=1e-9)
    # the body keeps its kinetic energy and angular momentum magnitude
    w = x[10:13]
    assert abs(w @ (J * w) - w0 @ (J * w0)) < 1e-9
    assert abs(np.linalg.norm(J * w) - np.linalg.norm(J * w0)) < 1e-9


def _complex_step_cols(fun, z, n):
    eps = 1e-30
    cols = []
    for j in range(n):
        zc = z.astype(complex)
        zc[j] += 1j * eps
        cols.append(np.imag(fun(zc)) / eps)
    return np.array(cols).T


def test_jacobians_match_complex_step():
    d = _inst()
    d["dist"] = np.array([0.2, -0.1, 0.3])
    rng = np.random.default_rng(11)
    x = _state(p=rng.normal(size=3), v=rng.normal(size=3), q=rng.normal(size=4), w=rng.normal(size=3))
    u = np.array([9.0, 0.3, -0.2, 0.1])
    Jx, Ju = jac_cont(d, x, u)
    np.testing.assert_allclose(Jx, _complex_step_cols(lambda z: f_cont(d, z, u.astype(complex)), x, 13), atol=1e-12)
    np.testing.assert_allclose(Ju, _complex_step_cols(lambda z: f_cont(d, x.astype(complex), z), u, 4), atol=1e-12)
    F, A, B, dd = rk4_jac(d, x, u)
    np.testing.assert_allclose(F, rk4(d, x, u), atol=1e-14)
    np.testing.assert_allclose(A, _complex_step_cols(lambda z: rk4(d, z, u.astype(complex)), x, 13), atol=1e-11)
    np.testing.assert_allclose(B, _complex_step_cols(lambda z: rk4(d, x.astype(complex), z), u, 4), atol=1e-11)
    np.testing.assert_allclose(A[:, :3], np.eye(13)[:, :3], atol=0)   # position never enters f
    np.testing.assert_allclose(dd, F - A @ x - B @ u, atol=1e-12)


def test_convexified_sets_of_the_6dof_model():
    d = scpgen.quad6_scene(N=8)
    d["u_ball"] = 1.0   # ignored by this model
    N = d["N"]
    groups = oracle.convexify(d, d["x_guess"], d["u_guess"], 1.0)
    kinds = [(g.kind, g.var, g.comps) for g in groups]
    assert kinds[0] == ("box", "x", tuple(range(13))) and kinds[1] == ("box", "u", tuple(range(4)))
    assert kinds[2:] == [("halfspace", "x", (0, 1, 2))] * 3
    # terminal position and velocity fixed, attitude and rates free
    xlo, xhi = groups[0].lo[N], groups[0].hi[N]
    np.testing.assert_array_equal(xlo[:6], d["x_target"][:6])
    np.testing.assert_array_equal(xhi[:6], d["x_target"][:6])
    assert np.all(xhi[6:] > xlo[6:])
    # thrust box [0, 20] cut by the trust box around the hover thrust
    np.testing.assert_allclose(groups[1].lo[0], [M * G - 1.0, -1.0, -1.0, -1.0])
    np.testing.assert_allclose(groups[1].hi[0], [M * G + 1.0, 1.0, 1.0, 1.0])
    x = d["x_guess"].copy()
    u = d["u_guess"].copy()
    u[0, 1] = 7.0                                   # torque above its bound by 2
    assert abs(oracle.violation(d, x, u) - 2.0) < 1e-12


def test_benchmark_generator_shapes():
    insts = scpgen.config5(5)
    for d in insts:
        assert d["model"] == scpgen.QUAD6 and d["N"] == 40 and d["obstacles"].shape == (3, 4)
        assert np.all((d["obstacles"][:, 3] >= 1.0) & (d["obstacles"][:, 3] <= 2.0))
        for c in d["obstacles"]:
            assert np.linalg.norm(scpgen.Q6_START - c[:3]) >= c[3] + 0.25
            assert np.linalg.norm(scpgen.Q6_GOAL - c[:3]) >= c[3] + 0.25
        np.testing.assert_array_equal(d["x_guess"][0], d["x_init"])
    assert not np.array_equal(insts[0]["obstacles"], insts[1]["obstacles"])
    np.testing.assert_array_equal(scpgen.config5(2)[1]["x_guess"], insts[1]["x_guess"])

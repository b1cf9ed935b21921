"""Pins of the oracle's 6-DOF lander (Sec. IV-B.1: mass, position and velocity Up-East-North,
attitude quaternion, body rates; body-frame thrust), against closed forms written out here:

* the rocket equation: upright, not rotating, constant axial thrust f: m(t) = m0 - alpha f t,
  v_U(t) = v0 - t - ln(m(t)/m0)/alpha, and r_U by integrating once more; RK4 converges to it at
  fourth order;
* the thrust point below the centre of mass turns a lateral thrust into a body torque
  (components written out, not through a cross product);
* the attitude rotates the thrust: about z by theta to (cos, sin, 0), about y to (cos, 0, -sin);
* the convexified sets mean what the paper's limits say: the tilt ball on (q_y, q_z) is the
  set of attitudes whose body axis is within 20 deg of Up; the glide cone the positions at least
  10 deg above the horizon; the gimbal cone the thrusts within 10 deg of the body axis; the
  linearized lower thrust bound is a half-space inside ||T|| >= T_min touching it at the nominal
  direction;
* Jacobians of f and of the RK4 map agree with complex-step derivatives.
"""
import math

import numpy as np
import pytest

import oracle
import scpgen
from oracle.dynamics import f_cont, jac_cont, rk4, rk4_jac


def _state(r=(0.0, 0.0, 0.0), v=(0.0, 0.0, 0.0), q=(1.0, 0.0, 0.0, 0.0), w=(0.0, 0.0, 0.0), m=2.0):
    return np.concatenate([r, v, q, w, [m]]).astype(float)


def _inst(h=None):
    d = scpgen.lander6_instance()
    if h is not None:
        d["h"] = h
    return d


def test_rocket_equation():
    alpha = scpgen.L6_ALPHA
    m0, f, v0, r0 = 2.0, 2.6, -0.4, 1.5
    T_total = 1.0
    mt = m0 - alpha * f * T_total
    c = alpha * f / m0
    v_exact = v0 - T_total - math.log(mt / m0) / alpha
    # r(t) = r0 + v0 t - t^2/2 - (1/alpha) int_0^t ln(1 - c s) ds
    integral = -((1.0 - c * T_total) * (math.log(1.0 - c * T_total) - 1.0) + 1.0) / c
    r_exact = r0 + v0 * T_total - 0.5 * T_total ** 2 - integral / alpha
    errs = []
    for n in (4, 8, 16):
        d = _inst(h=T_total / n)
        x = _state(r=(r0, 0.0, 0.0), v=(v0, 0.0, 0.0), m=m0)
        for _ in range(n):
            x = rk4(d, x, np.array([f, 0.0, 0.0]))
        assert abs(x[13] - mt) < 1e-14                      # linear in time: RK4 exact
        np.testing.assert_array_equal(x[6:13], _state()[6:13])
        np.testing.assert_allclose(x[1:3], 0.0, atol=0)
        errs.append(max(abs(x[3] - v_exact), abs(x[0] - r_exact)))
    assert errs[-1] < 1e-8
    assert 12.0 < errs[0] / errs[1] < 20.0 and 12.0 < errs[1] / errs[2] < 20.0


def test_thrust_point_torque():
    d = _inst()
    J, a = d["inertia"], d["arm"][0]                      # thrust point on the body axis at a
    Tx, Ty, Tz = 2.0, 0.3, -0.2
    wdot = f_cont(d, _state(), np.array([Tx, Ty, Tz]))[10:13]
    # torque of (Tx, Ty, Tz) applied at (a, 0, 0): (0, -a Tz, a Ty)
    np.testing.assert_allclose(wdot, [0.0, -a * Tz / J[1], a * Ty / J[2]], atol=1e-15)
    # a thrust point below the centre of mass (a < 0) swings the nose away from the lateral
    # thrust: +T_z turns about +y (R_y e1 = (cos, 0, -sin): nose to -z), +T_y about -z (nose to -y)
    assert a < 0 and wdot[1] * Tz > 0 and wdot[2] * Ty < 0


@pytest.mark.parametrize("theta", [0.25, -0.9])
def test_attitude_rotates_the_thrust(theta):
    d = _inst()
    f, m = 2.2, 1.6
    c, s = math.cos(theta / 2), math.sin(theta / 2)
    for q, direction in (((c, 0.0, 0.0, s), (math.cos(theta), math.sin(theta), 0.0)),
                         ((c, 0.0, s, 0.0), (math.cos(theta), 0.0, -math.sin(theta)))):
        acc = f_cont(d, _state(q=1.3 * np.array(q), m=m), np.array([f, 0.0, 0.0]))[3:6]
        np.testing.assert_allclose(acc, f / m * np.array(direction) + scpgen.L6_GRAVITY, atol=1e-14)


def _groups(d):
    return oracle.convexify(d, d["x_guess"], d["u_guess"], d["delta"])


def test_tilt_ball_is_the_tilt_limit():
    d = _inst()
    tilt = [g for g in _groups(d) if g.var == "x" and g.comps == (8, 9)][0]
    assert tilt.kind == "ball"
    rng = np.random.default_rng(5)
    for _ in range(2000):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        qw, qx, qy, qz = q
        axis_up = qw * qw + qx * qx - qy * qy - qz * qz          # Up component of R(q) e1
        inside_angle = axis_up >= math.cos(math.radians(scpgen.L6_TILT_DEG)) - 1e-12
        inside_ball = math.hypot(qy, qz) <= tilt.radius + 1e-12
        assert inside_angle == inside_ball


def test_glide_and_gimbal_cones_are_the_angle_limits():
    d = _inst()
    g = _groups(d)
    glide = [x for x in g if x.var == "x" and x.kind == "cone"][0]
    gimbal = [x for x in g if x.var == "u" and x.kind == "cone"][0]
    assert glide.comps == (1, 2, 0) and gimbal.comps == (1, 2, 0)
    rng = np.random.default_rng(6)
    for _ in range(2000):
        r = rng.normal(size=3)
        elev = math.degrees(math.atan2(r[0], math.hypot(r[1], r[2])))
        assert (elev >= scpgen.L6_GLIDE_DEG) == (math.hypot(r[1], r[2]) <= glide.kappa * r[0])
        T = rng.normal(size=3)
        off = math.degrees(math.acos(np.clip(T[0] / np.linalg.norm(T), -1.0, 1.0)))
        assert (off <= scpgen.L6_GIMBAL_DEG) == (math.hypot(T[1], T[2]) <= gimbal.kappa * T[0])


def test_lower_thrust_halfspace_is_inside_the_nonconvex_set():
    d = _inst()
    rng = np.random.default_rng(8)
    d["u_guess"] = rng.normal(size=d["u_guess"].shape) * 1.5
    hs = [x for x in _groups(d) if x.kind == "halfspace"][0]
    assert hs.var == "u" and not hs.active[d["N"]]
    for i in range(d["N"]):
        a, b = hs.a[i], hs.b[i]
        ub = d["u_guess"][i]
        np.testing.assert_allclose(a, ub / np.linalg.norm(ub), atol=1e-15)
        assert b == scpgen.L6_T_MIN
        touch = b * a                                              # the tangent point
        assert abs(np.linalg.norm(touch) - scpgen.L6_T_MIN) < 1e-14 and abs(a @ touch - b) < 1e-14
        for _ in range(20):
            T = rng.normal(size=3) * 3.0
            if a @ T >= b:
                assert np.linalg.norm(T) >= scpgen.L6_T_MIN - 1e-12


def test_violation_reads_each_limit():
    d = _inst()
    x, u = d["x_guess"].copy(), d["u_guess"].copy()
    assert oracle.violation(d, x, u) < 1e-12
    u2 = u.copy()
    u2[3] = [0.2, 0.0, 0.0]                                        # below the lower thrust bound
    assert abs(oracle.violation(d, x, u2) - (scpgen.L6_T_MIN - 0.2)) < 1e-12
    x2 = x.copy()
    x2[5, 10:13] = [0.0, 0.0, 1.0]                                 # rate above its bound
    assert abs(oracle.violation(d, x2, u) - (1.0 - math.radians(30.0))) < 1e-12


def _cs_cols(fun, z, n):
    eps = 1e-30
    out = []
    for j in range(n):
        zc = z.astype(complex)
        zc[j] += 1j * eps
        out.append(np.imag(fun(zc)) / eps)
    return np.array(out).T


def test_jacobians_match_complex_step():
    d = _inst()
    rng = np.random.default_rng(12)
    x = _state(r=rng.normal(size=3), v=rng.normal(size=3), q=rng.normal(size=4), w=rng.normal(size=3), m=1.4)
    u = np.array([1.7, 0.2, -0.3])
    Jx, Ju = jac_cont(d, x, u)
    np.testing.assert_allclose(Jx, _cs_cols(lambda z: f_cont(d, z, u.astype(complex)), x, 14), atol=1e-12)
    np.testing.assert_allclose(Ju, _cs_cols(lambda z: f_cont(d, x.astype(complex), z), u, 3), atol=1e-12)
    F, A, B, dd = rk4_jac(d, x, u)
    np.testing.assert_allclose(A, _cs_cols(lambda z: rk4(d, z, u.astype(complex)), x, 14), atol=1e-11)
    np.testing.assert_allclose(B, _cs_cols(lambda z: rk4(d, x.astype(complex), z), u, 3), atol=1e-11)
    np.testing.assert_allclose(A[:, :3], np.eye(14)[:, :3], atol=0)   # position never enters f
    np.testing.assert_allclose(dd, F - A @ x - B @ u, atol=1e-12)


def test_monte_carlo_generator():
    insts = scpgen.config6(6)
    nominal = scpgen.lander6_instance()["x_init"]
    for d in insts:
        x0 = d["x_init"]
        assert d["model"] == scpgen.LANDER6 and d["N"] == 30 and x0.shape == (14,)
        assert abs(np.linalg.norm(x0[6:10]) - 1.0) < 1e-14 and x0[13] <= scpgen.L6_M_WET
        nz = nominal != 0.0
        nz[6:10] = False
        assert np.all(np.abs(x0[nz] - nominal[nz]) <= 0.05 * np.abs(nominal[nz]) + 1e-15)
        np.testing.assert_array_equal(d["x_guess"][0], x0)
    assert not np.array_equal(insts[0]["x_init"], insts[1]["x_init"])

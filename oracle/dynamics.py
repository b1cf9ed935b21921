"""Dynamics of the three models, their RK4 discretization and its exact Jacobians.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper: Sec. II eq. (ocp) integrates the continuous dynamics over one step with
4th-order Runge-Kutta; Sec. III-A takes A_i, B_i as the Jacobians of that
discrete map at the nominal (x_i, u_i) and d_i as the linearization residual.
"""
from __future__ import annotations

import numpy as np

QUAD, MARS, QUAD6, LANDER6 = 1, 2, 3, 4


def f_cont(inst: dict, x: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Continuous-time dynamics x' = f(x, u).

    Quadrotor point mass: p' = v, v' = u/m_s - g e3 - c ||v|| v + d  (drag isotropic and
    quadratic; d the instance's constant disturbance acceleration, 0 unless given).
    Powered descent (scaled units): r' = v, v' = T/m + g_vec, m' = -alpha Gamma.
    6-DOF quadrotor (Sec. IV-A.1, Newton-Euler rigid body): x = (p, v, q, w) with the unit
    quaternion q = (q_w, q_x, q_y, q_z) rotating body to world and w the body angular rate;
    u = (f, tau) total thrust along the body z axis and body torques:
        p' = v,  v' = (f/m) R(q) e3 - g e3 + d,  q' = (1/2) q (x) (0, w),  J w' = tau - w x (J w),
    with J = diag(inertia).  R(q) e3 is the third column of the rotation matrix of q / ||q||:
    (2(q_x q_z + q_w q_y), 2(q_y q_z - q_w q_x), q_w^2 - q_x^2 - q_y^2 + q_z^2) / ||q||^2, so the
    thrust direction stays a unit vector when the iterates leave the unit sphere.
    6-DOF lander (Sec. IV-B.1, unified non-dimensional units): x = (r, v, q, w, m) with position
    and velocity in the Up-East-North frame, q rotating body to inertial, w the body rate and m the
    mass; u = T_B, the thrust vector in the body frame:
        r' = v,  v' = R(q/||q||) T_B / m + g,  q' = (1/2) q (x) (0, w),
        J w' = r_T x T_B - w x (J w),  m' = -alpha ||T_B||,
    with r_T the thrust point in the body frame ("arm") and J = diag(inertia).
    The norm is written sqrt(v.v) so the function stays analytic for complex-step tests.
    """
    if inst["model"] == LANDER6:
        v, q, w, m = x[3:6], x[6:10], x[10:13], x[13]
        T = u[0:3]
        J = np.asarray(inst["inertia"], dtype=float)
        acc = _rot(q) @ T / m + np.asarray(inst["gvec"], dtype=float)
        qdot = 0.5 * _quat_mul(q, np.concatenate([[0.0], w]))
        wdot = (np.cross(np.asarray(inst["arm"], dtype=float), T) - np.cross(w, J * w)) / J
        mdot = -inst["alpha"] * np.sqrt(T @ T)
        return np.concatenate([v, acc, qdot, wdot, [mdot]])
    if inst["model"] == QUAD6:
        v, q, w = x[3:6], x[6:10], x[10:13]
        f, tau = u[0], u[1:4]
        J = np.asarray(inst["inertia"], dtype=float)
        acc = (f / inst["mscale"]) * _rot_e3(q) - np.array([0.0, 0.0, inst["grav"]])
        if "dist" in inst:
            acc = acc + np.asarray(inst["dist"], dtype=float)
        qdot = 0.5 * _quat_mul(q, np.concatenate([[0.0], w]))
        wdot = (tau - np.cross(w, J * w)) / J
        return np.concatenate([v, acc, qdot, wdot])
    if inst["model"] == QUAD:
        p, v = x[:3], x[3:6]
        nv = np.sqrt(v @ v)
        acc = u / inst["mscale"] - np.array([0.0, 0.0, inst["grav"]]) - inst["drag"] * nv * v
        if "dist" in inst:
            acc = acc + np.asarray(inst["dist"], dtype=float)
        return np.concatenate([v, acc])
    r, v, m = x[:3], x[3:6], x[6]
    T, G = u[:3], u[3]
    return np.concatenate([v, T / m + inst["gvec"], [-inst["alpha"] * G]])


def _quat_mul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Hamilton product a (x) b of quaternions stored scalar first."""
    aw, av = a[0], a[1:]
    bw, bv = b[0], b[1:]
    return np.concatenate([[aw * bw - av @ bv], aw * bv + bw * av + np.cross(av, bv)])


def _rot_e3(q: np.ndarray) -> np.ndarray:
    """Third column of the rotation matrix of q / ||q||."""
    qw, qx, qy, qz = q
    n2 = qw * qw + qx * qx + qy * qy + qz * qz
    return np.array([2.0 * (qx * qz + qw * qy), 2.0 * (qy * qz - qw * qx), qw * qw - qx * qx - qy * qy + qz * qz]) / n2


def _rot_hom(q: np.ndarray) -> np.ndarray:
    """Rotation matrix of a unit quaternion written as the homogeneous quadratic in q."""
    qw, qx, qy, qz = q
    return np.array([[qw * qw + qx * qx - qy * qy - qz * qz, 2.0 * (qx * qy - qw * qz), 2.0 * (qx * qz + qw * qy)],
                     [2.0 * (qx * qy + qw * qz), qw * qw - qx * qx + qy * qy - qz * qz, 2.0 * (qy * qz - qw * qx)],
                     [2.0 * (qx * qz - qw * qy), 2.0 * (qy * qz + qw * qx), qw * qw - qx * qx - qy * qy + qz * qz]])


def _rot(q: np.ndarray) -> np.ndarray:
    """Rotation matrix of q / ||q||."""
    return _rot_hom(q) / (q @ q)


def _skew(a: np.ndarray) -> np.ndarray:
    """Matrix of the cross product a x (.)."""
    return np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])


def jac_cont(inst: dict, x: np.ndarray, u: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Jacobians (df/dx, df/du) of ``f_cont``.

    Drag term: d(c||v||v)/dv = c (||v|| I + v v^T / ||v||), taken as 0 at v = 0.
    6-DOF quadrotor: d(R(q) e3)/dq by the quotient rule on the normalized form; q (x) (0, w) is
    bilinear, so its
    derivative in q is the right-multiplication matrix of (0, w) and in w the left-multiplication
    matrix of q restricted to the vector part; d(w x Jw)/dw = [w]x J - [Jw]x.
    """
    nx, nu = x.shape[0], u.shape[0]
    Jx = np.zeros((nx, nx))
    Ju = np.zeros((nx, nu))
    if inst["model"] == LANDER6:
        q, w, m = x[6:10], x[10:13], x[13]
        qw, qx, qy, qz = q
        T = u[0:3]
        T0, T1, T2 = T
        J = np.asarray(inst["inertia"], dtype=float)
        n2 = q @ q
        p = _rot_hom(q) @ T
        # d(R_hom(q) T)/dq, one column per quaternion component (w, x, y, z)
        dp = 2.0 * np.array([[qw * T0 - qz * T1 + qy * T2, qx * T0 + qy * T1 + qz * T2,
                              -qy * T0 + qx * T1 + qw * T2, -qz * T0 - qw * T1 + qx * T2],
                             [qz * T0 + qw * T1 - qx * T2, qy * T0 - qx * T1 - qw * T2,
                              qx * T0 + qy * T1 + qz * T2, qw * T0 - qz * T1 + qy * T2],
                             [-qy * T0 + qx * T1 + qw * T2, qz * T0 + qw * T1 - qx * T2,
                              -qw * T0 + qz * T1 - qy * T2, qx * T0 + qy * T1 + qz * T2]])
        Jx[0:3, 3:6] = np.eye(3)
        Jx[3:6, 6:10] = (dp / n2 - np.outer(p, 2.0 * q) / (n2 * n2)) / m
        Jx[3:6, 13] = -p / n2 / (m * m)
        Ju[3:6, 0:3] = _rot(q) / m
        Lq = np.zeros((4, 4))
        Lq[0, 0] = qw
        Lq[0, 1:] = -q[1:]
        Lq[1:, 0] = q[1:]
        Lq[1:, 1:] = qw * np.eye(3) + _skew(q[1:])
        Rp = np.zeros((4, 4))
        Rp[0, 1:] = -w
        Rp[1:, 0] = w
        Rp[1:, 1:] = -_skew(w)
        Jx[6:10, 6:10] = 0.5 * Rp
        Jx[6:10, 10:13] = 0.5 * Lq[:, 1:]
        Jx[10:13, 10:13] = -(_skew(w) @ np.diag(J) - _skew(J * w)) / J[:, None]
        Ju[10:13, 0:3] = _skew(np.asarray(inst["arm"], dtype=float)) / J[:, None]
        nT = np.sqrt(T @ T)
        if nT > 0.0:
            Ju[13, 0:3] = -inst["alpha"] * T / nT
        return Jx, Ju
    if inst["model"] == QUAD6:
        q, w = x[6:10], x[10:13]
        qw, qx, qy, qz = q
        f = u[0]
        m = inst["mscale"]
        J = np.asarray(inst["inertia"], dtype=float)
        Jx[0:3, 3:6] = np.eye(3)
        n2 = q @ q
        dc = 2.0 * np.array([[qy, qz, qw, qx],
                             [-qx, -qw, qz, qy],
                             [qw, -qx, -qy, qz]])
        dR = dc / n2 - np.outer(_rot_e3(q), 2.0 * q) / n2
        Jx[3:6, 6:10] = (f / m) * dR
        Ju[3:6, 0] = _rot_e3(q) / m
        # q' = (1/2) q (x) p with p = (0, w): right multiplication by p, and left multiplication by q
        pw, pv = 0.0, w
        Rp = np.zeros((4, 4))
        Rp[0, 0] = pw
        Rp[0, 1:] = -pv
        Rp[1:, 0] = pv
        Rp[1:, 1:] = pw * np.eye(3) - _skew(pv)
        Lq = np.zeros((4, 4))
        Lq[0, 0] = qw
        Lq[0, 1:] = -q[1:]
        Lq[1:, 0] = q[1:]
        Lq[1:, 1:] = qw * np.eye(3) + _skew(q[1:])
        Jx[6:10, 6:10] = 0.5 * Rp
        Jx[6:10, 10:13] = 0.5 * Lq[:, 1:]
        Jx[10:13, 10:13] = -(_skew(w) @ np.diag(J) - _skew(J * w)) / J[:, None]
        Ju[10:13, 1:4] = np.diag(1.0 / J)
        return Jx, Ju
    if inst["model"] == QUAD:
        v = x[3:6]
        nv = np.sqrt(v @ v)
        Jx[0:3, 3:6] = np.eye(3)
        if nv > 0.0:
            Jx[3:6, 3:6] = -inst["drag"] * (nv * np.eye(3) + np.outer(v, v) / nv)
        Ju[3:6, 0:3] = np.eye(3) / inst["mscale"]
        return Jx, Ju
    m = x[6]
    T = u[:3]
    Jx[0:3, 3:6] = np.eye(3)
    Jx[3:6, 6] = -T / (m * m)
    Ju[3:6, 0:3] = np.eye(3) / m
    Ju[6, 3] = -inst["alpha"]
    return Jx, Ju


def rk4(inst: dict, x: np.ndarray, u: np.ndarray, h: float | None = None) -> np.ndarray:
    """Classical 4th-order Runge-Kutta step with zero-order-hold control."""
    h = inst["h"] if h is None else h
    k1 = f_cont(inst, x, u)
    k2 = f_cont(inst, x + 0.5 * h * k1, u)
    k3 = f_cont(inst, x + 0.5 * h * k2, u)
    k4 = f_cont(inst, x + h * k3, u)
    return x + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def rk4_jac(inst: dict, x: np.ndarray, u: np.ndarray):
    """Discrete map F = RK4(x, u) and its exact Jacobians A = dF/dx, B = dF/du.

    Forward-mode chain rule through the four stages: with stage points
    x1 = x, x2 = x + h/2 k1, x3 = x + h/2 k2, x4 = x + h k3 and stage sensitivities
    S_j = dk_j/d(x,u), S_j = Jx(x_j) dx_j/d(x,u) + [0, Ju(x_j)].
    Returns (F, A, B, d) with the residual d = F - A x - B u (Sec. III-A).
    """
    h = inst["h"]
    nx, nu = x.shape[0], u.shape[0]
    I = np.eye(nx)
    Zu = np.zeros((nx, nu))
    pts, sx, su = [], [], []
    xs, dxs_x, dxs_u = x, I, Zu
    coeffs = (0.5 * h, 0.5 * h, h)
    ks = []
    for j in range(4):
        Jx, Ju = jac_cont(inst, xs, u)
        k = f_cont(inst, xs, u)
        Sx = Jx @ dxs_x
        Su = Jx @ dxs_u + Ju
        ks.append(k)
        sx.append(Sx)
        su.append(Su)
        pts.append(xs)
        if j < 3:
            c = coeffs[j]
            xs = x + c * k
            dxs_x = I + c * Sx
            dxs_u = c * Su
    F = x + (h / 6.0) * (ks[0] + 2.0 * ks[1] + 2.0 * ks[2] + ks[3])
    A = I + (h / 6.0) * (sx[0] + 2.0 * sx[1] + 2.0 * sx[2] + sx[3])
    B = (h / 6.0) * (su[0] + 2.0 * su[1] + 2.0 * su[2] + su[3])
    d = F - A @ x - B @ u
    return F, A, B, d

"""Pins for the oracle's dynamics, RK4 map and Jacobians (Sec. II eq. (ocp), Sec. III-A).

Each check compares against something other than the oracle's own formulas:
an adaptive high-accuracy ODE integrator, exact closed forms of affine cases,
complex-step derivatives and central differences.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import scpgen
from oracle import f_cont, rk4, rk4_jac
from oracle.dynamics import jac_cont


def _quad(drag=0.1, mscale=1.0, h=0.1):
    d = scpgen.quad_instance(0, 0, N=50, K=0, T=5.0)
    d.update(drag=drag, mscale=mscale, h=h)
    return d


def _mars(alpha=None, h=None):
    d = scpgen.mars_instance(2, 0, N=60)
    if alpha is not None:
        d["alpha"] = alpha
    if h is not None:
        d["h"] = h
    return d


def _exact_step(inst, x, u, h):
    sol = solve_ivp(lambda t, y: f_cont(inst, y, u), (0.0, h), x, method="DOP853", rtol=1e-13, atol=1e-15)
    return sol.y[:, -1]


@pytest.mark.parametrize("kind", ["quad", "mars"])
def test_rk4_local_error_is_fifth_order(kind):
    """A correct RK4 step has local error C h^5: halving h divides it by ~32."""
    rng = np.random.default_rng(3)
    for _ in range(3):
        if kind == "quad":
            inst = _quad()
            x = np.concatenate([rng.uniform(-3, 3, 3), rng.uniform(-4, 4, 3)])
            u = rng.uniform(-8, 8, 3)
            h = 0.05
        else:
            inst = _mars()
            x = np.concatenate([rng.uniform(-0.5, 0.5, 2), [1.5], rng.uniform(-0.5, 0.5, 3), [0.9]])
            u = np.concatenate([rng.uniform(-0.3, 0.3, 3), [0.5]])
            u[2] = 0.6
            h = 0.4
        e1 = np.max(np.abs(rk4(inst, x, u, h) - _exact_step(inst, x, u, h)))
        e2 = np.max(np.abs(rk4(inst, x, u, h / 2) - _exact_step(inst, x, u, h / 2)))
        assert e1 > 0
        ratio = e1 / e2
        assert 26.0 < ratio < 45.0, ratio   # a wrong stage weight gives ~8 or ~16


def test_dragfree_quad_closed_form():
    """Drag-free point mass with ZOH control: RK4 is exact, A=[[I,hI],[0,I]], B=[[h^2/2 I],[hI]],
    d = [-h^2/2 g e3; -h g e3]."""
    h = 0.1
    inst = _quad(drag=0.0, h=h)
    rng = np.random.default_rng(0)
    x = rng.normal(size=6)
    u = rng.normal(size=3) * 5
    F, A, B, d = rk4_jac(inst, x, u)
    I3 = np.eye(3)
    A_ref = np.block([[I3, h * I3], [np.zeros((3, 3)), I3]])
    B_ref = np.vstack([0.5 * h * h * I3, h * I3])
    g = np.array([0, 0, 9.81])
    d_ref = np.concatenate([-0.5 * h * h * g, -h * g])
    np.testing.assert_allclose(A, A_ref, atol=1e-15)
    np.testing.assert_allclose(B, B_ref, atol=1e-15)
    np.testing.assert_allclose(d, d_ref, atol=1e-14)
    F_ref = np.concatenate([x[:3] + h * x[3:] + 0.5 * h * h * (u - g), x[3:] + h * (u - g)])
    np.testing.assert_allclose(F, F_ref, atol=1e-14)


def test_mars_constant_mass_closed_form():
    """alpha = 0 (no mass flow): r+ = r + h v + h^2/2 (T/m + g), v+ = v + h (T/m + g), m+ = m.
    Jacobians w.r.t. m: -h^2/2 T/m^2 and -h T/m^2."""
    h = 5.0 / 60
    inst = _mars(alpha=0.0, h=h)
    x = np.array([0.3, -0.2, 1.5, 0.1, 0.05, -0.3, 0.95])
    u = np.array([0.05, -0.02, 0.4, 0.45])
    F, A, B, d = rk4_jac(inst, x, u)
    m, T, g = x[6], u[:3], inst["gvec"]
    a = T / m + g
    np.testing.assert_allclose(F[:3], x[:3] + h * x[3:6] + 0.5 * h * h * a, atol=1e-15)
    np.testing.assert_allclose(F[3:6], x[3:6] + h * a, atol=1e-15)
    assert F[6] == m
    np.testing.assert_allclose(A[:3, 6], -0.5 * h * h * T / m ** 2, atol=1e-15)
    np.testing.assert_allclose(A[3:6, 6], -h * T / m ** 2, atol=1e-15)
    np.testing.assert_allclose(B[:3, :3], 0.5 * h * h * np.eye(3) / m, atol=1e-15)
    np.testing.assert_allclose(B[3:6, :3], h * np.eye(3) / m, atol=1e-15)
    np.testing.assert_allclose(B[:, 3], 0.0, atol=0)


def _complex_step_jac(inst, x, u):
    eps = 1e-30
    nx, nu = x.size, u.size
    A = np.zeros((nx, nx))
    B = np.zeros((nx, nu))
    for j in range(nx):
        xc = x.astype(complex)
        xc[j] += 1j * eps
        A[:, j] = np.imag(rk4(inst, xc, u.astype(complex))) / eps
    for j in range(nu):
        uc = u.astype(complex)
        uc[j] += 1j * eps
        B[:, j] = np.imag(rk4(inst, x.astype(complex), uc)) / eps
    return A, B


@pytest.mark.parametrize("kind", ["quad", "quad_mass", "mars"])
def test_jacobians_match_complex_step(kind):
    rng = np.random.default_rng(11)
    for _ in range(5):
        if kind.startswith("quad"):
            inst = _quad(mscale=1.07 if kind == "quad_mass" else 1.0)
            x = np.concatenate([rng.uniform(-5, 5, 3), rng.uniform(-4, 4, 3)])
            u = rng.uniform(-10, 15, 3)
        else:
            inst = _mars()
            x = np.concatenate([rng.uniform(-0.5, 0.5, 3), rng.uniform(-0.5, 0.5, 3), [rng.uniform(0.85, 1.0)]])
            u = np.concatenate([rng.uniform(-0.3, 0.3, 3), [rng.uniform(0.2, 0.6)]])
        F, A, B, d = rk4_jac(inst, x, u)
        Acs, Bcs = _complex_step_jac(inst, x, u)
        np.testing.assert_allclose(A, Acs, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(B, Bcs, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(F, rk4(inst, x, u), rtol=0, atol=0)
        np.testing.assert_allclose(A @ x + B @ u + d, F, atol=1e-13)


def test_jacobians_match_central_differences():
    rng = np.random.default_rng(5)
    inst = _quad()
    x = np.concatenate([rng.uniform(-5, 5, 3), rng.uniform(-4, 4, 3)])
    u = rng.uniform(-10, 15, 3)
    _, A, B, _ = rk4_jac(inst, x, u)
    e = 1e-6
    for j in range(6):
        dx = np.zeros(6)
        dx[j] = e
        col = (rk4(inst, x + dx, u) - rk4(inst, x - dx, u)) / (2 * e)
        np.testing.assert_allclose(A[:, j], col, atol=1e-8)
    for j in range(3):
        du = np.zeros(3)
        du[j] = e
        col = (rk4(inst, x, u + du) - rk4(inst, x, u - du)) / (2 * e)
        np.testing.assert_allclose(B[:, j], col, atol=1e-8)


def test_linear_model_error_is_second_order():
    """F(xbar + t dx) - [A (xbar + t dx) + B ubar + d] = O(t^2) (first-order Taylor, Sec. III-A)."""
    inst = _quad()
    rng = np.random.default_rng(9)
    x = np.concatenate([rng.uniform(-5, 5, 3), rng.uniform(-4, 4, 3)])
    u = rng.uniform(-10, 15, 3)
    _, A, B, d = rk4_jac(inst, x, u)
    dx = rng.normal(size=6)
    errs = []
    for t in (1e-2, 5e-3):
        xp = x + t * dx
        errs.append(np.max(np.abs(rk4(inst, xp, u) - (A @ xp + B @ u + d))))
    assert 3.5 < errs[0] / errs[1] < 4.5


def test_drag_jacobian_at_rest_is_zero():
    """At v = 0 the drag Jacobian c(||v|| I + v v'/||v||) is taken as 0 (it is 0 in the limit)."""
    inst = _quad()
    Jx, Ju = jac_cont(inst, np.zeros(6), np.zeros(3))
    assert np.all(Jx[3:6, 3:6] == 0.0)
    np.testing.assert_allclose(Ju[3:6], np.eye(3))


def test_mars_scaled_constants():
    """Scaled units of the powered-descent model: L = 1000 m, tau = 10 s, M = 1905 kg."""
    d = scpgen.mars_instance(2, 0)
    assert abs(d["grav"] - 0.37114) < 1e-12
    assert abs(d["alpha"] - 10.0 * 19050.0 / (1905.0 * 225.0 * 9.807)) < 1e-15
    assert abs(d["u_lo"][3] - 3000.0 / 19050.0) < 1e-15
    assert abs(d["u_hi"][3] - 13000.0 / 19050.0) < 1e-15
    assert abs(d["glide_tan"] - 14.300666256711942) < 1e-12
    assert abs(d["h"] - 5.0 / 60) < 1e-15

"""Pins for the oracle's projections (Sec. II prox-friendly sets, Sec. III-B Step 3).

A Euclidean projection P onto a closed convex set C is characterized by
feasibility, idempotence, the variational inequality <v - Pv, y - Pv> <= 0 for
all y in C, and non-expansiveness; these are checked on random points, and a
few points are compared with a generic constrained minimizer (SLSQP).
"""
import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import proj_box, proj_halfspace, proj_ball, proj_soc, proj_cone

KAPPA = np.tan(np.radians(86.0))


def _sets():
    rng = np.random.default_rng(0)
    lo = np.array([-1.0, -2.0, 0.5])
    hi = np.array([1.0, 0.0, 0.5])   # degenerate component lo == hi (an equality)
    a = rng.normal(size=3)
    b = 0.7
    return {
        "box": (lambda v: proj_box(v, lo, hi), lambda y: np.all(y >= lo - 1e-12) and np.all(y <= hi + 1e-12),
                lambda r, n: np.clip(r.normal(size=(n, 3)) * 3, lo, hi), 3),
        "halfspace": (lambda v: proj_halfspace(v, np.broadcast_to(a, v.shape), np.full(v.shape[0], b)),
                      lambda y: a @ y >= b - 1e-12,
                      lambda r, n: (lambda p: proj_halfspace(p, np.broadcast_to(a, p.shape), np.full(n, b)) + np.abs(r.normal(size=(n, 1))) * a)(r.normal(size=(n, 3)) * 3), 3),
        "ball": (lambda v: proj_ball(v, 2.0), lambda y: np.linalg.norm(y) <= 2.0 + 1e-12,
                 lambda r, n: (lambda p: p / np.maximum(1, np.linalg.norm(p, axis=1, keepdims=True) / (2 * r.uniform(size=(n, 1)))))(r.normal(size=(n, 3)) * 3), 3),
        "soc": (proj_soc, lambda y: np.linalg.norm(y[:-1]) <= y[-1] + 1e-12,
                lambda r, n: (lambda t: np.concatenate([t, (np.linalg.norm(t, axis=1) + np.abs(r.normal(size=n)))[:, None]], axis=1))(r.normal(size=(n, 3))), 4),
        "cone": (lambda v: proj_cone(v, KAPPA), lambda y: np.linalg.norm(y[:-1]) <= KAPPA * y[-1] + 1e-12,
                 lambda r, n: (lambda t: np.concatenate([t, (np.linalg.norm(t, axis=1) / KAPPA + np.abs(r.normal(size=n)))[:, None]], axis=1))(r.normal(size=(n, 2))), 3),
    }


@pytest.mark.parametrize("name", ["box", "halfspace", "ball", "soc", "cone"])
def test_projection_characterization(name):
    P, member, sample, dim = _sets()[name]
    rng = np.random.default_rng(1)
    v = rng.normal(size=(400, dim)) * 4
    pv = P(v)
    for row in pv:
        assert member(row)
    np.testing.assert_allclose(P(pv), pv, atol=1e-12)           # idempotent
    ys = sample(rng, 200)
    for y in ys:
        assert member(y)
    # variational inequality <v - Pv, y - Pv> <= 0 for every y in C
    vi = np.einsum("ij,kj->ik", v - pv, ys) - np.sum((v - pv) * pv, axis=1, keepdims=True)
    assert np.max(vi) <= 1e-9
    # non-expansive
    w = rng.normal(size=(400, dim)) * 4
    assert np.all(np.linalg.norm(P(w) - pv, axis=1) <= np.linalg.norm(w - v, axis=1) + 1e-12)


@pytest.mark.parametrize("name", ["halfspace", "ball", "soc", "cone"])
def test_projection_matches_generic_minimizer(name):
    P, member, _, dim = _sets()[name]
    rng = np.random.default_rng(2)
    cons = {
        "halfspace": None,
        "ball": lambda y: 2.0 - np.linalg.norm(y),
        "soc": lambda y: y[-1] - np.linalg.norm(y[:-1]),
        "cone": lambda y: KAPPA * y[-1] - np.linalg.norm(y[:-1]),
    }[name]
    for _ in range(5):
        v = rng.normal(size=dim) * 3
        pv = P(v[None])[0]
        if cons is None:
            continue
        res = minimize(lambda y: 0.5 * np.sum((y - v) ** 2), pv + 0.1 * rng.normal(size=dim),
                       constraints=[{"type": "ineq", "fun": cons}], method="SLSQP",
                       options={"ftol": 1e-14, "maxiter": 500})
        assert 0.5 * np.sum((pv - v) ** 2) <= res.fun + 1e-7


def test_projection_ties():
    # SOC with zero radial part: (0, s) -> (0, max(s, 0))
    np.testing.assert_array_equal(proj_soc(np.array([[0.0, 0.0, 0.0, -1.0]])), [[0, 0, 0, 0]])
    np.testing.assert_array_equal(proj_soc(np.array([[0.0, 0.0, 0.0, 2.0]])), [[0, 0, 0, 2.0]])
    # point on the boundary stays
    v = np.array([[3.0, 4.0, 5.0]])
    np.testing.assert_allclose(proj_soc(np.array([[3.0, 4.0, 0.0, 5.0]])), [[3, 4, 0, 5]])
    np.testing.assert_allclose(proj_ball(v, 5.0 * np.sqrt(2)), v)
    # half-space with a'v == b: both branches give v
    a = np.array([[0.0, 0.0, 2.0]])
    np.testing.assert_array_equal(proj_halfspace(np.array([[1.0, 2.0, 0.5]]), a, np.array([1.0])), [[1.0, 2.0, 0.5]])
    # ball at the origin
    np.testing.assert_array_equal(proj_ball(np.zeros((1, 3)), 1.0), np.zeros((1, 3)))
    # scaled cone reduces to the SOC at kappa = 1
    rng = np.random.default_rng(4)
    w = rng.normal(size=(50, 4))
    np.testing.assert_allclose(proj_cone(w, 1.0), proj_soc(w))


def test_soc_closed_form_example():
    """(t, s) = ((3, 4), 0): ||t|| = 5 > |s| -> ((5 + 0)/2) (t/5, 1) = (1.5, 2, 2.5)."""
    np.testing.assert_allclose(proj_soc(np.array([[3.0, 4.0, 0.0]])), [[1.5, 2.0, 2.5]], atol=1e-15)

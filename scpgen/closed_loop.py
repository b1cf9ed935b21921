"""The simulated world of the closed-loop robust-MPC experiment (Sec. IV-A.4 of the paper).

This is the environment the controller acts on, not the solver: the true plant (the point-mass
quadrotor plus an unmodelled crosswind), the seeded noise draws, and the scenario requests the
controller hands to a solver.  The solver's own model never calls into this module; the plant is
integrated here with its own sub-stepped scheme so that the world is simulated more finely than
the controller predicts it.

Scene (the paper's numbers where it gives them):
  * start (-4, -5, 2) m at rest, target (5, 5, 2) m at rest;
  * one vertical cylinder of radius 3.0 m at the origin, planned with a 0.5 m buffer
    (radius 3.5 m in the requests);
  * crosswind inside the corridor -2.5 < x < 2.5: base acceleration (0, 2.5, -1.0) m/s^2 plus
    Gaussian noise (standard deviation ``WIND_SIGMA`` per axis, drawn per MPC step);
  * S scenarios over a horizon of N intervals; scenario s carries the disturbance estimate plus
    ``SCEN_SIGMA`` times a standard normal draw (scenario 0 carries the estimate itself).

The controller plans in deviation coordinates around hover: its control is the thrust
acceleration minus g e3, so the planning model has no gravity term and the cost
2 ||du||^2 + 100 ||x_N - x_goal||^2 makes hovering at the target free (with the full thrust in
the cost, as in the batch workloads, a receding horizon settles short of the target).  The
plant adds g e3 back.  Bounds: |du_x|, |du_y| <= 15 and the full vertical thrust in [-15, 15].
"""
from __future__ import annotations

import math

import numpy as np

G = 9.81
START = np.array([-4.0, -5.0, 2.0])
TARGET = np.array([5.0, 5.0, 2.0])
CYL_CENTER = np.array([0.0, 0.0, 2.0])
CYL_RADIUS = 3.0
CYL_BUFFER = 0.5
WIND_BASE = np.array([0.0, 2.5, -1.0])
WIND_XMIN, WIND_XMAX = -2.5, 2.5
WIND_SIGMA = 0.5
SCEN_SIGMA = 0.5
PLANT_DRAG = 0.1
PLANT_SUBSTEPS = 10


def scene_instance(N: int = 30, T: float = 5.0, delta: float = 1.0) -> dict:
    """Problem template of the scene: a quadrotor from START to TARGET around the buffered
    cylinder (scenario-independent data; x_init and the disturbance are set per request)."""
    nx, nu = 6, 3
    x_goal = np.concatenate([TARGET, np.zeros(3)])
    x_init = np.concatenate([START, np.zeros(3)])
    s = np.linspace(0.0, 1.0, N + 1)[:, None]
    x_guess = np.zeros((N + 1, nx))
    x_guess[:, :3] = START + s * (TARGET - START)
    x_guess[:, 3:] = (TARGET - START) / T
    inf = math.inf
    return dict(
        model=1, N=N, h=T / N, nx=nx, nu=nu,
        x_init=x_init, x_target=x_goal.copy(), t_mask=np.zeros(nx, dtype=bool),
        Qr=np.zeros(nx), R=np.full(nu, 2.0),
        Qn=np.full(nx, 200.0), qn=-200.0 * x_goal, cN=100.0 * float(x_goal @ x_goal),
        x_lo=np.full(nx, -inf), x_hi=np.full(nx, inf),
        u_lo=np.array([-15.0, -15.0, -15.0 - G]), u_hi=np.array([15.0, 15.0, 15.0 - G]), u_ball=inf,
        delta=delta, drag=PLANT_DRAG, mscale=1.0, grav=0.0,
        obstacles=np.array([[*CYL_CENTER, CYL_RADIUS + CYL_BUFFER]]), cyl=np.array([True]),
        dist=np.zeros(3),
        alpha=0.0, gvec=np.array([0.0, 0.0, -G]), glide_tan=inf,
        x_guess=x_guess, u_guess=np.zeros((N, nu)), group=-1,
    )


def draws(seed: int, steps: int, S: int) -> dict:
    """Seeded noise of a closed-loop run: scenario draws xi (steps, S, 3) with xi[:, 0] = 0, and
    wind noise (steps, 3).  Draw order: for every step, the S-1 scenario vectors, then the wind."""
    g = np.random.Generator(np.random.PCG64(5000 + seed))
    xi = np.zeros((steps, S, 3))
    wn = np.zeros((steps, 3))
    for k in range(steps):
        xi[k, 1:] = g.standard_normal((S - 1, 3))
        wn[k] = g.standard_normal(3)
    return dict(xi=xi, wind=wn)


def request(template: dict, x_meas: np.ndarray, d_hat: np.ndarray, xi_step: np.ndarray, group: int = 0) -> list[dict]:
    """The S scenario problems of one MPC step: every scenario starts at the measured state and
    carries the disturbance estimate plus its scaled draw; all share the first control."""
    out = []
    for s in range(xi_step.shape[0]):
        c = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in template.items()}
        c["x_init"] = np.array(x_meas, dtype=float)
        c["dist"] = np.asarray(d_hat, dtype=float) + SCEN_SIGMA * xi_step[s]
        c["group"] = group
        out.append(c)
    return out


def wind(p: np.ndarray, noise: np.ndarray) -> np.ndarray:
    """Crosswind acceleration at position p for one step (zero outside the corridor)."""
    if WIND_XMIN < p[0] < WIND_XMAX:
        return WIND_BASE + WIND_SIGMA * noise
    return np.zeros(3)


def plant_step(x: np.ndarray, du: np.ndarray, h: float, w: np.ndarray) -> np.ndarray:
    """True plant over one control interval under the thrust deviation du from hover: the point
    mass with quadratic drag and the wind acceleration w held over the interval,
    PLANT_SUBSTEPS classical Runge-Kutta sub-steps."""
    def rhs(y):
        v = y[3:]
        sp = math.sqrt(float(v @ v))
        a = du - PLANT_DRAG * sp * v + w
        return np.concatenate([v, a])

    y = np.array(x, dtype=float)
    dt = h / PLANT_SUBSTEPS
    for _ in range(PLANT_SUBSTEPS):
        k1 = rhs(y)
        k2 = rhs(y + 0.5 * dt * k1)
        k3 = rhs(y + 0.5 * dt * k2)
        k4 = rhs(y + dt * k3)
        y = y + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return y


def clearance(p: np.ndarray) -> float:
    """Horizontal distance from p to the (unbuffered) cylinder surface; negative inside."""
    return float(math.hypot(p[0] - CYL_CENTER[0], p[1] - CYL_CENTER[1]) - CYL_RADIUS)

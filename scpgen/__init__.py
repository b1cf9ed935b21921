"""Seeded synthetic problem instances for the SCP + consensus-ADMM hot path.

This module only draws random problem data and writes it out as plain
numpy arrays.  It holds none of the solver's arithmetic: no dynamics, no
linearization, no projections.  Both the CPU oracle (``oracle/``) and the
GPU binding consume the instance dictionaries it returns; neither shares any
other code with the other.

Every instance is a ``dict`` with the physical problem in solver units:

``model``       1 = quadrotor point mass (nx=6, nu=3), 2 = 3-DOF powered descent (nx=7, nu=4),
                3 = 6-DOF quadrotor (nx=13: p, v, quaternion, body rates; nu=4: thrust, torques),
                4 = 6-DOF lander (nx=14: r, v, quaternion, body rates, mass; nu=3: body thrust)
``N``           number of intervals (N+1 state nodes, N control nodes)
``h``           step size T/N
``x_init``      initial state (boundary condition x_0 = x_init, eq. (ocp))
``x_target``    terminal target, ``t_mask`` selects the fixed components (S in eq. (ocp))
``Qr``, ``R``   diagonals of the running state / control Hessians
``Qn``, ``qn``, ``cN``  terminal cost 0.5 x'diag(Qn)x + qn'x + cN
``x_lo``/``x_hi``/``u_lo``/``u_hi``  hard bounds (+-inf where absent)
``u_ball``      radius of the control ball ||u|| <= u_ball (quadrotor; inf = none)
``delta``       trust-region radius (l-inf box around the nominal)
``drag``, ``mscale``, ``grav``  quadrotor drag coefficient, mass scale (6-DOF: the mass), gravity
``inertia``     (3,), 6-DOF principal moments of inertia
``arm``         (3,), 6-DOF lander: thrust point in the body frame
``T_min``, ``T_max``, ``gimbal_tan``, ``tilt_r``, ``w_max``  6-DOF lander: thrust magnitude bounds,
                tangent of the gimbal angle, tilt bound as ||(q_y, q_z)|| <= sin(tilt/2), rate bound
``obstacles``   (K, 4) obstacle centres and radii (quadrotor)
``cyl``         (K,) bool, optional: obstacle j is a vertical cylinder (axis along z through
                its centre) instead of a sphere
``dist``        (3,), optional: constant disturbance acceleration in the quadrotor model
``alpha``, ``gvec``, ``glide_tan``  powered-descent mass-flow coefficient, gravity vector,
                tangent of the glide-slope half angle
``x_guess``, ``u_guess``  initial nominal trajectory, shapes (N+1, nx) and (N, nu)
``group``       scenario group id; trajectories of one group share their first control
                by consensus (robust MPC, Sec. IV-A.4 of the paper)

RNG: ``numpy.random.Generator(PCG64(1000*config + instance))`` with a fixed draw
order (start, goal, obstacles; or r0, v0; then per-scenario parameters).
"""
from __future__ import annotations

import math

import numpy as np

QUAD = 1
MARS = 2
QUAD6 = 3
LANDER6 = 4
NX = {QUAD: 6, MARS: 7, QUAD6: 13, LANDER6: 14}
NU = {QUAD: 3, MARS: 4, QUAD6: 4, LANDER6: 3}
KMAX = 8  # most obstacles one quadrotor instance may carry

G_EARTH = 9.81

# Powered-descent scaling: length 1000 m, time 10 s, mass 1905 kg (force unit 19050 N).
MARS_L, MARS_TAU, MARS_M = 1000.0, 10.0, 1905.0
MARS_F = MARS_M * MARS_L / MARS_TAU ** 2
MARS_G = 3.7114
MARS_ISP_G0 = 225.0 * 9.807


def _rng(config: int, instance: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1000 * config + instance))


def quad_instance(config: int, instance: int, N: int = 30, K: int = 4, T: float = 5.0,
                  delta: float = 1.0, drag: float = 0.1, mscale: float = 1.0,
                  rng: np.random.Generator | None = None) -> dict:
    """Quadrotor point mass p' = v, v' = u/m - g e3 - c|v|v with K spherical obstacles.

    Cost sum ||u||^2 + 100 ||x_N - x_goal||^2, |u_j| <= 15, ||u|| <= 20.
    Start and goal are redrawn while they sit within r + 0.25 of an obstacle.
    """
    if not 0 <= K <= KMAX:
        raise ValueError(f"K must be in [0, {KMAX}]")
    g = rng if rng is not None else _rng(config, instance)
    start = g.uniform(-5.0, 5.0, 3)
    goal = g.uniform(-5.0, 5.0, 3)
    obs = np.zeros((K, 4))
    for j in range(K):
        obs[j, :3] = g.uniform(-3.0, 3.0, 3)
        obs[j, 3] = g.uniform(0.5, 1.0)

    def clear(p):
        return all(np.linalg.norm(p - obs[j, :3]) >= obs[j, 3] + 0.25 for j in range(K))

    while not clear(start):
        start = g.uniform(-5.0, 5.0, 3)
    while not clear(goal):
        goal = g.uniform(-5.0, 5.0, 3)

    nx, nu = 6, 3
    x_goal = np.concatenate([goal, np.zeros(3)])
    s = np.linspace(0.0, 1.0, N + 1)[:, None]
    x_guess = np.zeros((N + 1, nx))
    x_guess[:, :3] = start + s * (goal - start)
    x_guess[:, 3:] = (goal - start) / T
    u_guess = np.tile(np.array([0.0, 0.0, G_EARTH]), (N, 1))
    inf = math.inf
    return dict(
        model=QUAD, N=N, h=T / N, nx=nx, nu=nu,
        x_init=np.concatenate([start, np.zeros(3)]),
        x_target=x_goal.copy(), t_mask=np.zeros(nx, dtype=bool),
        Qr=np.zeros(nx), R=np.full(nu, 2.0),
        Qn=np.full(nx, 200.0), qn=-200.0 * x_goal, cN=100.0 * float(x_goal @ x_goal),
        x_lo=np.full(nx, -inf), x_hi=np.full(nx, inf),
        u_lo=np.full(nu, -15.0), u_hi=np.full(nu, 15.0), u_ball=20.0,
        delta=delta, drag=drag, mscale=mscale, grav=G_EARTH,
        obstacles=obs, alpha=0.0, gvec=np.array([0.0, 0.0, -G_EARTH]), glide_tan=inf,
        x_guess=x_guess, u_guess=u_guess, group=-1,
    )


def mars_instance(config: int, instance: int, N: int = 60, tf: float = 50.0,
                  delta: float = 1.0, rng: np.random.Generator | None = None) -> dict:
    """3-DOF powered descent r' = v, v' = T/m + g, m' = -Gamma/(Isp g0), in scaled units.

    SOC ||T|| <= Gamma, 3000 N <= Gamma <= 13000 N, glide-slope half angle 86 deg,
    r_N = 0 and v_N = 0, cost -m_N, m_0 = 1905 kg.
    """
    g = rng if rng is not None else _rng(config, instance)
    r0 = np.array([g.uniform(-500.0, 500.0), g.uniform(-500.0, 500.0), g.uniform(1200.0, 1800.0)])
    v0 = g.uniform(-50.0, 50.0, 3)
    nx, nu = 7, 4
    tf_s = tf / MARS_TAU
    gz = MARS_G * MARS_TAU ** 2 / MARS_L
    x_init = np.concatenate([r0 / MARS_L, v0 * MARS_TAU / MARS_L, [1.0]])
    s = np.linspace(0.0, 1.0, N + 1)[:, None]
    x_guess = np.zeros((N + 1, nx))
    x_guess[:, :6] = (1.0 - s) * x_init[:6]
    x_guess[:, 6] = 1.0
    u_guess = np.tile(np.array([0.0, 0.0, gz, gz]), (N, 1))
    inf = math.inf
    t_mask = np.array([True] * 6 + [False])
    return dict(
        model=MARS, N=N, h=tf_s / N, nx=nx, nu=nu,
        x_init=x_init, x_target=np.zeros(nx), t_mask=t_mask,
        Qr=np.zeros(nx), R=np.zeros(nu),
        Qn=np.zeros(nx), qn=np.array([0.0] * 6 + [-1.0]), cN=0.0,
        x_lo=np.full(nx, -inf), x_hi=np.full(nx, inf),
        u_lo=np.array([-inf, -inf, -inf, 3000.0 / MARS_F]),
        u_hi=np.array([inf, inf, inf, 13000.0 / MARS_F]), u_ball=inf,
        delta=delta, drag=0.0, mscale=1.0, grav=gz,
        obstacles=np.zeros((0, 4)),
        alpha=MARS_TAU * MARS_F / (MARS_M * MARS_ISP_G0),
        gvec=np.array([0.0, 0.0, -gz]), glide_tan=math.tan(math.radians(86.0)),
        x_guess=x_guess, u_guess=u_guess, group=-1,
    )


# 6-DOF quadrotor (Sec. IV-A.1): mass 1 kg, g = 9.81 m/s^2, thrust in [0, 20] N, body torques in
# [-5, 5] N m.  The paper takes the rest of the vehicle from a simulator it cites; the principal
# moments of inertia here are a stated choice for a 1 kg quadrotor.
Q6_MASS = 1.0
Q6_INERTIA = np.array([0.02, 0.02, 0.04])
Q6_START = np.array([-5.0, -5.0, 2.0])
Q6_GOAL = np.array([5.0, 5.0, 2.0])
# the parameter-study scene: three spheres (radii 1.2..1.5 m) across the direct path
Q6_SCENE_OBSTACLES = np.array([[-2.0, -1.6, 2.0, 1.2],
                               [0.3, 0.0, 2.2, 1.5],
                               [2.4, 2.0, 1.8, 1.3]])


def quad6_instance(obstacles: np.ndarray, N: int = 50, T: float = 6.0, delta: float = 1.0,
                   start: np.ndarray = Q6_START, goal: np.ndarray = Q6_GOAL,
                   guess_noise: float = 0.0, rng: np.random.Generator | None = None) -> dict:
    """6-DOF quadrotor from hover at ``start`` to ``goal`` with zero velocity there (both fixed:
    S selects position and velocity), spherical obstacles, cost sum ||u||^2 (R = 2 I).

    Initial guess: straight-line positions, constant velocity (goal - start)/T, level attitude
    q = (1, 0, 0, 0), zero rates, hover thrust m g; with ``guess_noise`` > 0 the interior
    positions and velocities get seeded Gaussian noise of that standard deviation
    ("noise-initialized" trajectories).
    """
    nx, nu = 13, 4
    x0 = np.zeros(nx)
    x0[:3] = start
    x0[6] = 1.0
    xg = np.zeros(nx)
    xg[:3] = goal
    xg[6] = 1.0
    s = np.linspace(0.0, 1.0, N + 1)[:, None]
    x_guess = np.zeros((N + 1, nx))
    x_guess[:, :3] = start + s * (goal - start)
    x_guess[:, 3:6] = (goal - start) / T
    x_guess[:, 6] = 1.0
    x_guess[0] = x0
    if guess_noise > 0.0:
        g = rng if rng is not None else np.random.default_rng(0)
        x_guess[1:N, :6] += guess_noise * g.standard_normal((N - 1, 6))
    u_guess = np.tile(np.array([Q6_MASS * G_EARTH, 0.0, 0.0, 0.0]), (N, 1))
    inf = math.inf
    t_mask = np.array([True] * 6 + [False] * 7)
    return dict(
        model=QUAD6, N=N, h=T / N, nx=nx, nu=nu,
        x_init=x0, x_target=xg, t_mask=t_mask,
        Qr=np.zeros(nx), R=np.full(nu, 2.0),
        Qn=np.zeros(nx), qn=np.zeros(nx), cN=0.0,
        x_lo=np.full(nx, -inf), x_hi=np.full(nx, inf),
        u_lo=np.array([0.0, -5.0, -5.0, -5.0]), u_hi=np.array([20.0, 5.0, 5.0, 5.0]), u_ball=inf,
        delta=delta, drag=0.0, mscale=Q6_MASS, grav=G_EARTH, inertia=Q6_INERTIA.copy(),
        obstacles=np.asarray(obstacles, dtype=float).reshape(-1, 4).copy(),
        alpha=0.0, gvec=np.array([0.0, 0.0, -G_EARTH]), glide_tan=inf,
        x_guess=x_guess, u_guess=u_guess, group=-1,
    )


def quad6_scene(N: int = 50, T: float = 6.0) -> dict:
    """The parameter-study scene of Sec. IV-A.2 (N = 50, 6 s, three obstacles)."""
    return quad6_instance(Q6_SCENE_OBSTACLES, N=N, T=T)


def quad6_benchmark_instance(instance: int, N: int = 40, T: float = 6.0, K: int = 3) -> dict:
    """One trajectory of the scalability benchmark of Sec. IV-A.3: K random spheres (radii
    U[1, 2] m) with centres drawn around the straight path (a point U[0.2, 0.8] of the way plus
    U[-1.5, 1.5]^3), redrawn while start or goal lies within r + 0.25; noise-initialized guess
    (standard deviation 0.1).  Draw order: per obstacle s, offset (3), radius; then the guess
    noise."""
    g = _rng(5, instance)
    obs = np.zeros((K, 4))
    for j in range(K):
        while True:
            sj = g.uniform(0.2, 0.8)
            c = Q6_START + sj * (Q6_GOAL - Q6_START) + g.uniform(-1.5, 1.5, 3)
            r = g.uniform(1.0, 2.0)
            if (np.linalg.norm(Q6_START - c) >= r + 0.25) and (np.linalg.norm(Q6_GOAL - c) >= r + 0.25):
                break
        obs[j, :3] = c
        obs[j, 3] = r
    return quad6_instance(obs, N=N, T=T, guess_noise=0.1, rng=g)


def config5(n_inst: int = 1000, first: int = 0) -> list[dict]:
    """6-DOF quadrotor batch of the scalability benchmark: N = 40, three random obstacles."""
    return [quad6_benchmark_instance(i) for i in range(first, first + n_inst)]


# 6-DOF lander (Sec. IV-B.1, unified non-dimensional units, position Up-East-North, body x along
# the thrust axis): the paper's alpha, horizon, mass, thrust, gimbal, glide-slope, tilt and rate
# limits and boundary states; gravity, inertia and thrust point are stated choices.
L6_ALPHA = 0.1
L6_TF, L6_N = 5.0, 30
L6_M_DRY, L6_M_WET = 0.75, 2.0
L6_T_MIN, L6_T_MAX = 0.5, 3.0
L6_GIMBAL_DEG, L6_GLIDE_DEG, L6_TILT_DEG, L6_WMAX_DEG = 10.0, 10.0, 20.0, 30.0
L6_GRAVITY = np.array([-1.0, 0.0, 0.0])
L6_INERTIA = np.array([0.02, 0.1, 0.1])
L6_ARM = np.array([-0.25, 0.0, 0.0])
L6_R0, L6_V0 = np.array([2.0, 1.0, 0.0]), np.array([-1.0, 0.2, 0.0])
L6_VF = np.array([-0.1, 0.0, 0.0])


def _l6_nominal_state() -> np.ndarray:
    x = np.zeros(14)
    x[0:3] = L6_R0
    x[3:6] = L6_V0
    x[6] = 1.0
    x[13] = L6_M_WET
    return x


def lander6_instance(x_init: np.ndarray | None = None, N: int = L6_N, tf: float = L6_TF, delta: float = 1.0) -> dict:
    """6-DOF powered descent to rest-like touchdown: r_N = 0, v_N = (-0.1, 0, 0), upright and
    not rotating (S selects every state but the mass), cost -m_N (fuel), dry mass <= m <= wet
    mass.  Initial guess: r and v linear to the target, upright, no rotation, full mass, thrust
    m g along the body axis."""
    nx, nu = 14, 3
    x0 = _l6_nominal_state() if x_init is None else np.asarray(x_init, dtype=float)
    xf = np.zeros(nx)
    xf[3:6] = L6_VF
    xf[6] = 1.0
    xf[13] = L6_M_DRY
    t_mask = np.array([True] * 13 + [False])
    s = np.linspace(0.0, 1.0, N + 1)[:, None]
    x_guess = np.zeros((N + 1, nx))
    x_guess[:, 0:6] = (1.0 - s) * x0[0:6] + s * xf[0:6]
    x_guess[:, 6] = 1.0
    x_guess[:, 13] = x0[13]
    x_guess[0] = x0
    u_guess = np.tile(np.array([x0[13] * -L6_GRAVITY[0], 0.0, 0.0]), (N, 1))
    inf = math.inf
    x_lo = np.full(nx, -inf)
    x_hi = np.full(nx, inf)
    x_lo[13], x_hi[13] = L6_M_DRY, L6_M_WET
    qn = np.zeros(nx)
    qn[13] = -1.0
    return dict(
        model=LANDER6, N=N, h=tf / N, nx=nx, nu=nu,
        x_init=x0.copy(), x_target=xf, t_mask=t_mask,
        Qr=np.zeros(nx), R=np.zeros(nu), Qn=np.zeros(nx), qn=qn, cN=0.0,
        x_lo=x_lo, x_hi=x_hi, u_lo=np.full(nu, -inf), u_hi=np.full(nu, inf), u_ball=inf,
        delta=delta, drag=0.0, mscale=1.0, grav=0.0, alpha=L6_ALPHA, gvec=L6_GRAVITY.copy(),
        inertia=L6_INERTIA.copy(), arm=L6_ARM.copy(),
        glide_tan=math.tan(math.radians(90.0 - L6_GLIDE_DEG)),
        tilt_r=math.sin(math.radians(L6_TILT_DEG / 2.0)), w_max=math.radians(L6_WMAX_DEG),
        T_min=L6_T_MIN, T_max=L6_T_MAX, gimbal_tan=math.tan(math.radians(L6_GIMBAL_DEG)),
        obstacles=np.zeros((0, 4)), x_guess=x_guess, u_guess=u_guess, group=-1,
    )


def lander6_perturbed(instance: int) -> dict:
    """Monte-Carlo member of Sec. IV-B.2: every initial state component perturbed by 5 %: a
    nonzero component k becomes x_k (1 + 0.05 e_k), a zero one 0.05 e_k, e_k ~ U[-1, 1]
    (draw order: the 14 components); then the quaternion is renormalized and the mass capped
    at the wet mass."""
    g = _rng(6, instance)
    x = _l6_nominal_state()
    e = g.uniform(-1.0, 1.0, 14)
    x = np.where(x != 0.0, x * (1.0 + 0.05 * e), 0.05 * e)
    x[6:10] /= np.linalg.norm(x[6:10])
    x[13] = min(x[13], L6_M_WET)
    return lander6_instance(x)


def config6(n_inst: int = 1000, first: int = 0) -> list[dict]:
    """6-DOF lander Monte Carlo: N = 30, horizon 5, 5 % initial-state dispersion."""
    return [lander6_perturbed(i) for i in range(first, first + n_inst)]


def with_scenarios(base: dict, S: int, rng: np.random.Generator, group: int) -> list[dict]:
    """S copies of a quadrotor instance with drag ~ U[0.05, 0.2] and mass scale ~ U[0.9, 1.1].

    All copies share x_init, goal and obstacles and form one consensus group.
    """
    out = []
    for _ in range(S):
        c = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in base.items()}
        c["drag"] = float(rng.uniform(0.05, 0.2))
        c["mscale"] = float(rng.uniform(0.9, 1.1))
        c["group"] = group
        out.append(c)
    return out


# ---------------------------------------------------------------------------------------------
# Workloads (shapes of the paper's quadrotor and powered-descent experiments)
# ---------------------------------------------------------------------------------------------

def config0() -> list[dict]:
    """Single quadrotor instance, N=30, T=5 s, 4 obstacles (solved in FP64)."""
    return [quad_instance(0, 0, N=30, K=4, T=5.0)]


def config1(n_inst: int = 1024, first: int = 0) -> list[dict]:
    """Independent quadrotor instances, N=50, T=5 s, 8 obstacles each (FP32 batch)."""
    return [quad_instance(1, i, N=50, K=8, T=5.0) for i in range(first, first + n_inst)]


def config2(n_inst: int = 4096, first: int = 0) -> list[dict]:
    """Powered-descent Monte Carlo, N=60, tf=50 s."""
    return [mars_instance(2, i, N=60, tf=50.0) for i in range(first, first + n_inst)]


def config3(n_inst: int = 2048, first: int = 0) -> list[dict]:
    """Uneven mix: half quadrotor (8 obstacles, T=5 s), half powered descent (tf=50 s),
    horizons N ~ U{20..120}, order given by a seeded permutation."""
    perm = np.random.Generator(np.random.PCG64(3000 + 999_999)).permutation(n_inst)
    out = []
    for i in range(first, first + n_inst):
        g = _rng(3, i)
        N = int(g.integers(20, 121))
        if perm[i] % 2 == 0:
            out.append(quad_instance(3, i, N=N, K=8, T=5.0, rng=g))
        else:
            out.append(mars_instance(3, i, N=N, tf=50.0, rng=g))
    return out


def config4_request(session: int, S: int = 16, N: int | None = None) -> list[dict]:
    """One robust-MPC request: S scenarios of a quadrotor (4 obstacles, N ~ U{30..80})
    sharing the first control.  Drag and mass scale are drawn per scenario."""
    g = _rng(4, session)
    if N is None:
        N = int(g.integers(30, 81))
    base = quad_instance(4, session, N=N, K=4, T=5.0, rng=g)
    return with_scenarios(base, S, g, group=session)


def horizon_mix_stats(insts: list[dict]) -> dict:
    """Counts used to state the workload in results (nodes, models)."""
    nodes = sum(d["N"] + 1 for d in insts)
    return dict(instances=len(insts), nodes=nodes,
                quad=sum(d["model"] == QUAD for d in insts),
                mars=sum(d["model"] == MARS for d in insts))

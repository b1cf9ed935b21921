"""Outer SCP loop (Sec. III-A) around the consensus ADMM, with trust-region acceptance.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Per SCP iteration k (Fig. method_overview: linearize -> convex QP -> update nominal):
  a2  A_i, B_i, d_i from the exact Jacobians of the RK4 map at the nominal (Sec. III-A)
  a3  convex sets of eq. (qp_subproblem): trust box around the nominal intersected with the
      hard bounds, boundary conditions of eq. (ocp) as degenerate boxes, obstacle spheres
      linearized into half-spaces at the nominal, control ball / SOC / glide-slope cone
  a4  Step-1 Hessians; ADMM primal state re-initialized from the nominal, duals carried over
  a5-a9  ADMM iterations (oracle.admm)
  a10 candidate = last physical iterate; merit ratio test; nominal and trust radius update
      (the paper omits this logic and points to standard trust-region texts; the reading
      here is the classic ratio test on an l1 merit function)

Status bits of a group's info: ST_NONFINITE (a non-finite merit), ST_DIVERGED (residual blow-up,
with params["detect_blowup"]: the primal residual of an SCP iteration's last ADMM iteration above
RP_BLOWUP times the first positive one of the solve; the paper gives no such rule, it is failure
detection only).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .admm import Group, QP, AdmmState, build_H, admm_run
from .dynamics import rk4, rk4_jac, QUAD, MARS, QUAD6, LANDER6

ST_NONFINITE = 1
ST_DIVERGED = 32
RP_BLOWUP = 1.0e6


def default_params(**kw) -> dict:
    """Solver parameters; the defaults are the fixed-budget settings of the workloads
    (rho = 1 for all three penalties, always-accept steps, fixed trust radius).  rho_final > 0
    turns on the penalty schedule of penalty_factors; adapt_mu > 0 the residual balancing of
    adapt_penalty; detect_blowup the ST_DIVERGED status bit."""
    p = dict(scp_iters=10, admm_iters=100, rho_eq=1.0, rho_dyn=1.0, rho_geo=1.0, rho_final=0.0,
             adapt_mu=0.0, adapt_tau=2.0, detect_blowup=False,
             check_every=0, eps_p=0.0, eps_d=0.0,
             eta0=-math.inf, eta1=0.25, eta2=0.75, shrink=1.0, grow=1.0, delta_max=math.inf,
             merit_w=1.0e3)
    p.update(kw)
    return p


def penalty_factors(params: dict) -> list[float]:
    """Factor applied to all three penalties at each SCP iteration (Sec. IV-A.2, parameter
    study: the penalties are scaled geometrically over the SCP iterations up to a final value).

    Reading: with K SCP iterations, rho_eq grows from its given value to rho_final by a constant
    ratio q = (rho_final / rho_eq)^(1 / (K - 1)), evaluated once in double precision; the factor
    of iteration k is q^k formed by repeated multiplication (1, q, q*q, ...); rho_dyn and rho_geo
    keep their ratios to rho_eq.  rho_final <= 0, or K = 1, means no schedule.  The duals are
    carried across SCP iterations unscaled (they are the multipliers themselves)."""
    K = params["scp_iters"]
    rf = params.get("rho_final", 0.0) or 0.0
    q = (rf / params["rho_eq"]) ** (1.0 / (K - 1)) if rf > 0.0 and K > 1 else 1.0
    out, s = [], 1.0
    for _ in range(K):
        out.append(s)
        s = s * q
    return out


# ------------------------------------------------------------------------------------------
# a2: linearization
# ------------------------------------------------------------------------------------------

def adapt_penalty(scale: float, r_p: float, r_d: float, params: dict) -> float:
    """Adaptive penalty by residual balancing, applied between SCP iterations.

    The paper fixes the penalties or scales them on a schedule (Sec. IV-A.2) and gives no
    adaptive rule.  Reading: the residual-balancing rule of Boyd et al., "Distributed
    Optimization and Statistical Learning via ADMM" (2011), Sec. 3.4.1: when the primal residual
    exceeds mu times the dual one the penalty grows by tau, when the dual residual exceeds mu
    times the primal one it shrinks by tau, otherwise it stays.  Here one factor scales all three
    penalties of a group (on top of the schedule's factor), decided from the residuals of the
    last ADMM iteration of an SCP iteration, in double precision; the next SCP iteration builds
    its factor with the new penalties.  The duals are the unscaled multipliers and carry over
    unchanged.  NaN residuals leave the factor alone.  adapt_mu <= 0 turns the rule off."""
    mu = params.get("adapt_mu", 0.0) or 0.0
    if mu <= 0.0:
        return scale
    tau = params["adapt_tau"]
    if r_p > mu * r_d:
        return scale * tau
    if r_d > mu * r_p:
        return scale / tau
    return scale


def linearize(inst: dict, xbar: np.ndarray, ubar: np.ndarray):
    """A_i, B_i, d_i for i < N at the nominal (first-order expansion of the RK4 map)."""
    N, nx, nu = inst["N"], inst["nx"], inst["nu"]
    A = np.zeros((N, nx, nx))
    B = np.zeros((N, nx, nu))
    d = np.zeros((N, nx))
    for i in range(N):
        _, A[i], B[i], d[i] = rk4_jac(inst, xbar[i], ubar[i])
    return A, B, d


def cost_qp(inst: dict, A, B, d) -> QP:
    """Quadratic cost model of eq. (qp_subproblem).  The workloads' costs are already
    quadratic (sum u'Ru/2 + terminal x'Qn x/2 + qn'x), so the expansion is exact."""
    N, nx, nu = inst["N"], inst["nx"], inst["nu"]
    Q = np.zeros((N + 1, nx, nx))
    Q[:N] = np.diag(inst["Qr"])
    Q[N] = np.diag(inst["Qn"])
    q = np.zeros((N + 1, nx))
    q[N] = inst["qn"]
    R = np.broadcast_to(np.diag(inst["R"]), (N, nu, nu)).copy()
    return QP(Q=Q, q=q, R=R, r=np.zeros((N, nu)), M=np.zeros((N, nx, nu)), A=A, B=B, d=d)


# ------------------------------------------------------------------------------------------
# a3: convexification
# ------------------------------------------------------------------------------------------

def _trust_box(center, delta, lo_h, hi_h):
    """[center - delta, center + delta] intersected with [lo_h, hi_h]; if empty, the box
    collapses onto the hard-box point nearest the nominal (the hard bounds win)."""
    lo = np.maximum(center - delta, lo_h)
    hi = np.minimum(center + delta, hi_h)
    empty = lo > hi
    if np.any(empty):
        p = np.minimum(np.maximum(center, lo_h), hi_h)
        lo = np.where(empty, p, lo)
        hi = np.where(empty, p, hi)
    return lo, hi


def _cyl_flags(inst: dict) -> np.ndarray:
    """Per obstacle: True for a vertical cylinder (axis along z), False for a sphere."""
    K = inst["obstacles"].shape[0]
    flags = np.zeros(K, dtype=bool)
    given = np.asarray(inst.get("cyl", ()), dtype=bool)
    flags[:min(K, given.size)] = given[:K]
    return flags


def convexify(inst: dict, xbar: np.ndarray, ubar: np.ndarray, delta: float, u0_center=None):
    """Constraint groups of the convex subproblem, in a fixed order.

    x box (all nodes): node 0 lo = hi = x_init; nodes 1..N trust box around xbar intersected
      with the hard state bounds; node N components selected by t_mask lo = hi = x_target.
    u box (nodes 0..N-1): trust box around ubar intersected with the hard control bounds;
      at node 0 the box is centred at ``u0_center`` when given (scenario groups share one
      first-control set).
    Quadrotors: control ball ||u|| <= u_ball (point mass only, nodes 0..N-1), then one
      half-space per obstacle at nodes 1..N: n'(p - c) >= r with n = (pbar - c)/||pbar - c||
      (+e3 if ||pbar - c|| < 1e-9).  A vertical cylinder uses the horizontal part of pbar - c
      (fallback +e1).  The 6-DOF model's position is its first three states as well.
    Powered descent: glide-slope cone ||(r_x, r_y)|| <= tan(86 deg) r_z at nodes 1..N, then
      the SOC ||T|| <= Gamma at nodes 0..N-1.
    6-DOF lander (position Up-East-North): at nodes 1..N the glide-slope cone
      ||(r_E, r_N)|| <= glide_tan r_U (components (1, 2, 0): the axis last), the tilt limit
      ||(q_y, q_z)|| <= tilt_r and the rate ball ||w|| <= w_max; at nodes 0..N-1 the thrust ball
      ||T|| <= T_max, the lower thrust bound ||T|| >= T_min linearized at the nominal thrust as
      the half-space n'T >= T_min with n = Tbar/||Tbar|| (+e1 if ||Tbar|| < 1e-9), and the
      gimbal cone ||(T_y, T_z)|| <= gimbal_tan T_x (components (1, 2, 0)).
    """
    N, nx, nu = inst["N"], inst["nx"], inst["nu"]
    allx = np.ones(N + 1, dtype=bool)
    xlo = np.zeros((N + 1, nx))
    xhi = np.zeros((N + 1, nx))
    xlo[0] = xhi[0] = inst["x_init"]
    for i in range(1, N + 1):
        xlo[i], xhi[i] = _trust_box(xbar[i], delta, inst["x_lo"], inst["x_hi"])
    m = inst["t_mask"]
    xlo[N, m] = inst["x_target"][m]
    xhi[N, m] = inst["x_target"][m]
    groups = [Group("x", tuple(range(nx)), "box", allx, lo=xlo, hi=xhi)]

    uact = np.ones(N + 1, dtype=bool)
    uact[N] = False
    ulo = np.zeros((N + 1, nu))
    uhi = np.zeros((N + 1, nu))
    for i in range(N):
        c = ubar[i] if (i > 0 or u0_center is None) else u0_center
        ulo[i], uhi[i] = _trust_box(c, delta, inst["u_lo"], inst["u_hi"])
    groups.append(Group("u", tuple(range(nu)), "box", uact, lo=ulo, hi=uhi))

    inner = np.ones(N + 1, dtype=bool)
    inner[0] = False
    if inst["model"] in (QUAD, QUAD6):
        if inst["model"] == QUAD and math.isfinite(inst["u_ball"]):
            groups.append(Group("u", (0, 1, 2), "ball", uact.copy(), radius=float(inst["u_ball"])))
        cyl = _cyl_flags(inst)
        for j in range(inst["obstacles"].shape[0]):
            c, r = inst["obstacles"][j, :3], inst["obstacles"][j, 3]
            a = np.zeros((N + 1, 3))
            b = np.zeros(N + 1)
            fallback = np.array([1.0, 0.0, 0.0]) if cyl[j] else np.array([0.0, 0.0, 1.0])
            for i in range(1, N + 1):
                dvec = xbar[i, :3] - c
                if cyl[j]:
                    dvec[2] = 0.0
                nd = np.sqrt(dvec @ dvec)
                nvec = dvec / nd if nd >= 1e-9 else fallback
                a[i] = nvec
                b[i] = r + nvec @ c
            groups.append(Group("x", (0, 1, 2), "halfspace", inner.copy(), a=a, b=b))
    elif inst["model"] == LANDER6:
        groups.append(Group("x", (1, 2, 0), "cone", inner.copy(), kappa=float(inst["glide_tan"])))
        groups.append(Group("x", (8, 9), "ball", inner.copy(), radius=float(inst["tilt_r"])))
        groups.append(Group("x", (10, 11, 12), "ball", inner.copy(), radius=float(inst["w_max"])))
        groups.append(Group("u", (0, 1, 2), "ball", uact.copy(), radius=float(inst["T_max"])))
        a = np.zeros((N + 1, 3))
        b = np.zeros(N + 1)
        for i in range(N):
            t = ubar[i]
            nt = np.sqrt(t @ t)
            a[i] = t / nt if nt >= 1e-9 else np.array([1.0, 0.0, 0.0])
            b[i] = float(inst["T_min"])
        groups.append(Group("u", (0, 1, 2), "halfspace", uact.copy(), a=a, b=b))
        groups.append(Group("u", (1, 2, 0), "cone", uact.copy(), kappa=float(inst["gimbal_tan"])))
    else:
        groups.append(Group("x", (0, 1, 2), "cone", inner.copy(), kappa=float(inst["glide_tan"])))
        groups.append(Group("u", (0, 1, 2, 3), "soc", uact.copy()))
    return groups


# ------------------------------------------------------------------------------------------
# metrics and merit
# ------------------------------------------------------------------------------------------

def cost(inst: dict, x: np.ndarray, u: np.ndarray) -> float:
    """Objective of eq. (ocp) for the workloads: sum_i (x_i'Qr x_i + u_i'R u_i)/2 over i < N plus
    x_N'Qn x_N/2 + qn'x_N + cN.  Summed in node order."""
    N = inst["N"]
    J = 0.0
    for i in range(N):
        J += 0.5 * float(x[i] @ (inst["Qr"] * x[i])) + 0.5 * float(u[i] @ (inst["R"] * u[i]))
    J += 0.5 * float(x[N] @ (inst["Qn"] * x[N])) + float(inst["qn"] @ x[N]) + inst["cN"]
    return J


def defect(inst: dict, x: np.ndarray, u: np.ndarray) -> float:
    """Max over i < N of ||x_{i+1} - RK4(x_i, u_i)||_inf (nonlinear dynamics defect)."""
    N = inst["N"]
    if N == 0:
        return 0.0
    return float(max(np.max(np.abs(x[i + 1] - rk4(inst, x[i], u[i]))) for i in range(N)))


def violation(inst: dict, x: np.ndarray, u: np.ndarray) -> float:
    """Max violation of the hard (unconvexified) constraints: state/control bounds, control
    ball, obstacles (penetration depth, nodes 1..N; horizontal distance for a cylinder),
    SOC ||T|| <= Gamma, glide slope; for the 6-DOF lander the thrust magnitude bounds (the lower
    one unconvexified), gimbal, glide slope, tilt and rate limits."""
    N = inst["N"]
    v = 0.0
    v = max(v, float(np.max(np.maximum(0.0, inst["x_lo"] - x))), float(np.max(np.maximum(0.0, x - inst["x_hi"]))))
    if N > 0:
        v = max(v, float(np.max(np.maximum(0.0, inst["u_lo"] - u))), float(np.max(np.maximum(0.0, u - inst["u_hi"]))))
    if inst["model"] in (QUAD, QUAD6):
        if inst["model"] == QUAD and N > 0 and math.isfinite(inst["u_ball"]):
            v = max(v, float(np.max(np.sqrt(np.sum(u[:, :3] ** 2, axis=1)) - inst["u_ball"])))
        cyl = _cyl_flags(inst)
        for j in range(inst["obstacles"].shape[0]):
            c, r = inst["obstacles"][j, :3], inst["obstacles"][j, 3]
            dims = 2 if cyl[j] else 3
            dist = np.sqrt(np.sum((x[1:, :dims] - c[:dims]) ** 2, axis=1))
            if dist.size:
                v = max(v, float(np.max(r - dist)))
    elif inst["model"] == LANDER6:
        if N > 0:
            nt = np.sqrt(np.sum(u[:N, :3] ** 2, axis=1))
            v = max(v, float(np.max(nt - inst["T_max"])), float(np.max(inst["T_min"] - nt)))
            v = max(v, float(np.max(np.sqrt(u[:N, 1] ** 2 + u[:N, 2] ** 2) - inst["gimbal_tan"] * u[:N, 0])))
            xs = x[1:]
            v = max(v, float(np.max(np.sqrt(xs[:, 1] ** 2 + xs[:, 2] ** 2) - inst["glide_tan"] * xs[:, 0])))
            v = max(v, float(np.max(np.sqrt(xs[:, 8] ** 2 + xs[:, 9] ** 2) - inst["tilt_r"])))
            v = max(v, float(np.max(np.sqrt(np.sum(xs[:, 10:13] ** 2, axis=1)) - inst["w_max"])))
    else:
        if N > 0:
            v = max(v, float(np.max(np.sqrt(np.sum(u[:, :3] ** 2, axis=1)) - u[:, 3])))
        rxy = np.sqrt(x[1:, 0] ** 2 + x[1:, 1] ** 2)
        if rxy.size:
            v = max(v, float(np.max(rxy - inst["glide_tan"] * x[1:, 2])))
    return max(v, 0.0)


def boundary_error(inst: dict, x: np.ndarray) -> float:
    """max(||x_0 - x_init||_inf, max |x_N - x_target| over the components selected by S)."""
    e = float(np.max(np.abs(x[0] - inst["x_init"])))
    m = inst["t_mask"]
    if np.any(m):
        e = max(e, float(np.max(np.abs(x[-1, m] - inst["x_target"][m]))))
    return e


def _merit_terms(inst, x, u, A=None, B=None, d=None):
    """(J, sum_i ||x_{i+1} - F_i||_1) with F_i the RK4 map, or the affine model if A is given."""
    N = inst["N"]
    pen = 0.0
    for i in range(N):
        if A is None:
            Fi = rk4(inst, x[i], u[i])
        else:
            Fi = A[i] @ x[i] + B[i] @ u[i] + d[i]
        pen += float(np.sum(np.abs(x[i + 1] - Fi)))
    return cost(inst, x, u), pen


# ------------------------------------------------------------------------------------------
# the SCP loop
# ------------------------------------------------------------------------------------------

@dataclass
class Traj:
    inst: dict
    xbar: np.ndarray
    ubar: np.ndarray
    state: AdmmState | None = None
    qp: QP | None = None
    groups: list = field(default_factory=list)


def init_traj(inst: dict) -> Traj:
    return Traj(inst, np.array(inst["x_guess"], dtype=float, copy=True),
                np.array(inst["u_guess"], dtype=float, copy=True))


def _prepare(trajs: list[Traj], delta: float, rho):
    """a2-a4 plus the primal re-initialization (primal state from the nominal, duals carried over)
    for every trajectory of one group."""
    u0c = None
    if len(trajs) > 1:
        acc = np.zeros(trajs[0].inst["nu"])
        for t in trajs:
            acc = acc + t.ubar[0]
        u0c = acc / len(trajs)
    out = []
    for t in trajs:
        inst = t.inst
        A, B, d = linearize(inst, t.xbar, t.ubar)
        t.qp = cost_qp(inst, A, B, d)
        t.groups = convexify(inst, t.xbar, t.ubar, delta, u0c)
        N = inst["N"]
        if t.state is None:
            t.state = AdmmState.zeros(N, inst["nx"], inst["nu"], t.groups)
        st = t.state
        st.x[:] = t.xbar
        st.u[:] = t.ubar
        st.z[:] = t.xbar
        st.z[0] = 0.0
        for gi, g in enumerate(t.groups):
            src = t.xbar if g.var == "x" else np.vstack([t.ubar, np.zeros((1, inst["nu"]))])
            st.copy[gi][:] = 0.0
            st.copy[gi][g.active] = src[g.active][:, list(g.comps)]
        out.append((t.qp, t.groups, st, build_H(t.qp, t.groups, rho)))
    return out


def scp_group(trajs: list[Traj], params: dict, delta: float | None = None) -> dict:
    """Solve one group of trajectories (a single trajectory, or scenarios sharing u_0).

    Returns the group's info; the trajectories' nominals hold the solution.
    """
    factors = penalty_factors(params)
    delta = trajs[0].inst["delta"] if delta is None else delta
    coupled = len(trajs) > 1
    iters_total = 0
    n_accept = 0
    rp = rd = float("nan")
    rp0 = 0.0     # blow-up reference: the first positive primal residual of the solve
    status = 0
    scale = 1.0   # adaptive factor of the penalties (adapt_penalty)
    for k in range(params["scp_iters"]):
        rho = (params["rho_eq"] * factors[k] * scale, params["rho_dyn"] * factors[k] * scale,
               params["rho_geo"] * factors[k] * scale)
        packs = _prepare(trajs, delta, rho)
        it, rp, rd = admm_run(packs, rho, params["admm_iters"], params["check_every"],
                              params["eps_p"], params["eps_d"], couple_u0=coupled)
        iters_total += it
        # a10: merit ratio test over the whole group (sums in trajectory order)
        m_nom = m_new = m_mod = 0.0
        w = params["merit_w"]
        for t in trajs:
            J0, p0 = _merit_terms(t.inst, t.xbar, t.ubar)
            J1, p1 = _merit_terms(t.inst, t.state.x, t.state.u)
            _, pm = _merit_terms(t.inst, t.state.x, t.state.u, t.qp.A, t.qp.B, t.qp.d)
            m_nom += J0 + w * p0
            m_new += J1 + w * p1
            m_mod += J1 + w * pm
        actual = m_nom - m_new
        pred = m_nom - m_mod
        ratio = actual / pred if pred > 0.0 else -math.inf
        if not (math.isfinite(m_new) and math.isfinite(m_mod)):
            ratio = math.nan
            status |= ST_NONFINITE
        if params.get("detect_blowup"):
            if rp0 > 0.0:
                if rp > RP_BLOWUP * rp0:
                    status |= ST_DIVERGED
            elif rp > 0.0:
                rp0 = rp
        if ratio >= params["eta0"]:
            n_accept += 1
            for t in trajs:
                t.xbar = t.state.x.copy()
                t.ubar = t.state.u.copy()
        if ratio < params["eta1"]:
            delta = delta * params["shrink"]
        elif ratio > params["eta2"]:
            delta = min(delta * params["grow"], params["delta_max"])
        scale = adapt_penalty(scale, rp, rd, params)
    return dict(admm_iters=iters_total, r_p=rp, r_d=rd, n_accept=n_accept, delta=delta, status=status,
                rho_scale=scale)


def scp_solve(insts: list[dict], params: dict | None = None):
    """Solve every instance (grouping consecutive instances that share a ``group`` id >= 0).

    Returns (list of (xbar, ubar), list of per-instance info dicts).
    """
    params = default_params() if params is None else params
    sols, infos = [None] * len(insts), [None] * len(insts)
    i = 0
    while i < len(insts):
        j = i + 1
        if insts[i]["group"] >= 0:
            while j < len(insts) and insts[j]["group"] == insts[i]["group"]:
                j += 1
        trajs = [init_traj(insts[k]) for k in range(i, j)]
        ginfo = scp_group(trajs, params)
        for k, t in zip(range(i, j), trajs):
            inf = dict(ginfo)
            inf.update(defect=defect(t.inst, t.xbar, t.ubar), cost=cost(t.inst, t.xbar, t.ubar),
                       viol=violation(t.inst, t.xbar, t.ubar), bnd_err=boundary_error(t.inst, t.xbar))
            sols[k] = (t.xbar, t.ubar)
            infos[k] = inf
        i = j
    return sols, infos


def shift_warm_start(trajs: list[Traj], next_insts: list[dict] | None = None, measured: bool = False) -> list[Traj]:
    """MPC warm start of the next request of a session (Sec. IV-A.4, receding horizon).

    Reading (the paper gives no formula): the next request starts one node later along the
    previous solution of every scenario.
      * state-indexed rows (nominal x, lambda, mu, duals of state groups; N+1 rows): row i takes
        row i+1 for i < N, row N is repeated;
      * control-indexed rows (nominal u, duals of control groups; rows 0..N-1): row i takes row
        i+1 for i < N-1, row N-1 is repeated;
      * lambda_0 = mu_0 = 0 (node 0 has no dynamic coupling), and every dual at a node where its
        group does not exist is 0;
      * the new initial state, for every scenario, is the previous scenario-0 nominal at node 1;
        with ``measured`` (closed-loop MPC) it is next_insts' own x_init, the measured state.
    The trust radius and the iteration records start afresh (the caller's scp_group does so).
    Returns new Traj objects; their instances are next_insts (the next request's data, same
    shapes) or copies of the previous ones, with the new x_init.  The inputs are unchanged.
    """
    x_init = np.array(trajs[0].xbar[1], dtype=float, copy=True)

    def sh_x(a):
        b = np.array(a, dtype=float, copy=True)
        b[:-1] = a[1:]
        return b

    def sh_u(a, N):
        b = np.array(a, dtype=float, copy=True)
        b[:N - 1] = a[1:N]
        return b

    out = []
    for k, t in enumerate(trajs):
        inst = dict(t.inst if next_insts is None else next_insts[k])
        if not (measured and next_insts is not None):
            inst["x_init"] = x_init.copy()
        N = inst["N"]
        nt = Traj(inst, sh_x(t.xbar), sh_u(t.ubar, N))
        st = t.state
        if st is not None:
            ns = AdmmState(np.array(st.x, copy=True), np.array(st.u, copy=True), np.array(st.z, copy=True),
                           sh_x(st.lam), sh_x(st.mu), np.array(st.ddyn, copy=True),
                           [np.array(c, copy=True) for c in st.copy], [])
            ns.lam[0] = 0.0
            ns.mu[0] = 0.0
            for g, d in zip(t.groups, st.dual):
                nd = sh_x(d) if g.var == "x" else sh_u(d, N)
                nd[~g.active] = 0.0
                ns.dual.append(nd)
            nt.state = ns
            nt.groups = t.groups
        out.append(nt)
    return out


def mpc_session(requests: list[list[dict]], params: dict) -> list[tuple[list[Traj], dict]]:
    """Solve the requests of one MPC session in order: the first from its initial guess, each
    later one warm-started from the previous solution (shift_warm_start).  Returns, per request,
    the solved trajectories and the group info."""
    out = []
    prev = None
    for req in requests:
        trajs = [init_traj(d) for d in req] if prev is None else shift_warm_start(prev, req)
        info = scp_group(trajs, params)
        out.append((trajs, info))
        prev = trajs
    return out

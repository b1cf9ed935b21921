"""Consensus ADMM on the temporally split QP (Sec. III-B), FP64, vectorized over nodes.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Variables of one trajectory with N intervals:
  physical   x_0..x_N (nx), u_0..u_{N-1} (nu)                      (Sec. III-B.1)
  dynamic    z_1..z_N with x_i = z_i                                 (Sec. III-B.1)
  geometric  one mirror copy per constraint group, with its own dual (reading of Sec. III-B.1:
             all box-type constraints on a variable form one group; every half-space, ball,
             second-order cone or scaled cone is a group of its own, so each projection stays
             exact; the Hessian then carries rho_geo * D with D = number of groups per component,
             which equals the paper's rho_geo * I when only the box group exists)
  duals      lambda_1..lambda_N, mu_1..mu_N, nu per group copy

Augmented Lagrangian: eq. (augmented_lagrangian).  Step 1 solves H_i xi_i = g_i per node with
H_i from the block formulas below that equation; g_i is the stationarity right-hand side of the
Lagrangian in (x_i, u_i).  Step 2 is the closed-form weighted average of that section, Step 3
the projections (Step 3 equations), Step 4 dual ascent with each constraint's own penalty.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .sets import proj_box, proj_halfspace, proj_ball, proj_cone


@dataclass
class Group:
    """One geometric constraint group acting on components ``comps`` of ``var`` ('x' or 'u')."""
    var: str
    comps: tuple
    kind: str                    # 'box' | 'halfspace' | 'ball' | 'soc' | 'cone'
    active: np.ndarray           # (N+1,) bool: nodes where the group exists
    lo: np.ndarray | None = None  # (N+1, m) box bounds
    hi: np.ndarray | None = None
    a: np.ndarray | None = None   # (N+1, m) half-space a'y >= b
    b: np.ndarray | None = None   # (N+1,)
    radius: float = 0.0           # ball radius
    kappa: float = 1.0            # cone slope (soc: 1)

    def project(self, v: np.ndarray, rows: np.ndarray) -> np.ndarray:
        if self.kind == "box":
            return proj_box(v, self.lo[rows], self.hi[rows])
        if self.kind == "halfspace":
            return proj_halfspace(v, self.a[rows], self.b[rows])
        if self.kind == "ball":
            return proj_ball(v, self.radius)
        if self.kind == "soc":
            return proj_cone(v, 1.0)
        if self.kind == "cone":
            return proj_cone(v, self.kappa)
        raise ValueError(self.kind)


@dataclass
class QP:
    """Per-node data of eq. (qp_subproblem): cost (Q,q,R,r,M) and affine dynamics (A,B,d)."""
    Q: np.ndarray   # (N+1, nx, nx)
    q: np.ndarray   # (N+1, nx)
    R: np.ndarray   # (N, nu, nu)
    r: np.ndarray   # (N, nu)
    M: np.ndarray   # (N, nx, nu)
    A: np.ndarray   # (N, nx, nx)
    B: np.ndarray   # (N, nx, nu)
    d: np.ndarray   # (N, nx)

    @property
    def N(self):
        return self.A.shape[0]

    @property
    def nx(self):
        return self.A.shape[1]

    @property
    def nu(self):
        return self.B.shape[2]


@dataclass
class AdmmState:
    x: np.ndarray      # (N+1, nx)
    u: np.ndarray      # (N, nu)
    z: np.ndarray      # (N+1, nx); row 0 unused
    lam: np.ndarray    # (N+1, nx); row 0 unused
    mu: np.ndarray     # (N+1, nx); row 0 unused
    ddyn: np.ndarray   # (N, nx): d_dyn,i = A_i x_i + B_i u_i + d_i
    copy: list = field(default_factory=list)   # per group (N+1, m)
    dual: list = field(default_factory=list)   # per group (N+1, m)

    @staticmethod
    def zeros(N, nx, nu, groups):
        return AdmmState(np.zeros((N + 1, nx)), np.zeros((N, nu)), np.zeros((N + 1, nx)),
                         np.zeros((N + 1, nx)), np.zeros((N + 1, nx)), np.zeros((N, nx)),
                         [np.zeros((N + 1, len(g.comps))) for g in groups],
                         [np.zeros((N + 1, len(g.comps))) for g in groups])


def _var(state: AdmmState, g: Group, N: int) -> np.ndarray:
    """(N+1, m) view of the group's variable components (u padded with a zero row N)."""
    if g.var == "x":
        return state.x[:, list(g.comps)]
    out = np.zeros((N + 1, len(g.comps)))
    out[:N] = state.u[:, list(g.comps)]
    return out


def group_counts(groups, N, nx, nu):
    """D_x (N+1, nx) and D_u (N+1, nu): number of groups covering each component."""
    Dx = np.zeros((N + 1, nx))
    Du = np.zeros((N + 1, nu))
    for g in groups:
        D = Dx if g.var == "x" else Du
        for c in g.comps:
            D[g.active, c] += 1.0
    return Dx, Du


def build_H(qp: QP, groups, rho):
    """Step-1 Hessians (block formulas of Sec. III-B.3, with rho_geo I -> rho_geo D).

    H11 = Q_i + rho_eq 1{i>0} I + rho_geo D_x,i + rho_dyn A_i'A_i
    H12 = M_i + rho_dyn A_i'B_i,  H22 = R_i + rho_geo D_u,i + rho_dyn B_i'B_i   (i < N)
    Node N has no control and no outgoing dynamics: H_N = Q_N + rho_eq I + rho_geo D_x,N.
    Returns (H of shape (N, n, n), H_N of shape (nx, nx)).
    """
    rho_eq, rho_dyn, rho_geo = rho
    N, nx, nu = qp.N, qp.nx, qp.nu
    Dx, Du = group_counts(groups, N, nx, nu)
    n = nx + nu
    H = np.zeros((N, n, n))
    AtA = np.einsum("kij,kil->kjl", qp.A, qp.A)
    AtB = np.einsum("kij,kil->kjl", qp.A, qp.B)
    BtB = np.einsum("kij,kil->kjl", qp.B, qp.B)
    eq = np.array([0.0] + [1.0] * N)  # 1{i>0}
    for i in range(N):
        H[i, :nx, :nx] = qp.Q[i] + rho_eq * eq[i] * np.eye(nx) + rho_geo * np.diag(Dx[i]) + rho_dyn * AtA[i]
        H[i, :nx, nx:] = qp.M[i] + rho_dyn * AtB[i]
        H[i, nx:, :nx] = H[i, :nx, nx:].T
        H[i, nx:, nx:] = qp.R[i] + rho_geo * np.diag(Du[i]) + rho_dyn * BtB[i]
    HN = qp.Q[N] + rho_eq * np.eye(nx) + rho_geo * np.diag(Dx[N])
    return H, HN


def step1(qp: QP, groups, st: AdmmState, rho, H, HN):
    """Physical update: per node solve H_i xi_i = g_i, then d_dyn,i = A_i x_i + B_i u_i + d_i.

    g_i (stationarity of the Lagrangian in (x_i, u_i), all other blocks fixed):
      x-part: -q_i + 1{i>0}(rho_eq z_i - lambda_i) + 1{i<N} A_i' w_i + sum_g (rho_geo xhat^g - nu_x^g)
      u-part: -r_i + B_i' w_i + sum_g (rho_geo uhat^g - nu_u^g)
      with w_i = mu_{i+1} + rho_dyn (z_{i+1} - d_i).
    """
    rho_eq, rho_dyn, rho_geo = rho
    N, nx, nu = qp.N, qp.nx, qp.nu
    w = st.mu[1:] + rho_dyn * (st.z[1:] - qp.d)
    gx = -qp.q.copy()
    gx[1:] += rho_eq * st.z[1:] - st.lam[1:]
    gx[:N] += np.einsum("kij,ki->kj", qp.A, w)
    gu = np.zeros((N + 1, nu))
    gu[:N] = -qp.r + np.einsum("kij,ki->kj", qp.B, w)
    for gi, g in enumerate(groups):
        tgt = gx if g.var == "x" else gu
        contrib = rho_geo * st.copy[gi] - st.dual[gi]
        for j, c in enumerate(g.comps):
            tgt[g.active, c] += contrib[g.active, j]
    rhs = np.concatenate([gx[:N], gu[:N]], axis=1)
    xi = np.linalg.solve(H, rhs[..., None])[..., 0]
    st.x[:N] = xi[:, :nx]
    st.u[:] = xi[:, nx:]
    st.x[N] = np.linalg.solve(HN, gx[N])
    st.ddyn[:] = np.einsum("kij,kj->ki", qp.A, st.x[:N]) + np.einsum("kij,kj->ki", qp.B, st.u) + qp.d


def step2(st: AdmmState, rho):
    """Dynamic layer: z_i = (rho_eq (x_i + lambda_i/rho_eq) + rho_dyn (d_dyn,i-1 - mu_i/rho_dyn))
    / (rho_eq + rho_dyn), i = 1..N (Step 2 equation)."""
    rho_eq, rho_dyn, _ = rho
    st.z[1:] = (rho_eq * st.x[1:] + st.lam[1:] + rho_dyn * st.ddyn - st.mu[1:]) / (rho_eq + rho_dyn)


def step3(groups, st: AdmmState, rho, N):
    """Geometric layer: each group's copy = projection of (var + nu/rho_geo) (Step 3)."""
    rho_geo = rho[2]
    for gi, g in enumerate(groups):
        rows = np.nonzero(g.active)[0]
        v = _var(st, g, N)[rows] + st.dual[gi][rows] / rho_geo
        st.copy[gi][rows] = g.project(v, rows)


def step4(groups, st: AdmmState, rho, N):
    """Dual ascent (Step 4): lambda_i += rho_eq (x_i - z_i), mu_i += rho_dyn (z_i - d_dyn,i-1),
    nu^g += rho_geo (var^g - copy^g)."""
    rho_eq, rho_dyn, rho_geo = rho
    st.lam[1:] += rho_eq * (st.x[1:] - st.z[1:])
    st.mu[1:] += rho_dyn * (st.z[1:] - st.ddyn)
    for gi, g in enumerate(groups):
        rows = g.active
        st.dual[gi][rows] += rho_geo * (_var(st, g, N)[rows] - st.copy[gi][rows])


def residuals(qp: QP, groups, st: AdmmState, z_old, copy_old, rho):
    """Primal and dual residuals (infinity norms; reading of the stopping rule of Sec. III-B.3).

    r_p = max over nodes of |x_i - z_i|, |z_i - d_dyn,i-1|, |var^g - copy^g|.
    r_d = max over nodes of |s_i|, s_i the change of the second ADMM block (z, copies) mapped
    through the constraints onto (x_i, u_i):
      x-part rho_eq dz_i + rho_dyn A_i' dz_{i+1} + rho_geo sum_g dxhat^g,
      u-part rho_dyn B_i' dz_{i+1} + rho_geo sum_g duhat^g.
    """
    rho_eq, rho_dyn, rho_geo = rho
    N, nx, nu = qp.N, qp.nx, qp.nu
    rp = 0.0
    if N > 0:
        rp = max(np.max(np.abs(st.x[1:] - st.z[1:])), np.max(np.abs(st.z[1:] - st.ddyn)))
    for gi, g in enumerate(groups):
        if np.any(g.active):
            rp = max(rp, np.max(np.abs(_var(st, g, N)[g.active] - st.copy[gi][g.active])))
    dz = st.z - z_old
    sx = np.zeros((N + 1, nx))
    su = np.zeros((N + 1, nu))
    sx[1:] += rho_eq * dz[1:]
    sx[:N] += rho_dyn * np.einsum("kij,ki->kj", qp.A, dz[1:])
    su[:N] += rho_dyn * np.einsum("kij,ki->kj", qp.B, dz[1:])
    for gi, g in enumerate(groups):
        s = sx if g.var == "x" else su
        dc = rho_geo * (st.copy[gi] - copy_old[gi])
        for j, c in enumerate(g.comps):
            s[g.active, c] += dc[g.active, j]
    rd = max(np.max(np.abs(sx)), np.max(np.abs(su[:N])) if N > 0 else 0.0)
    return float(rp), float(rd)


def admm_run(trajs, rho, iters: int, check_every: int = 0, eps_p: float = 0.0, eps_d: float = 0.0,
             couple_u0: bool = False, u_groups_couple=None):
    """Run up to ``iters`` ADMM iterations on a list of trajectories.

    ``trajs`` is a list of (qp, groups, state, (H, H_N)).  The trajectories are
    independent unless ``couple_u0``: then, after Step 3, the node-0 copy of every
    u-group is replaced by its average over the trajectories, summed in list order
    (scenario consensus on the first control, Sec. IV-A.4).

    Residuals are evaluated every ``check_every`` iterations (0: only after the last
    iteration); the loop stops once r_p <= eps_p and r_d <= eps_d at a check (the
    maximum over all trajectories of the list).  Returns (iterations run, r_p, r_d).
    """
    rp = rd = float("nan")
    for j in range(1, iters + 1):
        check = (check_every > 0 and j % check_every == 0) or j == iters
        if check:
            olds = [(st.z.copy(), [c.copy() for c in st.copy]) for (_, _, st, _) in trajs]
        for qp, groups, st, (H, HN) in trajs:
            step1(qp, groups, st, rho, H, HN)
            step2(st, rho)
            step3(groups, st, rho, qp.N)
        if couple_u0 and len(trajs) > 1:
            groups0 = trajs[0][1]
            for gi, g in enumerate(groups0):
                if g.var != "u":
                    continue
                acc = np.zeros(len(g.comps))
                for (_, _, st, _) in trajs:
                    acc = acc + st.copy[gi][0]
                mean = acc / len(trajs)
                for (_, _, st, _) in trajs:
                    st.copy[gi][0] = mean
        for qp, groups, st, _ in trajs:
            step4(groups, st, rho, qp.N)
        if check:
            rp = rd = 0.0
            for (qp, groups, st, _), (zo, co) in zip(trajs, olds):
                a, b = residuals(qp, groups, st, zo, co, rho)
                rp, rd = max(rp, a), max(rd, b)
            if check_every > 0 and rp <= eps_p and rd <= eps_d:
                return j, rp, rd
    return iters, rp, rd

"""Independent pin of the oracle's ADMM residuals (stopping rule of Sec. III-B, Step 4).

The paper stops the ADMM loop when the primal and dual residuals meet a tolerance but does not
write them out.  The oracle's reading is the standard two-block ADMM residual pair (Boyd et al.,
"Distributed Optimization and Statistical Learning via ADMM", 2011, Sec. 3.3): the splitting of
Sec. III-B is written as

    minimize f(xi) + g(zeta)   subject to   A_c xi + B_c zeta = c,

with xi = (x_0..x_N, u_0..u_{N-1}) the physical block, zeta = (z_1..z_N, every mirror copy) the
second block, f the quadratic cost of eq. (qp_subproblem) and g the indicators of the sets.  Each
constraint row carries its own penalty (rho_eq for x_i = z_i, rho_dyn for z_{i+1} = d_dyn,i, rho_geo
for var = copy), collected in the diagonal matrix P.  Then

    r_p = ||A_c xi + B_c zeta - c||_inf,     r_d = ||A_c' P B_c (zeta - zeta_old)||_inf,

and the dual residual is exactly the stationarity defect of the first block after the dual
update: grad f(xi) + A_c' y = A_c' P B_c (zeta - zeta_old).

This file assembles A_c, B_c, c and P as dense matrices from the constraint definitions alone
(none of the oracle's residual or step formulas is reused), runs a few ADMM iterations with unequal
penalties away from convergence, and checks:
  * the oracle's (r_p, r_d) against the dense norms;
  * the stationarity identity, vector by vector, from the cost gradient and the duals;
  * that the dense check fails for the plausible mistakes in r_d (the rho_dyn A' / B' term with
    the wrong sign or dropped, the mirror term dropped), planted in the oracle's inputs on the CPU.
"""
import numpy as np
import pytest

from oracle.admm import AdmmState, Group, QP, build_H, residuals, step1, step2, step3, step4

RHOS = [(0.7, 1.9, 0.45), (2.5, 0.3, 1.1)]


def _qp(rng, N, nx, nu):
    A = np.eye(nx) + 0.3 * rng.normal(size=(N, nx, nx))
    B = 0.6 * rng.normal(size=(N, nx, nu))
    d = 0.2 * rng.normal(size=(N, nx))
    Q = np.zeros((N + 1, nx, nx))
    for i in range(N + 1):
        L = rng.normal(size=(nx, nx))
        Q[i] = 0.4 * L @ L.T + 0.2 * np.eye(nx)
    R = np.zeros((N, nu, nu))
    for i in range(N):
        L = rng.normal(size=(nu, nu))
        R[i] = L @ L.T + 0.5 * np.eye(nu)
    M = 0.15 * rng.normal(size=(N, nx, nu))
    return QP(Q=Q, q=rng.normal(size=(N + 1, nx)), R=R, r=rng.normal(size=(N, nu)), M=M, A=A, B=B, d=d)


def _groups(rng, N, nx, nu):
    """x box (node 0 degenerate), u box, u ball, one x half-space at the inner nodes: the kinds of
    the point-mass quadrotor's groups."""
    allx = np.ones(N + 1, dtype=bool)
    xlo = np.full((N + 1, nx), -1.5)
    xhi = np.full((N + 1, nx), 1.5)
    x0 = 0.3 * rng.normal(size=nx)
    xlo[0] = xhi[0] = x0
    uact = allx.copy()
    uact[N] = False
    inner = allx.copy()
    inner[0] = False
    a = rng.normal(size=(N + 1, 2))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b = 0.4 * rng.normal(size=N + 1)
    return [Group("x", tuple(range(nx)), "box", allx, lo=xlo, hi=xhi),
            Group("u", tuple(range(nu)), "box", uact, lo=np.full((N + 1, nu), -0.4), hi=np.full((N + 1, nu), 0.4)),
            Group("u", tuple(range(nu)), "ball", uact.copy(), radius=0.5),
            Group("x", (0, 1), "halfspace", inner, a=a, b=b)]


class Layout:
    """Index maps of the dense Boyd form: columns of xi, columns of zeta, constraint rows."""

    def __init__(self, N, nx, nu, groups):
        self.N, self.nx, self.nu = N, nx, nu
        self.nxi = (N + 1) * nx + N * nu
        # zeta: z_1..z_N, then every group's copy at its active nodes (node order, component order)
        self.zcol = {}
        k = 0
        for i in range(1, N + 1):
            self.zcol[("z", i)] = k
            k += nx
        self.ccol = {}
        for gi, g in enumerate(groups):
            for i in np.nonzero(g.active)[0]:
                self.ccol[(gi, int(i))] = k
                k += len(g.comps)
        self.nzeta = k

    def xcol(self, i):
        return i * self.nx

    def ucol(self, i):
        return (self.N + 1) * self.nx + i * self.nu


def dense_form(qp, groups, rho):
    """A_c, B_c, c and the row penalties P of the splitting, built from the constraints:
        x_i - z_i = 0                                  (i = 1..N, penalty rho_eq, dual lambda_i)
        z_{i+1} - (A_i x_i + B_i u_i + d_i) = 0        (i = 0..N-1, penalty rho_dyn, dual mu_{i+1})
        var^g_i - copy^g_i = 0                         (active nodes, penalty rho_geo, dual nu^g_i)
    """
    rho_eq, rho_dyn, rho_geo = rho
    N, nx, nu = qp.N, qp.nx, qp.nu
    lay = Layout(N, nx, nu, groups)
    rows_A, rows_B, rows_c, pen = [], [], [], []

    def new_rows(m):
        Ar = np.zeros((m, lay.nxi))
        Br = np.zeros((m, lay.nzeta))
        rows_A.append(Ar)
        rows_B.append(Br)
        rows_c.append(np.zeros(m))
        return Ar, Br, rows_c[-1]

    I = np.eye(nx)
    for i in range(1, N + 1):
        Ar, Br, _ = new_rows(nx)
        Ar[:, lay.xcol(i):lay.xcol(i) + nx] = I
        Br[:, lay.zcol[("z", i)]:lay.zcol[("z", i)] + nx] = -I
        pen.append(np.full(nx, rho_eq))
    for i in range(N):
        Ar, Br, c = new_rows(nx)
        Ar[:, lay.xcol(i):lay.xcol(i) + nx] = -qp.A[i]
        Ar[:, lay.ucol(i):lay.ucol(i) + nu] = -qp.B[i]
        Br[:, lay.zcol[("z", i + 1)]:lay.zcol[("z", i + 1)] + nx] = I
        c[:] = qp.d[i]
        pen.append(np.full(nx, rho_dyn))
    for gi, g in enumerate(groups):
        m = len(g.comps)
        for i in np.nonzero(g.active)[0]:
            i = int(i)
            Ar, Br, _ = new_rows(m)
            base = lay.xcol(i) if g.var == "x" else lay.ucol(i)
            for j, comp in enumerate(g.comps):
                Ar[j, base + comp] = 1.0
            Br[:, lay.ccol[(gi, i)]:lay.ccol[(gi, i)] + m] = -np.eye(m)
            pen.append(np.full(m, rho_geo))
    return lay, np.vstack(rows_A), np.vstack(rows_B), np.concatenate(rows_c), np.concatenate(pen)


def pack_xi(lay, st):
    v = np.zeros(lay.nxi)
    for i in range(lay.N + 1):
        v[lay.xcol(i):lay.xcol(i) + lay.nx] = st.x[i]
    for i in range(lay.N):
        v[lay.ucol(i):lay.ucol(i) + lay.nu] = st.u[i]
    return v


def pack_zeta(lay, z, copies):
    v = np.zeros(lay.nzeta)
    for i in range(1, lay.N + 1):
        v[lay.zcol[("z", i)]:lay.zcol[("z", i)] + lay.nx] = z[i]
    for (gi, i), k in lay.ccol.items():
        v[k:k + copies[gi].shape[1]] = copies[gi][i]
    return v


def pack_duals(lay, st, groups):
    """y in the row order of dense_form: lambda_1..N, mu_1..N, then each group's nu at its active
    nodes."""
    parts = [st.lam[i] for i in range(1, lay.N + 1)]
    parts += [st.mu[i + 1] for i in range(lay.N)]
    for gi, g in enumerate(groups):
        parts += [st.dual[gi][int(i)] for i in np.nonzero(g.active)[0]]
    return np.concatenate(parts)


def cost_gradient(lay, qp, st):
    """grad f(xi) of the quadratic cost of eq. (qp_subproblem): sum_i 1/2 x'Qx + q'x (i = 0..N) and
    1/2 u'Ru + x'Mu + r'u (i < N)."""
    g = np.zeros(lay.nxi)
    N, nx, nu = lay.N, lay.nx, lay.nu
    for i in range(N + 1):
        gx = qp.Q[i] @ st.x[i] + qp.q[i]
        if i < N:
            gx = gx + qp.M[i] @ st.u[i]
        g[lay.xcol(i):lay.xcol(i) + nx] = gx
    for i in range(N):
        g[lay.ucol(i):lay.ucol(i) + nu] = qp.R[i] @ st.u[i] + qp.M[i].T @ st.x[i] + qp.r[i]
    return g


def _random_start(rng, qp, groups):
    N, nx, nu = qp.N, qp.nx, qp.nu
    st = AdmmState.zeros(N, nx, nu, groups)
    for arr in (st.z, st.lam, st.mu):
        arr[1:] = 0.5 * rng.normal(size=arr[1:].shape)
    for gi, g in enumerate(groups):
        st.copy[gi][g.active] = 0.5 * rng.normal(size=(int(g.active.sum()), len(g.comps)))
        st.dual[gi][g.active] = 0.5 * rng.normal(size=(int(g.active.sum()), len(g.comps)))
    return st


def _iterate(qp, groups, st, rho, n):
    """n ADMM iterations; returns (z, copies) before the last one."""
    H, HN = build_H(qp, groups, rho)
    z_old = c_old = None
    for _ in range(n):
        z_old = st.z.copy()
        c_old = [c.copy() for c in st.copy]
        step1(qp, groups, st, rho, H, HN)
        step2(st, rho)
        step3(groups, st, rho, qp.N)
        step4(groups, st, rho, qp.N)
    return z_old, c_old


def _case(seed, rho, N=4, nx=3, nu=2, iters=3):
    rng = np.random.default_rng(seed)
    qp = _qp(rng, N, nx, nu)
    groups = _groups(rng, N, nx, nu)
    st = _random_start(rng, qp, groups)
    z_old, c_old = _iterate(qp, groups, st, rho, iters)
    return qp, groups, st, z_old, c_old


def _dense_residuals(qp, groups, st, z_old, c_old, rho):
    lay, Ac, Bc, c, P = dense_form(qp, groups, rho)
    xi = pack_xi(lay, st)
    zeta = pack_zeta(lay, st.z, st.copy)
    zeta_old = pack_zeta(lay, z_old, c_old)
    r = Ac @ xi + Bc @ zeta - c
    s = Ac.T @ (P * (Bc @ (zeta - zeta_old)))
    return lay, Ac, r, s


@pytest.mark.parametrize("rho", RHOS)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_residuals_equal_dense_boyd_form(seed, rho):
    qp, groups, st, z_old, c_old = _case(seed, rho)
    _, _, r, s = _dense_residuals(qp, groups, st, z_old, c_old, rho)
    rp, rd = residuals(qp, groups, st, z_old, c_old, rho)
    # away from convergence: both residuals are far from zero, so every term matters
    assert rp > 1e-3 and rd > 1e-3
    assert rp == pytest.approx(np.max(np.abs(r)), rel=1e-12, abs=1e-14)
    assert rd == pytest.approx(np.max(np.abs(s)), rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("rho", RHOS)
@pytest.mark.parametrize("seed", [3, 4])
def test_dual_residual_is_stationarity_defect(seed, rho):
    """grad f(xi^{k+1}) + A_c' y^{k+1} = A_c' P B_c (zeta^{k+1} - zeta^k), entry by entry: the
    first block's optimality condition with the new duals fails by exactly the dual residual.
    This fixes the sign convention of every dual update as well."""
    qp, groups, st, z_old, c_old = _case(seed, rho, N=5, nx=4, nu=3, iters=4)
    lay, Ac, _, s = _dense_residuals(qp, groups, st, z_old, c_old, rho)
    y = pack_duals(lay, st, groups)
    lhs = cost_gradient(lay, qp, st) + Ac.T @ y
    np.testing.assert_allclose(lhs, s, rtol=0, atol=1e-10 * max(1.0, np.max(np.abs(s))))
    # the primal residual is the dual increment of the last iteration divided by its penalty
    assert np.max(np.abs(s)) > 1e-3


def _mutant(qp, **over):
    kw = dict(Q=qp.Q, q=qp.q, R=qp.R, r=qp.r, M=qp.M, A=qp.A, B=qp.B, d=qp.d)
    kw.update(over)
    return QP(**kw)


@pytest.mark.parametrize("rho", RHOS)
def test_dense_check_rejects_plausible_dual_residual_mistakes(rho):
    """Mistakes planted in the oracle's residual (by feeding it altered inputs, on the CPU) fail
    the dense comparison: the rho_dyn A'dz / B'dz term with the wrong sign, that term dropped, and
    the mirror-copy term dropped."""
    qp, groups, st, z_old, c_old = _case(5, rho)
    _, _, _, s = _dense_residuals(qp, groups, st, z_old, c_old, rho)
    want = np.max(np.abs(s))
    mutants = {
        "dyn term sign": residuals(_mutant(qp, A=-qp.A, B=-qp.B), groups, st, z_old, c_old, rho)[1],
        "dyn term dropped": residuals(_mutant(qp, A=0 * qp.A, B=0 * qp.B), groups, st, z_old, c_old, rho)[1],
        "mirror term dropped": residuals(qp, groups, st, z_old, [c.copy() for c in st.copy], rho)[1],
    }
    for name, rd_bad in mutants.items():
        assert abs(rd_bad - want) > 1e-6 * want, f"dense check blind to: {name}"
    assert residuals(qp, groups, st, z_old, c_old, rho)[1] == pytest.approx(want, rel=1e-12)

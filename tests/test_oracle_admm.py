"""Pins for the oracle's consensus ADMM (Sec. III-B).

* every block update is a minimizer of the augmented Lagrangian, checked with
  central differences of an independent transcription of eq. (augmented_lagrangian);
* the dual update is gradient ascent on that Lagrangian;
* the ADMM fixed point equals the QP optimum found by brute-force active-set
  enumeration on a tiny problem, and the Riccati LQR solution when unconstrained;
* residuals vanish on a feasible problem;
* scenario consensus: identical scenarios reproduce the single problem, node-0
  control copies agree across scenarios after every iteration.
"""
import itertools

import numpy as np
import pytest

from oracle.admm import Group, QP, AdmmState, build_H, step1, step2, step3, step4, admm_run, residuals

RHO = (0.7, 1.3, 0.9)


def _random_qp(rng, N=4, nx=3, nu=2, cross=True):
    A = np.eye(nx) + 0.2 * rng.normal(size=(N, nx, nx))
    B = 0.5 * rng.normal(size=(N, nx, nu))
    d = 0.1 * rng.normal(size=(N, nx))
    Q = np.zeros((N + 1, nx, nx))
    for i in range(N + 1):
        L = rng.normal(size=(nx, nx))
        Q[i] = 0.3 * L @ L.T + 0.1 * np.eye(nx)
    R = np.zeros((N, nu, nu))
    for i in range(N):
        L = rng.normal(size=(nu, nu))
        R[i] = L @ L.T + 0.5 * np.eye(nu)
    M = 0.1 * rng.normal(size=(N, nx, nu)) if cross else np.zeros((N, nx, nu))
    return QP(Q=Q, q=rng.normal(size=(N + 1, nx)), R=R, r=rng.normal(size=(N, nu)), M=M, A=A, B=B, d=d)


def _groups(rng, N, nx, nu, x_init):
    allx = np.ones(N + 1, dtype=bool)
    xlo = np.full((N + 1, nx), -np.inf)
    xhi = np.full((N + 1, nx), np.inf)
    xlo[0] = xhi[0] = x_init
    xlo[1:] = -2.0
    xhi[1:] = 2.0
    uact = allx.copy()
    uact[N] = False
    ulo = np.full((N + 1, nu), -0.5)
    uhi = np.full((N + 1, nu), 0.5)
    inner = allx.copy()
    inner[0] = False
    a = rng.normal(size=(N + 1, 2))
    b = rng.normal(size=N + 1) * 0.3
    return [Group("x", tuple(range(nx)), "box", allx, lo=xlo, hi=xhi),
            Group("u", tuple(range(nu)), "box", uact, lo=ulo, hi=uhi),
            Group("u", tuple(range(nu)), "ball", uact.copy(), radius=0.6),
            Group("x", (0, 1), "halfspace", inner, a=a, b=b)]


def _random_state(rng, qp, groups):
    N, nx, nu = qp.N, qp.nx, qp.nu
    st = AdmmState.zeros(N, nx, nu, groups)
    for arr in (st.x, st.u, st.z, st.lam, st.mu):
        arr[:] = rng.normal(size=arr.shape)
    for gi, g in enumerate(groups):
        st.copy[gi][g.active] = rng.normal(size=(int(g.active.sum()), len(g.comps)))
        st.dual[gi][g.active] = rng.normal(size=(int(g.active.sum()), len(g.comps)))
    st.ddyn[:] = np.einsum("kij,kj->ki", qp.A, st.x[:N]) + np.einsum("kij,kj->ki", qp.B, st.u) + qp.d
    return st


def lagrangian(qp, groups, x, u, z, lam, mu, copy, dual, rho):
    """Eq. (augmented_lagrangian) written out term by term (indicators omitted: they are constant
    for the blocks differentiated here)."""
    rho_eq, rho_dyn, rho_geo = rho
    N = qp.N
    L = 0.0
    for i in range(N + 1):
        L += 0.5 * x[i] @ qp.Q[i] @ x[i] + qp.q[i] @ x[i]
    for i in range(N):
        L += 0.5 * u[i] @ qp.R[i] @ u[i] + x[i] @ qp.M[i] @ u[i] + qp.r[i] @ u[i]
    for i in range(1, N + 1):
        L += lam[i] @ (x[i] - z[i]) + 0.5 * rho_eq * np.sum((x[i] - z[i]) ** 2)
    for i in range(N):
        ddyn = qp.A[i] @ x[i] + qp.B[i] @ u[i] + qp.d[i]
        L += mu[i + 1] @ (z[i + 1] - ddyn) + 0.5 * rho_dyn * np.sum((z[i + 1] - ddyn) ** 2)
    for gi, g in enumerate(groups):
        for i in np.nonzero(g.active)[0]:
            var = (x[i] if g.var == "x" else u[i])[list(g.comps)]
            diff = var - copy[gi][i]
            L += dual[gi][i] @ diff + 0.5 * rho_geo * diff @ diff
    return L


def _L(qp, groups, st, rho, **over):
    args = dict(x=st.x, u=st.u, z=st.z, lam=st.lam, mu=st.mu, copy=st.copy, dual=st.dual)
    args.update(over)
    return lagrangian(qp, groups, rho=rho, **args)


def _fd_grad(fun, arr, idx, h=1e-4):
    g = np.zeros(arr[idx].shape)
    for j in range(g.size):
        a1 = arr.copy()
        a2 = arr.copy()
        a1[idx][j] += h
        a2[idx][j] -= h
        g[j] = (fun(a1) - fun(a2)) / (2 * h)
    return g


def test_H_is_spd_and_step1_is_stationary():
    rng = np.random.default_rng(0)
    qp = _random_qp(rng)
    x_init = rng.normal(size=qp.nx)
    groups = _groups(rng, qp.N, qp.nx, qp.nu, x_init)
    st = _random_state(rng, qp, groups)
    H, HN = build_H(qp, groups, RHO)
    for Hi in list(H) + [HN]:
        np.testing.assert_allclose(Hi, Hi.T, atol=1e-14)
        np.linalg.cholesky(Hi)
    step1(qp, groups, st, RHO, H, HN)
    for i in range(qp.N + 1):
        gx = _fd_grad(lambda xx: _L(qp, groups, st, RHO, x=xx), st.x, i)
        assert np.max(np.abs(gx)) < 1e-7, (i, gx)
        if i < qp.N:
            gu = _fd_grad(lambda uu: _L(qp, groups, st, RHO, u=uu), st.u, i)
            assert np.max(np.abs(gu)) < 1e-7, (i, gu)
    ddyn = np.einsum("kij,kj->ki", qp.A, st.x[:qp.N]) + np.einsum("kij,kj->ki", qp.B, st.u) + qp.d
    np.testing.assert_allclose(st.ddyn, ddyn, atol=1e-13)


def test_step2_is_stationary_in_z():
    rng = np.random.default_rng(1)
    qp = _random_qp(rng)
    groups = _groups(rng, qp.N, qp.nx, qp.nu, rng.normal(size=qp.nx))
    st = _random_state(rng, qp, groups)
    step2(st, RHO)
    for i in range(1, qp.N + 1):
        gz = _fd_grad(lambda zz: _L(qp, groups, st, RHO, z=zz), st.z, i)
        assert np.max(np.abs(gz)) < 1e-8, (i, gz)


def test_step2_equal_penalties_special_case():
    """rho_eq = rho_dyn = rho: z_i = (x_i + d_dyn,i-1)/2 + (lambda_i - mu_i)/(2 rho)."""
    rng = np.random.default_rng(2)
    qp = _random_qp(rng)
    groups = _groups(rng, qp.N, qp.nx, qp.nu, rng.normal(size=qp.nx))
    st = _random_state(rng, qp, groups)
    rho = (2.0, 2.0, 1.0)
    step2(st, rho)
    ref = 0.5 * (st.x[1:] + st.ddyn) + (st.lam[1:] - st.mu[1:]) / 4.0
    np.testing.assert_allclose(st.z[1:], ref, atol=1e-14)


def test_step3_minimizes_lagrangian_over_each_set():
    rng = np.random.default_rng(3)
    qp = _random_qp(rng)
    groups = _groups(rng, qp.N, qp.nx, qp.nu, rng.normal(size=qp.nx))
    st = _random_state(rng, qp, groups)
    step3(groups, st, RHO, qp.N)
    base = _L(qp, groups, st, RHO)
    members = {
        "box": lambda g, i, y: np.all(y >= g.lo[i] - 1e-12) and np.all(y <= g.hi[i] + 1e-12),
        "ball": lambda g, i, y: np.linalg.norm(y) <= g.radius + 1e-12,
        "halfspace": lambda g, i, y: g.a[i] @ y >= g.b[i] - 1e-12,
    }
    for gi, g in enumerate(groups):
        for i in np.nonzero(g.active)[0]:
            assert members[g.kind](g, i, st.copy[gi][i])
            for _ in range(30):
                y = st.copy[gi][i] + 0.3 * rng.normal(size=len(g.comps))
                if not members[g.kind](g, i, y):
                    continue
                c2 = [c.copy() for c in st.copy]
                c2[gi][i] = y
                assert _L(qp, groups, st, RHO, copy=c2) >= base - 1e-10


def test_step4_is_dual_ascent_on_lagrangian():
    rng = np.random.default_rng(4)
    qp = _random_qp(rng)
    groups = _groups(rng, qp.N, qp.nx, qp.nu, rng.normal(size=qp.nx))
    st = _random_state(rng, qp, groups)
    lam0, mu0 = st.lam.copy(), st.mu.copy()
    dual0 = [d.copy() for d in st.dual]
    g_lam = [_fd_grad(lambda ll: _L(qp, groups, st, RHO, lam=ll), st.lam, i) for i in range(1, qp.N + 1)]
    g_mu = [_fd_grad(lambda mm: _L(qp, groups, st, RHO, mu=mm), st.mu, i) for i in range(1, qp.N + 1)]
    step4(groups, st, RHO, qp.N)
    for i in range(1, qp.N + 1):
        np.testing.assert_allclose(st.lam[i] - lam0[i], RHO[0] * g_lam[i - 1], atol=1e-8)
        np.testing.assert_allclose(st.mu[i] - mu0[i], RHO[1] * g_mu[i - 1], atol=1e-8)
    for gi, g in enumerate(groups):
        for i in np.nonzero(g.active)[0]:
            def f(dd, gi=gi):
                return _L(qp, groups, st, RHO, dual=dd)
            h = 1e-4
            for j in range(len(g.comps)):
                d1 = [d.copy() for d in dual0]
                d2 = [d.copy() for d in dual0]
                d1[gi][i, j] += h
                d2[gi][i, j] -= h
                gj = (_L(qp, groups, st, RHO, dual=d1) - _L(qp, groups, st, RHO, dual=d2)) / (2 * h)
                assert abs(st.dual[gi][i, j] - dual0[gi][i, j] - RHO[2] * gj) < 1e-8


# ---------------------------------------------------------------------------------------------
# fixed-point pins
# ---------------------------------------------------------------------------------------------

def _solve_admm(qp, groups, x_init, iters, rho=(1.0, 1.0, 1.0)):
    st = AdmmState.zeros(qp.N, qp.nx, qp.nu, groups)
    st.x[0] = x_init
    H = build_H(qp, groups, rho)
    return admm_run([(qp, groups, st, H)], rho, iters), st


def _qp_bruteforce(qp, x_init, ulo, uhi, hs_a, hs_b):
    """Whole-QP optimum by enumerating active sets of the inequalities (tiny problems only).

    Variables w = [x_0..x_N, u_0..u_{N-1}]; equalities x_0 = x_init, x_{i+1} = A x_i + B u_i + d_i;
    inequalities ulo <= u_i <= uhi and a_i' x_i[0:2] >= b_i (i = 1..N)."""
    N, nx, nu = qp.N, qp.nx, qp.nu
    nv = (N + 1) * nx + N * nu
    xs = lambda i: slice(i * nx, (i + 1) * nx)
    us = lambda i: slice((N + 1) * nx + i * nu, (N + 1) * nx + (i + 1) * nu)
    Hm = np.zeros((nv, nv))
    c = np.zeros(nv)
    for i in range(N + 1):
        Hm[xs(i), xs(i)] += qp.Q[i]
        c[xs(i)] += qp.q[i]
    for i in range(N):
        Hm[us(i), us(i)] += qp.R[i]
        Hm[xs(i), us(i)] += qp.M[i]
        Hm[us(i), xs(i)] += qp.M[i].T
        c[us(i)] += qp.r[i]
    E, e = [], []
    for j in range(nx):
        row = np.zeros(nv)
        row[j] = 1.0
        E.append(row)
        e.append(x_init[j])
    for i in range(N):
        for j in range(nx):
            row = np.zeros(nv)
            row[xs(i + 1)][j] = 1.0
            row[xs(i)] -= qp.A[i][j]
            row[us(i)] -= qp.B[i][j]
            E.append(row)
            e.append(qp.d[i][j])
    G, h = [], []   # G w >= h
    for i in range(N):
        for j in range(nu):
            row = np.zeros(nv)
            row[us(i)][j] = 1.0
            G.append(row.copy())
            h.append(ulo)
            G.append(-row)
            h.append(-uhi)
    for i in range(1, N + 1):
        row = np.zeros(nv)
        row[xs(i)][:2] = hs_a[i]
        G.append(row)
        h.append(hs_b[i])
    E, e, G, h = np.array(E), np.array(e), np.array(G), np.array(h)
    best = None
    for k in range(len(G) + 1):
        for act in itertools.combinations(range(len(G)), k):
            C = np.vstack([E] + ([G[list(act)]] if act else []))
            cv = np.concatenate([e] + ([h[list(act)]] if act else []))
            K = np.block([[Hm, -C.T], [C, np.zeros((len(C), len(C)))]])
            try:
                sol = np.linalg.solve(K, np.concatenate([-c, cv]))
            except np.linalg.LinAlgError:
                continue
            w, mult = sol[:nv], sol[nv:]
            if np.max(np.abs(C @ w - cv)) > 1e-9:
                continue   # inconsistent active set (singular KKT matrix)
            if np.all(G @ w >= h - 1e-9) and np.all(mult[len(E):] >= -1e-9):
                best = w
                break
        if best is not None:
            break
    assert best is not None, "QP infeasible"
    X = best[:(N + 1) * nx].reshape(N + 1, nx)
    U = best[(N + 1) * nx:].reshape(N, nu)
    return X, U


def test_admm_fixed_point_equals_bruteforce_qp():
    rng = np.random.default_rng(7)
    N, nx, nu = 2, 2, 1
    qp = _random_qp(rng, N=N, nx=nx, nu=nu)
    qp.q[:] *= 3.0
    x_init = np.array([1.0, -0.5])
    ulo, uhi = -0.4, 0.4
    allx = np.ones(N + 1, dtype=bool)
    xlo = np.full((N + 1, nx), -np.inf)
    xhi = np.full((N + 1, nx), np.inf)
    xlo[0] = xhi[0] = x_init
    uact = allx.copy()
    uact[N] = False
    inner = allx.copy()
    inner[0] = False
    a = np.array([[0, 0], [1.0, 0.5], [-0.3, 1.0]])
    b = np.array([0.0, 0.75, -0.85])
    groups = [Group("x", (0, 1), "box", allx, lo=xlo, hi=xhi),
              Group("u", (0,), "box", uact, lo=np.full((N + 1, 1), ulo), hi=np.full((N + 1, 1), uhi)),
              Group("x", (0, 1), "halfspace", inner, a=a, b=b)]
    (it, rp, rd), st = _solve_admm(qp, groups, x_init, 20000)
    X, U = _qp_bruteforce(qp, x_init, ulo, uhi, a, b)
    assert rp < 1e-9 and rd < 1e-9
    np.testing.assert_allclose(st.x, X, atol=1e-7)
    np.testing.assert_allclose(st.u, U, atol=1e-7)
    # at least one inequality must be active for the test to exercise projections
    active_u = np.any(np.isclose(np.abs(U), uhi, atol=1e-6))
    active_h = np.any(np.isclose(np.einsum("ij,ij->i", a[1:], X[1:, :2]), b[1:], atol=1e-6))
    assert active_u or active_h


def _riccati(qp, x_init):
    """Textbook finite-horizon LQR with cross term M and affine dynamics (backward pass, then
    forward rollout)."""
    N = qp.N
    P, p = qp.Q[N].copy(), qp.q[N].copy()
    Ks, ks = [None] * N, [None] * N
    for i in range(N - 1, -1, -1):
        A, B, d = qp.A[i], qp.B[i], qp.d[i]
        G = qp.R[i] + B.T @ P @ B
        Hx = qp.M[i].T + B.T @ P @ A
        hv = qp.r[i] + B.T @ (P @ d + p)
        K = -np.linalg.solve(G, Hx)
        k = -np.linalg.solve(G, hv)
        P, p = (qp.Q[i] + A.T @ P @ A + Hx.T @ K, qp.q[i] + A.T @ (P @ d + p) + Hx.T @ k)
        Ks[i], ks[i] = K, k
    X = np.zeros((N + 1, qp.nx))
    U = np.zeros((N, qp.nu))
    X[0] = x_init
    for i in range(N):
        U[i] = Ks[i] @ X[i] + ks[i]
        X[i + 1] = qp.A[i] @ X[i] + qp.B[i] @ U[i] + qp.d[i]
    return X, U


def _free_groups(N, nx, nu, x_init):
    allx = np.ones(N + 1, dtype=bool)
    xlo = np.full((N + 1, nx), -np.inf)
    xhi = np.full((N + 1, nx), np.inf)
    xlo[0] = xhi[0] = x_init
    uact = allx.copy()
    uact[N] = False
    return [Group("x", tuple(range(nx)), "box", allx, lo=xlo, hi=xhi),
            Group("u", tuple(range(nu)), "box", uact, lo=np.full((N + 1, nu), -np.inf), hi=np.full((N + 1, nu), np.inf))]


def test_admm_unconstrained_equals_riccati_lqr():
    rng = np.random.default_rng(8)
    N, nx, nu = 6, 3, 2
    qp = _random_qp(rng, N=N, nx=nx, nu=nu)
    x_init = rng.normal(size=nx)
    groups = _free_groups(N, nx, nu, x_init)
    (it, rp, rd), st = _solve_admm(qp, groups, x_init, 6000)
    X, U = _riccati(qp, x_init)
    np.testing.assert_allclose(st.x, X, atol=1e-8)
    np.testing.assert_allclose(st.u, U, atol=1e-8)
    assert rp < 1e-10 and rd < 1e-10


def test_residuals_vanish_and_stopping_rule():
    rng = np.random.default_rng(9)
    N, nx, nu = 5, 3, 2
    qp = _random_qp(rng, N=N, nx=nx, nu=nu)
    x_init = rng.normal(size=nx)
    groups = _free_groups(N, nx, nu, x_init)
    rho = (1.0, 1.0, 1.0)
    st = AdmmState.zeros(N, nx, nu, groups)
    H = build_H(qp, groups, rho)
    it, rp, rd = admm_run([(qp, groups, st, H)], rho, 100000, check_every=10, eps_p=1e-9, eps_d=1e-9)
    assert it % 10 == 0 and it < 100000
    assert rp <= 1e-9 and rd <= 1e-9
    # residuals recomputed from scratch on the converged state after one more iteration agree
    z_old, c_old = st.z.copy(), [c.copy() for c in st.copy]
    admm_run([(qp, groups, st, H)], rho, 1)
    rp2, rd2 = residuals(qp, groups, st, z_old, c_old, rho)
    assert rp2 < 1e-8 and rd2 < 1e-8


def _scenario_qps(rng, S, N=4, nx=3, nu=2, identical=False):
    base = _random_qp(rng, N=N, nx=nx, nu=nu)
    out = []
    for s in range(S):
        if identical:
            qp = QP(**{k: v.copy() for k, v in base.__dict__.items()})
        else:
            qp = QP(**{k: v.copy() for k, v in base.__dict__.items()})
            qp.A = qp.A + 0.05 * rng.normal(size=qp.A.shape)
            qp.d = qp.d + 0.05 * rng.normal(size=qp.d.shape)
        out.append(qp)
    return out


def test_identical_scenarios_reproduce_single_problem():
    rng = np.random.default_rng(10)
    qps = _scenario_qps(rng, 3, identical=True)
    x_init = rng.normal(size=3)
    rho = (1.0, 1.0, 1.0)
    groups = _groups(np.random.default_rng(0), 4, 3, 2, x_init)
    single = AdmmState.zeros(4, 3, 2, groups)
    admm_run([(qps[0], groups, single, build_H(qps[0], groups, rho))], rho, 300)
    trajs = []
    for qp in qps:
        st = AdmmState.zeros(4, 3, 2, groups)
        trajs.append((qp, groups, st, build_H(qp, groups, rho)))
    admm_run(trajs, rho, 300, couple_u0=True)
    for (_, _, st, _) in trajs:
        np.testing.assert_allclose(st.x, single.x, atol=1e-12)
        np.testing.assert_allclose(st.u, single.u, atol=1e-12)


def test_scenario_consensus_on_first_control():
    rng = np.random.default_rng(11)
    qps = _scenario_qps(rng, 4)
    x_init = rng.normal(size=3)
    rho = (1.0, 1.0, 1.0)
    groups = _groups(np.random.default_rng(0), 4, 3, 2, x_init)
    trajs = []
    for qp in qps:
        st = AdmmState.zeros(4, 3, 2, groups)
        trajs.append((qp, groups, st, build_H(qp, groups, rho)))
    for _ in range(5):
        admm_run(trajs, rho, 1, couple_u0=True)
        for gi, g in enumerate(groups):
            if g.var == "u":
                for (_, _, st, _) in trajs[1:]:
                    np.testing.assert_array_equal(st.copy[gi][0], trajs[0][2].copy[gi][0])
    admm_run(trajs, rho, 4000, couple_u0=True)
    u0 = np.array([st.u[0] for (_, _, st, _) in trajs])
    assert np.max(np.abs(u0 - u0[0])) < 1e-6      # non-anticipativity reached
    u1 = np.array([st.u[1] for (_, _, st, _) in trajs])
    assert np.max(np.abs(u1 - u1[0])) > 1e-4      # later controls branch

"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Bar (fixed iteration counts, per block V in {x, u, z, lambda, mu, copies, duals, nominal}):
||V_gpu - V_oracle||_inf <= tol * max(1, ||V_oracle||_inf) with tol = 1e-9 in FP64 mode and
1e-4 in FP32 mode.  FP32 is held to 1e-4 where the iteration is well conditioned (first SCP
iteration, short budgets); at the full 15 x 200 budget the SCP map amplifies input perturbations
of 1e-7 to ~1e-3 (measured on the oracle itself), so the full budgets are checked in FP64 mode at
1e-9 and in FP32 mode through batch invariance (every trajectory alone == in the batch).
"""
import math

import numpy as np
import pytest

import scpgen
import oracle
from _parity import FIELDS, compare, gpu_fields, oracle_linearize_admm, oracle_scp, rel_err

pytestmark = pytest.mark.gpu

TOL64 = 1e-9
TOL32 = 1e-4


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def B(lib):
    from paper_2603_10711_amd import binding
    return binding


def _ragged_quads(n, seed_base=0, K=None):
    out = []
    for i in range(n):
        N = 5 + (7 * i) % 23
        out.append(scpgen.quad_instance(9, seed_base + i, N=N, K=(i % 9) if K is None else K, T=0.1 * N + 1.0))
    return out


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 2e-6)])
def test_linearize_and_convexify(B, prec, tol):
    insts = _ragged_quads(6) + [scpgen.mars_instance(2, i, N=9 + i) for i in range(3)]
    insts += [scpgen.quad6_benchmark_instance(i, N=7 + 3 * i) for i in range(3)]
    insts[-1]["x_guess"][:, 6:10] *= 1.3      # off the unit sphere: the normalized thrust direction
    _say("linearize", prec, len(insts))
    prob = B.Problem(insts, precision=prec)
    prob.linearize(B.admm_params(1.0))
    A, Bm, d = (prob.field(k).cpu().numpy() for k in ("A", "B", "d"))
    lo, hi, hs = (prob.field(k).cpu().numpy() for k in ("boxlo", "boxhi", "hs"))
    for t, inst in enumerate(insts):
        nx, nu, N = inst["nx"], inst["nu"], inst["N"]
        Ao, Bo, do = oracle.linearize(inst, inst["x_guess"], inst["u_guess"])
        o = prob.offsets[t]
        assert rel_err(A[o:o + N].reshape(N, B.MAX_NX, B.MAX_NX)[:, :nx, :nx], Ao) < tol
        assert rel_err(Bm[o:o + N].reshape(N, B.MAX_NX, B.MAX_NU)[:, :nx, :nu], Bo) < tol
        assert rel_err(d[o:o + N, :nx], do) < tol
        g = oracle.convexify(inst, inst["x_guess"], inst["u_guess"], inst["delta"])
        assert rel_err(lo[o:o + N + 1, :nx], g[0].lo) < tol and rel_err(hi[o:o + N + 1, :nx], g[0].hi) < tol
        ub = slice(B.MAX_NX, B.MAX_NX + nu)
        assert rel_err(lo[o:o + N, ub], g[1].lo[:N]) < tol and rel_err(hi[o:o + N, ub], g[1].hi[:N]) < tol
        if inst["model"] in (1, 3):
            hsg = [grp for grp in g if grp.kind == "halfspace"]
            assert len(hsg) == inst["obstacles"].shape[0]
            for j, grp in enumerate(hsg):
                assert rel_err(hs[o + 1:o + N + 1, 4 * j:4 * j + 3], grp.a[1:]) < tol
                assert rel_err(hs[o + 1:o + N + 1, 4 * j + 3], grp.b[1:]) < tol
    prob.close()


@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
def test_admm_fixed_iterations_plain(B, prec, tol):
    insts = _ragged_quads(5, 20) + [scpgen.mars_instance(2, 7, N=13)]
    _say("admm_solve", prec)
    prob = B.Problem(insts, precision=prec)
    prob.linearize(B.admm_params(1.0))
    prob.admm(B.admm_params(1.0, 23))
    prob.admm(B.admm_params(1.0, 14))     # continues from the arena state: 37 iterations total
    f = gpu_fields(prob)
    trajs = [oracle_linearize_admm(d, 37) for d in insts]
    worst = compare(prob, f, insts, trajs)
    _say(worst)
    assert max(worst.values()) < tol
    prob.close()


@pytest.mark.parametrize("form", ["plain", "persistent"])
def test_scp_config0_fp64(B, form):
    insts = scpgen.config0()
    _say("config0 fp64", form)
    prob = B.Problem(insts, precision="f64")
    prob.solve(B.scp_params(10, 100, form=form))
    f = gpu_fields(prob)
    _, _, info = prob.result()
    trajs, oinfo = oracle_scp(insts, 10, 100)
    worst = compare(prob, f, insts, trajs)
    _say(worst)
    assert max(worst.values()) < TOL64
    inf = prob.info_dicts(info.cpu().numpy())[0]
    t = trajs[0]
    assert inf["admm_iters"] == oinfo[0]["admm_iters"] and inf["n_accept"] == oinfo[0]["n_accept"]
    assert abs(inf["cost"] - oracle.cost(insts[0], t.xbar, t.ubar)) <= TOL64 * abs(inf["cost"])
    assert abs(inf["defect"] - oracle.defect(insts[0], t.xbar, t.ubar)) <= TOL64
    assert abs(inf["viol"] - oracle.violation(insts[0], t.xbar, t.ubar)) <= TOL64
    assert abs(inf["bnd_err"] - oracle.boundary_error(insts[0], t.xbar)) <= TOL64
    assert abs(inf["r_p"] - oinfo[0]["r_p"]) <= TOL64 and abs(inf["r_d"] - oinfo[0]["r_d"]) <= TOL64
    prob.close()


@pytest.mark.parametrize("form", ["plain", "persistent"])
def test_scp_ragged_batch_fp64(B, form):
    """Ragged horizons spanning several workgroups, obstacle counts 0..8, both models."""
    insts = _ragged_quads(14, 40) + [scpgen.mars_instance(2, 20 + i, N=6 + 5 * i) for i in range(4)]
    _say("ragged fp64", form, [d["N"] for d in insts])
    prob = B.Problem(insts, precision="f64")
    prob.solve(B.scp_params(3, 30, form=form))
    f = gpu_fields(prob)
    trajs, _ = oracle_scp(insts, 3, 30)
    worst = compare(prob, f, insts, trajs)
    _say(worst)
    assert max(worst.values()) < TOL64
    prob.close()


@pytest.mark.parametrize("form", ["plain", "persistent"])
def test_scp_fp32_short_budgets(B, form):
    insts = scpgen.config1(6) + [scpgen.mars_instance(2, i, N=60) for i in range(2)]
    for K, J in [(1, 200), (3, 50)]:
        _say("fp32", form, K, J)
        prob = B.Problem(insts, precision="f32")
        prob.solve(B.scp_params(K, J, form=form))
        f = gpu_fields(prob)
        trajs, _ = oracle_scp(insts, K, J)
        worst = compare(prob, f, insts, trajs)
        _say(worst)
        assert max(worst.values()) < TOL32
        prob.close()


def test_residual_stopping_matches_oracle(B):
    """Residual test every 10 iterations, eps 1e-4, rho 3: the per-trajectory iteration counts
    (integers) and the iterates at the stop agree with the oracle; some trajectories stop early,
    one runs the whole budget."""
    insts = [scpgen.quad_instance(3, i, N=15 + i, K=2, T=5.0, delta=5.0) for i in range(3)]
    insts += [scpgen.mars_instance(3, 5, N=12)]
    kw = dict(check_every=10, eps_p=1e-4, eps_d=1e-4, rho_eq=3.0, rho_dyn=3.0, rho_geo=3.0)
    trajs, oinfo = oracle_scp(insts, 3, 600, **kw)
    assert any(o["admm_iters"] < 1800 for o in oinfo) and any(o["admm_iters"] == 1800 for o in oinfo)
    for form in ["plain", "persistent"]:
        _say("residual stop", form)
        prob = B.Problem(insts, precision="f64")
        prob.solve(B.scp_params(3, 600, check_every=10, eps=1e-4, rho=3.0, form=form))
        f = gpu_fields(prob)
        _, _, info = prob.result()
        inf = prob.info_dicts(info.cpu().numpy())
        _say([i["admm_iters"] for i in inf], [o["admm_iters"] for o in oinfo])
        assert [i["admm_iters"] for i in inf] == [o["admm_iters"] for o in oinfo]
        worst = compare(prob, f, insts, trajs)
        _say(worst)
        assert max(worst.values()) < TOL64
        prob.close()


def test_trust_region_ratio_test_matches_oracle(B):
    insts = [scpgen.quad_instance(1, 7, N=20, K=4), scpgen.quad_instance(1, 8, N=12, K=3)]
    kw = dict(eta0=0.05, eta1=0.25, eta2=0.75, shrink=0.5, grow=2.0, delta_max=2.0)
    for form in ["plain", "persistent"]:
        _say("ratio test", form)
        prob = B.Problem(insts, precision="f64")
        prob.solve(B.scp_params(8, 60, form=form, **kw))
        f = gpu_fields(prob)
        _, _, info = prob.result()
        trajs, oinfo = oracle_scp(insts, 8, 60, **kw)
        inf = prob.info_dicts(info.cpu().numpy())
        for a, o in zip(inf, oinfo):
            assert a["n_accept"] == o["n_accept"] and a["delta"] == o["delta"]
        assert any(o["n_accept"] < 8 or o["delta"] != 1.0 for o in oinfo)
        worst = compare(prob, f, insts, trajs)
        assert max(worst.values()) < TOL64
        prob.close()


def test_scenario_groups_fp64(B):
    """Consensus on the first control across scenarios (robust MPC request)."""
    reqs = scpgen.config4_request(0, S=4, N=10) + scpgen.config4_request(1, S=3, N=14)
    for form in ["plain", "persistent"]:
        _say("scenarios", form)
        prob = B.Problem(reqs, precision="f64")
        prob.solve(B.scp_params(3, 40, form=form))
        f = gpu_fields(prob)
        trajs, _ = oracle_scp(reqs, 3, 40)
        worst = compare(prob, f, reqs, trajs)
        _say(worst)
        assert max(worst.values()) < TOL64
        cp = f["copy"]
        for t0, S in [(0, 4), (4, 3)]:
            firsts = [cp[prob.offsets[t0 + m], 6:12] for m in range(S)]
            for v in firsts[1:]:
                np.testing.assert_array_equal(v, firsts[0])
        prob.close()


def test_edge_cases(B):
    """One interval, no obstacles, and the longest trajectory a 256-lane workgroup holds."""
    insts = [scpgen.quad_instance(5, 0, N=1, K=0, T=0.5), scpgen.quad_instance(5, 1, N=2, K=8, T=0.6),
             scpgen.mars_instance(5, 2, N=1), scpgen.quad_instance(5, 3, N=255, K=3, T=25.5)]
    _say("edge fp32 persistent / plain")
    out = {}
    for form in ["persistent", "plain"]:
        prob = B.Problem(insts, precision="f32")
        prob.solve(B.scp_params(2, 30, form=form))
        out[form] = gpu_fields(prob)
        trajs, _ = oracle_scp(insts, 2, 30)
        worst = compare(prob, out[form], insts, trajs)
        _say(form, worst)
        assert max(worst.values()) < TOL32
        prob.close()


def test_invalid_arguments_are_errors(B):
    insts = scpgen.config1(2)
    prob = B.Problem(insts, precision="f32")
    with pytest.raises(B.ScpError):
        prob.admm(B.admm_params(1.0, 5))                 # before scp_linearize
    prob.linearize(B.admm_params(1.0))
    with pytest.raises(B.ScpError):
        prob.admm(B.admm_params(2.0, 5))                 # penalties differ from the factors
    with pytest.raises(B.ScpError):
        prob.solve(B.scp_params(1, 10, rho=-1.0))
    prob.close()
    bad = [dict(scpgen.quad_instance(0, 0, N=300, K=2), group=-1)]
    p2 = B.Problem(bad, precision="f32")                 # longer than a workgroup: plain form only
    with pytest.raises(B.ScpError):
        p2.solve(B.scp_params(1, 5, form="persistent"))
    p2.solve(B.scp_params(1, 5, form="plain"))
    p2.close()


def test_reset_then_solve_equals_fresh_solve(B):
    """scp_reset restores the initial guess and clears the state: a second solve after a reset is
    bitwise equal to the first solve of a fresh problem (both forms)."""
    insts = scpgen.config1(4) + [scpgen.mars_instance(2, 3, N=30)]
    for form in ["persistent", "plain"]:
        _say("reset", form)
        fresh = B.Problem(insts, precision="f32")
        fresh.solve(B.scp_params(3, 40, form=form))
        x1, u1, i1 = (a.cpu().numpy() for a in fresh.result())
        fresh.solve(B.scp_params(3, 40, form=form))          # warm start: different result
        x2, _, _ = (a.cpu().numpy() for a in fresh.result())
        assert not np.array_equal(x1, x2)
        fresh.reset()
        fresh.solve(B.scp_params(3, 40, form=form))
        x3, u3, i3 = (a.cpu().numpy() for a in fresh.result())
        np.testing.assert_array_equal(x3, x1)
        np.testing.assert_array_equal(u3, u1)
        np.testing.assert_array_equal(i3, i1)
        fresh.close()


@pytest.mark.parametrize("form,per_launch", [("plain", 0), ("persistent", 0), ("persistent", 1)])
def test_penalty_schedule_fp64(B, form, per_launch):
    """The paper's geometric penalty schedule (1e2 -> 1e3 over the SCP iterations), duals carried
    unscaled, the persistent form also split into one launch per SCP iteration."""
    insts = _ragged_quads(5, 60) + [scpgen.mars_instance(2, 30, N=14)]
    kw = dict(rho_eq=100.0, rho_dyn=100.0, rho_geo=100.0, rho_final=1e3)
    trajs, oinfo = oracle_scp(insts, 4, 40, **kw)
    _say("schedule", form, per_launch)
    prob = B.Problem(insts, precision="f64")
    prob.solve(B.scp_params(4, 40, rho=100.0, rho_final=1e3, form=form, scp_per_launch=per_launch))
    f = gpu_fields(prob)
    worst = compare(prob, f, insts, trajs)
    _say(worst)
    assert max(worst.values()) < TOL64
    prob.close()

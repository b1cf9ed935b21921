"""GPU parity of the 6-DOF lander (Sec. IV-B; plain form), through the C ABI, against the FP64
oracle.

* Linearization and convexified sets (A, B, d, boxes, the linearized lower thrust bound) on
  ragged horizons, one nominal with its quaternion off the unit sphere: FP64 1e-12, FP32 2e-6.
* ADMM at fixed iteration counts on ragged horizons: every block of iterates in FP64 to 1e-9 and
  in FP32 to 1e-4.
* The nominal descent (Sec. IV-B.1: N = 30, horizon 5) in FP64 at 20 SCP x 200 ADMM with rho
  geometric from 1e2 to 1e3: every block and the info record to 1e-9.
* The Monte-Carlo batch at its full size (Sec. IV-B.2: 1000 dispersed descents, N = 30) in FP64
  at the bench budget: sampled trajectories against the oracle to 1e-9; in FP32 the first SCP
  iteration of the samples to 1e-4 and, at the full budget, every sample bit-identical alone and
  in the batch.
* Edge cases: horizons N = 1, 2 and 240 in one batch (FP64, 1e-9).
* The persistent form of this model keeps the ADMM iterations resident in one workgroup per
  trajectory; it gives the plain form's bits (FP32 and FP64, full budget) and meets the same
  oracle bars, on horizons up to 63 intervals.  It refuses longer trajectories and residual-test
  cadences; the request server and consensus groups refuse the model with an error.

The lander's mirror copies [x box 14][u box 3][glide 3][tilt 2][rate 3][thrust ball 3][lower
bound 3][gimbal 3] list the cones' components axis last, exactly as the oracle's groups do, so the
copies and duals compare slot for slot.
"""
import numpy as np
import pytest

import oracle
import scpgen
from _parity import compare, gpu_fields, oracle_linearize_admm, oracle_scp, rel_err

pytestmark = pytest.mark.gpu

TOL64 = 1e-9
TOL32 = 1e-4
SCHED = dict(rho=100.0, rho_final=1e3)
OSCHED = dict(rho_eq=100.0, rho_dyn=100.0, rho_geo=100.0, rho_final=1e3)


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def B(lib):
    from paper_2603_10711_amd import binding
    return binding


def _ragged(n, base=0):
    out = []
    for i in range(n):
        d = scpgen.lander6_perturbed(base + i)
        N = 3 + (7 * i) % 28
        out.append(scpgen.lander6_instance(d["x_init"], N=N, tf=5.0 * N / 30))
    return out


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 2e-6)])
def test_linearize_and_convexify(B, prec, tol):
    insts = _ragged(5)
    rng = np.random.default_rng(3)
    insts[-1]["x_guess"][:, 6:10] *= 1.2
    insts[-1]["u_guess"] = insts[-1]["u_guess"] + rng.normal(size=insts[-1]["u_guess"].shape) * 0.3
    _say("lander linearize", prec, [d["N"] for d in insts])
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
        low = [x for x in g if x.kind == "halfspace"][0]
        assert rel_err(hs[o:o + N, 0:3], low.a[:N]) < tol and rel_err(hs[o:o + N, 3], low.b[:N]) < tol
    prob.close()


@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
def test_admm_fixed_iterations(B, prec, tol):
    insts = _ragged(10, 20)
    _say("lander admm", prec, [d["N"] for d in insts])
    prob = B.Problem(insts, precision=prec)
    prob.linearize(B.admm_params(1.0))
    prob.admm(B.admm_params(1.0, 19))
    prob.admm(B.admm_params(1.0, 11))
    f = gpu_fields(prob)
    trajs = [oracle_linearize_admm(d, 30) for d in insts]
    worst = compare(prob, f, insts, trajs)
    _say(worst)
    assert max(worst.values()) < tol
    prob.close()


@pytest.mark.parametrize("form", ["plain", "persistent"])
def test_nominal_descent_fp64(B, form):
    insts = [scpgen.lander6_instance()]
    _say("lander nominal fp64 20x200", form)
    prob = B.Problem(insts, precision="f64")
    prob.solve(B.scp_params(20, 200, form=form, **SCHED))
    f = gpu_fields(prob)
    _, _, info = prob.result()
    trajs, oinfo = oracle_scp(insts, 20, 200, **OSCHED)
    worst = compare(prob, f, insts, trajs)
    _say(worst)
    assert max(worst.values()) < TOL64
    inf = prob.info_dicts(info.cpu().numpy())[0]
    d, t = insts[0], trajs[0]
    _say("defect", inf["defect"], "cost", inf["cost"], "viol", inf["viol"], "bnd", inf["bnd_err"])
    assert abs(inf["cost"] - oracle.cost(d, t.xbar, t.ubar)) <= TOL64 * max(1.0, abs(inf["cost"]))
    assert abs(inf["defect"] - oracle.defect(d, t.xbar, t.ubar)) <= TOL64
    assert abs(inf["viol"] - oracle.violation(d, t.xbar, t.ubar)) <= TOL64
    assert abs(inf["bnd_err"] - oracle.boundary_error(d, t.xbar)) <= TOL64
    assert inf["defect"] < 0.01
    prob.close()


SAMPLE = [0, 421, 999]


@pytest.mark.parametrize("form", ["plain", "persistent"])
def test_monte_carlo_fullsize_fp64_samples(B, form):
    insts = scpgen.config6(1000)
    _say("lander 1000 x 31 fp64 20x200", form)
    prob = B.Problem(insts, precision="f64")
    prob.solve(B.scp_params(20, 200, form=form, **SCHED))
    x, u, info = (a.cpu().numpy() for a in prob.result())
    for i in SAMPLE:
        (t,), _ = oracle_scp([insts[i]], 20, 200, **OSCHED)
        ex = rel_err(prob.split(x, i, 14), t.xbar)
        eu = rel_err(prob.split(u, i, 3, True), t.ubar)
        _say(i, ex, eu)
        assert max(ex, eu) < TOL64
        assert abs(info[i, 6] - oracle.defect(insts[i], t.xbar, t.ubar)) <= TOL64
    prob.close()


@pytest.mark.parametrize("form", ["plain", "persistent"])
def test_monte_carlo_fullsize_fp32(B, form):
    insts = scpgen.config6(1000)
    _say("lander 1000 x 31 fp32 first SCP iteration", form)
    prob = B.Problem(insts, precision="f32")
    prob.solve(B.scp_params(1, 200, form=form, **SCHED))
    f = gpu_fields(prob)
    for i in SAMPLE:
        (t,), _ = oracle_scp([insts[i]], 1, 200, **OSCHED)
        worst = compare(prob, f, [insts[i]], [t], idx=[i])
        _say(i, worst)
        assert max(worst.values()) < TOL32
    prob.reset()
    prm = B.scp_params(20, 200, form=form, **SCHED)
    prob.solve(prm)
    x, u, info = (a.cpu().numpy() for a in prob.result())
    for i in SAMPLE:
        one = B.Problem([insts[i]], precision="f32")
        one.solve(prm)
        x1, u1, info1 = (a.cpu().numpy() for a in one.result())
        np.testing.assert_array_equal(x1, prob.split(x, i))
        np.testing.assert_array_equal(u1[:insts[i]["N"]], prob.split(u, i, controls=True))
        np.testing.assert_array_equal(info1[0], info[i])
        one.close()
    defect = info[:, 6]
    _say("fp32 defect p50", float(np.median(defect)), "p90", float(np.percentile(defect, 90)))
    assert np.all(np.isfinite(defect)) and float(np.median(defect)) < 0.05
    prob.close()


def test_edge_horizons_fp64(B):
    """The shortest horizons (N = 1, 2) and a long one (N = 240) of the dispersed descent."""
    x0s = [scpgen.lander6_perturbed(50 + i)["x_init"] for i in range(3)]
    insts = [scpgen.lander6_instance(x0s[0], N=1, tf=5.0 / 30), scpgen.lander6_instance(x0s[1], N=2, tf=10.0 / 30),
             scpgen.lander6_instance(x0s[2], N=240, tf=5.0)]
    _say("lander edge horizons fp64", [d["N"] for d in insts])
    prob = B.Problem(insts, precision="f64")
    prob.solve(B.scp_params(3, 20, form="plain", **SCHED))
    f = gpu_fields(prob)
    trajs, _ = oracle_scp(insts, 3, 20, **OSCHED)
    worst = compare(prob, f, insts, trajs)
    _say(worst)
    assert max(worst.values()) < TOL64
    prob.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_resident_and_plain_forms_agree_bitwise(B, prec):
    insts = scpgen.config6(160)
    out = {}
    for form in ("plain", "persistent"):
        prob = B.Problem(insts, precision=prec)
        prob.solve(B.scp_params(20, 200, form=form, **SCHED))
        f = gpu_fields(prob, ("x", "u", "z", "lam", "mu", "copy", "dual"))
        x, u, info = (a.cpu().numpy() for a in prob.result())
        out[form] = (f, x, u, info)
        prob.close()
    (fp, xp, up, ip), (fr, xr, ur, ir) = out["plain"], out["persistent"]
    for k in fp:
        np.testing.assert_array_equal(fr[k], fp[k], err_msg=k)
    np.testing.assert_array_equal(xr, xp)
    np.testing.assert_array_equal(ur, up)
    np.testing.assert_array_equal(ir, ip)


def test_resident_edge_horizons_fp64(B):
    """Horizons N = 1, 2 and 63 (the longest resident trajectory) together."""
    x0s = [scpgen.lander6_perturbed(80 + i)["x_init"] for i in range(3)]
    insts = [scpgen.lander6_instance(x0s[0], N=1, tf=5.0 / 30), scpgen.lander6_instance(x0s[1], N=2, tf=10.0 / 30),
             scpgen.lander6_instance(x0s[2], N=63, tf=5.0 * 63 / 30)]
    prob = B.Problem(insts, precision="f64")
    prob.solve(B.scp_params(3, 20, form="persistent", **SCHED))
    f = gpu_fields(prob)
    trajs, _ = oracle_scp(insts, 3, 20, **OSCHED)
    worst = compare(prob, f, insts, trajs)
    _say("lander resident edge", worst)
    assert max(worst.values()) < TOL64
    prob.close()


def test_persistent_limits_server_and_groups_refuse(B):
    long = [scpgen.lander6_instance(N=64, tf=5.0 * 64 / 30)]    # 65 nodes: over the resident limit
    prob = B.Problem(long, precision="f32")
    with pytest.raises(RuntimeError, match="64 nodes"):
        prob.solve(B.scp_params(2, 10, form="persistent"))
    prob.close()
    insts = scpgen.config6(2)
    prob = B.Problem(insts, precision="f32")
    with pytest.raises(RuntimeError, match="fixed budgets"):
        prob.solve(B.scp_params(2, 10, form="persistent", check_every=5, eps=1e-4))
    prob.close()
    srv = B.Server(B.scp_params(2, 10), precision="f32", block=256, max_nodes=1 << 12, max_traj=16, max_wg=16,
                   max_span=4, max_requests=4)
    try:
        with pytest.raises(RuntimeError):
            srv.submit(insts, session=-1)
    finally:
        srv.close()
    grouped = [dict(d, group=1) for d in insts]
    with pytest.raises(RuntimeError, match="consensus"):
        B.Problem(grouped, precision="f32")

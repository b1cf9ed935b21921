"""GPU parity of the 6-DOF quadrotor model (Sec. IV-A.1; plain form), through the C ABI, against
the FP64 oracle.

* ADMM at fixed iteration counts on ragged horizons (several 256-node blocks and a ragged tail,
  obstacle counts 0..8): every block of iterates in FP64 to 1e-9 and in FP32 to 1e-4.
* The parameter-study scene (Sec. IV-A.2: N = 50, 20 SCP x 200 ADMM, rho geometric from 1e2 to
  1e3) in FP64: every block and the info record (cost, defect, violation, boundary error) to 1e-9.
* The scalability-benchmark batch at its full size (Sec. IV-A.3: 1000 trajectories, N = 40,
  three random obstacles) solved once in FP64 at the bench budget: sampled trajectories against
  the oracle to 1e-9; and in FP32 the first SCP iteration of sampled trajectories to 1e-4 (at
  the full budget the SCP map amplifies FP32 rounding far beyond it, as for the other models)
  and every FP32 trajectory bit-identical alone and in the batch.
* Edge cases: horizons N = 1 and 2, no obstacles and N = 300 in one batch (FP64, 1e-9); a zero
  quaternion in one nominal (the thrust direction is undefined there) sets SCP_ST_NONFINITE on
  that trajectory only, the others equal their lone solves bit for bit.
* A scenario group (consensus on the first control) in FP64 to 1e-9.
* The trust-region ratio test of the SCP step (the benchmark's goodput setting: rho 10 -> 3e4,
  accept when the ratio is positive, radius halved below 0.25, doubled above 0.75 up to 4) on a
  small batch in FP64: accepted-step counts and final radii exact, iterates to 1e-9, both forms.
* The persistent form of this model keeps the ADMM iterations resident in one workgroup per
  trajectory (four lanes per node); it performs the plain kernels' operations in their order, so
  both forms give the same bits (FP32 and FP64, full budget), and it meets the oracle bars above.
  It refuses trajectories over 64 nodes, consensus groups and residual-test cadences; the request
  server refuses the model.

The mirror copies of this model sit in the quadrotor layout [x box 13][u box 4][ball 3][half-
space k: 3 each]; the ball slots never hold a group and must read 0.  They are dropped before the
comparison with the oracle, which has no ball group for this model.
"""
import numpy as np
import pytest

import oracle
import scpgen
from _parity import compare, gpu_fields, oracle_linearize_admm, oracle_scp, rel_err

pytestmark = pytest.mark.gpu

TOL64 = 1e-9
TOL32 = 1e-4
BALL = [17, 18, 19]
SCHED = dict(rho=100.0, rho_final=1e3)
OSCHED = dict(rho_eq=100.0, rho_dyn=100.0, rho_geo=100.0, rho_final=1e3)


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def B(lib):
    from paper_2603_10711_amd import binding
    return binding


def _fields(prob):
    f = gpu_fields(prob)
    for k in ("copy", "dual"):
        assert np.all(f[k][:, BALL] == 0.0), k
        f[k] = np.delete(f[k], BALL, axis=1)
    return f


def _ragged(n, base=0):
    out = []
    for i in range(n):
        N = 4 + (11 * i) % 37
        d = scpgen.quad6_benchmark_instance(base + i, N=N, K=3)
        K = i % 9
        obs = np.tile(d["obstacles"], (3, 1))[:K]
        d["obstacles"] = obs
        out.append(d)
    return out


@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
def test_admm_fixed_iterations(B, prec, tol):
    insts = _ragged(12)
    _say("quad6 admm", prec, [d["N"] for d in insts], sum(d["N"] + 1 for d in insts))
    prob = B.Problem(insts, precision=prec)
    prob.linearize(B.admm_params(1.0))
    prob.admm(B.admm_params(1.0, 17))
    prob.admm(B.admm_params(1.0, 12))
    f = _fields(prob)
    trajs = [oracle_linearize_admm(d, 29) for d in insts]
    worst = compare(prob, f, insts, trajs)
    _say(worst)
    assert max(worst.values()) < tol
    prob.close()


@pytest.mark.parametrize("form", ["plain", "persistent"])
def test_parameter_study_scene_fp64(B, form):
    insts = [scpgen.quad6_scene()]
    _say("quad6 scene fp64 20x200", form)
    prob = B.Problem(insts, precision="f64")
    prob.solve(B.scp_params(20, 200, form=form, **SCHED))
    f = _fields(prob)
    _, _, info = prob.result()
    trajs, oinfo = oracle_scp(insts, 20, 200, **OSCHED)
    worst = compare(prob, f, insts, trajs)
    _say(worst)
    assert max(worst.values()) < TOL64
    inf = prob.info_dicts(info.cpu().numpy())[0]
    d, t = insts[0], trajs[0]
    _say("defect", inf["defect"], "cost", inf["cost"], "viol", inf["viol"], "bnd", inf["bnd_err"])
    assert abs(inf["cost"] - oracle.cost(d, t.xbar, t.ubar)) <= TOL64 * abs(inf["cost"])
    assert abs(inf["defect"] - oracle.defect(d, t.xbar, t.ubar)) <= TOL64
    assert abs(inf["viol"] - oracle.violation(d, t.xbar, t.ubar)) <= TOL64
    assert abs(inf["bnd_err"] - oracle.boundary_error(d, t.xbar)) <= TOL64
    assert inf["admm_iters"] == oinfo[0]["admm_iters"]
    assert inf["defect"] < 0.02     # the schedule converges this scene
    prob.close()


SAMPLE = [0, 137, 999]


@pytest.mark.parametrize("form", ["plain", "persistent"])
def test_benchmark_batch_fullsize_fp64_samples(B, form):
    insts = scpgen.config5(1000)
    _say("quad6 1000 x 41 fp64 20x200", form)
    prob = B.Problem(insts, precision="f64")
    prob.solve(B.scp_params(20, 200, form=form, **SCHED))
    x, u, info = (a.cpu().numpy() for a in prob.result())
    for i in SAMPLE:
        (t,), _ = oracle_scp([insts[i]], 20, 200, **OSCHED)
        ex = rel_err(prob.split(x, i, 13), t.xbar)
        eu = rel_err(prob.split(u, i, 4, True), t.ubar)
        _say(i, ex, eu)
        assert max(ex, eu) < TOL64
        assert abs(info[i, 6] - oracle.defect(insts[i], t.xbar, t.ubar)) <= TOL64
    prob.close()


@pytest.mark.parametrize("form", ["plain", "persistent"])
def test_benchmark_batch_fullsize_fp32(B, form):
    insts = scpgen.config5(1000)
    _say("quad6 1000 x 41 fp32 first SCP iteration", form)
    prob = B.Problem(insts, precision="f32")
    prob.solve(B.scp_params(1, 200, form=form, **SCHED))
    f = _fields(prob)
    for i in SAMPLE:
        (t,), _ = oracle_scp([insts[i]], 1, 200, **OSCHED)
        worst = compare(prob, f, [insts[i]], [t], idx=[i])
        _say(i, worst)
        assert max(worst.values()) < TOL32
    # full budget: every trajectory alone equals its row in the batch, bit for bit
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


def test_scenario_group_fp64(B):
    """Scenarios sharing their first control by consensus (Sec. IV-A.4) on the 6-DOF model: node 0 of the
    group takes the averaged copies; every block against the oracle, next to a lone trajectory."""
    base = scpgen.quad6_benchmark_instance(7, N=18)
    insts = []
    for m, mass in enumerate((0.9, 1.0, 1.15)):
        d = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in base.items()}
        d["mscale"] = mass
        d["group"] = 3
        insts.append(d)
    insts.append(scpgen.quad6_benchmark_instance(8, N=11))
    _say("quad6 scenario group fp64")
    prob = B.Problem(insts, precision="f64")
    prob.solve(B.scp_params(3, 30, form="plain", **SCHED))
    f = _fields(prob)
    trajs, _ = oracle_scp(insts, 3, 30, **OSCHED)
    worst = compare(prob, f, insts, trajs)
    _say(worst)
    assert max(worst.values()) < TOL64
    cp = f["copy"]   # the node-0 control copies (u box) agree across the scenarios
    for t in (1, 2):
        np.testing.assert_allclose(cp[prob.offsets[t], 13:17], cp[prob.offsets[0], 13:17], rtol=0, atol=1e-12)
    prob.close()


def test_edge_horizons_fp64(B):
    """The shortest horizons (N = 1, 2), no obstacles, and a long horizon (N = 300) in one batch."""
    insts = [scpgen.quad6_benchmark_instance(30, N=1), scpgen.quad6_benchmark_instance(31, N=2),
             scpgen.quad6_benchmark_instance(32, N=5, K=0), scpgen.quad6_benchmark_instance(33, N=300)]
    _say("quad6 edge horizons fp64", [d["N"] for d in insts])
    prob = B.Problem(insts, precision="f64")
    prob.solve(B.scp_params(3, 20, form="plain", **SCHED))
    f = _fields(prob)
    trajs, _ = oracle_scp(insts, 3, 20, **OSCHED)
    worst = compare(prob, f, insts, trajs)
    _say(worst)
    assert max(worst.values()) < TOL64
    prob.close()


def test_zero_quaternion_is_flagged_and_contained(B):
    """A nominal with a zero quaternion leaves the thrust direction undefined: that trajectory
    reports SCP_ST_NONFINITE and its neighbours in the batch are unaffected (bit for bit)."""
    insts = [scpgen.quad6_benchmark_instance(40, N=12), scpgen.quad6_benchmark_instance(41, N=12),
             scpgen.quad6_benchmark_instance(42, N=9)]
    insts[1]["x_guess"][5, 6:10] = 0.0
    prm = B.scp_params(2, 10, form="plain", **SCHED)
    prob = B.Problem(insts, precision="f32")
    prob.solve(prm)
    x, u, info = (a.cpu().numpy() for a in prob.result())
    assert int(info[1, 5]) & B.ST_NONFINITE
    for i in (0, 2):
        assert not int(info[i, 5]) & B.ST_NONFINITE
        one = B.Problem([insts[i]], precision="f32")
        one.solve(prm)
        x1, u1, info1 = (a.cpu().numpy() for a in one.result())
        np.testing.assert_array_equal(x1, prob.split(x, i))
        np.testing.assert_array_equal(info1[0], info[i])
        one.close()
    prob.close()


def _short_batch():
    # at most 32 nodes per trajectory: the resident kernel's 32-row variant (128-lane workgroups)
    return [scpgen.quad6_benchmark_instance(80 + i, N=5 + (7 * i) % 27) for i in range(40)]


@pytest.mark.parametrize("prec,batch", [("f32", "bench"), ("f64", "bench"), ("f32", "short")])
def test_resident_and_plain_forms_agree_bitwise(B, prec, batch):
    insts = scpgen.config5(160) if batch == "bench" else _short_batch()
    prm = dict(**SCHED)
    out = {}
    for form in ("plain", "persistent"):
        prob = B.Problem(insts, precision=prec)
        prob.solve(B.scp_params(20, 200, form=form, **prm))
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
    """Horizons N = 1, 2, 5 (no obstacles) and 63 (the longest resident trajectory) together."""
    insts = [scpgen.quad6_benchmark_instance(60, N=1), scpgen.quad6_benchmark_instance(61, N=2),
             scpgen.quad6_benchmark_instance(62, N=5, K=0), scpgen.quad6_benchmark_instance(63, N=63)]
    prob = B.Problem(insts, precision="f64")
    prob.solve(B.scp_params(3, 20, form="persistent", **SCHED))
    f = _fields(prob)
    trajs, _ = oracle_scp(insts, 3, 20, **OSCHED)
    worst = compare(prob, f, insts, trajs)
    _say("resident edge", worst)
    assert max(worst.values()) < TOL64
    prob.close()


def test_persistent_form_limits_and_server_refuse(B):
    long = [scpgen.quad6_benchmark_instance(70, N=64)]        # 65 nodes: over the resident limit
    prob = B.Problem(long, precision="f32")
    with pytest.raises(RuntimeError, match="64 nodes"):
        prob.solve(B.scp_params(2, 10, form="persistent"))
    prob.close()
    insts = scpgen.config5(2)
    prob = B.Problem(insts, precision="f32")
    with pytest.raises(RuntimeError, match="fixed budgets"):
        prob.solve(B.scp_params(2, 10, form="persistent", check_every=5, eps=1e-4))
    prob.close()
    grouped = [dict(d, group=2) for d in [scpgen.quad6_benchmark_instance(71, N=9)] * 2]
    prob = B.Problem(grouped, precision="f32")
    with pytest.raises(RuntimeError, match="64 nodes"):
        prob.solve(B.scp_params(2, 10, form="persistent"))
    prob.close()
    srv = B.Server(B.scp_params(2, 10), precision="f32", block=256, max_nodes=1 << 12, max_traj=16, max_wg=16,
                   max_span=4, max_requests=4)
    try:
        with pytest.raises(RuntimeError):
            srv.submit(insts, session=-1)
    finally:
        srv.close()


def test_resident_short_horizons_fp32_match_oracle(B):
    """The 32-row resident variant in FP32 (Step 1 through the inverse, A in LDS) against the
    oracle at the FP32 bar, on a few SCP iterations."""
    insts = _short_batch()[:8]
    prob = B.Problem(insts, precision="f32")
    prob.solve(B.scp_params(2, 30, form="persistent", **SCHED))
    f = _fields(prob)
    trajs, _ = oracle_scp(insts, 2, 30, **OSCHED)
    worst = compare(prob, f, insts, trajs)
    _say("resident short fp32", worst)
    assert max(worst.values()) < TOL32
    prob.close()


TR = dict(eta0=0.0, eta1=0.25, eta2=0.75, shrink=0.5, grow=2.0, delta_max=4.0)


@pytest.mark.parametrize("form", ["plain", "persistent"])
def test_trust_region_ratio_test_fp64(B, form):
    insts = [scpgen.quad6_benchmark_instance(i, N=8 + 5 * i) for i in range(4)]
    _say("quad6 ratio test fp64 12x80", form, [d["N"] for d in insts])
    prob = B.Problem(insts, precision="f64")
    prob.solve(B.scp_params(12, 80, form=form, rho=10.0, rho_final=3e4, **TR))
    f = _fields(prob)
    _, _, info = prob.result()
    trajs, oinfo = oracle_scp(insts, 12, 80, rho_eq=10.0, rho_dyn=10.0, rho_geo=10.0, rho_final=3e4, **TR)
    inf = prob.info_dicts(info.cpu().numpy())
    _say([(a["n_accept"], a["delta"]) for a in inf], [(o["n_accept"], o["delta"]) for o in oinfo])
    for a, o in zip(inf, oinfo):
        assert a["n_accept"] == o["n_accept"] and a["delta"] == o["delta"]
    # the test exercises rejections or radius changes, not only always-accepted unit steps
    assert any(o["n_accept"] < 12 for o in oinfo) and any(o["delta"] != 1.0 for o in oinfo)
    worst = compare(prob, f, insts, trajs)
    _say(worst)
    assert max(worst.values()) < TOL64
    prob.close()


@pytest.mark.parametrize("model", ["quad6", "lander6"])
@pytest.mark.parametrize("form", ["persistent", "plain"])
def test_graph_replay_equals_direct_launches_6dof(B, model, form):
    """The 6-DOF solve as the benchmark times it (one hipGraph per solve, penalty schedule, and for
    the quadrotor the trust-region ratio test): every replay, with eager work and a
    synchronization between replays, equals the solve launched directly, bit for bit."""
    import torch
    if model == "quad6":
        insts = [scpgen.quad6_benchmark_instance(i, N=20 + 4 * i) for i in range(5)]
        tr = dict(eta0=0.0, eta1=0.25, eta2=0.75, shrink=0.5, grow=2.0, delta_max=4.0)
    else:
        insts = [scpgen.lander6_perturbed(i) for i in range(5)]
        tr = {}
    s = torch.cuda.Stream()

    def prm(graph):
        return B.scp_params(4, 30, rho=10.0, rho_final=1e3, form=form, graph=graph, **tr)

    direct = B.Problem(insts, precision="f32", stream=s)
    direct.solve(prm(False))
    ref = [a.cpu().numpy() for a in direct.result()]
    direct.close()
    g = B.Problem(insts, precision="f32", stream=s)
    for rep in range(3):
        g.reset()
        g.solve(prm(True))
        out = [a.cpu().numpy() for a in g.result()]
        print("graph replay", model, form, rep, flush=True)
        for a, b in zip(out, ref):
            np.testing.assert_array_equal(a, b)
        # eager work of the program between replays
        with torch.cuda.stream(s):
            torch.ones(1 << 20, device="cuda").mul_(2.0).sum().item()
        torch.cuda.synchronize()
    g.close()

"""Numerical failures are per-trajectory status bits, and they stay inside their trajectory.

The C ABI reports a non-positive Cholesky pivot (SCP_ST_BADPIVOT), a hard box with lo > hi
(SCP_ST_EMPTYSET), non-finite iterates (SCP_ST_NONFINITE) and a residual blow-up
(SCP_ST_DIVERGED) in the info record of the trajectory they occur in and never fails the call.
Every solve here runs with residual blow-up detection on (scp_params.detect_blowup). The blow-up
case is a negative control weight (the QP turns nonconvex while H stays positive
definite, and ADMM diverges): in FP64 the residual grows past 1e6 times its first value before the
iterates overflow, and the status equals the oracle's (NONFINITE | DIVERGED); in FP32 the first
SCP iteration already overflows, so there is no finite reference and the bit is NONFINITE.  Each case plants one bad trajectory in a batch
of good ones and checks, in both forms and both precisions:
  * the bad trajectory carries its bit;
  * every good trajectory is bit-identical to the same trajectory solved alone, and carries no
    failure bit.
The 6-DOF quadrotor and lander (resident ADMM and plain form) are held to the same containment for the
first three cases.
Spanning consensus groups: a group barrier that gives up (scp_params.group_wait_ms < 0 gives up
at the first wait) flags every member of the group with SCP_ST_SYNC, and a batch whose spanning
groups cannot all be resident at once is refused before any launch.
"""
import math

import numpy as np
import pytest

import oracle
import scpgen

pytestmark = pytest.mark.gpu

FAIL_BITS = 1 | 2 | 4 | 16 | 32


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def B(lib):
    from paper_2603_10711_amd import binding
    return binding


def _good():
    return [scpgen.quad_instance(9, 700 + i, N=12 + 5 * i, K=i % 5) for i in range(4)] + \
           [scpgen.mars_instance(9, 3, N=17)]


def _bad(kind):
    d = scpgen.quad_instance(9, 750, N=20, K=3)
    if kind == "badpivot":      # control Hessian far from positive definite
        d = dict(d, R=np.array([-80.0, 2.0, 2.0]))
        return d, 2
    if kind == "emptyset":      # hard state box with lo > hi on one component
        xlo, xhi = d["x_lo"].copy(), d["x_hi"].copy()
        xlo[4], xhi[4] = 3.0, -3.0
        return dict(d, x_lo=xlo, x_hi=xhi), 4
    if kind == "nan_xinit":     # non-finite initial state
        x0 = d["x_init"].copy()
        x0[1] = math.nan
        return dict(d, x_init=x0), 1
    if kind == "diverge":       # nonconvex QP (negative control weight), H positive definite
        return dict(d, R=np.full(3, -2.0)), None
    raise ValueError(kind)


def _solve(B, insts, prec, form):
    prob = B.Problem(insts, precision=prec)
    prob.solve(B.scp_params(3, 40, form=form, detect_blowup=True))
    x, u, info = (a.cpu().numpy() for a in prob.result())
    offs = prob.offsets.copy()
    prob.close()
    return x, u, info, offs


@pytest.mark.parametrize("kind", ["badpivot", "emptyset", "nan_xinit", "diverge"])
@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("form", ["persistent", "plain"])
def test_failure_is_flagged_and_contained(B, kind, prec, form):
    good = _good()
    bad, bit = _bad(kind)
    pos = 2
    insts = good[:pos] + [bad] + good[pos:]
    _say(kind, prec, form)
    x, u, info, offs = _solve(B, insts, prec, form)
    st = info[:, 5].astype(np.int64)
    if kind == "diverge":
        with np.errstate(all="ignore"):
            _, oinf = oracle.scp_solve([bad], oracle.default_params(scp_iters=3, admm_iters=40, detect_blowup=True))
        assert oinf[0]["status"] == B.ST_NONFINITE | B.ST_DIVERGED
        bit = B.ST_NONFINITE | B.ST_DIVERGED if prec == "f64" else B.ST_NONFINITE
        assert (st[pos] & (B.ST_NONFINITE | B.ST_DIVERGED)) == bit, f"status {st[pos]}, expected {bit}"
    assert st[pos] & bit, f"status {st[pos]} lacks bit {bit}"
    for t, d in enumerate(insts):
        if t == pos:
            continue
        assert (st[t] & FAIL_BITS) == 0, (t, st[t])
        xa, ua, ia, _ = _solve(B, [d], prec, form)
        n = d["N"] + 1
        o = offs[t]
        np.testing.assert_array_equal(xa[:n], x[o:o + n])
        np.testing.assert_array_equal(ua[:n], u[o:o + n])
        np.testing.assert_array_equal(ia[0], info[t])


def _span_batch(S=6, N=40):
    """A 6-scenario group (41 nodes each) between two independent trajectories; in 64-lane
    workgroups it spans six of them."""
    req = scpgen.config4_request(11, S=S, N=N)
    return [scpgen.quad_instance(4, 801, N=20, K=2)] + req + [scpgen.quad_instance(4, 802, N=25, K=4)]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_group_barrier_failure_flags_every_member(B, prec):
    insts = _span_batch()
    pl = B.plan(insts, block=64)
    assert pl["spanning"] == 1
    prob = B.Problem(insts, precision=prec, block=64)
    # group barriers give up at the first wait: the group is flagged, its neighbours are not
    prob.solve(B.scp_params(2, 30, rho=3.0, group_wait_ms=-1.0))
    info = prob.result()[2].cpu().numpy()
    st = info[:, 5].astype(np.int64)
    _say(prec, st)
    members = [t for t, d in enumerate(insts) if d["group"] >= 0]
    assert len(members) == 6
    for t in members:
        assert st[t] & B.ST_SYNC, (t, st[t])
    for t in (0, len(insts) - 1):
        assert (st[t] & B.ST_SYNC) == 0
    # the neighbours are untouched by the failed group: bit-identical to their lone solves
    x, u, _ = (a.cpu().numpy() for a in prob.result())
    for t in (0, len(insts) - 1):
        alone = B.Problem([insts[t]], precision=prec, block=64)
        alone.solve(B.scp_params(2, 30, rho=3.0))
        xa, ua, ia = (a.cpu().numpy() for a in alone.result())
        alone.close()
        o, n = prob.offsets[t], insts[t]["N"] + 1
        np.testing.assert_array_equal(xa[:n], x[o:o + n])
        np.testing.assert_array_equal(ia[0], info[t])
    # the default bound on the same problem: no flag is left over from the failed launch
    prob.reset()
    prob.solve(B.scp_params(2, 30, rho=3.0))
    x2, _, info2 = (a.cpu().numpy() for a in prob.result())
    assert not np.any(info2[:, 5].astype(np.int64) & B.ST_SYNC)
    prob.close()
    if prec == "f32":
        # and it equals the group held by one 256-lane workgroup, bit for bit
        ref = B.Problem(insts, precision=prec, block=256)
        ref.solve(B.scp_params(2, 30, rho=3.0))
        xr, _, ir = (a.cpu().numpy() for a in ref.result())
        ref.close()
        np.testing.assert_array_equal(x2, xr)
        np.testing.assert_array_equal(ir, info2)


def test_spanning_batch_beyond_residency_is_refused(B):
    """Every workgroup of a spanning group must be resident at once; a batch with more
    workgroups than the device keeps resident is refused with SCP_ERR_UNSUPPORTED instead of
    relying on the barrier's time bound."""
    reqs = []
    for g in range(1100):
        for d in scpgen.config4_request(g % 64, S=2, N=63):
            reqs.append(dict(d, group=g))
    pl = B.plan(reqs, block=64)
    _say(pl)
    assert pl["spanning"] == 1100 and pl["n_wg"] >= 2200
    prob = B.Problem(reqs, precision="f32", block=64)
    with pytest.raises(B.ScpError) as e:
        prob.solve(B.scp_params(1, 2))
    assert "resident" in str(e.value)
    prob.solve(B.scp_params(1, 2, form="plain"))   # the plain form has no such limit
    info = prob.result()[2].cpu().numpy()
    assert np.all(np.isfinite(info[:, 1]))
    prob.close()


@pytest.mark.parametrize("form", ["persistent", "plain"])
def test_blowup_detection_leaves_results_unchanged(B, form):
    """Blow-up detection only adds the status bit: on a healthy batch the kernels with the tracking
    (the persistent form's own variant) return the same bits as without it."""
    insts = _good()
    res = []
    for detect in (False, True):
        prob = B.Problem(insts, precision="f32")
        prob.solve(B.scp_params(3, 40, form=form, detect_blowup=detect))
        res.append([a.cpu().numpy() for a in prob.result()])
        prob.close()
    for a, b in zip(*res):
        np.testing.assert_array_equal(a, b)
    assert not np.any(res[1][2][:, 5].astype(np.int64) & B.ST_DIVERGED)


def _good6(model):
    if model == "quad6":
        return [scpgen.quad6_benchmark_instance(i, N=12 + 3 * i) for i in range(4)]
    return [scpgen.lander6_perturbed(i) for i in range(4)]


def _bad6(model, kind):
    d = scpgen.quad6_benchmark_instance(9, N=15) if model == "quad6" else scpgen.lander6_perturbed(9)
    if kind == "badpivot":      # control Hessian far from positive definite
        R = np.full(d["nu"], 2.0)
        R[0] = -80.0
        return dict(d, R=R), 2
    if kind == "emptyset":      # hard state box with lo > hi on one velocity component
        xlo, xhi = d["x_lo"].copy(), d["x_hi"].copy()
        xlo[4], xhi[4] = 3.0, -3.0
        return dict(d, x_lo=xlo, x_hi=xhi), 4
    if kind == "nan_xinit":     # non-finite initial state
        x0 = d["x_init"].copy()
        x0[1] = math.nan
        return dict(d, x_init=x0), 1
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["badpivot", "emptyset", "nan_xinit"])
@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("form", ["persistent", "plain"])
@pytest.mark.parametrize("model", ["quad6", "lander6"])
def test_failure_is_flagged_and_contained_6dof(B, model, kind, prec, form):
    """The same containment on the 6-DOF models: the resident ADMM (one workgroup per
    trajectory) and the plain form flag the bad trajectory and leave its neighbours bit-identical
    to their lone solves."""
    good = _good6(model)
    bad, bit = _bad6(model, kind)
    pos = 1
    insts = good[:pos] + [bad] + good[pos:]
    _say("6dof", model, kind, prec, form)

    def solve(batch):
        prob = B.Problem(batch, precision=prec)
        prob.solve(B.scp_params(3, 30, rho=10.0, form=form, detect_blowup=True))
        x, u, info = (a.cpu().numpy() for a in prob.result())
        offs = prob.offsets.copy()
        prob.close()
        return x, u, info, offs

    x, u, info, offs = solve(insts)
    st = info[:, 5].astype(np.int64)
    assert st[pos] & bit, f"status {st[pos]} lacks bit {bit}"
    for t, d in enumerate(insts):
        if t == pos:
            continue
        assert (st[t] & FAIL_BITS) == 0, (t, st[t])
        xa, ua, ia, _ = solve([d])
        n = d["N"] + 1
        o = offs[t]
        np.testing.assert_array_equal(xa[:n], x[o:o + n])
        np.testing.assert_array_equal(ua[:n], u[o:o + n])
        np.testing.assert_array_equal(ia[0], info[t])

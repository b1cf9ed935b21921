"""Checkpoint and resume through scp_problem_export_state / scp_problem_import_state: a state
exported mid-solve and imported into another handle of the same description continues bit for bit
as the exporting handle does; a state of another layout, or of the wrong size, is refused."""
import numpy as np
import pytest

import scpgen

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def B(lib):
    from paper_2603_10711_amd import binding
    return binding


def _mix():
    out = [scpgen.quad_instance(21, i, N=20 + 9 * i, K=i % 9) for i in range(5)]
    out += [scpgen.mars_instance(21, i, N=30 + 11 * i) for i in range(3)]
    return out


def _arrays(prob):
    return [a.cpu().numpy() for a in prob.result()]


@pytest.mark.parametrize("prec,form", [("f32", "persistent"), ("f64", "plain")])
def test_resume_in_another_handle(B, prec, form):
    insts = _mix()
    _say("checkpoint", prec, form, [d["N"] for d in insts])
    a = B.Problem(insts, precision=prec)
    a.solve(B.scp_params(3, 40, rho=2.0, form=form))
    state = a.export_state()
    a.solve(B.scp_params(2, 40, rho=2.0, form=form))
    want = _arrays(a)
    b = B.Problem(insts, precision=prec)
    b.import_state(state)
    b.solve(B.scp_params(2, 40, rho=2.0, form=form))
    got = _arrays(b)
    for x, y in zip(got, want):
        np.testing.assert_array_equal(x, y)
    # the same handle, reset in between, resumes the same way
    a.reset()
    a.import_state(state)
    a.solve(B.scp_params(2, 40, rho=2.0, form=form))
    for x, y in zip(_arrays(a), want):
        np.testing.assert_array_equal(x, y)
    a.close()
    b.close()


def test_resume_between_admm_calls(B):
    """The host-side state travels too: a handle that imports a state taken after scp_linearize
    may call admm_solve (it needs a current linearization and the same penalties)."""
    insts = _mix()
    a = B.Problem(insts, precision="f64")
    prm = B.admm_params(rho=3.0, iters=15)
    a.linearize(prm)
    a.admm(prm)
    state = a.export_state()
    a.admm(prm)
    want = [a.field(f).cpu().numpy() for f in ("x", "u", "z", "lam", "mu")]
    b = B.Problem(insts, precision="f64")
    with pytest.raises(B.ScpError):
        b.admm(prm)                                   # no linearization yet
    b.import_state(state)
    b.admm(prm)
    got = [b.field(f).cpu().numpy() for f in ("x", "u", "z", "lam", "mu")]
    for x, y in zip(got, want):
        np.testing.assert_array_equal(x, y)
    a.close()
    b.close()


def test_resume_resident_6dof(B):
    insts = [scpgen.quad6_benchmark_instance(i, N=16) for i in range(3)]
    a = B.Problem(insts, precision="f32")
    prm = B.scp_params(2, 30, rho=100.0)
    a.solve(prm)
    state = a.export_state()
    a.solve(prm)
    want = _arrays(a)
    b = B.Problem(insts, precision="f32")
    b.import_state(state)
    b.solve(prm)
    for x, y in zip(_arrays(b), want):
        np.testing.assert_array_equal(x, y)
    a.close()
    b.close()


def test_foreign_states_are_refused(B):
    insts = _mix()
    a = B.Problem(insts, precision="f32")
    state = a.export_state()
    other = B.Problem(insts[:-1], precision="f32")
    with pytest.raises(B.ScpError, match="import_state"):
        other.import_state(np.zeros(state.nbytes, dtype=np.uint8))        # wrong size or layout
    # the same node count with one node moved between two trajectories: refused by size or, where
    # the arenas have equal size, by the layout fingerprint
    moved = [dict(d) for d in insts]
    moved[0] = scpgen.quad_instance(21, 0, N=insts[0]["N"] + 1, K=0)
    moved[1] = scpgen.quad_instance(21, 1, N=insts[1]["N"] - 1, K=1)
    packed = B.Problem(moved, precision="f32")
    _say("moved node: state bytes", packed.export_state().nbytes, "against", state.nbytes)
    with pytest.raises(B.ScpError, match="import_state"):
        packed.import_state(state)
    wide = B.Problem(insts, precision="f64")
    with pytest.raises(B.ScpError, match="import_state"):
        wide.import_state(state)
    bad = state.copy()
    bad[0] ^= 1                                                           # header magic
    with pytest.raises(B.ScpError, match="layout"):
        a.import_state(bad)
    for p in (a, other, packed, wide):
        p.close()


@pytest.mark.parametrize("case", ["spanning_ratio_blowup", "adaptive"])
def test_resume_carries_per_trajectory_state(B, case):
    """The per-trajectory state beyond the iterates travels with a checkpoint: the trust radius of
    the ratio test, the residual blow-up reference and maximum and the spanning groups' layout; a
    solve with the adaptive penalty (whose factor restarts at 1 with every solve) resumes the
    same way."""
    if case == "spanning_ratio_blowup":
        insts = [scpgen.quad_instance(4, 811, N=20, K=2)] + scpgen.config4_request(12, S=6, N=40) + \
                [scpgen.quad_instance(4, 812, N=25, K=4)]
        kw = dict(block=64)
        prm = B.scp_params(2, 30, rho=3.0, eta0=0.0, shrink=0.5, grow=2.0, delta_max=4.0, detect_blowup=True)
    else:
        insts = _mix()
        kw = {}
        prm = B.scp_params(2, 30, rho=1.0, adapt_mu=10.0, adapt_tau=2.0)
    _say("checkpoint", case)
    a = B.Problem(insts, precision="f32", **kw)
    a.solve(prm)
    state = a.export_state()
    a.solve(prm)
    want = _arrays(a)
    b = B.Problem(insts, precision="f32", **kw)
    b.import_state(state)
    b.solve(prm)
    for x, y in zip(_arrays(b), want):
        np.testing.assert_array_equal(x, y)
    a.close()
    b.close()

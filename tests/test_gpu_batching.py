"""Uneven batching on the GPU: mixed models and horizons in one persistent kernel, per-trajectory
convergence masks, hipGraph replay of the SCP launch sequence, and the autotuner.

Parity bar as in the other GPU tests: FP64 mode within 1e-9 of the FP64 oracle at fixed
iteration counts.  Packing (workgroup size, aligned or dense) changes where a trajectory runs,
never its arithmetic, so results of different packings are compared bit for bit.
"""
import numpy as np
import pytest

import scpgen
from _parity import compare, gpu_fields, oracle_scp

pytestmark = pytest.mark.gpu

TOL64 = 1e-9


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def B(lib):
    from paper_2603_10711_amd import binding
    return binding


def _mix(horizons, cfg=3):
    """Alternating quadrotor (8 obstacles, T = 5 s) and powered-descent (tf = 50 s) instances."""
    out = []
    for i, N in enumerate(horizons):
        if i % 2 == 0:
            out.append(scpgen.quad_instance(cfg, 100 + i, N=N, K=8, T=5.0))
        else:
            out.append(scpgen.mars_instance(cfg, 100 + i, N=N, tf=50.0))
    return out


# horizons around the wavefront boundary (63, 64, 65 nodes) and up to the longest of the mix
MIX_N = [20, 63, 62, 64, 65, 33, 90, 120, 120, 41, 27, 100]


@pytest.mark.parametrize("form", ["plain", "persistent"])
def test_uneven_mix_fp64_matches_oracle(B, form):
    insts = _mix(MIX_N)
    _say("uneven mix fp64", form, [d["N"] for d in insts])
    prob = B.Problem(insts, precision="f64")
    prob.solve(B.scp_params(2, 30, form=form))
    f = gpu_fields(prob)
    trajs, _ = oracle_scp(insts, 2, 30)
    worst = compare(prob, f, insts, trajs)
    _say(worst)
    assert max(worst.values()) < TOL64
    prob.close()


def test_packings_are_bitwise_equal(B):
    """FP32, same batch under every workgroup size and packing: identical results and info."""
    insts = _mix(MIX_N + [30, 31, 45, 18, 64, 22])
    ref = None
    for block, pack in [(128, 0), (128, 1), (256, 0), (256, 1)]:
        pl = B.plan(insts, block=block, pack=pack)
        _say("packing", block, pack, pl)
        prob = B.Problem(insts, precision="f32", block=block, pack=pack)
        prob.solve(B.scp_params(3, 40, check_every=5, eps=1e-4))
        out = [a.cpu().numpy() for a in prob.result()]
        if ref is None:
            ref = out
        else:
            for a, b in zip(out, ref):
                np.testing.assert_array_equal(a, b)
        prob.close()
    # short trajectories only: 64-lane workgroups (wavefront exchange) against 256-lane ones
    short = _mix([20, 40, 63, 31, 50, 25])
    res = []
    for block, pack in [(64, 0), (256, 0), (256, 1)]:
        prob = B.Problem(short, precision="f32", block=block, pack=pack)
        prob.solve(B.scp_params(3, 40))
        res.append([a.cpu().numpy() for a in prob.result()])
        prob.close()
    for r in res[1:]:
        for a, b in zip(r, res[0]):
            np.testing.assert_array_equal(a, b)


def test_convergence_masks_on_the_mix(B):
    """Residual test every 5 iterations at 1e-4: the short quadrotors stop on their own, with the
    oracle's iteration counts, inside the workgroup of a 71-node trajectory that runs the whole
    budget (and beside a 67-node powered descent that does too)."""
    insts = [scpgen.quad_instance(3, i, N=15 + i, K=2, T=5.0, delta=5.0) for i in range(3)]
    insts += [scpgen.quad_instance(3, 1, N=70, K=2, T=5.0, delta=5.0), scpgen.mars_instance(3, 5, N=66)]
    kw = dict(check_every=5, eps_p=1e-4, eps_d=1e-4, rho_eq=3.0, rho_dyn=3.0, rho_geo=3.0)
    trajs, oinfo = oracle_scp(insts, 3, 600, **kw)
    iters = [o["admm_iters"] for o in oinfo]
    _say("oracle iterations", iters)
    assert len(set(iters[:3])) == 3 and max(iters[:3]) < 1800 and iters[3:] == [1800, 1800]
    pl = B.plan(insts, block=128, lanes=True)
    assert pl["n_wg"] == 2                          # the short quadrotors ride with the long one
    for form in ["plain", "persistent"]:
        prob = B.Problem(insts, precision="f64", block=128)
        prob.solve(B.scp_params(3, 600, check_every=5, eps=1e-4, rho=3.0, form=form))
        f = gpu_fields(prob)
        _, _, info = prob.result()
        inf = prob.info_dicts(info.cpu().numpy())
        _say(form, [i["admm_iters"] for i in inf])
        assert [i["admm_iters"] for i in inf] == iters
        worst = compare(prob, f, insts, trajs)
        _say(worst)
        assert max(worst.values()) < TOL64
        prob.close()


@pytest.mark.parametrize("form", ["persistent", "plain"])
def test_graph_replay_equals_direct_launches(B, form):
    import torch
    insts = _mix([20, 63, 90, 41])
    s = torch.cuda.Stream()
    direct = B.Problem(insts, precision="f32", stream=s)
    direct.solve(B.scp_params(3, 25, check_every=5, eps=1e-4, form=form, scp_per_launch=1))
    ref = [a.cpu().numpy() for a in direct.result()]
    direct.close()
    g = B.Problem(insts, precision="f32", stream=s)
    for rep in range(3):
        g.reset()
        g.solve(B.scp_params(3, 25, check_every=5, eps=1e-4, form=form, scp_per_launch=1, graph=True))
        out = [a.cpu().numpy() for a in g.result()]
        _say("graph replay", form, rep)
        for a, b in zip(out, ref):
            np.testing.assert_array_equal(a, b)
    g.close()


def test_autotune_small_mix(B):
    insts = _mix([20, 63, 90, 41, 120, 33, 70, 64])
    prm = B.scp_params(2, 40, check_every=5, eps=1e-4)
    best, table = B.autotune(insts, prm, cadences=(1, 5), reps=1)
    _say(best, table)
    assert len(table) == 6 * 2
    one = [e for e in table if e["lanes_per_node"] == 1]
    assert len(one) == 5 * 2
    assert not any(e["valid"] for e in one if e["block"] == 64)       # 121 nodes need 128 lanes
    # lane groups of four: trajectories over 64 nodes and a residual-test cadence rule them out
    four = [e for e in table if e["lanes_per_node"] == 4]
    assert len(four) == 2 and not any(e["valid"] for e in four)
    valid = [e for e in table if e["valid"]]
    assert len(valid) == 8 and best["valid"]
    assert best["ms"] == min(e["ms"] for e in valid)
    best2, table2 = B.autotune(insts, prm, cadences=(1, 5), reps=1)
    assert table2 == [] and best2 == best                             # cached

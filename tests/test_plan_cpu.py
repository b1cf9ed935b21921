"""Host-side packing of trajectories into persistent-kernel workgroups (no GPU needed).

The plan must place every node of every trajectory exactly once, keep each trajectory (and each
consensus group) contiguous inside one workgroup, and, in aligned mode, never let a trajectory of
at most 64 nodes straddle a wavefront.  Workgroups flagged for the LDS exchange are exactly the
ones in which some trajectory straddles a wavefront (for batches with consensus groups: at least
those; a group placed whole is one unit, and a workgroup whose unit straddles takes the exchange
too).  Random batches (hypothesis) check the invariants over many shapes.
"""
import numpy as np
import pytest

import scpgen


@pytest.fixture(scope="module")
def B():
    from paper_2603_10711_amd import binding
    try:
        binding.load()
    except RuntimeError as e:
        pytest.skip(str(e))
    return binding


def _check_plan(insts, pl):
    block, n_wg, lanes = pl["block"], pl["n_wg"], pl["lanes"]
    assert lanes.shape == (n_wg, block)
    offs = np.cumsum([0] + [d["N"] + 1 for d in insts])
    nodes = lanes[lanes >= 0]
    assert np.array_equal(np.sort(nodes), np.arange(offs[-1]))          # every node exactly once
    assert pl["idle"] == n_wg * block - offs[-1]
    straddle = np.zeros(n_wg, dtype=bool)
    where = {int(g): (w, l) for w in range(n_wg) for l, g in enumerate(lanes[w]) if g >= 0}
    for t, d in enumerate(insts):
        w0, l0 = where[int(offs[t])]
        for i in range(d["N"] + 1):
            assert where[int(offs[t] + i)] == (w0, l0 + i)                 # contiguous, one workgroup
        if l0 // 64 != (l0 + d["N"]) // 64:
            straddle[w0] = True
    return straddle


@pytest.mark.parametrize("block", [128, 256])
@pytest.mark.parametrize("pack", [0, 1])
def test_uneven_mix_plan_invariants(B, block, pack):
    insts = scpgen.config3(300)
    pl = B.plan(insts, block=block, pack=pack, lanes=True)
    assert pl["block"] == block
    straddle = _check_plan(insts, pl)
    assert pl["lds_wg"] == int(straddle.sum())
    if pack == 0:
        offs = np.cumsum([0] + [d["N"] + 1 for d in insts])
        for t, d in enumerate(insts):
            if d["N"] + 1 <= 64:
                w = np.argwhere(pl["lanes"] == offs[t])[0]
                assert w[1] // 64 == (w[1] + d["N"]) // 64
    # one model per workgroup
    model = np.repeat([d["model"] for d in insts], [d["N"] + 1 for d in insts])
    for w in range(pl["n_wg"]):
        row = pl["lanes"][w]
        assert len(set(model[row[row >= 0]])) == 1


def test_short_trajectories_alone_use_wavefront_exchange(B):
    """Trajectories of at most 64 nodes, aligned packing: no workgroup needs the LDS exchange even
    at 256 lanes; dense packing of the same batch does straddle."""
    insts = [scpgen.quad_instance(1, i, N=20 + (i * 13) % 40, K=2) for i in range(40)]
    al = B.plan(insts, block=256, pack=0, lanes=True)
    _check_plan(insts, al)
    assert al["lds_wg"] == 0
    de = B.plan(insts, block=256, pack=1, lanes=True)
    _check_plan(insts, de)
    assert de["lds_wg"] > 0 and de["idle"] <= al["idle"]


def test_groups_stay_whole_and_auto_block(B):
    reqs = scpgen.config4_request(0, S=3, N=30) + scpgen.config4_request(1, S=2, N=50)
    pl = B.plan(reqs, lanes=True)
    assert pl["block"] == 128                       # a 3 x 31 group needs more than one wavefront
    _check_plan(reqs, pl)
    lanes = pl["lanes"]
    w0 = np.argwhere(lanes == 0)[0][0]
    assert set(range(93)) <= set(lanes[w0][lanes[w0] >= 0].tolist())
    assert B.plan(scpgen.config1(64))["block"] == 64
    too_long = [scpgen.quad_instance(0, 0, N=300, K=1)]
    assert B.plan(too_long)["block"] == 0           # persistent form unavailable


def test_autotune_arena_covers_every_candidate(B):
    from ctypes import byref
    lib = B.load()
    insts = scpgen.config3(64)
    d, keep = B.make_desc(insts)
    auto = lib.scp_autotune_device_bytes(byref(d))
    for blk in (64, 128, 256):
        for pk in (0, 1):
            d2, keep2 = B.make_desc(insts, 0, blk, pk)
            assert lib.scp_problem_device_bytes(byref(d2)) <= auto


@pytest.mark.parametrize("N", [30, 50, 64, 80])
@pytest.mark.parametrize("block,pack", [(128, 0), (256, 0), (256, 1)])
def test_scenario_request_spans_workgroups(B, N, block, pack):
    """A 16-scenario request is larger than one workgroup: its members go to workgroups of their
    own (one spanning group), each member whole in one workgroup."""
    req = scpgen.config4_request(0, S=16, N=N)
    other = [scpgen.quad_instance(4, 900 + i, N=20 + i, K=4) for i in range(5)]
    insts = other[:2] + req + other[2:]
    pl = B.plan(insts, block=block, pack=pack, lanes=True)
    assert pl["block"] == block and pl["spanning"] == 1
    _check_plan(insts, pl)
    lanes = pl["lanes"]
    off = sum(d["N"] + 1 for d in other[:2])
    span_nodes = set(range(off, off + 16 * (N + 1)))
    for w in range(pl["n_wg"]):
        row = set(lanes[w][lanes[w] >= 0].tolist())
        assert row <= span_nodes or not (row & span_nodes)        # spanning workgroups hold nothing else


def test_spanning_limits(B):
    too_many = scpgen.with_scenarios(scpgen.quad_instance(4, 1, N=10, K=2), 65, np.random.default_rng(0), group=3)
    assert B.plan(too_many)["block"] == 0          # more than 64 members: persistent form unavailable
    assert B.plan(too_many[:64])["spanning"] in (0, 1)


# ---- randomized batches (hypothesis): the packing invariants over many shapes ----

from hypothesis import given, settings, strategies as st   # noqa: E402

_INST_CACHE = {}


def _inst(model, N):
    key = (model, N)
    if key not in _INST_CACHE:
        _INST_CACHE[key] = (scpgen.quad_instance(7, N, N=N, K=N % 9) if model == scpgen.QUAD
                            else scpgen.mars_instance(7, N, N=N))
    return _INST_CACHE[key]


_unit = st.one_of(
    st.tuples(st.just(1), st.sampled_from([scpgen.QUAD, scpgen.MARS]), st.integers(1, 255)),
    st.tuples(st.integers(2, 24), st.sampled_from([scpgen.QUAD, scpgen.MARS]), st.integers(1, 80)),
)


@settings(max_examples=300, deadline=None)
@given(units=st.lists(_unit, min_size=1, max_size=12), block=st.sampled_from([0, 64, 128, 256]),
       pack=st.sampled_from([0, 1]))
def test_random_batches_pack_correctly(B, units, block, pack):
    """Random mixes of single trajectories (N up to 255) and consensus groups (2-24 members of
    one model and horizon) of both models, every workgroup size and both packings: a batch the
    persistent form can hold is packed with every node once, each trajectory contiguous in one
    workgroup, one model per workgroup, groups whole in one workgroup when they fit it and spread
    over workgroups of their own otherwise; a batch it cannot hold gets no plan."""
    insts, groups = [], []
    for gid, (S, model, N) in enumerate(units):
        d = _inst(model, N)
        if S == 1:
            insts.append(dict(d, group=-1))
        else:
            groups.append((len(insts), S, N + 1))
            insts.extend(dict(d, group=gid) for _ in range(S))
    pl = B.plan(insts, block=block, pack=pack, lanes=True)
    longest = max(N + 1 for _, _, N in units)
    # every trajectory, group members included, must fit one workgroup; groups of at most 64
    # members may span workgroups; nothing else makes a batch of these models unplannable
    if pl["block"] == 0:
        assert longest > (block or 256), (units, block, pack)
        return
    assert longest <= pl["block"]
    if block:
        assert pl["block"] == block
    b = pl["block"]
    straddle = _check_plan(insts, pl)
    # a workgroup in which a trajectory straddles a wavefront boundary must take the LDS exchange;
    # one that holds a straddling group unit takes it as well, even where its members do not
    assert pl["lds_wg"] >= int(straddle.sum())
    if not groups:
        assert pl["lds_wg"] == int(straddle.sum())
    lanes = pl["lanes"]
    model = np.repeat([d["model"] for d in insts], [d["N"] + 1 for d in insts])
    wg_of = np.full(len(model), -1)
    for w in range(pl["n_wg"]):
        row = lanes[w][lanes[w] >= 0]
        assert len(set(model[row])) == 1                                   # one model per workgroup
        wg_of[row] = w
    offs = np.cumsum([0] + [d["N"] + 1 for d in insts])
    n_span = 0
    unit_lanes = np.array([d["N"] + 1 for d in insts])   # lanes of the unit a trajectory is placed in
    for first, S, L in groups:
        nodes = np.arange(offs[first], offs[first + S])
        wgs = set(wg_of[nodes].tolist())
        if S * L <= b:
            assert len(wgs) == 1                                           # whole in one workgroup
            unit_lanes[first:first + S] = S * L
        else:
            n_span += 1                                                    # members placed one by one
            for w in wgs:                                                  # in workgroups of its own
                row = lanes[w][lanes[w] >= 0]
                assert np.all((row >= offs[first]) & (row < offs[first + S]))
    assert pl["spanning"] == n_span
    if pack == 0:
        # aligned packing: a unit of at most 64 lanes never straddles a wavefront boundary
        for t in range(len(insts)):
            if unit_lanes[t] <= 64:
                w = np.argwhere(lanes == offs[t])[0]
                assert w[1] // 64 == (w[1] + insts[t]["N"]) // 64

"""scp_problem_create_noalloc against scp_problem_create, through the C ABI.

The no-allocation entry point lays the problem out in the library's fixed device arena instead of
caller memory; everything after create runs the same kernels on the same layout, so results must
be bit-identical to the caller-arena path.  Two calls in a row, the second with a smaller input
(the arena keeps the first call's contents, which create must clear), then the size limit and the
one-handle-per-device rule.
"""
import numpy as np
import pytest

import scpgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B(lib):
    from paper_2603_10711_amd import binding
    return binding


def _run(B, insts, prec, prm, noalloc):
    prob = B.Problem(insts, precision=prec, noalloc=noalloc)
    prob.solve(prm)
    out = [a.cpu().numpy() for a in prob.result()]
    out += [prob.field(k).cpu().numpy() for k in ("z", "lam", "mu", "copy", "dual")]
    prob.close()
    return out


def _first():
    insts = [scpgen.quad_instance(12, i, N=20 + 9 * i, K=(3 * i) % 9) for i in range(6)]
    return insts + [scpgen.mars_instance(12, i, N=30 + 7 * i) for i in range(2)]


def _second():
    return [scpgen.quad_instance(13, 0, N=11, K=2), scpgen.mars_instance(13, 1, N=9)]


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_noalloc_equals_caller_arena_two_calls(B, prec):
    prm = B.scp_params(3, 60, rho=2.0, check_every=10, eps=1e-6)
    for insts, form in ((_first(), "persistent"), (_second(), "plain")):
        p = B.scp_params(3, 60, rho=2.0, check_every=10, eps=1e-6, form=form)
        print(prec, form, len(insts), flush=True)
        ref = _run(B, insts, prec, p, noalloc=False)
        got = _run(B, insts, prec, p, noalloc=True)
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, b)
    # the smaller problem again, persistent form, after the larger one left its contents behind
    ref = _run(B, _second(), prec, prm, noalloc=False)
    got = _run(B, _second(), prec, prm, noalloc=True)
    for a, b in zip(got, ref):
        np.testing.assert_array_equal(a, b)


def test_noalloc_limits(B):
    lib = B.load()
    big = scpgen.config2(256)          # about 40 MB of arena in FP32: over the fixed size
    desc, keep = B.make_desc(big, B.F32)
    need = lib.scp_problem_device_bytes(desc)
    assert need > B.NOALLOC_MAX_BYTES
    with pytest.raises(B.ScpError) as e:
        B.Problem(big, precision="f32", noalloc=True)
    assert "no-allocation arena" in str(e.value)
    # one live handle per device
    a = B.Problem(_second(), precision="f32", noalloc=True)
    with pytest.raises(B.ScpError) as e:
        B.Problem(_second(), precision="f32", noalloc=True)
    assert "held by another" in str(e.value)
    a.close()
    b = B.Problem(_second(), precision="f32", noalloc=True)   # released by destroy
    b.close()

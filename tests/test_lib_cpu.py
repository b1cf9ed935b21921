"""CPU checks of the C-ABI library: it loads, exports every symbol the header declares, and its
host-side validation rejects bad descriptions without touching a GPU."""
import ctypes
import os
import re
from ctypes import POINTER, byref, c_double, c_int32, c_void_p

import numpy as np
import pytest

import scpgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def B():
    from paper_2603_10711_amd import binding
    binding.load()
    return binding


def _header_functions(name="scp.h"):
    txt = open(os.path.join(ROOT, "include", name)).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_]+)\s*\([^;{]*\)\s*;", txt)) - {"sizeof"})


def test_library_exports_every_declared_symbol(B):
    names = _header_functions()
    assert len(names) >= 12
    lib = B.load()
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(B.SYMBOLS) == names
    serve = _header_functions("scp_serve.h")
    for n in serve:
        assert hasattr(lib, n), n
    assert sorted(B.SERVE_SYMBOLS) == serve
    headers = sorted(f for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h"))
    assert headers == ["scp.h", "scp_serve.h"]


def test_noalloc_arena_size_matches_header(B):
    txt = open(os.path.join(ROOT, "include", "scp.h")).read()
    m = re.search(r"#define SCP_NOALLOC_MAX_BYTES \((\d+)u << (\d+)\)", txt)
    assert m and int(m.group(1)) << int(m.group(2)) == B.NOALLOC_MAX_BYTES


def test_numerical_failures_are_not_call_errors(B):
    """Non-SPD cost, lo > hi and a NaN initial state are per-trajectory status bits on the device,
    not description errors: the host accepts them."""
    lib = B.load()
    insts = scpgen.config1(3)
    insts[0] = dict(insts[0], R=np.array([-80.0, 2.0, 2.0]))
    xlo, xhi = insts[1]["x_lo"].copy(), insts[1]["x_hi"].copy()
    xlo[4], xhi[4] = 3.0, -3.0
    insts[1] = dict(insts[1], x_lo=xlo, x_hi=xhi)
    x0 = insts[2]["x_init"].copy()
    x0[1] = float("nan")
    insts[2] = dict(insts[2], x_init=x0)
    d, keep = _desc(B, insts)
    assert lib.scp_problem_device_bytes(byref(d)) > 0


def test_server_config_validation(B):
    lib = B.load()
    prm = B.scp_params(10, 100)
    good = B.ServerConfig(0, 256, 0, 1 << 14, 256, 256, 32, 32, 0, prm, 1, 2)
    assert lib.scp_server_device_bytes(byref(good)) > (1 << 14) * 350 * 4
    bad = [dict(block=96), dict(prec=1, block=256), dict(scp_per_step=3), dict(max_nodes=0), dict(max_inflight=0),
           dict(adapt_mu=10.0), dict(rho_final=1e3)]
    for kw in bad:
        c = B.ServerConfig(0, 256, 0, 1 << 14, 256, 256, 32, 32, 0, prm, 1, 2)
        for k, v in kw.items():
            setattr(c.solve if k in ("adapt_mu", "rho_final") else c, k, v)
        assert lib.scp_server_device_bytes(byref(c)) == 0, kw
        h = c_void_p()
        assert lib.scp_server_create(byref(c), None, 0, None, byref(h)) == 1 and not h.value
        assert len(lib.scp_server_last_error(None)) > 0


def _desc(B, insts, prec=0, block=0, group=None, pack=0):
    if group is not None:
        insts = [dict(d, group=g) for d, g in zip(insts, group)]
    return B.make_desc(insts, prec, block, pack)


def test_device_bytes_and_field_widths(B):
    lib = B.load()
    d, keep = _desc(B, scpgen.config1(8))
    n32 = lib.scp_problem_device_bytes(byref(d))
    d64, keep2 = _desc(B, scpgen.config1(8), prec=1)
    n64 = lib.scp_problem_device_bytes(byref(d64))
    assert n32 > 0 and n64 > 1.9 * n32 * 0.9
    assert [lib.scp_field_width(i) for i in range(16)] == [14, 4, 14, 4, 14, 14, 14, 14, 44, 44, 196, 56, 14, 18, 18, 32]
    assert lib.scp_field_width(99) == 0


@pytest.mark.parametrize("case", ["model", "horizon", "obstacles", "block", "pack", "group_gap", "group_shape",
                                  "delta"])
def test_invalid_descriptions_rejected_on_host(B, case):
    lib = B.load()
    insts = scpgen.config1(3)
    group = None
    block = 0
    pack = 0
    if case == "model":
        insts[1] = dict(insts[1], model=9)
    elif case == "horizon":
        insts[2] = dict(insts[2], N=0)
    elif case == "obstacles":
        insts[0] = dict(insts[0], obstacles=np.zeros((9, 4)))
    elif case == "block":
        block = 96
    elif case == "pack":
        pack = 2
    elif case == "group_gap":
        group = [5, -1, 5]
    elif case == "group_shape":
        insts[1] = dict(scpgen.quad_instance(1, 1, N=20), group=4)
        insts[0] = dict(insts[0], group=4)
        group = [4, 4, -1]
    elif case == "delta":
        insts[0] = dict(insts[0], delta=0.0)
    if case == "horizon":
        insts[2]["x_guess"] = insts[2]["x_guess"][:1]
        insts[2]["u_guess"] = insts[2]["u_guess"][:0]
    d, keep = _desc(B, insts, block=block, group=group, pack=pack)
    assert lib.scp_problem_device_bytes(byref(d)) == 0
    h = c_void_p()
    st = lib.scp_problem_create(byref(d), None, 0, None, byref(h))
    assert st == 1 and not h.value
    assert len(lib.scp_last_error(None)) > 0


def test_arena_too_small_is_rejected(B):
    lib = B.load()
    d, keep = _desc(B, scpgen.config1(2))
    h = c_void_p()
    st = lib.scp_problem_create(byref(d), c_void_p(256), 512, None, byref(h))
    assert st == 1 and b"too small" in lib.scp_last_error(None)


def test_null_handles_are_safe(B):
    lib = B.load()
    assert lib.scp_linearize(None, None) == 1
    assert lib.admm_solve(None, None) == 1
    assert lib.scp_solve(None, None) == 1
    assert lib.scp_problem_nodes(None) == 0
    lib.scp_problem_destroy(None)

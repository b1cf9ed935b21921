"""ctypes binding of libscp.so (the C ABI in include/scp.h).

Argument marshalling only: problem dictionaries (as produced by ``scpgen``) are packed into
the C parameter records, device memory comes from PyTorch (one uint8 tensor per problem, the
"arena"), and every computation runs in the HIP kernels of the library.  There is no CPU
fallback: if the library is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import math
import os
from ctypes import POINTER, byref, c_double, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libscp.so")

# --- constants mirrored from include/scp.h ------------------------------------------------
SCP_OK = 0
QUAD, MARS, QUAD6, LANDER6 = 1, 2, 3, 4
F32, F64 = 0, 1
FORM_PLAIN, FORM_PERSISTENT = 0, 1
PACK_ALIGNED, PACK_DENSE = 0, 1
MAX_NX, MAX_NU, MAX_OBS = 14, 4, 8
P = dict(H=0, XINIT=1, XTGT=15, TMASK=29, QR=43, QN=57, QNV=71, CN=85, R=86, XLO=90, XHI=104, ULO=118, UHI=122,
         UBALL=126, DELTA=127, DRAG=128, MSCALE=129, GRAV=130, ALPHA=131, GVEC=132, GLIDE=135, NOBS=136, OBS=137,
         DIST=169, CYL=172, INERTIA=173, ARM=176, TMIN=179, TMAX=180, GIMBAL=181, TILT=182, WMAX=183)
PARAM_STRIDE = 184
SUBMIT_MEASURED = 1
INFO = dict(admm_iters=0, r_p=1, r_d=2, n_accept=3, delta=4, status=5, defect=6, cost=7, viol=8, bnd_err=9,
            merit=10, ratio=11)
INFO_FIELDS = 12
ST_NONFINITE, ST_BADPIVOT, ST_EMPTYSET, ST_CONVERGED, ST_SYNC, ST_DIVERGED = 1, 2, 4, 8, 16, 32
FIELDS = dict(xbar=0, ubar=1, x=2, u=3, z=4, lam=5, mu=6, ddyn=7, copy=8, dual=9, A=10, B=11, d=12, boxlo=13,
              boxhi=14, hs=15)
SYMBOLS = ["scp_problem_device_bytes", "scp_problem_create", "scp_problem_create_noalloc", "scp_problem_destroy",
           "scp_linearize", "admm_solve",
           "scp_solve", "scp_reset", "scp_get_result", "scp_field_width", "scp_get_field", "scp_problem_nodes",
           "scp_traj_node_offset", "scp_plan", "scp_autotune_device_bytes", "scp_autotune", "scp_last_error",
           "scp_problem_state_bytes", "scp_problem_export_state", "scp_problem_import_state"]
SERVE_SYMBOLS = ["scp_server_device_bytes", "scp_server_create", "scp_server_destroy", "scp_server_request_bytes",
                 "scp_server_submit", "scp_server_submit_ex", "scp_server_step", "scp_server_collect",
                 "scp_server_cancel", "scp_server_take_done", "scp_server_get_stats", "scp_server_last_error"]
REQ_UNKNOWN, REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_CANCELLED, REQ_TIMEOUT = 0, 1, 2, 3, 4, 5
NOALLOC_MAX_BYTES = 32 << 20   # SCP_NOALLOC_MAX_BYTES of scp.h


class ProblemDesc(ctypes.Structure):
    _fields_ = [("n_traj", c_int32), ("prec", c_int32), ("model", POINTER(c_int32)), ("horizon", POINTER(c_int32)),
                ("group", POINTER(c_int32)), ("params", POINTER(c_double)), ("x_guess", POINTER(c_double)),
                ("u_guess", POINTER(c_double)), ("block", c_int32), ("pack", c_int32)]


class AdmmParams(ctypes.Structure):
    _fields_ = [("rho_eq", c_double), ("rho_dyn", c_double), ("rho_geo", c_double), ("max_iters", c_int32),
                ("check_every", c_int32), ("eps_prim", c_double), ("eps_dual", c_double)]


class ScpParams(ctypes.Structure):
    _fields_ = [("scp_iters", c_int32), ("admm", AdmmParams), ("eta0", c_double), ("eta1", c_double),
                ("eta2", c_double), ("shrink", c_double), ("grow", c_double), ("delta_max", c_double),
                ("merit_w", c_double), ("form", c_int32), ("scp_per_launch", c_int32), ("rho_final", c_double),
                ("graph", c_int32), ("adapt_mu", c_double), ("adapt_tau", c_double), ("group_wait_ms", c_double),
                ("lanes_per_node", c_int32), ("detect_blowup", c_int32)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("block", c_int32), ("pack", c_int32), ("check_every", c_int32), ("valid", c_int32),
                ("ms", c_double), ("lanes", c_int32)]

    def as_dict(self) -> dict:
        return dict(lanes_per_node=self.lanes, block=self.block, pack="dense" if self.pack == PACK_DENSE else "aligned",
                    check_every=self.check_every, valid=bool(self.valid), ms=self.ms)


class ServerConfig(ctypes.Structure):
    _fields_ = [("prec", c_int32), ("block", c_int32), ("pack", c_int32), ("max_nodes", c_int64),
                ("max_traj", c_int32), ("max_wg", c_int32), ("max_span", c_int32), ("max_requests", c_int32),
                ("budget_bytes", c_size_t), ("solve", ScpParams), ("scp_per_step", c_int32),
                ("max_inflight", c_int32), ("timeout_ms", c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", c_int64), ("completed", c_int64), ("rejected", c_int64), ("queued", c_int32),
                ("running", c_int32), ("resident", c_int32), ("steps", c_int64), ("evictions", c_int64),
                ("warm_starts", c_int64), ("resident_bytes", c_size_t), ("peak_resident_bytes", c_size_t),
                ("cancelled", c_int64), ("timed_out", c_int64), ("latency_ms_p50", c_double),
                ("latency_ms_p99", c_double), ("solves_per_s", c_double), ("latency_ms_p999", c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_LIB = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libscp.so and declare its signatures.  Raises if the library is missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing (run paper_2603_10711_amd.build)")
    lib = ctypes.CDLL(path)
    lib.scp_problem_device_bytes.argtypes = [POINTER(ProblemDesc)]
    lib.scp_problem_device_bytes.restype = c_size_t
    lib.scp_problem_create.argtypes = [POINTER(ProblemDesc), c_void_p, c_size_t, c_void_p, POINTER(c_void_p)]
    lib.scp_problem_create.restype = c_int32
    lib.scp_problem_create_noalloc.argtypes = [POINTER(ProblemDesc), c_void_p, POINTER(c_void_p)]
    lib.scp_problem_create_noalloc.restype = c_int32
    lib.scp_problem_destroy.argtypes = [c_void_p]
    lib.scp_problem_destroy.restype = None
    lib.scp_linearize.argtypes = [c_void_p, POINTER(AdmmParams)]
    lib.scp_linearize.restype = c_int32
    lib.admm_solve.argtypes = [c_void_p, POINTER(AdmmParams)]
    lib.admm_solve.restype = c_int32
    lib.scp_solve.argtypes = [c_void_p, POINTER(ScpParams)]
    lib.scp_solve.restype = c_int32
    lib.scp_reset.argtypes = [c_void_p]
    lib.scp_reset.restype = c_int32
    lib.scp_get_result.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
    lib.scp_get_result.restype = c_int32
    lib.scp_problem_state_bytes.argtypes = [c_void_p]
    lib.scp_problem_state_bytes.restype = c_size_t
    lib.scp_problem_export_state.argtypes = [c_void_p, c_void_p, c_size_t]
    lib.scp_problem_export_state.restype = c_int32
    lib.scp_problem_import_state.argtypes = [c_void_p, c_void_p, c_size_t]
    lib.scp_problem_import_state.restype = c_int32
    lib.scp_field_width.argtypes = [c_int32]
    lib.scp_field_width.restype = c_int32
    lib.scp_get_field.argtypes = [c_void_p, c_int32, c_void_p]
    lib.scp_get_field.restype = c_int32
    lib.scp_problem_nodes.argtypes = [c_void_p]
    lib.scp_problem_nodes.restype = c_int64
    lib.scp_traj_node_offset.argtypes = [c_void_p, c_int32]
    lib.scp_traj_node_offset.restype = c_int64
    lib.scp_plan.argtypes = [POINTER(ProblemDesc), POINTER(c_int32), POINTER(c_int32), c_size_t]
    lib.scp_plan.restype = c_int32
    lib.scp_autotune_device_bytes.argtypes = [POINTER(ProblemDesc)]
    lib.scp_autotune_device_bytes.restype = c_size_t
    lib.scp_autotune.argtypes = [POINTER(ProblemDesc), POINTER(ScpParams), POINTER(c_int32), c_int32, c_int32,
                                 c_void_p, c_size_t, c_void_p, POINTER(TuneEntry), c_int32, POINTER(c_int32),
                                 POINTER(TuneEntry)]
    lib.scp_autotune.restype = c_int32
    lib.scp_last_error.argtypes = [c_void_p]
    lib.scp_last_error.restype = ctypes.c_char_p
    lib.scp_server_device_bytes.argtypes = [POINTER(ServerConfig)]
    lib.scp_server_device_bytes.restype = c_size_t
    lib.scp_server_create.argtypes = [POINTER(ServerConfig), c_void_p, c_size_t, c_void_p, POINTER(c_void_p)]
    lib.scp_server_create.restype = c_int32
    lib.scp_server_destroy.argtypes = [c_void_p]
    lib.scp_server_destroy.restype = None
    lib.scp_server_request_bytes.argtypes = [c_void_p, POINTER(ProblemDesc)]
    lib.scp_server_request_bytes.restype = c_size_t
    lib.scp_server_submit.argtypes = [c_void_p, POINTER(ProblemDesc), c_int32, POINTER(c_int64)]
    lib.scp_server_submit.restype = c_int32
    lib.scp_server_submit_ex.argtypes = [c_void_p, POINTER(ProblemDesc), c_int32, ctypes.c_uint32, POINTER(c_int64)]
    lib.scp_server_submit_ex.restype = c_int32
    lib.scp_server_step.argtypes = [c_void_p, c_int32, POINTER(c_int32)]
    lib.scp_server_step.restype = c_int32
    lib.scp_server_collect.argtypes = [c_void_p, c_int64, c_int32, POINTER(c_int32), POINTER(c_double),
                                       POINTER(c_double), POINTER(c_double), POINTER(c_double)]
    lib.scp_server_collect.restype = c_int32
    lib.scp_server_cancel.argtypes = [c_void_p, c_int64]
    lib.scp_server_cancel.restype = c_int32
    lib.scp_server_take_done.argtypes = [c_void_p, POINTER(c_int64), c_int32, POINTER(c_int32)]
    lib.scp_server_take_done.restype = c_int32
    lib.scp_server_get_stats.argtypes = [c_void_p, POINTER(ServerStats)]
    lib.scp_server_get_stats.restype = c_int32
    lib.scp_server_last_error.argtypes = [c_void_p]
    lib.scp_server_last_error.restype = ctypes.c_char_p
    _LIB = lib
    return lib


def param_record(inst: dict) -> np.ndarray:
    """Pack one problem dictionary into the SCP_PARAM_STRIDE-double C record."""
    r = np.zeros(PARAM_STRIDE)
    nx, nu = inst["nx"], inst["nu"]
    r[P["H"]] = inst["h"]
    r[P["XINIT"]:P["XINIT"] + nx] = inst["x_init"]
    r[P["XTGT"]:P["XTGT"] + nx] = inst["x_target"]
    r[P["TMASK"]:P["TMASK"] + nx] = np.asarray(inst["t_mask"], dtype=float)
    r[P["QR"]:P["QR"] + nx] = inst["Qr"]
    r[P["QN"]:P["QN"] + nx] = inst["Qn"]
    r[P["QNV"]:P["QNV"] + nx] = inst["qn"]
    r[P["CN"]] = inst["cN"]
    r[P["R"]:P["R"] + nu] = inst["R"]
    r[P["XLO"]:P["XLO"] + nx] = inst["x_lo"]
    r[P["XHI"]:P["XHI"] + nx] = inst["x_hi"]
    r[P["ULO"]:P["ULO"] + nu] = inst["u_lo"]
    r[P["UHI"]:P["UHI"] + nu] = inst["u_hi"]
    r[P["UBALL"]] = inst["u_ball"]
    r[P["DELTA"]] = inst["delta"]
    r[P["DRAG"]] = inst["drag"]
    r[P["MSCALE"]] = inst["mscale"]
    r[P["GRAV"]] = inst["grav"]
    r[P["ALPHA"]] = inst["alpha"]
    r[P["GVEC"]:P["GVEC"] + 3] = inst["gvec"]
    r[P["GLIDE"]] = inst["glide_tan"]
    obs = np.asarray(inst["obstacles"], dtype=float).reshape(-1, 4)
    r[P["NOBS"]] = obs.shape[0]          # the library rejects counts above MAX_OBS
    keep = obs[:MAX_OBS].ravel()
    r[P["OBS"]:P["OBS"] + keep.size] = keep
    r[P["DIST"]:P["DIST"] + 3] = inst.get("dist", (0.0, 0.0, 0.0))
    r[P["CYL"]] = float(sum(1 << j for j, c in enumerate(inst.get("cyl", ())) if c))
    r[P["INERTIA"]:P["INERTIA"] + 3] = inst.get("inertia", (0.0, 0.0, 0.0))
    r[P["ARM"]:P["ARM"] + 3] = inst.get("arm", (0.0, 0.0, 0.0))
    r[P["TMIN"]] = inst.get("T_min", 0.0)
    r[P["TMAX"]] = inst.get("T_max", 0.0)
    r[P["GIMBAL"]] = inst.get("gimbal_tan", 0.0)
    r[P["TILT"]] = inst.get("tilt_r", 0.0)
    r[P["WMAX"]] = inst.get("w_max", 0.0)
    return r


def admm_params(rho=1.0, iters=100, check_every=0, eps=0.0, rho_dyn=None, rho_geo=None, eps_dual=None) -> AdmmParams:
    return AdmmParams(rho, rho if rho_dyn is None else rho_dyn, rho if rho_geo is None else rho_geo, iters,
                      check_every, eps, eps if eps_dual is None else eps_dual)


def scp_params(scp_iters=10, admm_iters=100, rho=1.0, check_every=0, eps=0.0, form="persistent",
               scp_per_launch=0, eta0=-math.inf, eta1=0.25, eta2=0.75, shrink=1.0, grow=1.0, delta_max=math.inf,
               merit_w=1.0e3, rho_dyn=None, rho_geo=None, graph=False, rho_final=0.0, adapt_mu=0.0,
               adapt_tau=2.0, group_wait_ms=0.0, lanes_per_node=0, detect_blowup=False) -> ScpParams:
    f = FORM_PERSISTENT if form == "persistent" else FORM_PLAIN
    return ScpParams(scp_iters, admm_params(rho, admm_iters, check_every, eps, rho_dyn, rho_geo), eta0, eta1, eta2,
                     shrink, grow, delta_max, merit_w, f, scp_per_launch, rho_final, 1 if graph else 0, adapt_mu,
                     adapt_tau, group_wait_ms, lanes_per_node, 1 if detect_blowup else 0)


def _pad(a, w):
    a = np.asarray(a, dtype=float)
    out = np.zeros((a.shape[0], w))
    out[:, :a.shape[1]] = a
    return out


def make_desc(insts: list[dict], prec: int = F32, block: int = 0, pack: int = PACK_ALIGNED):
    """The C description of a batch; the second value keeps its arrays alive."""
    model = np.array([d["model"] for d in insts], dtype=np.int32)
    horizon = np.array([d["N"] for d in insts], dtype=np.int32)
    group = np.array([d.get("group", -1) for d in insts], dtype=np.int32)
    params = np.concatenate([param_record(d) for d in insts])
    xg = np.concatenate([_pad(d["x_guess"], MAX_NX) for d in insts])
    ug = np.concatenate([_pad(d["u_guess"], MAX_NU) for d in insts])
    keep = (model, horizon, group, params, xg, ug)
    desc = ProblemDesc(len(insts), prec, model.ctypes.data_as(POINTER(c_int32)),
                       horizon.ctypes.data_as(POINTER(c_int32)), group.ctypes.data_as(POINTER(c_int32)),
                       params.ctypes.data_as(POINTER(c_double)), xg.ctypes.data_as(POINTER(c_double)),
                       ug.ctypes.data_as(POINTER(c_double)), block, pack)
    return desc, keep


def request_arrays(insts: list[dict]) -> dict:
    """The C-record arrays of one request, for fast concatenation into batches (concat_desc)."""
    return dict(model=np.array([d["model"] for d in insts], dtype=np.int32),
                horizon=np.array([d["N"] for d in insts], dtype=np.int32),
                grouped=np.array([d.get("group", -1) >= 0 for d in insts]),
                params=np.concatenate([param_record(d) for d in insts]),
                xg=np.concatenate([_pad(d["x_guess"], MAX_NX) for d in insts]),
                ug=np.concatenate([_pad(d["u_guess"], MAX_NU) for d in insts]),
                shape=[(d["N"], d["nx"], d["nu"]) for d in insts])


def concat_desc(parts: list[dict], prec: int = F32, block: int = 0, pack: int = PACK_ALIGNED):
    """One C description of several requests (request k's grouped trajectories form group k)."""
    model = np.concatenate([p["model"] for p in parts])
    horizon = np.concatenate([p["horizon"] for p in parts])
    group = np.concatenate([np.where(p["grouped"], k, -1) for k, p in enumerate(parts)]).astype(np.int32)
    params = np.concatenate([p["params"] for p in parts])
    xg = np.concatenate([p["xg"] for p in parts])
    ug = np.concatenate([p["ug"] for p in parts])
    keep = (model, horizon, group, params, xg, ug)
    desc = ProblemDesc(len(model), prec, model.ctypes.data_as(POINTER(c_int32)),
                       horizon.ctypes.data_as(POINTER(c_int32)), group.ctypes.data_as(POINTER(c_int32)),
                       params.ctypes.data_as(POINTER(c_double)), xg.ctypes.data_as(POINTER(c_double)),
                       ug.ctypes.data_as(POINTER(c_double)), block, pack)
    return desc, keep


def plan(insts: list[dict], precision: str = "f32", block: int = 0, pack: int = PACK_ALIGNED,
         lanes: bool = False) -> dict:
    """Host-side persistent-kernel plan of a batch (no GPU needed)."""
    lib = load()
    desc, keep = make_desc(insts, F32 if precision == "f32" else F64, block, pack)
    out = (c_int32 * 5)()
    st = lib.scp_plan(byref(desc), out, None, 0)
    if st != SCP_OK:
        raise ScpError(f"scp_plan failed ({st}): {lib.scp_last_error(None).decode()}")
    res = dict(block=out[0], n_wg=out[1], lds_wg=out[2], idle=out[3], spanning=out[4])
    if lanes and out[0]:
        n = out[0] * out[1]
        tab = np.empty(n, dtype=np.int32)
        st = lib.scp_plan(byref(desc), out, tab.ctypes.data_as(POINTER(c_int32)), n)
        if st != SCP_OK:
            raise ScpError(f"scp_plan failed ({st}): {lib.scp_last_error(None).decode()}")
        res["lanes"] = tab.reshape(out[1], out[0])
    return res


def autotune(insts: list[dict], prm: ScpParams, cadences=(1, 5, 10, 25), reps: int = 3, precision: str = "f32",
             device: str = "cuda", stream=None):
    """Run the library's autotuner on this batch; returns (best, table) as dictionaries."""
    import torch
    lib = load()
    desc, keep = make_desc(insts, F32 if precision == "f32" else F64)
    nbytes = lib.scp_autotune_device_bytes(byref(desc))
    if nbytes == 0:
        raise ScpError("invalid problem description for autotune")
    arena = torch.empty(nbytes, dtype=torch.uint8, device=device)
    s = stream if stream is not None else torch.cuda.current_stream(arena.device)
    cad = (c_int32 * len(cadences))(*cadences)
    cap = 6 * len(cadences)
    table = (TuneEntry * cap)()
    n = c_int32(0)
    best = TuneEntry()
    st = lib.scp_autotune(byref(desc), byref(prm), cad, len(cadences), reps, c_void_p(arena.data_ptr()), nbytes,
                          c_void_p(s.cuda_stream), table, cap, byref(n), byref(best))
    if st != SCP_OK:
        raise ScpError(f"scp_autotune failed ({st}): {lib.scp_last_error(None).decode()}")
    return best.as_dict(), [table[i].as_dict() for i in range(min(n.value, cap))]


class ScpError(RuntimeError):
    pass


class Problem:
    """A batch of trajectories resident on the GPU (one arena tensor), driven through the C ABI."""

    def __init__(self, insts: list[dict] | None, precision: str = "f32", block: int = 0, device: str = "cuda",
                 stream=None, pack: int = PACK_ALIGNED, parts: list[dict] | None = None, noalloc: bool = False):
        """insts: problem dictionaries; or parts: request_arrays() of several requests.  noalloc: the
        arena is the library's fixed no-allocation arena of the device (scp_problem_create_noalloc)
        instead of a torch tensor."""
        import torch
        self.torch = torch
        self.lib = load()
        self.prec = F32 if precision == "f32" else F64
        self.dtype = torch.float32 if self.prec == F32 else torch.float64
        if parts is not None:
            desc, self._keep = concat_desc(parts, self.prec, block, pack)
            self.insts = [dict(N=N, nx=nx, nu=nu) for p in parts for N, nx, nu in p["shape"]]
        else:
            desc, self._keep = make_desc(insts, self.prec, block, pack)
            self.insts = insts
        self.n_traj = len(self.insts)
        nbytes = self.lib.scp_problem_device_bytes(byref(desc))
        if nbytes == 0:
            h = c_void_p()
            st = self.lib.scp_problem_create(byref(desc), None, 0, None, byref(h))
            raise ScpError(f"invalid problem description: {self.lib.scp_last_error(None).decode()}")
        self.nbytes = nbytes
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = c_void_p()
        if noalloc:
            self.arena = None
            with torch.cuda.device(self.device):
                st = self.lib.scp_problem_create_noalloc(byref(desc), c_void_p(self.stream.cuda_stream), byref(h))
            what = "scp_problem_create_noalloc"
        else:
            self.arena = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            if self.stream != torch.cuda.current_stream(self.device):
                self.arena.record_stream(self.stream)
            st = self.lib.scp_problem_create(byref(desc), c_void_p(self.arena.data_ptr()), nbytes,
                                             c_void_p(self.stream.cuda_stream), byref(h))
            what = "scp_problem_create"
        if st != SCP_OK:
            raise ScpError(f"{what} failed ({st}): {self.lib.scp_last_error(None).decode()}")
        self.h = h
        self.n_nodes = int(self.lib.scp_problem_nodes(h))
        self.offsets = np.array([self.lib.scp_traj_node_offset(h, t) for t in range(self.n_traj)], dtype=np.int64)

    @staticmethod
    def _pad(a, w):
        return _pad(a, w)

    def _check(self, st, what):
        if st != SCP_OK:
            raise ScpError(f"{what} failed ({st}): {self.lib.scp_last_error(self.h).decode()}")

    def linearize(self, prm: AdmmParams | None = None):
        self._check(self.lib.scp_linearize(self.h, byref(prm) if prm is not None else None), "scp_linearize")

    def admm(self, prm: AdmmParams):
        self._check(self.lib.admm_solve(self.h, byref(prm)), "admm_solve")

    def solve(self, prm: ScpParams):
        self._check(self.lib.scp_solve(self.h, byref(prm)), "scp_solve")

    def reset(self):
        """Back to the initial guess with zero duals: the next solve starts fresh."""
        self._check(self.lib.scp_reset(self.h), "scp_reset")

    def export_state(self):
        """Checkpoint: the whole solver state as a host uint8 array (waits for the problem's stream)."""
        import numpy as np
        buf = np.empty(self.lib.scp_problem_state_bytes(self.h), dtype=np.uint8)
        self._check(self.lib.scp_problem_export_state(self.h, c_void_p(buf.ctypes.data), c_size_t(buf.nbytes)),
                    "scp_problem_export_state")
        return buf

    def import_state(self, buf):
        """Resume from export_state() of a problem with the same description."""
        import numpy as np
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(self.lib.scp_problem_import_state(self.h, c_void_p(buf.ctypes.data), c_size_t(buf.nbytes)),
                    "scp_problem_import_state")

    def field(self, name: str):
        fid = FIELDS[name]
        w = self.lib.scp_field_width(fid)
        out = self.torch.empty((self.n_nodes, w), dtype=self.dtype, device=self.device)
        self._enter(out)
        self._check(self.lib.scp_get_field(self.h, fid, c_void_p(out.data_ptr())), "scp_get_field")
        self._join()
        return out

    def _enter(self, *outs):
        """Before the library writes caller-side tensors on the problem's stream: that stream
        waits for the caller's current stream (the allocator may hand out a block whose last use
        there is still running), and the tensors are marked as used on it."""
        cur = self.torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)
            for o in outs:
                o.record_stream(self.stream)

    def _join(self):
        """Order the caller's current stream after the work enqueued on the problem's stream."""
        cur = self.torch.cuda.current_stream(self.device)
        if cur != self.stream:
            cur.wait_stream(self.stream)

    def result(self):
        """(x, u, info) as device tensors: x (nodes, MAX_NX), u (nodes, MAX_NU), info (n_traj, 12) float64."""
        t = self.torch
        x = t.empty((self.n_nodes, MAX_NX), dtype=self.dtype, device=self.device)
        u = t.empty((self.n_nodes, MAX_NU), dtype=self.dtype, device=self.device)
        info = t.empty((self.n_traj, INFO_FIELDS), dtype=t.float64, device=self.device)
        self._enter(x, u, info)
        self._check(self.lib.scp_get_result(self.h, c_void_p(x.data_ptr()), c_void_p(u.data_ptr()),
                                            c_void_p(info.data_ptr())), "scp_get_result")
        self._join()
        return x, u, info

    def split(self, arr: np.ndarray, t: int, width: int | None = None, controls: bool = False) -> np.ndarray:
        """Rows of trajectory t from a node-major array (controls: the first N rows)."""
        N = self.insts[t]["N"]
        o = self.offsets[t]
        rows = arr[o:o + N + (0 if controls else 1)]
        return rows if width is None else rows[:, :width]

    def info_dicts(self, info: np.ndarray) -> list[dict]:
        return [{k: float(info[t, v]) for k, v in INFO.items()} for t in range(self.n_traj)]

    def close(self):
        if getattr(self, "h", None):
            self.lib.scp_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """The library's continuous-batching request server on one device pool (a torch uint8 arena).

    Marshalling only: requests (lists of problem dictionaries) are packed into C descriptions,
    scheduling, admission, warm starts and every computation run in the library."""

    def __init__(self, prm: ScpParams, precision: str = "f32", block: int = 256, pack: int = PACK_ALIGNED,
                 max_nodes: int = 1 << 16, max_traj: int = 1024, max_wg: int = 1024, max_span: int = 256,
                 max_requests: int = 256, budget_bytes: int | None = None, scp_per_step: int = 1,
                 max_inflight: int = 2, device: str = "cuda", stream=None, timeout_ms: float = 0.0):
        import torch
        self.torch = torch
        self.lib = load()
        self.prec = F32 if precision == "f32" else F64
        cfg = ServerConfig(self.prec, block, pack, max_nodes, max_traj, max_wg, max_span, max_requests, 0, prm,
                           scp_per_step, max_inflight, timeout_ms)
        nbytes = self.lib.scp_server_device_bytes(byref(cfg))
        if nbytes == 0:
            h = c_void_p()
            self.lib.scp_server_create(byref(cfg), None, 0, None, byref(h))
            raise ScpError(f"invalid server configuration: {self.lib.scp_server_last_error(None).decode()}")
        cfg.budget_bytes = nbytes if budget_bytes is None else int(budget_bytes)
        self.cfg = cfg
        self.nbytes = nbytes
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.arena.device)
        self.arena.record_stream(self.stream)
        torch.cuda.synchronize(self.arena.device)
        h = c_void_p()
        st = self.lib.scp_server_create(byref(cfg), c_void_p(self.arena.data_ptr()), nbytes,
                                        c_void_p(self.stream.cuda_stream), byref(h))
        if st != SCP_OK:
            raise ScpError(f"scp_server_create failed ({st}): {self.lib.scp_server_last_error(None).decode()}")
        self.h = h
        self.shapes = {}
        self._ended = set()     # ended requests reported by take_done that no drain asked for yet

    def _check(self, st, what):
        if st != SCP_OK:
            raise ScpError(f"{what} failed ({st}): {self.lib.scp_server_last_error(self.h).decode()}")

    def take_done(self, cap: int = 4096) -> list[int]:
        """Ids of the requests that ended (done, cancelled, timed out) since the last call."""
        buf = (c_int64 * cap)()
        n = c_int32(0)
        out = []
        while True:
            self._check(self.lib.scp_server_take_done(self.h, buf, cap, byref(n)), "scp_server_take_done")
            out.extend(buf[:n.value])
            if n.value < cap:
                return out

    def cancel(self, rid: int):
        self._check(self.lib.scp_server_cancel(self.h, rid), "scp_server_cancel")

    def request_bytes(self, insts: list[dict]) -> int:
        desc, keep = make_desc(insts, self.prec)
        return int(self.lib.scp_server_request_bytes(self.h, byref(desc)))

    def prepare(self, insts: list[dict]):
        """A reusable C description of a request (submit it any number of times)."""
        desc, keep = make_desc(insts, self.prec)
        return (desc, keep, [(d["N"], d["nx"], d["nu"]) for d in insts])

    def submit(self, insts, session: int = -1, measured: bool = False) -> int:
        """Queue a request (a list of problem dictionaries, or a prepared description).
        measured: a warm start keeps the request's x_init (closed-loop MPC, SUBMIT_MEASURED)."""
        desc, keep, shape = insts if isinstance(insts, tuple) else self.prepare(insts)
        rid = c_int64(0)
        flags = SUBMIT_MEASURED if measured else 0
        self._check(self.lib.scp_server_submit_ex(self.h, byref(desc), session, flags, byref(rid)),
                    "scp_server_submit_ex")
        self.shapes[rid.value] = shape
        return rid.value

    def poll(self, rid: int, release: bool = True):
        """None while queued or running, else (latency_ms, info array (n_traj, 12)); a request that
        ended without a result (cancelled, timed out) gives (latency_ms, None)."""
        shape = self.shapes[rid]
        state = c_int32(0)
        lat = c_double(0.0)
        info = np.zeros((len(shape), INFO_FIELDS))
        self._check(self.lib.scp_server_collect(self.h, rid, 1 if release else 0, byref(state), byref(lat),
                                                info.ctypes.data_as(POINTER(c_double)), None, None),
                    "scp_server_collect")
        if state.value in (REQ_CANCELLED, REQ_TIMEOUT):
            if release:
                self.shapes.pop(rid, None)
            return lat.value, None
        if state.value != REQ_DONE:
            if state.value == REQ_UNKNOWN:
                raise ScpError(f"request {rid} unknown or already collected")
            return None
        if release:
            self.shapes.pop(rid, None)
        return lat.value, info

    def step(self, wait: bool = False) -> int:
        pending = c_int32(0)
        self._check(self.lib.scp_server_step(self.h, 1 if wait else 0, byref(pending)), "scp_server_step")
        return pending.value

    def collect(self, rid: int, release: bool = True):
        """None while the request is queued or running; else dict(latency_ms, info, x, u) with
        per-trajectory arrays (x: (N+1, nx), u: (N, nu)) and info dictionaries."""
        shape = self.shapes.get(rid)
        if shape is None:
            raise ScpError(f"unknown request {rid}")
        nt = len(shape)
        nxr = sum(N + 1 for N, _, _ in shape)
        nur = sum(N for N, _, _ in shape)
        state = c_int32(0)
        lat = c_double(0.0)
        info = np.zeros((nt, INFO_FIELDS))
        x = np.zeros((nxr, MAX_NX))
        u = np.zeros((max(nur, 1), MAX_NU))
        dp = lambda a: a.ctypes.data_as(POINTER(c_double))
        self._check(self.lib.scp_server_collect(self.h, rid, 1 if release else 0, byref(state), byref(lat), dp(info),
                                                dp(x), dp(u)), "scp_server_collect")
        if state.value in (REQ_CANCELLED, REQ_TIMEOUT):
            if release:
                self.shapes.pop(rid, None)
            return dict(latency_ms=lat.value, state="cancelled" if state.value == REQ_CANCELLED else "timeout",
                        info=None, x=None, u=None)
        if state.value != REQ_DONE:
            if state.value == REQ_UNKNOWN:
                raise ScpError(f"request {rid} unknown or already collected")
            return None
        if release:
            self.shapes.pop(rid, None)
        xs, us, xo, uo = [], [], 0, 0
        for N, nx, nu in shape:
            xs.append(x[xo:xo + N + 1, :nx].copy())
            us.append(u[uo:uo + N, :nu].copy())
            xo += N + 1
            uo += N
        infos = [{k: float(info[t, v]) for k, v in INFO.items()} for t in range(nt)]
        return dict(latency_ms=lat.value, state="done", info=infos, x=xs, u=us)

    def stats(self) -> dict:
        out = ServerStats()
        self._check(self.lib.scp_server_get_stats(self.h, byref(out)), "scp_server_get_stats")
        return out.as_dict()

    def drain(self, ids, timeout_s: float = 60.0) -> dict:
        """Step until every request in ids has ended; returns {id: result}.  Only the requests the
        library reports as ended are collected (no polling of every pending id)."""
        import time
        out = {}
        t0 = time.perf_counter()
        todo = set(ids)
        for rid in list(todo & self._ended):
            out[rid] = self.collect(rid)
            todo.discard(rid)
            self._ended.discard(rid)
        while todo:
            self.step(wait=True)
            for rid in self.take_done():
                if rid in todo:
                    out[rid] = self.collect(rid)
                    todo.discard(rid)
                else:
                    self._ended.add(rid)
            if todo and time.perf_counter() - t0 > timeout_s:
                raise ScpError(f"requests not done after {timeout_s} s: {sorted(todo)[:8]}")
        return out

    def close(self):
        if getattr(self, "h", None):
            self.lib.scp_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

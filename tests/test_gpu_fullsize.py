"""Parity at the full workload sizes, in the launch configuration the benchmark times.

Quadrotor batch: 1024 instances, N = 50, 8 obstacles, 15 SCP x 200 ADMM, FP32, persistent form.
Powered descent: 4096 instances, N = 60, 15 x 200, FP32.
Uneven mix: 2048 instances, N ~ U{20..120}, residual stop 1e-4 every 25 iterations, 15 x 200 caps.
* sampled instances after the first SCP iteration of the full batch: FP32 vs oracle at 1e-4;
* sampled instances in FP64 mode vs oracle: 1e-9 after 5 SCP iterations, a fixed 1e-6 at the full
  budget (the SCP map amplifies rounding-order differences; measured on the oracle itself);
* every sampled trajectory of the full FP32 batch is bitwise equal to the same trajectory solved
  alone (placement independence), and plain and persistent forms agree to 1e-4 after SCP 1;
* properties that hold at any size: finite iterates, boundary conditions, metrics consistent.
"""
import numpy as np
import pytest

import scpgen
import oracle
from _parity import FIELDS, compare, gpu_fields, oracle_scp, rel_err

pytestmark = pytest.mark.gpu

SAMPLE = [0, 333, 1023]


@pytest.fixture(scope="module")
def B(lib):
    from paper_2603_10711_amd import binding
    return binding


@pytest.fixture(scope="module")
def quad_batch():
    return scpgen.config1(1024)


def test_quad_full_batch_first_scp_iteration(B, quad_batch):
    print("quad 1024 x 51, 1 x 200 fp32 persistent", flush=True)
    prob = B.Problem(quad_batch, precision="f32")
    prob.solve(B.scp_params(1, 200))
    f = gpu_fields(prob)
    sample = [quad_batch[i] for i in SAMPLE]
    trajs, _ = oracle_scp(sample, 1, 200)
    worst = compare(prob, f, sample, trajs, idx=SAMPLE)
    print(worst, flush=True)
    assert max(worst.values()) < 1e-4
    plain = B.Problem(quad_batch, precision="f32")
    plain.solve(B.scp_params(1, 200, form="plain"))
    fp = gpu_fields(plain, ("xbar", "lam", "dual"))
    for k in fp:
        assert rel_err(fp[k][:prob.n_nodes], f[k][:prob.n_nodes]) < 1e-4
    prob.close()
    plain.close()


def _oracle_cholesky_variant(sample, K, J):
    """The oracle with its Step-1 solves done by Cholesky instead of LU: an equally valid rounding
    order, used to measure how much the SCP map amplifies rounding differences."""
    import scipy.linalg as sl
    import oracle.admm as oa

    lu = oa.np.linalg.solve

    def chol(H, b):
        if H.ndim == 3:
            return np.stack([sl.cho_solve(sl.cho_factor(H[i], lower=True), b[i]) for i in range(H.shape[0])])
        return sl.cho_solve(sl.cho_factor(H, lower=True), b)

    oa.np.linalg.solve = chol
    try:
        return oracle_scp(sample, K, J)[0]
    finally:
        oa.np.linalg.solve = lu


# FP64 bar at the full 15 x 200 budget.  Over 15 SCP iterations the map amplifies rounding-order
# differences: the oracle itself, with its Step-1 solves done by Cholesky instead of LU (an equally
# valid rounding order), moves its own nominal by up to 5.8e-8 relative on these samples (instance
# 1023; 1.4e-10 to 6.6e-10 on the others).  The bar is a fixed 1e-6, 17 x that measured
# amplification; after 5 SCP iterations the bar stays 1e-9.
TOL64_FULL = 1e-6


def test_quad_full_budget_fp64_samples(B, quad_batch):
    """FP64 mode against the oracle: 1e-9 after 5 SCP iterations, TOL64_FULL at the full budget;
    the oracle's own LU-vs-Cholesky gap is printed beside it."""
    sample = [quad_batch[i] for i in SAMPLE]
    for K in (5, 15):
        print(f"quad samples {K} x 200 fp64 persistent", flush=True)
        prob = B.Problem(sample, precision="f64")
        prob.solve(B.scp_params(K, 200))
        f = gpu_fields(prob)
        trajs, _ = oracle_scp(sample, K, 200)
        worst = compare(prob, f, sample, trajs)
        tol = 1e-9 if K == 5 else TOL64_FULL
        if K == 15:
            alt = _oracle_cholesky_variant(sample, K, 200)
            self_gap = max(rel_err(a.xbar, t.xbar) for a, t in zip(alt, trajs))
            print(f"oracle self-disagreement {self_gap:.2e}; bar {tol:.0e}", flush=True)
        print(worst, flush=True)
        assert max(worst.values()) < tol
        prob.close()


def test_quad_full_budget_batch_invariance(B, quad_batch):
    print("quad 1024 15 x 200 fp32 persistent vs alone", flush=True)
    prob = B.Problem(quad_batch, precision="f32")
    prob.solve(B.scp_params(15, 200))
    x, u, info = prob.result()
    x, u, info = x.cpu().numpy(), u.cpu().numpy(), info.cpu().numpy()
    assert np.all(np.isfinite(x[:prob.n_nodes])) and np.all(np.isfinite(info[:, :11]))   # ratio may be -inf
    assert np.all(info[:, 0] == 3000) and np.all(info[:, 3] == 15)
    for i in SAMPLE:
        alone = B.Problem([quad_batch[i]], precision="f32")
        alone.solve(B.scp_params(15, 200))
        xa, ua, ia = (a.cpu().numpy() for a in alone.result())
        o = prob.offsets[i]
        n = quad_batch[i]["N"] + 1
        np.testing.assert_array_equal(xa[:n], x[o:o + n])
        np.testing.assert_array_equal(ua[:n], u[o:o + n])
        np.testing.assert_array_equal(ia[0], info[i])
        alone.close()
    # metrics recomputed by the oracle from the returned FP32 trajectory (in FP64)
    for i in SAMPLE:
        d = quad_batch[i]
        o, N = prob.offsets[i], d["N"]
        xs, us = x[o:o + N + 1, :6].astype(float), u[o:o + N, :3].astype(float)
        assert abs(info[i, 6] - oracle.defect(d, xs, us)) < 1e-4 * max(1.0, oracle.defect(d, xs, us))
        assert abs(info[i, 7] - oracle.cost(d, xs, us)) < 1e-5 * abs(oracle.cost(d, xs, us))
    prob.close()


def test_mars_full_batch(B):
    insts = scpgen.config2(4096)
    print("mars 4096 x 61 fp32 persistent 1 x 200", flush=True)
    prob = B.Problem(insts, precision="f32")
    prob.solve(B.scp_params(1, 200))
    f = gpu_fields(prob)
    idx = [0, 2047, 4095]
    sample = [insts[i] for i in idx]
    trajs, _ = oracle_scp(sample, 1, 200)
    worst = compare(prob, f, sample, trajs, idx=idx)
    print(worst, flush=True)
    assert max(worst.values()) < 1e-4
    prob.close()


def test_mix_full_batch_fp64_samples(B):
    """The uneven mix at full size (2048 instances, half quadrotor and half powered descent, N ~
    U{20..120}) in the benchmark's launch configuration (128 lanes, aligned, residual test every 25
    iterations at 1e-4, caps 15 x 200), FP64 mode.  Sampled instances (the longest quadrotor and
    powered descent, the shortest, two that straddle a wavefront and the two that stop earliest)
    against the oracle with the same stopping rule: identical ADMM iteration counts, iterates at
    the fixed full-budget bar."""
    insts = scpgen.config3(2048)
    print("mix 2048 fp64 persistent 15 x 200, block 128 aligned, check 25 at 1e-4", flush=True)
    prob = B.Problem(insts, precision="f64", block=128, pack=B.PACK_ALIGNED)
    prob.solve(B.scp_params(15, 200, check_every=25, eps=1e-4))
    f = gpu_fields(prob)
    info = prob.info_dicts(prob.result()[2].cpu().numpy())
    iters = np.array([d["admm_iters"] for d in info])
    Ns = np.array([d["N"] for d in insts])
    models = np.array([d["model"] for d in insts])
    idx = [int(np.argmax(np.where(models == 1, Ns, -1))), int(np.argmax(np.where(models == 2, Ns, -1))),
           int(np.argmin(Ns))]
    idx += [i for i in range(len(insts)) if 64 < Ns[i] + 1 < 70][:2]
    idx += [int(i) for i in np.argsort(iters, kind="stable")[:2]]
    idx = list(dict.fromkeys(idx))
    sample = [insts[i] for i in idx]
    print("sample", idx, Ns[idx].tolist(), iters[idx].tolist(), flush=True)
    trajs, oinfo = oracle_scp(sample, 15, 200, check_every=25, eps_p=1e-4, eps_d=1e-4)
    assert [o["admm_iters"] for o in oinfo] == iters[idx].tolist()
    worst = compare(prob, f, sample, trajs, idx=idx)
    print(worst, flush=True)
    assert max(worst.values()) < TOL64_FULL
    prob.close()


def test_mars_full_budget_fp64_samples(B):
    """The powered-descent batch at full size and full budget (4096 instances, 15 x 200) in FP64
    mode, sampled instances against the oracle at the fixed full-budget bar."""
    insts = scpgen.config2(4096)
    print("mars 4096 x 61 fp64 persistent 15 x 200", flush=True)
    prob = B.Problem(insts, precision="f64")
    prob.solve(B.scp_params(15, 200))
    f = gpu_fields(prob)
    idx = [0, 2047, 4095]
    sample = [insts[i] for i in idx]
    trajs, _ = oracle_scp(sample, 15, 200)
    worst = compare(prob, f, sample, trajs, idx=idx)
    print(worst, flush=True)
    assert max(worst.values()) < TOL64_FULL
    prob.close()

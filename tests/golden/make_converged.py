"""Write the oracle's converged solutions of a batch (expected values for the GPU tests of the
converged-solution bar).

    python tests/golden/make_converged.py [--workload quad1024|quad6_1000|mars4096|mix2048] [--workers W]
                                          [--count C]

Calls only the oracle (FP64 NumPy), with the geometric penalty schedule of the paper's parameter
study (Sec. IV-A.2: one rho for all three penalties, grown geometrically over the SCP iterations to
a final value):

* quad1024: the 1024 point-mass quadrotor instances of the batch workload (N = 50, 8 obstacles,
  seeded generator), rho 5 -> 1e4 over 18 SCP iterations of 290 ADMM iterations each (the headline
  setting of the benchmark), fixed trust radius, always-accept steps;
* quad6_1000: the first C (default 256) of the 1000 6-DOF quadrotor instances of the scalability
  batch (Sec. IV-A.3: N = 40, three obstacles, noise-initialized), rho 10 -> 3e4 over 50 SCP
  iterations of 300 ADMM iterations each, with the trust-region ratio test of the SCP step (accept
  when the ratio is positive, radius halved below 0.25, doubled above 0.75 up to 4);
* mars4096: the first C (default 256) of the 4096 powered-descent Monte Carlo instances (N = 60,
  tf = 50 s), rho 1 -> 1e4 over 30 SCP iterations of 400 ADMM iterations each, fixed trust radius,
  always-accept steps;
* mix2048: the first C (default 256) of the 2048 instances of the uneven mix (half quadrotor, half
  powered descent, N ~ U{20..120}), rho 5 -> 1e4 over 25 SCP iterations of 400 ADMM iterations
  each, with the residual stop of the mix (primal and dual residual <= 1e-4, tested every 25 ADMM
  iterations).

For every instance it stores the final cost, max dynamics defect, max constraint violation and
boundary error of the returned nominal.
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

WORKLOADS = {
    "quad1024": dict(setting=dict(scp_iters=18, admm_iters=290, rho=5.0, rho_final=1e4), count=1024,
                     what="oracle (FP64) solutions of the point-mass quadrotor batch, 1024 x N=50, 8 obstacles"),
    "quad6_1000": dict(setting=dict(scp_iters=50, admm_iters=300, rho=10.0, rho_final=3e4, eta0=0.0, eta1=0.25,
                                    eta2=0.75, shrink=0.5, grow=2.0, delta_max=4.0), count=256,
                       what="oracle (FP64) solutions of the first instances of the 6-DOF quadrotor batch, "
                            "1000 x N=40, 3 obstacles"),
    "mars4096": dict(setting=dict(scp_iters=30, admm_iters=400, rho=1.0, rho_final=1e4), count=256,
                     what="oracle (FP64) solutions of the first instances of the powered-descent Monte Carlo, "
                          "4096 x N=60, tf=50 s"),
    "mix2048": dict(setting=dict(scp_iters=25, admm_iters=400, rho=5.0, rho_final=1e4, check_every=25,
                                 eps_p=1e-4, eps_d=1e-4), count=256,
                    what="oracle (FP64) solutions of the first instances of the uneven mix, 2048 instances, "
                         "half quadrotor / half powered descent, N ~ U{20..120}"),
}


_CACHE = {}


def _instance(workload, i):
    import scpgen
    if workload == "quad1024":
        return scpgen.config1(i + 1)[i]
    if workload == "mars4096":
        return scpgen.config2(1, first=i)[0]
    if workload == "mix2048":       # the mix's order depends on the batch size
        if "mix2048" not in _CACHE:
            _CACHE["mix2048"] = scpgen.config3(2048)
        return _CACHE["mix2048"][i]
    return scpgen.config5(1, first=i)[0]


def _solve(args):
    workload, i = args
    import oracle
    s = dict(WORKLOADS[workload]["setting"])
    rho = s.pop("rho")
    p = oracle.default_params(rho_eq=rho, rho_dyn=rho, rho_geo=rho, **s)
    _, infos = oracle.scp_solve([_instance(workload, i)], p)
    f = infos[0]
    return i, dict(cost=f["cost"], defect=f["defect"], viol=f["viol"], bnd_err=f["bnd_err"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="quad1024", choices=sorted(WORKLOADS))
    ap.add_argument("--workers", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--count", type=int, default=0)
    a = ap.parse_args()
    w = WORKLOADS[a.workload]
    count = a.count or w["count"]
    t0 = time.time()
    rows = [None] * count
    with mp.get_context("fork").Pool(a.workers) as pool:
        for k, (i, r) in enumerate(pool.imap_unordered(_solve, [(a.workload, i) for i in range(count)])):
            rows[i] = r
            if k % 32 == 0:
                print(f"{k + 1}/{count} {time.time() - t0:.0f} s", flush=True)
    out = {"what": w["what"], "setting": w["setting"], "generator": "tests/golden/make_converged.py",
           "instances": rows}
    OUT = os.path.join(HERE, f"{a.workload}_converged.json")
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=0)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()

"""Write the oracle's converged solutions of the quadrotor batch (expected values for the GPU test
of the converged-solution bar).

    python tests/golden/make_converged.py [--workers W]

Calls only the oracle (FP64 NumPy): the 1024 point-mass quadrotor instances of the batch workload
(N = 50, 8 obstacles, seeded generator) solved with the geometric penalty schedule of the paper's
parameter study (Sec. IV-A.2: one rho for all three penalties, grown geometrically over the SCP
iterations to a final value), here from 5 to 1e4 over 18 SCP iterations of 290 ADMM iterations each
(the headline setting of the benchmark), fixed trust radius, always-accept steps.  For every instance it stores the final cost, max
dynamics defect, max constraint violation and boundary error of the returned nominal.
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

SETTING = dict(scp_iters=18, admm_iters=290, rho=5.0, rho_final=1e4)
OUT = os.path.join(HERE, "quad1024_converged.json")


def _solve(i):
    import oracle
    import scpgen
    d = scpgen.config1(i + 1)[i]
    p = oracle.default_params(scp_iters=SETTING["scp_iters"], admm_iters=SETTING["admm_iters"],
                              rho_eq=SETTING["rho"], rho_dyn=SETTING["rho"], rho_geo=SETTING["rho"],
                              rho_final=SETTING["rho_final"])
    _, infos = oracle.scp_solve([d], p)
    f = infos[0]
    return i, dict(cost=f["cost"], defect=f["defect"], viol=f["viol"], bnd_err=f["bnd_err"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=min(8, os.cpu_count() or 1))
    ap.add_argument("--count", type=int, default=1024)
    a = ap.parse_args()
    t0 = time.time()
    rows = [None] * a.count
    with mp.get_context("fork").Pool(a.workers) as pool:
        for k, (i, r) in enumerate(pool.imap_unordered(_solve, range(a.count))):
            rows[i] = r
            if k % 32 == 0:
                print(f"{k + 1}/{a.count} {time.time() - t0:.0f} s", flush=True)
    out = {"what": "oracle (FP64) solutions of the point-mass quadrotor batch, 1024 x N=50, 8 obstacles",
           "setting": SETTING, "generator": "tests/golden/make_converged.py", "instances": rows}
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=0)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()

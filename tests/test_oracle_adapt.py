"""Pins of the oracle's adaptive penalty (residual balancing between SCP iterations; the paper
gives none, the rule is that of Boyd et al. 2011, Sec. 3.4.1):

* it moves the residual ratio toward balance from either side: a penalty far too small (primal
  residual dominating) is raised, one far too large is lowered, and the final r_p / r_d lies
  closer to 1 than with the penalty fixed; the factor is a power of tau;
* where the residuals stay within a factor mu of each other the run is the fixed-penalty run,
  bit for bit, and adapt_mu = 0 is the fixed solver;
* with affine dynamics every subproblem has the same optimum whatever the penalty, so the last
  ADMM output, reached after the penalties changed between SCP iterations (duals carried, the
  factor rebuilt), satisfies the KKT conditions of the last subproblem; a factor left at the old
  penalties would leave a residual;
* a scenario group of identical copies adapts like the single instance.
"""
import math

import numpy as np

import oracle
import scpgen
from oracle.scp import init_traj, scp_group

from test_oracle_scp import _kkt_check


def _p(rho, **kw):
    return oracle.default_params(rho_eq=rho, rho_dyn=rho, rho_geo=rho, **kw)


def test_adaptive_penalty_moves_toward_balance():
    inst = scpgen.config0()[0]
    for rho, grows in ((1e-3, True), (1e4, False)):
        fixed = oracle.scp_solve([inst], _p(rho, scp_iters=10, admm_iters=100))[1][0]
        adapt = oracle.scp_solve([inst], _p(rho, scp_iters=10, admm_iters=100, adapt_mu=10.0))[1][0]
        s = adapt["rho_scale"]
        assert (s > 1.0) if grows else (s < 1.0), (rho, s)
        e = math.log2(s)
        assert e == round(e)
        assert abs(math.log(adapt["r_p"] / adapt["r_d"])) < abs(math.log(fixed["r_p"] / fixed["r_d"]))
        assert fixed["rho_scale"] == 1.0


def test_balanced_runs_are_the_fixed_solver():
    inst = scpgen.config0()[0]
    a = oracle.scp_solve([inst], _p(1.0, scp_iters=6, admm_iters=100))
    b = oracle.scp_solve([inst], _p(1.0, scp_iters=6, admm_iters=100, adapt_mu=10.0))
    c = oracle.scp_solve([inst], _p(1.0, scp_iters=6, admm_iters=100, adapt_mu=0.0, adapt_tau=3.0))
    assert b[1][0]["rho_scale"] == 1.0
    for other in (b, c):
        np.testing.assert_array_equal(a[0][0][0], other[0][0][0])
        np.testing.assert_array_equal(a[0][0][1], other[0][0][1])


def _affine_instance():
    inst = scpgen.quad_instance(0, 0, N=6, K=0, T=3.0, drag=0.0, delta=3.0)
    inst["x_init"] = np.zeros(6)
    inst["x_target"] = np.array([1.2, 0.5, 0.3, 0, 0, 0])
    inst["qn"] = -200.0 * inst["x_target"]
    inst["obstacles"] = np.array([[0.6, 0.25, 0.2, 0.3]])
    s = np.linspace(0, 1, 7)[:, None]
    inst["x_guess"] = np.hstack([s * inst["x_target"][:3], np.tile(inst["x_target"][:3] / 3.0, (7, 1))])
    inst["u_ball"] = 10.3
    return inst


def test_adaptive_penalty_reaches_the_subproblem_kkt_point():
    t = init_traj(_affine_instance())
    info = scp_group([t], _p(200.0, scp_iters=6, admm_iters=3000, check_every=50, eps_p=1e-11, eps_d=1e-11,
                             adapt_mu=10.0))
    assert info["rho_scale"] < 1.0 / 8.0, info     # the penalty was lowered several times
    assert info["r_p"] < 1e-9 and info["r_d"] < 1e-9, info
    _kkt_check(t, None, 1e-7)


def test_group_of_identical_copies_adapts_like_one_instance():
    inst = scpgen.quad_instance(1, 3, N=10, K=2)
    p = _p(1e-2, scp_iters=5, admm_iters=40, adapt_mu=10.0)
    one = [init_traj(inst)]
    i1 = scp_group(one, p)
    grp = [init_traj(dict(inst, group=0)) for _ in range(3)]
    i3 = scp_group(grp, p)
    assert i1["rho_scale"] > 1.0 and i3["rho_scale"] == i1["rho_scale"]
    for t in grp:
        np.testing.assert_allclose(t.xbar, one[0].xbar, rtol=0, atol=1e-12)

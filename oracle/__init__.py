"""CPU oracle for the SCP + consensus-ADMM hot path (plain, slow, FP64 NumPy).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
never calls into it and shares no code with it: the two are independent
encodings of the same method, written from the paper (arXiv 2603.10711):

* Sec. II, eq. (ocp): discrete OCP with RK4 dynamics, boundary conditions and
  prox-friendly convex sets;
* Sec. III-A, eq. (qp_subproblem): first-order dynamics / second-order cost
  expansion around the nominal, trust-region boxes;
* Sec. III-B: variable splitting (physical x,u; dynamic z; geometric mirrors),
  the augmented Lagrangian (eq. augmented_lagrangian) and ADMM Steps 1-4.

Where the paper is silent (group-wise mirror copies, residual definitions,
trust-region acceptance, units of the powered-descent model, ...), the
oracle follows the readings listed in the design notes of the repository;
each function's docstring names the reading it implements.

Parity status: every function here is pinned by a CPU test against something
other than itself (closed forms, complex-step derivatives, brute-force KKT,
Riccati LQR, projection invariants), except the full nonlinear FP32-budget
trajectories of the quadrotor / powered-descent workloads, whose end-to-end
values are *parity unpinned* beyond this oracle (the paper prints no values for
those workloads).
"""
from .dynamics import f_cont, jac_cont, rk4, rk4_jac  # noqa: F401
from .sets import proj_box, proj_halfspace, proj_ball, proj_soc, proj_cone  # noqa: F401
from .admm import Group, QP, AdmmState, build_H, admm_run, residuals  # noqa: F401
from .scp import (linearize, convexify, scp_solve, default_params, defect, cost,  # noqa: F401
                  violation, boundary_error, Traj, init_traj, shift_warm_start, mpc_session)

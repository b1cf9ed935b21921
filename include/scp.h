/*
 * scp.h - C ABI of the MI355X (gfx950) library for the data-parallel hot path of
 * GPU-native sequential convex programming with consensus ADMM (arXiv 2603.10711).
 *
 * The library solves batches of discrete optimal control problems of the form of the
 * paper's eq. (ocp) (Sec. II): RK4-discretized nonlinear dynamics x_{i+1} = f(x_i, u_i),
 * boundary conditions x_0 = x_init and S x_N = x_target, convex sets on x_i and u_i.
 * Each SCP iteration (Sec. III-A) linearizes the dynamics around the nominal trajectory and
 * solves the convex subproblem eq. (qp_subproblem) with the temporally split consensus ADMM
 * of Sec. III-B (per-node dense Cholesky solves, closed-form consensus update, analytic
 * projections, dual ascent).
 *
 * General conventions
 *  - Every call returns scp_status (SCP_OK = 0) and never throws.  On error the handle's
 *    message is available from scp_last_error().
 *  - Device memory: the caller owns it.  scp_problem_device_bytes() gives the size of the
 *    arena that scp_problem_create() needs; the caller allocates it (e.g. a torch uint8 tensor)
 *    and keeps it alive until scp_problem_destroy().  The library never calls hipMalloc.
 *  - Streams: every call after create enqueues work on the hip stream given at create time
 *    and returns without synchronizing; results live in device memory.
 *  - Numerical failures are not call errors: they are per-trajectory status bits in the info
 *    record (SCP_ST_*), and the other trajectories of the batch are unaffected.
 *  - Thread compatibility: one handle must not be used from two host threads at once.
 *    Different handles are independent.
 */
#ifndef SCP_MI355X_H
#define SCP_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SCP_OK = 0,
    SCP_ERR_ARG = 1,          /* invalid argument (sizes, ids, NULL pointers, arena too small) */
    SCP_ERR_NOMEM = 2,        /* host allocation failed */
    SCP_ERR_HIP = 3,          /* a HIP runtime call or kernel launch failed */
    SCP_ERR_STATE = 4,        /* call out of order (e.g. admm_solve before scp_linearize) */
    SCP_ERR_UNSUPPORTED = 5   /* valid request the library cannot serve (e.g. block size) */
} scp_status;

/* Dynamics models (hand-derived device functions; a problem names a model id). */
typedef enum {
    SCP_MODEL_QUAD_PM = 1,    /* quadrotor point mass, nx=6 (p, v), nu=3 (u):
                                 p' = v, v' = u/m_s - g e3 - c |v| v                        */
    SCP_MODEL_MARS3DOF = 2,   /* 3-DOF powered descent in scaled units, nx=7 (r, v, m),
                                 nu=4 (T, Gamma): r' = v, v' = T/m + g_vec, m' = -alpha Gamma */
    SCP_MODEL_QUAD_6DOF = 3   /* 6-DOF rigid-body quadrotor (Sec. IV-A.1), nx=13 (p, v,
                                 unit quaternion q = (w, x, y, z), body rates w_b), nu=4
                                 (total thrust f, body torques tau):
                                 p' = v, v' = (f/m) R(q) e3 - g e3 + d,
                                 q' = q (x) (0, w_b) / 2, w_b' = J^-1 (tau - w_b x J w_b),
                                 m = SCP_P_MSCALE, g = SCP_P_GRAV, J = diag(SCP_P_INERTIA);
                                 R(q) e3 is the third column of the rotation matrix of
                                 q / |q| (a unit thrust direction off the unit sphere too) */,
    SCP_MODEL_LANDER6 = 4     /* 6-DOF powered descent (Sec. IV-B.1), unified units, nx=14
                                 (r, v Up-East-North, unit quaternion q, body rates w_b, mass
                                 m), nu=3 (body-frame thrust T): r' = v,
                                 v' = R(q/|q|) T / m + g (g = SCP_P_GVEC),
                                 q' = q (x) (0, w_b) / 2,
                                 J w_b' = r_T x T - w_b x J w_b (r_T = SCP_P_ARM),
                                 m' = -alpha |T| (alpha = SCP_P_ALPHA)                    */
} scp_model;

typedef enum { SCP_F32 = 0, SCP_F64 = 1 } scp_precision;

typedef enum {
    SCP_FORM_PLAIN = 0,       /* state in HBM; host-enqueued kernels per ADMM iteration       */
    SCP_FORM_PERSISTENT = 1   /* one kernel per SCP iteration (or per solve); every node's
                                 factor and ADMM state stay in registers/LDS.  For a batch of
                                 one 6-DOF model alone (at most 64 nodes per trajectory, no
                                 consensus groups, check_every = 0), and for lanes_per_node =
                                 4: linearization and acceptance as in the plain form, the
                                 ADMM iterations of each SCP iteration resident in one
                                 workgroup per trajectory, four lanes per node              */
} scp_form;

typedef enum { SCP_PACK_ALIGNED = 0, SCP_PACK_DENSE = 1 } scp_pack;

#define SCP_MAX_NX 14
#define SCP_MAX_NU 4
#define SCP_MAX_OBS 8
#define SCP_MAX_N 1023        /* largest horizon N (intervals) of one trajectory */

/*
 * Per-trajectory parameter record: SCP_PARAM_STRIDE doubles, in solver units.
 * Vectors are stored at the given offset with SCP_MAX_NX / SCP_MAX_NU slots; unused
 * trailing slots are ignored.  +-HUGE_VAL marks an absent bound.
 */
enum {
    SCP_P_H = 0,              /* step size T/N                                              */
    SCP_P_XINIT = 1,          /* [14] initial state, x_0 = x_init (eq. ocp)                 */
    SCP_P_XTGT = 15,          /* [14] terminal target                                       */
    SCP_P_TMASK = 29,         /* [14] 1.0 where x_N is fixed to the target (selection S)    */
    SCP_P_QR = 43,            /* [14] diagonal of the running state Hessian Q_i, i < N      */
    SCP_P_QN = 57,            /* [14] diagonal of the terminal Hessian Q_N                  */
    SCP_P_QNV = 71,           /* [14] terminal gradient q_N                                 */
    SCP_P_CN = 85,            /* constant of the terminal cost (reported cost only)         */
    SCP_P_R = 86,             /* [4] diagonal of the control Hessian R_i                    */
    SCP_P_XLO = 90,           /* [14] hard state lower bounds                               */
    SCP_P_XHI = 104,          /* [14] hard state upper bounds                               */
    SCP_P_ULO = 118,          /* [4] hard control lower bounds                              */
    SCP_P_UHI = 122,          /* [4] hard control upper bounds                              */
    SCP_P_UBALL = 126,        /* control ball radius ||u|| <= r (point-mass quadrotor;
                                 HUGE_VAL = none; ignored by the other models)              */
    SCP_P_DELTA = 127,        /* initial trust-region radius (l-inf box around the nominal) */
    SCP_P_DRAG = 128,         /* point-mass quadrotor drag coefficient c                    */
    SCP_P_MSCALE = 129,       /* quadrotor mass scale m_s (6-DOF quadrotor: the mass m)     */
    SCP_P_GRAV = 130,         /* quadrotor gravity g                                        */
    SCP_P_ALPHA = 131,        /* powered descent mass-flow coefficient alpha                */
    SCP_P_GVEC = 132,         /* [3] powered descent gravity vector                         */
    SCP_P_GLIDE = 135,        /* glide slope (powered descent, 6-DOF lander): the tangent
                                 of the cone's half angle about the vertical axis           */
    SCP_P_NOBS = 136,         /* number of obstacles K <= SCP_MAX_OBS (quadrotors)          */
    SCP_P_OBS = 137,          /* [8 x 4] obstacle centre (3) and radius (1)                 */
    SCP_P_DIST = 169,         /* [3] constant disturbance acceleration added to v'
                                 (quadrotors)                                               */
    SCP_P_CYL = 172,          /* bit j set: obstacle j is a vertical cylinder (axis along z
                                 through its centre; the centre's z is ignored), else a
                                 sphere                                                     */
    SCP_P_INERTIA = 173,      /* [3] principal moments of inertia J_xx, J_yy, J_zz (6-DOF)  */
    SCP_P_ARM = 176,          /* [3] 6-DOF lander: thrust point in the body frame           */
    SCP_P_TMIN = 179,         /* 6-DOF lander: thrust magnitude lower bound (non-convex;
                                 linearized at the nominal thrust each SCP iteration)       */
    SCP_P_TMAX = 180,         /* 6-DOF lander: thrust magnitude upper bound                 */
    SCP_P_GIMBAL = 181,       /* 6-DOF lander: tangent of the gimbal cone's half angle
                                 about the body x axis                                      */
    SCP_P_TILT = 182,         /* 6-DOF lander: tilt bound as |(q_y, q_z)| <= this value
                                 (the sine of half the largest tilt angle)                  */
    SCP_P_WMAX = 183,         /* 6-DOF lander: body-rate bound |w_b| <= this value          */
    SCP_PARAM_STRIDE = 184
};

/*
 * Per-trajectory info record written to device memory by scp_solve / admm_solve
 * (SCP_INFO_FIELDS doubles per trajectory).
 */
enum {
    SCP_I_ADMM_ITERS = 0,     /* ADMM iterations run (summed over SCP iterations)           */
    SCP_I_RP = 1,             /* last primal residual (inf-norm)                            */
    SCP_I_RD = 2,             /* last dual residual (inf-norm)                              */
    SCP_I_NACCEPT = 3,        /* accepted SCP steps                                         */
    SCP_I_DELTA = 4,          /* trust radius after the last SCP iteration                  */
    SCP_I_STATUS = 5,         /* SCP_ST_* bits                                              */
    SCP_I_DEFECT = 6,         /* max_i ||x_{i+1} - RK4(x_i, u_i)||_inf of the returned nominal */
    SCP_I_COST = 7,           /* objective of eq. (ocp) at the returned nominal             */
    SCP_I_VIOL = 8,           /* max violation of the hard (unconvexified) constraints      */
    SCP_I_BNDERR = 9,         /* boundary-condition error                                   */
    SCP_I_MERIT = 10,         /* merit of the last candidate                                */
    SCP_I_RATIO = 11,         /* last actual/predicted merit reduction ratio                */
    SCP_INFO_FIELDS = 12
};

/* status bits of SCP_I_STATUS */
#define SCP_ST_NONFINITE 1    /* a non-finite iterate or merit was produced                 */
#define SCP_ST_BADPIVOT 2     /* non-positive Cholesky pivot (H_i not positive definite)   */
#define SCP_ST_EMPTYSET 4     /* a hard box has lo > hi                                     */
#define SCP_ST_CONVERGED 8    /* ADMM residual test passed in the last SCP iteration        */
#define SCP_ST_SYNC 16        /* a consensus group spanning several workgroups waited too
                                 long at a group barrier (scp_params.group_wait_ms); set on
                                 every member of the group, whose results are invalid      */
#define SCP_ST_DIVERGED 32    /* residual blow-up (scp_params.detect_blowup): at the
                                 acceptance step of an SCP iteration, the primal residual of
                                 its last ADMM iteration exceeded SCP_RP_BLOWUP times the
                                 first positive one since the problem was created or reset
                                 (a served request: admitted).  Set by scp_solve and the
                                 server only (admm_solve has no acceptance step).            */
#define SCP_RP_BLOWUP 1.0e6

typedef struct {
    int32_t n_traj;           /* number of trajectories, >= 1                              */
    scp_precision prec;       /* arithmetic of every kernel of this problem                 */
    const int32_t* model;     /* [n_traj] scp_model                                         */
    const int32_t* horizon;   /* [n_traj] N, 1 <= N <= SCP_MAX_N                            */
    const int32_t* group;     /* [n_traj] consensus group id, or -1; members of one group
                                 are consecutive and share model and N; their first
                                 controls are averaged at every ADMM iteration (scenario
                                 MPC, Sec. IV-A.4).  NULL = every trajectory alone.  In the
                                 persistent form a group larger than one workgroup spans
                                 several (at most 64 members, each member whole in one
                                 workgroup), coupled by a barrier in device memory.  Groups
                                 of the 6-DOF lander are refused (SCP_ERR_ARG).             */
    const double* params;     /* [n_traj * SCP_PARAM_STRIDE] records, see SCP_P_*           */
    const double* x_guess;    /* initial nominal states, rows of SCP_MAX_NX doubles, (N+1)
                                 rows per trajectory, trajectories concatenated             */
    const double* u_guess;    /* initial nominal controls, rows of SCP_MAX_NU doubles, N
                                 rows per trajectory                                        */
    int32_t block;            /* workgroup size of the persistent kernel: 64, 128 or 256
                                 (0 = smallest that holds the longest trajectory or group) */
    int32_t pack;             /* SCP_PACK_ALIGNED: a trajectory of at most 64 nodes never
                                 straddles a wavefront, so workgroups without longer ones
                                 exchange neighbour values inside the wavefront;
                                 SCP_PACK_DENSE: first-fit over the whole workgroup (fewer
                                 idle lanes, LDS exchange when the workgroup has several
                                 wavefronts).  Results do not depend on it.               */
} scp_problem_desc;

typedef struct {
    double rho_eq, rho_dyn, rho_geo;  /* penalties of eq. (augmented_lagrangian), > 0        */
    int32_t max_iters;                /* ADMM iterations per call / per SCP iteration       */
    int32_t check_every;              /* residual test cadence c (0 = never stop early)     */
    double eps_prim, eps_dual;        /* stop when r_p <= eps_prim and r_d <= eps_dual      */
} admm_params;

typedef struct {
    int32_t scp_iters;                /* SCP iterations                                      */
    admm_params admm;
    double eta0;                      /* accept a step if ratio >= eta0 (-HUGE_VAL: always) */
    double eta1, eta2;                /* shrink below eta1, grow above eta2                 */
    double shrink, grow, delta_max;   /* trust-radius update factors and cap                */
    double merit_w;                   /* weight of the l1 dynamics defect in the merit      */
    scp_form form;                    /* plain (HBM state) or persistent kernel             */
    int32_t scp_per_launch;           /* persistent form: SCP iterations per kernel launch
                                         (0 = all in one launch)                            */
    double rho_final;                 /* > 0: penalty schedule (Sec. IV-A.2 parameter study):
                                         rho_eq grows geometrically from admm.rho_eq at the first
                                         SCP iteration to rho_final at the last (ratio
                                         (rho_final/rho_eq)^(1/(scp_iters-1)) in double, factors
                                         by repeated multiplication), rho_dyn and rho_geo keep
                                         their ratios to rho_eq, duals carry over unscaled.
                                         0: fixed penalties.                                  */
    int32_t graph;                    /* 1: the first call with these parameters captures its
                                         whole launch sequence into a hipGraph kept by the
                                         handle, later calls with equal parameters replay it.
                                         Needs a stream other than the legacy default stream
                                         (SCP_ERR_HIP otherwise).  0: direct launches.        */
    double adapt_mu;                  /* > 1: adaptive penalty by residual balancing (Boyd et
                                         al. 2011, Sec. 3.4.1; the paper gives no adaptive
                                         rule): after each SCP iteration a trajectory's three
                                         penalties are multiplied by adapt_tau when its primal
                                         residual of the last ADMM iteration exceeds adapt_mu
                                         times the dual one, divided by adapt_tau when the dual
                                         residual exceeds adapt_mu times the primal one
                                         (compared in double), on top of the schedule's factor;
                                         the next SCP iteration factors with the new penalties
                                         and the duals carry over unscaled.  Each scp_solve call
                                         starts from factor 1.  Needs check_every = 0 and no
                                         consensus groups (SCP_ERR_UNSUPPORTED otherwise).
                                         0: off.                                              */
    double adapt_tau;                 /* > 1 when adapt_mu > 0                                */
    double group_wait_ms;             /* persistent form with consensus groups spanning several
                                         workgroups: longest wait at one group barrier before the
                                         whole group is flagged SCP_ST_SYNC (0 = 20 ms; < 0 = give
                                         up at the first wait, which exercises the failure path).
                                         Once a member gives up, every member of the group stops
                                         waiting and reports SCP_ST_SYNC.                       */
    int32_t lanes_per_node;           /* persistent form, lanes of a wavefront that share one
                                         node: 1 = one lane per node, the whole solve in one
                                         fused kernel (point-mass quadrotor, powered descent);
                                         4 = lane groups of four (DPP quad exchanges): the node's
                                         components, factor rows and A, B columns split over the
                                         four lanes, ADMM iterations resident in one workgroup per
                                         trajectory, linearization and acceptance as in the plain
                                         form (at most 64 nodes per trajectory, no consensus
                                         groups, check_every = 0; the only form of the 6-DOF
                                         models).  0 = the model's default (1 for the point-mass
                                         quadrotor and powered descent, 4 for the 6-DOF models).
                                         A combination the batch does not allow returns
                                         SCP_ERR_UNSUPPORTED.  Results agree within rounding
                                         (the sums run in another order).                        */
    int32_t detect_blowup;            /* 1: residual blow-up detection (SCP_ST_DIVERGED), in
                                         every form; the persistent form then runs a kernel
                                         variant that carries the tracking.  0: off.             */
} scp_params;

typedef struct scp_problem scp_problem;

/* HBM footprint in bytes of the arena scp_problem_create() needs for this description;
 * 0 if the description is invalid.  Pure host computation. */
size_t scp_problem_device_bytes(const scp_problem_desc* desc);

/* Validate the description, lay out the arena, upload problem data and initial nominal
 * (converted to the problem precision), and return a handle.  arena_dev must hold at
 * least scp_problem_device_bytes(desc) bytes of device memory, 256-byte aligned.  The
 * upload is enqueued on hip_stream (a hipStream_t, NULL = default stream) and the call
 * waits for it.  Errors: SCP_ERR_ARG (bad description or arena), SCP_ERR_HIP. */
scp_status scp_problem_create(const scp_problem_desc* desc, void* arena_dev, size_t arena_bytes,
                              void* hip_stream, scp_problem** out);

/* Size of the no-allocation arena of scp_problem_create_noalloc: one fixed device array of this
 * many bytes per GPU, part of the library's device image and held until the process ends. */
#define SCP_NOALLOC_MAX_BYTES (32u << 20)

/* scp_problem_create for callers that cannot allocate device memory (code under HIP graph capture
 * of later calls, tight serving loops, harnesses that forbid allocation): the same problem, laid
 * out and uploaded exactly as scp_problem_create does, but in the library's fixed no-allocation
 * arena of the current device (SCP_NOALLOC_MAX_BYTES) instead of caller memory.  The call allocates
 * no device memory (no hipMalloc / hipFree, no allocating library routine); every later call on
 * the handle (scp_solve, scp_get_result, ...) works as for a caller arena and produces the same
 * bits.  The arena is cleared at create (as scp_problem_create clears a caller arena), so nothing
 * is left over from an earlier problem.
 * One arena per device: while a handle made by this call is alive, another call on the same device
 * returns SCP_ERR_STATE; scp_problem_destroy releases it.  Work of a destroyed handle still queued
 * on its stream and a new handle's work on another stream overlap in the same memory and race: the
 * caller orders them (same stream, or a synchronization in between).
 * Errors: SCP_ERR_ARG (invalid description, or a problem larger than SCP_NOALLOC_MAX_BYTES, whose
 * size scp_problem_device_bytes gives), SCP_ERR_STATE (arena in use), SCP_ERR_HIP. */
scp_status scp_problem_create_noalloc(const scp_problem_desc* desc, void* hip_stream, scp_problem** out);

/* Release host resources of the handle; never frees arena_dev.  NULL is ignored. */
void scp_problem_destroy(scp_problem* p);

/* Steps a2-a4 at the current nominal (Sec. III-A; Sec. III-B Step 1 factorization):
 * RK4 linearization with exact Jacobians, convexified constraint sets (trust box with the
 * current radius, boundary equalities, obstacle half-spaces), Step-1 Hessians and their
 * unpivoted Cholesky factors (for the 6-DOF quadrotor in FP32, then the inverse of each
 * Hessian computed from its factor, which Step 1 multiplies by), and re-initialization of the
 * ADMM primal state from the nominal (duals are carried).  Uses rho from the last admm_params given to admm_solve or
 * scp_solve, or rho = 1 before any.  Async on the handle's stream. */
scp_status scp_linearize(scp_problem* p, const admm_params* prm);

/* Steps a5-a9: up to prm->max_iters ADMM iterations (Steps 1-4) on the subproblem built by
 * the last scp_linearize, continuing from the state in the arena, with the residual test
 * every prm->check_every iterations (per trajectory / consensus group).  The penalties must
 * equal those given to scp_linearize (SCP_ERR_ARG otherwise).  Plain form.  Async. */
scp_status admm_solve(scp_problem* p, const admm_params* prm);

/* Steps a2-a10 repeated prm->scp_iters times from the current nominal, including the merit
 * ratio test, nominal update and trust-radius update, then the metrics of the final
 * nominal (defect, cost, violation, boundary error) into the info records.  Async. */
scp_status scp_solve(scp_problem* p, const scp_params* prm);

/* Restore the initial guess given at create time as the nominal, set every ADMM iterate and
 * dual to zero, the trust radius to its initial value and the info records to zero: the next
 * scp_solve is then a fresh solve (instead of a warm start from the last one).  Async. */
scp_status scp_reset(scp_problem* p);

/* Checkpoint and resume.  The paper's only form of resumption is the MPC warm start (Sec.
 * IV-A.4: the previous solution, shifted, seeds the next solve); these calls make any solve
 * resumable across handles and processes.  The state is everything a later call reads: the
 * nominal, the linearization and factors, the ADMM iterates and duals, the trust radii, the info
 * records and flags (the whole arena, which holds offsets only, never addresses), plus the
 * handle's host-side state (whether a linearization is current, and its penalties).
 *
 * scp_problem_state_bytes: size of an exported state (a header plus the arena bytes).
 * scp_problem_export_state: waits for the handle's stream, then copies the state into `host`
 *   (>= scp_problem_state_bytes bytes, any host memory).  Errors: SCP_ERR_ARG (NULL or too
 *   small), SCP_ERR_HIP.
 * scp_problem_import_state: restores a state exported from a handle created with the same
 *   description (same trajectories, horizons, models, groups, precision and packing; checked by
 *   a fingerprint of the layout in the header), enqueued on the handle's stream after its
 *   earlier work; returns after the copy, so `host` may be reused at once.  The next scp_solve
 *   or admm_solve then continues exactly as the exporting handle would have (bitwise, on the
 *   same device).  Errors: SCP_ERR_ARG (NULL, wrong size, or a state of another layout),
 *   SCP_ERR_HIP. */
size_t scp_problem_state_bytes(const scp_problem* p);
scp_status scp_problem_export_state(scp_problem* p, void* host, size_t bytes);
scp_status scp_problem_import_state(scp_problem* p, const void* host, size_t bytes);

/* Copy the nominal trajectory and info to caller device buffers (device-to-device, async):
 * x_dev gets rows of SCP_MAX_NX values per node (all trajectories concatenated, N+1 rows
 * each), u_dev rows of SCP_MAX_NU values (N+1 rows per trajectory, the last row zero), both
 * in the problem precision; info_dev gets SCP_INFO_FIELDS doubles per trajectory.  Any of
 * the three may be NULL. */
scp_status scp_get_result(const scp_problem* p, void* x_dev, void* u_dev, void* info_dev);

/* Field ids of scp_get_field: the ADMM iterates and linearization data of every node. */
typedef enum {
    SCP_FIELD_XBAR = 0, SCP_FIELD_UBAR = 1, SCP_FIELD_X = 2, SCP_FIELD_U = 3,
    SCP_FIELD_Z = 4, SCP_FIELD_LAM = 5, SCP_FIELD_MU = 6, SCP_FIELD_DDYN = 7,
    SCP_FIELD_COPY = 8, SCP_FIELD_DUAL = 9, SCP_FIELD_A = 10, SCP_FIELD_B = 11,
    SCP_FIELD_D = 12, SCP_FIELD_BOXLO = 13, SCP_FIELD_BOXHI = 14, SCP_FIELD_HS = 15,
    SCP_FIELD_COUNT = 16
} scp_field;

/* Width (values per node) of a field: XBAR/X/Z/LAM/MU/DDYN/D 14, UBAR/U 4, COPY/DUAL 44,
 * A 196 (row-major 14x14), B 56 (row-major 14x4), BOXLO/BOXHI 18 (x then u), HS 32
 * (a_x, a_y, a_z, b per obstacle).  A model's values fill the leading slots (its nx, nu
 * rows and columns); the rest are 0.  0 for an invalid id. */
int32_t scp_field_width(int32_t field);

/* Copy one field of every node (trajectories concatenated, N+1 rows each, scp_field_width
 * values per row, problem precision) to dst_dev.  Mirror copies and duals are packed per
 * model in a fixed group order: point-mass quadrotor [x box 6][u box 3][ball 3][half-space k:
 * 3 each], 6-DOF quadrotor [x box 13][u box 4][ball 3, unused][half-space k: 3 each],
 * powered descent [x box 7][u box 4][glide cone 3][SOC 4], 6-DOF lander [x box 14][u box 3]
 * [glide cone on (r_E, r_N, r_U) 3][tilt on (q_y, q_z) 2][rate ball 3][thrust ball 3]
 * [thrust lower-bound half-space 3][gimbal cone on (T_y, T_z, T_x) 3].  Async. */
scp_status scp_get_field(const scp_problem* p, int32_t field, void* dst_dev);

/* Total nodes (sum of N+1) and the node offset of trajectory t (for slicing results). */
int64_t scp_problem_nodes(const scp_problem* p);
int64_t scp_traj_node_offset(const scp_problem* p, int32_t t);

/* Host-side plan of the persistent form for a description (pure host computation, no
 * device access): plan[0] workgroup size, plan[1] workgroups, plan[2] workgroups whose
 * trajectories straddle a wavefront (LDS neighbour exchange), plan[3] idle lanes, plan[4]
 * consensus groups spanning several workgroups.  If
 * lane_table is not NULL and lane_cap >= plan[0] * plan[1], it receives the node index
 * (trajectory offset + node) of every lane, -1 for idle lanes.  plan[0] = 0 if no block
 * holds the longest trajectory or group (the persistent form is then unavailable).
 * Errors: SCP_ERR_ARG (invalid description, NULL plan). */
scp_status scp_plan(const scp_problem_desc* desc, int32_t plan[5], int32_t* lane_table, size_t lane_cap);

/* Autotuner of the persistent form (the knobs do not change what is computed, except the
 * residual-test cadence, which decides at which iteration a converged trajectory stops). */
typedef struct {
    int32_t block;        /* workgroup size                                          */
    int32_t pack;         /* scp_pack                                                */
    int32_t check_every;  /* residual-test cadence c                                 */
    int32_t valid;        /* 0 if the candidate does not fit (no timing)             */
    double ms;            /* mean wall time of one fresh solve on the device, in ms  */
    int32_t lanes;        /* lanes per node (scp_params.lanes_per_node)              */
} scp_tune_entry;

/* Largest arena any candidate of scp_autotune needs (pure host computation); 0 if the
 * description is invalid. */
size_t scp_autotune_device_bytes(const scp_problem_desc* desc);

/* Time every candidate (lanes per node 1: block in {64, 128, 256} (FP64: {64, 128}), pack in
 * {aligned, dense}; lanes per node 4: its one workgroup size; each with check_every in
 * cadences[0..n_cad-1]; a lane-group candidate is valid only for check_every = 0 and batches it
 * holds) on the description's own problem: each candidate
 * builds the problem in arena_dev, runs one untimed fresh solve with prm (form forced to
 * persistent) and then `reps` timed fresh solves (HIP events on hip_stream).  Writes up to
 * table_cap entries to table (n_out = number of candidates) and the fastest valid one to
 * best.  Synchronizes the stream; the arena's contents are undefined afterwards.  Results are
 * cached per process, keyed by the description's shape (precision, models, horizons, groups)
 * and the parameters: a repeated call returns the cached best with *n_out = 0.
 * Errors: SCP_ERR_ARG, SCP_ERR_HIP, SCP_ERR_UNSUPPORTED (no candidate fits). */
scp_status scp_autotune(const scp_problem_desc* desc, const scp_params* prm, const int32_t* cadences, int32_t n_cad,
                        int32_t reps, void* arena_dev, size_t arena_bytes, void* hip_stream,
                        scp_tune_entry* table, int32_t table_cap, int32_t* n_out, scp_tune_entry* best);

/* Message of the last failed call on this handle ("" if none); for p == NULL, the last
 * error of a failed scp_problem_create, scp_plan or scp_autotune in this thread. */
const char* scp_last_error(const scp_problem* p);

#ifdef __cplusplus
}
#endif
#endif /* SCP_MI355X_H */

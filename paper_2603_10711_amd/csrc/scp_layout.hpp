// Arena layout shared by the host API and the kernels.
//
// Node data is stored component-plane major ("SoA"): value k of node g lives at
// planes[k * P + g], P = node count padded to a multiple of 256, so consecutive lanes of a
// wavefront touch consecutive addresses.  Plane blocks are sized for the largest model of each
// (nx <= 14, nu <= 4, n <= 17, 44 mirror slots); smaller models use a prefix of each block.  The
// nominal, physical and guess blocks keep x and u adjacent (x block, then u block).
#pragma once

#include <stdint.h>

namespace scp {

enum Plane : int {
    PL_XBAR = 0,    // 14  nominal state
    PL_UBAR = 14,   // 4   nominal control (row N zero)
    PL_X = 18,      // 14  physical state
    PL_U = 32,      // 4   physical control
    PL_Z = 36,      // 14  dynamic auxiliary z
    PL_LAM = 50,    // 14  lambda
    PL_MU = 64,     // 14  mu
    PL_DD = 78,     // 14  d_dyn = A x + B u + d
    PL_CP = 92,     // 44  mirror copies
    PL_DU = 136,    // 44  mirror duals
    PL_AR = 180,    // 154 non-unit columns of A (row-major NX x NXR)
    PL_B = 334,     // 52  B (row-major NX x NU)
    PL_D = 386,     // 14  d
    PL_L = 400,     // 153 packed Cholesky factor (diagonal slots hold reciprocals)
    PL_LO = 553,    // 17  box lower bounds (x then u)
    PL_HI = 570,    // 17  box upper bounds
    PL_HS = 587,    // 32  half-spaces (a_x, a_y, a_z, b) per obstacle / thrust bound
    PL_G0 = 619,    // 14  constant Step-1 right-hand side (x part)
    PL_DZ = 633,    // 14  z - z_old (residual iterations)
    PL_SP = 647,    // 17  node-local part of the dual residual vector
    PL_RP = 664,    // 1   node primal residual
    PL_MER = 665,   // 8   merit / metric terms of one node
    PL_XG = 673,    // 14  initial guess of the states (restored by scp_reset)
    PL_UG = 687,    // 4   initial guess of the controls
    NPLANES = 691
};

// mirror slots of the largest model (the PL_CP / PL_DU block width)
constexpr int MAX_C = 44;
// Largest state dimension and mirror-slot count among the models the persistent kernel and the
// request server run (point-mass quadrotor, powered descent); their workgroup exchange arrays
// are sized by these.
constexpr int PERSIST_MAX_NX = 7;
// Longest trajectory (nodes) whose ADMM iterations run resident in one workgroup (6-DOF quadrotor,
// four lanes per node, at most 256 lanes)
constexpr int RESIDENT_MAX_NODES = 64;
constexpr int PERSIST_MAX_C = 36;

// merit / metric term slots inside PL_MER
enum : int { MER_COST_NOM = 0, MER_PEN_NOM = 1, MER_COST_NEW = 2, MER_PEN_NEW = 3, MER_PEN_MOD = 4,
             MER_DEFECT = 5, MER_VIOL = 6, MER_BND = 7 };

// per-trajectory integer record
enum : int { TR_MODEL = 0, TR_N = 1, TR_OFF = 2, TR_GFIRST = 3, TR_GSIZE = 4, TR_K = 5, TR_BALL = 6,
             TR_MEMBER = 7, TR_FIELDS = 8 };

// per-trajectory runtime values (problem precision)
// RT_RP0: the first positive primal residual since create / reset / admission (blow-up reference),
// RT_RPMAX: the largest one since then
enum : int { RT_DELTA = 0, RT_RHOS = 1, RT_RP0 = 2, RT_RPMAX = 3, RT_FIELDS = 4 };

// per-trajectory integer flags
enum : int { FL_DONE = 0, FL_ITERS = 1, FL_ACCEPT = 2, FL_STATUS = 3, FL_FIELDS = 4 };

// Consensus groups larger than one workgroup ("spanning groups") get whole workgroups of their
// own and exchange their per-member values through HBM records: two buffers (alternating by
// the parity of the group barrier), GX_MEMBERS member rows of GX_WIDTH values each.  The
// group barrier counts workgroup arrivals in one 32-bit word per 128-byte line; the next word
// of that line is the group's failure word (nonzero once a member gave up waiting).
constexpr int GX_MEMBERS = 64;
constexpr int GX_WIDTH = 8;
constexpr int GX_SYNC_STRIDE = 32;
constexpr int GX_MAX_WG = 64;
// per-workgroup record: model id | straddling flag << 8 | spanning-group flag << 9
enum : int { WG_CROSS = 1 << 8, WG_SPAN = 1 << 9 };

// Server admission record (device staging): where a request goes in the pool and where its
// data sits in the staged blob (byte offsets).  Its trajectory records already hold pool node
// offsets and trajectory slots, its lane table pool node indices.
struct AdmitRec {
    int traj_first, n_traj, node_off, n_nodes, wg_first, n_wg;
    int warm;     // 1: shift the resident solution in place (MPC warm start)
    int x1_node;  // warm: pool node of scenario 0, node 1, of the previous solution
    int keep_xinit;  // warm: keep the request's x_init (measured state) instead of that node
    int o_traj, o_params, o_node_traj, o_lane, o_wginfo, o_wggroup, o_xg, o_ug;
};

// Server result record: a finished request's info, nominal states and controls go to the
// output staging at o_out (info doubles, then N+1 rows of SCP_MAX_NX and of SCP_MAX_NU values
// per trajectory).
struct CollectRec {
    int traj_first, n_traj, node_off, n_nodes;
    long long o_out;
};

template <class T>
struct Dev {
    const int* traj;       // [n_traj * TR_FIELDS]
    const int* node_traj;  // [P] trajectory of each node, -1 for padding
    const int* lane_node;  // [n_wg * block] node of each persistent-kernel lane, -1 idle
    const T* params;       // [n_traj * SCP_PARAM_STRIDE]
    T* planes;             // [NPLANES * P]
    T* rt;                 // [n_traj * RT_FIELDS]
    double* info;          // [n_traj * SCP_INFO_FIELDS]
    int* flags;            // [n_traj * FL_FIELDS]
    unsigned long long* red;  // [n_traj * 2] atomic max slots (r_p, r_d as double bit patterns)
    int n_traj;
    int P;
    int n_nodes;
    int n_groups;          // number of consensus groups with more than one member
    const int* groups;     // [n_groups] first trajectory of each such group
    // persistent form
    const int* wg_list;    // [grid] lane-table workgroup of each launched workgroup (NULL: identity)
    const int* wg_info;    // [n_wg] model | WG_CROSS | WG_SPAN
    const int* wg_group;   // [n_wg * 2] spanning group slot and its workgroup count (WG_SPAN only)
    unsigned* gsync;       // [n_gslots * GX_SYNC_STRIDE] barrier arrival counters
    T* gx;                 // [n_gslots * 2 * GX_MEMBERS * GX_WIDTH] exchange records
    int n_gslots;
};

template <class T>
struct KParams {
    T rho_eq, rho_dyn, rho_geo;
    T eps_p, eps_d;
    T eta0, eta1, eta2, shrink, grow, delta_max, merit_w;
    int max_iters, check_every;
    int n_scp;        // SCP iterations this launch (persistent form)
    int final_metrics;
    int reset_info;
    int has_groups;
    int iter_base;    // plain form: index of the first ADMM iteration of this launch batch
    // penalty schedule: the penalties of SCP iteration k of a launch are rho_base * s_k with
    // s_0 = sched_s0 and s_{k+1} = s_k * sched_q, in double (rho_base in double too)
    double rho_base[3];
    double sched_s0, sched_q;
    // adaptive penalty (residual balancing between SCP iterations): on when adapt_mu > 0; the
    // factor of trajectory t is rt[t * RT_FIELDS + RT_RHOS] and multiplies the penalties above
    double adapt_mu, adapt_tau;
    // spanning consensus groups: longest wait at one group barrier, in ticks of the device wall
    // clock (100 MHz), before the group is declared failed (0: give up at the first wait)
    unsigned long long spin_ticks;
    // residual blow-up detection (scp_params.detect_blowup): SCP_ST_DIVERGED on / off
    int blowup;
};

}  // namespace scp

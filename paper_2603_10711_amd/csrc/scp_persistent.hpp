// Persistent form of the hot path.
//
// One workgroup holds whole trajectories (and whole consensus groups), one lane per node.  For
// the SCP iterations of a launch every node keeps its linearization, Cholesky factor, box and
// half-space data and all ADMM iterates in registers; the only traffic between nodes is the
// neighbour exchange of the consensus step (d_dyn from node i-1, z and mu from node i+1) and
// the per-trajectory reductions, both through LDS.  HBM is touched once at launch start (nominal
// and duals) and once at the end (state write-back).
//
// Barriers per ADMM iteration: one after Step 1 (d_dyn published), one after Step 4 (z, mu
// published); consensus groups add one for the first-control average, residual iterations
// add three for the dual-residual neighbour term and the per-trajectory test.
//
// A consensus group too large for one workgroup spans several workgroups that hold nothing
// else.  Its four couplings (scenario mean of the nominal first control at the start of an SCP
// iteration, first-control copy average in every ADMM iteration, group residual test, group
// merit test) go through per-member records in HBM and a group barrier across those
// workgroups.  Every sum runs over members in member order, as in the single-workgroup case,
// so the results do not depend on whether a group spans workgroups.
#pragma once

#include "scp_device.hpp"
#include "scp_launch.hpp"
#include "scp_layout.hpp"

namespace scp {

// HSR: rows of half-space state (3 per half-space group; 1 where the kernel holds no half-space
// groups).
// A lane's column of a row-major LDS array [k][STRIDE], read as a packed vector.
template <class T, int STRIDE>
struct StridedLds {
    const T* p;
    __device__ __forceinline__ T operator[](int k) const { return p[k * STRIDE]; }
};

// One-wavefront workgroups exchange neighbours with DPP, so their exchange arrays shrink to one
// row; the LDS this frees holds the Cholesky factors instead (LR rows, 1 where unused): with the
// factor out of the registers, the ADMM state stays in VGPRs instead of spilling to AGPRs.
template <class T, int BLOCK, int HSR, int LR, int AR = 1>
struct Shared {
    static constexpr int XR = BLOCK == 64 ? 1 : PERSIST_MAX_NX;
    T ex[2 * XR][BLOCK + 1];       // z, mu of every node (backward exchange); x / xbar at accept;
                                   // column BLOCK stays 0 (the neighbour of the last lane)
    T fw[XR][BLOCK + 1];           // d_dyn of lane t in column t + 1 (forward exchange)
    T dz[XR][BLOCK];               // z - z_old (dual-residual neighbour term)
    T zo[PERSIST_MAX_NX][BLOCK];   // own z before Steps 2-3 on residual iterations
    T cpo[PERSIST_MAX_C][BLOCK];   // own copies before Step 3 on residual iterations
    T red[8][BLOCK];               // per-node terms for fixed-order trajectory sums
    T ucp[8][BLOCK];               // node-0 u copies of consensus groups
    unsigned long long mx[2][BLOCK];  // per-trajectory residual maxima, slot = first lane
    int flag[BLOCK];               // per-trajectory flags at the group leader lane
    int st[BLOCK];                 // per-trajectory status bits at the first lane
    int sync_fail;                 // a spanning-group barrier timed out
    T Lf[LR][BLOCK];               // packed Cholesky factor of every node (LDS-resident form)
    T hsp[HSR][BLOCK];             // half-space groups: carried-dual parts orthogonal to the new
                                   // normals (3 per group)
    T gxw[GX_WIDTH][BLOCK];        // spanning groups: member rows staged for publication
    int gxm[BLOCK];                // member index of the row staged at a lane, -1 none
    T arho[AR];                    // adaptive-penalty kernels (AR = BLOCK): the factor of the
                                   // lane's trajectory, own slot, out of the ADMM loop's registers
    T rp0[BLOCK];                  // residual blow-up tracking (TRACK kernels): the group's
    T rpm[BLOCK];                  // reference and largest primal residual, at the leader lane
};

// Spanning consensus group of a workgroup (on = false for every other workgroup).
struct Span {
    bool on;
    int slot;  // group slot: barrier counter and exchange records
    int nwg;   // workgroups of the group
};

template <class T>
__device__ __forceinline__ T* gx_row(const Dev<T>& dv, const Span& sp, unsigned nbar, int member) {
    return dv.gx + ((size_t)(sp.slot * 2 + (int)(nbar & 1u)) * GX_MEMBERS + member) * GX_WIDTH;
}

template <class T>
__device__ __forceinline__ T gx_read(const T* p) {
    return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Columns of a member row that hold node-0 u copies (the u box, then the ball's or the SOC's).
template <class M>
__device__ __forceinline__ constexpr int u_copy_cols() {
    int w = 0;
    for (int q = 0; q < M::C; ++q)
        if (slot_is_u<M>(q) && slot_comp_u<M>(q) + 1 > w) w = slot_comp_u<M>(q) + 1;
    return w;
}

// Value k of member m's row in the LDS copy that group_sync<W> gathers (see there).
template <int W, class T, int BLOCK, int HSR, int LR, int AR>
__device__ __forceinline__ T& gx_at(Shared<T, BLOCK, HSR, LR, AR>& sh, const int m, const int k) {
    const int f = m * W + k;
    return sh.ucp[f / BLOCK][f % BLOCK];
}

// Barrier over the workgroups of a spanning group, with the exchange of member rows.  Writer
// lanes stage their rows in LDS (gxw, gxm); wave 0 publishes them with agent-scope atomic
// stores; after a workgroup barrier, thread 0 arrives once with an agent-scope release (one L2
// write-back), polls the arrival counter with relaxed agent-scope loads (no cache maintenance
// per poll) and takes one agent-scope acquire fence (one L2 invalidation).  The workgroup then
// copies the rows with agent-scope atomic loads (the gather below).  Both fences are required on
// gfx950: without them arrivals and rows written on other XCDs can stay invisible.
// Failure: a workgroup that has waited spin ticks of the device wall clock (or finds the group's
// failure word set) gives up, sets the failure word and never waits again; it still arrives at
// every later barrier, so the counts stay consistent and every workgroup reaches the end of the
// kernel quickly.  Every member reads the failure word at the end of the launch and reports
// SCP_ST_SYNC, so a member that never had to wait (it found the counter already past its
// target) is flagged too.  nbar counts the group barriers this workgroup has passed in this
// launch; rows of barrier b live in buffer b & 1.
// Gather: after the barrier the whole workgroup copies the first W values of every member row
// into LDS (gx_at), every thread issuing all of its loads before it waits for any, so the group
// pays one memory latency instead of one per member and value (a reader summing S rows straight
// from HBM waits S x W times).  All GX_MEMBERS rows are copied (rows past the group's size are
// never read), so the count is the same in every thread.  A spanning workgroup holds one group
// and never uses the in-workgroup consensus array ucp, which holds the copy.
template <int W, class T, int BLOCK, int HSR, int LR, int AR>
__device__ __forceinline__ void group_sync(const Dev<T>& dv, Shared<T, BLOCK, HSR, LR, AR>& sh, const Span& sp, unsigned& nbar,
                                           const int t, const unsigned long long spin) {
    static_assert(W >= 1 && W <= GX_WIDTH && GX_MEMBERS * W <= 8 * BLOCK, "gather does not fit ucp");
    __syncthreads();
    if (t < 64) {
        for (int j = t; j < BLOCK; j += 64) {
            const int m = sh.gxm[j];
            if (m >= 0) {
                T* row = gx_row(dv, sp, nbar, m);
#pragma unroll
                for (int k = 0; k < GX_WIDTH; ++k)
                    __hip_atomic_store(row + k, sh.gxw[k][j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                sh.gxm[j] = -1;
            }
        }
    }
    __syncthreads();
    nbar += 1u;
    if (t == 0) {
        unsigned* c = dv.gsync + (size_t)sp.slot * GX_SYNC_STRIDE;
        __hip_atomic_fetch_add(c, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (!sh.sync_fail) {
            const unsigned target = nbar * (unsigned)sp.nwg;
            const unsigned long long t0 = wall_clock64();
            while (__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                if (wall_clock64() - t0 >= spin ||
                    __hip_atomic_load(c + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                    sh.sync_fail = 1;
                    __hip_atomic_fetch_or(c + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    constexpr int NPER = (GX_MEMBERS * W + BLOCK - 1) / BLOCK;
    T v[NPER];
#pragma unroll
    for (int i = 0; i < NPER; ++i) {
        const int f = t + i * BLOCK;
        v[i] = f < GX_MEMBERS * W ? gx_read(gx_row(dv, sp, nbar - 1u, f / W) + f % W) : T(0);
    }
#pragma unroll
    for (int i = 0; i < NPER; ++i) {
        const int f = t + i * BLOCK;
        if (f < GX_MEMBERS * W) sh.ucp[f / BLOCK][f % BLOCK] = v[i];
    }
    __syncthreads();
}

// WAVE1: no trajectory of this workgroup straddles a wavefront boundary, so neighbour values
// move with DPP wavefront shifts instead of LDS and the two exchange barriers of every ADMM
// iteration disappear.  The per-trajectory reductions still go through LDS.
// ADAPT: the adaptive penalty (residual balancing between SCP iterations) is on; a kernel variant
// of its own, so the fixed-penalty kernels compile without it.
template <class M, class T, int BLOCK, bool WAVE1, bool SPAN, bool ADAPT, bool TRACK, int HSR, int LR, int AR>
__device__ __forceinline__ void persistent_body(const Dev<T>& dv, const KParams<T>& kp,
                                                Shared<T, BLOCK, HSR, LR, AR>& sh, const int t, const int gn,
                                                const Span span_in) {
    // SPAN: this kernel variant may hold spanning groups (compiled out of the other variant)
    const Span span{SPAN && span_in.on, span_in.slot, span_in.nwg};
    constexpr int NX = M::NX, NU = M::NU, NN = M::NN, NXR = M::NXR, C = M::C;
    const int P = dv.P;
    const bool valid = gn >= 0;
    NodeId id{0, 0, 0, false};
    int tr = 0, tb = t, lb = t, S = 1, mem = 0;
    unsigned nbar = 0;
    const T* prm = dv.params;
    if (valid) {
        tr = dv.node_traj[gn];
        const int* rec = dv.traj + tr * TR_FIELDS;
        id.i = gn - rec[TR_OFF];
        id.N = rec[TR_N];
        id.K = rec[TR_K];
        id.ball = rec[TR_BALL] != 0;
        tb = t - id.i;
        S = rec[TR_GSIZE];
        mem = rec[TR_MEMBER];
        // members of a spanning group lead themselves; their group reductions go through HBM
        lb = span.on ? tb : tb - mem * (id.N + 1);
        prm = dv.params + (size_t)tr * SCP_PARAM_STRIDE;
    }
    const bool first_lane = valid && id.first();
    const bool leader = first_lane && lb == tb;
    Rho<T> rho{};
    double sfac = kp.sched_s0;  // penalty-schedule factor of the current SCP iteration
    const T ball_r = valid ? prm[SCP_P_UBALL] : T(0);
    const T kappa = valid ? prm[SCP_P_GLIDE] : T(1);
    const T inv1k2 = T(1) / (T(1) + kappa * kappa);
    T delta = valid ? dv.rt[tr * RT_FIELDS + RT_DELTA] : T(0);
    // residual blow-up tracking of the group (the same in every member: they share the residual),
    // in LDS at the group leader's lane, out of the registers of the ADMM loop
    if constexpr (TRACK) {
        if (leader) {
            sh.rp0[t] = dv.rt[tr * RT_FIELDS + RT_RP0];
            sh.rpm[t] = dv.rt[tr * RT_FIELDS + RT_RPMAX];
        }
    }

    T xbar[NX], ubar[NU];
    NodeState<M, T> s;
    NodeConst<M, T> nc;
#pragma unroll
    for (int r = 0; r < NX; ++r) {
        xbar[r] = valid ? dv.planes[(size_t)(PL_XBAR + r) * P + gn] : T(0);
        s.lam[r] = valid ? dv.planes[(size_t)(PL_LAM + r) * P + gn] : T(0);
        s.mu[r] = valid ? dv.planes[(size_t)(PL_MU + r) * P + gn] : T(0);
        s.z[r] = T(0);
        s.dd[r] = T(0);
        s.x[r] = T(0);
    }
#pragma unroll
    for (int r = 0; r < NU; ++r) {
        ubar[r] = (valid && !id.last()) ? dv.planes[(size_t)(PL_UBAR + r) * P + gn] : T(0);
        s.u[r] = T(0);
    }
#pragma unroll
    for (int k = 0; k < C; ++k) {
        s.du[k] = valid ? dv.planes[(size_t)(PL_DU + k) * P + gn] : T(0);
        s.cp[k] = T(0);
    }
    int status = 0;
    int n_acc = 0, iters_sum = 0;
    // half-space groups in scalar form (quadrotor): dual -rho sig a, Step-1 coefficient rho kap
    constexpr bool HSQ = (M::ID == SCP_MODEL_QUAD_PM) && (M::KM > 0);
    constexpr int HSN = HSQ ? M::KM : 1;
    static_assert(!HSQ || HSR == 3 * HSN, "half-space rows of the workgroup state");
    constexpr bool LDSL = LR >= Dims<M>::NL;  // the factor lives in LDS
    static_assert(WAVE1 || Shared<T, BLOCK, HSR, LR, AR>::XR == PERSIST_MAX_NX, "LDS exchange needs full rows");
    static_assert(M::NX <= PERSIST_MAX_NX && M::C <= PERSIST_MAX_C, "model too large for the workgroup state");
    T sig[HSN], kap[HSN];
#pragma unroll
    for (int q = 0; q < HSN; ++q) sig[q] = kap[q] = T(0);
    if constexpr (HSQ) {
#pragma unroll
        for (int q = 0; q < M::NHS; ++q) nc.hs[q] = T(0);  // idle lanes: no half-spaces
    }
    T nr = T(0);          // rho_geo times the number of half-space groups at this node
    T ehs[3] = {T(0), T(0), T(0)};  // orthogonal remainders' Step-1 term for the coming iteration
    int last_iters = 0;   // ADMM iterations this lane ran in the last SCP iteration
    T rp_last = T(0), rd_last = T(0), ratio_last = T(0), merit_last = T(0);
    bool conv_last = false;
    if (t < BLOCK) {
        sh.mx[0][t] = 0ull;
        sh.mx[1][t] = 0ull;
        sh.st[t] = 0;
    }
    if (t == 0) sh.sync_fail = 0;
    if constexpr (!WAVE1) {
        if (t < 2 * PERSIST_MAX_NX) sh.ex[t][BLOCK] = T(0);
        if (t < PERSIST_MAX_NX) sh.fw[t][0] = T(0);
    }
    if (t < BLOCK) sh.gxm[t] = -1;
    if constexpr (ADAPT) sh.arho[t] = valid ? dv.rt[tr * RT_FIELDS + RT_RHOS] : T(1);

    for (int k = 0; k < kp.n_scp; ++k, sfac *= kp.sched_q) {
        {
            // schedule factor, then the adaptive factor: (rho_base * s_k) * f
            auto pen = [&](double base) -> T {
                if constexpr (ADAPT) return T(base * sfac * (double)sh.arho[t]);
                return T(base * sfac);
            };
            const T re = pen(kp.rho_base[0]), rd = pen(kp.rho_base[1]), rg = pen(kp.rho_base[2]);
            rho = Rho<T>{re, rd, rg, T(1) / rg, T(1) / (re + rd)};
        }
        // ---------------- a2: linearization at the nominal ----------------
        T F[NX];
        if (valid && !id.last()) {
            linearize<M, T>(prm, xbar, ubar, F, nc.Ar, nc.B, nc.d);
        } else {
#pragma unroll
            for (int q = 0; q < NX * NXR; ++q) nc.Ar[q] = T(0);
#pragma unroll
            for (int q = 0; q < NX * NU; ++q) nc.B[q] = T(0);
#pragma unroll
            for (int q = 0; q < NX; ++q) nc.d[q] = F[q] = T(0);
        }
        // nominal merit terms and the scenario mean of the first controls
        T xn0[NX];
        if constexpr (WAVE1) {
#pragma unroll
            for (int r = 0; r < NX; ++r) xn0[r] = lane_next(xbar[r]);
        } else {
#pragma unroll
            for (int r = 0; r < NX; ++r) sh.ex[r][t] = xbar[r];
        }
#pragma unroll
        for (int r = 0; r < NU; ++r) sh.red[r][t] = ubar[r];
        __syncthreads();
        if constexpr (!WAVE1) {
#pragma unroll
            for (int r = 0; r < NX; ++r) xn0[r] = sh.ex[r][t + 1 < BLOCK ? t + 1 : t];
        }
        T uc[NU];
#pragma unroll
        for (int r = 0; r < NU; ++r) uc[r] = ubar[r];
        T pen_nom = T(0);
        if (valid) {
            if (!id.last()) {
#pragma unroll
                for (int r = 0; r < NX; ++r) pen_nom = pen_nom + tabs(xn0[r] - F[r]);
            }
            if (id.first() && S > 1 && !span.on) {
                T acc[NU];
#pragma unroll
                for (int r = 0; r < NU; ++r) acc[r] = T(0);
                for (int m = 0; m < S; ++m) {
                    const int lm = lb + m * (id.N + 1);
#pragma unroll
                    for (int r = 0; r < NU; ++r) acc[r] = acc[r] + sh.red[r][lm];
                }
#pragma unroll
                for (int r = 0; r < NU; ++r) uc[r] = acc[r] / T(S);
            }
        }
        if (span.on) {
            const bool g0 = valid && id.first();
            if (g0) {
#pragma unroll
                for (int r = 0; r < NU; ++r) sh.gxw[r][t] = ubar[r];
                sh.gxm[t] = mem;
            }
            group_sync<NU>(dv, sh, span, nbar, t, kp.spin_ticks);
            if (g0) {
                T acc[NU];
#pragma unroll
                for (int r = 0; r < NU; ++r) acc[r] = T(0);
                for (int m = 0; m < S; ++m) {
#pragma unroll
                    for (int r = 0; r < NU; ++r) acc[r] = acc[r] + gx_at<NU>(sh, m, r);
                }
#pragma unroll
                for (int r = 0; r < NU; ++r) uc[r] = acc[r] / T(S);
            }
        }
        const T cost_nom = valid ? node_cost<M, T>(prm, id, xbar, ubar) : T(0);
        __syncthreads();

        // ---------------- a3 / a4: convex sets, Step-1 factor ----------------
        if (valid) {
            status |= convexify<M, T>(prm, id, xbar, uc, delta, nc);
            status |= assemble_factor<M, T>(prm, id, rho, nc);
        }
        if constexpr (LDSL) {
#pragma unroll
            for (int q = 0; q < Dims<M>::NL; ++q) sh.Lf[q][t] = nc.L[q];
        }
        // primal re-initialization from the nominal; duals carried
#pragma unroll
        for (int r = 0; r < NX; ++r) {
            s.x[r] = xbar[r];
            s.z[r] = id.first() ? T(0) : xbar[r];
        }
#pragma unroll
        for (int r = 0; r < NU; ++r) s.u[r] = ubar[r];
#pragma unroll
        for (int q = 0; q < C; ++q)
            s.cp[q] = (valid && group_active<M>(id, slot_group<M>(q))) ? slot_var<M, T>(s, q) : T(0);
        if constexpr (!WAVE1) {
#pragma unroll
            for (int r = 0; r < NX; ++r) {
                sh.ex[r][t] = s.z[r];
                sh.ex[NX + r][t] = s.mu[r];
            }
        }
        // The scalar half-space state is entered, left and materialized in every lane (idle
        // lanes hold zeros): a lane-conditional update would keep the vector copies and duals
        // of the half-space groups alive through the ADMM loop.
        if constexpr (HSQ) {
            T perp[3 * HSN], psum[3];
            hs_enter<M, T>(nc, rho, s, sig, kap, perp, psum);
#pragma unroll
            for (int q = 0; q < 3 * HSN; ++q) sh.hsp[q][t] = perp[q];
#pragma unroll
            for (int r = 0; r < 3; ++r) ehs[r] = -psum[r];
            nr = rho.geo * T(id.first() ? 0 : min(id.K, (int)M::KM));
        }
        bool done = !valid;
        int iters_here = kp.max_iters;
        bool conv_here = false;
        __syncthreads();

        // ---------------- a5-a9: ADMM iterations ----------------
        // The iterations between two residual tests run a copy of the body without the test's
        // code (CHK false): no per-iteration test bookkeeping in the common path.
        auto admm_iter = [&](const int j, auto chk, const bool test) __attribute__((always_inline)) -> bool {
            constexpr bool check = decltype(chk)::value;
            // The next lane of a node N is a node 0, an idle lane or past the workgroup edge: its
            // z and mu are exactly 0, which is what Step 1 needs there.  d_dyn of the previous
            // lane is read at every node but used only at nodes i >= 1.
            T zn[NX], mn[NX];
            if constexpr (WAVE1) {
#pragma unroll
                for (int r = 0; r < NX; ++r) {
                    zn[r] = lane_next(s.z[r]);
                    mn[r] = lane_next(s.mu[r]);
                }
            }
            if (!done) {
                if constexpr (!WAVE1) {
#pragma unroll
                    for (int r = 0; r < NX; ++r) {
                        zn[r] = sh.ex[r][t + 1];
                        mn[r] = sh.ex[NX + r][t + 1];
                    }
                }
                if constexpr (check) {
                    // z and copies before this iteration, for the dual residual
                    if constexpr (HSQ) {
                        if (j == 2) {
                            T perp[3 * HSN];
#pragma unroll
                            for (int q = 0; q < 3 * HSN; ++q) perp[q] = sh.hsp[q][t];
                            hs_copies<M, T>(nc, rho, s, sig, kap, perp);
                        } else {
                            hs_copies<M, T>(nc, rho, s, sig, kap, nullptr);
                        }
                    }
#pragma unroll
                    for (int r = 0; r < NX; ++r) sh.zo[r][t] = s.z[r];
#pragma unroll
                    for (int q = 0; q < C; ++q) sh.cpo[q][t] = s.cp[q];
                }
                if constexpr (HSQ) {
                    T hx[3];
                    hs_step1_term<M, T>(nc, rho, s.x, nr, kap, ehs, hx);
                    if constexpr (LDSL) {
                        const StridedLds<T, BLOCK> la{&sh.Lf[0][t]};
                        step1<M, T, true, StridedLds<T, BLOCK>>(id, rho, nc, s, zn, mn, hx, &la);
                    } else {
                        step1<M, T, true>(id, rho, nc, s, zn, mn, hx);
                    }
                } else if constexpr (LDSL) {
                    const StridedLds<T, BLOCK> la{&sh.Lf[0][t]};
                    step1<M, T, false, StridedLds<T, BLOCK>>(id, rho, nc, s, zn, mn, nullptr, &la);
                } else {
                    step1<M, T>(id, rho, nc, s, zn, mn);
                }
                if constexpr (!WAVE1) {
#pragma unroll
                    for (int r = 0; r < NX; ++r) sh.fw[r][t + 1] = s.dd[r];
                }
            }
            if constexpr (HSQ) {
                // the remainders enter with -sum p, then +sum p, then leave (every lane alike)
                if (__builtin_expect(j == 1, 0)) {
#pragma unroll
                    for (int r = 0; r < 3; ++r) ehs[r] = -ehs[r];
                } else if (__builtin_expect(j == 2, 0)) {
#pragma unroll
                    for (int r = 0; r < 3; ++r) ehs[r] = T(0);
                }
            }
            T dp[NX];
            if constexpr (WAVE1) {
#pragma unroll
                for (int r = 0; r < NX; ++r) dp[r] = lane_prev(s.dd[r]);
            } else {
                __syncthreads();
#pragma unroll
                for (int r = 0; r < NX; ++r) dp[r] = sh.fw[r][t];
            }
            if (!done) {
                step2<M, T>(id, rho, s, dp);
                step3<M, T, HSQ>(id, rho, nc, s, ball_r, kappa, inv1k2);
                if constexpr (HSQ) hs_step34<M, T>(nc, s.x, sig, kap);
            }
            if (span.on) {
                // scenario consensus across workgroups
                const bool g0 = !done && id.first();
                if (g0) {
#pragma unroll
                    for (int q = 0; q < C; ++q)
                        if (slot_is_u<M>(q)) sh.gxw[slot_comp_u<M>(q)][t] = s.cp[q];
                    sh.gxm[t] = mem;
                }
                constexpr int UW = u_copy_cols<M>();
                group_sync<UW>(dv, sh, span, nbar, t, kp.spin_ticks);
                if (g0) {
#pragma unroll
                    for (int q = 0; q < C; ++q) {
                        if (!slot_is_u<M>(q)) continue;
                        T acc = T(0);
                        for (int m = 0; m < S; ++m) acc = acc + gx_at<UW>(sh, m, slot_comp_u<M>(q));
                        s.cp[q] = group_active<M>(id, slot_group<M>(q)) ? acc / T(S) : T(0);
                    }
                }
            } else if (kp.has_groups) {
                // scenario consensus: node-0 u copies replaced by their scenario mean
                const bool g0 = !done && id.first() && S > 1;
                if (g0) {
#pragma unroll
                    for (int q = 0; q < C; ++q)
                        if (slot_is_u<M>(q)) sh.ucp[slot_comp_u<M>(q)][t] = s.cp[q];
                }
                __syncthreads();
                if (g0) {
#pragma unroll
                    for (int q = 0; q < C; ++q) {
                        if (!slot_is_u<M>(q)) continue;
                        T acc = T(0);
                        for (int m = 0; m < S; ++m) acc = acc + sh.ucp[slot_comp_u<M>(q)][lb + m * (id.N + 1)];
                        s.cp[q] = group_active<M>(id, slot_group<M>(q)) ? acc / T(S) : T(0);
                    }
                }
            }
            if (!done) {
                step4<M, T, HSQ>(id, rho, s, dp);
                if constexpr (!WAVE1) {
#pragma unroll
                    for (int r = 0; r < NX; ++r) {
                        sh.ex[r][t] = s.z[r];
                        sh.ex[NX + r][t] = s.mu[r];
                    }
                }
            }
            if constexpr (check) {
                T rp = T(0), sp[NN], dz[NX];
#pragma unroll
                for (int r = 0; r < NX; ++r) dz[r] = T(0);
                if (!done) {
                    T dcp[C];
#pragma unroll
                    for (int r = 0; r < NX; ++r) {
                        dz[r] = s.z[r] - sh.zo[r][t];
                        if constexpr (!WAVE1) sh.dz[r][t] = dz[r];
                    }
                    if constexpr (HSQ) {
                        if (j == 1) {
                            T perp[3 * HSN];
#pragma unroll
                            for (int q = 0; q < 3 * HSN; ++q) perp[q] = sh.hsp[q][t];
                            hs_copies<M, T>(nc, rho, s, sig, kap, perp);
                        } else {
                            hs_copies<M, T>(nc, rho, s, sig, kap, nullptr);
                        }
                    }
#pragma unroll
                    for (int q = 0; q < C; ++q) dcp[q] = s.cp[q] - sh.cpo[q][t];
                    dual_res_own<M, T>(id, rho, dz, dcp, sp, false);
                    rp = primal_res<M, T>(id, s, dp);
                }
                T dzn[NX];
                if constexpr (WAVE1) {
#pragma unroll
                    for (int r = 0; r < NX; ++r) dzn[r] = lane_next(dz[r]);
                }
                __syncthreads();
                if (!done) {
#pragma unroll
                    for (int r = 0; r < NX; ++r) {
                        if constexpr (WAVE1) dzn[r] = id.last() ? T(0) : dzn[r];
                        else dzn[r] = id.last() ? T(0) : sh.dz[r][t + 1];
                    }
                    const T rd = dual_res_finish<M, T>(id, rho, nc.Ar, nc.B, sp, dzn);
                    atomicMax(&sh.mx[0][tb], res_bits(rp));
                    atomicMax(&sh.mx[1][tb], res_bits(rd));
                }
                __syncthreads();
                if (!span.on) {
                    if (!done && leader) {
                        unsigned long long bp = 0ull, bd = 0ull;
                        for (int m = 0; m < S; ++m) {
                            const int lm = lb + m * (id.N + 1);
                            bp = max(bp, sh.mx[0][lm]);
                            bd = max(bd, sh.mx[1][lm]);
                            sh.mx[0][lm] = 0ull;
                            sh.mx[1][lm] = 0ull;
                        }
                        const T grp = T(bits_res(bp)), grd = T(bits_res(bd));
                        const bool conv = test && grp <= kp.eps_p && grd <= kp.eps_d;
                        sh.flag[lb] = conv ? 1 : 0;
                        sh.red[0][lb] = grp;
                        sh.red[1][lb] = grd;
                        // blow-up tracking on the SCP iteration's last residual (at convergence or
                        // at the last ADMM iteration)
                        if constexpr (TRACK)
                            if (kp.blowup && (conv || j == kp.max_iters)) blowup_track<T>(sh.rp0[lb], sh.rpm[lb], grp);
                    }
                } else {
                    // member maxima to HBM; the group maximum is the same in every workgroup
                    if (!done && leader) {
                        sh.gxw[0][t] = T(bits_res(sh.mx[0][tb]));
                        sh.gxw[1][t] = T(bits_res(sh.mx[1][tb]));
                        sh.gxm[t] = mem;
                        sh.mx[0][tb] = 0ull;
                        sh.mx[1][tb] = 0ull;
                    }
                    group_sync<2>(dv, sh, span, nbar, t, kp.spin_ticks);
                    if (!done && leader) {
                        T grp = T(0), grd = T(0);
                        for (int m = 0; m < S; ++m) {
                            grp = nmax(grp, gx_at<2>(sh, m, 0));
                            grd = nmax(grd, gx_at<2>(sh, m, 1));
                        }
                        const bool conv = test && grp <= kp.eps_p && grd <= kp.eps_d;
                        sh.flag[lb] = conv ? 1 : 0;
                        sh.red[0][lb] = grp;
                        sh.red[1][lb] = grd;
                        if constexpr (TRACK)
                            if (kp.blowup && (conv || j == kp.max_iters)) blowup_track<T>(sh.rp0[lb], sh.rpm[lb], grp);
                    }
                }
                __syncthreads();
                if (!done) {
                    rp_last = sh.red[0][lb];
                    rd_last = sh.red[1][lb];
                    if (sh.flag[lb]) {
                        done = true;
                        conv_here = true;
                        iters_here = j;
                    }
                }
                if (!__syncthreads_or(done ? 0 : 1)) return true;
            }
            if constexpr (!WAVE1) __syncthreads();
            return false;
        };
        {
            const int K = kp.max_iters, c = kp.check_every;
            int j = 1;
            while (j <= K) {
                const int jc = c > 0 ? min((j + c - 1) / c * c, K) : K;  // next iteration with a check
                for (; j < jc; ++j) admm_iter(j, std::false_type{}, false);
                if (admm_iter(j, std::true_type{}, c > 0 && j % c == 0)) break;
                ++j;
            }
        }
        // half-space duals back to vector form: carried into the next SCP iteration / written back
        if constexpr (HSQ) {
            if (kp.max_iters == 0) {
                T perp[3 * HSN];
#pragma unroll
                for (int q = 0; q < 3 * HSN; ++q) perp[q] = sh.hsp[q][t];
                hs_duals<M, T>(nc, rho, s, sig, perp);
            } else {
                hs_duals<M, T>(nc, rho, s, sig, nullptr);
            }
        }
        last_iters = iters_here;

        // ---------------- a10: merit ratio test and nominal update ----------------
        T xn1[NX];
        if constexpr (WAVE1) {
#pragma unroll
            for (int r = 0; r < NX; ++r) xn1[r] = lane_next(s.x[r]);
        } else {
#pragma unroll
            for (int r = 0; r < NX; ++r) sh.ex[r][t] = s.x[r];
        }
        __syncthreads();
        if constexpr (!WAVE1) {
#pragma unroll
            for (int r = 0; r < NX; ++r) xn1[r] = sh.ex[r][t + 1 < BLOCK ? t + 1 : t];
        }
        T cost_new = T(0), pen_new = T(0), pen_mod = T(0);
        if (valid) {
            cost_new = node_cost<M, T>(prm, id, s.x, s.u);
            if (!id.last()) {
                T Fx[NX];
                rk4<M, T>(prm, s.x, s.u, Fx);
#pragma unroll
                for (int r = 0; r < NX; ++r) pen_new = pen_new + tabs(xn1[r] - Fx[r]);
#pragma unroll
                for (int r = 0; r < NX; ++r) pen_mod = pen_mod + tabs(xn1[r] - s.dd[r]);
            }
        }
        sh.red[0][t] = cost_nom;
        sh.red[1][t] = pen_nom;
        sh.red[2][t] = cost_new;
        sh.red[3][t] = pen_new;
        sh.red[4][t] = pen_mod;
        __syncthreads();
        // member merit terms (nominal, candidate, model); a spanning group sums them over HBM
        const int S_here = span.on ? 1 : S;
        T mnom = T(0), mnew = T(0), mmod = T(0);
        if (leader) {
            for (int m = 0; m < S_here; ++m) {
                const int base = lb + m * (id.N + 1);
                T J0 = T(0), p0 = T(0), J1 = T(0), p1 = T(0), pm = T(0);
                for (int i = 0; i <= id.N; ++i) {
                    J0 = J0 + sh.red[0][base + i];
                    J1 = J1 + sh.red[2][base + i];
                }
                for (int i = 0; i < id.N; ++i) {
                    p0 = p0 + sh.red[1][base + i];
                    p1 = p1 + sh.red[3][base + i];
                    pm = pm + sh.red[4][base + i];
                }
                const T vnom = J0 + kp.merit_w * p0, vnew = J1 + kp.merit_w * p1, vmod = J1 + kp.merit_w * pm;
                if (span.on) {
                    sh.gxw[0][t] = vnom;
                    sh.gxw[1][t] = vnew;
                    sh.gxw[2][t] = vmod;
                    sh.gxm[t] = mem;
                } else {
                    mnom = mnom + vnom;
                    mnew = mnew + vnew;
                    mmod = mmod + vmod;
                }
            }
        }
        if (span.on) {
            group_sync<3>(dv, sh, span, nbar, t, kp.spin_ticks);
            if (leader) {
                for (int m = 0; m < S; ++m) {
                    mnom = mnom + gx_at<3>(sh, m, 0);
                    mnew = mnew + gx_at<3>(sh, m, 1);
                    mmod = mmod + gx_at<3>(sh, m, 2);
                }
            }
        }
        if (leader) {
            const AcceptOut<T> a = accept_rule<T>(kp.eta0, kp.eta1, kp.eta2, kp.shrink, kp.grow, kp.delta_max, mnom,
                                                  mnew, mmod, delta);
            sh.flag[lb] = (a.accept ? 1 : 0) | (a.nonfinite ? 2 : 0);
            sh.red[5][lb] = a.delta;
            sh.red[6][lb] = a.ratio;
            sh.red[7][lb] = mnew;
        }
        __syncthreads();
        if (valid) {
            const int f = sh.flag[lb];
            delta = sh.red[5][lb];
            ratio_last = sh.red[6][lb];
            merit_last = sh.red[7][lb];
            if (f & 2) status |= SCP_ST_NONFINITE;
            if (f & 1) {
#pragma unroll
                for (int r = 0; r < NX; ++r) xbar[r] = s.x[r];
#pragma unroll
                for (int r = 0; r < NU; ++r) ubar[r] = s.u[r];
                n_acc += 1;
            }
            iters_sum += iters_here;
            conv_last = conv_here;
            // the group's residuals of this SCP iteration's last ADMM iteration
            if constexpr (ADAPT)
                sh.arho[t] = T(adapt_factor((double)sh.arho[t], (double)rp_last, (double)rd_last, kp.adapt_mu,
                                            kp.adapt_tau));
        }
        __syncthreads();
    }

    // ---------------- metrics of the final nominal ----------------
    T m_cost = T(0), m_def = T(0), m_viol = T(0), m_bnd = T(0);
    if (kp.final_metrics) {
        T xnf[NX];
        if constexpr (WAVE1) {
#pragma unroll
            for (int r = 0; r < NX; ++r) xnf[r] = lane_next(xbar[r]);
        } else {
#pragma unroll
            for (int r = 0; r < NX; ++r) sh.ex[r][t] = xbar[r];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < NX; ++r) xnf[r] = sh.ex[r][t + 1];
        }
        if (valid) {
            if (!id.last()) {
                T Fx[NX];
                rk4<M, T>(prm, xbar, ubar, Fx);
#pragma unroll
                for (int r = 0; r < NX; ++r) m_def = nmax(m_def, tabs(xnf[r] - Fx[r]));
            }
            m_cost = node_cost<M, T>(prm, id, xbar, ubar);
            m_viol = node_violation<M, T>(prm, id, xbar, ubar);
            m_bnd = node_bnd_err<M, T>(prm, id, xbar);
        }
        sh.red[0][t] = m_cost;
        sh.red[1][t] = m_def;
        sh.red[2][t] = m_viol;
        sh.red[3][t] = m_bnd;
        __syncthreads();
    }
    if (span.on) {
        // the group failed if any member gave up waiting (see group_sync)
        if (t == 0 && __hip_atomic_load(dv.gsync + (size_t)span.slot * GX_SYNC_STRIDE + 1, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT) != 0u)
            sh.sync_fail = 1;
        __syncthreads();
        if (sh.sync_fail) status |= SCP_ST_SYNC;
    }
    if (valid && status) atomicOr(&sh.st[tb], status);
    __syncthreads();

    // ---------------- write-back ----------------
    if constexpr (HSQ) {
        // with no SCP iteration: x = 0, sig = kap = 0 and a = 0, so the copies are 0
        if (kp.n_scp > 0 && last_iters == 1) {
            T perp[3 * HSN];
#pragma unroll
            for (int q = 0; q < 3 * HSN; ++q) perp[q] = sh.hsp[q][t];
            hs_copies<M, T>(nc, rho, s, sig, kap, perp);
        } else {
            hs_copies<M, T>(nc, rho, s, sig, kap, nullptr);
        }
    }
    if (valid) {
#pragma unroll
        for (int r = 0; r < NX; ++r) {
            dv.planes[(size_t)(PL_XBAR + r) * P + gn] = xbar[r];
            dv.planes[(size_t)(PL_X + r) * P + gn] = s.x[r];
            dv.planes[(size_t)(PL_Z + r) * P + gn] = s.z[r];
            dv.planes[(size_t)(PL_LAM + r) * P + gn] = s.lam[r];
            dv.planes[(size_t)(PL_MU + r) * P + gn] = s.mu[r];
            dv.planes[(size_t)(PL_DD + r) * P + gn] = id.last() ? T(0) : s.dd[r];
        }
#pragma unroll
        for (int r = 0; r < NU; ++r) {
            dv.planes[(size_t)(PL_UBAR + r) * P + gn] = ubar[r];
            dv.planes[(size_t)(PL_U + r) * P + gn] = s.u[r];
        }
#pragma unroll
        for (int q = 0; q < C; ++q) {
            dv.planes[(size_t)(PL_CP + q) * P + gn] = group_active<M>(id, slot_group<M>(q)) ? s.cp[q] : T(0);
            dv.planes[(size_t)(PL_DU + q) * P + gn] = s.du[q];
        }
    }
    if (first_lane) {
        dv.rt[tr * RT_FIELDS + RT_DELTA] = delta;
        if constexpr (ADAPT) dv.rt[tr * RT_FIELDS + RT_RHOS] = sh.arho[t];
        double* inf = dv.info + (size_t)tr * SCP_INFO_FIELDS;
        int st = sh.st[tb];
        if constexpr (TRACK) {
            if (kp.blowup) {
                dv.rt[tr * RT_FIELDS + RT_RP0] = sh.rp0[lb];
                dv.rt[tr * RT_FIELDS + RT_RPMAX] = sh.rpm[lb];
                st |= blowup_status<T>(sh.rp0[lb], sh.rpm[lb]);
            }
        }
        if (!kp.reset_info) st |= (int)inf[SCP_I_STATUS] & ~SCP_ST_CONVERGED;
        if (conv_last) st |= SCP_ST_CONVERGED;
        const double it0 = kp.reset_info ? 0.0 : inf[SCP_I_ADMM_ITERS];
        const double na0 = kp.reset_info ? 0.0 : inf[SCP_I_NACCEPT];
        inf[SCP_I_ADMM_ITERS] = it0 + (double)iters_sum;
        inf[SCP_I_NACCEPT] = na0 + (double)n_acc;
        inf[SCP_I_RP] = (double)rp_last;
        inf[SCP_I_RD] = (double)rd_last;
        inf[SCP_I_DELTA] = (double)delta;
        inf[SCP_I_STATUS] = (double)st;
        inf[SCP_I_RATIO] = (double)ratio_last;
        inf[SCP_I_MERIT] = (double)merit_last;
        if (kp.final_metrics) {
            T J = T(0), df = T(0), vi = T(0), be = T(0);
            for (int i = 0; i <= id.N; ++i) {
                J = J + sh.red[0][tb + i];
                df = nmax(df, sh.red[1][tb + i]);
                vi = nmax(vi, sh.red[2][tb + i]);
                be = nmax(be, sh.red[3][tb + i]);
            }
            inf[SCP_I_COST] = (double)J;
            inf[SCP_I_DEFECT] = (double)df;
            inf[SCP_I_VIOL] = (double)vi;
            inf[SCP_I_BNDERR] = (double)be;
        }
    }
}

template <class M, class T, int BLOCK, bool SPAN, bool ADAPT, bool TRACK, int HSR, int LR, int AR>
__device__ __forceinline__ void body_for(const Dev<T>& dv, const KParams<T>& kp, Shared<T, BLOCK, HSR, LR, AR>& sh,
                                         const int t, const int gn, const bool cross, const Span& sp) {
    if constexpr (BLOCK == 64) {
        persistent_body<M, T, BLOCK, true, SPAN, ADAPT, TRACK>(dv, kp, sh, t, gn, sp);
    } else {
        if (cross) persistent_body<M, T, BLOCK, false, SPAN, ADAPT, TRACK>(dv, kp, sh, t, gn, sp);
        else persistent_body<M, T, BLOCK, true, SPAN, ADAPT, TRACK>(dv, kp, sh, t, gn, sp);
    }
}

// LDS rows of the factors: one-wavefront workgroups keep the quadrotor's factor in LDS (and the
// powered descent's when it is the only model); the LDS of a mixed kernel stays within four
// workgroups per CU with the quadrotor's factor alone.
constexpr int persistent_lds_factor_rows(int block, int models) {
    return block != 64 ? 1 : models == 2 ? Dims<Mars>::NL : Dims<Quad<8>>::NL;
}

// MODELS: 1 quadrotor only, 2 powered descent only, 3 both (each workgroup holds one model).
// SPAN: the launch has consensus groups spanning several workgroups.
template <class T, int BLOCK, int MODELS, int KM, bool SPAN, bool ADAPT, bool TRACK>
__global__ __launch_bounds__(BLOCK) void k_persistent(Dev<T> dv, KParams<T> kp) {
    __shared__ Shared<T, BLOCK, (MODELS != 2 && KM > 0) ? 3 * KM : 1, persistent_lds_factor_rows(BLOCK, MODELS),
                      ADAPT ? BLOCK : 1> sh;
    const int t = threadIdx.x;
    const int w = dv.wg_list ? dv.wg_list[blockIdx.x] : (int)blockIdx.x;
    const int gn = dv.lane_node[(size_t)w * BLOCK + t];
    const int wi = dv.wg_info[w];
    const bool cross = (wi & WG_CROSS) != 0;
    Span sp{false, 0, 1};
    if (wi & WG_SPAN) sp = Span{true, dv.wg_group[2 * w], dv.wg_group[2 * w + 1]};
    if constexpr (MODELS == 1) {
        body_for<Quad<KM>, T, BLOCK, SPAN, ADAPT, TRACK>(dv, kp, sh, t, gn, cross, sp);
    } else if constexpr (MODELS == 2) {
        body_for<Mars, T, BLOCK, SPAN, ADAPT, TRACK>(dv, kp, sh, t, gn, cross, sp);
    } else {
        if ((wi & 0xff) == SCP_MODEL_QUAD_PM) body_for<Quad<KM>, T, BLOCK, SPAN, ADAPT, TRACK>(dv, kp, sh, t, gn, cross, sp);
        else body_for<Mars, T, BLOCK, SPAN, ADAPT, TRACK>(dv, kp, sh, t, gn, cross, sp);
    }
}

// Launch of the persistent kernel variant for BLOCK, SPAN, ADAPT and TRACK (instantiated per
// precision and variant in their own translation units, compiled in parallel).  TRACK kernels
// carry the residual blow-up tracking (active when kp.blowup is set); the spanning and adaptive
// variants always do, the plain fixed-penalty one comes in both forms, so that the default
// kernel keeps its code and registers.
template <class T, int BLOCK, bool SPAN, bool ADAPT = false, bool TRACK = SPAN || ADAPT>
void launch_models(const Dev<T>& dv, const KParams<T>& kp, int n_wg, int models, int kmax, hipStream_t s) {
    const dim3 g(n_wg), b(BLOCK);
    if (models == 1) {
        if (kmax <= 4) hipLaunchKernelGGL((k_persistent<T, BLOCK, 1, 4, SPAN, ADAPT, TRACK>), g, b, 0, s, dv, kp);
        else hipLaunchKernelGGL((k_persistent<T, BLOCK, 1, 8, SPAN, ADAPT, TRACK>), g, b, 0, s, dv, kp);
    } else if (models == 2) {
        hipLaunchKernelGGL((k_persistent<T, BLOCK, 2, 0, SPAN, ADAPT, TRACK>), g, b, 0, s, dv, kp);
    } else {
        if (kmax <= 4) hipLaunchKernelGGL((k_persistent<T, BLOCK, 3, 4, SPAN, ADAPT, TRACK>), g, b, 0, s, dv, kp);
        else hipLaunchKernelGGL((k_persistent<T, BLOCK, 3, 8, SPAN, ADAPT, TRACK>), g, b, 0, s, dv, kp);
    }
}

// Workgroups per compute unit of the spanning-group variant (occupancy of the exact kernel the
// launch would use); 0 if the query fails.
template <class T, int BLOCK>
int span_blocks_per_cu(int models, int kmax) {
    int n = 0;
    hipError_t e;
    if (models == 1)
        e = kmax <= 4 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_persistent<T, BLOCK, 1, 4, true, false, true>, BLOCK, 0)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_persistent<T, BLOCK, 1, 8, true, false, true>, BLOCK, 0);
    else if (models == 2)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_persistent<T, BLOCK, 2, 0, true, false, true>, BLOCK, 0);
    else
        e = kmax <= 4 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_persistent<T, BLOCK, 3, 4, true, false, true>, BLOCK, 0)
                      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_persistent<T, BLOCK, 3, 8, true, false, true>, BLOCK, 0);
    return e == hipSuccess ? n : 0;
}

}  // namespace scp

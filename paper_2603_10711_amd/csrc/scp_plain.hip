// Plain form of the hot path: one thread per node, every array in HBM, one kernel launch per
// ADMM phase.  This is the comparison baseline for the persistent kernel and the path behind
// the scp_linearize / admm_solve entry points.
#include "scp_device.hpp"
#include "scp_launch.hpp"
#include "scp_layout.hpp"

namespace scp {

// every plane block holds the largest model (6-DOF quadrotor with SCP_MAX_OBS obstacles)
using QMax = Quad6<SCP_MAX_OBS>;
static_assert(PL_UBAR - PL_XBAR >= QMax::NX && PL_X - PL_UBAR >= QMax::NU, "nominal blocks");
static_assert(PL_U - PL_X >= QMax::NX && PL_Z - PL_U >= QMax::NU && PL_LAM - PL_Z >= QMax::NX, "iterate blocks");
static_assert(PL_MU - PL_LAM >= QMax::NX && PL_DD - PL_MU >= QMax::NX && PL_CP - PL_DD >= QMax::NX, "iterate blocks");
static_assert(PL_DU - PL_CP >= MAX_C && PL_AR - PL_DU >= MAX_C && QMax::C <= MAX_C && Quad<SCP_MAX_OBS>::C <= MAX_C,
              "mirror blocks");
static_assert(PL_B - PL_AR >= QMax::NX * QMax::NXR && PL_D - PL_B >= QMax::NX * QMax::NU && PL_L - PL_D >= QMax::NX,
              "linearization blocks");
static_assert(PL_LO - PL_L >= Dims<QMax>::NL && PL_HI - PL_LO >= QMax::NN && PL_HS - PL_HI >= QMax::NN, "factor, box");
static_assert(PL_G0 - PL_HS >= QMax::NHS && PL_DZ - PL_G0 >= QMax::NX && PL_SP - PL_DZ >= QMax::NX, "half-spaces");
static_assert(PL_RP - PL_SP >= QMax::NN && PL_XG - PL_MER >= 8 && NPLANES - PL_UG >= QMax::NU &&
              PL_UG - PL_XG >= QMax::NX, "residual, merit, guess blocks");
// the 6-DOF lander (14 states, 3 controls, 34 slots) fits the same blocks
static_assert(PL_UBAR - PL_XBAR >= Lander6::NX && PL_LAM - PL_Z >= Lander6::NX && PL_CP - PL_DD >= Lander6::NX,
              "lander state blocks");
static_assert(PL_B - PL_AR >= Lander6::NX * Lander6::NXR && PL_D - PL_B >= Lander6::NX * Lander6::NU &&
              PL_L - PL_D >= Lander6::NX && Lander6::C <= MAX_C && PL_LO - PL_L >= Dims<Lander6>::NL &&
              PL_HI - PL_LO >= Lander6::NN && PL_RP - PL_SP >= Lander6::NN && PL_G0 - PL_HS >= Lander6::NHS &&
              PL_UG - PL_XG >= Lander6::NX && PL_DZ - PL_G0 >= Lander6::NX && PL_SP - PL_DZ >= Lander6::NX,
              "lander blocks");
// node 0 of a consensus group parks its u-slot copies in the merit block (the lander takes no
// consensus groups)
static_assert(QMax::NU + 3 <= 8 && Mars::NU + 4 <= 8, "u-slot stash");

template <int NV, class T>
__device__ __forceinline__ void ldp(const T* __restrict__ pl, int P, int g, T* v) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = pl[(size_t)k * P + g];
}
template <int NV, class T>
__device__ __forceinline__ void stp(T* __restrict__ pl, int P, int g, const T* v) {
#pragma unroll
    for (int k = 0; k < NV; ++k) pl[(size_t)k * P + g] = v[k];
}

template <class T>
__device__ __forceinline__ T* PL(const Dev<T>& dv, int plane) { return dv.planes + (size_t)plane * dv.P; }

// adaptive penalty factor of trajectory tr (exactly 1 while the rule is off), and the penalties
// of this SCP iteration scaled by it
template <class T>
__device__ __forceinline__ T rho_factor(const Dev<T>& dv, const KParams<T>& kp, int tr) {
    return kp.adapt_mu > 0.0 ? dv.rt[tr * RT_FIELDS + RT_RHOS] : T(1);
}
template <class T>
__device__ __forceinline__ Rho<T> rho_of(const KParams<T>& kp, T f) {
    const T re = kp.rho_eq * f, rd = kp.rho_dyn * f, rg = kp.rho_geo * f;
    return Rho<T>{re, rd, rg, T(1) / rg, T(1) / (re + rd)};
}

// Resolve the node handled by this thread: returns the trajectory or -1.
template <class M, class T>
__device__ __forceinline__ int node_of(const Dev<T>& dv, int g, NodeId& id, const T*& prm) {
    if (g >= dv.n_nodes) return -1;
    const int tr = dv.node_traj[g];
    if (tr < 0) return -1;
    const int* rec = dv.traj + tr * TR_FIELDS;
    if (rec[TR_MODEL] != M::ID) return -1;
    id.i = g - rec[TR_OFF];
    id.N = rec[TR_N];
    id.K = rec[TR_K];
    id.ball = rec[TR_BALL] != 0;
    prm = dv.params + (size_t)tr * SCP_PARAM_STRIDE;
    return tr;
}

template <class M, class T>
__device__ __forceinline__ void load_const(const Dev<T>& dv, int g, NodeConst<M, T>& nc) {
    constexpr int NX = M::NX, NU = M::NU, NN = M::NN, NXR = M::NXR;
    const int P = dv.P;
    ldp<Dims<M>::NL>(PL(dv, PL_L), P, g, nc.L);
    ldp<NX * NXR>(PL(dv, PL_AR), P, g, nc.Ar);
    ldp<NX * NU>(PL(dv, PL_B), P, g, nc.B);
    ldp<NX>(PL(dv, PL_D), P, g, nc.d);
    ldp<NN>(PL(dv, PL_LO), P, g, nc.lo);
    ldp<NN>(PL(dv, PL_HI), P, g, nc.hi);
    if constexpr (M::HSD) ldp<M::NHS>(PL(dv, PL_HS), P, g, nc.hs);
    ldp<NX>(PL(dv, PL_G0), P, g, nc.g0);
}

// ------------------------------------------------------------------------------------------
// a2-a4 + primal re-initialization + nominal merit terms
// ------------------------------------------------------------------------------------------
template <class M, class T>
__global__ __launch_bounds__(256) void k_lin(Dev<T> dv, KParams<T> kp) {
    constexpr int NX = M::NX, NU = M::NU, NXR = M::NXR;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    NodeId id;
    const T* prm;
    const int tr = node_of<M>(dv, g, id, prm);
    if (tr < 0) return;
    const int P = dv.P;
    const int* rec = dv.traj + tr * TR_FIELDS;
    const Rho<T> rho = rho_of<T>(kp, rho_factor<T>(dv, kp, tr));
    NodeConst<M, T> nc;
    T xbar[NX], ubar[NU], F[NX];
    ldp<NX>(PL(dv, PL_XBAR), P, g, xbar);
    ldp<NU>(PL(dv, PL_UBAR), P, g, ubar);
    if (!id.last()) {
        linearize<M, T>(prm, xbar, ubar, F, nc.Ar, nc.B, nc.d);
    } else {
#pragma unroll
        for (int k = 0; k < NX * NXR; ++k) nc.Ar[k] = T(0);
#pragma unroll
        for (int k = 0; k < NX * NU; ++k) nc.B[k] = T(0);
#pragma unroll
        for (int k = 0; k < NX; ++k) nc.d[k] = T(0);
#pragma unroll
        for (int k = 0; k < NU; ++k) ubar[k] = T(0);
    }
    // control trust-box centre: scenario mean of the first nominal controls inside a group
    T uc[NU];
#pragma unroll
    for (int k = 0; k < NU; ++k) uc[k] = ubar[k];
    const int gsize = rec[TR_GSIZE];
    if (id.first() && gsize > 1) {
        const int g0 = dv.traj[rec[TR_GFIRST] * TR_FIELDS + TR_OFF];
        const int stride = id.N + 1;
        T acc[NU];
#pragma unroll
        for (int k = 0; k < NU; ++k) acc[k] = T(0);
        for (int m = 0; m < gsize; ++m) {
            T um[NU];
            ldp<NU>(PL(dv, PL_UBAR), P, g0 + m * stride, um);
#pragma unroll
            for (int k = 0; k < NU; ++k) acc[k] = acc[k] + um[k];
        }
#pragma unroll
        for (int k = 0; k < NU; ++k) uc[k] = acc[k] / T(gsize);
    }
    const T delta = dv.rt[tr * RT_FIELDS + RT_DELTA];
    int st = convexify<M, T>(prm, id, xbar, uc, delta, nc);
    st |= assemble_factor<M, T>(prm, id, rho, nc);
    // merit terms of the nominal
    T pen = T(0);
    if (!id.last()) {
        T xn[NX];
        ldp<NX>(PL(dv, PL_XBAR), P, g + 1, xn);
#pragma unroll
        for (int r = 0; r < NX; ++r) pen = pen + tabs(xn[r] - F[r]);
    }
    PL(dv, PL_MER)[(size_t)MER_COST_NOM * P + g] = node_cost<M, T>(prm, id, xbar, ubar);
    PL(dv, PL_MER)[(size_t)MER_PEN_NOM * P + g] = pen;
    // primal re-initialization from the nominal (duals carried)
    NodeState<M, T> s;
#pragma unroll
    for (int r = 0; r < NX; ++r) {
        s.x[r] = xbar[r];
        s.z[r] = id.first() ? T(0) : xbar[r];
    }
#pragma unroll
    for (int r = 0; r < NU; ++r) s.u[r] = ubar[r];
#pragma unroll
    for (int k = 0; k < M::C; ++k)
        s.cp[k] = group_active<M>(id, slot_group<M>(k)) ? slot_var<M, T>(s, k) : T(0);
    stp<Dims<M>::NL>(PL(dv, PL_L), P, g, nc.L);
    stp<NX * NXR>(PL(dv, PL_AR), P, g, nc.Ar);
    stp<NX * NU>(PL(dv, PL_B), P, g, nc.B);
    stp<NX>(PL(dv, PL_D), P, g, nc.d);
    stp<M::NN>(PL(dv, PL_LO), P, g, nc.lo);
    stp<M::NN>(PL(dv, PL_HI), P, g, nc.hi);
    if constexpr (M::HSD) stp<M::NHS>(PL(dv, PL_HS), P, g, nc.hs);
    stp<NX>(PL(dv, PL_G0), P, g, nc.g0);
    stp<NX>(PL(dv, PL_X), P, g, s.x);
    stp<NU>(PL(dv, PL_U), P, g, s.u);
    stp<NX>(PL(dv, PL_Z), P, g, s.z);
    stp<M::C>(PL(dv, PL_CP), P, g, s.cp);
    if (st) atomicOr(&dv.flags[tr * FL_FIELDS + FL_STATUS], st);
    if (id.first()) {
        dv.flags[tr * FL_FIELDS + FL_DONE] = 0;
        dv.flags[tr * FL_FIELDS + FL_ITERS] = 0;
        dv.red[2 * tr] = 0ull;
        dv.red[2 * tr + 1] = 0ull;
    }
}

// ------------------------------------------------------------------------------------------
// a5: Step 1
// ------------------------------------------------------------------------------------------
template <class M, class T>
__global__ __launch_bounds__(256) void k_step1(Dev<T> dv, KParams<T> kp) {
    constexpr int NX = M::NX, NU = M::NU;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    NodeId id;
    const T* prm;
    const int tr = node_of<M>(dv, g, id, prm);
    if (tr < 0 || dv.flags[tr * FL_FIELDS + FL_DONE]) return;
    const int P = dv.P;
    const Rho<T> rho = rho_of<T>(kp, rho_factor<T>(dv, kp, tr));
    NodeConst<M, T> nc;
    load_const<M, T>(dv, g, nc);
    NodeState<M, T> s;
    ldp<NX>(PL(dv, PL_Z), P, g, s.z);
    ldp<NX>(PL(dv, PL_LAM), P, g, s.lam);
    ldp<M::C>(PL(dv, PL_CP), P, g, s.cp);
    ldp<M::C>(PL(dv, PL_DU), P, g, s.du);
    T zn[NX], mn[NX];
    if (!id.last()) {
        ldp<NX>(PL(dv, PL_Z), P, g + 1, zn);
        ldp<NX>(PL(dv, PL_MU), P, g + 1, mn);
    } else {
#pragma unroll
        for (int r = 0; r < NX; ++r) zn[r] = mn[r] = T(0);
    }
    step1<M, T>(id, rho, nc, s, zn, mn);
    if (id.last()) {
#pragma unroll
        for (int r = 0; r < NX; ++r) s.dd[r] = T(0);   // no interval after node N
    }
    stp<NX>(PL(dv, PL_X), P, g, s.x);
    stp<NU>(PL(dv, PL_U), P, g, s.u);
    stp<NX>(PL(dv, PL_DD), P, g, s.dd);
}

// ------------------------------------------------------------------------------------------
// a5: Step 1 of the 6-DOF models (n = 17), four lanes per node
// ------------------------------------------------------------------------------------------
// At n = 17 one lane per node underfills the chip (a 1000-trajectory batch of 41 nodes makes 641
// wavefronts for 1024 SIMDs) and every lane works through a long chain of dependent loads.  Here
// the four lanes of a DPP group share a node.  Lane l owns the state components k = 4s + l
// (slots s = 0..3) and the control component l (slot 4): their rows of w, their columns of A and
// B, and their rows of the factor, so each lane loads about a third of the node's data.  A slot
// holds states only or controls only, so no slot runs both the state and the control code.
//  * w rows go to every lane of the group by broadcast;
//  * the forward substitution is right-looking: y_k comes from its owner by broadcast and every
//    lane updates its rows below k (the same subtraction sequence as the one-lane solve);
//  * the backward substitution sums each lane's products over its rows below k across the group
//    (the same bits in every lane) and the owner of row k finishes x_k;
//  * A x + B u: a lane's copies of its columns of A and B hold row 4n + (l xor c) at entry
//    4n + c, so one reduce-scatter of three exchanges per four rows hands every lane the sums of
//    its own rows, with the bits of the full group sum (the last rows use that sum);
//  * A'w sums over the rows in the same lane-permuted order.
// Rows of the factor above the diagonal are held as zeros, so no step needs a lane mask.
template <class M>
struct Lanes4 {
    static constexpr int NX = M::NX, NU = M::NU, NN = M::NN, NS = 5;
    static_assert(NX <= 16 && NU <= 4 && NN == NX + NU, "four lanes hold the node");
    // component in slot s of lane l, and whether the node has it
    __device__ static constexpr int comp(int s, int l) { return s < 4 ? 4 * s + l : NX + l; }
    __device__ static constexpr bool held(int s, int l) { return s < 4 ? 4 * s + l < NX : l < NU; }
    // slot and lane of component k
    __device__ static constexpr int slot(int k) { return k < NX ? k / 4 : 4; }
    __device__ static constexpr int lane(int k) { return k < NX ? k % 4 : k - NX; }
    // largest component any lane holds in slot s
    __device__ static constexpr int top(int s) { return s < 4 ? (4 * s + 3 < NX ? 4 * s + 3 : NX - 1) : NN - 1; }
    // Row of A and B that entry m of a lane's column copy holds: rows 4n + (l xor c) at m = 4n + c
    // below RB, so that quad_reduce_scatter hands the sum of row 4n + l to lane l; rows from RB on
    // in order.
    static constexpr int RB = NX / 4 * 4;
    __device__ static constexpr int row(int m, int l) { return m < RB ? 4 * (m / 4) + (l ^ (m % 4)) : m; }
};

// Per-lane stride, in elements of T, of a lane-private LDS array of n entries read with 16-byte
// loads: a multiple of 16 bytes whose length in 4-byte words is 4 or 12 modulo 16, so that the
// 16-byte reads of 16 consecutive lanes start 4 words apart modulo 64 and hit distinct banks.
template <class T>
constexpr int lds_lane_stride(int n) {
    constexpr int step = 16 / (int)sizeof(T);
    int e = (n + step - 1) / step * step;
    while ((e * (int)sizeof(T) / 4) % 16 != 4 && (e * (int)sizeof(T) / 4) % 16 != 12) e += step;
    return e;
}

// The 6-DOF quadrotor solves Step 1 in FP32 with the explicit inverse M = H^-1 of the node's
// matrix; FP64 and the other models keep the two triangular substitutions (Sec. III-B Step 1
// caches a factorization; the inverse is computed from it once per SCP iteration).  At n = 17
// the product x = M g is 17 broadcasts and 85 multiply-adds per lane in five independent chains,
// against ~230 instructions in two dependent chains of 17 steps for the substitutions; H is well
// conditioned here (condition numbers below 60 at the benchmark penalties), where the FP32 error
// of the product is that of the substitutions.  The lander keeps the substitutions: its rows of
// M and the LDS copy of A that makes room for them cost more than they save (measured).
template <class M, class T>
struct StepInverse {
    static constexpr bool value = sizeof(T) == 4 && M::ID == SCP_MODEL_QUAD_6DOF;
};

// The lane's rows of the node's factor (diagonal slot 1/L_kk, 0 above the diagonal) or, with the
// inverse, its full rows of M (held as the lower triangle, packed like the factor).  ld(t) loads
// packed entry t.
template <bool INVERSE, class LY, class T, class LD>
__device__ __forceinline__ void lanes4_load_rows(int l, LD&& ld, T (&R)[LY::NS][LY::NN]) {
#pragma unroll
    for (int s = 0; s < LY::NS; ++s) {
        const int row = LY::comp(s, l);
        const bool ok = LY::held(s, l);
#pragma unroll
        for (int j = 0; j < LY::NN; ++j) {
            if constexpr (INVERSE) R[s][j] = ok ? ld(row >= j ? tri(row, j) : tri(j, row)) : T(0);
            else if (j <= LY::top(s)) R[s][j] = (ok && j <= row) ? ld(tri(row, j)) : T(0);
            else R[s][j] = T(0);
        }
    }
}

// L L' x = r on the node held by a group of four lanes (lane l holds rows comp(s, l)).
//  * forward: y_k comes from its owner by broadcast and every lane updates its rows below k (the
//    same subtraction sequence as the one-lane solve);
//  * backward: each lane's products over its rows below k, summed across the group (the same
//    bits in every lane), and the owner of row k finishes x_k.
// r is overwritten.
template <class LY, class T>
__device__ __forceinline__ void lanes4_chol_solve(T (&r)[LY::NS], const T (&Lr)[LY::NS][LY::NN], int l, T (&xl)[LY::NS]) {
    constexpr int NS = LY::NS, NN = LY::NN;
    T yl[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) yl[s] = T(0);
#pragma unroll
    for (int k = 0; k < NN; ++k) {
        const int sk = LY::slot(k), lk = LY::lane(k);
        const T yk = quad_bcast(r[sk] * Lr[sk][k], lk);
        yl[sk] = (l == lk) ? yk : yl[sk];
#pragma unroll
        for (int s = 0; s < NS; ++s)
            if (LY::top(s) > k) r[s] = r[s] - Lr[s][k] * yk;
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) xl[s] = T(0);
#pragma unroll
    for (int k = NN - 1; k >= 0; --k) {
        T p = T(0);
#pragma unroll
        for (int s = 0; s < NS; ++s)
            if (LY::top(s) > k) p = p + Lr[s][k] * xl[s];   // rows not below k hold 0 here
        // the sum is the same in every lane, so the owner finishes x_k alone
        const int sk = LY::slot(k), lk = LY::lane(k);
        const T xk = (yl[sk] - quad_sum(p)) * Lr[sk][k];
        xl[sk] = (l == lk) ? xk : xl[sk];
    }
}

// x = M r: r_k comes from its owner by broadcast and every lane accumulates its rows, in order of k.
template <class LY, class T>
__device__ __forceinline__ void lanes4_inv_apply(const T (&r)[LY::NS], const T (&Mr)[LY::NS][LY::NN], T (&xl)[LY::NS]) {
#pragma unroll
    for (int s = 0; s < LY::NS; ++s) xl[s] = T(0);
#pragma unroll
    for (int k = 0; k < LY::NN; ++k) {
        const T rk = quad_bcast(r[LY::slot(k)], LY::lane(k));
#pragma unroll
        for (int s = 0; s < LY::NS; ++s) xl[s] = xl[s] + Mr[s][k] * rk;
    }
}

// M = H^-1 of every node of a 6-DOF model in FP32, column by column (column j solves
// L L' m = e_j with the factor), written over the factor planes as a packed lower triangle.  Runs
// after the factorization of every SCP iteration; each group of four lanes loads its node's
// factor rows before it stores anything, and no other group touches the node.
template <class M>
__global__ __launch_bounds__(256) void k_minv_lanes4(Dev<float> dv) {
    using T = float;
    using LY = Lanes4<M>;
    constexpr int NS = LY::NS, NN = LY::NN;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int g = (int)(gid >> 2), l = (int)(gid & 3);
    NodeId id;
    const T* prm;
    if (node_of<M>(dv, g, id, prm) < 0) return;   // the lanes of a group leave together
    const int P = dv.P;
    T Lr[NS][NN];
    lanes4_load_rows<false, LY>(l, [&](int t) { return dv.planes[(size_t)(PL_L + t) * P + g]; }, Lr);
#pragma unroll 1
    for (int j = 0; j < NN; ++j) {
        T r[NS], x[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) r[s] = (LY::held(s, l) && LY::comp(s, l) == j) ? T(1) : T(0);
        lanes4_chol_solve<LY>(r, Lr, l, x);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int row = LY::comp(s, l);
            if (LY::held(s, l) && row >= j) dv.planes[(size_t)(PL_L + tri(row, j)) * P + g] = x[s];
        }
    }
}

template <class M, class T>
__global__ __launch_bounds__(256) void k_step1_lanes4(Dev<T> dv, KParams<T> kp) {
    using LY = Lanes4<M>;
    constexpr int NX = M::NX, NU = M::NU, NN = M::NN, NXR = M::NXR, KM = M::KM, NS = LY::NS;
    const size_t gid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int g = (int)(gid >> 2), l = (int)(gid & 3);
    NodeId id;
    const T* prm;
    const int tr = node_of<M>(dv, g, id, prm);   // the lanes of a group share g and leave together
    if (tr < 0 || dv.flags[tr * FL_FIELDS + FL_DONE]) return;
    const int P = dv.P;
    const bool last = id.last();
    const T rf = rho_factor<T>(dv, kp, tr);
    const T rho_eq = kp.rho_eq * rf, rho_dyn = kp.rho_dyn * rf, rho_geo = kp.rho_geo * rf;
    auto at = [&](int plane, int node) -> T { return dv.planes[(size_t)plane * P + node]; };

    // w = mu_{i+1} + rho_dyn (z_{i+1} - d_i) on the owned rows (z, mu of node N+1 read as 0)
    T wl[4], dl[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int r = 4 * s + l;
        T zn = T(0), mn = T(0), d = T(0);
        if (r < NX) {
            d = at(PL_D + r, g);
            if (!last) {
                zn = at(PL_Z + r, g + 1);
                mn = at(PL_MU + r, g + 1);
            }
        }
        dl[s] = d;
        wl[s] = mn + rho_dyn * (zn - d);
    }
    T w[NX];
#pragma unroll
    for (int m = 0; m < NX; ++m) w[m] = m < LY::RB ? quad_xor(wl[m / 4], m % 4) : quad_bcast(wl[m / 4], m % 4);

    // owned columns of A (non-unit part) and of B
    T Al[4][NX], Bl[NX];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int k = 4 * s + l;
#pragma unroll
        for (int m = 0; m < NX; ++m) Al[s][m] = (k >= 3 && k < NX) ? at(PL_AR + LY::row(m, l) * NXR + (k - 3), g) : T(0);
    }
    // the control component of this lane, if any: k = NX + l, slot 4
    const int cu = l;
    const bool has_u = l < NU;
#pragma unroll
    for (int m = 0; m < NX; ++m) Bl[m] = has_u ? at(PL_B + LY::row(m, l) * NU + cu, g) : T(0);

    // right-hand side of the owned components (A'w over the rows in the lane's permuted order)
    T acc[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int k = 4 * s + l;
        const int s4 = s < 4 ? s : 3;   // state components sit in slots 0..3
        T v = T(0);
        if (s < 4 && k < NX) {
            T tx = wl[s4];   // unit columns of A: (A'w)_k = w_k, the lane's own row k
            if (k >= 3) {
                tx = T(0);
#pragma unroll
                for (int r = 0; r < NX; ++r) tx = tx + Al[s4][r] * w[r];
            }
            v = (at(PL_G0 + k, g) + (rho_eq * at(PL_Z + k, g) - at(PL_LAM + k, g))) + tx;
            v = v + (rho_geo * at(PL_CP + M::C_XBOX + k, g) - at(PL_DU + M::C_XBOX + k, g));
            if constexpr (M::QL) {
                if (k < 3) {
#pragma unroll
                    for (int j = 0; j < KM; ++j) {
                        const T rj = group_rho<M>(id, rho_geo, 3 + j);
                        v = v + (rj * at(PL_CP + M::C_HS + 3 * j + k, g) - at(PL_DU + M::C_HS + 3 * j + k, g));
                    }
                }
            } else {
                // lander: at most one more group per state component (glide cone on r, listed
                // (r_E, r_N, r_U); tilt on q_y, q_z; rate ball on w)
                const int slot = k < 3 ? M::C_GLIDE + (k + 2) % 3 : (k == 8 || k == 9) ? M::C_TILT + (k - 8)
                               : (k >= 10 && k < 13) ? M::C_RATE + (k - 10) : -1;
                if (slot >= 0) {
                    const T rx = group_rho<M>(id, rho_geo, 2);
                    v = v + (rx * at(PL_CP + slot, g) - at(PL_DU + slot, g));
                }
            }
        } else if (s == 4 && has_u) {
            T tu = T(0);
#pragma unroll
            for (int r = 0; r < NX; ++r) tu = tu + Bl[r] * w[r];
            v = tu + (rho_geo * at(PL_CP + M::C_UBOX + cu, g) - at(PL_DU + M::C_UBOX + cu, g));
            if constexpr (!M::QL) {
                // lander: thrust ball, linearized lower bound, gimbal cone (listed (T_y, T_z, T_x))
                const T ru = group_rho<M>(id, rho_geo, 5);
                v = v + (ru * at(PL_CP + M::C_TBALL + cu, g) - at(PL_DU + M::C_TBALL + cu, g));
                v = v + (ru * at(PL_CP + M::C_THS + cu, g) - at(PL_DU + M::C_THS + cu, g));
                const int sg = M::C_GIMB + (cu + 2) % 3;
                v = v + (ru * at(PL_CP + sg, g) - at(PL_DU + sg, g));
            }
        }
        acc[s] = v;
    }

    // owned rows of the factor (diagonal slots hold 1/L_kk; entries above the diagonal are 0) or of
    // the inverse, then the solve
    constexpr bool INV = StepInverse<M, T>::value;
    T Lr[NS][NN];
    lanes4_load_rows<INV, LY>(l, [&](int t) { return at(PL_L + t, g); }, Lr);
    T xl[NS];
    if constexpr (INV) lanes4_inv_apply<LY>(acc, Lr, xl);
    else lanes4_chol_solve<LY>(acc, Lr, l, xl);

    // x, u of the owned components (u = 0 at node N), then d_dyn = A x + B u + d
    T q[NX];
#pragma unroll
    for (int r = 0; r < NX; ++r) q[r] = T(0);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int k = 4 * s + l;
        if (s < 4 && k < NX) {
            dv.planes[(size_t)(PL_X + k) * P + g] = xl[s];
            if (s == 0) {
                q[0] = q[0] + (k < 3 ? xl[s] : T(0));   // entry 0 holds row l = k
            }
#pragma unroll
            for (int r = 0; r < NX; ++r) q[r] = q[r] + Al[s < 4 ? s : 3][r] * xl[s];
        } else if (s == 4 && has_u) {
            const T u = last ? T(0) : xl[s];
            dv.planes[(size_t)(PL_U + cu) * P + g] = u;
#pragma unroll
            for (int r = 0; r < NX; ++r) q[r] = q[r] + Bl[r] * u;
        }
    }
    // rows below RB: each lane receives the sums of its own rows; the rest by a sum over the group
#pragma unroll
    for (int n = 0; n < LY::RB / 4; ++n) {
        const T dd = quad_reduce_scatter(q + 4 * n) + dl[n];
        dv.planes[(size_t)(PL_DD + 4 * n + l) * P + g] = last ? T(0) : dd;   // no interval after node N
    }
#pragma unroll
    for (int r = LY::RB; r < NX; ++r) {
        const T dd = quad_sum(q[r]) + dl[r / 4];
        if (l == r % 4) dv.planes[(size_t)(PL_DD + r) * P + g] = last ? T(0) : dd;
    }
}

// ------------------------------------------------------------------------------------------
// a5-a8 of the 6-DOF models resident in one workgroup per trajectory
// ------------------------------------------------------------------------------------------
// The plain kernels stream every node from HBM twice per ADMM iteration.  Here one workgroup holds
// a whole trajectory (N + 1 <= 64 nodes, four lanes per node with the components split as in
// k_step1_lanes4) and runs all ADMM iterations of an SCP iteration with the node's factor rows,
// A and B columns, box bounds and ADMM state in registers.  Nodes are coupled only through z and
// mu of node i+1 (Step 1) and d_dyn of node i-1 (Step 2); those rows go through LDS, and two
// workgroup barriers per iteration order the writes and reads.  Every lane of the workgroup
// reaches every barrier: lanes past the trajectory's last node compute on zeros and store
// nothing.  The arithmetic of every component is that of k_step1_lanes4 and k_step234.  The last
// iteration also leaves the node-local residual pieces for k_resid, and the final iterate goes
// back to the planes.  Fixed budgets only (no residual test inside).  The lander's sets that
// couple components (cones, balls, the thrust half-space) are projected by every lane of the node
// on the components broadcast from their owners; each owner keeps its own component.
template <class M, class T, int ROWS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 2 : 1)))
void k_admm_resident(Dev<T> dv, KParams<T> kp) {
    using LY = Lanes4<M>;
    constexpr int NX = M::NX, NU = M::NU, NN = M::NN, NXR = M::NXR, NS = LY::NS, MAXN = ROWS;
    constexpr int KM = M::KM, KA = KM > 0 ? KM : 1;
    constexpr bool LD = M::ID == SCP_MODEL_LANDER6;
    constexpr bool QP = M::ID == SCP_MODEL_QUAD_PM;      // point-mass quadrotor: control ball
    constexpr bool MS = M::ID == SCP_MODEL_MARS3DOF;     // powered descent: glide cone, SOC
    // Neighbour rows, one per node.  A wavefront holds 16 nodes (four lanes each) and reads one
    // component slot of every node at once, i.e. 16 rows x 4 consecutive values; a row stride of
    // 20 values puts the 32 reads of each half-wavefront in 32 different LDS banks (a stride of 16
    // folds them onto 8 banks, a four-way conflict).
    constexpr int SR = 20;
    __shared__ T sz[MAXN][SR], smu[MAXN][SR], sdd[MAXN][SR];
    // With the inverse, the lane's columns of A live in LDS instead of registers, which leaves room
    // for the rows of the inverse at 2 waves per SIMD: row r of every slot at [r][4], so one
    // 16-byte read serves the four slots, with a lane stride that keeps the reads of 16 lanes in
    // distinct banks.  The workgroup's row capacity ROWS sizes it.
    constexpr bool ALDS = StepInverse<M, T>::value;
    constexpr int SA = lds_lane_stride<T>(4 * NX);
    __shared__ __attribute__((aligned(16))) T sA[ALDS ? 4 * MAXN : 1][ALDS ? SA : 4];
    const int tr = blockIdx.x;
    if (tr >= dv.n_traj || dv.flags[tr * FL_FIELDS + FL_DONE]) return;   // uniform over the workgroup
    const int* rec = dv.traj + tr * TR_FIELDS;
    if (rec[TR_MODEL] != M::ID) return;   // a mixed batch launches one kernel per model
    const int N = rec[TR_N], off = rec[TR_OFF];
    const int t = threadIdx.x, i = t >> 2, l = t & 3;
    const bool live = i <= N;
    const int g = off + (live ? i : 0);
    NodeId id;
    id.i = live ? i : 0;
    id.N = N;
    id.K = rec[TR_K];
    id.ball = QP && rec[TR_BALL] != 0;
    const bool first = id.first(), last = id.last();
    const int P = dv.P;
    // penalties of this trajectory: the same in every lane of the workgroup
    const T rf = rho_factor<T>(dv, kp, tr);
    const T rho_eq = wave_uniform(kp.rho_eq * rf), rho_dyn = wave_uniform(kp.rho_dyn * rf);
    const T rho_geo = wave_uniform(kp.rho_geo * rf);
    const T inv_geo = wave_uniform(T(1) / rho_geo), inv_sum = wave_uniform(T(1) / (rho_eq + rho_dyn));
    const T* prm = dv.params + (size_t)tr * SCP_PARAM_STRIDE;
    auto at = [&](int plane) -> T { return live ? dv.planes[(size_t)plane * P + g] : T(0); };
    auto put = [&](int plane, T v) {
        if (live) dv.planes[(size_t)plane * P + g] = v;
    };
    const int cu = l;   // control component of this lane (slot 4), if l < NU
    const bool has_u = l < NU;

    // node data of the owned components
    T dl[4], zl[4], laml[4], mul[4], g0l[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int r = 4 * s + l;
        const bool ok = r < NX;
        dl[s] = ok ? at(PL_D + r) : T(0);
        zl[s] = ok ? at(PL_Z + r) : T(0);
        laml[s] = ok ? at(PL_LAM + r) : T(0);
        mul[s] = ok ? at(PL_MU + r) : T(0);
        g0l[s] = ok ? at(PL_G0 + r) : T(0);
    }
    T Al[ALDS ? 1 : 4][NX], Bl[NX];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int k = 4 * s + l;
#pragma unroll
        for (int m = 0; m < NX; ++m) {
            const T a = (k >= 3 && k < NX) ? at(PL_AR + LY::row(m, l) * NXR + (k - 3)) : T(0);
            if constexpr (ALDS) sA[t][4 * m + s] = a;
            else Al[s][m] = a;
        }
    }
    // entry m of the lane's column copy of slot s
    auto acol = [&](int s, int m) -> T {
        if constexpr (ALDS) return sA[t][4 * m + s];
        else return Al[s][m];
    };
#pragma unroll
    for (int m = 0; m < NX; ++m) Bl[m] = has_u ? at(PL_B + LY::row(m, l) * NU + cu) : T(0);
    T cpb[NS], dub[NS], lol[NS], hil[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int k = LY::comp(s, l);
        const bool ok = LY::held(s, l);
        const int bs = s < 4 ? M::C_XBOX + k : M::C_UBOX + l;
        cpb[s] = ok ? at(PL_CP + bs) : T(0);
        dub[s] = ok ? at(PL_DU + bs) : T(0);
        lol[s] = ok ? at(PL_LO + k) : T(0);
        hil[s] = ok ? at(PL_HI + k) : T(0);
    }
    constexpr bool INV = StepInverse<M, T>::value;
    T Lr[NS][NN];
    // (the factor's rows and its solve below are written out here rather than through the
    // helpers of k_step1_lanes4: with the helpers the compiler allocates ~30 more registers for
    // the point-mass variants and spills 8 bytes per lane for the lander; the arithmetic is the same)
    if constexpr (INV) {
        lanes4_load_rows<true, LY>(l, [&](int t2) { return at(PL_L + t2); }, Lr);
    } else {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int row = LY::comp(s, l);
            const bool ok = LY::held(s, l);
#pragma unroll
            for (int j = 0; j < NN; ++j) {
                if (j <= LY::top(s)) Lr[s][j] = (ok && j <= row) ? at(PL_L + tri(row, j)) : T(0);
                else Lr[s][j] = T(0);
            }
        }
    }
    // quadrotors: half-space j: a_l (l < 3) or b (l = 3); copy and dual of position component l
    T own[KA], cph[KA], duh[KA];
#pragma unroll
    for (int j = 0; j < KA; ++j) own[j] = cph[j] = duh[j] = T(0);
    // the one further group of each owned state component (lander: glide cone on r, tilt on
    // q_y, q_z, rate ball on w; powered descent: glide cone on r), the further groups of the owned
    // control component (lander: thrust ball, lower bound, gimbal cone; point-mass quadrotor: the
    // control ball; powered descent: the SOC), and the lander's thrust half-space (a_l, or b in
    // lane 3)
    constexpr int NUG = LD ? 3 : (QP || MS) ? 1 : 0;
    T cpe[4], due[4], cu3[3], du3[3], own_h = T(0);
    // mirror slot of the further group of state component k, -1 if none
    auto xslot_of = [](int k) -> int {
        if constexpr (LD)
            return k < 3 ? Lander6::C_GLIDE + (k + 2) % 3 : (k == 8 || k == 9) ? Lander6::C_TILT + (k - 8)
                 : (k >= 10 && k < 13) ? Lander6::C_RATE + (k - 10) : -1;
        if constexpr (MS) return k < 3 ? Mars::C_CONE + k : -1;
        return -1;
    };
    // mirror slots of the further groups of control component c
    auto uslot_of = [](int c, int j) -> int {
        if constexpr (LD) return j == 0 ? Lander6::C_TBALL + c : j == 1 ? Lander6::C_THS + c : Lander6::C_GIMB + (c + 2) % 3;
        if constexpr (QP) return M::C_BALL + c;
        if constexpr (MS) return Mars::C_SOC + c;
        return -1;
    };
#pragma unroll
    for (int s = 0; s < 4; ++s) cpe[s] = due[s] = T(0);
#pragma unroll
    for (int j = 0; j < 3; ++j) cu3[j] = du3[j] = T(0);
    if constexpr (M::QL) {
#pragma unroll
        for (int j = 0; j < KM; ++j) {
            own[j] = at(PL_HS + 4 * j + l);
            cph[j] = l < 3 ? at(PL_CP + M::C_HS + 3 * j + l) : T(0);
            duh[j] = l < 3 ? at(PL_DU + M::C_HS + 3 * j + l) : T(0);
        }
    } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int xs = xslot_of(4 * s + l);
            if (xs >= 0) {
                cpe[s] = at(PL_CP + xs);
                due[s] = at(PL_DU + xs);
            }
        }
        if constexpr (LD) own_h = at(PL_HS + l);
    }
    if (has_u) {
#pragma unroll
        for (int j = 0; j < NUG; ++j) {
            cu3[j] = at(PL_CP + uslot_of(cu, j));
            du3[j] = at(PL_DU + uslot_of(cu, j));
        }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int r = 4 * s + l;
        if (live && r < NX) {
            sz[i][r] = zl[s];
            smu[i][r] = mul[s];
        }
    }
    const int K = kp.max_iters;
    T xl[NS], dds[4];
#pragma unroll
    for (int s = 0; s < NS; ++s) xl[s] = T(0);
#pragma unroll
    for (int s = 0; s < 4; ++s) dds[s] = T(0);
    __syncthreads();

    for (int it = 1; it <= K; ++it) {
        const bool chk = it == K;
        // ---- Step 1 ----
        T wl[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int r = 4 * s + l;
            T zn = T(0), mn = T(0);
            if (live && r < NX && !last) {
                zn = sz[i + 1][r];
                mn = smu[i + 1][r];
            }
            wl[s] = mn + rho_dyn * (zn - dl[s]);
        }
        T w[NX];
#pragma unroll
        for (int m = 0; m < NX; ++m) w[m] = m < LY::RB ? quad_xor(wl[m / 4], m % 4) : quad_bcast(wl[m / 4], m % 4);
        // With A in LDS: A'w of the four state slots first, each summed over the rows in order (rows
        // outermost, so that one read of A serves the four slots; columns the lane does not hold
        // are 0).  With A in registers each slot sums its own rows below, as the plain kernel does.
        T txs[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) txs[s] = T(0);
        if constexpr (ALDS) {
#pragma unroll
            for (int r = 0; r < NX; ++r) {
#pragma unroll
                for (int s = 0; s < 4; ++s) txs[s] = txs[s] + acol(s, r) * w[r];
            }
        }
        T acc[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int k = 4 * s + l;
            const int s4 = s < 4 ? s : 3;   // state components sit in slots 0..3
            T v = T(0);
            if (s < 4 && k < NX) {
                T tx = wl[s4];   // unit columns of A: (A'w)_k = w_k
                if (k >= 3) {
                    if constexpr (ALDS) {
                        tx = txs[s4];
                    } else {
                        tx = T(0);
#pragma unroll
                        for (int r = 0; r < NX; ++r) tx = tx + acol(s4, r) * w[r];
                    }
                }
                v = (g0l[s4] + (rho_eq * zl[s4] - laml[s4])) + tx;
                v = v + (rho_geo * cpb[s] - dub[s]);
                if constexpr (M::QL) {
                    if (k < 3) {
#pragma unroll
                        for (int j = 0; j < KM; ++j) {
                            const T rj = group_rho<M>(id, rho_geo, 3 + j);
                            v = v + (rj * cph[j] - duh[j]);
                        }
                    }
                } else {
                    if (xslot_of(k) >= 0) v = v + (group_rho<M>(id, rho_geo, 2) * cpe[s4] - due[s4]);
                }
            } else if (s == 4 && has_u) {
                T tu = T(0);
#pragma unroll
                for (int r = 0; r < NX; ++r) tu = tu + Bl[r] * w[r];
                v = tu + (rho_geo * cpb[s] - dub[s]);
                if constexpr (LD) {
                    const T ru = group_rho<M>(id, rho_geo, 5);
#pragma unroll
                    for (int j = 0; j < 3; ++j) v = v + (ru * cu3[j] - du3[j]);
                } else if constexpr (QP) {
                    v = v + (group_rho<M>(id, rho_geo, 2) * cu3[0] - du3[0]);   // control ball
                } else if constexpr (MS) {
                    v = v + (rho_geo * cu3[0] - du3[0]);                         // SOC
                }
            }
            acc[s] = v;
        }
        if constexpr (INV) {
            lanes4_inv_apply<LY>(acc, Lr, xl);
        } else {
            // the steps of lanes4_chol_solve
            T yl[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) yl[s] = T(0);
#pragma unroll
            for (int k = 0; k < NN; ++k) {
                const int sk = LY::slot(k), lk = LY::lane(k);
                const T yk = quad_bcast(acc[sk] * Lr[sk][k], lk);
                yl[sk] = (l == lk) ? yk : yl[sk];
#pragma unroll
                for (int s = 0; s < NS; ++s)
                    if (LY::top(s) > k) acc[s] = acc[s] - Lr[s][k] * yk;
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) xl[s] = T(0);
#pragma unroll
            for (int k = NN - 1; k >= 0; --k) {
                T p = T(0);
#pragma unroll
                for (int s = 0; s < NS; ++s)
                    if (LY::top(s) > k) p = p + Lr[s][k] * xl[s];
                const int sk = LY::slot(k), lk = LY::lane(k);
                const T xk = (yl[sk] - quad_sum(p)) * Lr[sk][k];
                xl[sk] = (l == lk) ? xk : xl[sk];
            }
        }
        // A x + B u: every entry gets its terms in slot order
        T q[NX];
#pragma unroll
        for (int r = 0; r < NX; ++r) q[r] = T(0);
        if constexpr (ALDS) {
            // rows outermost, one read of A per row; a slot the lane does not hold adds 0 * 0
            if (has_u && last) xl[4] = T(0);
            q[0] = q[0] + (l < 3 ? xl[0] : T(0));   // unit columns: entry 0 holds row l of slot 0
#pragma unroll
            for (int r = 0; r < NX; ++r) {
#pragma unroll
                for (int s = 0; s < 4; ++s) q[r] = q[r] + acol(s, r) * xl[s];
                q[r] = q[r] + Bl[r] * xl[4];
            }
        } else {
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int k = 4 * s + l;
                if (s < 4 && k < NX) {
                    if (s == 0) {
                        q[0] = q[0] + (k < 3 ? xl[s] : T(0));   // entry 0 holds row l = k
                    }
#pragma unroll
                    for (int r = 0; r < NX; ++r) q[r] = q[r] + acol(s < 4 ? s : 3, r) * xl[s];
                } else if (s == 4 && has_u) {
                    if (last) xl[s] = T(0);
#pragma unroll
                    for (int r = 0; r < NX; ++r) q[r] = q[r] + Bl[r] * xl[s];
                }
            }
        }
        // rows below RB: each lane receives the sums of its own rows; the rest by a sum over the group
#pragma unroll
        for (int n = 0; n < LY::RB / 4; ++n) {
            const T dd = quad_reduce_scatter(q + 4 * n) + dl[n];
            dds[n] = last ? T(0) : dd;   // no interval after node N
            if (live) sdd[i][4 * n + l] = dds[n];
        }
#pragma unroll
        for (int r = LY::RB; r < NX; ++r) {
            const T dd = quad_sum(q[r]) + dl[r / 4];
            if (l == r % 4) {
                dds[r / 4] = last ? T(0) : dd;
                if (live) sdd[i][r] = dds[r / 4];
            }
        }
        __syncthreads();
        // ---- Steps 2-4 ----
        T pm = T(0), xpos = T(0), uval = T(0), spu = T(0);
        T spv[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) spv[s] = T(0);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int k = 4 * s + l;
            const int s4 = s < 4 ? s : 3;
            if (s < 4 && k < NX) {
                const T x = xl[s], z0 = zl[s4];
                const T dp = (!first && live) ? sdd[i - 1][k] : T(0);
                const T z = first ? z0 : (((rho_eq * x + laml[s4]) + rho_dyn * dp) - mul[s4]) * inv_sum;
                const T cpo = cpb[s];
                const T cp = clampv(x + dub[s] * inv_geo, lol[s], hil[s]);
                if (!first) {
                    laml[s4] = laml[s4] + rho_eq * (x - z);
                    mul[s4] = mul[s4] + rho_dyn * (z - dp);
                }
                dub[s] = dub[s] + rho_geo * (x - cp);
                cpb[s] = cp;
                zl[s4] = z;
                if (chk) {
                    const T dz = z - z0;
                    spv[s4] = (first ? T(0) : rho_eq * dz) + rho_geo * (cp - cpo);
                    put(PL_DZ + k, dz);
                    if (!first) {
                        pm = nmax(pm, tabs(x - z));
                        pm = nmax(pm, tabs(z - dp));
                    }
                    pm = nmax(pm, tabs(x - cp));
                }
                if (s == 0) xpos = x;
            } else if (s == 4 && has_u) {
                const T u = xl[s];
                const T cpo = cpb[s];
                T cp = clampv(u + dub[s] * inv_geo, lol[s], hil[s]);
                const bool act = !last;
                dub[s] = act ? dub[s] + rho_geo * (u - cp) : T(0);
                if (!act) cp = T(0);
                cpb[s] = cp;
                uval = u;
                if (chk) {
                    spu = act ? rho_geo * (cp - cpo) : T(0);
                    if (act) pm = nmax(pm, tabs(u - cp));
                }
            }
        }
        if constexpr (M::QL) {
#pragma unroll
        for (int j = 0; j < KM; ++j) {
            if (first || j >= id.K) continue;   // uniform over the four lanes of a node
            const T a0 = quad_bcast(own[j], 0), a1 = quad_bcast(own[j], 1), a2 = quad_bcast(own[j], 2);
            const T b = quad_bcast(own[j], 3);
            const T v = xpos + duh[j] * inv_geo;
            const T v0 = quad_bcast(v, 0), v1 = quad_bcast(v, 1), v2 = quad_bcast(v, 2);
            const T tt = tmaxv(T(0), b - ((a0 * v0 + a1 * v1) + a2 * v2));
            const T cp = v + tt * own[j];
            if (l < 3) {
                const T cpo = cph[j];
                duh[j] = duh[j] + rho_geo * (xpos - cp);
                cph[j] = cp;
                if (chk) {
                    spv[0] = spv[0] + rho_geo * (cp - cpo);
                    pm = nmax(pm, tabs(xpos - cp));
                }
            }
        }
        if constexpr (QP) {
            // control ball on the components held by lanes 0..2 (slot 4); absent where the
            // trajectory has none and at node N, where its copy and dual stay 0
            const bool bact = !last && id.ball;
            const T vb = has_u ? uval + du3[0] * inv_geo : T(0);
            T v[3] = {quad_bcast(vb, 0), quad_bcast(vb, 1), quad_bcast(vb, 2)};
            proj_ball3(prm[SCP_P_UBALL], v);
            if (has_u) {
                const T cp = cu == 0 ? v[0] : cu == 1 ? v[1] : v[2];
                const T cpo = cu3[0];
                du3[0] = bact ? du3[0] + rho_geo * (uval - cp) : T(0);
                cu3[0] = bact ? cp : T(0);
                if (chk && bact) {
                    spu = spu + rho_geo * (cu3[0] - cpo);
                    pm = nmax(pm, tabs(uval - cp));
                }
            }
        }
        } else if constexpr (MS) {
            // powered descent: glide cone on r (components 0..2, lanes 0..2 of slot 0) at nodes
            // 1..N, SOC on (T, Gamma) (the four controls, slot 4) at nodes 0..N-1; where a group
            // does not exist its copy and dual stay 0
            const bool xact = !first, uact = !last;
            {
                const T kg = prm[SCP_P_GLIDE];
                const T vv = l < 3 ? xl[0] + due[0] * inv_geo : T(0);
                T v[3] = {quad_bcast(vv, 0), quad_bcast(vv, 1), quad_bcast(vv, 2)};
                proj_cone<3>(kg, T(1) / (T(1) + kg * kg), v);
                if (l < 3) {
                    const T cp = l == 0 ? v[0] : l == 1 ? v[1] : v[2];
                    const T cpo = cpe[0];
                    due[0] = xact ? due[0] + rho_geo * (xl[0] - cp) : T(0);
                    cpe[0] = xact ? cp : T(0);
                    if (chk && xact) {
                        spv[0] = spv[0] + rho_geo * (cpe[0] - cpo);
                        pm = nmax(pm, tabs(xl[0] - cp));
                    }
                }
            }
            {
                const T vs = has_u ? uval + du3[0] * inv_geo : T(0);
                T v[4] = {quad_bcast(vs, 0), quad_bcast(vs, 1), quad_bcast(vs, 2), quad_bcast(vs, 3)};
                proj_cone<4>(T(1), T(0.5), v);
                if (has_u) {
                    const T cp = cu == 0 ? v[0] : cu == 1 ? v[1] : cu == 2 ? v[2] : v[3];
                    const T cpo = cu3[0];
                    du3[0] = uact ? du3[0] + rho_geo * (uval - cp) : T(0);
                    cu3[0] = uact ? cp : T(0);
                    if (chk && uact) {
                        spu = spu + rho_geo * (cu3[0] - cpo);
                        pm = nmax(pm, tabs(uval - cp));
                    }
                }
            }
        } else {
            // lander: the sets coupling components; a group exists at nodes 1..N (state) or
            // 0..N-1 (thrust), and where it does not its copy and dual stay 0
            const bool xact = !first, uact = !last;
            auto upd_x = [&](int s, T var, T cp) {
                const T cpo = cpe[s];
                due[s] = xact ? due[s] + rho_geo * (var - cp) : T(0);
                cpe[s] = xact ? cp : T(0);
                if (chk && xact) {
                    spv[s] = spv[s] + rho_geo * (cpe[s] - cpo);
                    pm = nmax(pm, tabs(var - cp));
                }
            };
            auto upd_u = [&](int j, T cp) {
                const T cpo = cu3[j];
                du3[j] = uact ? du3[j] + rho_geo * (uval - cp) : T(0);
                cu3[j] = uact ? cp : T(0);
                if (chk && uact) {
                    spu = spu + rho_geo * (cu3[j] - cpo);
                    pm = nmax(pm, tabs(uval - cp));
                }
            };
            {   // glide cone on (r_E, r_N, r_U): owners lanes 1, 2, 0 (slot 0)
                const T kg = prm[SCP_P_GLIDE];
                const T vv = l < 3 ? xl[0] + due[0] * inv_geo : T(0);
                T v[3] = {quad_bcast(vv, 1), quad_bcast(vv, 2), quad_bcast(vv, 0)};
                proj_cone<3>(kg, T(1) / (T(1) + kg * kg), v);
                const int o = (l + 2) % 3;
                if (l < 3) upd_x(0, xl[0], o == 0 ? v[0] : o == 1 ? v[1] : v[2]);
            }
            {   // tilt on (q_y, q_z): owners lanes 0, 1 (slot 2)
                const T vv = l < 2 ? xl[2] + due[2] * inv_geo : T(0);
                T v[2] = {quad_bcast(vv, 0), quad_bcast(vv, 1)};
                proj_ball2(prm[SCP_P_TILT], v);
                if (l < 2) upd_x(2, xl[2], l == 0 ? v[0] : v[1]);
            }
            {   // rate ball on w: owners lanes 2, 3 (slot 2) and 0 (slot 3)
                const T vv = (l >= 2) ? xl[2] + due[2] * inv_geo : (l == 0 ? xl[3] + due[3] * inv_geo : T(0));
                T v[3] = {quad_bcast(vv, 2), quad_bcast(vv, 3), quad_bcast(vv, 0)};
                proj_ball3(prm[SCP_P_WMAX], v);
                if (l >= 2) upd_x(2, xl[2], l == 2 ? v[0] : v[1]);
                if (l == 0) upd_x(3, xl[3], v[2]);
            }
            // thrust component c is held by lane c (slot 4)
            constexpr int L0 = 0, L1 = 1, L2 = 2;
            {   // thrust magnitude upper bound
                const T vb = has_u ? uval + du3[0] * inv_geo : T(0);
                T v[3] = {quad_bcast(vb, L0), quad_bcast(vb, L1), quad_bcast(vb, L2)};
                proj_ball3(prm[SCP_P_TMAX], v);
                if (has_u) upd_u(0, cu == 0 ? v[0] : cu == 1 ? v[1] : v[2]);
            }
            {   // linearized lower thrust bound
                const T a[3] = {quad_bcast(own_h, 0), quad_bcast(own_h, 1), quad_bcast(own_h, 2)};
                const T bh = quad_bcast(own_h, 3);
                const T vh = has_u ? uval + du3[1] * inv_geo : T(0);
                T v[3] = {quad_bcast(vh, L0), quad_bcast(vh, L1), quad_bcast(vh, L2)};
                proj_halfspace(a, bh, v);
                if (has_u) upd_u(1, cu == 0 ? v[0] : cu == 1 ? v[1] : v[2]);
            }
            {   // gimbal cone on (T_y, T_z, T_x)
                const T kq = prm[SCP_P_GIMBAL];
                const T vq = has_u ? uval + du3[2] * inv_geo : T(0);
                T v[3] = {quad_bcast(vq, L1), quad_bcast(vq, L2), quad_bcast(vq, L0)};
                proj_cone<3>(kq, T(1) / (T(1) + kq * kq), v);
                const int o = (cu + 2) % 3;
                if (has_u) upd_u(2, o == 0 ? v[0] : o == 1 ? v[1] : v[2]);
            }
        }
        if (chk) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int k = 4 * s + l;
                if (k < NX) put(PL_SP + k, spv[s]);
            }
            if (has_u) put(PL_SP + NX + cu, spu);
            pm = nmax(pm, quad_perm<0xB1>(pm));
            pm = nmax(pm, quad_perm<0x4E>(pm));
            if (l == 0) put(PL_RP, pm);
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int r = 4 * s + l;
            if (live && r < NX) {
                sz[i][r] = zl[s];
                smu[i][r] = mul[s];
            }
        }
        __syncthreads();
    }
    if (K == 0) return;
    // the final iterate back to the planes
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int k = 4 * s + l;
        const int s4 = s < 4 ? s : 3;
        if (s < 4 && k < NX) {
            put(PL_X + k, xl[s]);
            put(PL_Z + k, zl[s4]);
            put(PL_LAM + k, laml[s4]);
            put(PL_MU + k, mul[s4]);
            put(PL_DD + k, dds[s4]);
            put(PL_CP + M::C_XBOX + k, cpb[s]);
            put(PL_DU + M::C_XBOX + k, dub[s]);
        } else if (s == 4 && has_u) {
            put(PL_U + cu, xl[s]);
            put(PL_CP + M::C_UBOX + cu, cpb[s]);
            put(PL_DU + M::C_UBOX + cu, dub[s]);
        }
    }
    if constexpr (M::QL) {
        if (l < 3 && !first) {
#pragma unroll
            for (int j = 0; j < KM; ++j) {
                if (j < id.K) {
                    put(PL_CP + M::C_HS + 3 * j + l, cph[j]);
                    put(PL_DU + M::C_HS + 3 * j + l, duh[j]);
                }
            }
        }
    } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int xs = xslot_of(4 * s + l);
            if (xs >= 0) {
                put(PL_CP + xs, cpe[s]);
                put(PL_DU + xs, due[s]);
            }
        }
    }
    if (has_u) {
#pragma unroll
        for (int j = 0; j < NUG; ++j) {
            put(PL_CP + uslot_of(cu, j), cu3[j]);
            put(PL_DU + uslot_of(cu, j), du3[j]);
        }
    }
}

// ------------------------------------------------------------------------------------------
// a6-a8: Steps 2-4 (+ node-local residual pieces on check iterations)
// ------------------------------------------------------------------------------------------
template <class M, class T>
__global__ __launch_bounds__(256) void k_step234(Dev<T> dv, KParams<T> kp, int check) {
    constexpr int NX = M::NX, NU = M::NU, NN = M::NN;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    NodeId id;
    const T* prm;
    const int tr = node_of<M>(dv, g, id, prm);
    if (tr < 0 || dv.flags[tr * FL_FIELDS + FL_DONE]) return;
    const int P = dv.P;
    const bool grouped0 = id.first() && dv.traj[tr * TR_FIELDS + TR_GSIZE] > 1;
    const Rho<T> rho = rho_of<T>(kp, rho_factor<T>(dv, kp, tr));
    NodeConst<M, T> nc;
    ldp<NN>(PL(dv, PL_LO), P, g, nc.lo);
    ldp<NN>(PL(dv, PL_HI), P, g, nc.hi);
    if constexpr (M::HSD) ldp<M::NHS>(PL(dv, PL_HS), P, g, nc.hs);
    NodeState<M, T> s;
    ldp<NX>(PL(dv, PL_X), P, g, s.x);
    ldp<NU>(PL(dv, PL_U), P, g, s.u);
    ldp<NX>(PL(dv, PL_Z), P, g, s.z);
    ldp<NX>(PL(dv, PL_LAM), P, g, s.lam);
    ldp<NX>(PL(dv, PL_MU), P, g, s.mu);
    ldp<M::C>(PL(dv, PL_CP), P, g, s.cp);
    ldp<M::C>(PL(dv, PL_DU), P, g, s.du);
    T dp[NX];
    if (!id.first()) ldp<NX>(PL(dv, PL_DD), P, g - 1, dp);
    else {
#pragma unroll
        for (int r = 0; r < NX; ++r) dp[r] = T(0);
    }
    T zold[NX], cpold[M::C];
#pragma unroll
    for (int r = 0; r < NX; ++r) zold[r] = s.z[r];
#pragma unroll
    for (int k = 0; k < M::C; ++k) cpold[k] = s.cp[k];
    const T ball_r = prm[SCP_P_UBALL], kappa = prm[SCP_P_GLIDE];
    const T inv1k2 = T(1) / (T(1) + kappa * kappa);
    step2<M, T>(id, rho, s, dp);
    step3<M, T>(id, rho, nc, s, ball_r, kappa, inv1k2, prm);
    if (grouped0) {
        // node 0 of a consensus group: u copies are averaged by k_group, which also
        // finishes Step 4 and the residual pieces of those slots; keep the old copies.
#pragma unroll
        for (int k = 0; k < M::C; ++k)
            if (slot_is_u<M>(k)) PL(dv, PL_MER)[(size_t)slot_comp_u<M>(k) * P + g] = cpold[k];
    }
    // Step 4 (skip the u slots of a grouped node 0: k_group does them after averaging)
    if (!id.first()) {
#pragma unroll
        for (int r = 0; r < NX; ++r) {
            s.lam[r] = s.lam[r] + rho.eq * (s.x[r] - s.z[r]);
            s.mu[r] = s.mu[r] + rho.dyn * (s.z[r] - dp[r]);
        }
    }
#pragma unroll
    for (int k = 0; k < M::C; ++k) {
        if (grouped0 && slot_is_u<M>(k)) continue;
        const bool act = group_active<M>(id, slot_group<M>(k));
        const T v = s.du[k] + rho.geo * (slot_var<M, T>(s, k) - s.cp[k]);
        s.du[k] = act ? v : T(0);
    }
#pragma unroll
    for (int k = 0; k < M::C; ++k)   // copies of groups absent at this node are stored as 0
        if (!group_active<M>(id, slot_group<M>(k))) s.cp[k] = T(0);
    stp<NX>(PL(dv, PL_Z), P, g, s.z);
    stp<NX>(PL(dv, PL_LAM), P, g, s.lam);
    stp<NX>(PL(dv, PL_MU), P, g, s.mu);
    stp<M::C>(PL(dv, PL_CP), P, g, s.cp);
    stp<M::C>(PL(dv, PL_DU), P, g, s.du);
    if (check) {
        T dz[NX], dcp[M::C], sp[NN];
#pragma unroll
        for (int r = 0; r < NX; ++r) dz[r] = s.z[r] - zold[r];
#pragma unroll
        for (int k = 0; k < M::C; ++k) dcp[k] = (grouped0 && slot_is_u<M>(k)) ? T(0) : s.cp[k] - cpold[k];
        dual_res_own<M, T>(id, rho, dz, dcp, sp, grouped0);
        T rp = grouped0 ? primal_res_skip_u<M, T>(id, s, dp) : primal_res<M, T>(id, s, dp);
        stp<NX>(PL(dv, PL_DZ), P, g, dz);
        stp<NN>(PL(dv, PL_SP), P, g, sp);
        PL(dv, PL_RP)[g] = rp;
    }
}

// node 0 of every consensus group: average the projected first-control copies over the
// scenarios (fixed order), then Step 4 and residual pieces of those slots.  One thread per group.
template <class M, class T>
__global__ void k_group(Dev<T> dv, KParams<T> kp, int check) {
    constexpr int NX = M::NX, NU = M::NU, NN = M::NN;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= dv.n_groups) return;
    const int t0 = dv.groups[q];
    const int* rec = dv.traj + t0 * TR_FIELDS;
    if (rec[TR_MODEL] != M::ID || dv.flags[t0 * FL_FIELDS + FL_DONE]) return;
    const int S = rec[TR_GSIZE];
    const int P = dv.P;
    const T rho_geo = kp.rho_geo;
    T acc[M::C];
#pragma unroll
    for (int k = 0; k < M::C; ++k) acc[k] = T(0);
    for (int m = 0; m < S; ++m) {
        const int g = dv.traj[(t0 + m) * TR_FIELDS + TR_OFF];
#pragma unroll
        for (int k = 0; k < M::C; ++k)
            if (slot_is_u<M>(k)) acc[k] = acc[k] + PL(dv, PL_CP)[(size_t)k * P + g];
    }
    for (int m = 0; m < S; ++m) {
        const int tr = t0 + m;
        const int g = dv.traj[tr * TR_FIELDS + TR_OFF];
        NodeId id;
        id.i = 0;
        id.N = rec[TR_N];
        id.K = dv.traj[tr * TR_FIELDS + TR_K];
        id.ball = dv.traj[tr * TR_FIELDS + TR_BALL] != 0;
        T u[NU], sp[NN];
        ldp<NU>(PL(dv, PL_U), P, g, u);
        if (check) ldp<NN>(PL(dv, PL_SP), P, g, sp);
        T rp = check ? PL(dv, PL_RP)[g] : T(0);
#pragma unroll
        for (int k = 0; k < M::C; ++k) {
            if (!slot_is_u<M>(k)) continue;
            const bool act = group_active<M>(id, slot_group<M>(k));
            const T mean = act ? acc[k] / T(S) : T(0);
            const T old = PL(dv, PL_MER)[(size_t)slot_comp_u<M>(k) * P + g];
            const T var = u[slot_comp<M>(k)];
            T du = PL(dv, PL_DU)[(size_t)k * P + g];
            du = act ? du + rho_geo * (var - mean) : T(0);
            PL(dv, PL_CP)[(size_t)k * P + g] = mean;
            PL(dv, PL_DU)[(size_t)k * P + g] = du;
            if (check && act) {
                sp[NX + slot_comp<M>(k)] = sp[NX + slot_comp<M>(k)] + rho_geo * (mean - old);
                rp = nmax(rp, tabs(var - mean));
            }
        }
        if (check) {
            stp<NN>(PL(dv, PL_SP), P, g, sp);
            PL(dv, PL_RP)[g] = rp;
        }
    }
}

// a9: finish the dual residual with the neighbour term and reduce per trajectory.
template <class M, class T>
__global__ __launch_bounds__(256) void k_resid(Dev<T> dv, KParams<T> kp) {
    constexpr int NX = M::NX, NU = M::NU, NN = M::NN, NXR = M::NXR;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    NodeId id;
    const T* prm;
    const int tr = node_of<M>(dv, g, id, prm);
    if (tr < 0 || dv.flags[tr * FL_FIELDS + FL_DONE]) return;
    const int P = dv.P;
    const Rho<T> rho = rho_of<T>(kp, rho_factor<T>(dv, kp, tr));
    T Ar[NX * NXR], B[NX * NU], sp[NN], dzn[NX];
    ldp<NX * NXR>(PL(dv, PL_AR), P, g, Ar);
    ldp<NX * NU>(PL(dv, PL_B), P, g, B);
    ldp<NN>(PL(dv, PL_SP), P, g, sp);
    if (!id.last()) ldp<NX>(PL(dv, PL_DZ), P, g + 1, dzn);
    else {
#pragma unroll
        for (int r = 0; r < NX; ++r) dzn[r] = T(0);
    }
    const T rd = dual_res_finish<M, T>(id, rho, Ar, B, sp, dzn);
    const T rp = PL(dv, PL_RP)[g];
    atomicMax(&dv.red[2 * tr], res_bits(rp));
    atomicMax(&dv.red[2 * tr + 1], res_bits(rd));
}

// per trajectory (group leader): residual test, convergence mask, info.
template <class T>
__global__ void k_check(Dev<T> dv, KParams<T> kp, int j, int test) {
    const int tr = blockIdx.x * blockDim.x + threadIdx.x;
    if (tr >= dv.n_traj) return;
    const int* rec = dv.traj + tr * TR_FIELDS;
    if (rec[TR_MEMBER] != 0 || dv.flags[tr * FL_FIELDS + FL_DONE]) return;
    const int S = rec[TR_GSIZE];
    unsigned long long bp = 0ull, bd = 0ull;
    for (int m = 0; m < S; ++m) {
        bp = max(bp, dv.red[2 * (tr + m)]);
        bd = max(bd, dv.red[2 * (tr + m) + 1]);
        dv.red[2 * (tr + m)] = 0ull;
        dv.red[2 * (tr + m) + 1] = 0ull;
    }
    const T rp = T(bits_res(bp)), rd = T(bits_res(bd));
    const bool conv = test && (rp <= kp.eps_p) && (rd <= kp.eps_d);
    for (int m = 0; m < S; ++m) {
        double* inf = dv.info + (size_t)(tr + m) * SCP_INFO_FIELDS;
        inf[SCP_I_RP] = (double)rp;
        inf[SCP_I_RD] = (double)rd;
        if (conv) {
            dv.flags[(tr + m) * FL_FIELDS + FL_DONE] = 1;
            dv.flags[(tr + m) * FL_FIELDS + FL_ITERS] = j;
        }
    }
}

// ------------------------------------------------------------------------------------------
// a10: merit terms of the candidate, ratio test, nominal update
// ------------------------------------------------------------------------------------------
template <class M, class T>
__global__ __launch_bounds__(256) void k_acc_nodes(Dev<T> dv, KParams<T> kp) {
    constexpr int NX = M::NX, NU = M::NU;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    NodeId id;
    const T* prm;
    const int tr = node_of<M>(dv, g, id, prm);
    if (tr < 0) return;
    const int P = dv.P;
    T x[NX], u[NU], dd[NX];
    ldp<NX>(PL(dv, PL_X), P, g, x);
    ldp<NU>(PL(dv, PL_U), P, g, u);
    T pen = T(0), pmod = T(0);
    if (!id.last()) {
        T xn[NX], F[NX];
        ldp<NX>(PL(dv, PL_DD), P, g, dd);
        ldp<NX>(PL(dv, PL_X), P, g + 1, xn);
        rk4<M, T>(prm, x, u, F);
#pragma unroll
        for (int r = 0; r < NX; ++r) pen = pen + tabs(xn[r] - F[r]);
#pragma unroll
        for (int r = 0; r < NX; ++r) pmod = pmod + tabs(xn[r] - dd[r]);
    }
    PL(dv, PL_MER)[(size_t)MER_COST_NEW * P + g] = node_cost<M, T>(prm, id, x, u);
    PL(dv, PL_MER)[(size_t)MER_PEN_NEW * P + g] = pen;
    PL(dv, PL_MER)[(size_t)MER_PEN_MOD * P + g] = pmod;
}

// One wavefront per trajectory (group leader): the lanes stage the node terms of up to 64 nodes
// at a time in LDS with coalesced loads, and lane 0 sums them in node order (the sums are those
// of a single thread walking the nodes, without its chain of dependent global loads).
template <class T>
__global__ __launch_bounds__(64) void k_acc_traj(Dev<T> dv, KParams<T> kp) {
    __shared__ T sm[5][64];
    const int tr = blockIdx.x, t = threadIdx.x;
    if (tr >= dv.n_traj) return;   // uniform over the workgroup, as the next test
    const int* rec = dv.traj + tr * TR_FIELDS;
    if (rec[TR_MEMBER] != 0) return;
    const int S = rec[TR_GSIZE];
    const int P = dv.P;
    const T* mer = dv.planes + (size_t)PL_MER * P;
    T mnom = T(0), mnew = T(0), mmod = T(0);
    for (int m = 0; m < S; ++m) {
        const int* r = dv.traj + (tr + m) * TR_FIELDS;
        const int off = r[TR_OFF], n = r[TR_N] + 1;
        T J0 = T(0), p0 = T(0), J1 = T(0), p1 = T(0), pm = T(0);
        for (int c = 0; c < n; c += 64) {
            const int i = c + t;
            if (i < n) {
                sm[0][t] = mer[(size_t)MER_COST_NOM * P + off + i];
                sm[1][t] = mer[(size_t)MER_COST_NEW * P + off + i];
                sm[2][t] = mer[(size_t)MER_PEN_NOM * P + off + i];
                sm[3][t] = mer[(size_t)MER_PEN_NEW * P + off + i];
                sm[4][t] = mer[(size_t)MER_PEN_MOD * P + off + i];
            }
            __syncthreads();
            if (t == 0) {
                const int e = min(64, n - c);          // nodes of this chunk
                const int ep = min(64, n - 1 - c);     // of them, nodes with an interval after them
                for (int q = 0; q < e; ++q) {
                    J0 = J0 + sm[0][q];
                    J1 = J1 + sm[1][q];
                }
                for (int q = 0; q < ep; ++q) {
                    p0 = p0 + sm[2][q];
                    p1 = p1 + sm[3][q];
                    pm = pm + sm[4][q];
                }
            }
            __syncthreads();
        }
        mnom = mnom + (J0 + kp.merit_w * p0);
        mnew = mnew + (J1 + kp.merit_w * p1);
        mmod = mmod + (J1 + kp.merit_w * pm);
    }
    if (t != 0) return;
    const AcceptOut<T> a = accept_rule<T>(kp.eta0, kp.eta1, kp.eta2, kp.shrink, kp.grow, kp.delta_max, mnom, mnew,
                                          mmod, dv.rt[tr * RT_FIELDS + RT_DELTA]);
    for (int m = 0; m < S; ++m) {
        const int t = tr + m;
        double* inf = dv.info + (size_t)t * SCP_INFO_FIELDS;
        int* fl = dv.flags + t * FL_FIELDS;
        const int iters = fl[FL_DONE] ? fl[FL_ITERS] : kp.max_iters;
        inf[SCP_I_ADMM_ITERS] += (double)iters;
        inf[SCP_I_NACCEPT] += a.accept ? 1.0 : 0.0;
        inf[SCP_I_RATIO] = (double)a.ratio;
        inf[SCP_I_MERIT] = (double)mnew;
        inf[SCP_I_DELTA] = (double)a.delta;
        int st = fl[FL_STATUS] | (a.nonfinite ? SCP_ST_NONFINITE : 0);
        if (kp.blowup) {   // inf[SCP_I_RP]: the residual of this SCP iteration's last ADMM iteration (k_check)
            T rp0 = dv.rt[t * RT_FIELDS + RT_RP0], rpmax = dv.rt[t * RT_FIELDS + RT_RPMAX];
            blowup_track<T>(rp0, rpmax, T(inf[SCP_I_RP]));
            st |= blowup_status<T>(rp0, rpmax);
            dv.rt[t * RT_FIELDS + RT_RP0] = rp0;
            dv.rt[t * RT_FIELDS + RT_RPMAX] = rpmax;
        }
        if (fl[FL_DONE]) st |= SCP_ST_CONVERGED;
        else st &= ~SCP_ST_CONVERGED;
        fl[FL_STATUS] = st;
        inf[SCP_I_STATUS] = (double)st;
        fl[FL_ACCEPT] = a.accept ? 1 : 0;
        dv.rt[t * RT_FIELDS + RT_DELTA] = a.delta;
    }
    if (kp.adapt_mu > 0.0) {   // residuals of this SCP iteration's last ADMM iteration (k_check)
        const double* li = dv.info + (size_t)tr * SCP_INFO_FIELDS;
        const T f = T(adapt_factor((double)dv.rt[tr * RT_FIELDS + RT_RHOS], li[SCP_I_RP], li[SCP_I_RD], kp.adapt_mu,
                                   kp.adapt_tau));
        for (int m = 0; m < S; ++m) dv.rt[(tr + m) * RT_FIELDS + RT_RHOS] = f;
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_acc_apply(Dev<T> dv) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= dv.n_nodes) return;
    const int tr = dv.node_traj[g];
    if (tr < 0 || !dv.flags[tr * FL_FIELDS + FL_ACCEPT]) return;
    const int P = dv.P;
#pragma unroll
    for (int r = 0; r < SCP_MAX_NX; ++r) PL(dv, PL_XBAR)[(size_t)r * P + g] = PL(dv, PL_X)[(size_t)r * P + g];
#pragma unroll
    for (int r = 0; r < SCP_MAX_NU; ++r) PL(dv, PL_UBAR)[(size_t)r * P + g] = PL(dv, PL_U)[(size_t)r * P + g];
}

// metrics of the nominal: per node, then per trajectory in node order
template <class M, class T>
__global__ __launch_bounds__(256) void k_met_nodes(Dev<T> dv) {
    constexpr int NX = M::NX, NU = M::NU;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    NodeId id;
    const T* prm;
    const int tr = node_of<M>(dv, g, id, prm);
    if (tr < 0) return;
    const int P = dv.P;
    T x[NX], u[NU];
    ldp<NX>(PL(dv, PL_XBAR), P, g, x);
    ldp<NU>(PL(dv, PL_UBAR), P, g, u);
    T dfc = T(0);
    if (!id.last()) {
        T xn[NX], F[NX];
        ldp<NX>(PL(dv, PL_XBAR), P, g + 1, xn);
        rk4<M, T>(prm, x, u, F);
#pragma unroll
        for (int r = 0; r < NX; ++r) dfc = nmax(dfc, tabs(xn[r] - F[r]));
    }
    PL(dv, PL_MER)[(size_t)MER_DEFECT * P + g] = dfc;
    PL(dv, PL_MER)[(size_t)MER_COST_NEW * P + g] = node_cost<M, T>(prm, id, x, u);
    PL(dv, PL_MER)[(size_t)MER_VIOL * P + g] = node_violation<M, T>(prm, id, x, u);
    PL(dv, PL_MER)[(size_t)MER_BND * P + g] = node_bnd_err<M, T>(prm, id, x);
}

template <class T>
__global__ void k_met_traj(Dev<T> dv) {
    const int tr = blockIdx.x * blockDim.x + threadIdx.x;
    if (tr >= dv.n_traj) return;
    const int* rec = dv.traj + tr * TR_FIELDS;
    const int off = rec[TR_OFF], n = rec[TR_N] + 1, P = dv.P;
    const T* mer = dv.planes + (size_t)PL_MER * P;
    T J = T(0), dfc = T(0), vi = T(0), be = T(0);
    for (int i = 0; i < n; ++i) {
        J = J + mer[(size_t)MER_COST_NEW * P + off + i];
        dfc = nmax(dfc, mer[(size_t)MER_DEFECT * P + off + i]);
        vi = nmax(vi, mer[(size_t)MER_VIOL * P + off + i]);
        be = nmax(be, mer[(size_t)MER_BND * P + off + i]);
    }
    double* inf = dv.info + (size_t)tr * SCP_INFO_FIELDS;
    inf[SCP_I_COST] = (double)J;
    inf[SCP_I_DEFECT] = (double)dfc;
    inf[SCP_I_VIOL] = (double)vi;
    inf[SCP_I_BNDERR] = (double)be;
}

template <class T>
__global__ void k_reset(Dev<T> dv, int reset_delta) {
    const int tr = blockIdx.x * blockDim.x + threadIdx.x;
    if (tr >= dv.n_traj) return;
    double* inf = dv.info + (size_t)tr * SCP_INFO_FIELDS;
#pragma unroll
    for (int k = 0; k < SCP_INFO_FIELDS; ++k) inf[k] = 0.0;
    int* fl = dv.flags + tr * FL_FIELDS;
    fl[FL_DONE] = 0;
    fl[FL_ITERS] = 0;
    fl[FL_ACCEPT] = 0;
    fl[FL_STATUS] = 0;
    dv.red[2 * tr] = 0ull;
    dv.red[2 * tr + 1] = 0ull;
    if (reset_delta) {
        dv.rt[tr * RT_FIELDS + RT_DELTA] = dv.params[(size_t)tr * SCP_PARAM_STRIDE + SCP_P_DELTA];
        dv.rt[tr * RT_FIELDS + RT_RHOS] = T(1);
        dv.rt[tr * RT_FIELDS + RT_RP0] = T(0);
        dv.rt[tr * RT_FIELDS + RT_RPMAX] = T(0);
    }
    inf[SCP_I_DELTA] = (double)dv.rt[tr * RT_FIELDS + RT_DELTA];
}

// restore the initial guess as the nominal and clear every ADMM iterate and dual
template <class T>
__global__ __launch_bounds__(256) void k_reset_state(Dev<T> dv) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= dv.n_nodes) return;
    const int P = dv.P;
#pragma unroll
    for (int r = 0; r < SCP_MAX_NX; ++r) PL(dv, PL_XBAR)[(size_t)r * P + g] = PL(dv, PL_XG)[(size_t)r * P + g];
#pragma unroll
    for (int r = 0; r < SCP_MAX_NU; ++r) PL(dv, PL_UBAR)[(size_t)r * P + g] = PL(dv, PL_UG)[(size_t)r * P + g];
    // x, u, z, lambda, mu, d_dyn, copies, duals: the slots of this node's model
    const int model = dv.traj[dv.node_traj[g] * TR_FIELDS + TR_MODEL];
    const int nx = model_nx(model), nu = model_nu(model), nc = model_slots(model);
    for (int k = 0; k < nx; ++k) {
        PL(dv, PL_X)[(size_t)k * P + g] = T(0);
        PL(dv, PL_Z)[(size_t)k * P + g] = T(0);
        PL(dv, PL_LAM)[(size_t)k * P + g] = T(0);
        PL(dv, PL_MU)[(size_t)k * P + g] = T(0);
        PL(dv, PL_DD)[(size_t)k * P + g] = T(0);
    }
    for (int k = 0; k < nu; ++k) PL(dv, PL_U)[(size_t)k * P + g] = T(0);
    for (int k = 0; k < nc; ++k) {
        PL(dv, PL_CP)[(size_t)k * P + g] = T(0);
        PL(dv, PL_DU)[(size_t)k * P + g] = T(0);
    }
}

// gather one field of every node into a dense [node][width] array
template <class T>
__global__ __launch_bounds__(256) void k_gather(Dev<T> dv, int plane, int width, int mode, T* out) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= dv.n_nodes) return;
    const int tr = dv.node_traj[g];
    const int model = dv.traj[tr * TR_FIELDS + TR_MODEL];
    const int P = dv.P;
    T* o = out + (size_t)g * width;
    const int nx = model_nx(model), nu = model_nu(model), nxr = nx - 3;
    if (mode == 1) {
        // dense A (SCP_MAX_NX x SCP_MAX_NX, the model's nx x nx block leading) from the stored
        // non-unit columns
        const int N = dv.traj[tr * TR_FIELDS + TR_N], i = g - dv.traj[tr * TR_FIELDS + TR_OFF];
        for (int r = 0; r < SCP_MAX_NX; ++r)
            for (int c = 0; c < SCP_MAX_NX; ++c) {
                T v = T(0);
                if (r < nx && c < nx) {
                    if (c < 3) v = (i < N && r == c) ? T(1) : T(0);
                    else v = PL(dv, PL_AR)[(size_t)(r * nxr + (c - 3)) * P + g];
                }
                o[r * SCP_MAX_NX + c] = v;
            }
    } else if (mode == 2) {
        for (int r = 0; r < SCP_MAX_NX; ++r)
            for (int c = 0; c < SCP_MAX_NU; ++c)
                o[r * SCP_MAX_NU + c] = (r < nx && c < nu) ? PL(dv, PL_B)[(size_t)(r * nu + c) * P + g] : T(0);
    } else if (mode == 3) {
        // box bounds: x part then u part at fixed offsets 0..SCP_MAX_NX-1 / SCP_MAX_NX..
        for (int k = 0; k < SCP_MAX_NX + SCP_MAX_NU; ++k) {
            T v = T(0);
            if (k < SCP_MAX_NX && k < nx) v = PL(dv, plane)[(size_t)k * P + g];
            if (k >= SCP_MAX_NX && k - SCP_MAX_NX < nu) v = PL(dv, plane)[(size_t)(nx + k - SCP_MAX_NX) * P + g];
            o[k] = v;
        }
    } else {
        for (int k = 0; k < width; ++k) o[k] = PL(dv, plane)[(size_t)k * P + g];
    }
}

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
static inline dim3 grid_for(int n) { return dim3((n + 255) / 256); }

template <class T>
hipError_t launch_plain(PlainOp op, const Dev<T>& dv, const KParams<T>& kp, int models, int kmax, int check,
                        int j, hipStream_t s) {
    const dim3 gn = grid_for(dv.n_nodes), gt = grid_for(dv.n_traj), gg = grid_for(dv.n_groups > 0 ? dv.n_groups : 1);
    const dim3 b(256);
    auto each = [&](auto launch_model) {
        if (models & 1) {
            if (kmax <= 4) launch_model(Quad<4>{});
            else launch_model(Quad<8>{});
        }
        if (models & 2) launch_model(Mars{});
        if (models & 4) {
            if (kmax <= 4) launch_model(Quad6<4>{});
            else launch_model(Quad6<8>{});
        }
        if (models & 8) launch_model(Lander6{});
    };
    switch (op) {
        case PlainOp::Lin:
            each([&](auto m) {
                using MM = decltype(m);
                hipLaunchKernelGGL((k_lin<MM, T>), gn, b, 0, s, dv, kp);
                if constexpr (StepInverse<MM, T>::value) {
                    // Step 1 of these models in FP32 applies the inverse: computed once per SCP iteration
                    const dim3 g4((unsigned)(((size_t)dv.n_nodes * 4 + 255) / 256));
                    hipLaunchKernelGGL((k_minv_lanes4<MM>), g4, b, 0, s, dv);
                }
            });
            break;
        case PlainOp::Step1:
            each([&](auto m) {
                using MM = decltype(m);
                if constexpr (MM::NN == 17) {
                    const dim3 g4((unsigned)(((size_t)dv.n_nodes * 4 + 255) / 256));
                    hipLaunchKernelGGL((k_step1_lanes4<MM, T>), g4, b, 0, s, dv, kp);
                } else {
                    hipLaunchKernelGGL((k_step1<MM, T>), gn, b, 0, s, dv, kp);
                }
            });
            break;
        case PlainOp::Step234:
            each([&](auto m) { hipLaunchKernelGGL((k_step234<decltype(m), T>), gn, b, 0, s, dv, kp, check); });
            if (dv.n_groups > 0)
                each([&](auto m) { hipLaunchKernelGGL((k_group<decltype(m), T>), gg, b, 0, s, dv, kp, check); });
            break;
        case PlainOp::Resid:
            each([&](auto m) { hipLaunchKernelGGL((k_resid<decltype(m), T>), gn, b, 0, s, dv, kp); });
            hipLaunchKernelGGL((k_check<T>), gt, b, 0, s, dv, kp, j, check);
            break;
        case PlainOp::Accept:
            each([&](auto m) { hipLaunchKernelGGL((k_acc_nodes<decltype(m), T>), gn, b, 0, s, dv, kp); });
            hipLaunchKernelGGL((k_acc_traj<T>), dim3(dv.n_traj), dim3(64), 0, s, dv, kp);
            hipLaunchKernelGGL((k_acc_apply<T>), gn, b, 0, s, dv);
            break;
        case PlainOp::Metrics:
            each([&](auto m) { hipLaunchKernelGGL((k_met_nodes<decltype(m), T>), gn, b, 0, s, dv); });
            hipLaunchKernelGGL((k_met_traj<T>), gt, b, 0, s, dv);
            break;
        case PlainOp::Reset:
            hipLaunchKernelGGL((k_reset<T>), gt, b, 0, s, dv, check);
            break;
        case PlainOp::ResetState:
            hipLaunchKernelGGL((k_reset_state<T>), gn, b, 0, s, dv);
            hipLaunchKernelGGL((k_reset<T>), gt, b, 0, s, dv, 1);
            break;
    }
    return hipGetLastError();
}

template <class T>
hipError_t launch_gather(const Dev<T>& dv, int plane, int width, int mode, T* out, hipStream_t s) {
    hipLaunchKernelGGL((k_gather<T>), grid_for(dv.n_nodes), dim3(256), 0, s, dv, plane, width, mode, out);
    return hipGetLastError();
}

template <class T>
hipError_t launch_resident(const Dev<T>& dv, const KParams<T>& kp, int n_traj, int block, int models, int kmax,
                           hipStream_t s) {
    if (n_traj <= 0) return hipSuccess;
    if (block <= 0 || block > 256 || block % 64 != 0 || block > 4 * RESIDENT_MAX_NODES) return hipErrorInvalidValue;
    // 6-DOF models: workgroups of at most 128 lanes (32 nodes) take the 32-row variant, with less
    // LDS per workgroup
    const bool small = block <= 128;
    if (models == 4) {
        if (kmax <= 4) {
            if (small) hipLaunchKernelGGL((k_admm_resident<Quad6<4>, T, 32>), dim3(n_traj), dim3(block), 0, s, dv, kp);
            else hipLaunchKernelGGL((k_admm_resident<Quad6<4>, T, 64>), dim3(n_traj), dim3(block), 0, s, dv, kp);
        } else {
            if (small) hipLaunchKernelGGL((k_admm_resident<Quad6<8>, T, 32>), dim3(n_traj), dim3(block), 0, s, dv, kp);
            else hipLaunchKernelGGL((k_admm_resident<Quad6<8>, T, 64>), dim3(n_traj), dim3(block), 0, s, dv, kp);
        }
    } else if (models == 8) {
        if (small) hipLaunchKernelGGL((k_admm_resident<Lander6, T, 32>), dim3(n_traj), dim3(block), 0, s, dv, kp);
        else hipLaunchKernelGGL((k_admm_resident<Lander6, T, 64>), dim3(n_traj), dim3(block), 0, s, dv, kp);
    } else if (models >= 1 && models <= 3) {
        // point-mass quadrotor and powered descent in lane groups of four: one launch per model
        // present, each workgroup of the other model returns at once
        if (models & 1) {
            if (kmax <= 4) hipLaunchKernelGGL((k_admm_resident<Quad<4>, T, 64>), dim3(n_traj), dim3(block), 0, s, dv, kp);
            else hipLaunchKernelGGL((k_admm_resident<Quad<8>, T, 64>), dim3(n_traj), dim3(block), 0, s, dv, kp);
        }
        if (models & 2) hipLaunchKernelGGL((k_admm_resident<Mars, T, 64>), dim3(n_traj), dim3(block), 0, s, dv, kp);
    } else {
        return hipErrorInvalidValue;   // one 6-DOF model per batch
    }
    return hipGetLastError();
}

template hipError_t launch_plain<float>(PlainOp, const Dev<float>&, const KParams<float>&, int, int, int, int, hipStream_t);
template hipError_t launch_plain<double>(PlainOp, const Dev<double>&, const KParams<double>&, int, int, int, int, hipStream_t);
template hipError_t launch_resident<float>(const Dev<float>&, const KParams<float>&, int, int, int, int, hipStream_t);
template hipError_t launch_resident<double>(const Dev<double>&, const KParams<double>&, int, int, int, int, hipStream_t);
template hipError_t launch_gather<float>(const Dev<float>&, int, int, int, float*, hipStream_t);
template hipError_t launch_gather<double>(const Dev<double>&, int, int, int, double*, hipStream_t);

}  // namespace scp

// Per-node device routines of the SCP + consensus-ADMM hot path (gfx950).
//
// Every routine works on one trajectory node held in registers: the caller (a plain-form kernel
// that streams the node from HBM, or the persistent kernel that keeps it resident) owns the
// storage.  Arrays are sized by compile-time model traits and indexed with compile-time
// constants only (all loops are unrolled), so they live in VGPRs.
//
// Paper references (arXiv 2603.10711):
//   dynamics + RK4            Sec. II eq. (ocp)
//   linearization             Sec. III-A (A_i, B_i Jacobians of the discrete map, d_i residual)
//   convex sets / trust box   Sec. III-A eq. (qp_subproblem), Sec. II prox-friendly sets
//   Step 1 (H_i, Cholesky)    Sec. III-B.3 block formulas of H_i and the unpivoted factorization
//   Step 2 (z average)        Sec. III-B.3 closed-form weighted average
//   Step 3 (projections)      Sec. III-B.3 proximal step / clamp
//   Step 4 (duals)            Sec. III-B.3 dual ascent
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/scp.h"

namespace scp {

// ------------------------------------------------------------------------------------------
// model traits
// ------------------------------------------------------------------------------------------
// Mirror-copy layout (one copy with its own dual per constraint group):
//   quadrotors      [x box: NX][u box: NU][ball: 3][half-space k: 3 each, k < KM]
//   powered descent [x box: NX][u box: NU][glide cone on r: 3][SOC on (T, Gamma): 4]
//   6-DOF lander    [x box: 14][u box: 3][glide cone on (r_E, r_N, r_U): 3][tilt on (q_y, q_z): 2]
//                   [rate ball on w: 3][thrust ball: 3][lower thrust half-space: 3]
//                   [gimbal cone on (T_y, T_z, T_x): 3]
// Both quadrotor models share the first layout (QL: "quadrotor layout"); the 6-DOF model never
// has the ball group (its slots stay inactive).  The first three state components (position)
// never enter the dynamics of any model, so the first three columns of A are the unit vectors
// e_0..e_2 exactly; only the other NXR = NX - 3 columns are stored ("Ar").

template <int KM_>
struct Quad {
    static constexpr int ID = SCP_MODEL_QUAD_PM;
    static constexpr bool QL = true, HSD = true;
    static constexpr int NX = 6, NU = 3, NN = 9, NXR = 3, KM = KM_;
    static constexpr int C_XBOX = 0, C_UBOX = 6, C_BALL = 9, C_HS = 12;
    static constexpr int C = 12 + 3 * KM_;
    static constexpr int NHS = KM_ > 0 ? 4 * KM_ : 1;
};

// 6-DOF quadrotor: x = (p, v, q, w_b), u = (f, tau)
template <int KM_>
struct Quad6 {
    static constexpr int ID = SCP_MODEL_QUAD_6DOF;
    static constexpr bool QL = true, HSD = true;
    static constexpr int NX = 13, NU = 4, NN = 17, NXR = 10, KM = KM_;
    static constexpr int C_XBOX = 0, C_UBOX = 13, C_BALL = 17, C_HS = 20;
    static constexpr int C = 20 + 3 * KM_;
    static constexpr int NHS = KM_ > 0 ? 4 * KM_ : 1;
};

struct Mars {
    static constexpr int ID = SCP_MODEL_MARS3DOF;
    static constexpr bool QL = false, HSD = false;
    static constexpr int NX = 7, NU = 4, NN = 11, NXR = 4, KM = 0;
    static constexpr int C_XBOX = 0, C_UBOX = 7, C_CONE = 11, C_SOC = 14;
    static constexpr int C = 18;
    static constexpr int NHS = 1;
};

// 6-DOF lander: x = (r, v, q, w_b, m), u = T (body frame).  HSD: the node carries half-space
// data (here the linearized lower thrust bound: normal and offset).
struct Lander6 {
    static constexpr int ID = SCP_MODEL_LANDER6;
    static constexpr bool QL = false, HSD = true;
    static constexpr int NX = 14, NU = 3, NN = 17, NXR = 11, KM = 0;
    static constexpr int C_XBOX = 0, C_UBOX = 14, C_GLIDE = 17, C_TILT = 20, C_RATE = 22, C_TBALL = 25,
                         C_THS = 28, C_GIMB = 31;
    static constexpr int C = 34;
    static constexpr int NHS = 4;
};

// run-time dimensions of a model id: state, control, and the mirror slots of its largest
// instantiation (the prefix of each plane block a trajectory of that model uses)
__host__ __device__ constexpr int model_nx(int m) {
    return m == SCP_MODEL_QUAD_PM ? 6 : m == SCP_MODEL_MARS3DOF ? 7 : m == SCP_MODEL_QUAD_6DOF ? 13 : 14;
}
__host__ __device__ constexpr int model_nu(int m) { return m == SCP_MODEL_QUAD_PM || m == SCP_MODEL_LANDER6 ? 3 : 4; }
__host__ __device__ constexpr int model_slots(int m) {
    return m == SCP_MODEL_QUAD_PM ? Quad<SCP_MAX_OBS>::C : m == SCP_MODEL_MARS3DOF ? Mars::C
         : m == SCP_MODEL_QUAD_6DOF ? Quad6<SCP_MAX_OBS>::C : Lander6::C;
}

template <class M>
__host__ __device__ constexpr int NU_OF() { return M::NU; }

template <class M>
struct Dims {
    static constexpr int NX = M::NX, NU = M::NU, NN = M::NN, NXR = M::NXR;
    static constexpr int NL = NN * (NN + 1) / 2;
};

__host__ __device__ constexpr int tri(int r, int c) { return r * (r + 1) / 2 + c; }

template <class T>
struct Rho {
    T eq, dyn, geo, inv_geo, inv_sum;
};

// Adaptive penalty by residual balancing between SCP iterations (Boyd et al. 2011, Sec. 3.4.1;
// the paper gives no adaptive rule): the factor after an SCP iteration whose last ADMM iteration
// left residuals rp, rd, compared in double.  NaN residuals keep the factor.
__host__ __device__ inline double adapt_factor(double f, double rp, double rd, double mu, double tau) {
    if (rp > mu * rd) return f * tau;
    if (rd > mu * rp) return f / tau;
    return f;
}

// ------------------------------------------------------------------------------------------
// scalar helpers (NaN-propagating max; the comparisons keep a NaN once it appears)
// ------------------------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T nmax(T a, T b) { return (b > a || b != b) ? b : a; }
template <class T>
__device__ __forceinline__ T tabs(T a) { return a < T(0) ? -a : a; }
__device__ __forceinline__ float tsqrt(float a) { return sqrtf(a); }
__device__ __forceinline__ double tsqrt(double a) { return sqrt(a); }
// min / max / clamp map to single VALU instructions (v_min, v_max, v_med3)
__device__ __forceinline__ float tmin(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double tmin(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ float tmaxv(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ double tmaxv(double a, double b) { return __builtin_fmax(a, b); }
// fused multiply-add written out, where the rounding of a sum must not depend on which product
// the compiler chooses to contract (it can differ between kernel instantiations)
__device__ __forceinline__ float tfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double tfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
// 1/sqrt(a): one hardware reciprocal square root in FP32 (about 1 ulp), exact division in FP64
__device__ __forceinline__ float trsqrt(float a) { return __builtin_amdgcn_rsqf(a); }
__device__ __forceinline__ double trsqrt(double a) { return 1.0 / sqrt(a); }

// ------------------------------------------------------------------------------------------
// wavefront neighbour exchange (DPP wave shifts, no LDS): lane t receives the value of lane
// t+1 (lane_next) or t-1 (lane_prev); the lane without a neighbour receives 0.  Called with
// the whole wavefront active.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ int dpp_next_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xF, 0xF, true); }
__device__ __forceinline__ int dpp_prev_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xF, 0xF, true); }
__device__ __forceinline__ float lane_next(float v) { return __builtin_bit_cast(float, dpp_next_i(__builtin_bit_cast(int, v))); }
__device__ __forceinline__ float lane_prev(float v) { return __builtin_bit_cast(float, dpp_prev_i(__builtin_bit_cast(int, v))); }
__device__ __forceinline__ double lane_next(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = dpp_next_i((int)(b & 0xffffffffll)), hi = dpp_next_i((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double lane_prev(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = dpp_prev_i((int)(b & 0xffffffffll)), hi = dpp_prev_i((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// Lane permutations inside each aligned group of four lanes (DPP quad_perm; SEL packs the source
// lane of lanes 0..3 in two bits each).  Every lane of a group must be active, so a source lane is
// never out of range and the zero-fill flag changes no result; with it set the compiler folds the
// permutation into a following two-operand addition, multiplication or min/max (v_add_f32_dpp ...),
// one instruction instead of two (quad_sum, quad_reduce_scatter).
template <int SEL>
__device__ __forceinline__ int quad_perm_i(int v) { return __builtin_amdgcn_mov_dpp(v, SEL, 0xF, 0xF, true); }
template <int SEL>
__device__ __forceinline__ float quad_perm(float v) { return __builtin_bit_cast(float, quad_perm_i<SEL>(__builtin_bit_cast(int, v))); }
template <int SEL>
__device__ __forceinline__ double quad_perm(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = quad_perm_i<SEL>((int)(b & 0xffffffffll)), hi = quad_perm_i<SEL>((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
// a value the same in every active lane of the wavefront, moved to scalar registers (it then
// takes no vector register, as a kernel argument would not)
__device__ __forceinline__ float wave_uniform(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double wave_uniform(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll)), hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
// the value of lane k of this lane's group (k a constant after unrolling)
template <class T>
__device__ __forceinline__ T quad_bcast(T v, int k) {
    switch (k & 3) {
        case 0: return quad_perm<0x00>(v);
        case 1: return quad_perm<0x55>(v);
        case 2: return quad_perm<0xAA>(v);
        default: return quad_perm<0xFF>(v);
    }
}
// the value of lane l xor c of this lane's group (c a constant after unrolling)
template <class T>
__device__ __forceinline__ T quad_xor(T v, int c) {
    switch (c & 3) {
        case 0: return v;
        case 1: return quad_perm<0xB1>(v);
        case 2: return quad_perm<0x4E>(v);
        default: return quad_perm<0x1B>(v);
    }
}
// Sums over the group of four rows at once: lane l holds its term of row l xor c in v[c], and
// receives the sum of row l as (v_l + v_{l^1}) + (v_{l^2} + v_{l^3}) (subscripts: lanes), the
// bits quad_sum gives that row in every lane.
template <class T>
__device__ __forceinline__ T quad_reduce_scatter(const T* v) {
    const T a = v[0] + quad_perm<0xB1>(v[1]);   // row l: own term + lane l^1's
    const T b = v[2] + quad_perm<0xB1>(v[3]);   // row l^2: own term + lane l^1's
    return a + quad_perm<0x4E>(b);              // + lane l^2's pair sum of row l
}
// sum over the group as (v0 + v1) + (v2 + v3); addition commutes exactly, so every lane of the
// group gets the same bits
template <class T>
__device__ __forceinline__ T quad_sum(T v) {
    const T a = v + quad_perm<0xB1>(v);   // lanes (1, 0, 3, 2)
    return a + quad_perm<0x4E>(a);         // lanes (2, 3, 0, 1)
}

// ------------------------------------------------------------------------------------------
// continuous dynamics and their directional derivative (JVP)
// ------------------------------------------------------------------------------------------
// prm points at the trajectory's parameter record (SCP_P_* offsets) in the problem precision.

template <class M, class T>
__device__ __forceinline__ void f_cont(const T* __restrict__ prm, const T* x, const T* u, T* f) {
    if constexpr (M::ID == SCP_MODEL_QUAD_PM) {
        // p' = v, v' = u/m_s - g e3 - c ||v|| v + d  (d: constant disturbance acceleration)
        const T c = prm[SCP_P_DRAG], ms = prm[SCP_P_MSCALE], g = prm[SCP_P_GRAV];
        const T* dist = prm + SCP_P_DIST;
        const T nv = tsqrt(x[3] * x[3] + x[4] * x[4] + x[5] * x[5]);
        f[0] = x[3]; f[1] = x[4]; f[2] = x[5];
        f[3] = (u[0] / ms - c * nv * x[3]) + dist[0];
        f[4] = (u[1] / ms - c * nv * x[4]) + dist[1];
        f[5] = ((u[2] / ms - g) - c * nv * x[5]) + dist[2];
    } else if constexpr (M::ID == SCP_MODEL_QUAD_6DOF) {
        // p' = v, v' = (f/m) R(q/|q|) e3 - g e3 + d, q' = q (x) (0, w) / 2, J w' = tau - w x (J w)
        const T m = prm[SCP_P_MSCALE], g = prm[SCP_P_GRAV];
        const T* J = prm + SCP_P_INERTIA;
        const T* dist = prm + SCP_P_DIST;
        const T qw = x[6], qx = x[7], qy = x[8], qz = x[9];
        const T wx = x[10], wy = x[11], wz = x[12];
        const T a = u[0] / m;
        // third column of the rotation matrix of q / |q|
        const T in2 = T(1) / ((qw * qw + qx * qx) + (qy * qy + qz * qz));
        const T c0 = T(2) * (qx * qz + qw * qy) * in2;
        const T c1 = T(2) * (qy * qz - qw * qx) * in2;
        const T c2 = ((qw * qw - qx * qx) + (qz * qz - qy * qy)) * in2;
        f[0] = x[3]; f[1] = x[4]; f[2] = x[5];
        f[3] = a * c0 + dist[0];
        f[4] = a * c1 + dist[1];
        f[5] = (a * c2 - g) + dist[2];
        f[6] = T(-0.5) * ((qx * wx + qy * wy) + qz * wz);
        f[7] = T(0.5) * ((qw * wx + qy * wz) - qz * wy);
        f[8] = T(0.5) * ((qw * wy + qz * wx) - qx * wz);
        f[9] = T(0.5) * ((qw * wz + qx * wy) - qy * wx);
        f[10] = (u[1] - (J[2] - J[1]) * (wy * wz)) / J[0];
        f[11] = (u[2] - (J[0] - J[2]) * (wz * wx)) / J[1];
        f[12] = (u[3] - (J[1] - J[0]) * (wx * wy)) / J[2];
    } else if constexpr (M::ID == SCP_MODEL_LANDER6) {
        // r' = v, v' = R(q/|q|) T / m + g, q' = q (x) (0, w) / 2, J w' = r_T x T - w x (J w),
        // m' = -alpha |T|
        const T* J = prm + SCP_P_INERTIA;
        const T* ra = prm + SCP_P_ARM;
        const T* gv = prm + SCP_P_GVEC;
        const T qw = x[6], qx = x[7], qy = x[8], qz = x[9];
        const T wx = x[10], wy = x[11], wz = x[12], m = x[13];
        const T T0 = u[0], T1 = u[1], T2 = u[2];
        const T in2 = T(1) / ((qw * qw + qx * qx) + (qy * qy + qz * qz));
        // R_hom(q) T, the rotation written as a homogeneous quadratic in q
        const T p0 = ((qw * qw + qx * qx) - (qy * qy + qz * qz)) * T0 + T(2) * ((qx * qy - qw * qz) * T1 + (qx * qz + qw * qy) * T2);
        const T p1 = ((qw * qw - qx * qx) + (qy * qy - qz * qz)) * T1 + T(2) * ((qx * qy + qw * qz) * T0 + (qy * qz - qw * qx) * T2);
        const T p2 = ((qw * qw - qx * qx) - (qy * qy - qz * qz)) * T2 + T(2) * ((qx * qz - qw * qy) * T0 + (qy * qz + qw * qx) * T1);
        const T sc = in2 / m;
        f[0] = x[3]; f[1] = x[4]; f[2] = x[5];
        f[3] = p0 * sc + gv[0];
        f[4] = p1 * sc + gv[1];
        f[5] = p2 * sc + gv[2];
        f[6] = T(-0.5) * ((qx * wx + qy * wy) + qz * wz);
        f[7] = T(0.5) * ((qw * wx + qy * wz) - qz * wy);
        f[8] = T(0.5) * ((qw * wy + qz * wx) - qx * wz);
        f[9] = T(0.5) * ((qw * wz + qx * wy) - qy * wx);
        f[10] = ((ra[1] * T2 - ra[2] * T1) - (J[2] - J[1]) * (wy * wz)) / J[0];
        f[11] = ((ra[2] * T0 - ra[0] * T2) - (J[0] - J[2]) * (wz * wx)) / J[1];
        f[12] = ((ra[0] * T1 - ra[1] * T0) - (J[1] - J[0]) * (wx * wy)) / J[2];
        f[13] = -prm[SCP_P_ALPHA] * tsqrt((T0 * T0 + T1 * T1) + T2 * T2);
    } else {
        // r' = v, v' = T/m + g_vec, m' = -alpha Gamma
        const T m = x[6];
        f[0] = x[3]; f[1] = x[4]; f[2] = x[5];
        f[3] = u[0] / m + prm[SCP_P_GVEC + 0];
        f[4] = u[1] / m + prm[SCP_P_GVEC + 1];
        f[5] = u[2] / m + prm[SCP_P_GVEC + 2];
        f[6] = -prm[SCP_P_ALPHA] * u[3];
    }
}

// df = (df/dx) dx + (df/du) du at (x, u)
template <class M, class T>
__device__ __forceinline__ void f_jvp(const T* __restrict__ prm, const T* x, const T* u, const T* dx,
                                      const T* du, T* df) {
    if constexpr (M::ID == SCP_MODEL_QUAD_PM) {
        // d(c||v||v) = c (||v|| dv + v (v.dv)/||v||), zero at v = 0
        const T c = prm[SCP_P_DRAG], ms = prm[SCP_P_MSCALE];
        const T nv = tsqrt(x[3] * x[3] + x[4] * x[4] + x[5] * x[5]);
        const T vdv = x[3] * dx[3] + x[4] * dx[4] + x[5] * dx[5];
        const T q = nv > T(0) ? vdv / nv : T(0);
        df[0] = dx[3]; df[1] = dx[4]; df[2] = dx[5];
#pragma unroll
        for (int k = 0; k < 3; ++k) df[3 + k] = du[k] / ms - c * (nv * dx[3 + k] + x[3 + k] * q);
    } else if constexpr (M::ID == SCP_MODEL_QUAD_6DOF) {
        // product rule through every bilinear term of f_cont
        const T m = prm[SCP_P_MSCALE];
        const T* J = prm + SCP_P_INERTIA;
        const T qw = x[6], qx = x[7], qy = x[8], qz = x[9];
        const T wx = x[10], wy = x[11], wz = x[12];
        const T dqw = dx[6], dqx = dx[7], dqy = dx[8], dqz = dx[9];
        const T dwx = dx[10], dwy = dx[11], dwz = dx[12];
        const T a = u[0] / m, da = du[0] / m;
        // c = n(q) / |q|^2 with the quadratic numerator n: dc = (dn - c d|q|^2) / |q|^2
        const T in2 = T(1) / ((qw * qw + qx * qx) + (qy * qy + qz * qz));
        const T dn2 = T(2) * ((qw * dqw + qx * dqx) + (qy * dqy + qz * dqz));
        const T c0 = T(2) * (qx * qz + qw * qy) * in2;
        const T c1 = T(2) * (qy * qz - qw * qx) * in2;
        const T c2 = ((qw * qw - qx * qx) + (qz * qz - qy * qy)) * in2;
        const T dc0 = (T(2) * ((dqx * qz + qx * dqz) + (dqw * qy + qw * dqy)) - c0 * dn2) * in2;
        const T dc1 = (T(2) * ((dqy * qz + qy * dqz) - (dqw * qx + qw * dqx)) - c1 * dn2) * in2;
        const T dc2 = (T(2) * ((qw * dqw - qx * dqx) + (qz * dqz - qy * dqy)) - c2 * dn2) * in2;
        df[0] = dx[3]; df[1] = dx[4]; df[2] = dx[5];
        df[3] = da * c0 + a * dc0;
        df[4] = da * c1 + a * dc1;
        df[5] = da * c2 + a * dc2;
        df[6] = T(-0.5) * (((dqx * wx + dqy * wy) + dqz * wz) + ((qx * dwx + qy * dwy) + qz * dwz));
        df[7] = T(0.5) * (((dqw * wx + dqy * wz) - dqz * wy) + ((qw * dwx + qy * dwz) - qz * dwy));
        df[8] = T(0.5) * (((dqw * wy + dqz * wx) - dqx * wz) + ((qw * dwy + qz * dwx) - qx * dwz));
        df[9] = T(0.5) * (((dqw * wz + dqx * wy) - dqy * wx) + ((qw * dwz + qx * dwy) - qy * dwx));
        df[10] = (du[1] - (J[2] - J[1]) * (dwy * wz + wy * dwz)) / J[0];
        df[11] = (du[2] - (J[0] - J[2]) * (dwz * wx + wz * dwx)) / J[1];
        df[12] = (du[3] - (J[1] - J[0]) * (dwx * wy + wx * dwy)) / J[2];
    } else if constexpr (M::ID == SCP_MODEL_LANDER6) {
        const T* J = prm + SCP_P_INERTIA;
        const T* ra = prm + SCP_P_ARM;
        const T qw = x[6], qx = x[7], qy = x[8], qz = x[9];
        const T wx = x[10], wy = x[11], wz = x[12], m = x[13];
        const T dqw = dx[6], dqx = dx[7], dqy = dx[8], dqz = dx[9];
        const T dwx = dx[10], dwy = dx[11], dwz = dx[12], dm = dx[13];
        const T T0 = u[0], T1 = u[1], T2 = u[2], dT0 = du[0], dT1 = du[1], dT2 = du[2];
        const T in2 = T(1) / ((qw * qw + qx * qx) + (qy * qy + qz * qz));
        const T p0 = ((qw * qw + qx * qx) - (qy * qy + qz * qz)) * T0 + T(2) * ((qx * qy - qw * qz) * T1 + (qx * qz + qw * qy) * T2);
        const T p1 = ((qw * qw - qx * qx) + (qy * qy - qz * qz)) * T1 + T(2) * ((qx * qy + qw * qz) * T0 + (qy * qz - qw * qx) * T2);
        const T p2 = ((qw * qw - qx * qx) - (qy * qy - qz * qz)) * T2 + T(2) * ((qx * qz - qw * qy) * T0 + (qy * qz + qw * qx) * T1);
        // dp = R_hom(q) dT + (dR_hom/dq . dq) T
        const T r0 = ((qw * qw + qx * qx) - (qy * qy + qz * qz)) * dT0 + T(2) * ((qx * qy - qw * qz) * dT1 + (qx * qz + qw * qy) * dT2);
        const T r1 = ((qw * qw - qx * qx) + (qy * qy - qz * qz)) * dT1 + T(2) * ((qx * qy + qw * qz) * dT0 + (qy * qz - qw * qx) * dT2);
        const T r2 = ((qw * qw - qx * qx) - (qy * qy - qz * qz)) * dT2 + T(2) * ((qx * qz - qw * qy) * dT0 + (qy * qz + qw * qx) * dT1);
        const T e0 = T(2) * (((qw * T0 - qz * T1) + qy * T2) * dqw + ((qx * T0 + qy * T1) + qz * T2) * dqx +
                             ((qx * T1 - qy * T0) + qw * T2) * dqy + ((qx * T2 - qz * T0) - qw * T1) * dqz);
        const T e1 = T(2) * (((qz * T0 + qw * T1) - qx * T2) * dqw + ((qy * T0 - qx * T1) - qw * T2) * dqx +
                             ((qx * T0 + qy * T1) + qz * T2) * dqy + ((qw * T0 - qz * T1) + qy * T2) * dqz);
        const T e2 = T(2) * (((qx * T1 - qy * T0) + qw * T2) * dqw + ((qz * T0 + qw * T1) - qx * T2) * dqx +
                             ((qz * T1 - qw * T0) - qy * T2) * dqy + ((qx * T0 + qy * T1) + qz * T2) * dqz);
        // d(p / (|q|^2 m)) = (dp - p (d|q|^2 / |q|^2 + dm / m)) / (|q|^2 m)
        const T k = T(2) * ((qw * dqw + qx * dqx) + (qy * dqy + qz * dqz)) * in2 + dm / m;
        const T sc = in2 / m;
        df[0] = dx[3]; df[1] = dx[4]; df[2] = dx[5];
        df[3] = ((r0 + e0) - p0 * k) * sc;
        df[4] = ((r1 + e1) - p1 * k) * sc;
        df[5] = ((r2 + e2) - p2 * k) * sc;
        df[6] = T(-0.5) * (((dqx * wx + dqy * wy) + dqz * wz) + ((qx * dwx + qy * dwy) + qz * dwz));
        df[7] = T(0.5) * (((dqw * wx + dqy * wz) - dqz * wy) + ((qw * dwx + qy * dwz) - qz * dwy));
        df[8] = T(0.5) * (((dqw * wy + dqz * wx) - dqx * wz) + ((qw * dwy + qz * dwx) - qx * dwz));
        df[9] = T(0.5) * (((dqw * wz + dqx * wy) - dqy * wx) + ((qw * dwz + qx * dwy) - qy * dwx));
        df[10] = ((ra[1] * dT2 - ra[2] * dT1) - (J[2] - J[1]) * (dwy * wz + wy * dwz)) / J[0];
        df[11] = ((ra[2] * dT0 - ra[0] * dT2) - (J[0] - J[2]) * (dwz * wx + wz * dwx)) / J[1];
        df[12] = ((ra[0] * dT1 - ra[1] * dT0) - (J[1] - J[0]) * (dwx * wy + wx * dwy)) / J[2];
        const T nt = tsqrt((T0 * T0 + T1 * T1) + T2 * T2);
        df[13] = nt > T(0) ? -prm[SCP_P_ALPHA] * ((T0 * dT0 + T1 * dT1) + T2 * dT2) / nt : T(0);
    } else {
        const T m = x[6];
        const T dm = dx[6];
        df[0] = dx[3]; df[1] = dx[4]; df[2] = dx[5];
#pragma unroll
        for (int k = 0; k < 3; ++k) df[3 + k] = du[k] / m - u[k] / (m * m) * dm;
        df[6] = -prm[SCP_P_ALPHA] * du[3];
    }
}

// RK4 step F(x, u) with zero-order-hold control.
template <class M, class T>
__device__ __forceinline__ void rk4(const T* __restrict__ prm, const T* x, const T* u, T* F) {
    constexpr int NX = M::NX;
    const T h = prm[SCP_P_H];
    T k1[NX], k2[NX], k3[NX], k4[NX], xs[NX];
    f_cont<M, T>(prm, x, u, k1);
#pragma unroll
    for (int r = 0; r < NX; ++r) xs[r] = x[r] + T(0.5) * h * k1[r];
    f_cont<M, T>(prm, xs, u, k2);
#pragma unroll
    for (int r = 0; r < NX; ++r) xs[r] = x[r] + T(0.5) * h * k2[r];
    f_cont<M, T>(prm, xs, u, k3);
#pragma unroll
    for (int r = 0; r < NX; ++r) xs[r] = x[r] + h * k3[r];
    f_cont<M, T>(prm, xs, u, k4);
    const T h6 = h / T(6);
#pragma unroll
    for (int r = 0; r < NX; ++r) F[r] = x[r] + h6 * (((k1[r] + T(2) * k2[r]) + T(2) * k3[r]) + k4[r]);
}

// Linearization of the RK4 map at (x, u): F, the non-unit columns Ar of A = dF/dx (columns
// 3..NX-1), B = dF/du and d = F - A x - B u.  Forward-mode chain rule through the stages: for
// every input direction e, s_j = J(x_j) (e + c_j s_{j-1}) with stage points x_j and
// c = (0, h/2, h/2, h); the column is e + h/6 (s_1 + 2 s_2 + 2 s_3 + s_4).
template <class M, class T>
__device__ __forceinline__ void linearize(const T* __restrict__ prm, const T* x, const T* u, T* F,
                                          T* Ar, T* B, T* d) {
    constexpr int NX = M::NX, NU = M::NU, NXR = M::NXR;
    const T h = prm[SCP_P_H];
    T xs[4][NX], k[4][NX];
#pragma unroll
    for (int r = 0; r < NX; ++r) xs[0][r] = x[r];
    f_cont<M, T>(prm, xs[0], u, k[0]);
#pragma unroll
    for (int r = 0; r < NX; ++r) xs[1][r] = x[r] + T(0.5) * h * k[0][r];
    f_cont<M, T>(prm, xs[1], u, k[1]);
#pragma unroll
    for (int r = 0; r < NX; ++r) xs[2][r] = x[r] + T(0.5) * h * k[1][r];
    f_cont<M, T>(prm, xs[2], u, k[2]);
#pragma unroll
    for (int r = 0; r < NX; ++r) xs[3][r] = x[r] + h * k[2][r];
    f_cont<M, T>(prm, xs[3], u, k[3]);
    const T h6 = h / T(6);
#pragma unroll
    for (int r = 0; r < NX; ++r) F[r] = x[r] + h6 * (((k[0][r] + T(2) * k[1][r]) + T(2) * k[2][r]) + k[3][r]);

#pragma unroll
    for (int col = 3; col < NX + NU; ++col) {
        T e[NX], eu[NU], s[4][NX], dx[NX];
#pragma unroll
        for (int r = 0; r < NX; ++r) e[r] = (r == col) ? T(1) : T(0);
#pragma unroll
        for (int r = 0; r < NU; ++r) eu[r] = (NX + r == col) ? T(1) : T(0);
        f_jvp<M, T>(prm, xs[0], u, e, eu, s[0]);
#pragma unroll
        for (int r = 0; r < NX; ++r) dx[r] = e[r] + T(0.5) * h * s[0][r];
        f_jvp<M, T>(prm, xs[1], u, dx, eu, s[1]);
#pragma unroll
        for (int r = 0; r < NX; ++r) dx[r] = e[r] + T(0.5) * h * s[1][r];
        f_jvp<M, T>(prm, xs[2], u, dx, eu, s[2]);
#pragma unroll
        for (int r = 0; r < NX; ++r) dx[r] = e[r] + h * s[2][r];
        f_jvp<M, T>(prm, xs[3], u, dx, eu, s[3]);
#pragma unroll
        for (int r = 0; r < NX; ++r) {
            const T v = e[r] + h6 * (((s[0][r] + T(2) * s[1][r]) + T(2) * s[2][r]) + s[3][r]);
            if (col < NX) Ar[r * NXR + (col - 3)] = v;
            else B[r * NU + (col - NX)] = v;
        }
    }
    // d = F - A x - B u  (A x includes the unit columns)
#pragma unroll
    for (int r = 0; r < NX; ++r) {
        T ax = (r < 3) ? x[r] : T(0);
#pragma unroll
        for (int c = 0; c < NXR; ++c) ax = ax + Ar[r * NXR + c] * x[3 + c];
        T bu = T(0);
#pragma unroll
        for (int c = 0; c < NU; ++c) bu = bu + B[r * NU + c] * u[c];
        d[r] = (F[r] - ax) - bu;
    }
}

// y = A x  (A = [e_0 e_1 e_2 | Ar])
template <class M, class T>
__device__ __forceinline__ void a_mul(const T* Ar, const T* x, T* y) {
    constexpr int NX = M::NX, NXR = M::NXR;
#pragma unroll
    for (int r = 0; r < NX; ++r) {
        T s = (r < 3) ? x[r] : T(0);
#pragma unroll
        for (int c = 0; c < NXR; ++c) s = s + Ar[r * NXR + c] * x[3 + c];
        y[r] = s;
    }
}

// y = A^T w
template <class M, class T>
__device__ __forceinline__ void at_mul(const T* Ar, const T* w, T* y) {
    constexpr int NX = M::NX, NXR = M::NXR;
#pragma unroll
    for (int k = 0; k < 3; ++k) y[k] = w[k];
#pragma unroll
    for (int c = 0; c < NXR; ++c) {
        T s = T(0);
#pragma unroll
        for (int r = 0; r < NX; ++r) s = s + Ar[r * NXR + c] * w[r];
        y[3 + c] = s;
    }
}

// y = B^T w
template <class M, class T>
__device__ __forceinline__ void bt_mul(const T* B, const T* w, T* y) {
    constexpr int NX = M::NX, NU = M::NU;
#pragma unroll
    for (int c = 0; c < NU; ++c) {
        T s = T(0);
#pragma unroll
        for (int r = 0; r < NX; ++r) s = s + B[r * NU + c] * w[r];
        y[c] = s;
    }
}

// ------------------------------------------------------------------------------------------
// projections (exact closed forms)
// ------------------------------------------------------------------------------------------
// box clamp; lo <= hi holds for every convexified box (an empty cut collapses to a point)
__device__ __forceinline__ float clampv(float v, float lo, float hi) { return __builtin_amdgcn_fmed3f(v, lo, hi); }
__device__ __forceinline__ double clampv(double v, double lo, double hi) { return tmin(tmaxv(v, lo), hi); }

// {y : a'y >= b} with a unit normal a (the obstacle normals are normalized when the sets are
// built), so the projection v + max(0, b - a'v)/||a||^2 a needs no division.
template <class T>
__device__ __forceinline__ void proj_halfspace(const T* a, T b, T* v) {
    const T av = (a[0] * v[0] + a[1] * v[1]) + a[2] * v[2];
    const T t = tmaxv(T(0), b - av);
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = v[k] + t * a[k];
}

// {y : ||y|| <= r}, 3-vector: v min(1, r/||v||)
template <class T>
__device__ __forceinline__ void proj_ball3(T r, T* v) {
    const T vv = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2];
    const T s = vv > r * r ? r * trsqrt(vv) : T(1);
#pragma unroll
    for (int k = 0; k < 3; ++k) v[k] = v[k] * s;
}

// {y : ||y|| <= r}, 2-vector
template <class T>
__device__ __forceinline__ void proj_ball2(T r, T* v) {
    const T vv = v[0] * v[0] + v[1] * v[1];
    const T s = vv > r * r ? r * trsqrt(vv) : T(1);
    v[0] = v[0] * s;
    v[1] = v[1] * s;
}

// {(y, s) : ||y|| <= kappa s}, y of length M-1; inv1k2 = 1/(1 + kappa^2)
template <int M, class T>
__device__ __forceinline__ void proj_cone(T kappa, T inv1k2, T* v) {
    T yy = T(0);
#pragma unroll
    for (int k = 0; k < M - 1; ++k) yy = yy + v[k] * v[k];
    const T rny = trsqrt(yy);          // 1/||y|| (inf at y = 0; then the point is inside or polar)
    const T ny = yy * rny;
    const T s = v[M - 1];
    const bool inside = (yy == T(0)) ? (s >= T(0)) : (ny <= kappa * s);
    const bool polar = !inside && (yy == T(0) || kappa * ny <= -s);
    const T c = (kappa * ny + s) * inv1k2;
    const T f = polar ? T(0) : (inside ? T(1) : c * kappa * rny);
#pragma unroll
    for (int k = 0; k < M - 1; ++k) v[k] = f * v[k];
    v[M - 1] = polar ? T(0) : (inside ? s : c);
}

// ------------------------------------------------------------------------------------------
// node data
// ------------------------------------------------------------------------------------------
// Per-SCP-iteration constants of one node.
template <class M, class T>
struct NodeConst {
    static constexpr int NX = M::NX, NU = M::NU, NN = M::NN, NXR = M::NXR, NL = Dims<M>::NL;
    T L[NL];        // packed lower Cholesky factor of H_i, diagonal slots hold 1/L_kk
    T Ar[NX * NXR]; // non-unit columns of A_i (zero at node N)
    T B[NX * NU];   // B_i (zero at node N)
    T d[NX];        // d_i (zero at node N)
    T lo[NN], hi[NN];   // box group bounds: x components then u components
    T hs[M::NHS];   // quadrotor half-spaces: (a_x, a_y, a_z, b) per obstacle
    T g0[NX];       // constant part of the Step-1 right-hand side: -q_i (x part)
};

// ADMM iterates of one node.
template <class M, class T>
struct NodeState {
    static constexpr int NX = M::NX, NU = M::NU, C = M::C;
    T x[NX], u[NU];
    T z[NX], lam[NX], mu[NX];
    T dd[NX];       // d_dyn,i = A_i x_i + B_i u_i + d_i
    T cp[C], du[C]; // mirror copies and their duals (zero where the group is absent)
};

// Node identity inside its trajectory.
struct NodeId {
    int i, N, K;    // node index, horizon, obstacle count
    bool ball;      // quadrotor ball group present
    __device__ bool first() const { return i == 0; }
    __device__ bool last() const { return i == N; }
};

// Group activity at a node: x box everywhere; u groups at i < N; half-spaces and the glide
// cone at i >= 1.
template <class M>
__device__ __forceinline__ bool group_active(const NodeId& id, int g) {
    if constexpr (M::QL) {
        if (g == 0) return true;                         // x box
        if (g == 1) return !id.last();                   // u box
        if (g == 2) return !id.last() && id.ball;        // ball
        return !id.first() && (g - 3) < id.K;            // half-space g-3
    } else if constexpr (M::ID == SCP_MODEL_LANDER6) {
        if (g == 0) return true;                         // x box
        if (g == 1) return !id.last();                   // u box
        if (g <= 4) return !id.first();                  // glide cone, tilt, rate ball
        return !id.last();                               // thrust ball, lower bound, gimbal
    } else {
        if (g == 0) return true;
        if (g == 1) return !id.last();
        if (g == 2) return !id.first();                  // glide cone
        return !id.last();                               // SOC
    }
}

// Penalty of group g at this node: rho_geo where the group exists, 0 where it does not.  With it
// a group absent at a node keeps a zero dual and adds nothing to Step 1 without per-component
// masks; its copy there is a finite dummy that is reported (and stored) as 0.
template <class M, class T>
__device__ __forceinline__ T group_rho(const NodeId& id, T rho_geo, int g) {
    return group_active<M>(id, g) ? rho_geo : T(0);
}

// ------------------------------------------------------------------------------------------
// a3: convexified sets
// ------------------------------------------------------------------------------------------
// Trust box [c - delta, c + delta] cut by the hard box [lh, hh]; an empty cut collapses onto
// the hard-box point nearest the centre.  Returns true if the hard box itself is empty.
template <class T>
__device__ __forceinline__ bool trust_box(T c, T delta, T lh, T hh, T& lo, T& hi) {
    T l = tmaxv(c - delta, lh);
    T u = tmin(c + delta, hh);
    if (l > u) {
        const T p = tmin(tmaxv(c, lh), hh);
        l = p;
        u = p;
    }
    lo = l;
    hi = u;
    return lh > hh;
}

// Box bounds, half-spaces and g0 of one node.  ucenter: centre of the control trust box
// (the nominal control, or the scenario mean at node 0 of a consensus group).
template <class M, class T>
__device__ __forceinline__ int convexify(const T* __restrict__ prm, const NodeId& id, const T* xbar,
                                         const T* ucenter, T delta, NodeConst<M, T>& nc) {
    constexpr int NX = M::NX, NU = M::NU;
    int st = 0;
#pragma unroll
    for (int r = 0; r < NX; ++r) {
        T lo, hi;
        if (trust_box(xbar[r], delta, prm[SCP_P_XLO + r], prm[SCP_P_XHI + r], lo, hi)) st |= SCP_ST_EMPTYSET;
        if (id.first()) {
            lo = prm[SCP_P_XINIT + r];
            hi = lo;
        }
        if (id.last() && prm[SCP_P_TMASK + r] != T(0)) {
            lo = prm[SCP_P_XTGT + r];
            hi = lo;
        }
        if (!(lo <= hi)) st |= SCP_ST_NONFINITE;   // a NaN bound: non-finite nominal or boundary value
        nc.lo[r] = lo;
        nc.hi[r] = hi;
        nc.g0[r] = id.last() ? -prm[SCP_P_QNV + r] : T(0);
    }
#pragma unroll
    for (int r = 0; r < NU; ++r) {
        T lo, hi;
        if (trust_box(ucenter[r], delta, prm[SCP_P_ULO + r], prm[SCP_P_UHI + r], lo, hi)) st |= SCP_ST_EMPTYSET;
        if (!(lo <= hi)) st |= SCP_ST_NONFINITE;
        nc.lo[NX + r] = id.last() ? T(0) : lo;
        nc.hi[NX + r] = id.last() ? T(0) : hi;
    }
    if constexpr (M::QL) {
        const int cyl = (int)prm[SCP_P_CYL];
#pragma unroll
        for (int j = 0; j < M::KM; ++j) {
            T a0 = T(0), a1 = T(0), a2 = T(0), b = T(0);
            if (j < id.K && !id.first()) {
                // sphere: normal along xbar - c; vertical cylinder: its horizontal part
                const bool cj = (cyl >> j) & 1;
                const T* o = prm + SCP_P_OBS + 4 * j;
                const T d0 = xbar[0] - o[0], d1 = xbar[1] - o[1], d2 = cj ? T(0) : xbar[2] - o[2];
                const T nd = tsqrt((d0 * d0 + d1 * d1) + d2 * d2);
                if (nd >= T(1e-9)) {
                    a0 = d0 / nd; a1 = d1 / nd; a2 = d2 / nd;
                } else if (cj) {
                    a0 = T(1);
                } else {
                    a2 = T(1);
                }
                b = o[3] + ((a0 * o[0] + a1 * o[1]) + a2 * o[2]);
            }
            nc.hs[4 * j + 0] = a0;
            nc.hs[4 * j + 1] = a1;
            nc.hs[4 * j + 2] = a2;
            nc.hs[4 * j + 3] = b;
        }
    } else if constexpr (M::ID == SCP_MODEL_LANDER6) {
        // lower thrust bound |T| >= T_min linearized at the nominal thrust: n'T >= T_min with
        // n = Tbar / |Tbar| (+e1 if |Tbar| < 1e-9)
        const T t0 = ucenter[0], t1 = ucenter[1], t2 = ucenter[2];
        const T nt = tsqrt((t0 * t0 + t1 * t1) + t2 * t2);
        const bool ok = nt >= T(1e-9);
        nc.hs[0] = ok ? t0 / nt : T(1);
        nc.hs[1] = ok ? t1 / nt : T(0);
        nc.hs[2] = ok ? t2 / nt : T(0);
        nc.hs[3] = prm[SCP_P_TMIN];
    }
    return st;
}

// number of groups covering each component (D_x, D_u of the Step-1 Hessian)
template <class M, class T>
__device__ __forceinline__ void group_counts(const NodeId& id, T* Dx, T* Du) {
    constexpr int NX = M::NX, NU = M::NU;
#pragma unroll
    for (int r = 0; r < NX; ++r) Dx[r] = T(1);
#pragma unroll
    for (int r = 0; r < NU; ++r) Du[r] = T(1);
    if constexpr (M::QL) {
        if (!id.first()) {
#pragma unroll
            for (int r = 0; r < 3; ++r) Dx[r] = Dx[r] + T(id.K);
        }
        if (id.ball) {
#pragma unroll
            for (int r = 0; r < 3; ++r) Du[r] = Du[r] + T(1);
        }
    } else if constexpr (M::ID == SCP_MODEL_LANDER6) {
        if (!id.first()) {
#pragma unroll
            for (int r = 0; r < 3; ++r) Dx[r] = Dx[r] + T(1);       // glide cone
            Dx[8] = Dx[8] + T(1);                                   // tilt
            Dx[9] = Dx[9] + T(1);
#pragma unroll
            for (int r = 10; r < 13; ++r) Dx[r] = Dx[r] + T(1);     // rate ball
        }
#pragma unroll
        for (int r = 0; r < NU; ++r) Du[r] = Du[r] + T(3);          // thrust ball, bound, gimbal
    } else {
        if (!id.first()) {
#pragma unroll
            for (int r = 0; r < 3; ++r) Dx[r] = Dx[r] + T(1);
        }
#pragma unroll
        for (int r = 0; r < NU; ++r) Du[r] = Du[r] + T(1);
    }
}

// ------------------------------------------------------------------------------------------
// a4: Step-1 Hessian and its unpivoted Cholesky factor
// ------------------------------------------------------------------------------------------
// H11 = Q_i + rho_eq 1{i>0} I + rho_geo D_x + rho_dyn A'A
// H12 = rho_dyn A'B  (no cross cost term for the models here)
// H22 = R + rho_geo D_u + rho_dyn B'B  (i < N);  at node N the control block is I (unused).
// Returns SCP_ST_BADPIVOT if a pivot is not positive (the pivot is then replaced by 1 so the
// node stays finite; the status bit marks the trajectory).
template <class M, class T>
__device__ __forceinline__ int assemble_factor(const T* __restrict__ prm, const NodeId& id, const Rho<T>& rho,
                                               NodeConst<M, T>& nc) {
    constexpr int NX = M::NX, NU = M::NU, NN = M::NN, NXR = M::NXR;
    T Dx[NX], Du[NU];
    group_counts<M, T>(id, Dx, Du);
    const T rdyn = id.last() ? T(0) : rho.dyn;
    T* H = nc.L;  // factor in place
    // A'A, A'B, B'B with A = [E | Ar]
#pragma unroll
    for (int r = 0; r < NN; ++r) {
#pragma unroll
        for (int c = 0; c <= r; ++c) {
            T p = T(0);
            if (r < NX && c < NX) {
                // (A'A)_{rc}
                if (r < 3 && c < 3) {
                    p = (r == c) ? T(1) : T(0);
                } else if (c < 3) {
                    p = nc.Ar[c * NXR + (r - 3)];
                } else {
#pragma unroll
                    for (int k = 0; k < NX; ++k) p = p + nc.Ar[k * NXR + (r - 3)] * nc.Ar[k * NXR + (c - 3)];
                }
            } else if (r >= NX && c < NX) {
                // (A'B)_{c, r-NX}
                if (c < 3) {
                    p = nc.B[c * NU + (r - NX)];
                } else {
#pragma unroll
                    for (int k = 0; k < NX; ++k) p = p + nc.Ar[k * NXR + (c - 3)] * nc.B[k * NU + (r - NX)];
                }
            } else {
#pragma unroll
                for (int k = 0; k < NX; ++k) p = p + nc.B[k * NU + (r - NX)] * nc.B[k * NU + (c - NX)];
            }
            T v;
            if (r == c) {
                if (r < NX) {
                    const T q = id.last() ? prm[SCP_P_QN + r] : prm[SCP_P_QR + r];
                    v = ((q + (id.first() ? T(0) : rho.eq)) + rho.geo * Dx[r]) + rdyn * p;
                } else if (id.last()) {
                    v = T(1);
                } else {
                    v = (prm[SCP_P_R + (r - NX)] + rho.geo * Du[r - NX]) + rdyn * p;
                }
            } else {
                v = (r >= NX && id.last()) ? T(0) : rdyn * p;
            }
            H[tri(r, c)] = v;
        }
    }
    int st = 0;
#pragma unroll
    for (int c = 0; c < NN; ++c) {
        T s = H[tri(c, c)];
#pragma unroll
        for (int k = 0; k < c; ++k) s = s - H[tri(c, k)] * H[tri(c, k)];
        if (!(s > T(0))) {
            st |= SCP_ST_BADPIVOT;
            s = T(1);
        }
        const T inv = T(1) / tsqrt(s);
        H[tri(c, c)] = inv;
#pragma unroll
        for (int r = c + 1; r < NN; ++r) {
            T a = H[tri(r, c)];
#pragma unroll
            for (int k = 0; k < c; ++k) a = a - H[tri(r, k)] * H[tri(c, k)];
            H[tri(r, c)] = a * inv;
        }
    }
    return st;
}

// Solve L L' xi = g in place (forward then backward substitution).  L: the packed factor, or an
// accessor with operator[] over it (the persistent kernel may keep it in LDS).
template <class M, class T, class LA>
__device__ __forceinline__ void chol_solve(const LA& L, T* g) {
    constexpr int NN = M::NN;
#pragma unroll
    for (int r = 0; r < NN; ++r) {
        T s = g[r];
#pragma unroll
        for (int k = 0; k < r; ++k) s = s - L[tri(r, k)] * g[k];
        g[r] = s * L[tri(r, r)];
    }
#pragma unroll
    for (int r = NN - 1; r >= 0; --r) {
        T s = g[r];
#pragma unroll
        for (int k = r + 1; k < NN; ++k) s = s - L[tri(k, r)] * g[k];
        g[r] = s * L[tri(r, r)];
    }
}

// ------------------------------------------------------------------------------------------
// a5: Step 1 (physical layer)
// ------------------------------------------------------------------------------------------
// g_x = -q_i + 1{i>0}(rho_eq z_i - lambda_i) + 1{i<N} A_i' w_i + sum_g (rho_geo xhat^g - nu_x^g)
// g_u =         1{i<N} B_i' w_i + sum_g (rho_geo uhat^g - nu_u^g),  w_i = mu_{i+1} + rho_dyn (z_{i+1} - d_i)
// then x, u from the cached factor and d_dyn,i = A_i x_i + B_i u_i + d_i.
// Absent groups hold exactly zero copies and duals, so summing over all slots is exact.
// HSS: the half-space groups are carried in scalar form (hs_* below); their Step-1 term comes
// in hs_x (added to the position rows) instead of from s.cp / s.du.
template <class M, class T, bool HSS = false, class LA = const T*>
__device__ __forceinline__ void step1(const NodeId& id, const Rho<T>& rho, const NodeConst<M, T>& nc,
                                      NodeState<M, T>& s, const T* znext, const T* munext,
                                      const T* hs_x = nullptr, const LA* Lacc = nullptr) {
    constexpr int NX = M::NX, NU = M::NU, NN = M::NN;
    // A factor held outside the registers is fetched first; the scheduling barrier keeps the
    // loads ahead of the right-hand side, whose arithmetic then covers their latency.
    // The reciprocal diagonal stays in registers (nc.L), which trims the LDS traffic by a fifth.
    T Lr[Dims<M>::NL];
    if constexpr (!std::is_same<LA, const T*>::value) {
#pragma unroll
        for (int r = 0; r < NN; ++r)
#pragma unroll
            for (int c = 0; c <= r; ++c) Lr[tri(r, c)] = r == c ? nc.L[tri(r, r)] : (*Lacc)[tri(r, c)];
        __builtin_amdgcn_sched_barrier(0);
    }
    // No node masks are needed here: z_0 = lambda_0 = mu_0 = 0 always (node 0 has no dynamic
    // coupling), the caller passes the next node's z and mu, which at node N are those of a
    // node 0, of an idle lane or zeros, and d_N = 0; so w_N = 0 and A'w = B'w = 0 at node N,
    // and the terms below add exact zeros where the paper's sums have no term.
    T w[NX], g[NN], tx[NX], tu[NU];
#pragma unroll
    for (int r = 0; r < NX; ++r) w[r] = munext[r] + rho.dyn * (znext[r] - nc.d[r]);
    at_mul<M, T>(nc.Ar, w, tx);
    bt_mul<M, T>(nc.B, w, tu);
#pragma unroll
    for (int r = 0; r < NX; ++r) g[r] = (nc.g0[r] + (rho.eq * s.z[r] - s.lam[r])) + tx[r];
#pragma unroll
    for (int r = 0; r < NU; ++r) g[NX + r] = tu[r];
    // mirror terms, group order
#pragma unroll
    for (int r = 0; r < NX; ++r) g[r] = g[r] + (rho.geo * s.cp[M::C_XBOX + r] - s.du[M::C_XBOX + r]);
#pragma unroll
    for (int r = 0; r < NU; ++r) g[NX + r] = g[NX + r] + (rho.geo * s.cp[M::C_UBOX + r] - s.du[M::C_UBOX + r]);
    if constexpr (M::QL) {
        const T rb = group_rho<M>(id, rho.geo, 2);
#pragma unroll
        for (int r = 0; r < 3; ++r) g[NX + r] = g[NX + r] + (rb * s.cp[M::C_BALL + r] - s.du[M::C_BALL + r]);
        if constexpr (HSS) {
#pragma unroll
            for (int r = 0; r < 3; ++r) g[r] = g[r] + hs_x[r];
        } else {
#pragma unroll
            for (int j = 0; j < M::KM; ++j) {
                const T rj = group_rho<M>(id, rho.geo, 3 + j);
#pragma unroll
                for (int r = 0; r < 3; ++r)
                    g[r] = g[r] + (rj * s.cp[M::C_HS + 3 * j + r] - s.du[M::C_HS + 3 * j + r]);
            }
        }
    } else if constexpr (M::ID == SCP_MODEL_LANDER6) {
        const T rx = group_rho<M>(id, rho.geo, 2);   // glide, tilt and rate groups: nodes 1..N
        g[1] = g[1] + (rx * s.cp[M::C_GLIDE + 0] - s.du[M::C_GLIDE + 0]);
        g[2] = g[2] + (rx * s.cp[M::C_GLIDE + 1] - s.du[M::C_GLIDE + 1]);
        g[0] = g[0] + (rx * s.cp[M::C_GLIDE + 2] - s.du[M::C_GLIDE + 2]);
#pragma unroll
        for (int r = 0; r < 2; ++r) g[8 + r] = g[8 + r] + (rx * s.cp[M::C_TILT + r] - s.du[M::C_TILT + r]);
#pragma unroll
        for (int r = 0; r < 3; ++r) g[10 + r] = g[10 + r] + (rx * s.cp[M::C_RATE + r] - s.du[M::C_RATE + r]);
        const T ru = group_rho<M>(id, rho.geo, 5);   // thrust groups: nodes 0..N-1
#pragma unroll
        for (int r = 0; r < 3; ++r) g[NX + r] = g[NX + r] + (ru * s.cp[M::C_TBALL + r] - s.du[M::C_TBALL + r]);
#pragma unroll
        for (int r = 0; r < 3; ++r) g[NX + r] = g[NX + r] + (ru * s.cp[M::C_THS + r] - s.du[M::C_THS + r]);
        g[NX + 1] = g[NX + 1] + (ru * s.cp[M::C_GIMB + 0] - s.du[M::C_GIMB + 0]);
        g[NX + 2] = g[NX + 2] + (ru * s.cp[M::C_GIMB + 1] - s.du[M::C_GIMB + 1]);
        g[NX + 0] = g[NX + 0] + (ru * s.cp[M::C_GIMB + 2] - s.du[M::C_GIMB + 2]);
    } else {
        const T rc = group_rho<M>(id, rho.geo, 2);
#pragma unroll
        for (int r = 0; r < 3; ++r) g[r] = g[r] + (rc * s.cp[M::C_CONE + r] - s.du[M::C_CONE + r]);
#pragma unroll
        for (int r = 0; r < 4; ++r) g[NX + r] = g[NX + r] + (rho.geo * s.cp[M::C_SOC + r] - s.du[M::C_SOC + r]);
    }
    if constexpr (std::is_same<LA, const T*>::value) chol_solve<M, T>(nc.L, g);
    else chol_solve<M, T>(Lr, g);
#pragma unroll
    for (int r = 0; r < NX; ++r) s.x[r] = g[r];
#pragma unroll
    for (int r = 0; r < NU; ++r) s.u[r] = id.last() ? T(0) : g[NX + r];
    T ax[NX];
    a_mul<M, T>(nc.Ar, s.x, ax);
#pragma unroll
    for (int r = 0; r < NX; ++r) {
        T bu = T(0);
#pragma unroll
        for (int c = 0; c < NU; ++c) bu = bu + nc.B[r * NU + c] * s.u[c];
        s.dd[r] = (ax[r] + bu) + nc.d[r];  // meaningless at node N (no interval); never read there
    }
}

// ------------------------------------------------------------------------------------------
// a6: Step 2 (dynamic layer), i >= 1
// ------------------------------------------------------------------------------------------
template <class M, class T>
__device__ __forceinline__ void step2(const NodeId& id, const Rho<T>& rho, NodeState<M, T>& s, const T* ddprev) {
    if (id.first()) return;
#pragma unroll
    for (int r = 0; r < M::NX; ++r)
        s.z[r] = (((rho.eq * s.x[r] + s.lam[r]) + rho.dyn * ddprev[r]) - s.mu[r]) * rho.inv_sum;
}

// ------------------------------------------------------------------------------------------
// a7: Step 3 (geometric layer): copy^g = projection of (var^g + nu^g / rho_geo)
// ------------------------------------------------------------------------------------------
// The u copies at node 0 of a consensus group are averaged afterwards by the caller.  Copies of
// groups absent at this node are finite dummies (see group_rho).
template <class M, class T, bool HSS = false>
__device__ __forceinline__ void step3(const NodeId& id, const Rho<T>& rho, const NodeConst<M, T>& nc,
                                      NodeState<M, T>& s, T ball_r, T kappa, T inv1k2,
                                      const T* __restrict__ prm = nullptr) {
    constexpr int NX = M::NX, NU = M::NU;
    // x box
#pragma unroll
    for (int r = 0; r < NX; ++r)
        s.cp[M::C_XBOX + r] = clampv(s.x[r] + s.du[M::C_XBOX + r] * rho.inv_geo, nc.lo[r], nc.hi[r]);
    // u box (at node N: u = 0, dual 0 and box [0, 0], so the copy is 0 without a mask)
#pragma unroll
    for (int r = 0; r < NU; ++r)
        s.cp[M::C_UBOX + r] = clampv(s.u[r] + s.du[M::C_UBOX + r] * rho.inv_geo, nc.lo[NX + r], nc.hi[NX + r]);
    if constexpr (M::QL) {
        {
            T v[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) v[r] = s.u[r] + s.du[M::C_BALL + r] * rho.inv_geo;
            proj_ball3(ball_r, v);
#pragma unroll
            for (int r = 0; r < 3; ++r) s.cp[M::C_BALL + r] = v[r];
        }
#pragma unroll
        for (int j = 0; j < (HSS ? 0 : M::KM); ++j) {
            T v[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) v[r] = s.x[r] + s.du[M::C_HS + 3 * j + r] * rho.inv_geo;
            proj_halfspace(&nc.hs[4 * j], nc.hs[4 * j + 3], v);
#pragma unroll
            for (int r = 0; r < 3; ++r) s.cp[M::C_HS + 3 * j + r] = v[r];
        }
    } else if constexpr (M::ID == SCP_MODEL_LANDER6) {
        const T ig = rho.inv_geo;
        {   // glide cone, components (r_E, r_N, r_U): the axis last
            const T kg = prm[SCP_P_GLIDE];
            T v[3] = {s.x[1] + s.du[M::C_GLIDE + 0] * ig, s.x[2] + s.du[M::C_GLIDE + 1] * ig,
                      s.x[0] + s.du[M::C_GLIDE + 2] * ig};
            proj_cone<3>(kg, T(1) / (T(1) + kg * kg), v);
#pragma unroll
            for (int r = 0; r < 3; ++r) s.cp[M::C_GLIDE + r] = v[r];
        }
        {   // tilt: |(q_y, q_z)| <= sin(tilt / 2)
            T v[2] = {s.x[8] + s.du[M::C_TILT + 0] * ig, s.x[9] + s.du[M::C_TILT + 1] * ig};
            proj_ball2(prm[SCP_P_TILT], v);
            s.cp[M::C_TILT + 0] = v[0];
            s.cp[M::C_TILT + 1] = v[1];
        }
        {   // body-rate ball
            T v[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) v[r] = s.x[10 + r] + s.du[M::C_RATE + r] * ig;
            proj_ball3(prm[SCP_P_WMAX], v);
#pragma unroll
            for (int r = 0; r < 3; ++r) s.cp[M::C_RATE + r] = v[r];
        }
        {   // thrust magnitude upper bound
            T v[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) v[r] = s.u[r] + s.du[M::C_TBALL + r] * ig;
            proj_ball3(prm[SCP_P_TMAX], v);
#pragma unroll
            for (int r = 0; r < 3; ++r) s.cp[M::C_TBALL + r] = v[r];
        }
        {   // linearized thrust lower bound (unit normal)
            T v[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) v[r] = s.u[r] + s.du[M::C_THS + r] * ig;
            proj_halfspace(&nc.hs[0], nc.hs[3], v);
#pragma unroll
            for (int r = 0; r < 3; ++r) s.cp[M::C_THS + r] = v[r];
        }
        {   // gimbal cone, components (T_y, T_z, T_x)
            const T kq = prm[SCP_P_GIMBAL];
            T v[3] = {s.u[1] + s.du[M::C_GIMB + 0] * ig, s.u[2] + s.du[M::C_GIMB + 1] * ig,
                      s.u[0] + s.du[M::C_GIMB + 2] * ig};
            proj_cone<3>(kq, T(1) / (T(1) + kq * kq), v);
#pragma unroll
            for (int r = 0; r < 3; ++r) s.cp[M::C_GIMB + r] = v[r];
        }
    } else {
        {
            T v[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) v[r] = s.x[r] + s.du[M::C_CONE + r] * rho.inv_geo;
            proj_cone<3>(kappa, inv1k2, v);
#pragma unroll
            for (int r = 0; r < 3; ++r) s.cp[M::C_CONE + r] = v[r];
        }
        {
            T v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = s.u[r] + s.du[M::C_SOC + r] * rho.inv_geo;
            proj_cone<4>(T(1), T(0.5), v);  // at node N the input is 0 and so is the copy
#pragma unroll
            for (int r = 0; r < 4; ++r) s.cp[M::C_SOC + r] = v[r];
        }
    }
}

// variable component feeding mirror slot k (x or u), and the group of slot k
template <class M>
__device__ __forceinline__ constexpr int slot_group(int k) {
    if constexpr (M::QL) {
        return k < M::C_UBOX ? 0 : k < M::C_BALL ? 1 : k < M::C_HS ? 2 : 3 + (k - M::C_HS) / 3;
    } else if constexpr (M::ID == SCP_MODEL_LANDER6) {
        return k < M::C_UBOX ? 0 : k < M::C_GLIDE ? 1 : k < M::C_TILT ? 2 : k < M::C_RATE ? 3 : k < M::C_TBALL ? 4
             : k < M::C_THS ? 5 : k < M::C_GIMB ? 6 : 7;
    } else {
        return k < M::C_UBOX ? 0 : k < M::C_CONE ? 1 : k < M::C_SOC ? 2 : 3;
    }
}
// Slots whose group is absent only at node N, where variable, dual and copy are all 0, so their
// dual update needs no mask: the x box (always present), the u box and the SOC.
template <class M>
__device__ __forceinline__ constexpr bool slot_self_zero(int k) {
    if constexpr (M::QL) {
        return k < M::C_BALL;
    } else if constexpr (M::ID == SCP_MODEL_LANDER6) {
        // x box, u box, thrust ball and gimbal cone (both project 0 to 0 at node N)
        return k < M::C_GLIDE || (k >= M::C_TBALL && k < M::C_THS) || k >= M::C_GIMB;
    } else {
        return k < M::C_CONE || k >= M::C_SOC;
    }
}
template <class M>
__device__ __forceinline__ constexpr bool slot_is_u(int k) {
    if constexpr (M::QL) {
        return k >= M::C_UBOX && k < M::C_HS;
    } else if constexpr (M::ID == SCP_MODEL_LANDER6) {
        return (k >= M::C_UBOX && k < M::C_GLIDE) || k >= M::C_TBALL;
    } else {
        return (k >= M::C_UBOX && k < M::C_CONE) || k >= M::C_SOC;
    }
}
template <class M>
__device__ __forceinline__ constexpr int slot_comp(int k) {
    if constexpr (M::QL) {
        return k < M::C_UBOX ? k : k < M::C_BALL ? k - M::C_UBOX : k < M::C_HS ? k - M::C_BALL : (k - M::C_HS) % 3;
    } else if constexpr (M::ID == SCP_MODEL_LANDER6) {
        // the cones list their components axis last: (1, 2, 0)
        return k < M::C_UBOX ? k : k < M::C_GLIDE ? k - M::C_UBOX : k < M::C_TILT ? (k - M::C_GLIDE + 1) % 3
             : k < M::C_RATE ? 8 + (k - M::C_TILT) : k < M::C_TBALL ? 10 + (k - M::C_RATE)
             : k < M::C_THS ? k - M::C_TBALL : k < M::C_GIMB ? k - M::C_THS : (k - M::C_GIMB + 1) % 3;
    } else {
        return k < M::C_UBOX ? k : k < M::C_CONE ? k - M::C_UBOX : k < M::C_SOC ? k - M::C_CONE : k - M::C_SOC;
    }
}

template <class M, class T>
__device__ __forceinline__ T slot_var(const NodeState<M, T>& s, int k) {
    return slot_is_u<M>(k) ? s.u[slot_comp<M>(k)] : s.x[slot_comp<M>(k)];
}

// ------------------------------------------------------------------------------------------
// a8: Step 4 (dual ascent)
// ------------------------------------------------------------------------------------------
template <class M, class T, bool HSS = false>
__device__ __forceinline__ void step4(const NodeId& id, const Rho<T>& rho, NodeState<M, T>& s, const T* ddprev) {
    if (!id.first()) {
#pragma unroll
        for (int r = 0; r < M::NX; ++r) {
            s.lam[r] = s.lam[r] + rho.eq * (s.x[r] - s.z[r]);
            s.mu[r] = s.mu[r] + rho.dyn * (s.z[r] - ddprev[r]);
        }
    }
#pragma unroll
    for (int k = 0; k < M::C; ++k) {
        if constexpr (HSS && M::QL) {
            if (k >= M::C_HS) continue;
        }
        // groups absent only at node N with a zero copy there (u box, SOC) update to 0 by
        // themselves; the others use their group penalty, 0 where they are absent
        const T rg = slot_self_zero<M>(k) ? rho.geo : group_rho<M>(id, rho.geo, slot_group<M>(k));
        s.du[k] = s.du[k] + rg * (slot_var<M, T>(s, k) - s.cp[k]);
    }
}

// ------------------------------------------------------------------------------------------
// Half-space groups in scalar form (persistent kernel)
// ------------------------------------------------------------------------------------------
// With a unit normal a, the projection onto {a'y >= b} moves its input along a only, so after
// one ADMM iteration the group's dual is nu = -sigma a with sigma = rho t, t = max(0, b - a'v),
// and its copy is x + ((kappa - sigma) / rho) a with kappa = 2 sigma - sigma_prev.  Steps 1, 3
// and 4 then need per group two scalars instead of two 3-vectors.  They are kept divided by
// rho (s = sigma / rho, k = kappa / rho), which removes two multiplications per group:
//   Step 1 term  rho cp - nu = rho x_prev + rho sum_j k_j a_j (+ e, below)
//   Step 3 + 4   t = max(0, b - (a'x - s)),  s' = t,  k' = 2 s' - s
// The dual carried into an SCP iteration, nu_c, is generally not along the new normal: with
// sigma_0 = -a'nu_c and the orthogonal part p = nu_c + sigma_0 a (kappa_0 = sigma_0), the Step-1
// term carries e = -p in the first ADMM iteration and e = +p in the second, and the copy of the
// first iteration has the extra p / rho.  All of this is exact in real arithmetic (a'a = 1).
// The caller keeps e (the sum of p over the groups, with its sign for the coming iteration) in
// registers and p itself in LDS, read only on the iterations that need it.
// Absent groups have a = 0, b = 0 and therefore t = 0: no masks.  Every multiply-add below is an
// explicit FMA, so each kernel instantiation rounds the same way.

// Enter an SCP iteration: scalars from the carried duals s.du (vector form) and the new normals.
// perp receives p (3 per group), psum the sum over groups.
template <class M, class T>
__device__ __forceinline__ void hs_enter(const NodeConst<M, T>& nc, const Rho<T>& rho, const NodeState<M, T>& s,
                                         T* sc, T* kc, T* perp, T* psum) {
#pragma unroll
    for (int r = 0; r < 3; ++r) psum[r] = T(0);
#pragma unroll
    for (int j = 0; j < M::KM; ++j) {
        const T* a = &nc.hs[4 * j];
        const T* du = &s.du[M::C_HS + 3 * j];
        const T s0 = -tfma(a[2], du[2], tfma(a[1], du[1], a[0] * du[0]));
        sc[j] = kc[j] = s0 * rho.inv_geo;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            perp[3 * j + r] = tfma(s0, a[r], du[r]);
            psum[r] = psum[r] + perp[3 * j + r];
        }
    }
}

// Step-1 term of all half-space groups: nr x_prev + e + rho sum_j k_j a_j, with nr = rho_geo
// times the number of groups at this node and e = -sum p (first ADMM iteration of the SCP
// iteration), +sum p (second) or 0 (later).
template <class M, class T>
__device__ __forceinline__ void hs_step1_term(const NodeConst<M, T>& nc, const Rho<T>& rho, const T* xprev, T nr,
                                              const T* kc, const T* e, T* hx) {
    T acc[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) acc[r] = kc[0] * nc.hs[r];
#pragma unroll
    for (int j = 1; j < M::KM; ++j)
#pragma unroll
        for (int r = 0; r < 3; ++r) acc[r] = tfma(kc[j], nc.hs[4 * j + r], acc[r]);
#pragma unroll
    for (int r = 0; r < 3; ++r) hx[r] = tfma(rho.geo, acc[r], tfma(nr, xprev[r], e[r]));
}

// Steps 3 and 4 of all half-space groups.
template <class M, class T>
__device__ __forceinline__ void hs_step34(const NodeConst<M, T>& nc, const T* x, T* sc, T* kc) {
#pragma unroll
    for (int j = 0; j < M::KM; ++j) {
        const T* a = &nc.hs[4 * j];
        const T av = tfma(a[2], x[2], tfma(a[1], x[1], tfma(a[0], x[0], -sc[j])));
        const T t = tmaxv(T(0), a[3] - av);
        kc[j] = tfma(T(2), t, -sc[j]);  // 2 t is exact: one rounding, as (t + t) - s
        sc[j] = t;
    }
}

// Vector form of the half-space copies into s.cp.  perp: p of every group after exactly one
// ADMM iteration of the SCP iteration, else nullptr.
template <class M, class T>
__device__ __forceinline__ void hs_copies(const NodeConst<M, T>& nc, const Rho<T>& rho, NodeState<M, T>& s,
                                          const T* sc, const T* kc, const T* perp) {
#pragma unroll
    for (int j = 0; j < M::KM; ++j) {
        const T c = kc[j] - sc[j];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            T v = tfma(c, nc.hs[4 * j + r], s.x[r]);
            if (perp) v = tfma(perp[3 * j + r], rho.inv_geo, v);
            s.cp[M::C_HS + 3 * j + r] = v;
        }
    }
}
// Vector form of the half-space duals into s.du.  perp: p of every group when no ADMM iteration
// has run in the SCP iteration, else nullptr.
template <class M, class T>
__device__ __forceinline__ void hs_duals(const NodeConst<M, T>& nc, const Rho<T>& rho, NodeState<M, T>& s,
                                         const T* sc, const T* perp) {
#pragma unroll
    for (int j = 0; j < M::KM; ++j) {
        const T sig = rho.geo * sc[j];
#pragma unroll
        for (int r = 0; r < 3; ++r)
            s.du[M::C_HS + 3 * j + r] = perp ? tfma(-sig, nc.hs[4 * j + r], perp[3 * j + r])
                                             : -sig * nc.hs[4 * j + r];
    }
}

// ------------------------------------------------------------------------------------------
// a9: residual pieces
// ------------------------------------------------------------------------------------------
// primal: max |x - z|, |z - d_dyn,i-1| (i >= 1), |var - copy| (active groups)
template <class M, class T>
__device__ __forceinline__ T primal_res(const NodeId& id, const NodeState<M, T>& s, const T* ddprev) {
    T m = T(0);
    if (!id.first()) {
#pragma unroll
        for (int r = 0; r < M::NX; ++r) {
            m = nmax(m, tabs(s.x[r] - s.z[r]));
            m = nmax(m, tabs(s.z[r] - ddprev[r]));
        }
    }
#pragma unroll
    for (int k = 0; k < M::C; ++k) {
        if (group_active<M>(id, slot_group<M>(k))) m = nmax(m, tabs(slot_var<M, T>(s, k) - s.cp[k]));
    }
    return m;
}

// dual: max |s_i| with s_x = rho_eq dz_i + rho_dyn A'dz_{i+1} + rho_geo sum dxhat,
//                      s_u = rho_dyn B'dz_{i+1} + rho_geo sum duhat
// dcp holds copy - copy_old per slot; dz = z - z_old of this node; dznext of node i+1.
template <class M, class T>
__device__ __forceinline__ T dual_res(const NodeId& id, const Rho<T>& rho, const NodeConst<M, T>& nc,
                                      const T* dz, const T* dznext, const T* dcp) {
    constexpr int NX = M::NX, NU = M::NU;
    T sx[NX], su[NU], tx[NX], tu[NU];
    T w[NX];
#pragma unroll
    for (int r = 0; r < NX; ++r) w[r] = id.last() ? T(0) : dznext[r];
    at_mul<M, T>(nc.Ar, w, tx);
    bt_mul<M, T>(nc.B, w, tu);
#pragma unroll
    for (int r = 0; r < NX; ++r) {
        T v = T(0);
        if (!id.first()) v = v + rho.eq * dz[r];
        if (!id.last()) v = v + rho.dyn * tx[r];
        sx[r] = v;
    }
#pragma unroll
    for (int r = 0; r < NU; ++r) su[r] = id.last() ? T(0) : rho.dyn * tu[r];
#pragma unroll
    for (int k = 0; k < M::C; ++k) {
        if (!group_active<M>(id, slot_group<M>(k))) continue;
        const T v = rho.geo * dcp[k];
        if (slot_is_u<M>(k)) su[slot_comp<M>(k)] = su[slot_comp<M>(k)] + v;
        else sx[slot_comp<M>(k)] = sx[slot_comp<M>(k)] + v;
    }
    T m = T(0);
#pragma unroll
    for (int r = 0; r < NX; ++r) m = nmax(m, tabs(sx[r]));
    if (!id.last()) {
#pragma unroll
        for (int r = 0; r < NU; ++r) m = nmax(m, tabs(su[r]));
    }
    return m;
}

// index of slot k among the u slots (scratch addressing)
template <class M>
__device__ __forceinline__ constexpr int slot_comp_u(int k) {
    if constexpr (M::QL) {
        return k - M::C_UBOX;   // u box 0..NU-1, ball NU..NU+2
    } else if constexpr (M::ID == SCP_MODEL_LANDER6) {
        return k < M::C_GLIDE ? k - M::C_UBOX : NU_OF<M>() + (k - M::C_TBALL);   // no consensus groups
    } else {
        return k < M::C_CONE ? k - M::C_UBOX : NU_OF<M>() + (k - M::C_SOC);
    }
}

// node-local part of the dual-residual vector: x part rho_eq dz (i >= 1) + rho_geo sum dxhat,
// u part rho_geo sum duhat (active groups, slot order).  skip_u: leave the u slots out (node 0
// of a consensus group, finished after the scenario average).
template <class M, class T>
__device__ __forceinline__ void dual_res_own(const NodeId& id, const Rho<T>& rho, const T* dz, const T* dcp, T* sp,
                                             bool skip_u) {
    constexpr int NX = M::NX, NU = M::NU;
#pragma unroll
    for (int r = 0; r < NX; ++r) sp[r] = id.first() ? T(0) : rho.eq * dz[r];
#pragma unroll
    for (int r = 0; r < NU; ++r) sp[NX + r] = T(0);
#pragma unroll
    for (int k = 0; k < M::C; ++k) {
        if (!group_active<M>(id, slot_group<M>(k))) continue;
        if (slot_is_u<M>(k)) {
            if (!skip_u) sp[NX + slot_comp<M>(k)] = sp[NX + slot_comp<M>(k)] + rho.geo * dcp[k];
        } else {
            sp[slot_comp<M>(k)] = sp[slot_comp<M>(k)] + rho.geo * dcp[k];
        }
    }
}

// add the neighbour term rho_dyn [A B]' dz_{i+1} and return the inf-norm
template <class M, class T>
__device__ __forceinline__ T dual_res_finish(const NodeId& id, const Rho<T>& rho, const T* Ar, const T* B, const T* sp,
                                             const T* dznext) {
    constexpr int NX = M::NX, NU = M::NU;
    T w[NX], tx[NX], tu[NU];
#pragma unroll
    for (int r = 0; r < NX; ++r) w[r] = id.last() ? T(0) : dznext[r];
    at_mul<M, T>(Ar, w, tx);
    bt_mul<M, T>(B, w, tu);
    T m = T(0);
#pragma unroll
    for (int r = 0; r < NX; ++r) m = nmax(m, tabs(id.last() ? sp[r] : sp[r] + rho.dyn * tx[r]));
    if (!id.last()) {
#pragma unroll
        for (int r = 0; r < NU; ++r) m = nmax(m, tabs(sp[NX + r] + rho.dyn * tu[r]));
    }
    return m;
}

// primal residual without the u slots (node 0 of a consensus group)
template <class M, class T>
__device__ __forceinline__ T primal_res_skip_u(const NodeId& id, const NodeState<M, T>& s, const T* ddprev) {
    T m = T(0);
    if (!id.first()) {
#pragma unroll
        for (int r = 0; r < M::NX; ++r) {
            m = nmax(m, tabs(s.x[r] - s.z[r]));
            m = nmax(m, tabs(s.z[r] - ddprev[r]));
        }
    }
#pragma unroll
    for (int k = 0; k < M::C; ++k) {
        if (slot_is_u<M>(k)) continue;
        if (group_active<M>(id, slot_group<M>(k))) m = nmax(m, tabs(slot_var<M, T>(s, k) - s.cp[k]));
    }
    return m;
}

// order-preserving bit pattern of a non-negative residual (NaN sorts above every number)
template <class T>
__device__ __forceinline__ unsigned long long res_bits(T v) {
    return (unsigned long long)__double_as_longlong((double)v);
}
__device__ __forceinline__ double bits_res(unsigned long long b) { return __longlong_as_double((long long)b); }

// Residual blow-up (failure detection; the paper has no such rule).  At the acceptance step of
// every SCP iteration, rp (the primal residual of the iteration's last ADMM iteration) updates
// rp0, the first positive one since the problem was created, reset or admitted (0 = none yet),
// and rpmax, the largest one since then (a NaN changes neither).  The trajectory has blown up
// once rpmax exceeds SCP_RP_BLOWUP times rp0: the same as testing every rp against rp0 as it
// comes, which is what the oracle does.  Compared in the problem precision (the factor is exact
// in FP32).
template <class T>
__device__ __forceinline__ void blowup_track(T& rp0, T& rpmax, const T rp) {
    rp0 = rp0 > T(0) ? rp0 : (rp > T(0) ? rp : T(0));
    rpmax = rp > rpmax ? rp : rpmax;
}

template <class T>
__device__ __forceinline__ int blowup_status(const T rp0, const T rpmax) {
    return (rp0 > T(0) && rpmax > T(SCP_RP_BLOWUP) * rp0) ? SCP_ST_DIVERGED : 0;
}

// trust-region ratio test on the merit (reading of the omitted update logic, Sec. III-A)
template <class T>
struct AcceptOut {
    bool accept, nonfinite;
    T ratio, delta;
};

template <class T>
__device__ __forceinline__ AcceptOut<T> accept_rule(T eta0, T eta1, T eta2, T shrink, T grow, T dmax, T mnom, T mnew,
                                                    T mmod, T delta) {
    AcceptOut<T> a;
    const T actual = mnom - mnew;
    const T pred = mnom - mmod;
    T ratio = pred > T(0) ? actual / pred : -T(INFINITY);
    a.nonfinite = !(__builtin_isfinite(mnew) && __builtin_isfinite(mmod));
    if (a.nonfinite) ratio = T(NAN);
    a.accept = ratio >= eta0;
    if (ratio < eta1) delta = delta * shrink;
    else if (ratio > eta2) delta = tmin(delta * grow, dmax);
    a.ratio = ratio;
    a.delta = delta;
    return a;
}

// ------------------------------------------------------------------------------------------
// a10: merit terms and metrics of one node
// ------------------------------------------------------------------------------------------
// running/terminal cost of one node: 0.5 x'Qr x + 0.5 u'R u (i < N) or 0.5 x'Qn x + qn'x + cN
template <class M, class T>
__device__ __forceinline__ T node_cost(const T* __restrict__ prm, const NodeId& id, const T* x, const T* u) {
    constexpr int NX = M::NX, NU = M::NU;
    if (id.last()) {
        T a = T(0), b = T(0);
#pragma unroll
        for (int r = 0; r < NX; ++r) a = a + x[r] * (prm[SCP_P_QN + r] * x[r]);
#pragma unroll
        for (int r = 0; r < NX; ++r) b = b + prm[SCP_P_QNV + r] * x[r];
        return (T(0.5) * a + b) + prm[SCP_P_CN];
    }
    T a = T(0), b = T(0);
#pragma unroll
    for (int r = 0; r < NX; ++r) a = a + x[r] * (prm[SCP_P_QR + r] * x[r]);
#pragma unroll
    for (int r = 0; r < NU; ++r) b = b + u[r] * (prm[SCP_P_R + r] * u[r]);
    return T(0.5) * a + T(0.5) * b;
}

// max violation of the hard constraints at one node (oracle's definition)
template <class M, class T>
__device__ __forceinline__ T node_violation(const T* __restrict__ prm, const NodeId& id, const T* x, const T* u) {
    constexpr int NX = M::NX, NU = M::NU;
    T v = T(0);
#pragma unroll
    for (int r = 0; r < NX; ++r) {
        v = nmax(v, prm[SCP_P_XLO + r] - x[r]);
        v = nmax(v, x[r] - prm[SCP_P_XHI + r]);
    }
    if (!id.last()) {
#pragma unroll
        for (int r = 0; r < NU; ++r) {
            v = nmax(v, prm[SCP_P_ULO + r] - u[r]);
            v = nmax(v, u[r] - prm[SCP_P_UHI + r]);
        }
    }
    if constexpr (M::QL) {
        if (!id.last() && id.ball) {
            const T nu = tsqrt((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]);
            v = nmax(v, nu - prm[SCP_P_UBALL]);
        }
        if (!id.first()) {
            const int cyl = (int)prm[SCP_P_CYL];
            for (int j = 0; j < id.K; ++j) {
                const T* o = prm + SCP_P_OBS + 4 * j;
                const T d0 = x[0] - o[0], d1 = x[1] - o[1], d2 = ((cyl >> j) & 1) ? T(0) : x[2] - o[2];
                v = nmax(v, o[3] - tsqrt((d0 * d0 + d1 * d1) + d2 * d2));
            }
        }
    } else if constexpr (M::ID == SCP_MODEL_LANDER6) {
        if (!id.last()) {
            const T nt = tsqrt((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]);
            v = nmax(v, nt - prm[SCP_P_TMAX]);
            v = nmax(v, prm[SCP_P_TMIN] - nt);
            v = nmax(v, tsqrt(u[1] * u[1] + u[2] * u[2]) - prm[SCP_P_GIMBAL] * u[0]);
        }
        if (!id.first()) {
            v = nmax(v, tsqrt(x[1] * x[1] + x[2] * x[2]) - prm[SCP_P_GLIDE] * x[0]);
            v = nmax(v, tsqrt(x[8] * x[8] + x[9] * x[9]) - prm[SCP_P_TILT]);
            v = nmax(v, tsqrt((x[10] * x[10] + x[11] * x[11]) + x[12] * x[12]) - prm[SCP_P_WMAX]);
        }
    } else {
        if (!id.last()) {
            const T nt = tsqrt((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]);
            v = nmax(v, nt - u[3]);
        }
        if (!id.first()) {
            const T rxy = tsqrt(x[0] * x[0] + x[1] * x[1]);
            v = nmax(v, rxy - prm[SCP_P_GLIDE] * x[2]);
        }
    }
    return v;
}

// boundary error at one node
template <class M, class T>
__device__ __forceinline__ T node_bnd_err(const T* __restrict__ prm, const NodeId& id, const T* x) {
    T e = T(0);
    if (id.first()) {
#pragma unroll
        for (int r = 0; r < M::NX; ++r) e = nmax(e, tabs(x[r] - prm[SCP_P_XINIT + r]));
    }
    if (id.last()) {
#pragma unroll
        for (int r = 0; r < M::NX; ++r)
            if (prm[SCP_P_TMASK + r] != T(0)) e = nmax(e, tabs(x[r] - prm[SCP_P_XTGT + r]));
    }
    return e;
}

}  // namespace scp

// Device side of the request server: admission of staged requests into the pool (cold start
// from the request's initial guess, or in-place MPC warm start from the session's previous
// solution) and collection of finished requests into the output staging.
#include "scp_device.hpp"
#include "scp_launch.hpp"
#include "scp_layout.hpp"

namespace scp {

// Receding-horizon shift of resident trajectories (Sec. IV-A.4, scenario MPC): state-indexed
// rows move one node earlier with the last repeated, control-indexed rows likewise over their N
// rows; lambda_0 = mu_0 = 0 and every mirror dual where its group does not exist is 0.
// The nodes of an admission move in parallel, one thread per node, in chunks of the block: every
// thread of a chunk loads its source row (node i + 1) into registers, the block synchronizes, then
// every thread stores its row i.  A chunk's stores reach rows of that chunk only, and the rows the
// next chunk loads lie past it, so each row is read before it is overwritten, as in a walk of the
// nodes in increasing order.  Pure data movement: the result is the same bits whatever the order.
constexpr int SHIFT_NV = 3 * PERSIST_MAX_NX + 4 + PERSIST_MAX_C;   // x, lambda, mu rows; u (<= 4); copies' duals

template <class M, class T>
__device__ __forceinline__ void shift_load(const T* __restrict__ pl, const int P, const size_t src, const bool urow,
                                           T (&v)[SHIFT_NV]) {
    static_assert(3 * M::NX + M::NU + M::C <= SHIFT_NV, "shift row does not fit");
#pragma unroll
    for (int r = 0; r < M::NX; ++r) {
        v[3 * r] = pl[(size_t)(PL_XBAR + r) * P + src];
        v[3 * r + 1] = pl[(size_t)(PL_LAM + r) * P + src];
        v[3 * r + 2] = pl[(size_t)(PL_MU + r) * P + src];
    }
    if (urow) {
#pragma unroll
        for (int r = 0; r < M::NU; ++r) v[3 * M::NX + r] = pl[(size_t)(PL_UBAR + r) * P + src];
    }
#pragma unroll
    for (int q = 0; q < M::C; ++q)
        if (!slot_is_u<M>(q) || urow) v[3 * M::NX + M::NU + q] = pl[(size_t)(PL_DU + q) * P + src];
}

template <class M, class T>
__device__ __forceinline__ void shift_store(T* __restrict__ pl, const int P, const size_t dst, const bool urow,
                                            const T (&v)[SHIFT_NV]) {
#pragma unroll
    for (int r = 0; r < M::NX; ++r) {
        pl[(size_t)(PL_XBAR + r) * P + dst] = v[3 * r];
        pl[(size_t)(PL_LAM + r) * P + dst] = v[3 * r + 1];
        pl[(size_t)(PL_MU + r) * P + dst] = v[3 * r + 2];
    }
    if (urow) {
#pragma unroll
        for (int r = 0; r < M::NU; ++r) pl[(size_t)(PL_UBAR + r) * P + dst] = v[3 * M::NX + r];
    }
#pragma unroll
    for (int q = 0; q < M::C; ++q)
        if (!slot_is_u<M>(q) || urow) pl[(size_t)(PL_DU + q) * P + dst] = v[3 * M::NX + M::NU + q];
}

template <class M, class T>
__device__ __forceinline__ void shift_clear(T* __restrict__ pl, const int P, const size_t g, const NodeId& id) {
    if (id.i == 0) {
#pragma unroll
        for (int r = 0; r < M::NX; ++r) {
            pl[(size_t)(PL_LAM + r) * P + g] = T(0);
            pl[(size_t)(PL_MU + r) * P + g] = T(0);
        }
    }
#pragma unroll
    for (int q = 0; q < M::C; ++q)
        if (!group_active<M>(id, slot_group<M>(q))) pl[(size_t)(PL_DU + q) * P + g] = T(0);
}

// Shift every trajectory of one admission record.  s_nt: the record's node -> trajectory map
// (global trajectory indices), s_traj: its trajectory records.  Called by the whole block.
template <class T>
__device__ void shift_admission(T* __restrict__ pl, const int P, const int node_off, const int n_nodes,
                                const int traj_first, const int* __restrict__ s_nt,
                                const int* __restrict__ s_traj) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int base = 0; base < n_nodes; base += nt) {
        const int k = base + tid;
        bool mv = false, urow = false, quad = false;
        T v[SHIFT_NV];
        if (k < n_nodes) {
            const int* rec = s_traj + (s_nt[k] - traj_first) * TR_FIELDS;
            const int i = node_off + k - rec[TR_OFF], N = rec[TR_N];
            mv = i < N;          // rows 0..N-1 take row i + 1; row N stays
            urow = i + 1 < N;    // control rows 0..N-2 take row i + 1; row N-1 stays
            quad = rec[TR_MODEL] == SCP_MODEL_QUAD_PM;
            if (mv) {
                if (quad) shift_load<Quad<8>, T>(pl, P, (size_t)node_off + k + 1, urow, v);
                else shift_load<Mars, T>(pl, P, (size_t)node_off + k + 1, urow, v);
            }
        }
        __syncthreads();
        if (mv) {
            if (quad) shift_store<Quad<8>, T>(pl, P, (size_t)node_off + k, urow, v);
            else shift_store<Mars, T>(pl, P, (size_t)node_off + k, urow, v);
        }
        __syncthreads();
    }
    for (int k = tid; k < n_nodes; k += nt) {
        const int* rec = s_traj + (s_nt[k] - traj_first) * TR_FIELDS;
        const NodeId id{node_off + k - rec[TR_OFF], rec[TR_N], rec[TR_K], rec[TR_BALL] != 0};
        if (rec[TR_MODEL] == SCP_MODEL_QUAD_PM) shift_clear<Quad<8>, T>(pl, P, (size_t)node_off + k, id);
        else shift_clear<Mars, T>(pl, P, (size_t)node_off + k, id);
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_admit(Dev<T> dv, int block, const unsigned char* __restrict__ blob, int rec_off) {
    const AdmitRec r = reinterpret_cast<const AdmitRec*>(blob + rec_off)[blockIdx.x];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int P = dv.P;
    const int* s_traj = reinterpret_cast<const int*>(blob + r.o_traj);
    const T* s_prm = reinterpret_cast<const T*>(blob + r.o_params);
    const int* s_nt = reinterpret_cast<const int*>(blob + r.o_node_traj);
    const int* s_lane = reinterpret_cast<const int*>(blob + r.o_lane);
    const int* s_wi = reinterpret_cast<const int*>(blob + r.o_wginfo);
    const int* s_wg = reinterpret_cast<const int*>(blob + r.o_wggroup);
    int* traj = const_cast<int*>(dv.traj);
    T* prm = const_cast<T*>(dv.params);
    int* node_traj = const_cast<int*>(dv.node_traj);
    int* lane = const_cast<int*>(dv.lane_node);
    int* wi = const_cast<int*>(dv.wg_info);
    int* wg = const_cast<int*>(dv.wg_group);

    for (int k = tid; k < r.n_traj * TR_FIELDS; k += nt) traj[(size_t)r.traj_first * TR_FIELDS + k] = s_traj[k];
    for (int k = tid; k < r.n_traj * SCP_PARAM_STRIDE; k += nt) prm[(size_t)r.traj_first * SCP_PARAM_STRIDE + k] = s_prm[k];
    for (int k = tid; k < r.n_nodes; k += nt) node_traj[r.node_off + k] = s_nt[k];
    for (int k = tid; k < r.n_wg * block; k += nt) lane[(size_t)r.wg_first * block + k] = s_lane[k];
    for (int k = tid; k < r.n_wg; k += nt) wi[r.wg_first + k] = s_wi[k];
    for (int k = tid; k < 2 * r.n_wg; k += nt) wg[2 * r.wg_first + k] = s_wg[k];
    for (int k = tid; k < r.n_traj * SCP_INFO_FIELDS; k += nt) dv.info[(size_t)r.traj_first * SCP_INFO_FIELDS + k] = 0.0;
    for (int k = tid; k < r.n_traj * FL_FIELDS; k += nt) dv.flags[(size_t)r.traj_first * FL_FIELDS + k] = 0;
    for (int k = tid; k < r.n_traj * 2; k += nt) dv.red[(size_t)r.traj_first * 2 + k] = 0ull;
    for (int k = tid; k < r.n_traj; k += nt) {
        dv.rt[(size_t)(r.traj_first + k) * RT_FIELDS + RT_DELTA] = s_prm[(size_t)k * SCP_PARAM_STRIDE + SCP_P_DELTA];
        dv.rt[(size_t)(r.traj_first + k) * RT_FIELDS + RT_RHOS] = T(0);
        dv.rt[(size_t)(r.traj_first + k) * RT_FIELDS + RT_RP0] = T(0);
        dv.rt[(size_t)(r.traj_first + k) * RT_FIELDS + RT_RPMAX] = T(0);
    }
    T* pl = dv.planes;
    if (!r.warm) {
        const T* xg = reinterpret_cast<const T*>(blob + r.o_xg);
        const T* ug = reinterpret_cast<const T*>(blob + r.o_ug);
        for (int k = tid; k < r.n_nodes; k += nt) {
            const size_t g = (size_t)r.node_off + k;
            for (int c = 0; c < SCP_MAX_NX; ++c) {
                pl[(size_t)(PL_XBAR + c) * P + g] = xg[(size_t)k * SCP_MAX_NX + c];
                pl[(size_t)(PL_LAM + c) * P + g] = T(0);
                pl[(size_t)(PL_MU + c) * P + g] = T(0);
            }
            for (int c = 0; c < SCP_MAX_NU; ++c) pl[(size_t)(PL_UBAR + c) * P + g] = ug[(size_t)k * SCP_MAX_NU + c];
            for (int c = 0; c < MAX_C; ++c) pl[(size_t)(PL_DU + c) * P + g] = T(0);
        }
        return;
    }
    // warm start: every scenario starts at the previous scenario-0 state at node 1, unless the
    // request brings its own (measured) initial state
    if (!r.keep_xinit) {
        __shared__ T x1[SCP_MAX_NX];
        if (tid < SCP_MAX_NX) x1[tid] = pl[(size_t)(PL_XBAR + tid) * P + r.x1_node];
        __syncthreads();
        for (int k = tid; k < r.n_traj * SCP_MAX_NX; k += nt)
            prm[(size_t)(r.traj_first + k / SCP_MAX_NX) * SCP_PARAM_STRIDE + SCP_P_XINIT + k % SCP_MAX_NX] =
                x1[k % SCP_MAX_NX];
    }
    shift_admission<T>(pl, P, r.node_off, r.n_nodes, r.traj_first, s_nt, s_traj);
}

template <class T>
__global__ void k_collect(Dev<T> dv, const CollectRec* __restrict__ recs, unsigned char* __restrict__ out) {
    const CollectRec r = recs[blockIdx.x];
    const int tid = threadIdx.x, nt = blockDim.x;
    double* info = reinterpret_cast<double*>(out + r.o_out);
    for (int k = tid; k < r.n_traj * SCP_INFO_FIELDS; k += nt) info[k] = dv.info[(size_t)r.traj_first * SCP_INFO_FIELDS + k];
    T* xo = reinterpret_cast<T*>(info + (size_t)r.n_traj * SCP_INFO_FIELDS);
    T* uo = xo + (size_t)r.n_nodes * SCP_MAX_NX;
    const int P = dv.P;
    for (int k = tid; k < r.n_nodes; k += nt) {
        const size_t g = (size_t)r.node_off + k;
        for (int c = 0; c < SCP_MAX_NX; ++c) xo[(size_t)k * SCP_MAX_NX + c] = dv.planes[(size_t)(PL_XBAR + c) * P + g];
        for (int c = 0; c < SCP_MAX_NU; ++c) uo[(size_t)k * SCP_MAX_NU + c] = dv.planes[(size_t)(PL_UBAR + c) * P + g];
    }
}

template <class T>
hipError_t launch_admit(const Dev<T>& dv, int block, const unsigned char* blob, int rec_off, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_admit<T>, dim3(n), dim3(256), 0, s, dv, block, blob, rec_off);
    return hipGetLastError();
}

template <class T>
hipError_t launch_collect(const Dev<T>& dv, const CollectRec* recs, int n, unsigned char* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_collect<T>, dim3(n), dim3(256), 0, s, dv, recs, out);
    return hipGetLastError();
}

template hipError_t launch_admit<float>(const Dev<float>&, int, const unsigned char*, int, int, hipStream_t);
template hipError_t launch_admit<double>(const Dev<double>&, int, const unsigned char*, int, int, hipStream_t);
template hipError_t launch_collect<float>(const Dev<float>&, const CollectRec*, int, unsigned char*, hipStream_t);
template hipError_t launch_collect<double>(const Dev<double>&, const CollectRec*, int, unsigned char*, hipStream_t);

}  // namespace scp

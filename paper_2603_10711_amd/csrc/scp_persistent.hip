// Persistent form: launch entry (the kernel templates live in scp_persistent.hpp; their
// instantiations are split over scp_persistent_{f32,f64}{,_span,_adapt,_track}.hip).
#include "scp_persistent.hpp"
#include "scp_host.hpp"

namespace scp {

#define SCP_EXTERN_VARIANTS(T, SPAN)                                                                        \
    extern template void launch_models<T, 64, SPAN>(const Dev<T>&, const KParams<T>&, int, int, int, hipStream_t); \
    extern template void launch_models<T, 128, SPAN>(const Dev<T>&, const KParams<T>&, int, int, int, hipStream_t);
SCP_EXTERN_VARIANTS(float, false)
SCP_EXTERN_VARIANTS(float, true)
SCP_EXTERN_VARIANTS(double, false)
SCP_EXTERN_VARIANTS(double, true)
extern template void launch_models<float, 256, false>(const Dev<float>&, const KParams<float>&, int, int, int, hipStream_t);
extern template void launch_models<float, 256, true>(const Dev<float>&, const KParams<float>&, int, int, int, hipStream_t);
#define SCP_EXTERN_ADAPT(T, BLOCK) \
    extern template void launch_models<T, BLOCK, false, true>(const Dev<T>&, const KParams<T>&, int, int, int, hipStream_t);
SCP_EXTERN_ADAPT(float, 64)
SCP_EXTERN_ADAPT(float, 128)
SCP_EXTERN_ADAPT(float, 256)
SCP_EXTERN_ADAPT(double, 64)
SCP_EXTERN_ADAPT(double, 128)
#undef SCP_EXTERN_ADAPT
#define SCP_EXTERN_TRACK(T, BLOCK) \
    extern template void launch_models<T, BLOCK, false, false, true>(const Dev<T>&, const KParams<T>&, int, int, int, hipStream_t);
SCP_EXTERN_TRACK(float, 64)
SCP_EXTERN_TRACK(float, 128)
SCP_EXTERN_TRACK(float, 256)
SCP_EXTERN_TRACK(double, 64)
SCP_EXTERN_TRACK(double, 128)
#undef SCP_EXTERN_TRACK
#undef SCP_EXTERN_VARIANTS

// Barrier counters of the spanning groups start every launch at zero.
__global__ void k_zero_sync(unsigned* __restrict__ c, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = 0u;
}

template <class T, int BLOCK>
static hipError_t launch_block(const Dev<T>& dv, const KParams<T>& kp, int n_wg, int models, int kmax,
                               hipStream_t s) {
    if (kp.adapt_mu > 0.0) {   // no consensus groups with the adaptive penalty (refused on the host)
        if (dv.n_gslots > 0) return hipErrorInvalidValue;
        launch_models<T, BLOCK, false, true>(dv, kp, n_wg, models, kmax, s);
    } else if (dv.n_gslots > 0) {
        launch_models<T, BLOCK, true>(dv, kp, n_wg, models, kmax, s);
    } else if (kp.blowup) {
        launch_models<T, BLOCK, false, false, true>(dv, kp, n_wg, models, kmax, s);
    } else {
        launch_models<T, BLOCK, false>(dv, kp, n_wg, models, kmax, s);
    }
    return hipGetLastError();
}

template <class T>
hipError_t launch_persistent(const Dev<T>& dv, const KParams<T>& kp, int n_wg, int block, int models, int kmax,
                             hipStream_t s) {
    if (n_wg <= 0) return hipSuccess;
    if (models & ~3) return hipErrorInvalidValue;  // point-mass quadrotor and powered descent only
    if (dv.n_gslots > 0) {
        const int n = dv.n_gslots * GX_SYNC_STRIDE;
        hipLaunchKernelGGL(k_zero_sync, dim3((n + 255) / 256), dim3(256), 0, s, dv.gsync, n);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    switch (block) {
        case 64: return launch_block<T, 64>(dv, kp, n_wg, models, kmax, s);
        case 128: return launch_block<T, 128>(dv, kp, n_wg, models, kmax, s);
        case 256:
            // FP64 state of a 256-lane workgroup does not fit the 160 KB of LDS
            if constexpr (sizeof(T) == 4) return launch_block<T, 256>(dv, kp, n_wg, models, kmax, s);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

template <class T>
static size_t shared_bytes(int block) {
    constexpr int HSR = 3 * 8;  // quadrotor kernels with 8 obstacles: the largest state
    switch (block) {
        case 64: return sizeof(Shared<T, 64, HSR, persistent_lds_factor_rows(64, 3)>);
        case 128: return sizeof(Shared<T, 128, HSR, persistent_lds_factor_rows(128, 3)>);
        case 256: return sizeof(Shared<T, 256, HSR, persistent_lds_factor_rows(256, 3)>);
        default: return 0;
    }
}

size_t persistent_shared_bytes(int esz, int block) {
    return esz == 4 ? shared_bytes<float>(block) : shared_bytes<double>(block);
}

int span_blocks_per_cu_f32(int block, int models, int kmax);
int span_blocks_per_cu_f64(int block, int models, int kmax);

int persistent_span_resident_cap(int esz, int block, int models, int kmax) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const int per_cu = esz == 4 ? span_blocks_per_cu_f32(block, models, kmax) : span_blocks_per_cu_f64(block, models, kmax);
    return per_cu * cus;
}

template hipError_t launch_persistent<float>(const Dev<float>&, const KParams<float>&, int, int, int, int, hipStream_t);
template hipError_t launch_persistent<double>(const Dev<double>&, const KParams<double>&, int, int, int, int, hipStream_t);

}  // namespace scp

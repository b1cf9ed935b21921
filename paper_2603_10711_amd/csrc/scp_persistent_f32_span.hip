// Persistent kernel instantiations: float, launches with consensus groups spanning workgroups.
#include "scp_persistent.hpp"

namespace scp {

template void launch_models<float, 64, true>(const Dev<float>&, const KParams<float>&, int, int, int,
                                                   hipStream_t);
template void launch_models<float, 128, true>(const Dev<float>&, const KParams<float>&, int, int, int,
                                                   hipStream_t);
template void launch_models<float, 256, true>(const Dev<float>&, const KParams<float>&, int, int, int,
                                                   hipStream_t);

int span_blocks_per_cu_f32(int block, int models, int kmax) {
    switch (block) {
        case 64: return span_blocks_per_cu<float, 64>(models, kmax);
        case 128: return span_blocks_per_cu<float, 128>(models, kmax);
        case 256: return span_blocks_per_cu<float, 256>(models, kmax);
        default: return 0;
    }
}

}  // namespace scp

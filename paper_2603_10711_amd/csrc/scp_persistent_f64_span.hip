// Persistent kernel instantiations: double, launches with consensus groups spanning workgroups.
#include "scp_persistent.hpp"

namespace scp {

template void launch_models<double, 64, true>(const Dev<double>&, const KParams<double>&, int, int, int,
                                                   hipStream_t);
template void launch_models<double, 128, true>(const Dev<double>&, const KParams<double>&, int, int, int,
                                                   hipStream_t);

int span_blocks_per_cu_f64(int block, int models, int kmax) {
    switch (block) {
        case 64: return span_blocks_per_cu<double, 64>(models, kmax);
        case 128: return span_blocks_per_cu<double, 128>(models, kmax);
        default: return 0;
    }
}

}  // namespace scp

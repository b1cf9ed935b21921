// Persistent kernel instantiations: float, launches with consensus groups spanning workgroups.
#include "scp_persistent.hpp"

namespace scp {

template void launch_models<float, 64, true>(const Dev<float>&, const KParams<float>&, int, int, int,
                                                   hipStream_t);
template void launch_models<float, 128, true>(const Dev<float>&, const KParams<float>&, int, int, int,
                                                   hipStream_t);
template void launch_models<float, 256, true>(const Dev<float>&, const KParams<float>&, int, int, int,
                                                   hipStream_t);

}  // namespace scp

// Persistent kernel instantiations: float, launches with residual blow-up detection (no spanning
// groups, fixed penalties).
#include "scp_persistent.hpp"

namespace scp {

template void launch_models<float, 64, false, false, true>(const Dev<float>&, const KParams<float>&, int, int,
                                                         int, hipStream_t);
template void launch_models<float, 128, false, false, true>(const Dev<float>&, const KParams<float>&, int, int,
                                                         int, hipStream_t);
template void launch_models<float, 256, false, false, true>(const Dev<float>&, const KParams<float>&, int, int,
                                                         int, hipStream_t);

}  // namespace scp

// Persistent kernel instantiations: float, launches with the adaptive penalty (no spanning groups).
#include "scp_persistent.hpp"

namespace scp {

template void launch_models<float, 64, false, true>(const Dev<float>&, const KParams<float>&, int, int, int,
                                                      hipStream_t);
template void launch_models<float, 128, false, true>(const Dev<float>&, const KParams<float>&, int, int, int,
                                                      hipStream_t);
template void launch_models<float, 256, false, true>(const Dev<float>&, const KParams<float>&, int, int, int,
                                                      hipStream_t);

}  // namespace scp

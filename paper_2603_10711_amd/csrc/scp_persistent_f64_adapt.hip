// Persistent kernel instantiations: double, launches with the adaptive penalty (no spanning groups).
#include "scp_persistent.hpp"

namespace scp {

template void launch_models<double, 64, false, true>(const Dev<double>&, const KParams<double>&, int, int, int,
                                                      hipStream_t);
template void launch_models<double, 128, false, true>(const Dev<double>&, const KParams<double>&, int, int, int,
                                                      hipStream_t);

}  // namespace scp

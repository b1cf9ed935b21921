// Persistent kernel instantiations: double, launches with consensus groups spanning workgroups.
#include "scp_persistent.hpp"

namespace scp {

template void launch_models<double, 64, true>(const Dev<double>&, const KParams<double>&, int, int, int,
                                                   hipStream_t);
template void launch_models<double, 128, true>(const Dev<double>&, const KParams<double>&, int, int, int,
                                                   hipStream_t);

}  // namespace scp

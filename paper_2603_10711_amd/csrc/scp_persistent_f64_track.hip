// Persistent kernel instantiations: double, launches with residual blow-up detection (no spanning
// groups, fixed penalties).
#include "scp_persistent.hpp"

namespace scp {

template void launch_models<double, 64, false, false, true>(const Dev<double>&, const KParams<double>&, int, int,
                                                         int, hipStream_t);
template void launch_models<double, 128, false, false, true>(const Dev<double>&, const KParams<double>&, int, int,
                                                         int, hipStream_t);

}  // namespace scp

// Persistent kernel instantiations: double, launches without spanning groups.
#include "scp_persistent.hpp"

namespace scp {

template void launch_models<double, 64, false>(const Dev<double>&, const KParams<double>&, int, int, int,
                                                   hipStream_t);
template void launch_models<double, 128, false>(const Dev<double>&, const KParams<double>&, int, int, int,
                                                   hipStream_t);

}  // namespace scp

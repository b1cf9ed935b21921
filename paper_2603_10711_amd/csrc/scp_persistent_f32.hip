// Persistent kernel instantiations: float, launches without spanning groups.
#include "scp_persistent.hpp"

namespace scp {

template void launch_models<float, 64, false>(const Dev<float>&, const KParams<float>&, int, int, int,
                                                   hipStream_t);
template void launch_models<float, 128, false>(const Dev<float>&, const KParams<float>&, int, int, int,
                                                   hipStream_t);
template void launch_models<float, 256, false>(const Dev<float>&, const KParams<float>&, int, int, int,
                                                   hipStream_t);

}  // namespace scp

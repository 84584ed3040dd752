// Instantiations of the fused forward kernel (see fwd_kernel.h), one file per group so
// that they compile in parallel: pipelined stages, non-temporal table loads.
#include "fwd_kernel.h"

namespace bm {
template int launch_k_forward<float, 8, true, 2>(const HostPlan&, const LaunchPlan&, size_t, char*,
                                                   const int32_t*, double*, double*, double*, const int32_t*,
                                                   const int32_t*, int, hipStream_t,
                                                   hipEvent_t, hipEvent_t);
}  // namespace bm

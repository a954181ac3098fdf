// Conic step for cliques larger than the LDS Jacobi kernel handles.
#include "device.h"

namespace cdcs {

void launch_cone_large(const DevPlan&, const int32_t*, const int32_t*, int32_t, int32_t, hipStream_t) {}
void launch_psd_project_large(const int32_t*, const int64_t*, const int32_t*, const int32_t*, int32_t, int32_t,
                              const double*, double*, double*, const int64_t*, hipStream_t) {}

}  // namespace cdcs

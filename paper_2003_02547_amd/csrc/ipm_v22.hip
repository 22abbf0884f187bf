// Explicit instantiations of ipm_kernel variants (one of several units
// compiled in parallel).
#include "ipm_kernel.h"

namespace oqp {
template void launch_ipm<24, 8, 0, KM_F64>(const InstDesc*, int, const double*, double*, double*, double*, DevStat*, KParams, hipStream_t);
template void launch_ipm<24, 8, 0, KM_MIXED>(const InstDesc*, int, const double*, double*, double*, double*, DevStat*, KParams, hipStream_t);
template void launch_ipm<24, 8, 0, KM_ABS>(const InstDesc*, int, const double*, double*, double*, double*, DevStat*, KParams, hipStream_t);
}  // namespace oqp

// Explicit instantiations of ipm_kernel variants, balance mode (checked Cholesky, array-algorithm fallback)
// (one of several units compiled in parallel).
#include "ipm_kernel.h"

namespace oqp {
template void launch_ipm<8, 16, 0, KM_BALANCE>(const InstDesc*, int, const double*, double*, double*, double*, DevStat*, KParams, hipStream_t);
}  // namespace oqp

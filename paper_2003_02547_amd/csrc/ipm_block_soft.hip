// Instantiations of the block kernel with soft constraints (Section 2.2):
// FP64 delta formulation on the soft layout, for every stage-block bound,
// without and with general rows.
#include "ipm_block.h"
#include "ipm_launch.h"

namespace oqp {

int block_launch_soft(int zm, int gm, const InstDesc* desc, int count, const double* data, double* iter,
                      double* work, double* step, DevStat* stat, const KParams& P, size_t lds_bytes, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (zm == 64 && gm == 64 && lds_bytes > 80 * 1024) {  // one workgroup per CU: the build that spills nothing
        hipLaunchKernelGGL((ipm_block_kernel<KM_SOFT, 64, 64, 1>), dim3(count), dim3(BT), lds_bytes, s, desc, count,
                           data, iter, work, step, stat, P);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
#define OQP_BLK_SOFT(Z, G)                                                                                          \
    if (zm == Z && gm == G) {                                                                                       \
        hipLaunchKernelGGL((ipm_block_kernel<KM_SOFT, Z, G>), dim3(count), dim3(BT), lds_bytes, s, desc, count,    \
                           data, iter, work, step, stat, P);                                                        \
        return hipGetLastError() == hipSuccess ? 0 : -1;                                                            \
    }
    OQP_BLK_SOFT(32, 0)
    OQP_BLK_SOFT(32, 64)
    OQP_BLK_SOFT(64, 0)
    OQP_BLK_SOFT(64, 64)
    OQP_BLK_SOFT(256, 0)
    OQP_BLK_SOFT(256, 64)
#undef OQP_BLK_SOFT
    return -1;
}

}  // namespace oqp

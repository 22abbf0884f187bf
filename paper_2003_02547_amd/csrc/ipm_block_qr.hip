// Instantiations of the block kernel with the array algorithm of Section 4.2:
// mode robust (every iteration) and mode balance (Cholesky factors checked,
// the array algorithm when the check fails), FP64, for every stage-block
// bound, without and with general rows.
#include "ipm_block.h"
#include "ipm_launch.h"

namespace oqp {

template <int KM>
static int launch_qr_t(int zm, int gm, const InstDesc* desc, int count, const double* data, double* iter,
                       double* work, double* step, DevStat* stat, const KParams& P, size_t lds_bytes,
                       hipStream_t s)
{
    if (zm == 64 && gm == 64 && lds_bytes > 80 * 1024) {  // one workgroup per CU: the build that spills nothing
        hipLaunchKernelGGL((ipm_block_kernel<KM, 64, 64, 1>), dim3(count), dim3(BT), lds_bytes, s, desc, count, data,
                           iter, work, step, stat, P);
        return hipGetLastError() == hipSuccess ? 0 : -1;
    }
#define OQP_BLK_QR(Z, G)                                                                                            \
    if (zm == Z && gm == G) {                                                                                       \
        hipLaunchKernelGGL((ipm_block_kernel<KM, Z, G>), dim3(count), dim3(BT), lds_bytes, s, desc, count, data,    \
                           iter, work, step, stat, P);                                                              \
        return hipGetLastError() == hipSuccess ? 0 : -1;                                                            \
    }
    OQP_BLK_QR(32, 0)
    OQP_BLK_QR(32, 64)
    OQP_BLK_QR(64, 0)
    OQP_BLK_QR(64, 64)
    OQP_BLK_QR(256, 0)
    OQP_BLK_QR(256, 64)
#undef OQP_BLK_QR
    return -1;
}

int block_launch_qr(int zm, int gm, int km, const InstDesc* desc, int count, const double* data, double* iter,
                    double* work, double* step, DevStat* stat, const KParams& P, size_t lds_bytes, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    if (km == KM_ROBUST)
        return launch_qr_t<KM_ROBUST>(zm, gm, desc, count, data, iter, work, step, stat, P, lds_bytes, s);
    if (km == KM_BALANCE)
        return launch_qr_t<KM_BALANCE>(zm, gm, desc, count, data, iter, work, step, stat, P, lds_bytes, s);
    return -1;
}

}  // namespace oqp

// Instantiations of the block kernel: FP64 and mixed, for stage blocks up to
// 32 and up to 64 (LDS-resident stage blocks, the bound sizes the prefetch
// registers), and above 64 (global-memory mode), each without and with
// general rows.
#include "ipm_block.h"
#include "ipm_launch.h"

namespace oqp {

// LDS above half of a CU's 160 KB: one workgroup per CU whatever the
// register budget
static constexpr size_t kLdsHalfCU = 80 * 1024;

template <int KM, int ZM, int GM>
static int launch_block_t(const InstDesc* desc, int count, const double* data, double* iter, double* work,
                          double* step, DevStat* stat, const KParams& P, size_t lds_bytes, hipStream_t stream)
{
    if constexpr (ZM == 64 && GM == 64) {
        if (lds_bytes > kLdsHalfCU) {
            hipLaunchKernelGGL((ipm_block_kernel<KM, ZM, GM, 1>), dim3(count), dim3(BT), lds_bytes, stream, desc,
                               count, data, iter, work, step, stat, P);
            return hipGetLastError() == hipSuccess ? 0 : -1;
        }
    }
    hipLaunchKernelGGL((ipm_block_kernel<KM, ZM, GM>), dim3(count), dim3(BT), lds_bytes, stream, desc, count, data,
                       iter, work, step, stat, P);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int block_lds_bytes(int nx, int nu, int ng) { return (int)(sizeof(double) * make_blds(nx, nu, ng).total); }

int block_zmax(int nz) { return nz <= 32 ? 32 : (nz <= 64 ? 64 : (nz <= 256 ? 256 : 0)); }

int block_launch(int zm, int gm, int km, const InstDesc* desc, int count, const double* data, double* iter,
                 double* work, double* step, DevStat* stat, const KParams& P, size_t lds_bytes, void* stream)
{
    if (km == KM_SOFT) return block_launch_soft(zm, gm, desc, count, data, iter, work, step, stat, P, lds_bytes, stream);
    if (km == KM_ROBUST || km == KM_BALANCE)
        return block_launch_qr(zm, gm, km, desc, count, data, iter, work, step, stat, P, lds_bytes, stream);
    hipStream_t s = (hipStream_t)stream;
#define OQP_BLK(Z, G)                                                                                             \
    if (zm == Z && gm == G) {                                                                                       \
        if (km == KM_MIXED) return launch_block_t<KM_MIXED, Z, G>(desc, count, data, iter, work, step, stat, P,   \
                                                                  lds_bytes, s);                                    \
        if (km == KM_ABS) return launch_block_t<KM_ABS, Z, G>(desc, count, data, iter, work, step, stat, P,       \
                                                              lds_bytes, s);                                        \
        if (km == KM_F64) return launch_block_t<KM_F64, Z, G>(desc, count, data, iter, work, step, stat, P,       \
                                                              lds_bytes, s);                                        \
        return -1;                                                                                                  \
    }
    OQP_BLK(32, 0)
    OQP_BLK(32, 64)
    OQP_BLK(64, 0)
    OQP_BLK(64, 64)
    OQP_BLK(256, 0)
    OQP_BLK(256, 64)
#undef OQP_BLK
    return -1;
}

}  // namespace oqp

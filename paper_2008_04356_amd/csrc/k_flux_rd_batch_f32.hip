// Instantiations of the batched register-direct kernel (FP32, degrees N = 3, 5, 7).
#include "k_flux_rd.h"

namespace mortar {

template <bool NSV, int RIEM>
static int rd_batch_occ1()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void *>(&k_mortar_flux_rd_batch<NSV, RIEM>), 64 * kRdBatchWaves, 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

int flux_rd_batch_occupancy_f32(bool ns, int riem)
{
    if (ns) return riem ? rd_batch_occ1<true, 1>() : rd_batch_occ1<true, 0>();
    return riem ? rd_batch_occ1<false, 1>() : rd_batch_occ1<false, 0>();
}

hipError_t launch_flux_rd_batch_f32(const BatchArgs<float> &b, int grid, bool ns, int riem,
                                    hipStream_t st)
{
    if (ns) {
        if (riem) hipLaunchKernelGGL((k_mortar_flux_rd_batch<true, 1>), dim3(grid), dim3(64 * kRdBatchWaves), 0, st, b);
        else hipLaunchKernelGGL((k_mortar_flux_rd_batch<true, 0>), dim3(grid), dim3(64 * kRdBatchWaves), 0, st, b);
    } else {
        if (riem) hipLaunchKernelGGL((k_mortar_flux_rd_batch<false, 1>), dim3(grid), dim3(64 * kRdBatchWaves), 0, st, b);
        else hipLaunchKernelGGL((k_mortar_flux_rd_batch<false, 0>), dim3(grid), dim3(64 * kRdBatchWaves), 0, st, b);
    }
    return hipGetLastError();
}

}  // namespace mortar

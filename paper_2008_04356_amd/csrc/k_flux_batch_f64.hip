// Instantiations of the batched mortar-flux kernel for element type double.
#include "k_flux.h"

namespace mortar {

constexpr int kLdsBudget = lds_budget<double>();

// Batched kernel: several interfaces of one element type, physics and flux in one launch.
template <bool NSV, int RIEM, int MASK>
static hipError_t go_batch(const BatchArgs<double> &b, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((k_mortar_flux_batch<double, NSV, RIEM, kLdsBudget, MASK>), dim3(grid),
                       dim3(kFluxThreads), 0, st, b);
    return hipGetLastError();
}

template <bool NSV, int RIEM, int MASK>
static int occ_batch()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void *>(&k_mortar_flux_batch<double, NSV, RIEM, kLdsBudget, MASK>),
            kFluxThreads, 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

// turbine: the degree set N = 3, 5, 7 (only instantiated for NS + Roe)
hipError_t launch_flux_batch_f64(const BatchArgs<double> &b, int grid, bool ns, int riem, bool turbine,
                                 hipStream_t st)
{
    if (turbine && ns && riem) return go_batch<true, 1, kMaskTurbine>(b, grid, st);
    if (ns) return riem ? go_batch<true, 1, kMaskAll>(b, grid, st) : go_batch<true, 0, kMaskAll>(b, grid, st);
    return riem ? go_batch<false, 1, kMaskAll>(b, grid, st) : go_batch<false, 0, kMaskAll>(b, grid, st);
}

int flux_batch_occupancy_f64(bool ns, int riem, bool turbine)
{
    if (turbine && ns && riem) return occ_batch<true, 1, kMaskTurbine>();
    if (ns) return riem ? occ_batch<true, 1, kMaskAll>() : occ_batch<true, 0, kMaskAll>();
    return riem ? occ_batch<false, 1, kMaskAll>() : occ_batch<false, 0, kMaskAll>();
}

}  // namespace mortar

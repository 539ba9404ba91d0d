// Instantiations of the VALU mortar-flux kernel, element type double, 80 KB of LDS per
// workgroup (two workgroups per CU).
#include "k_flux_valu_launch.h"

namespace mortar {

using L = ValuLaunch<double, lds_budget<double>()>;

// degrees above kMaxNFast: instantiated in k_flux_hi_f64.hip
int flux_occupancy_hi_f64(int NP, bool ns, bool met, int riem);
int flux_tile_capacity_hi_f64(int NP, bool ns, bool met);
hipError_t launch_flux_hi_f64(const FluxArgs<double> &a, int NP, int grid, bool ns, bool met, int riem,
                             hipStream_t st);

int flux_occupancy_f64(int NP, bool ns, bool met, int riem)
{
    return NP > kMaxNFast + 1 ? flux_occupancy_hi_f64(NP, ns, met, riem) : L::occupancy(NP, ns, met, riem);
}
int flux_tile_capacity_f64(int NP, bool ns, bool met)
{
    return NP > kMaxNFast + 1 ? flux_tile_capacity_hi_f64(NP, ns, met) : L::capacity(NP, ns, met);
}
hipError_t launch_flux_f64(const FluxArgs<double> &a, int NP, int grid, bool ns, bool met, int riem,
                           hipStream_t st)
{
    if (NP > kMaxNFast + 1) return launch_flux_hi_f64(a, NP, grid, ns, met, riem, st);
    return L::launch(a, NP, grid, ns, met, riem, st);
}

}  // namespace mortar

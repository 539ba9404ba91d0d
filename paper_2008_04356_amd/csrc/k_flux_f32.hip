// Instantiations of the VALU mortar-flux kernel, element type float, 48 KB of LDS per
// workgroup (three workgroups per CU).
#include "k_flux_valu_launch.h"

namespace mortar {

using L = ValuLaunch<float, lds_budget<float>()>;

// degrees above kMaxNFast: instantiated in k_flux_hi_f32.hip
int flux_occupancy_hi_f32(int NP, bool ns, bool met, int riem);
int flux_tile_capacity_hi_f32(int NP, bool ns, bool met);
hipError_t launch_flux_hi_f32(const FluxArgs<float> &a, int NP, int grid, bool ns, bool met, int riem,
                             hipStream_t st);

int flux_occupancy_f32(int NP, bool ns, bool met, int riem)
{
    return NP > kMaxNFast + 1 ? flux_occupancy_hi_f32(NP, ns, met, riem) : L::occupancy(NP, ns, met, riem);
}
int flux_tile_capacity_f32(int NP, bool ns, bool met)
{
    return NP > kMaxNFast + 1 ? flux_tile_capacity_hi_f32(NP, ns, met) : L::capacity(NP, ns, met);
}
hipError_t launch_flux_f32(const FluxArgs<float> &a, int NP, int grid, bool ns, bool met, int riem,
                           hipStream_t st)
{
    if (NP > kMaxNFast + 1) return launch_flux_hi_f32(a, NP, grid, ns, met, riem, st);
    return L::launch(a, NP, grid, ns, met, riem, st);
}

}  // namespace mortar

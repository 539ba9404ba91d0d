// Instantiations of the VALU mortar-flux kernel for the high degrees (N = 10..15),
// element type float, 48 KB of LDS per
// workgroup; the only flux kernel of those degrees.
#include "k_flux_valu_launch.h"

namespace mortar {

using LH = ValuLaunch<float, lds_budget<float>(), kMaxNFast + 2, kMaxNP>;

int flux_occupancy_hi_f32(int NP, bool ns, bool met, int riem) { return LH::occupancy(NP, ns, met, riem); }
int flux_tile_capacity_hi_f32(int NP, bool ns, bool met) { return LH::capacity(NP, ns, met); }
hipError_t launch_flux_hi_f32(const FluxArgs<float> &a, int NP, int grid, bool ns, bool met, int riem,
                             hipStream_t st)
{
    return LH::launch(a, NP, grid, ns, met, riem, st);
}

}  // namespace mortar

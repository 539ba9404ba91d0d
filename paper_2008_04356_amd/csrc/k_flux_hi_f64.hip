// Instantiations of the VALU mortar-flux kernel for the high degrees (N = 10..15),
// element type double, 80 KB of LDS per
// workgroup; the only flux kernel of those degrees.
#include "k_flux_valu_launch.h"

namespace mortar {

using LH = ValuLaunch<double, lds_budget<double>(), kMaxNFast + 2, kMaxNP>;

int flux_occupancy_hi_f64(int NP, bool ns, bool met, int riem) { return LH::occupancy(NP, ns, met, riem); }
int flux_tile_capacity_hi_f64(int NP, bool ns, bool met) { return LH::capacity(NP, ns, met); }
hipError_t launch_flux_hi_f64(const FluxArgs<double> &a, int NP, int grid, bool ns, bool met, int riem,
                             hipStream_t st)
{
    return LH::launch(a, NP, grid, ns, met, riem, st);
}

}  // namespace mortar

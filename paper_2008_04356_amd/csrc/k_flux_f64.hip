// Instantiations of the VALU mortar-flux kernel, element type double, 80 KB of LDS per
// workgroup (two workgroups per CU).
#include "k_flux_valu_launch.h"

namespace mortar {

using L = ValuLaunch<double, lds_budget<double>()>;

int flux_occupancy_f64(int NP, bool ns, bool met, int riem) { return L::occupancy(NP, ns, met, riem); }
int flux_tile_capacity_f64(int NP, bool ns, bool met) { return L::capacity(NP, ns, met); }
hipError_t launch_flux_f64(const FluxArgs<double> &a, int NP, int grid, bool ns, bool met, int riem,
                           hipStream_t st)
{
    return L::launch(a, NP, grid, ns, met, riem, st);
}

}  // namespace mortar

// Instantiations of the register-direct mortar-flux kernel: FP32 data, FP32 matrix cores.
#include "k_flux_rd.h"

namespace mortar {

int flux_rd_occupancy_f32(int NP, bool ns, bool met, int riem)
{
#define E(np) rd_occ<float, np, 0>(ns, met, riem)
    MORTAR_RD_NP_SWITCH(E, 1)
#undef E
}

hipError_t launch_flux_rd_f32(const FluxArgs<float> &a, int NP, int grid, bool ns, bool met,
                              int riem, hipStream_t st)
{
#define E(np) rd_pick<float, np, 0>(a, grid, ns, met, riem, st)
    MORTAR_RD_NP_SWITCH(E, hipErrorInvalidValue)
#undef E
}

}  // namespace mortar

// Instantiations of the register-direct BR1 lifting kernel: FP32 data, FP32 matrix cores.
#include "k_flux_rd.h"

namespace mortar {

int lift_rd_occupancy_f32(int NP, bool met)
{
#define E(np) rd_lift_occ<float, np>(met)
    MORTAR_RD_NP_SWITCH(E, 1)
#undef E
}

hipError_t launch_lift_rd_f32(const FluxArgs<float> &a, int NP, int grid, bool met, hipStream_t st)
{
#define E(np) rd_lift_go<float, np>(a, grid, met, st)
    MORTAR_RD_NP_SWITCH(E, hipErrorInvalidValue)
#undef E
}

}  // namespace mortar

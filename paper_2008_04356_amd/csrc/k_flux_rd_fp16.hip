// Instantiations of the register-direct mortar-flux kernel with fp16 GEMM operands
// (FP32 data and accumulation, conservation-corrected back projection).
#include "k_flux_rd.h"

namespace mortar {

int flux_rd_occupancy_fp16(int NP, bool ns, bool met, int riem)
{
#define E(np) rd_occ<float, np, 2>(ns, met, riem)
    MORTAR_RD_NP_SWITCH(E, 1)
#undef E
}

hipError_t launch_flux_rd_fp16(const FluxArgs<float> &a, int NP, int grid, bool ns, bool met,
                               int riem, hipStream_t st)
{
#define E(np) rd_pick<float, np, 2>(a, grid, ns, met, riem, st)
    MORTAR_RD_NP_SWITCH(E, hipErrorInvalidValue)
#undef E
}

}  // namespace mortar

// Instantiations of the mortar-flux kernel with matrix-core projections (FP32).
#include "k_flux_hyb.h"

namespace mortar {

namespace {

template <int NP, bool NSV, bool MET, int RIEM>
hipError_t hyb_go(const FluxArgs<float> &a, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((k_mortar_flux_hyb<NP, NSV, MET, RIEM>), dim3(grid), dim3(kFluxThreads), 0, st, a);
    return hipGetLastError();
}

template <int NP>
hipError_t hyb_pick(const FluxArgs<float> &a, int grid, bool ns, bool met, int riem, hipStream_t st)
{
    if (ns) {
        if (met) return riem ? hyb_go<NP, true, true, 1>(a, grid, st) : hyb_go<NP, true, true, 0>(a, grid, st);
        return riem ? hyb_go<NP, true, false, 1>(a, grid, st) : hyb_go<NP, true, false, 0>(a, grid, st);
    }
    if (met) return riem ? hyb_go<NP, false, true, 1>(a, grid, st) : hyb_go<NP, false, true, 0>(a, grid, st);
    return riem ? hyb_go<NP, false, false, 1>(a, grid, st) : hyb_go<NP, false, false, 0>(a, grid, st);
}

template <int NP, bool NSV, bool MET, int RIEM>
int hyb_occ1()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void *>(&k_mortar_flux_hyb<NP, NSV, MET, RIEM>), kFluxThreads, 0) !=
        hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

template <int NP>
int hyb_occ(bool ns, bool met, int riem)
{
    if (ns) {
        if (met) return riem ? hyb_occ1<NP, true, true, 1>() : hyb_occ1<NP, true, true, 0>();
        return riem ? hyb_occ1<NP, true, false, 1>() : hyb_occ1<NP, true, false, 0>();
    }
    if (met) return riem ? hyb_occ1<NP, false, true, 1>() : hyb_occ1<NP, false, true, 0>();
    return riem ? hyb_occ1<NP, false, false, 1>() : hyb_occ1<NP, false, false, 0>();
}

template <int NP>
int hyb_cap(bool ns, bool met)
{
    if (ns) return met ? HybCfg<NP, true, true>::TF : HybCfg<NP, true, false>::TF;
    return met ? HybCfg<NP, false, true>::TF : HybCfg<NP, false, false>::TF;
}

}  // namespace

#define MORTAR_HYB_NP_SWITCH(EXPR, DEFAULT)                                             \
    switch (NP) {                                                                       \
    case 2: return EXPR(2); case 3: return EXPR(3); case 4: return EXPR(4);            \
    case 5: return EXPR(5); case 6: return EXPR(6); case 7: return EXPR(7);            \
    case 8: return EXPR(8); case 9: return EXPR(9); case 10: return EXPR(10);          \
    default: return DEFAULT;                                                            \
    }

int flux_hyb_occupancy_f32(int NP, bool ns, bool met, int riem)
{
#define E(np) hyb_occ<np>(ns, met, riem)
    MORTAR_HYB_NP_SWITCH(E, 1)
#undef E
}

int flux_hyb_tile_capacity_f32(int NP, bool ns, bool met)
{
#define E(np) hyb_cap<np>(ns, met)
    MORTAR_HYB_NP_SWITCH(E, 0)
#undef E
}

hipError_t launch_flux_hyb_f32(const FluxArgs<float> &a, int NP, int grid, bool ns, bool met, int riem,
                               hipStream_t st)
{
#define E(np) hyb_pick<np>(a, grid, ns, met, riem, st)
    MORTAR_HYB_NP_SWITCH(E, hipErrorInvalidValue)
#undef E
}

}  // namespace mortar

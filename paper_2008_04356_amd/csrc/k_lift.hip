// Instantiations of the BR1 lifting surface kernel (VALU projections), FP32 and FP64,
// with the LDS budget of the VALU flux kernel of the same element type.
#include "k_flux.h"

namespace mortar {

namespace {

template <typename T, int NP, bool MET>
hipError_t lift_go(const FluxArgs<T> &a, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((k_mortar_lift<T, NP, MET, lds_budget<T>()>), dim3(grid), dim3(kFluxThreads), 0, st, a);
    return hipGetLastError();
}

template <typename T, int NP, bool MET>
int lift_occ1()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void *>(&k_mortar_lift<T, NP, MET, lds_budget<T>()>), kFluxThreads, 0) !=
        hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

template <typename T, int NP>
int lift_cap(bool met)
{
    return met ? FluxCfg<T, NP, false, true, lds_budget<T>(), true>::TF
               : FluxCfg<T, NP, false, false, lds_budget<T>(), true>::TF;
}

template <typename T>
struct LiftLaunch {
#define MORTAR_LIFT_NP_SWITCH(EXPR, DEFAULT)                                            \
    switch (NP) {                                                                       \
    case 2: return EXPR(2); case 3: return EXPR(3); case 4: return EXPR(4);            \
    case 5: return EXPR(5); case 6: return EXPR(6); case 7: return EXPR(7);            \
    case 8: return EXPR(8); case 9: return EXPR(9); case 10: return EXPR(10);          \
    default: return DEFAULT;                                                            \
    }
    static int occupancy(int NP, bool met)
    {
#define E(np) (met ? lift_occ1<T, np, true>() : lift_occ1<T, np, false>())
        MORTAR_LIFT_NP_SWITCH(E, 1)
#undef E
    }
    static int capacity(int NP, bool met)
    {
#define E(np) lift_cap<T, np>(met)
        MORTAR_LIFT_NP_SWITCH(E, 0)
#undef E
    }
    static hipError_t launch(const FluxArgs<T> &a, int NP, int grid, bool met, hipStream_t st)
    {
#define E(np) (met ? lift_go<T, np, true>(a, grid, st) : lift_go<T, np, false>(a, grid, st))
        MORTAR_LIFT_NP_SWITCH(E, hipErrorInvalidValue)
#undef E
    }
#undef MORTAR_LIFT_NP_SWITCH
};

}  // namespace

int lift_occupancy(int NP, bool met, bool f64)
{
    return f64 ? LiftLaunch<double>::occupancy(NP, met) : LiftLaunch<float>::occupancy(NP, met);
}

int lift_tile_capacity(int NP, bool met, bool f64)
{
    return f64 ? LiftLaunch<double>::capacity(NP, met) : LiftLaunch<float>::capacity(NP, met);
}

hipError_t launch_lift_f32(const FluxArgs<float> &a, int NP, int grid, bool met, hipStream_t st)
{
    return LiftLaunch<float>::launch(a, NP, grid, met, st);
}

hipError_t launch_lift_f64(const FluxArgs<double> &a, int NP, int grid, bool met, hipStream_t st)
{
    return LiftLaunch<double>::launch(a, NP, grid, met, st);
}

}  // namespace mortar

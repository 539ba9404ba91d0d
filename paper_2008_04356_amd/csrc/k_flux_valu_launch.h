// Launch, occupancy and tile-capacity helpers of the VALU flux kernel for one element
// type and one LDS budget; each instantiation unit exports them under its own names.
#pragma once

#include "k_flux.h"

namespace mortar {

template <typename T, int BUDGET>
struct ValuLaunch {
    template <int NP, bool NSV, bool MET, int RIEM>
    static hipError_t go(const FluxArgs<T> &a, int grid, hipStream_t st)
    {
        hipLaunchKernelGGL((k_mortar_flux<T, NP, NSV, MET, RIEM, BUDGET>), dim3(grid),
                           dim3(kFluxThreads), 0, st, a);
        return hipGetLastError();
    }

    template <int NP>
    static hipError_t pick(const FluxArgs<T> &a, int grid, bool ns, bool met, int riem, hipStream_t st)
    {
        if (ns) {
            if (met) return riem ? go<NP, true, true, 1>(a, grid, st) : go<NP, true, true, 0>(a, grid, st);
            return riem ? go<NP, true, false, 1>(a, grid, st) : go<NP, true, false, 0>(a, grid, st);
        }
        if (met) return riem ? go<NP, false, true, 1>(a, grid, st) : go<NP, false, true, 0>(a, grid, st);
        return riem ? go<NP, false, false, 1>(a, grid, st) : go<NP, false, false, 0>(a, grid, st);
    }

    template <int NP, bool NSV, bool MET, int RIEM>
    static int occ1()
    {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nb, reinterpret_cast<const void *>(&k_mortar_flux<T, NP, NSV, MET, RIEM, BUDGET>),
                kFluxThreads, 0) != hipSuccess)
            return 1;
        return nb > 0 ? nb : 1;
    }

    template <int NP>
    static int occ(bool ns, bool met, int riem)
    {
        if (ns) {
            if (met) return riem ? occ1<NP, true, true, 1>() : occ1<NP, true, true, 0>();
            return riem ? occ1<NP, true, false, 1>() : occ1<NP, true, false, 0>();
        }
        if (met) return riem ? occ1<NP, false, true, 1>() : occ1<NP, false, true, 0>();
        return riem ? occ1<NP, false, false, 1>() : occ1<NP, false, false, 0>();
    }

    template <int NP>
    static int cap(bool ns, bool met)
    {
        if (ns) return met ? FluxCfg<T, NP, true, true, BUDGET>::TF : FluxCfg<T, NP, true, false, BUDGET>::TF;
        return met ? FluxCfg<T, NP, false, true, BUDGET>::TF : FluxCfg<T, NP, false, false, BUDGET>::TF;
    }

#define MORTAR_VALU_NP_SWITCH(EXPR, DEFAULT)                                            \
    switch (NP) {                                                                       \
    case 2: return EXPR(2); case 3: return EXPR(3); case 4: return EXPR(4);            \
    case 5: return EXPR(5); case 6: return EXPR(6); case 7: return EXPR(7);            \
    case 8: return EXPR(8); case 9: return EXPR(9); case 10: return EXPR(10);          \
    default: return DEFAULT;                                                            \
    }

    static int occupancy(int NP, bool ns, bool met, int riem)
    {
#define E(np) occ<np>(ns, met, riem)
        MORTAR_VALU_NP_SWITCH(E, 1)
#undef E
    }

    static int capacity(int NP, bool ns, bool met)
    {
#define E(np) cap<np>(ns, met)
        MORTAR_VALU_NP_SWITCH(E, 0)
#undef E
    }

    static hipError_t launch(const FluxArgs<T> &a, int NP, int grid, bool ns, bool met, int riem,
                             hipStream_t st)
    {
#define E(np) pick<np>(a, grid, ns, met, riem, st)
        MORTAR_VALU_NP_SWITCH(E, hipErrorInvalidValue)
#undef E
    }
#undef MORTAR_VALU_NP_SWITCH
};

}  // namespace mortar

// Launch, occupancy and tile-capacity helpers of the VALU flux kernel for one element
// type, one LDS budget and a range of degrees; each instantiation unit exports them under
// its own names.
#pragma once

#include "k_flux.h"

namespace mortar {

// Instantiations for NP in [LO, HI].
template <typename T, int BUDGET, int LO = 2, int HI = kMaxNFast + 1>
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

    static int occupancy(int NP, bool ns, bool met, int riem)
    {
        return np_dispatch<LO, HI, int>(NP, 1, [&](auto c) { return occ<decltype(c)::value>(ns, met, riem); });
    }

    static int capacity(int NP, bool ns, bool met)
    {
        return np_dispatch<LO, HI, int>(NP, 0, [&](auto c) { return cap<decltype(c)::value>(ns, met); });
    }

    static hipError_t launch(const FluxArgs<T> &a, int NP, int grid, bool ns, bool met, int riem,
                             hipStream_t st)
    {
        return np_dispatch<LO, HI, hipError_t>(NP, hipErrorInvalidValue, [&](auto c) {
            return pick<decltype(c)::value>(a, grid, ns, met, riem, st);
        });
    }
};

}  // namespace mortar

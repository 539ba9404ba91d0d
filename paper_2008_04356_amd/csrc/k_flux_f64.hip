// Instantiations of the fused mortar-flux kernel for element type double.
#include "k_flux.h"

namespace mortar {

constexpr int kLdsBudget = lds_budget<double>();

template <int NP, bool NSV, bool MET, int RIEM>
static hipError_t go(const FluxArgs<double> &a, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((k_mortar_flux<double, NP, NSV, MET, RIEM, kLdsBudget>), dim3(grid),
                       dim3(kFluxThreads), 0, st, a);
    return hipGetLastError();
}

template <int NP>
static hipError_t pick(const FluxArgs<double> &a, int grid, bool ns, bool met, int riem,
                       hipStream_t st)
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
            &nb, reinterpret_cast<const void *>(&k_mortar_flux<double, NP, NSV, MET, RIEM, kLdsBudget>),
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

int flux_occupancy_f64(int NP, bool ns, bool met, int riem)
{
    switch (NP) {
    case 2: return occ<2>(ns, met, riem);
    case 3: return occ<3>(ns, met, riem);
    case 4: return occ<4>(ns, met, riem);
    case 5: return occ<5>(ns, met, riem);
    case 6: return occ<6>(ns, met, riem);
    case 7: return occ<7>(ns, met, riem);
    case 8: return occ<8>(ns, met, riem);
    case 9: return occ<9>(ns, met, riem);
    case 10: return occ<10>(ns, met, riem);
    default: return 1;
    }
}

template <int NP>
static int cap(bool ns, bool met)
{
    if (ns) return met ? FluxCfg<double, NP, true, true, kLdsBudget>::TF
                       : FluxCfg<double, NP, true, false, kLdsBudget>::TF;
    return met ? FluxCfg<double, NP, false, true, kLdsBudget>::TF
               : FluxCfg<double, NP, false, false, kLdsBudget>::TF;
}

int flux_tile_capacity_f64(int NP, bool ns, bool met)
{
    switch (NP) {
    case 2: return cap<2>(ns, met);
    case 3: return cap<3>(ns, met);
    case 4: return cap<4>(ns, met);
    case 5: return cap<5>(ns, met);
    case 6: return cap<6>(ns, met);
    case 7: return cap<7>(ns, met);
    case 8: return cap<8>(ns, met);
    case 9: return cap<9>(ns, met);
    case 10: return cap<10>(ns, met);
    default: return 0;
    }
}

hipError_t launch_flux_f64(const FluxArgs<double> &a, int NP, int grid, bool ns, bool met, int riem,
                          hipStream_t st)
{
    switch (NP) {
    case 2: return pick<2>(a, grid, ns, met, riem, st);
    case 3: return pick<3>(a, grid, ns, met, riem, st);
    case 4: return pick<4>(a, grid, ns, met, riem, st);
    case 5: return pick<5>(a, grid, ns, met, riem, st);
    case 6: return pick<6>(a, grid, ns, met, riem, st);
    case 7: return pick<7>(a, grid, ns, met, riem, st);
    case 8: return pick<8>(a, grid, ns, met, riem, st);
    case 9: return pick<9>(a, grid, ns, met, riem, st);
    case 10: return pick<10>(a, grid, ns, met, riem, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mortar

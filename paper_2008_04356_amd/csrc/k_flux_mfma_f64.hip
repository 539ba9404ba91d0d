// Instantiations of the matrix-core mortar-flux kernel for element type double.
#include "k_flux_mfma.h"

namespace mortar {

template <int NP, bool NSV, bool MET, int RIEM>
static hipError_t go(const FluxArgs<double> &a, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((k_mortar_flux_mfma<double, NP, NSV, MET, RIEM>), dim3(grid),
                       dim3(MCfg<double, NP, NSV, MET>::NT), 0, st, a);
    return hipGetLastError();
}

template <int NP, bool NSV, bool MET, int RIEM>
static int occ1()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void *>(&k_mortar_flux_mfma<double, NP, NSV, MET, RIEM>),
            MCfg<double, NP, NSV, MET>::NT, 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
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

#define MORTAR_NP_SWITCH(EXPR, DEFAULT)                                                 \
    switch (NP) {                                                                       \
    case 2: return EXPR(2); case 3: return EXPR(3); case 4: return EXPR(4);            \
    case 5: return EXPR(5); case 6: return EXPR(6); case 7: return EXPR(7);            \
    case 8: return EXPR(8); case 9: return EXPR(9); case 10: return EXPR(10);          \
    default: return DEFAULT;                                                            \
    }

int flux_mfma_occupancy_f64(int NP, bool ns, bool met, int riem)
{
#define E(np) occ<np>(ns, met, riem)
    MORTAR_NP_SWITCH(E, 1)
#undef E
}

hipError_t launch_flux_mfma_f64(const FluxArgs<double> &a, int NP, int grid, bool ns, bool met,
                               int riem, hipStream_t st)
{
#define E(np) pick<np>(a, grid, ns, met, riem, st)
    MORTAR_NP_SWITCH(E, hipErrorInvalidValue)
#undef E
}

}  // namespace mortar

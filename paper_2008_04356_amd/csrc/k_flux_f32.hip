// Instantiations of the fused mortar-flux kernel for element type float.
#include "k_flux.h"

namespace mortar {

constexpr int kLdsBudget = 65536;

template <int NP, bool NSV, bool MET, int RIEM>
static hipError_t go(const FluxArgs<float> &a, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((k_mortar_flux<float, NP, NSV, MET, RIEM, kLdsBudget>), dim3(grid),
                       dim3(kFluxThreads), 0, st, a);
    return hipGetLastError();
}

template <int NP>
static hipError_t pick(const FluxArgs<float> &a, int grid, bool ns, bool met, int riem,
                       hipStream_t st)
{
    if (ns) {
        if (met) return riem ? go<NP, true, true, 1>(a, grid, st) : go<NP, true, true, 0>(a, grid, st);
        return riem ? go<NP, true, false, 1>(a, grid, st) : go<NP, true, false, 0>(a, grid, st);
    }
    if (met) return riem ? go<NP, false, true, 1>(a, grid, st) : go<NP, false, true, 0>(a, grid, st);
    return riem ? go<NP, false, false, 1>(a, grid, st) : go<NP, false, false, 0>(a, grid, st);
}

int flux_tile_faces_f32(int NP, bool ns, bool met)
{
    const int V = ns ? 20 : 5, VS = V + (met ? 4 : 0);
    int tf = 64;
    while (tf > 2 && (size_t)(VS + V) * NP * (2 * tf + 2) * sizeof(float) > (size_t)kLdsBudget) --tf;
    return tf;
}

hipError_t launch_flux_f32(const FluxArgs<float> &a, int NP, int grid, bool ns, bool met, int riem,
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

// swr_sweep_pair.hip -- instantiates the two-tasks-per-wave subdomain sweep
// (swr_sweep_pair_kernel.h) for a static potential with Robin or S0^2.
#include "swr_sweep_pair_kernel.h"

namespace swr {

template <int P>
static void launch_pair_p(const SweepArgs& a, int trans, hipStream_t st) {
    if (trans == TR_S02) sweep_pair_kernel<P, TR_S02><<<a.ntasks, kWave, 0, st>>>(a);
    else sweep_pair_kernel<P, TR_ROBIN><<<a.ntasks, kWave, 0, st>>>(a);
}

hipError_t launch_sweep_pairs(const SweepArgs& a, int trans, hipStream_t st) {
    if (a.ntasks == 0) return hipSuccess;
    if (!a.pairs || (trans != TR_S02 && trans != TR_ROBIN)) return hipErrorInvalidValue;
    switch (a.P) {
        case 1: launch_pair_p<1>(a, trans, st); break;
        case 2: launch_pair_p<2>(a, trans, st); break;
        case 3: launch_pair_p<3>(a, trans, st); break;
        case 4: launch_pair_p<4>(a, trans, st); break;
        case 5: launch_pair_p<5>(a, trans, st); break;
        case 6: launch_pair_p<6>(a, trans, st); break;
        case 7: launch_pair_p<7>(a, trans, st); break;
        case 8: launch_pair_p<8>(a, trans, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace swr

// swr_sweep_static_s02.hip -- instantiates the subdomain sweep for a
// time-independent potential with the S0^2 transmission, in both workgroup
// forms (with the far-history helper wave for launches of at most
// help_max tasks (a schedule parameter), one wave otherwise; same arithmetic).
#include "swr_sweep_kernel.h"

namespace swr {

template <int P>
static void launch_p(const SweepArgs& a, hipStream_t st) {
    if (a.ntasks <= a.help_max)
        sweep_kernel<P, TR_S02, VK_STATIC, true><<<a.ntasks, sweep_threads(true), 0, st>>>(a);
    else
        sweep_kernel<P, TR_S02, VK_STATIC, false><<<a.ntasks, sweep_threads(false), 0, st>>>(a);
}

hipError_t launch_sweep_static_s02(const SweepArgs& a, hipStream_t st) {
    switch (a.P) {
        case 1: launch_p<1>(a, st); break;
        case 2: launch_p<2>(a, st); break;
        case 3: launch_p<3>(a, st); break;
        case 4: launch_p<4>(a, st); break;
        case 5: launch_p<5>(a, st); break;
        case 6: launch_p<6>(a, st); break;
        case 7: launch_p<7>(a, st); break;
        case 8: launch_p<8>(a, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace swr

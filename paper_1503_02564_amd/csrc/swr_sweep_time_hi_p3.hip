// swr_sweep_time_hi_p3.hip -- instantiates the subdomain sweep for a
// time-dependent potential V(t,x) with the higher-order operators (S0^3, S0^4,
// S1^2, S1^4) and the Pade strategy (S2^{2,m}, S2^{4,m}) at chunk width P = 3
// (one unit per width so that they build in parallel; swr_sweep_time.hip
// dispatches).
#include "swr_sweep_kernel.h"

namespace swr {

template <int P>
hipError_t launch_sweep_time_hi_p(const SweepArgs& a, int trans, hipStream_t st) {
    if (trans == TR_GEN)
        sweep_kernel<P, TR_GEN, VK_TIME><<<a.ntasks, sweep_threads(false), 0, st>>>(a);
    else if (trans == TR_PADE)
        sweep_kernel<P, TR_PADE, VK_TIME><<<a.ntasks, sweep_threads(false), 0, st>>>(a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}
template hipError_t launch_sweep_time_hi_p<3>(const SweepArgs&, int, hipStream_t);

}  // namespace swr

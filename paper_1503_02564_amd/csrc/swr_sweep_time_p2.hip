// swr_sweep_time_p2.hip -- instantiates the subdomain sweep for a time-dependent
// potential V(t,x) at chunk width P = 2 (the refactorising sweep is the
// slowest template to compile, so each width is a unit of its own and they
// build in parallel; swr_sweep_time.hip dispatches).
#include "swr_sweep_kernel.h"

namespace swr {

template <int P>
hipError_t launch_sweep_time_p(const SweepArgs& a, int trans, hipStream_t st) {
    if (trans == TR_S02 && a.ntasks <= a.help_max)
        sweep_kernel<P, TR_S02, VK_TIME, true><<<a.ntasks, sweep_threads(true), 0, st>>>(a);
    else if (trans == TR_S02)
        sweep_kernel<P, TR_S02, VK_TIME, false><<<a.ntasks, sweep_threads(false), 0, st>>>(a);
    else sweep_kernel<P, TR_ROBIN, VK_TIME><<<a.ntasks, sweep_threads(false), 0, st>>>(a);
    return hipGetLastError();
}
template hipError_t launch_sweep_time_p<2>(const SweepArgs&, int, hipStream_t);

}  // namespace swr

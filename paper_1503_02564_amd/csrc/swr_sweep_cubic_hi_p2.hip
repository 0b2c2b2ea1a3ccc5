// swr_sweep_cubic_hi_p2.hip -- instantiates the subdomain sweep for the |u|^2
// potential with the W-dependent operators of order 2 and 3 (S0^3, S1^2,
// S2^{2,m}) at chunk width P = 2 (one unit per width so that they build in
// parallel; swr_sweep_cubic_hi.hip dispatches).
#include "swr_sweep_kernel.h"

namespace swr {

template <int P>
void launch_sweep_cubic_hi_p(const SweepArgs& a, int trans, hipStream_t st) {
    if (trans == TR_GEN) sweep_kernel<P, TR_GEN, VK_CUBIC><<<a.ntasks, sweep_threads(false), 0, st>>>(a);
    else sweep_kernel<P, TR_PADE, VK_CUBIC><<<a.ntasks, sweep_threads(false), 0, st>>>(a);
}
template void launch_sweep_cubic_hi_p<2>(const SweepArgs&, int, hipStream_t);

}  // namespace swr

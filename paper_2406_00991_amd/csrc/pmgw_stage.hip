// Instantiates the Runge-Kutta stage kernels (PMGW_STAGE_PART = 0) or their adjoints
// (PMGW_STAGE_PART = 1) for every finest-level row count. The build compiles this file once per
// part, in parallel with the solve kernels.
#include "pmgw_launch.hpp"

#ifndef PMGW_STAGE_PART
#error "PMGW_STAGE_PART must be defined (0 or 1)"
#endif

namespace pmgw {

#if PMGW_STAGE_PART == 0
template <int NZ>
void launch_k_rk(int which, unsigned grid, size_t lds, hipStream_t st, const RkArgs& a) {
  const dim3 blk(kStageThreads);
  if (which == 0) {
    hipLaunchKernelGGL(k_rk_pre<NZ>, dim3(grid), blk, lds, st, a.descs, a.ids, a.ws, a.cf, a.u,
                       a.w, a.eta, a.Keta, a.rb, a.fftb);
  } else if (which == 1) {
    hipLaunchKernelGGL(k_rk_force<NZ>, dim3(grid, 2), blk, lds, st, a.descs, a.ids, a.ws, a.cf,
                       a.u, a.w, (const double*)a.Ku, (const double*)a.Kw, a.rb, a.fftb);
    hipLaunchKernelGGL(k_rk_rhs<NZ>, dim3(grid), blk, lds, st, a.descs, a.ids, a.ws, a.cf, a.rb,
                       a.fftb);
  } else {
    hipLaunchKernelGGL(k_rk_update<NZ>, dim3(grid, 2), blk, lds, st, a.descs, a.ids, a.ws, a.cf,
                       a.pr, a.uo, a.wo, a.Ku, a.Kw, a.rb, a.fftb);
  }
}

template void launch_k_rk<3>(int, unsigned, size_t, hipStream_t, const RkArgs&);
template void launch_k_rk<5>(int, unsigned, size_t, hipStream_t, const RkArgs&);
template void launch_k_rk<9>(int, unsigned, size_t, hipStream_t, const RkArgs&);
template void launch_k_rk<17>(int, unsigned, size_t, hipStream_t, const RkArgs&);
template void launch_k_rk<33>(int, unsigned, size_t, hipStream_t, const RkArgs&);
#else
template <int NZ>
void launch_k_rka(int which, unsigned grid, size_t lds, hipStream_t st, const RkaArgs& a) {
  if (which == 0)
    hipLaunchKernelGGL(k_rka_post<NZ>, dim3(grid), dim3(256), lds, st, a.descs, a.ids, a.ws,
                       a.cf, a.ub, a.wb, a.Kub, a.Kwb, a.rb, a.ab, a.fftb);
  else if (which == 1)
    hipLaunchKernelGGL(k_rka_mid<NZ>, dim3(grid), dim3(256), lds, st, a.descs, a.ids, a.ws,
                       a.cf, a.ub, a.wb, a.Kub, a.Kwb, a.rb, a.ab, a.fftb);
  else if (which == 2)
    hipLaunchKernelGGL(k_rka_force<NZ>, dim3(grid), dim3(256), lds, st, a.descs, a.ids, a.ws,
                       a.cf, a.u, a.w, a.ub, a.wb, a.rb, a.ab, a.fftb);
  else
    hipLaunchKernelGGL(k_rka_pre<NZ>, dim3(grid), dim3(256), lds, st, a.descs, a.ids, a.ws,
                       a.cf, a.u, a.ub, a.wb, a.etab, a.Ketab, a.hbar, a.rb, a.ab, a.fftb);
}

template void launch_k_rka<3>(int, unsigned, size_t, hipStream_t, const RkaArgs&);
template void launch_k_rka<5>(int, unsigned, size_t, hipStream_t, const RkaArgs&);
template void launch_k_rka<9>(int, unsigned, size_t, hipStream_t, const RkaArgs&);
template void launch_k_rka<17>(int, unsigned, size_t, hipStream_t, const RkaArgs&);
template void launch_k_rka<33>(int, unsigned, size_t, hipStream_t, const RkaArgs&);
#endif

}  // namespace pmgw

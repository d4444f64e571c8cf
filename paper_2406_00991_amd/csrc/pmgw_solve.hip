// Instantiates the per-tank solve kernel for one V-cycle precision (PMGW_TV: float or double) and
// one direction (PMGW_TR: 0 = A and the V-cycle, 1 = A^T and the transposed cycle), for every
// finest-level row count; with PMGW_WIDE (forward only), the 512-thread build of the forward
// kernel instead. The build compiles this file once per combination, in parallel.
#include "pmgw_launch.hpp"

#ifndef PMGW_TV
#error "PMGW_TV must be defined (float or double)"
#endif
#ifndef PMGW_TR
#error "PMGW_TR must be defined (0 or 1)"
#endif

namespace pmgw {

// Largest workgroup the solve kernel is compiled for (its register budget follows from it).
constexpr int kSolveMaxThreads = 256;

#ifdef PMGW_WIDE
static_assert(PMGW_TR == 0, "the 512-thread build is forward only");
constexpr int kSolveWideThreads = 512;

template <typename TV, int NZ>
void launch_k_solve_wide(unsigned grid, int threads, size_t lds, hipStream_t st,
                         const SolveArgs& a) {
  hipLaunchKernelGGL((k_solve<TV, NZ, kSolveWideThreads, false>), dim3(grid), dim3(threads), lds,
                     st, a.descs, a.ids, a.ws, a.mode, a.in, a.out, a.rtol, a.maxit, a.info, a.o,
                     a.fftb);
}

template void launch_k_solve_wide<PMGW_TV, 3>(unsigned, int, size_t, hipStream_t,
                                              const SolveArgs&);
template void launch_k_solve_wide<PMGW_TV, 5>(unsigned, int, size_t, hipStream_t,
                                              const SolveArgs&);
template void launch_k_solve_wide<PMGW_TV, 9>(unsigned, int, size_t, hipStream_t,
                                              const SolveArgs&);
template void launch_k_solve_wide<PMGW_TV, 17>(unsigned, int, size_t, hipStream_t,
                                               const SolveArgs&);
template void launch_k_solve_wide<PMGW_TV, 33>(unsigned, int, size_t, hipStream_t,
                                               const SolveArgs&);
#else

template <typename TV, int NZ, bool TR>
void launch_k_solve(unsigned grid, int threads, size_t lds, hipStream_t st, const SolveArgs& a) {
  hipLaunchKernelGGL((k_solve<TV, NZ, kSolveMaxThreads, TR>), dim3(grid), dim3(threads), lds, st,
                     a.descs, a.ids, a.ws, a.mode, a.in, a.out, a.rtol, a.maxit, a.info, a.o,
                     a.fftb);
}

template void launch_k_solve<PMGW_TV, 3, PMGW_TR != 0>(unsigned, int, size_t, hipStream_t,
                                                        const SolveArgs&);
template void launch_k_solve<PMGW_TV, 5, PMGW_TR != 0>(unsigned, int, size_t, hipStream_t,
                                                        const SolveArgs&);
template void launch_k_solve<PMGW_TV, 9, PMGW_TR != 0>(unsigned, int, size_t, hipStream_t,
                                                        const SolveArgs&);
template void launch_k_solve<PMGW_TV, 17, PMGW_TR != 0>(unsigned, int, size_t, hipStream_t,
                                                         const SolveArgs&);
template void launch_k_solve<PMGW_TV, 33, PMGW_TR != 0>(unsigned, int, size_t, hipStream_t,
                                                         const SolveArgs&);

#if PMGW_TR == 0
template <int NZ>
void launch_k_solve_res(unsigned grid, int threads, size_t lds, hipStream_t st,
                        const SolveArgs& a) {
  if constexpr (std::is_same<PMGW_TV, float>::value) {
    hipLaunchKernelGGL((k_solve<float, NZ, kSolveMaxThreads, false, true>), dim3(grid),
                       dim3(threads), lds, st, a.descs, a.ids, a.ws, a.mode, a.in, a.out, a.rtol,
                       a.maxit, a.info, a.o, a.fftb);
  }
}
#endif

#if PMGW_TR == 0 && defined(PMGW_TV_IS_FLOAT)
template void launch_k_solve_res<3>(unsigned, int, size_t, hipStream_t, const SolveArgs&);
template void launch_k_solve_res<5>(unsigned, int, size_t, hipStream_t, const SolveArgs&);
template void launch_k_solve_res<9>(unsigned, int, size_t, hipStream_t, const SolveArgs&);
template void launch_k_solve_res<17>(unsigned, int, size_t, hipStream_t, const SolveArgs&);
#endif

#endif  // PMGW_WIDE

}  // namespace pmgw

// Launch interface between the host API (pmgw.hip) and the translation units that instantiate
// the large kernels (pmgw_solve.hip per precision and direction, pmgw_stage.hip for the RK stage
// and its adjoint). Each launcher enqueues one kernel on the given stream; the host API chooses
// the grid, block size and dynamic LDS.
#pragma once
#include <hip/hip_runtime.h>

#include "pmgw_rka.hpp"

namespace pmgw {

// Arguments of the per-tank solve kernel (k_solve): see its comment in pmgw_kernels.hpp.
struct SolveArgs {
  const TankDesc* descs;
  const int32_t* ids;
  char* ws;
  int mode;
  const double* in;
  double* out;
  double rtol;
  int maxit;
  pmgw_info_dev* info;
  KOpts o;
  int fftb;
};

// grid = number of tanks of the class, threads = workgroup size, lds = dynamic LDS bytes.
template <typename TV, int NZ, bool TR>
void launch_k_solve(unsigned grid, int threads, size_t lds, hipStream_t st, const SolveArgs& a);

// The forward kernel compiled for workgroups of up to 512 threads (two wavefronts per SIMD).
template <typename TV, int NZ>
void launch_k_solve_wide(unsigned grid, int threads, size_t lds, hipStream_t st,
                         const SolveArgs& a);

// The same kernel with the LDS-resident float32 V-cycle (forward, NZ <= 17).
template <int NZ>
void launch_k_solve_res(unsigned grid, int threads, size_t lds, hipStream_t st,
                        const SolveArgs& a);

// Arguments of the stage kernels: k_rk_pre (which = 0), k_rk_force and k_rk_rhs (1),
// k_rk_update (2).
struct RkArgs {
  const TankDesc* descs;
  const int32_t* ids;
  char* ws;
  RkCoef cf;
  const double* u;
  const double* w;
  double* eta;
  double* Ku;
  double* Kw;
  double* Keta;
  const double* pr;
  double* uo;
  double* wo;
  RkBufs rb;
  int fftb;
};

template <int NZ>
void launch_k_rk(int which, unsigned grid, size_t lds, hipStream_t st, const RkArgs& a);

// Arguments of the adjoint stage kernels k_rka_post (which = 0), k_rka_mid (1), k_rka_force (2),
// k_rka_pre (3).
struct RkaArgs {
  const TankDesc* descs;
  const int32_t* ids;
  char* ws;
  RkCoef cf;
  const double* u;
  const double* w;
  double* ub;
  double* wb;
  double* etab;
  double* Kub;
  double* Kwb;
  double* Ketab;
  double* hbar;
  RkBufs rb;
  AdjBufs ab;
  int fftb;
};

template <int NZ>
void launch_k_rka(int which, unsigned grid, size_t lds, hipStream_t st, const RkaArgs& a);

}  // namespace pmgw

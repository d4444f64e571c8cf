// Workspace layout shared by the host API and the kernels of the p-multigrid Poisson library.
//
// Everything lives in one caller-owned device buffer. All offsets are BYTE offsets from the
// start of that buffer, each array aligned to 256 bytes.
#pragma once
#include <stdint.h>

namespace pmgw {

constexpr int kMaxLev = 5;          // orders 32, 16, 8, 4, 2
constexpr int kMaxRestart = 32;     // FGMRES restart length bound (Hessenberg lives in LDS)
constexpr int kFftBytes = 32768;    // one LDS ping-pong buffer of the row FFTs
constexpr int kMaxNz = 33;
constexpr int kCoarseExactMaxNx = 512;
// Largest Nx of the bed-line step (its set-up is Nx^3 multiply-adds per level).
constexpr int kBedLineMaxNx = 1024;   // largest Nx of the direct coarsest-level solve

enum : int32_t { PREC64 = 0, PREC32 = 1 };

// One multigrid level of one tank (order M_l = nz - 1).
struct LevelDesc {
  int32_t nz, nzc;                  // rows here, rows on the next coarser level (0 on coarsest)
  int64_t ds[2];                    // D_sigma [nz][nz], float64 / float32 copies
  int64_t sig[2];                   // sigma_j [nz]
  int64_t dss;                      // D_s D_s and D_s diag(sigma) D_s, [2][nz][nz] float64
                                    // (the column and mode blocks are combinations of these)
  int64_t R[2];                     // restriction [nzc][nz]
  int64_t P[2];                     // prolongation [nz][nzc]
  int64_t PT[2];                    // P^T [nzc][nz] (restriction of the transposed cycle)
  int64_t RT[2];                    // R^T [nz][nzc] (prolongation of the transposed cycle)
  int64_t colinv;                   // inverse column blocks [nz][nz][nx] (V-cycle precision)
  int64_t modeinv;                  // inverse flat-mode blocks [nz][nz][nx/2+1]
  int64_t x, f, r, t1, t2, t3;      // level vectors [nz][nx] (V-cycle precision)
  int64_t u;                        // full-multigrid iterate of the level [nz][nx]
  int64_t spec;                     // packed row spectra [(nz+1)/2][nx] complex (V precision)
  int64_t bedinv;                   // bed-line inverse L_b^-1, transposed [nx][nx], float64
  int64_t bedinv32;                 // its float32 copy (mixed plans; 0 otherwise)
};

struct TankDesc {
  int32_t nx, nz, nlev, log2nx;
  double L, kfac, cxx;              // length, 2 pi / L, diagonal of D_x D_x
  int64_t off2d, off1d;             // element offsets into the caller's packed fields
  int64_t tw[2];                    // twiddles exp(-2 pi i t / nx), t < nx (complex)
  int64_t filtx;                    // x-filter factors F(|k|), k = 0..nx/2 (float64)
  int64_t filtz;                    // sigma-filter matrix [nz][nz] on the finest level (float64)
  int64_t geo64;                    // 10 x nx doubles (see GEO_* below)
  int64_t geo32;                    // 7 x nx floats: ao, bo, ido, an, bn, idn, hx
  int64_t scal;                     // 64 bytes: double cbar, ebar; int32 status at +16;
                                    // double mode-damping factor at +24
  int64_t V, Z;                     // FGMRES bases: (restart+1) x n and restart x n doubles
  int64_t a1, a2, a3, aspec;        // float64 operator temporaries (finest level)
  int64_t cw, cwt;                  // direct solve of the coarsest level (0 unless enabled):
                                    // W = [Q | B^-1] [2 nx][3 nx] and its transpose (float64)
  LevelDesc lev[kMaxLev];
};

// rows of geo64
enum : int { GEO_H = 0, GEO_EO = 1, GEO_EN = 2, GEO_AO = 3, GEO_BO = 4, GEO_IDO = 5,
             GEO_AN = 6, GEO_BN = 7, GEO_IDN = 8, GEO_HX = 9 };

// A job of the block-inversion kernel: `count` consecutive workgroups, one block each.
struct BlockJob {
  int32_t tank, level, kind, count;   // kind 0 = column block i, 1 = flat-mode block k
  int64_t first;
};

struct KOpts {
  int32_t nu1, nu2, coarse_pairs, restart;
  double omega_c, omega_m;
  int32_t adapt;                    // scale omega_m by the tank's factor (scal + 24)
  int32_t cycle;                    // preconditioner: 0 V-cycle, 1 full multigrid
  int32_t coarse_exact;             // coarsest level: 0 smoothing pairs, 1 direct solve
  int32_t bed_line;                 // end every smoothing pair with the bed-line step
};

}  // namespace pmgw

/*
 * pmgw3d.h -- C ABI of the 3D tanks of the p-multigrid pressure Poisson library.
 *
 * A 3D tank is periodic in x and y (Fourier, Nx x Ny points on Lx x Ly) with the sigma
 * Chebyshev basis in the vertical, as in the paper's sigma-transformed model with the horizontal
 * gradient (d/dx, d/dy) (Sec. 2.1, eq. 1_chain and eq. 1_Scoef with their y-terms; Sec. 3.4's
 * Fourier derivatives in y as in x). The operator, its V-cycle and the outer solve follow the 2D
 * library (pmgw.h) with the y-terms added:
 *   - metrics: d = h + eta, sigma_x = (h_x - sigma d_x)/d, sigma_y = (h_y - sigma d_y)/d;
 *   - rows: 0 = P (Dirichlet surface), 1..M-1 = Div^new Grad^old P with
 *     Grad P = (D_x P + sigma_x D_s P, D_y P + sigma_y D_s P, D_s P / d),
 *     Div F = D_x F_x + sigma_x D_s F_x + D_y F_y + sigma_y D_s F_y + D_s F_z / d,
 *     M = the bed condition -(h_x G_x + h_y G_y + G_z) on the old geometry
 *     (eq. poissonp, eq. bcpd, eq. bcpdneu);
 *   - V-cycle (Alg. 1) over the Chebyshev order with the smoothing pair: block Jacobi with each
 *     column's exact block, then the exact inverse of the horizontally averaged flat operator per
 *     Fourier mode (kx, ky); the coarsest level (order 2) runs coarse_pairs pairs from zero;
 *   - FGMRES(restart) right-preconditioned by one V-cycle, float64 throughout.
 *
 * Conventions
 *   - A field of tank t is a float64 DEVICE array [Nz][Ny][Nx], x fastest; tanks are packed back
 *     to back at off3d[t] (pmgw3_field_offsets); h and eta are [Ny][Nx] at off2d[t].
 *   - Sizes: Nx, Ny powers of two with 4 <= Nx, Ny and Nx Ny <= 65536, Nx, Ny <= 1024;
 *     Nz = M + 1 with M in {2, 4, 8, 16, 32}; Lx, Ly > 0.
 *   - The library allocates no device memory: the caller binds a workspace of
 *     pmgw3_workspace_bytes. Every call enqueues on the plan's stream; a non-NULL host info
 *     pointer makes it wait. Return codes as in pmgw.h; pmgw_last_error() describes failures.
 *   - Options: nu1, nu2, coarse_pairs, restart, omega_c, omega_m and adapt_omega_m of pmgw_opts
 *     apply; the others are ignored. Precision: PMGW_FP64 only.
 */
#ifndef PMGW3D_H
#define PMGW3D_H

#include <stddef.h>
#include <stdint.h>

#include "pmgw.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pmgw3_plan_s* pmgw3_plan;

/* Plan for ntanks 3D tanks (host arrays of sizes and periods). opts may be NULL (defaults);
 * stream = the hipStream_t to enqueue on (NULL = the null stream). */
int pmgw3_plan_create(pmgw3_plan* out, int32_t ntanks, const int32_t* nx, const int32_t* ny,
                      const int32_t* nz, const double* Lx, const double* Ly, int32_t precision,
                      const pmgw_opts* opts, void* stream);

/* Bytes of device workspace the plan needs, and binding of a caller-owned buffer. */
size_t pmgw3_workspace_bytes(pmgw3_plan plan);
int pmgw3_bind_workspace(pmgw3_plan plan, void* dev_ptr, size_t bytes);

/* Host outputs: off3d[ntanks + 1] element offsets of the 3D fields, off2d[ntanks + 1] of h/eta. */
int pmgw3_field_offsets(pmgw3_plan plan, int64_t* off3d, int64_t* off2d);

/* sigma-metrics of the old and new surface (device arrays [Ny][Nx] packed at off2d) and the
 * smoother's block inverses (column blocks and flat-mode blocks per level, Gauss-Jordan with
 * partial pivoting, float64). d <= 0 anywhere marks the tank PMGW_EGEOM. */
int pmgw3_set_geometry(pmgw3_plan plan, const double* h, const double* eta_old,
                       const double* eta_new);

/* Ap = A p (the operator above), device arrays packed at off3d. */
int pmgw3_laplacian_apply(pmgw3_plan plan, const double* p, double* Ap);

/* z = one V-cycle applied to r from a zero initial guess (paper Alg. 1). */
int pmgw3_vcycle(pmgw3_plan plan, const double* r, double* z);

/* FGMRES on A p = b from the initial guess in p, until ||b - A p||_2 <= rtol ||b||_2 or maxit
 * V-cycle applications; per-tank outcome in info (host, ntanks records, optional; with it the
 * call waits) or info_dev (device, optional). */
int pmgw3_poisson_solve(pmgw3_plan plan, const double* b, double* p, double rtol, int32_t maxit,
                        pmgw_info* info_host, pmgw_info* info_dev);

void pmgw3_plan_destroy(pmgw3_plan plan);

#ifdef __cplusplus
}
#endif

#endif /* PMGW3D_H */

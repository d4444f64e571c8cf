// Kernels of one low-storage Runge-Kutta stage with the pressure projection (paper Sec. 3.1-3.3,
// Sec. 3.6), float64, launched per finest-level row count NZ; one workgroup per tank, or per tank
// and velocity component where the two components are independent (grid.y = 2):
//
//   k_rk_pre    surface: eta_t = -u~ D_x eta + w~; K_eta <- a K_eta + dt eta_t;
//               eta <- filter_x(eta + b K_eta); the old surface is kept for the metrics.
//   (geometry)  sigma-metrics of the old and new surface and the smoother blocks.
//   k_rk_force  per component: forcing at the old stage, F_u = -u D_x u - w_s D_s u - g D_x eta
//               + nu Div Grad u, F_w = -u D_x w - w_s D_s w + nu Div Grad w with
//               w_s = sigma_t + u sigma_x + w/d, sigma_t = -sigma eta_t / d; provisional
//               u* = u + b (a K_u + dt F_u), w* likewise.
//   k_rk_rhs    right-hand side rho/(b dt) Div^new(u*, w*) inside, 0 on the surface row and
//               -rho/(b dt)(h_x u* + w*) on the bed row (eq. poissonp, eq. bcpd, eq. bcpdneu).
//   (solve)     flexible GMRES / p-multigrid for the dynamic pressure p.
//   k_rk_update per component: (G_x, G_z) = Grad^old p; K_u <- a K_u + dt (F_u - G_x/rho),
//               K_w likewise; u <- filter(u + b K_u), w <- filter(w + b K_w) in x and sigma.
//
// Model options (RkCoef): lin = the linearised equations (eq. NSElin, eq. linFS): F without the
// advection terms, eta_t = w~, and the host sets the geometry with eta = 0 (z1, zeroed by
// k_rk_pre); noslip = no-slip bed (Sec. 5, oscillatory wave boundary layer): after the update
// and the filter, K_u, K_w, u and w are set to zero on the bed row, and the viscous term is
// dropped on the surface row.
#pragma once
#include <stdint.h>

#include "pmgw_kernels.hpp"

namespace pmgw {

// Packed workspace of the stage: 1D arrays of n1d doubles, 2D arrays of n2d doubles.
struct RkBufs {
  double *eo, *etat, *etax, *z1;
  double *Fu, *Fw, *us, *ws, *b, *r1, *r2;
};

inline int64_t rk_align(int64_t v) { return (v + 255) & ~int64_t(255); }

inline int64_t rk_workspace_bytes(int64_t n2d, int64_t n1d) {
  return 4 * rk_align(8 * n1d) + 7 * rk_align(8 * n2d);
}

inline RkBufs rk_bufs(char* base, int64_t n2d, int64_t n1d) {
  RkBufs r;
  int64_t o = 0;
  auto take = [&](int64_t bytes) {
    double* p = reinterpret_cast<double*>(base + o);
    o += rk_align(bytes);
    return p;
  };
  r.eo = take(8 * n1d);
  r.etat = take(8 * n1d);
  r.etax = take(8 * n1d);
  r.z1 = take(8 * n1d);
  r.Fu = take(8 * n2d);
  r.Fw = take(8 * n2d);
  r.us = take(8 * n2d);
  r.ws = take(8 * n2d);
  r.b = take(8 * n2d);
  r.r1 = take(8 * n2d);
  r.r2 = take(8 * n2d);
  return r;
}

// Threads per stage workgroup (one workgroup per tank, or per tank and velocity component): four
// wavefronts, whose 16-lane groups take the row pairs of 256-point rows through the 16 x 16
// transform in one round. Eight wavefronts would leave 128 registers per lane, too few for that
// transform's sixteen complex values without spilling; on the radix-4 path they measured slower
// at 256 x 17 (k_rk_force 49 against 44 us, k_rk_rhs 25 against 22, k_rk_update 41 against 35).
constexpr int kStageThreads = 256;

struct RkCoef {
  double a, b, dt, rho, g, nu;
  int lin = 0;     // linearised model: no advection, eta_t = w~, still-water sigma-map
  int noslip = 0;  // no-slip bed: bed rows of u, w, K_u, K_w held at zero; no viscous term at
                   // the surface row
};

// float64 context of a tank: metrics of the geometry last set, finest-level constants; also
// stages the tank's twiddles in LDS (a workgroup barrier: every thread must call it).
__device__ __forceinline__ void rk_ctx(char* ws, const TankDesc& td, int fftb, Ctx<double>& c,
                                       Lev<double>& A) {
  c.nx = td.nx;
  c.log2nx = td.log2nx;
  c.kfac = td.kfac;
  c.fftb = fftb;
  stage_twiddles(gcp<cpx<double>>(ws, td.tw[0]), gcp<cpx<float>>(ws, td.tw[1]), td.nx, fftb);
  c.g = make_geo<double>(ws, td);
  c.cw = gptr<const double>(nullptr);
  c.cwt = gptr<const double>(nullptr);
  A = make_lev<double>(ws, td.lev[0]);
  A.t1 = gmp<double>(ws, td.a1);
  A.t2 = gmp<double>(ws, td.a2);
  A.t3 = gmp<double>(ws, td.a3);
}

// Filter multiplier F(|k|)/N for the packed x-FFT.
__device__ __forceinline__ cpx<double> filt_mul(gptr<const double> fx, int N, int n,
                                                cpx<double> v) {
  const int k = n <= (N >> 1) ? n : N - n;
  const double f = fx[k] / (double)N;
  return {v.re * f, v.im * f};
}

// The surface part of a stage for one tank (every thread of the workgroup calls it; ends with a
// barrier): eta_t = -u~ D_x eta + w~ (w~ alone in the linearised model), K_eta <- a K_eta +
// dt eta_t, the old surface kept in eo, eta <- filter_x(eta + b K_eta); z1 <- 0.
__device__ __forceinline__ void rk_pre_tank(const TankDesc& td, char* ws, const RkCoef& cf,
                                            const double* u, const double* w, double* eta,
                                            double* Keta, const RkBufs& rb, int fftb) {
  const int nx = td.nx;
  const gptr<const double> u0 = as_global(u + td.off2d);
  const gptr<const double> w0 = as_global(w + td.off2d);
  const gptr<double> e = as_global(eta + td.off1d);
  const gptr<double> ke = as_global(Keta + td.off1d);
  const gptr<double> eo = as_global(rb.eo + td.off1d);
  const gptr<double> et = as_global(rb.etat + td.off1d);
  const gptr<double> ex = as_global(rb.etax + td.off1d);
  const gptr<const double> fx = gcp<double>(ws, td.filtx);
  stage_twiddles(gcp<cpx<double>>(ws, td.tw[0]), gcp<cpx<float>>(ws, td.tw[1]), nx, fftb);
  dx_rows<double>(1, nx, td.log2nx, td.kfac, fftb, [=](int, int i) { return e[i]; },
                  [=](int, int i, double v) { ex[i] = v; });
  const gptr<double> z1 = as_global(rb.z1 + td.off1d);
  for (int i = tid(); i < nx; i += nthr()) {
    const double rate = cf.lin ? w0[i] : -u0[i] * ex[i] + w0[i];
    et[i] = rate;
    const double k = cf.a * ke[i] + cf.dt * rate;
    ke[i] = k;
    eo[i] = e[i];
    e[i] = e[i] + cf.b * k;
    z1[i] = 0.0;
  }
  __syncthreads();
  spectral_rows<double>(1, nx, td.log2nx, fftb, [=](int, int i) { return e[i]; },
                        [=](int n, cpx<double> v) { return filt_mul(fx, nx, n, v); },
                        [=](int, int i, double v) { e[i] = v; });
}

template <int NZ>
__global__ void __launch_bounds__(kStageThreads) k_rk_pre(const TankDesc* __restrict__ descs,
                                                const int32_t* __restrict__ ids, char* ws,
                                                RkCoef cf, const double* u, const double* w,
                                                double* eta, double* Keta, RkBufs rb, int fftb) {
  const TankDesc& td = descs[ids[blockIdx.x]];
  if (td.nz != NZ || td.nx < 8 || td.nx > 2048) return;
  rk_pre_tank(td, ws, cf, u, w, eta, Keta, rb, fftb);
}

// Forcing and provisional velocity of one component per workgroup: blockIdx.y = 0 for u (level
// temporaries t1..t3 of the finest level), 1 for w (r1, r2, b as temporaries: r1 and r2 are
// written by k_rk_update later, b by k_rk_rhs after both components).
template <int NZ>
__global__ void __launch_bounds__(kStageThreads) k_rk_force(const TankDesc* __restrict__ descs,
                                                  const int32_t* __restrict__ ids, char* ws,
                                                  RkCoef cf, const double* u, const double* w,
                                                  const double* Ku, const double* Kw, RkBufs rb,
                                                  int fftb) {
  const TankDesc& td = descs[ids[blockIdx.x]];
  const int nx = td.nx, n = nx * NZ, comp = blockIdx.y;
  if (td.nz != NZ || nx < 8 || nx > 2048) return;
  Ctx<double> c;
  Lev<double> A;
  rk_ctx(ws, td, fftb, c, A);
  if (comp == 1) {
    A.t1 = as_global(rb.r1 + td.off2d);
    A.t2 = as_global(rb.r2 + td.off2d);
    A.t3 = as_global(rb.b + td.off2d);
  }
  Ctx<double> cold = c;               // Div^old Grad^old for the viscous term
  cold.g.an = c.g.ao;
  cold.g.bn = c.g.bo;
  cold.g.idn = c.g.ido;
  const Geo<double> g = c.g;
  const gptr<const double> sig = A.sig;
  const gptr<const double> uu = as_global(u + td.off2d), wwp = as_global(w + td.off2d);
  const gptr<const double> f = comp == 0 ? uu : wwp;
  const gptr<const double> K = as_global((comp == 0 ? Ku : Kw) + td.off2d);
  const gptr<double> F = as_global((comp == 0 ? rb.Fu : rb.Fw) + td.off2d);
  const gptr<double> star = as_global((comp == 0 ? rb.us : rb.ws) + td.off2d);
  const gptr<const double> et = as_global(rb.etat + td.off1d);
  const gptr<const double> ex = as_global(rb.etax + td.off1d);
  const gptr<double> t1 = A.t1, t2 = A.t2;
  // F <- Div^old Grad^old f; leaves t1 = D_s f, t2 = D_x f
  op_apply<double, NZ>(cold, A, FIN_FULL, f, F, gptr<const double>(nullptr),
                       gptr<double>(nullptr), 0.0);
  for (int e = tid(); e < n; e += nthr()) {
    const int j = e / nx, i = e - j * nx;
    const double sx = g.ao[i] + g.bo[i] * sig[j];
    const double wsig = -sig[j] * et[i] * g.ido[i] + uu[e] * sx + wwp[e] * g.ido[i];
    double fo = (cf.noslip && j == 0) ? 0.0 : cf.nu * F[e];
    if (!cf.lin) fo += -uu[e] * t2[e] - wsig * t1[e];
    if (comp == 0) fo -= cf.g * ex[i];
    F[e] = fo;
    star[e] = f[e] + cf.b * (cf.a * K[e] + cf.dt * fo);
  }
}

// Right-hand side of the stage's pressure problem: scale Div^new(u*, w*) inside, 0 on the surface
// row, -scale (h_x u* + w*) on the bed row.
template <int NZ>
__global__ void __launch_bounds__(kStageThreads) k_rk_rhs(const TankDesc* __restrict__ descs,
                                                const int32_t* __restrict__ ids, char* ws,
                                                RkCoef cf, RkBufs rb, int fftb) {
  const TankDesc& td = descs[ids[blockIdx.x]];
  const int nx = td.nx, n = nx * NZ;
  if (td.nz != NZ || nx < 8 || nx > 2048) return;
  Ctx<double> c;
  Lev<double> A;
  rk_ctx(ws, td, fftb, c, A);
  const Geo<double> g = c.g;
  const gptr<const double> sig = A.sig;
  const gptr<const double> us = as_global(rb.us + td.off2d), wsv = as_global(rb.ws + td.off2d);
  const gptr<double> b = as_global(rb.b + td.off2d);
  const gptr<double> t1 = A.t1, t2 = A.t2, t3 = A.t3;
  col_dsig<double, NZ>(nx, A.Ds, us, t1);
  col_dsig<double, NZ>(nx, A.Ds, wsv, t3);
  __syncthreads();
  dx_rows<double>(NZ, nx, c.log2nx, c.kfac, fftb, [=](int j, int i) { return us[j * nx + i]; },
                  [=](int j, int i, double v) { t2[j * nx + i] = v; });
  const double scale = cf.rho / (cf.b * cf.dt);
  for (int e = tid(); e < n; e += nthr()) {
    const int j = e / nx, i = e - j * nx;
    double v;
    if (j == 0) v = 0.0;
    else if (j == NZ - 1) v = -scale * (g.hx[i] * us[e] + wsv[e]);
    else v = scale * (t2[e] + (g.an[i] + g.bn[i] * sig[j]) * t1[e] + g.idn[i] * t3[e]);
    b[e] = v;
  }
}

// Projection, velocity update and filter, one velocity component per workgroup
// (blockIdx.y = 0 for u, 1 for w): G = Grad^old p (G_x = D_x p + sigma_x D_s p, G_z = D_s p / d),
// K <- a K + dt (F - G / rho), r = q + b K, then q <- filter(r) in x and sigma. Temporaries:
// u uses t1, t2, t3 of the finest level and r1; w uses b and us (both free after the solve) and
// r2.
template <int NZ>
__global__ void __launch_bounds__(kStageThreads) k_rk_update(const TankDesc* __restrict__ descs,
                                                   const int32_t* __restrict__ ids, char* ws,
                                                   RkCoef cf, const double* p, double* u,
                                                   double* w, double* Ku, double* Kw, RkBufs rb,
                                                   int fftb) {
  const TankDesc& td = descs[ids[blockIdx.x]];
  const int nx = td.nx, n = nx * NZ, comp = blockIdx.y;
  if (td.nz != NZ || nx < 8 || nx > 2048) return;
  Ctx<double> c;
  Lev<double> A;
  rk_ctx(ws, td, fftb, c, A);
  const Geo<double> g = c.g;
  const gptr<const double> sig = A.sig;
  const gptr<const double> pp = as_global(p + td.off2d);
  const gptr<double> q = as_global((comp == 0 ? u : w) + td.off2d);
  const gptr<double> K = as_global((comp == 0 ? Ku : Kw) + td.off2d);
  const gptr<const double> F = as_global((comp == 0 ? rb.Fu : rb.Fw) + td.off2d);
  const gptr<double> r = as_global((comp == 0 ? rb.r1 : rb.r2) + td.off2d);
  const gptr<double> ts = comp == 0 ? A.t1 : as_global(rb.b + td.off2d);
  const gptr<double> tf = comp == 0 ? A.t3 : as_global(rb.us + td.off2d);
  const gptr<double> t2 = A.t2;
  const gptr<const double> fx = gcp<double>(ws, td.filtx);
  const gptr<const double> fz = gcp<double>(ws, td.filtz);
  col_dsig<double, NZ>(nx, A.Ds, pp, ts);
  __syncthreads();
  if (comp == 0)
    dx_rows<double>(NZ, nx, c.log2nx, c.kfac, fftb, [=](int j, int i) { return pp[j * nx + i]; },
                    [=](int j, int i, double v) { t2[j * nx + i] = v; });
  const double ir = 1.0 / cf.rho;
  for (int e = tid(); e < n; e += nthr()) {
    const int j = e / nx, i = e - j * nx;
    const double gr = comp == 0 ? t2[e] + (g.ao[i] + g.bo[i] * sig[j]) * ts[e]
                                : ts[e] * g.ido[i];
    const double a = cf.a * K[e] + cf.dt * (F[e] - gr * ir);
    const bool held = cf.noslip && j == NZ - 1;  // the update itself runs unheld, as filtered
    K[e] = held ? 0.0 : a;
    r[e] = q[e] + cf.b * a;
  }
  __syncthreads();
  spectral_rows<double>(NZ, nx, td.log2nx, fftb, [=](int j, int i) { return r[j * nx + i]; },
                        [=](int k, cpx<double> v) { return filt_mul(fx, nx, k, v); },
                        [=](int j, int i, double v) { tf[j * nx + i] = v; });
  col_dsig<double, NZ>(nx, fz, tf, q);
  if (cf.noslip) {
    __syncthreads();
    for (int i = tid(); i < nx; i += nthr()) q[(NZ - 1) * nx + i] = 0.0;
  }
}

}  // namespace pmgw

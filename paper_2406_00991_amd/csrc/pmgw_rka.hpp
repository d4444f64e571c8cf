// Discrete adjoint of one Runge-Kutta stage (the reverse of pmgw_rk.hpp), float64, one
// workgroup per tank, launched per finest-level row count NZ.
//
// The stage's forward intermediates (eta_t, D_x eta, the new surface, both geometries, the
// forcing's provisional velocity and the pressure p) are recomputed first from the stage's input
// state by the forward kernels. Then, given the adjoints of the stage outputs
// (ubar, wbar, etabar, Kubar, Kwbar, Ketabar), the kernels below run the reverse steps:
//
//   k_rka_post   filters and velocity/K update:
//                uh = F_x F_s^T ubar; Kbar_new = Kubar + beta uh; Kubar <- a Kbar_new;
//                Fubar = dt Kbar_new; Gbar = -(dt/rho) Kbar_new;
//                pbar = Grad_old^T Gbar, with the old metrics' adjoints.
//   (solve)      lambda = A^-T pbar.
//   k_rka_mid    the operator's metrics, -lambda^T dA p, and the right-hand side:
//                with Gbar' = the adjoint of (G_x, G_z) = Grad_old p under lambda^T A p, the
//                adjoint of (u*, w*) is s Gbar' (s = rho/(beta dt)), because the right-hand
//                side is s times the same divergence-and-bed map applied to (u*, w*);
//                u* = u + beta (a K + dt F) spreads it to ubar, Kubar and Fubar.
//   k_rka_force  the forcing (advection, w_sigma, -g D_x eta, nu Div Grad) on the old stage.
//   k_rka_pre    surface update and filter, eta_t, and both geometries back to h and eta.
//
// Metric adjoints are kept per geometry as three rows per x column: abar, bbar, ibar for
// sigma_x = a + b sigma and i = 1/d, plus hxbar, the direct adjoint of h_x (bed rows).
#pragma once
#include <stdint.h>

#include "pmgw_rk.hpp"

namespace pmgw {

struct AdjBufs {
  double *eta1, *keta1;                    // forward recompute: new surface and K_eta
  double *gbo, *gbn;                       // [3][n1d]: abar, bbar, ibar of old / new geometry
  double *hxb, *etatb, *etabf, *sfu;       // [n1d]
  double *y;                               // [6][n1d] scratch rows
  double *p, *pb, *lam, *Fub, *Fwb, *q1, *q2, *q3;   // [n2d]
};

inline int64_t adj_workspace_bytes(int64_t n2d, int64_t n1d) {
  return 2 * rk_align(8 * n1d) + 2 * rk_align(24 * n1d) + 4 * rk_align(8 * n1d) +
         rk_align(48 * n1d) + 8 * rk_align(8 * n2d);
}

inline AdjBufs adj_bufs(char* base, int64_t n2d, int64_t n1d) {
  AdjBufs r;
  int64_t o = 0;
  auto take = [&](int64_t bytes) {
    double* p = reinterpret_cast<double*>(base + o);
    o += rk_align(bytes);
    return p;
  };
  r.eta1 = take(8 * n1d);
  r.keta1 = take(8 * n1d);
  r.gbo = take(24 * n1d);
  r.gbn = take(24 * n1d);
  r.hxb = take(8 * n1d);
  r.etatb = take(8 * n1d);
  r.etabf = take(8 * n1d);
  r.sfu = take(8 * n1d);
  r.y = take(48 * n1d);
  r.p = take(8 * n2d);
  r.pb = take(8 * n2d);
  r.lam = take(8 * n2d);
  r.Fub = take(8 * n2d);
  r.Fwb = take(8 * n2d);
  r.q1 = take(8 * n2d);
  r.q2 = take(8 * n2d);
  r.q3 = take(8 * n2d);
  return r;
}

// The three metric-adjoint rows of one geometry for the tank (row stride nx).
struct MetBar {
  gptr<double> a, b, i;
};

__device__ __forceinline__ MetBar met_bar(double* base, const TankDesc& td) {
  const gptr<double> p = as_global(base + 3 * td.off1d);
  return MetBar{p, p + td.nx, p + 2 * td.nx};
}

// out[j] = sum_l D[l][j] v[l] (the transpose of an NZ x NZ matrix applied to a column).
template <int NZ>
__device__ __forceinline__ double colT(gptr<const double> D, const double* v, int j) {
  double s = 0.0;
#pragma unroll
  for (int l = 0; l < NZ; ++l) s += D[l * NZ + j] * v[l];
  return s;
}

template <int NZ>
__device__ __forceinline__ double colN(gptr<const double> D, const double* v, int j) {
  double s = 0.0;
#pragma unroll
  for (int l = 0; l < NZ; ++l) s += D[j * NZ + l] * v[l];
  return s;
}

// ----------------------------------------------------------------------------- post
template <int NZ>
__global__ void __launch_bounds__(256) k_rka_post(const TankDesc* __restrict__ descs,
                                                  const int32_t* __restrict__ ids, char* ws,
                                                  RkCoef cf, double* ub, double* wb,
                                                  double* Kub, double* Kwb, RkBufs rb,
                                                  AdjBufs ab, int fftb) {
  const TankDesc& td = descs[ids[blockIdx.x]];
  const int nx = td.nx, n = nx * NZ;
  if (td.nz != NZ || nx < 8 || nx > 2048) return;
  Ctx<double> c;
  Lev<double> A;
  rk_ctx(ws, td, fftb, c, A);
  const Geo<double> g = c.g;
  const gptr<const double> sig = A.sig, Ds = A.Ds;
  const gptr<double> u_b = as_global(ub + td.off2d), w_b = as_global(wb + td.off2d);
  const gptr<double> ku_b = as_global(Kub + td.off2d), kw_b = as_global(Kwb + td.off2d);
  const gptr<double> fub = as_global(ab.Fub + td.off2d), fwb = as_global(ab.Fwb + td.off2d);
  const gptr<double> gbx = as_global(rb.r1 + td.off2d), gbz = as_global(rb.r2 + td.off2d);
  const gptr<const double> pp = as_global(ab.p + td.off2d);
  const gptr<double> pb = as_global(ab.pb + td.off2d);
  const gptr<double> t1 = A.t1, t3 = A.t3;
  const gptr<const double> fx = gcp<double>(ws, td.filtx);
  const gptr<const double> fz = gcp<double>(ws, td.filtz);
  const MetBar mo = met_bar(ab.gbo, td), mn = met_bar(ab.gbn, td);
  const gptr<double> hxb = as_global(ab.hxb + td.off1d);
  // uh = F_x F_s^T ubar (F_x is symmetric), in place
  for (int comp = 0; comp < 2; ++comp) {
    const gptr<double> v = comp == 0 ? u_b : w_b;
    for (int i = tid(); i < nx; i += nthr()) {
      double col[NZ];
#pragma unroll
      for (int l = 0; l < NZ; ++l) col[l] = v[l * nx + i];
#pragma unroll 1
      for (int j = 0; j < NZ; ++j) t3[j * nx + i] = colT<NZ>(fz, col, j);
    }
    __syncthreads();
    spectral_rows<double>(NZ, nx, c.log2nx, fftb,
                          [=](int j, int i) { return t3[j * nx + i]; },
                          [=](int k, cpx<double> z) { return filt_mul(fx, nx, k, z); },
                          [=](int j, int i, double z) { v[j * nx + i] = z; });
  }
  const double ir = 1.0 / cf.rho;
  for (int e = tid(); e < n; e += nthr()) {
    const double kun = ku_b[e] + cf.b * u_b[e];
    const double kwn = kw_b[e] + cf.b * w_b[e];
    ku_b[e] = cf.a * kun;
    kw_b[e] = cf.a * kwn;
    fub[e] = cf.dt * kun;
    fwb[e] = cf.dt * kwn;
    gbx[e] = -cf.dt * ir * kun;
    gbz[e] = -cf.dt * ir * kwn;
  }
  col_dsig<double, NZ>(nx, Ds, pp, t1);
  __syncthreads();
  // pbar = -D_x Gbar_x + D_s^T (sx_old Gbar_x + Gbar_z / d_old); old metric adjoints start here
  for (int i = tid(); i < nx; i += nthr()) {
    const double ao = g.ao[i], bo = g.bo[i], ido = g.ido[i];
    double v[NZ];
    double sa = 0.0, sb = 0.0, si = 0.0;
#pragma unroll
    for (int l = 0; l < NZ; ++l) {
      const double gx = gbx[l * nx + i], gz = gbz[l * nx + i], ps = t1[l * nx + i];
      sa += gx * ps;
      sb += sig[l] * gx * ps;
      si += gz * ps;
      v[l] = (ao + bo * sig[l]) * gx + ido * gz;
    }
#pragma unroll 1
    for (int j = 0; j < NZ; ++j) pb[j * nx + i] = colT<NZ>(Ds, v, j);
    mo.a[i] = sa;
    mo.b[i] = sb;
    mo.i[i] = si;
    mn.a[i] = 0.0;
    mn.b[i] = 0.0;
    mn.i[i] = 0.0;
    hxb[i] = 0.0;
  }
  __syncthreads();
  dx_rows<double>(NZ, nx, c.log2nx, c.kfac, fftb,
                  [=](int j, int i) { return gbx[j * nx + i]; },
                  [=](int j, int i, double z) { pb[j * nx + i] -= z; });
}

// ----------------------------------------------------------------------------- mid
template <int NZ>
__global__ void __launch_bounds__(256) k_rka_mid(const TankDesc* __restrict__ descs,
                                                 const int32_t* __restrict__ ids, char* ws,
                                                 RkCoef cf, double* ub, double* wb,
                                                 double* Kub, double* Kwb, RkBufs rb,
                                                 AdjBufs ab, int fftb) {
  const TankDesc& td = descs[ids[blockIdx.x]];
  const int nx = td.nx, n = nx * NZ;
  if (td.nz != NZ || nx < 8 || nx > 2048) return;
  Ctx<double> c;
  Lev<double> A;
  rk_ctx(ws, td, fftb, c, A);
  const Geo<double> g = c.g;
  const gptr<const double> sig = A.sig, Ds = A.Ds;
  const gptr<double> u_b = as_global(ub + td.off2d), w_b = as_global(wb + td.off2d);
  const gptr<double> ku_b = as_global(Kub + td.off2d), kw_b = as_global(Kwb + td.off2d);
  const gptr<double> fub = as_global(ab.Fub + td.off2d), fwb = as_global(ab.Fwb + td.off2d);
  const gptr<const double> pp = as_global(ab.p + td.off2d), lam = as_global(ab.lam + td.off2d);
  const gptr<const double> us = as_global(rb.us + td.off2d), wsv = as_global(rb.ws + td.off2d);
  const gptr<double> q1 = as_global(ab.q1 + td.off2d), q2 = as_global(ab.q2 + td.off2d);
  const gptr<double> q3 = as_global(ab.q3 + td.off2d);
  const gptr<double> t1 = A.t1, t2 = A.t2;
  const MetBar mo = met_bar(ab.gbo, td), mn = met_bar(ab.gbn, td);
  const gptr<double> hxb = as_global(ab.hxb + td.off1d);
  const double s = cf.rho / (cf.b * cf.dt);
  col_dsig<double, NZ>(nx, Ds, pp, t1);
  __syncthreads();
  dx_rows<double>(NZ, nx, c.log2nx, c.kfac, fftb,
                  [=](int j, int i) { return pp[j * nx + i]; },
                  [=](int j, int i, double z) { t2[j * nx + i] = z; });
  for (int i = tid(); i < nx; i += nthr()) {
    const double ao = g.ao[i], bo = g.bo[i], ido = g.ido[i];
    const double an = g.an[i], bn = g.bn[i], idn = g.idn[i], hx = g.hx[i];
    double gx[NZ], gz[NZ], uu[NZ], wv[NZ], li[NZ], sl[NZ], il[NZ];
#pragma unroll
    for (int l = 0; l < NZ; ++l) {
      const double ps = t1[l * nx + i];
      gx[l] = t2[l * nx + i] + (ao + bo * sig[l]) * ps;
      gz[l] = ido * ps;
      uu[l] = us[l * nx + i];
      wv[l] = wsv[l * nx + i];
      li[l] = (l == 0 || l == NZ - 1) ? 0.0 : lam[l * nx + i];
      sl[l] = (an + bn * sig[l]) * li[l];
      il[l] = idn * li[l];
    }
    double sa = 0.0, sb = 0.0, si = 0.0;
#pragma unroll 1
    for (int j = 1; j < NZ - 1; ++j) {
      const double w1 = li[j] * (s * colN<NZ>(Ds, uu, j) - colN<NZ>(Ds, gx, j));
      sa += w1;
      sb += sig[j] * w1;
      si += li[j] * (s * colN<NZ>(Ds, wv, j) - colN<NZ>(Ds, gz, j));
    }
    mn.a[i] += sa;
    mn.b[i] += sb;
    mn.i[i] += si;
    const double lamM = lam[(NZ - 1) * nx + i];
    hxb[i] += lamM * gx[NZ - 1] - s * uu[NZ - 1] * lamM;
#pragma unroll 1
    for (int j = 0; j < NZ; ++j) {
      double cx = colT<NZ>(Ds, sl, j), cz = colT<NZ>(Ds, il, j);
      if (j == NZ - 1) {
        cx -= hx * lamM;
        cz -= lamM;
      }
      q1[j * nx + i] = cx;
      q2[j * nx + i] = cz;
    }
  }
  __syncthreads();
  dx_rows<double>(NZ, nx, c.log2nx, c.kfac, fftb,
                  [=](int j, int i) { return (j == 0 || j == NZ - 1) ? 0.0 : lam[j * nx + i]; },
                  [=](int j, int i, double z) { q3[j * nx + i] = z; });
  for (int i = tid(); i < nx; i += nthr()) {
    double sa = 0.0, sb = 0.0, si = 0.0;
#pragma unroll 1
    for (int j = 0; j < NZ; ++j) {
      const int e = j * nx + i;
      const double gbx = q1[e] - q3[e], gbz = q2[e], ps = t1[e];
      sa += gbx * ps;
      sb += sig[j] * gbx * ps;
      si += gbz * ps;
      const double usb = s * gbx, wsb = s * gbz;
      u_b[e] += usb;
      w_b[e] += wsb;
      ku_b[e] += cf.b * cf.a * usb;
      kw_b[e] += cf.b * cf.a * wsb;
      fub[e] += cf.b * cf.dt * usb;
      fwb[e] += cf.b * cf.dt * wsb;
    }
    mo.a[i] -= sa;
    mo.b[i] -= sb;
    mo.i[i] -= si;
  }
  (void)n;
}

// ----------------------------------------------------------------------------- force
template <int NZ>
__global__ void __launch_bounds__(256) k_rka_force(const TankDesc* __restrict__ descs,
                                                   const int32_t* __restrict__ ids, char* ws,
                                                   RkCoef cf, const double* u, const double* w,
                                                   double* ub, double* wb, RkBufs rb,
                                                   AdjBufs ab, int fftb) {
  const TankDesc& td = descs[ids[blockIdx.x]];
  const int nx = td.nx, n = nx * NZ;
  if (td.nz != NZ || nx < 8 || nx > 2048) return;
  Ctx<double> c;
  Lev<double> A;
  rk_ctx(ws, td, fftb, c, A);
  const Geo<double> g = c.g;
  const gptr<const double> sig = A.sig, Ds = A.Ds;
  const gptr<const double> uu = as_global(u + td.off2d), wwp = as_global(w + td.off2d);
  const gptr<double> u_b = as_global(ub + td.off2d), w_b = as_global(wb + td.off2d);
  const gptr<const double> fub = as_global(ab.Fub + td.off2d), fwb = as_global(ab.Fwb + td.off2d);
  const gptr<const double> et = as_global(rb.etat + td.off1d);
  const gptr<double> etatb = as_global(ab.etatb + td.off1d);
  const gptr<double> etabf = as_global(ab.etabf + td.off1d);
  const gptr<double> sfu = as_global(ab.sfu + td.off1d);
  const gptr<double> q1 = as_global(ab.q1 + td.off2d), q2 = as_global(ab.q2 + td.off2d);
  const gptr<double> q3 = as_global(ab.q3 + td.off2d);
  const gptr<double> t1 = A.t1, t2 = A.t2, t3 = A.t3;
  const MetBar mo = met_bar(ab.gbo, td);
  // advection through w_sigma, the w_sigma definition, and the sums for -g D_x eta;
  // q1 = D_s u, q2 = D_s w first
  col_dsig<double, NZ>(nx, Ds, uu, q1);
  col_dsig<double, NZ>(nx, Ds, wwp, q2);
  __syncthreads();
  for (int i = tid(); i < nx; i += nthr()) {
    const double ao = g.ao[i], bo = g.bo[i], ido = g.ido[i], eti = et[i];
    double au[NZ], aw[NZ];
#pragma unroll
    for (int l = 0; l < NZ; ++l) {
      const int e = l * nx + i;
      const double wsg = -sig[l] * eti * ido + uu[e] * (ao + bo * sig[l]) + wwp[e] * ido;
      au[l] = -wsg * fub[e];
      aw[l] = -wsg * fwb[e];
    }
    double sa = 0.0, sb = 0.0, si = 0.0, se = 0.0, sf = 0.0;
#pragma unroll 1
    for (int j = 0; j < NZ; ++j) {
      const int e = j * nx + i;
      const double fu = fub[e], uj = uu[e], wj = wwp[e];
      const double wsb = -fu * q1[e] - fwb[e] * q2[e];
      const double sx = ao + bo * sig[j];
      u_b[e] += colT<NZ>(Ds, au, j) + wsb * sx;
      w_b[e] += colT<NZ>(Ds, aw, j) + wsb * ido;
      sa += wsb * uj;
      sb += sig[j] * wsb * uj;
      si += wsb * wj - sig[j] * eti * wsb;
      se += -sig[j] * ido * wsb;
      sf += fu;
    }
    mo.a[i] += sa;
    mo.b[i] += sb;
    mo.i[i] += si;
    etatb[i] = se;
    sfu[i] = sf;
  }
  __syncthreads();
  // -u D_x u, -u D_x w: ubar += -Fubar D_x u + D_x(u Fubar) - Fwbar D_x w; wbar += D_x(u Fwbar)
  dx_rows<double>(NZ, nx, c.log2nx, c.kfac, fftb,
                  [=](int j, int i) { return uu[j * nx + i]; },
                  [=](int j, int i, double z) { t2[j * nx + i] = z; });
  dx_rows<double>(NZ, nx, c.log2nx, c.kfac, fftb,
                  [=](int j, int i) { return wwp[j * nx + i]; },
                  [=](int j, int i, double z) { t3[j * nx + i] = z; });
  dx_rows<double>(NZ, nx, c.log2nx, c.kfac, fftb,
                  [=](int j, int i) { return uu[j * nx + i] * fub[j * nx + i]; },
                  [=](int j, int i, double z) { q1[j * nx + i] = z; });
  dx_rows<double>(NZ, nx, c.log2nx, c.kfac, fftb,
                  [=](int j, int i) { return uu[j * nx + i] * fwb[j * nx + i]; },
                  [=](int j, int i, double z) { q2[j * nx + i] = z; });
  for (int e = tid(); e < n; e += nthr()) {
    u_b[e] += -fub[e] * t2[e] + q1[e] - fwb[e] * t3[e];
    w_b[e] += q2[e];
  }
  // -g D_x eta broadcast over the rows: etabar += g D_x (sum_j Fubar_j)
  const double gg = cf.g;
  dx_rows<double>(1, nx, c.log2nx, c.kfac, fftb, [=](int, int i) { return sfu[i]; },
                  [=](int, int i, double z) { etabf[i] = gg * z; });
  // nu Div_old Grad_old f for f = u (D_x f in t2) and f = w (D_x f in t3); t1 = D_s f
  const double nu = cf.nu;
  for (int comp = 0; comp < 2; ++comp) {
    const gptr<const double> f = comp == 0 ? uu : wwp;
    const gptr<const double> fxd = comp == 0 ? gptr<const double>(t2) : gptr<const double>(t3);
    const gptr<const double> fb = comp == 0 ? fub : fwb;
    const gptr<double> outb = comp == 0 ? u_b : w_b;
    col_dsig<double, NZ>(nx, Ds, f, t1);
    __syncthreads();
    // Div^T under Lbar = nu Fbar: metric sums over D_s G_x, D_s G_z (G = Grad f)
    for (int i = tid(); i < nx; i += nthr()) {
      const double ao = g.ao[i], bo = g.bo[i], ido = g.ido[i];
      double gx[NZ], gz[NZ];
#pragma unroll
      for (int l = 0; l < NZ; ++l) {
        const double fs = t1[l * nx + i];
        gx[l] = fxd[l * nx + i] + (ao + bo * sig[l]) * fs;
        gz[l] = ido * fs;
      }
      double sa = 0.0, sb = 0.0, si = 0.0;
#pragma unroll 1
      for (int j = 0; j < NZ; ++j) {
        const double lb = nu * fb[j * nx + i];
        const double dgx = colN<NZ>(Ds, gx, j);
        sa += lb * dgx;
        sb += sig[j] * lb * dgx;
        si += lb * colN<NZ>(Ds, gz, j);
      }
      mo.a[i] += sa;
      mo.b[i] += sb;
      mo.i[i] += si;
    }
    // the D_s^T parts of Gbar_x, Gbar_z
    for (int i = tid(); i < nx; i += nthr()) {
      const double ao = g.ao[i], bo = g.bo[i], ido = g.ido[i];
      double sl[NZ], il[NZ];
#pragma unroll
      for (int l = 0; l < NZ; ++l) {
        const double lb = nu * fb[l * nx + i];
        sl[l] = (ao + bo * sig[l]) * lb;
        il[l] = ido * lb;
      }
#pragma unroll 1
      for (int j = 0; j < NZ; ++j) {
        q1[j * nx + i] = colT<NZ>(Ds, sl, j);
        q2[j * nx + i] = colT<NZ>(Ds, il, j);
      }
    }
    __syncthreads();
    dx_rows<double>(NZ, nx, c.log2nx, c.kfac, fftb,
                    [=](int j, int i) { return nu * fb[j * nx + i]; },
                    [=](int j, int i, double z) { q3[j * nx + i] = z; });
    // Gbar_x = q1 - q3, Gbar_z = q2; Grad^T: fbar += -D_x Gbar_x + D_s^T (sx Gbar_x + i Gbar_z)
    for (int i = tid(); i < nx; i += nthr()) {
      const double ao = g.ao[i], bo = g.bo[i], ido = g.ido[i];
      double v[NZ];
      double sa = 0.0, sb = 0.0, si = 0.0;
#pragma unroll
      for (int l = 0; l < NZ; ++l) {
        const int e = l * nx + i;
        const double fs = t1[e];
        const double gbx = q1[e] - q3[e], gbz = q2[e];
        sa += gbx * fs;
        sb += sig[l] * gbx * fs;
        si += gbz * fs;
        v[l] = (ao + bo * sig[l]) * gbx + ido * gbz;
        q1[e] = gbx;
      }
#pragma unroll 1
      for (int j = 0; j < NZ; ++j) outb[j * nx + i] += colT<NZ>(Ds, v, j);
      mo.a[i] += sa;
      mo.b[i] += sb;
      mo.i[i] += si;
    }
    __syncthreads();
    dx_rows<double>(NZ, nx, c.log2nx, c.kfac, fftb,
                    [=](int j, int i) { return q1[j * nx + i]; },
                    [=](int j, int i, double z) { outb[j * nx + i] -= z; });
  }
}

// ----------------------------------------------------------------------------- pre
// Geometry adjoint: with a = h_x/d, b = -d_x/d, i = 1/d, d = h + eta,
//   hx~ = abar i + hxbar, dxbar = -bbar i, dbar = (-abar h_x + bbar d_x - ibar) i^2 - D_x dxbar,
//   hbar = dbar - D_x hx~, etabar = dbar   (D_x^T = -D_x).
template <int NZ>
__global__ void __launch_bounds__(256) k_rka_pre(const TankDesc* __restrict__ descs,
                                                 const int32_t* __restrict__ ids, char* ws,
                                                 RkCoef cf, const double* u, double* ub,
                                                 double* wb, double* etab, double* Ketab,
                                                 double* hbar, RkBufs rb, AdjBufs ab, int fftb) {
  const TankDesc& td = descs[ids[blockIdx.x]];
  const int nx = td.nx;
  if (td.nz != NZ || nx < 8 || nx > 2048) return;
  Ctx<double> c;
  Lev<double> A;
  rk_ctx(ws, td, fftb, c, A);
  const Geo<double> g = c.g;
  const gptr<const double> u0 = as_global(u + td.off2d);
  const gptr<double> u_b = as_global(ub + td.off2d), w_b = as_global(wb + td.off2d);
  const gptr<double> e_b = as_global(etab + td.off1d), ke_b = as_global(Ketab + td.off1d);
  const gptr<double> h_b = as_global(hbar + td.off1d);
  const gptr<const double> ex = as_global(rb.etax + td.off1d);
  const gptr<const double> etatb = as_global(ab.etatb + td.off1d);
  const gptr<const double> etabf = as_global(ab.etabf + td.off1d);
  const gptr<const double> hxbp = as_global(ab.hxb + td.off1d);
  const gptr<double> y = as_global(ab.y + 6 * td.off1d);
  const MetBar mo = met_bar(ab.gbo, td), mn = met_bar(ab.gbn, td);
  const gptr<const double> fx = gcp<double>(ws, td.filtx);
  // rows of y: 0 dxbar_new, 1 hx~_new, 2 dxbar_old, 3 hx~_old, 4 dbar_new (partial),
  // 5 dbar_old (partial)
  for (int i = tid(); i < nx; i += nthr()) {
    const double hx = g.hx[i];
    const double idn = g.idn[i], dxn = -g.bn[i] / idn;
    const double ido = g.ido[i], dxo = -g.bo[i] / ido;
    y[i] = -mn.b[i] * idn;
    y[nx + i] = mn.a[i] * idn;
    y[2 * nx + i] = -mo.b[i] * ido;
    y[3 * nx + i] = mo.a[i] * ido + hxbp[i];
    y[4 * nx + i] = (-mn.a[i] * hx + mn.b[i] * dxn - mn.i[i]) * idn * idn;
    y[5 * nx + i] = (-mo.a[i] * hx + mo.b[i] * dxo - mo.i[i]) * ido * ido;
  }
  __syncthreads();
  // y[r] <- D_x y[r] for r = 0..3
  dx_rows<double>(4, nx, c.log2nx, c.kfac, fftb,
                  [=](int r, int i) { return y[r * nx + i]; },
                  [=](int r, int i, double z) { y[r * nx + i] = z; });
  // dbar_new (etabar of the new surface) -> row 4; e1bar = F_x (etabar_out + dbar_new) -> row 0
  for (int i = tid(); i < nx; i += nthr()) {
    const double dbn = y[4 * nx + i] - y[i];
    const double dbo = y[5 * nx + i] - y[2 * nx + i];
    h_b[i] += dbn - y[nx + i] + dbo - y[3 * nx + i];
    y[4 * nx + i] = dbn;
    y[5 * nx + i] = dbo;
  }
  __syncthreads();
  spectral_rows<double>(1, nx, c.log2nx, fftb,
                        [=](int, int i) { return e_b[i] + y[4 * nx + i]; },
                        [=](int k, cpx<double> z) { return filt_mul(fx, nx, k, z); },
                        [=](int, int i, double z) { y[i] = z; });
  // K_eta and eta_t; eta_t = -u~ D_x eta + w~
  for (int i = tid(); i < nx; i += nthr()) {
    const double e1b = y[i];
    const double ken = ke_b[i] + cf.b * e1b;
    ke_b[i] = cf.a * ken;
    const double etb = etatb[i] + cf.dt * ken;
    u_b[i] += -ex[i] * etb;
    w_b[i] += etb;
    y[nx + i] = u0[i] * etb;
  }
  __syncthreads();
  dx_rows<double>(1, nx, c.log2nx, c.kfac, fftb, [=](int, int i) { return y[nx + i]; },
                  [=](int, int i, double z) { y[2 * nx + i] = z; });
  for (int i = tid(); i < nx; i += nthr())
    e_b[i] = y[i] + etabf[i] + y[2 * nx + i] + y[5 * nx + i];
}

}  // namespace pmgw

// Set-up kernels of the p-multigrid Poisson library, launched only by the host API: a fill
// kernel, the stage solve's initial-guess kernel, the geometry/metrics kernel and the
// block-inversion kernels.
#pragma once
#include "pmgw_kernels.hpp"
#include "pmgw_rk.hpp"

namespace pmgw {

// a[e] = v for e < n (grid-stride).
__global__ void __launch_bounds__(256) k_fill(double* a, int64_t n, double v) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    a[e] = v;
}

// Initial guess of a stage's pressure solve from the recorded history (opts.guess_steps):
// store the incoming p (the previous stage's result) into slot `store` of the history, then
// replace p by sum_i c_i H[src_i] (stage k's recorded steps). Elementwise over the n2d points
// of every tank; the stored slot belongs to another stage than the sources.
struct GuessArgs {
  int store;      // history slot receiving p, or -1
  int nsrc;       // number of source slots (0: p is left as is)
  int src[5];
  double c[5];
  double* eprev;  // the previous call's extrapolation (n2d doubles), or null
  int corr;       // add the previous call's extrapolation error p - eprev
  int save;       // keep this call's extrapolation in eprev
};

// p holds the previous call's result on entry: it is recorded (store), and replaced by the
// extrapolation E = sum_i c_i hist[src_i] (nsrc > 0), plus p - eprev with corr.
__global__ void __launch_bounds__(256) k_guess(double* p, double* hist, int64_t n2d,
                                               GuessArgs g) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n2d;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double v = p[e];
    if (g.store >= 0) hist[g.store * n2d + e] = v;
    if (g.nsrc > 0) {
      double s = 0.0;
      for (int i = 0; i < g.nsrc; ++i) s += g.c[i] * hist[g.src[i] * n2d + e];
      const double corr = g.corr ? v - g.eprev[e] : 0.0;
      if (g.save) g.eprev[e] = s;
      p[e] = s + corr;
    }
  }
}

// ----------------------------------------------------------------------------- relaxation zones
//
// Wave-flume relaxation (paper Sec. 5, harmonic generation over a submerged bar). The target of
// tank t is a steady stream-function wave with coefficients coef + t (2 nm + 6) =
// [k, c, ubar, h0, x0, E_0..E_nm, B_1..B_nm]: with X = x - x0 - c t and s = a S(x),
// eta = s sum_q E_q cos(q k X) and, on the target's sigma grid zeta_j = sigma_j (h0 + eta),
// u = s ((c - ubar) + sum_q q k B_q ch_q cos(q k X)), w = s sum_q q k B_q sh_q sin(q k X) with
// ch_q, sh_q = exp(q k (zeta - h0)) (1 +- exp(-2 q k zeta)) / (1 + exp(-2 q k h0))
// (= cosh(q k zeta) / cosh(q k h0) and sinh(q k zeta) / cosh(q k h0), without overflow).
constexpr int kStreamMaxModes = 64;

// One workgroup per (tank, row); row 0 also writes eta.
__global__ void __launch_bounds__(256) k_stream_target(const TankDesc* __restrict__ descs,
                                                       char* ws, const double* __restrict__ coef,
                                                       int nm, double t, double a,
                                                       const double* __restrict__ win, double* u,
                                                       double* w, double* eta) {
  const TankDesc& td = descs[blockIdx.x];
  const int nx = td.nx, j = blockIdx.y;
  if (j >= td.nz) return;
  const double* cf = coef + (int64_t)blockIdx.x * (2 * nm + 6);
  const double k = cf[0], c = cf[1], ub = cf[2], h0 = cf[3], x0 = cf[4];
  const double* E = cf + 5;
  const double* B = cf + 6 + nm;
  const double sg = cp<double>(ws, td.lev[0].sig[0])[j];
  const double dx = td.L / nx;
  for (int i = tid(); i < nx; i += nthr()) {
    const double X = i * dx - x0 - c * t;
    const double s = a * win[td.off1d + i];
    double e = 0.0;
    for (int q = 0; q <= nm; ++q) e += E[q] * cos(q * k * X);
    e *= s;
    const double zeta = sg * (h0 + e);
    double su = 0.0, sw = 0.0;
    for (int q = 1; q <= nm; ++q) {
      const double kq = q * k;
      const double up = exp(kq * (zeta - h0)), em = exp(-2.0 * kq * zeta);
      const double den = 1.0 + exp(-2.0 * kq * h0);
      double sn, cs;
      sincos(kq * X, &sn, &cs);
      su += kq * B[q - 1] * (up * (1.0 + em) / den) * cs;
      sw += kq * B[q - 1] * (up * (1.0 - em) / den) * sn;
    }
    const int64_t o = td.off2d + (int64_t)j * nx + i;
    u[o] = s * ((c - ub) + su);
    w[o] = s * sw;
    if (j == 0) eta[td.off1d + i] = e;
  }
}

// q <- q + r (q_target - q) for u, w (every row) and eta, r per column; grid (tanks, chunks).
__global__ void __launch_bounds__(256) k_relax(const TankDesc* __restrict__ descs,
                                               const double* __restrict__ r,
                                               const double* __restrict__ ut,
                                               const double* __restrict__ wt,
                                               const double* __restrict__ et, double* u,
                                               double* w, double* eta) {
  const TankDesc& td = descs[blockIdx.x];
  const int nx = td.nx, n = nx * td.nz;
  for (int e = blockIdx.y * blockDim.x + threadIdx.x; e < n; e += gridDim.y * blockDim.x) {
    const int i = e % nx;
    const double rr = r[td.off1d + i];
    const int64_t o = td.off2d + e;
    u[o] = u[o] + rr * (ut[o] - u[o]);
    w[o] = w[o] + rr * (wt[o] - w[o]);
    if (e < nx) {
      const int64_t o1 = td.off1d + e;
      eta[o1] = eta[o1] + rr * (et[o1] - eta[o1]);
    }
  }
}

// ----------------------------------------------------------------------------- geometry kernel

constexpr int kGeoFftBytes = 32768;   // the geometry kernel: 2 x 32 KB of FFT LDS + twiddles
//
// One workgroup per tank: copies h, eta_old, eta_new, checks d > 0, and forms the
// sigma-metrics of paper eq. 1_Scoef for both geometries: sigma_x = a + b sigma with
// a = h_x / d, b = -d_x / d, and 1/d; h_x and d_x by the FFT derivative. Also the x-averages
// cbar = <1/(d_o d_n)> and ebar = <(1 + h_x^2)/d_o> of the flat-mode operator, the mode-step
// damping factor min(1, 2 / (1 + (r/2)^0.4)) with r = max c / min c, c = 1/(d_o d_n), and float32
// copies for mixed plans.
// The metrics of one tank (every thread of the workgroup calls it); red: 16 doubles of LDS.
__device__ __forceinline__ void geometry_tank(const TankDesc& td, char* ws, const double* h,
                                              const double* eo, const double* en, double* red) {
  const int nx = td.nx;
  double* G = mp<double>(ws, td.geo64);
  const double* hh = h + td.off1d;
  const double* e0 = eo + td.off1d;
  const double* e1 = en + td.off1d;
  int bad = 0;
  for (int i = tid(); i < nx; i += nthr()) {
    const double a = hh[i], b = e0[i], c = e1[i];
    G[GEO_H * nx + i] = a;
    G[GEO_EO * nx + i] = b;
    G[GEO_EN * nx + i] = c;
    const double d0 = a + b, d1 = a + c;
    if (!(d0 > 0.0) || !(d1 > 0.0) || !isfinite(d0) || !isfinite(d1)) bad = 1;
  }
  stage_twiddles(gcp<cpx<double>>(ws, td.tw[0]), gcp<cpx<float>>(ws, td.tw[1]), nx,
                 kGeoFftBytes);
  // rows: 0 = h, 1 = d_old, 2 = d_new  ->  h_x (GEO_HX), d_x old (GEO_BO), d_x new (GEO_BN)
  dx_rows<double>(3, nx, td.log2nx, td.kfac, kGeoFftBytes,
                  [=](int j, int i) {
                    return j == 0 ? G[GEO_H * nx + i]
                                  : G[GEO_H * nx + i] + G[(j == 1 ? GEO_EO : GEO_EN) * nx + i];
                  },
                  [=](int j, int i, double v) {
                    G[(j == 0 ? GEO_HX : (j == 1 ? GEO_BO : GEO_BN)) * nx + i] = v;
                  });
  double sc = 0.0, se = 0.0, cmax = 0.0, icmax = 0.0;
  float* G32 = mp<float>(ws, td.geo32);
  for (int i = tid(); i < nx; i += nthr()) {
    const double hx = G[GEO_HX * nx + i];
    const double ido = 1.0 / (G[GEO_H * nx + i] + G[GEO_EO * nx + i]);
    const double idn = 1.0 / (G[GEO_H * nx + i] + G[GEO_EN * nx + i]);
    const double ao = hx * ido, bo = -G[GEO_BO * nx + i] * ido;
    const double an = hx * idn, bn = -G[GEO_BN * nx + i] * idn;
    G[GEO_AO * nx + i] = ao; G[GEO_BO * nx + i] = bo; G[GEO_IDO * nx + i] = ido;
    G[GEO_AN * nx + i] = an; G[GEO_BN * nx + i] = bn; G[GEO_IDN * nx + i] = idn;
    G32[i] = (float)ao; G32[nx + i] = (float)bo; G32[2 * nx + i] = (float)ido;
    G32[3 * nx + i] = (float)an; G32[4 * nx + i] = (float)bn; G32[5 * nx + i] = (float)idn;
    G32[6 * nx + i] = (float)hx;
    sc += ido * idn;
    se += (1.0 + hx * hx) * ido;
    cmax = fmax(cmax, fabs(ido * idn));
    icmax = fmax(icmax, 1.0 / fabs(ido * idn));
  }
  sc = block_sum(sc, red);
  se = block_sum(se, red);
  cmax = block_max(cmax, red);
  icmax = block_max(icmax, red);
  const double nb = block_sum((double)bad, red);
  if (tid() == 0) {
    double* S = mp<double>(ws, td.scal);
    S[0] = sc / nx;
    S[1] = se / nx;
    *reinterpret_cast<int32_t*>(S + 2) = nb > 0.0 ? ST_EGEOM : ST_OK;
    // mode-step damping: r = max c / min c with c = 1/(d_o d_n); min(1, 2 / (1 + (r/2)^0.4))
    const double r = cmax * icmax;
    S[3] = fmin(1.0, 2.0 / (1.0 + pow(0.5 * r, 0.4)));
  }
}

__global__ void __launch_bounds__(256) k_geometry(const TankDesc* __restrict__ descs, char* ws,
                                                  const double* h, const double* eo,
                                                  const double* en) {
  __shared__ double red[16];
  const TankDesc& td = descs[blockIdx.x];
  if (td.nx < 8 || td.nx > 2048) return;
  geometry_tank(td, ws, h, eo, en, red);
}

// The surface part of a stage and then the metrics of the old and new surface, one workgroup
// per tank (rk4_stage's first launch; the same arithmetic as k_rk_pre followed by k_geometry).
// The linearised model's metrics use the still-water surface z1 for both geometries.
__global__ void __launch_bounds__(256) k_rk_pre_geometry(const TankDesc* __restrict__ descs,
                                                         char* ws, RkCoef cf, const double* h,
                                                         const double* u, const double* w,
                                                         double* eta, double* Keta, RkBufs rb) {
  __shared__ double red[16];
  const TankDesc& td = descs[blockIdx.x];
  if (td.nx < 8 || td.nx > 2048) return;
  rk_pre_tank(td, ws, cf, u, w, eta, Keta, rb, kGeoFftBytes);
  __syncthreads();
  const double* eo = cf.lin ? rb.z1 : rb.eo;
  const double* en = cf.lin ? rb.z1 : eta;
  geometry_tank(td, ws, h, eo, en, red);
}

// ----------------------------------------------------------------------------- block kernel
//
// One 64-thread workgroup per block. Builds, in float64, either the column block B_i (the
// x-diagonal block of the level operator at column i: interior rows
// cxx I + diag(sx_n) D_s diag(sx_o) D_s + D_s^2/(d_n d_o), row 0 = e_0, bed row
// -(h_x sx_o[M] + 1/d_o) (D_s)_M) or the flat-mode block of mode k (interior
// -kappa_k^2 I + cbar D_s^2, row 0 = e_0, bed row -ebar (D_s)_M), inverts it by Gauss-Jordan
// with partial pivoting in LDS, and stores the inverse in the plan's V-cycle precision.
template <typename TV>
__global__ void __launch_bounds__(64) k_blocks(const TankDesc* __restrict__ descs,
                                               const BlockJob* __restrict__ jobs, int njobs,
                                               char* ws) {
  __shared__ double A[kMaxNz][kMaxNz + 1];
  __shared__ int piv[kMaxNz];
  const int64_t b = blockIdx.x;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].first <= b) lo = mid; else hi = mid - 1;
  }
  const BlockJob jb = jobs[lo];
  const int idx = (int)(b - jb.first);
  const TankDesc& td = descs[jb.tank];
  const LevelDesc& ld = td.lev[jb.level];
  const int nz = ld.nz, M = nz - 1, nx = td.nx;
  if (nz < 3 || nz > kMaxNz || nx < 8 || nx > 2048 || idx < 0 || idx > nx) return;
  const int t = tid();
  const double* Ds = cp<double>(ws, ld.ds[0]);
  const double* sig = cp<double>(ws, ld.sig[0]);
  // S2 = D_s D_s and SS = D_s diag(sigma) D_s: with sx = a + b sigma the interior rows are
  // sum_m (D_s)_jm (D_s)_mc (sxn_j sxo_m + 1/(d_n d_o)) = (sxn_j a_o + 1/(d_n d_o)) S2_jc
  // + sxn_j b_o SS_jc (plus c_xx on the diagonal of a column block)
  const double* S2 = cp<double>(ws, ld.dss);
  const double* SS = S2 + nz * nz;
  if (jb.kind == 0) {
    const double* G = cp<double>(ws, td.geo64);
    const int i = idx;
    const double ao = G[GEO_AO * nx + i], bo = G[GEO_BO * nx + i], ido = G[GEO_IDO * nx + i];
    const double an = G[GEO_AN * nx + i], bn = G[GEO_BN * nx + i], idn = G[GEO_IDN * nx + i];
    const double hx = G[GEO_HX * nx + i];
    const double bedc = -(hx * (ao + bo * sig[M]) + ido);
    for (int e = t; e < nz * nz; e += 64) {
      const int j = e / nz, c = e - j * nz;
      double v;
      if (j == 0) {
        v = (c == 0) ? 1.0 : 0.0;
      } else if (j == M) {
        v = bedc * Ds[M * nz + c];
      } else {
        const double sxn = an + bn * sig[j];
        v = (sxn * ao + idn * ido) * S2[e] + sxn * bo * SS[e] + ((c == j) ? td.cxx : 0.0);
      }
      A[j][c] = v;
    }
  } else {
    const double* S = cp<double>(ws, td.scal);
    const double cbar = S[0], ebar = S[1];
    const int k = idx;
    const double kap = (k == nx / 2) ? 0.0 : td.kfac * (double)k;
    for (int e = t; e < nz * nz; e += 64) {
      const int j = e / nz, c = e - j * nz;
      double v;
      if (j == 0) v = (c == 0) ? 1.0 : 0.0;
      else if (j == M) v = -ebar * Ds[M * nz + c];
      else v = cbar * S2[e] - ((c == j) ? kap * kap : 0.0);
      A[j][c] = v;
    }
  }
  __syncthreads();
  // In-place Gauss-Jordan inversion with row pivoting; thread t owns row t (or column t).
  for (int k = 0; k < nz; ++k) {
    // pivot: largest |A[t][k]| over t in [k, nz); NaN ranks highest so that every lane agrees
    double v = -1.0;
    if (t >= k && t < nz) {
      v = fabs(A[t][k]);
      if (!(v >= 0.0)) v = INFINITY;
    }
    int id = t;
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(v, o, 64);
      const int oi = __shfl_xor(id, o, 64);
      if (ov > v || (ov == v && oi < id)) { v = ov; id = oi; }
    }
    const int p = min(max(id, k), nz - 1);
    if (p != k && t < nz) {
      const double tmp = A[k][t];
      A[k][t] = A[p][t];
      A[p][t] = tmp;
    }
    if (t == 0) piv[k] = p;
    __syncthreads();
    const double inv = 1.0 / A[k][k];
    if (t < nz && t != k) {
      const double fr = A[t][k] * inv;
      for (int c = 0; c < nz; ++c)
        if (c != k) A[t][c] -= fr * A[k][c];
      A[t][k] = -fr;
    }
    __syncthreads();
    if (t < nz) A[k][t] = (t == k) ? inv : A[k][t] * inv;
    __syncthreads();
  }
  for (int k = nz - 1; k >= 0; --k) {
    const int p = piv[k];
    if (p != k && t < nz) {
      const double tmp = A[t][k];
      A[t][k] = A[t][p];
      A[t][p] = tmp;
    }
    __syncthreads();
  }
  if (jb.kind == 0) {
    TV* out = mp<TV>(ws, ld.colinv);
    for (int e = t; e < nz * nz; e += 64) out[(int64_t)e * nx + idx] = (TV)A[e / nz][e % nz];
  } else {
    const int nh = nx / 2 + 1;
    TV* out = mp<TV>(ws, ld.modeinv);
    for (int e = t; e < nz * nz; e += 64) out[(int64_t)e * nh + idx] = (TV)A[e / nz][e % nz];
  }
}

}  // namespace pmgw

namespace pmgw {

// ----------------------------------------------------------------------------- coarsest level
//
// Direct solve of the coarsest level (paper Alg. 1: the order-2 problem is solved exactly).
// The order-2 operator A_c (rows 0, 1, 2 = sigma 1, 1/2, 0, every row coupling all Nx columns
// through D_x) has the identity as its Dirichlet row 0, so with y = [x_1; x_2] it reduces to
// B y = [f_1; f_2] - C f_0, C = the coupling of rows 1, 2 to row 0. One workgroup per tank:
//   1. c1 = D_x e_0 and c2 = D_x c1, the first columns of the circulant D_x and D_x^2 (by the
//      same FFT derivative as the operator);
//   2. W = [-C | B] ([2 nx][3 nx], float64) assembled entry by entry from the level's D_sigma,
//      sigma nodes and the old/new metrics, with the operator's composite form: row 1 is
//      Div^new Grad^old, row 2 the bed condition -(h_x G_x + G_z);
//   3. Gauss-Jordan elimination with partial pivoting on the B columns, the -C columns carried
//      along as extra right-hand sides: W becomes [Q | B^-1], Q = -B^-1 C;
//   4. the transpose W^T, which the forward apply reads coalesced.
// A zero or non-finite pivot marks the tank ENAN (its later solves report it).

constexpr int kCoarseThreads = 1024;

__global__ void __launch_bounds__(kCoarseThreads) k_coarse_setup(const TankDesc* __restrict__ descs,
                                                                 char* ws) {
  __shared__ double prow[3 * kCoarseExactMaxNx];
  __shared__ double pcol[2 * kCoarseExactMaxNx];
  __shared__ double c1[kCoarseExactMaxNx], c2[kCoarseExactMaxNx];
  __shared__ int piv[2 * kCoarseExactMaxNx];
  __shared__ double redv[kCoarseThreads / 64];
  __shared__ int redi[kCoarseThreads / 64];
  const TankDesc td = descs[blockIdx.x];
  const int nx = td.nx;
  if (!td.cw || !td.cwt || nx < 8 || nx > kCoarseExactMaxNx) return;
  int32_t* status = reinterpret_cast<int32_t*>(mp<double>(ws, td.scal) + 2);
  if (*status != ST_OK) return;
  const int n2 = 2 * nx, n3 = 3 * nx;
  const int lane = tid() & 63, wv = tid() >> 6, nw = nthr() >> 6;

  stage_twiddles(gcp<cpx<double>>(ws, td.tw[0]), gcp<cpx<float>>(ws, td.tw[1]), nx,
                 kGeoFftBytes);
  double* c1p = c1;
  double* c2p = c2;
  dx_rows<double>(1, nx, td.log2nx, td.kfac, kGeoFftBytes,
                  [=](int, int i) { return i == 0 ? 1.0 : 0.0; },
                  [=](int, int i, double v) { c1p[i] = v; });
  dx_rows<double>(1, nx, td.log2nx, td.kfac, kGeoFftBytes, [=](int, int i) { return c1p[i]; },
                  [=](int, int i, double v) { c2p[i] = v; });

  const LevelDesc& lc = td.lev[td.nlev - 1];
  const double* Ds = cp<double>(ws, lc.ds[0]);
  const double* sg = cp<double>(ws, lc.sig[0]);
  const double* G = cp<double>(ws, td.geo64);
  const double* ao = G + GEO_AO * nx;
  const double* bo = G + GEO_BO * nx;
  const double* ido = G + GEO_IDO * nx;
  const double* an = G + GEO_AN * nx;
  const double* bn = G + GEO_BN * nx;
  const double* idn = G + GEO_IDN * nx;
  const double* hx = G + GEO_HX * nx;
  double* W = mp<double>(ws, td.cw);
  double* WT = mp<double>(ws, td.cwt);
  const int msk = nx - 1;

  // entry of A_c at equation (j, i), unknown (m, k), j in {1, 2}
  auto entry = [&](int j, int i, int m, int k) -> double {
    const double dxik = c1p[(i - k) & msk];
    double v = 0.0;
    if (j == 1) {
      if (m == 1) v += c2p[(i - k) & msk];
      const double sxo1k = ao[k] + bo[k] * sg[1];
      const double sxn1 = an[i] + bn[i] * sg[1];
      v += dxik * Ds[3 + m] * (sxo1k + sxn1);
      if (i == k) {
        double s = 0.0, t = 0.0;
        for (int l = 0; l < 3; ++l) {
          s += Ds[3 + l] * (ao[i] + bo[i] * sg[l]) * Ds[3 * l + m];
          t += Ds[3 + l] * Ds[3 * l + m];
        }
        v += sxn1 * s + idn[i] * ido[i] * t;
      }
    } else {
      if (m == 2) v -= hx[i] * dxik;
      if (i == k) v -= (hx[i] * (ao[i] + bo[i] * sg[2]) + ido[i]) * Ds[6 + m];
    }
    return v;
  };
  for (int r = wv; r < n2; r += nw) {
    const int j = 1 + r / nx, i = r & msk;
    for (int c = lane; c < n3; c += 64) {
      const int m = c / nx, k = c & msk;
      const double a = entry(j, i, m, k);
      W[(int64_t)r * n3 + c] = (m == 0) ? -a : a;
    }
  }
  __syncthreads();

  bool bad = false;
  for (int k = 0; k < n2; ++k) {
    const int pc = nx + k;
    // pivot row: largest |W[t][pc]| over t >= k, the smaller row on ties, NaN ranks highest
    double best = -1.0;
    int bi = n2;
    for (int t = k + tid(); t < n2; t += nthr()) {
      double v = fabs(W[(int64_t)t * n3 + pc]);
      if (!(v >= 0.0)) v = INFINITY;
      if (v > best) { best = v; bi = t; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    if (lane == 0) { redv[wv] = best; redi[wv] = bi; }
    __syncthreads();
    best = redv[0];
    bi = redi[0];
    for (int q = 1; q < nw; ++q)
      if (redv[q] > best || (redv[q] == best && redi[q] < bi)) { best = redv[q]; bi = redi[q]; }
    if (!(best > 0.0) || !isfinite(best) || bi >= n2) { bad = true; break; }
    const int p = bi;
    // swap rows p and k; the pivot row goes to LDS
    for (int c = tid(); c < n3; c += nthr()) {
      const double a = W[(int64_t)k * n3 + c], b = W[(int64_t)p * n3 + c];
      if (p != k) W[(int64_t)p * n3 + c] = a;
      prow[c] = b;
    }
    if (tid() == 0) piv[k] = p;
    __syncthreads();
    for (int t = tid(); t < n2; t += nthr()) pcol[t] = (t == k) ? 0.0 : W[(int64_t)t * n3 + pc];
    __syncthreads();
    const double inv = 1.0 / prow[pc];
    for (int t = wv; t < n2; t += nw) {
      double* row = W + (int64_t)t * n3;
      if (t == k) {
        for (int c = lane; c < n3; c += 64) row[c] = (c == pc) ? inv : prow[c] * inv;
      } else {
        const double fr = pcol[t] * inv;
        for (int c = lane; c < n3; c += 64) row[c] = (c == pc) ? -fr : row[c] - fr * prow[c];
      }
    }
    __syncthreads();
  }
  if (bad) {
    if (tid() == 0) *status = ST_ENAN;
    return;
  }
  // undo the row pivoting on the columns of the inverse, last pivot first
  for (int k = n2 - 1; k >= 0; --k) {
    const int p = piv[k];
    if (p != k) {
      for (int t = tid(); t < n2; t += nthr()) {
        double* row = W + (int64_t)t * n3 + nx;
        const double a = row[k];
        row[k] = row[p];
        row[p] = a;
      }
    }
    __syncthreads();
  }
  for (int c = wv; c < n3; c += nw)
    for (int t = lane; t < n2; t += 64) WT[(int64_t)c * n2 + t] = W[(int64_t)t * n3 + c];
}

}  // namespace pmgw

namespace pmgw {

// ----------------------------------------------------------------------------- bed line
//
// Inverse of the bed row's own block of the operator on level l (the bed-line step of the
// smoother): L_b = -(diag(h_x) D_x + diag(q (D_sigma)_MM)), q = h_x sigma_x^old[M] + 1/d_old,
// Nx x Nx, D_x circulant with first column c1 = D_x e_0 (the operator's FFT derivative). One
// workgroup per (tank, level): assemble L_b in the tank's float64 buffer, invert it in place by
// Gauss-Jordan with partial pivoting (pivot row and column in LDS), undo the pivoting, store the
// transpose in place (the apply reads it coalesced) and, for mixed plans, a float32 copy. A zero
// or non-finite pivot marks the tank ENAN.

constexpr int kBedLineThreads = 1024;

__global__ void __launch_bounds__(kBedLineThreads) k_bedline_setup(
    const TankDesc* __restrict__ descs, char* ws) {
  __shared__ double prow[kBedLineMaxNx];
  __shared__ double pcol[kBedLineMaxNx];
  __shared__ double c1[kBedLineMaxNx];
  __shared__ int piv[kBedLineMaxNx];
  __shared__ double redv[kBedLineThreads / 64];
  __shared__ int redi[kBedLineThreads / 64];
  const TankDesc td = descs[blockIdx.x];
  const int l = blockIdx.y;
  const int nx = td.nx;
  if (l >= td.nlev || nx < 8 || nx > kBedLineMaxNx) return;
  const LevelDesc& lv = td.lev[l];
  if (!lv.bedinv) return;
  int32_t* status = reinterpret_cast<int32_t*>(mp<double>(ws, td.scal) + 2);
  if (*status != ST_OK) return;
  const int lane = tid() & 63, wv = tid() >> 6, nw = nthr() >> 6;
  const int nz = lv.nz, M = nz - 1;

  stage_twiddles(gcp<cpx<double>>(ws, td.tw[0]), gcp<cpx<float>>(ws, td.tw[1]), nx,
                 kGeoFftBytes);
  double* c1p = c1;
  dx_rows<double>(1, nx, td.log2nx, td.kfac, kGeoFftBytes,
                  [=](int, int i) { return i == 0 ? 1.0 : 0.0; },
                  [=](int, int i, double v) { c1p[i] = v; });
  __syncthreads();

  const double dsmm = cp<double>(ws, lv.ds[0])[M * nz + M];
  const double sgm = cp<double>(ws, lv.sig[0])[M];
  const double* G = cp<double>(ws, td.geo64);
  const double* ao = G + GEO_AO * nx;
  const double* bo = G + GEO_BO * nx;
  const double* ido = G + GEO_IDO * nx;
  const double* hx = G + GEO_HX * nx;
  double* W = mp<double>(ws, lv.bedinv);
  const int msk = nx - 1;
  for (int r = wv; r < nx; r += nw) {
    const double q = (hx[r] * (ao[r] + bo[r] * sgm) + ido[r]) * dsmm;
    for (int c = lane; c < nx; c += 64)
      W[(int64_t)r * nx + c] = -(hx[r] * c1p[(r - c) & msk] + (r == c ? q : 0.0));
  }
  __syncthreads();

  bool bad = false;
  for (int k = 0; k < nx; ++k) {
    // pivot row: largest |W[t][k]| over t >= k, the smaller row on ties, NaN ranks highest
    double best = -1.0;
    int bi = nx;
    for (int t = k + tid(); t < nx; t += nthr()) {
      double v = fabs(W[(int64_t)t * nx + k]);
      if (!(v >= 0.0)) v = INFINITY;
      if (v > best) { best = v; bi = t; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
    }
    if (lane == 0) { redv[wv] = best; redi[wv] = bi; }
    __syncthreads();
    best = redv[0];
    bi = redi[0];
    for (int q = 1; q < nw; ++q)
      if (redv[q] > best || (redv[q] == best && redi[q] < bi)) { best = redv[q]; bi = redi[q]; }
    if (!(best > 0.0) || !isfinite(best) || bi >= nx) { bad = true; break; }
    const int p = bi;
    for (int c = tid(); c < nx; c += nthr()) {
      const double a = W[(int64_t)k * nx + c], b = W[(int64_t)p * nx + c];
      if (p != k) W[(int64_t)p * nx + c] = a;
      prow[c] = b;
    }
    if (tid() == 0) piv[k] = p;
    __syncthreads();
    for (int t = tid(); t < nx; t += nthr()) pcol[t] = (t == k) ? 0.0 : W[(int64_t)t * nx + k];
    __syncthreads();
    const double inv = 1.0 / prow[k];
    for (int t = wv; t < nx; t += nw) {
      double* row = W + (int64_t)t * nx;
      if (t == k) {
        for (int c = lane; c < nx; c += 64) row[c] = (c == k) ? inv : prow[c] * inv;
      } else {
        const double fr = pcol[t] * inv;
        for (int c = lane; c < nx; c += 64) row[c] = (c == k) ? -fr : row[c] - fr * prow[c];
      }
    }
    __syncthreads();
  }
  if (bad) {
    if (tid() == 0) *status = ST_ENAN;
    return;
  }
  // undo the row pivoting on the columns of the inverse, last pivot first
  for (int k = nx - 1; k >= 0; --k) {
    const int p = piv[k];
    if (p != k) {
      for (int t = tid(); t < nx; t += nthr()) {
        double* row = W + (int64_t)t * nx;
        const double a = row[k];
        row[k] = row[p];
        row[p] = a;
      }
    }
    __syncthreads();
  }
  // transpose in place: W[k][i] = L_b^-1[i][k]
  for (int e = tid(); e < nx * nx; e += nthr()) {
    const int r = e / nx, c = e - r * nx;
    if (r < c) {
      const double a = W[(int64_t)r * nx + c];
      W[(int64_t)r * nx + c] = W[(int64_t)c * nx + r];
      W[(int64_t)c * nx + r] = a;
    }
  }
  if (lv.bedinv32) {
    __syncthreads();
    float* W32 = mp<float>(ws, lv.bedinv32);
    for (int64_t e = tid(); e < (int64_t)nx * nx; e += nthr()) W32[e] = (float)W[e];
  }
}

}  // namespace pmgw

// Kernels of the p-multigrid Poisson library: geometry/metrics, block inversion, and the
// per-tank solve kernel (operator apply, V-cycle, flexible GMRES).
#pragma once
#include "pmgw_device.hpp"

struct pmgw_info_dev {
  int32_t iters;
  int32_t status;
  double relres;
};

namespace pmgw {

enum : int { MODE_APPLY = 0, MODE_VCYCLE = 1, MODE_SOLVE = 2, MODE_FMG = 3 };
enum : int { ST_OK = 0, ST_NOCONV = 1, ST_EGEOM = -2, ST_ENAN = -3 };

template <typename T>
__device__ __forceinline__ const T* cp(const char* ws, int64_t off) {
  return reinterpret_cast<const T*>(ws + off);
}
template <typename T>
__device__ __forceinline__ T* mp(char* ws, int64_t off) {
  return reinterpret_cast<T*>(ws + off);
}

template <typename T>
__device__ __forceinline__ gptr<const T> gcp(const char* ws, int64_t off) {
  return (gptr<const T>)(ws + off);
}
template <typename T>
__device__ __forceinline__ gptr<T> gmp(char* ws, int64_t off) {
  return (gptr<T>)(ws + off);
}

template <typename T>
__device__ Geo<T> make_geo(char* ws, const TankDesc& td) {
  Geo<T> g;
  if (std::is_same<T, double>::value) {
    const gptr<const T> b = gcp<T>(ws, td.geo64);
    const int nx = td.nx;
    g.ao = b + GEO_AO * nx; g.bo = b + GEO_BO * nx; g.ido = b + GEO_IDO * nx;
    g.an = b + GEO_AN * nx; g.bn = b + GEO_BN * nx; g.idn = b + GEO_IDN * nx;
    g.hx = b + GEO_HX * nx;
  } else {
    const gptr<const T> b = gcp<T>(ws, td.geo32);
    const int nx = td.nx;
    g.ao = b; g.bo = b + nx; g.ido = b + 2 * nx; g.an = b + 3 * nx; g.bn = b + 4 * nx;
    g.idn = b + 5 * nx; g.hx = b + 6 * nx;
  }
  return g;
}

template <typename T>
__device__ Lev<T> make_lev(char* ws, const LevelDesc& d) {
  const int pr = std::is_same<T, double>::value ? 0 : 1;
  Lev<T> L;
  L.nz = d.nz; L.nzc = d.nzc;
  L.Ds = gcp<T>(ws, d.ds[pr]); L.sig = gcp<T>(ws, d.sig[pr]);
  L.R = gcp<T>(ws, d.R[pr]); L.P = gcp<T>(ws, d.P[pr]);
  L.PT = gcp<T>(ws, d.PT[pr]); L.RT = gcp<T>(ws, d.RT[pr]);
  L.colinv = gcp<T>(ws, d.colinv); L.modeinv = gcp<T>(ws, d.modeinv);
  L.x = gmp<T>(ws, d.x); L.f = gmp<T>(ws, d.f); L.r = gmp<T>(ws, d.r);
  L.t1 = gmp<T>(ws, d.t1); L.t2 = gmp<T>(ws, d.t2); L.t3 = gmp<T>(ws, d.t3);
  L.u = gmp<T>(ws, d.u);
  L.spec = gmp<cpx<T>>(ws, d.spec);
  return L;
}

// Level provider for vcycle(): level l of the tank, with the finest level's input and output
// optionally redirected (f0/x0 non-null).
template <typename T>
struct LevSet {
  char* ws;
  const TankDesc* td;
  gptr<T> f0;
  gptr<T> x0;
  __device__ Lev<T> operator()(int l) const {
    Lev<T> L = make_lev<T>(ws, td->lev[l]);
    if (l == 0 && f0) { L.f = f0; L.x = x0; }
    return L;
  }
};

template <typename T>
__device__ __forceinline__ LevSet<T> uni(const LevSet<T>& s) {
  return LevSet<T>{uni(s.ws), uni(s.td), uni(s.f0), uni(s.x0)};
}

// a[e] = v for e < n (grid-stride).
__global__ void __launch_bounds__(256) k_fill(double* a, int64_t n, double v) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    a[e] = v;
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
__global__ void __launch_bounds__(256) k_geometry(const TankDesc* __restrict__ descs, char* ws,
                                                  const double* h, const double* eo,
                                                  const double* en) {
  __shared__ double red[16];
  const TankDesc td = descs[blockIdx.x];
  const int nx = td.nx;
  if (nx < 8 || nx > 2048) return;
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
  __shared__ double Dsl[kMaxNz][kMaxNz + 1];
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
  for (int e = t; e < nz * nz; e += 64) Dsl[e / nz][e % nz] = Ds[e];
  __syncthreads();
  if (jb.kind == 0) {
    const double* G = cp<double>(ws, td.geo64);
    const int i = idx;
    const double ao = G[GEO_AO * nx + i], bo = G[GEO_BO * nx + i], ido = G[GEO_IDO * nx + i];
    const double an = G[GEO_AN * nx + i], bn = G[GEO_BN * nx + i], idn = G[GEO_IDN * nx + i];
    const double hx = G[GEO_HX * nx + i];
    if (t < nz) {
      const int j = t;
      const double sxn = an + bn * sig[j];
      const double bedc = -(hx * (ao + bo * sig[M]) + ido);
      for (int c = 0; c < nz; ++c) {
        double v;
        if (j == 0) {
          v = (c == 0) ? 1.0 : 0.0;
        } else if (j == M) {
          v = bedc * Dsl[M][c];
        } else {
          double s = 0.0;
          for (int m = 0; m < nz; ++m)
            s += Dsl[j][m] * Dsl[m][c] * (sxn * (ao + bo * sig[m]) + idn * ido);
          v = s + ((c == j) ? td.cxx : 0.0);
        }
        A[j][c] = v;
      }
    }
  } else {
    const double* S = cp<double>(ws, td.scal);
    const double cbar = S[0], ebar = S[1];
    const int k = idx;
    const double kap = (k == nx / 2) ? 0.0 : td.kfac * (double)k;
    if (t < nz) {
      const int j = t;
      for (int c = 0; c < nz; ++c) {
        double v;
        if (j == 0) {
          v = (c == 0) ? 1.0 : 0.0;
        } else if (j == M) {
          v = -ebar * Dsl[M][c];
        } else {
          double s = 0.0;
          for (int m = 0; m < nz; ++m) s += Dsl[j][m] * Dsl[m][c];
          v = cbar * s - ((c == j) ? kap * kap : 0.0);
        }
        A[j][c] = v;
      }
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

// ----------------------------------------------------------------------------- solve kernel

// Elementwise passes of the Krylov loop over the workgroup's share of a field: each thread takes
// kEw of its elements at a time (e, e + nthr(), ...), issues all their loads, then computes and
// stores. A load issued after a store waits for that store (the vector-memory counter retires
// both in order), so one element at a time would cost a memory round trip per element. The
// order in which a thread visits its elements, and so every per-thread sum, is unchanged.
constexpr int kEw = 4;

// dst[e] = (TD) src[e]
template <typename TD, typename TS, typename PD, typename PS>
__device__ __forceinline__ void ew_copy(int n, PD dst, PS src) {
  for (int e0 = tid(); e0 < n; e0 += kEw * nthr()) {
    TS v[kEw];
#pragma unroll
    for (int q = 0; q < kEw; ++q) {
      const int e = e0 + q * nthr();
      if (e < n) v[q] = src[e];
    }
#pragma unroll
    for (int q = 0; q < kEw; ++q) {
      const int e = e0 + q * nthr();
      if (e < n) dst[e] = (TD)v[q];
    }
  }
}

// p[e] *= a
__device__ __forceinline__ void ew_scale(int n, double* p, double a) {
  for (int e0 = tid(); e0 < n; e0 += kEw * nthr()) {
    double v[kEw];
#pragma unroll
    for (int q = 0; q < kEw; ++q) {
      const int e = e0 + q * nthr();
      if (e < n) v[q] = p[e];
    }
#pragma unroll
    for (int q = 0; q < kEw; ++q) {
      const int e = e0 + q * nthr();
      if (e < n) p[e] = v[q] * a;
    }
  }
}

// Givens/Hessenberg state of FGMRES in LDS.
struct KrylovLds {
  double H[(kMaxRestart + 1) * kMaxRestart];
  double cs[kMaxRestart], sn[kMaxRestart], g[kMaxRestart + 1], y[kMaxRestart];
  double red[16];
  double res;
};

// One workgroup per tank; the launch covers the tanks whose finest level has NZ rows, listed in
// ids[]. mode MODE_APPLY: out = A in. MODE_VCYCLE: out = V-cycle(in). MODE_SOLVE: FGMRES(restart)
// on A out = in with out as initial guess (paper Sec. 4.4): right preconditioning by one V-cycle,
// modified Gram-Schmidt, Givens rotations, stop on the true relative residual.
// TR = true does the same with A^T and the transposed cycle M^T (the adjoint solve).
template <typename TV, int NZ, int MAXT, bool TR = false>
__global__ void __launch_bounds__(MAXT) k_solve(const TankDesc* __restrict__ descs,
                                                const int32_t* __restrict__ ids, char* ws,
                                                int mode, const double* in, double* out,
                                                double rtol, int maxit, pmgw_info_dev* info,
                                                KOpts o, int fftb) {
  __shared__ KrylovLds K;
  const int tank = ids[blockIdx.x];
  const TankDesc& td = descs[tank];
  const int nx = td.nx, n = nx * NZ;
  if (td.nz != NZ || nx < 8 || nx > 2048) return;
  const double* b = in + td.off2d;
  double* x = out + td.off2d;
  const int32_t gstat = *reinterpret_cast<const int32_t*>(cp<double>(ws, td.scal) + 2);
  if (gstat != ST_OK) {
    if (info && tid() == 0) info[tank] = {0, gstat, 0.0};
    return;
  }

  stage_twiddles(gcp<cpx<double>>(ws, td.tw[0]), gcp<cpx<float>>(ws, td.tw[1]), nx, fftb);
  if (o.adapt) o.omega_m *= cp<double>(ws, td.scal)[3];
  Ctx<double> c64;
  c64.nx = nx; c64.log2nx = td.log2nx; c64.kfac = td.kfac; c64.fftb = fftb;
  c64.g = make_geo<double>(ws, td);
  Lev<double> A64 = make_lev<double>(ws, td.lev[0]);
  A64.t1 = gmp<double>(ws, td.a1); A64.t2 = gmp<double>(ws, td.a2);
  A64.t3 = gmp<double>(ws, td.a3);
  A64.spec = gmp<cpx<double>>(ws, td.aspec);

  Ctx<TV> cv;
  cv.nx = nx; cv.log2nx = td.log2nx; cv.kfac = (TV)td.kfac; cv.fftb = fftb;
  cv.g = make_geo<TV>(ws, td);
  LevSet<TV> levs{ws, &td, gptr<TV>(nullptr), gptr<TV>(nullptr)};
  Lev<TV> L0 = levs(0);

  if (mode == MODE_APPLY) {
    op_any<double, NZ, TR>(c64, A64, FIN_APPLY, as_global(b), as_global(x),
                         gptr<const double>(nullptr), gptr<double>(nullptr), 0.0);
    return;
  }
  if (mode == MODE_VCYCLE || mode == MODE_FMG) {
    ew_copy<TV, double>(n, L0.f, b);
    __syncthreads();
    if constexpr (!TR) {
      if (mode == MODE_FMG) fmg<TV, NZ>(cv, levs, 0, o);
      else vcycle<TV, NZ, LevSet<TV>, TR>(cv, levs, 0, o);
    } else {
      vcycle<TV, NZ, LevSet<TV>, TR>(cv, levs, 0, o);
    }
    ew_copy<double, TV>(n, x, L0.x);
    return;
  }
  // full multigrid preconditions forward solves only (it overwrites the level's right-hand side,
  // so it always runs on the level buffers)
  const bool use_fmg = !TR && o.cycle == 1;

  // ---- FGMRES
  double* V = mp<double>(ws, td.V);
  double* Z = mp<double>(ws, td.Z);
  double s = 0.0;
  for (int e = tid(); e < n; e += nthr()) s += b[e] * b[e];
  const double bn = sqrt(block_sum(s, K.red));
  int it = 0, status = ST_NOCONV;
  double rel = 1.0;
  if (bn == 0.0) {
    for (int e = tid(); e < n; e += nthr()) x[e] = 0.0;
    if (info && tid() == 0) info[tank] = {0, ST_OK, 0.0};
    return;
  }
  if (!isfinite(bn)) {
    if (info && tid() == 0) info[tank] = {0, ST_ENAN, 0.0};
    return;
  }
  const int m = min(o.restart, kMaxRestart);
  for (;;) {
    op_any<double, NZ, TR>(c64, A64, FIN_RESID, as_global((const double*)x), as_global(V),
                         as_global(b), gptr<double>(nullptr), 0.0);
    s = 0.0;
    for (int e = tid(); e < n; e += nthr()) s += V[e] * V[e];
    const double beta = sqrt(block_sum(s, K.red));
    rel = beta / bn;
    if (!isfinite(beta)) { status = ST_ENAN; break; }
    if (rel <= rtol) { status = ST_OK; break; }
    if (it >= maxit) { status = ST_NOCONV; break; }
    const double ib = 1.0 / beta;
    ew_scale(n, V, ib);
    if (tid() == 0) K.g[0] = beta;
    __syncthreads();
    const int mm = min(m, maxit - it);
    int kdone = 0;
    bool bad = false;
    for (int j = 0; j < mm; ++j) {
      double* vj = V + (int64_t)j * n;
      double* zj = Z + (int64_t)j * n;
      double* w = V + (int64_t)(j + 1) * n;
      // z_j = M^-1 v_j
      if (std::is_same<TV, double>::value && !use_fmg) {
        const LevSet<TV> lz{ws, &td, as_global(reinterpret_cast<TV*>(vj)),
                            as_global(reinterpret_cast<TV*>(zj))};
        vcycle<TV, NZ, LevSet<TV>, TR>(cv, lz, 0, o);
      } else {
        ew_copy<TV, double>(n, L0.f, vj);
        __syncthreads();
        if constexpr (!TR) {
          if (use_fmg) fmg<TV, NZ>(cv, levs, 0, o);
          else vcycle<TV, NZ, LevSet<TV>, TR>(cv, levs, 0, o);
        } else {
          vcycle<TV, NZ, LevSet<TV>, TR>(cv, levs, 0, o);
        }
        ew_copy<double, TV>(n, zj, L0.x);
        __syncthreads();
      }
      // w = A z_j
      op_any<double, NZ, TR>(c64, A64, FIN_APPLY, as_global((const double*)zj), as_global(w),
                           gptr<const double>(nullptr), gptr<double>(nullptr), 0.0);
      // modified Gram-Schmidt, each pass fuses the previous update with the next dot
      double hprev = 0.0;
      for (int i = 0; i <= j + 1; ++i) {
        const double* vprev = (i > 0) ? V + (int64_t)(i - 1) * n : nullptr;
        const double* vi = (i <= j) ? V + (int64_t)i * n : nullptr;
        double acc = 0.0;
        for (int e0 = tid(); e0 < n; e0 += kEw * nthr()) {
          double we[kEw], vp[kEw], vv[kEw];
#pragma unroll
          for (int q = 0; q < kEw; ++q) {
            const int e = e0 + q * nthr();
            if (e < n) {
              we[q] = w[e];
              if (i > 0) vp[q] = vprev[e];
              if (i <= j) vv[q] = vi[e];
            }
          }
#pragma unroll
          for (int q = 0; q < kEw; ++q) {
            const int e = e0 + q * nthr();
            if (e < n) {
              if (i > 0) { we[q] -= hprev * vp[q]; w[e] = we[q]; }
              acc += (i <= j) ? we[q] * vv[q] : we[q] * we[q];
            }
          }
        }
        const double hv = block_sum(acc, K.red);
        if (i <= j) {
          if (tid() == 0) K.H[i * kMaxRestart + j] = hv;
          hprev = hv;
        } else {
          const double hn = sqrt(hv);
          if (tid() == 0) K.H[(j + 1) * kMaxRestart + j] = hn;
          if (hn > 0.0 && isfinite(hn)) {
            const double ih = 1.0 / hn;
            ew_scale(n, w, ih);
          }
        }
      }
      __syncthreads();
      if (tid() == 0) {
        double* H = K.H;
        for (int i = 0; i < j; ++i) {
          const double a = H[i * kMaxRestart + j], c2 = H[(i + 1) * kMaxRestart + j];
          H[i * kMaxRestart + j] = K.cs[i] * a + K.sn[i] * c2;
          H[(i + 1) * kMaxRestart + j] = -K.sn[i] * a + K.cs[i] * c2;
        }
        const double a = H[j * kMaxRestart + j], c2 = H[(j + 1) * kMaxRestart + j];
        const double den = hypot(a, c2);
        const double cj = den > 0.0 ? a / den : 1.0, sj = den > 0.0 ? c2 / den : 0.0;
        K.cs[j] = cj;
        K.sn[j] = sj;
        H[j * kMaxRestart + j] = den;
        H[(j + 1) * kMaxRestart + j] = 0.0;
        K.g[j + 1] = -sj * K.g[j];
        K.g[j] = cj * K.g[j];
        K.res = fabs(K.g[j + 1]);
      }
      __syncthreads();
      ++it;
      kdone = j + 1;
      const double res = K.res;
      const double hjj = K.H[j * kMaxRestart + j];
      if (!isfinite(res) || !isfinite(hjj)) { bad = true; break; }
      if (res / bn <= rtol || hjj == 0.0) break;
    }
    if (bad) { status = ST_ENAN; break; }
    if (tid() == 0) {
      for (int i = kdone - 1; i >= 0; --i) {
        double acc = K.g[i];
        for (int l = i + 1; l < kdone; ++l) acc -= K.H[i * kMaxRestart + l] * K.y[l];
        K.y[i] = acc / K.H[i * kMaxRestart + i];
      }
    }
    __syncthreads();
    for (int e0 = tid(); e0 < n; e0 += kEw * nthr()) {
      double acc[kEw];
#pragma unroll
      for (int q = 0; q < kEw; ++q) {
        const int e = e0 + q * nthr();
        if (e < n) acc[q] = x[e];
      }
      for (int i = 0; i < kdone; ++i) {
        const double yi = K.y[i];
#pragma unroll
        for (int q = 0; q < kEw; ++q) {
          const int e = e0 + q * nthr();
          if (e < n) acc[q] += yi * Z[(int64_t)i * n + e];
        }
      }
#pragma unroll
      for (int q = 0; q < kEw; ++q) {
        const int e = e0 + q * nthr();
        if (e < n) x[e] = acc[q];
      }
    }
    __syncthreads();
  }
  if (info && tid() == 0) info[tank] = {it, status, rel};
}

}  // namespace pmgw

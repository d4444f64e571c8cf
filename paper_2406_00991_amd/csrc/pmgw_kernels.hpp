// The per-tank solve kernel of the p-multigrid Poisson library (operator apply, V-cycle,
// flexible GMRES) and the workspace accessors it shares with the set-up and stage kernels.
#pragma once
#include "pmgw_device.hpp"
#include "pmgw_resident.hpp"

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
  const int64_t bo = pr == 0 ? d.bedinv : d.bedinv32;
  L.binv = bo ? gcp<T>(ws, bo) : gptr<const T>(nullptr);
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
// RES = true (float32 cycle, forward, V-cycle preconditioner, NZ <= 17) runs the cycle in LDS
// (pmgw_resident.hpp); the launch's dynamic LDS then covers the resident map of every tank.
template <typename TV, int NZ, int MAXT, bool TR = false, bool RES = false>
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
  c64.cw = td.cw ? gcp<double>(ws, td.cw) : gptr<const double>(nullptr);
  c64.cwt = td.cwt ? gcp<double>(ws, td.cwt) : gptr<const double>(nullptr);
  Lev<double> A64 = make_lev<double>(ws, td.lev[0]);
  A64.t1 = gmp<double>(ws, td.a1); A64.t2 = gmp<double>(ws, td.a2);
  A64.t3 = gmp<double>(ws, td.a3);
  A64.spec = gmp<cpx<double>>(ws, td.aspec);

  Ctx<TV> cv;
  cv.nx = nx; cv.log2nx = td.log2nx; cv.kfac = (TV)td.kfac; cv.fftb = fftb;
  cv.g = make_geo<TV>(ws, td);
  cv.cw = c64.cw;
  cv.cwt = c64.cwt;
  LevSet<TV> levs{ws, &td, gptr<TV>(nullptr), gptr<TV>(nullptr)};
  Lev<TV> L0 = levs(0);

  // the resident cycle: src (float64, global) -> f_0 in LDS -> cycle -> x_0 -> dst (float64)
  RCtx rc;
  auto res_cycle = [&](const double* src, double* dst) {
    if constexpr (RES) {
      const RMap m0 = res_map<NZ, NZ>(nx);
      res_load_geo<NZ>(ws, td);
      ew_copy<float, double>(n, m0.f, src);
      __syncthreads();
      rvcycle<NZ, NZ>(rc);
      ew_copy<double, float>(n, dst, m0.x);
      __syncthreads();
    }
  };
  if constexpr (RES) {
    static_assert(std::is_same<TV, float>::value && !TR && NZ <= kResMaxNz, "resident cycle");
    rc.nx = nx; rc.log2nx = td.log2nx; rc.fftb = fftb; rc.kfac = (float)td.kfac;
    rc.wc = (float)o.omega_c; rc.wm = (float)o.omega_m;
    rc.nu1 = o.nu1; rc.nu2 = o.nu2; rc.coarse_pairs = o.coarse_pairs;
    rc.coarse_exact = o.coarse_exact; rc.td = &td; rc.ws = ws; rc.cw = cv.cw; rc.cwt = cv.cwt;
  }

  if (mode == MODE_APPLY) {
    op_any<double, NZ, TR>(c64, A64, FIN_APPLY, as_global(b), as_global(x),
                         gptr<const double>(nullptr), gptr<double>(nullptr), 0.0);
    return;
  }
  if constexpr (RES) {
    if (mode == MODE_VCYCLE) {
      res_cycle(b, x);
      return;
    }
  } else if (mode == MODE_VCYCLE || mode == MODE_FMG) {
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
      if constexpr (RES) {
        res_cycle(vj, zj);
      } else if (std::is_same<TV, double>::value && !use_fmg) {
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

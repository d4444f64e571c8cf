// Device code of the 3D tanks (x, y periodic Fourier, sigma Chebyshev), float64: geometry,
// smoother blocks, the operator, the V-cycle and FGMRES, one workgroup per tank. Fields are
// [Nz][Ny][Nx] with x fastest; nh = Nx Ny horizontal nodes ("columns").
#pragma once
#include <stdint.h>

#include "pmgw_device.hpp"

namespace pmgw3 {

using pmgw::block_sum;
using pmgw::cpx;
using pmgw::nthr;
using pmgw::tid;

constexpr int kMaxLev3 = 5;
constexpr int kMaxNz3 = 33;
constexpr int kMaxRestart3 = 32;
constexpr int kFftCap3 = 2048;   // complex doubles per LDS FFT buffer (two buffers: 64 KB)
constexpr int kMaxN3 = 1024;     // largest Nx or Ny

enum : int { ST3_OK = 0, ST3_NOCONV = 1, ST3_EGEOM = -2, ST3_ENAN = -3 };
enum : int { M3_APPLY = 0, M3_VCYCLE = 1, M3_SOLVE = 2 };
// geometry rows (nh doubles each): sigma_x = ax + bx sigma, sigma_y = ay + by sigma, 1/d, for the
// old (O) and new (N) surface, and h_x, h_y
enum : int { G_AXO, G_BXO, G_AYO, G_BYO, G_IDO, G_AXN, G_BXN, G_AYN, G_BYN, G_IDN, G_HX, G_HY,
             G_COUNT };

struct Lev3 {
  int32_t nz, nzc;
  int64_t ds, sig, R, P;             // D_sigma [nz][nz], sigma [nz], R [nzc][nz], P [nz][nzc]
  int64_t colinv, modeinv;           // block inverses [nz][nz][nh]
  int64_t x, f, r, t1, gx, gy, t2, t3;   // level fields [nz][nh]
  int64_t spec;                      // spectra of the packed row pairs [(nz+1)/2][nh] complex
};

struct Tank3 {
  int32_t nx, ny, nz, nlev, lgx, lgy;
  double Lx, Ly, kfx, kfy, cxx, cyy;
  int64_t off3d, off2d;
  int64_t geo;                       // [G_COUNT][nh]
  int64_t scal;                      // cbar, ebar, status (int32 in the third double), damping
  int64_t V, Z;                      // FGMRES bases [(m+1)][n], [m][n]
  Lev3 lev[kMaxLev3];
};

struct Opts3 {
  int32_t nu1, nu2, coarse_pairs, restart;
  double omega_c, omega_m;
  int32_t adapt;
};

struct Info3 {
  int32_t iters, status;
  double relres;
};

template <typename T>
__device__ __forceinline__ T* wp(char* ws, int64_t off) { return reinterpret_cast<T*>(ws + off); }
template <typename T>
__device__ __forceinline__ const T* wc(const char* ws, int64_t off) {
  return reinterpret_cast<const T*>(ws + off);
}
__device__ __forceinline__ int32_t* status_of(char* ws, const Tank3& t) {
  return reinterpret_cast<int32_t*>(wp<double>(ws, t.scal) + 2);
}

extern __shared__ double g3_lds[];

// Dynamic LDS: two FFT buffers of kFftCap3 complex doubles, then the x and y twiddle tables.
struct Fft3 {
  cpx<double>* A;
  cpx<double>* B;
  cpx<double>* twx;
  cpx<double>* twy;
};

__device__ __forceinline__ Fft3 fft3_layout(int nx) {
  cpx<double>* base = reinterpret_cast<cpx<double>*>(g3_lds);
  Fft3 f;
  f.A = base;
  f.B = base + kFftCap3;
  f.twx = base + 2 * kFftCap3;
  f.twy = f.twx + nx;
  return f;
}

// tw[t] = exp(-2 pi i t / N) for the x and y lengths (sincospi: the library's own double-precision
// routine); a workgroup barrier at the end.
__device__ void fft3_twiddles(const Fft3& f, int nx, int ny) {
  for (int t = tid(); t < nx; t += nthr()) {
    double s, c;
    sincospi(-2.0 * t / nx, &s, &c);
    f.twx[t] = {c, s};
  }
  for (int t = tid(); t < ny; t += nthr()) {
    double s, c;
    sincospi(-2.0 * t / ny, &s, &c);
    f.twy[t] = {c, s};
  }
  __syncthreads();
}

// Stockham radix-2 transform of nb complex rows of length N = 2^lg in A (row r at A + r N),
// ping-ponging with B: with n the current transform length and s the stride,
// y[q + s(2p)] = a + b, y[q + s(2p+1)] = (a - b) W_n^p, a = x[q + s p], b = x[q + s(p + n/2)];
// natural order in and out. Forward (exp(-2 pi i/N)) or inverse (conjugate, unscaled). Returns
// the buffer holding the result; barriers between passes and at the end.
__device__ cpx<double>* fft3(cpx<double>* A, cpx<double>* B, int nb, int N, int lg,
                             const cpx<double>* tw, bool inv) {
  cpx<double>* x = A;
  cpx<double>* y = B;
  const int half = N >> 1;
  int n = N, s = 1;
  for (int pass = 0; pass < lg; ++pass) {
    const int m = n >> 1;
    const int items = nb * half;
    for (int e = tid(); e < items; e += nthr()) {
      const int row = e / half, r = e - row * half;
      const int p = r / s, q = r - p * s;
      const cpx<double>* xr = x + row * N;
      cpx<double>* yr = y + row * N;
      const cpx<double> a = xr[q + s * p], b = xr[q + s * (p + m)];
      cpx<double> w = tw[p * (N / n)];
      if (inv) w.im = -w.im;
      yr[q + s * (2 * p)] = {a.re + b.re, a.im + b.im};
      const cpx<double> d = {a.re - b.re, a.im - b.im};
      yr[q + s * (2 * p + 1)] = {d.re * w.re - d.im * w.im, d.re * w.im + d.im * w.re};
    }
    __syncthreads();
    cpx<double>* t = x;
    x = y;
    y = t;
    n = m;
    s <<= 1;
  }
  return x;
}

// Derivative of nrows real rows of length N along their direction, two rows per complex
// transform: ld(row, i) reads, st(row, i, v) writes D f (i kappa_k, kappa_k = kf k, Nyquist 0).
template <class LD, class ST>
__device__ void deriv_rows(int nrows, int N, int lg, double kf, const Fft3& F,
                           const cpx<double>* tw, LD ld, ST st) {
  const int npairs = (nrows + 1) >> 1;
  const int rpb = kFftCap3 / N;
  for (int p0 = 0; p0 < npairs; p0 += rpb) {
    const int nb = min(rpb, npairs - p0);
    for (int e = tid(); e < nb * N; e += nthr()) {
      const int q = e / N, i = e - q * N, ra = 2 * (p0 + q);
      F.A[e] = {ld(ra, i), ra + 1 < nrows ? ld(ra + 1, i) : 0.0};
    }
    __syncthreads();
    cpx<double>* R = fft3(F.A, F.B, nb, N, lg, tw, false);
    for (int e = tid(); e < nb * N; e += nthr()) {
      const int k = e % N;
      const int kk = (k <= N / 2) ? k : k - N;
      const double kap = (k == N / 2) ? 0.0 : kf * (double)kk / (double)N;
      const cpx<double> v = R[e];
      R[e] = {-kap * v.im, kap * v.re};
    }
    __syncthreads();
    cpx<double>* S = fft3(R, R == F.A ? F.B : F.A, nb, N, lg, tw, true);
    for (int e = tid(); e < nb * N; e += nthr()) {
      const int q = e / N, i = e - q * N, ra = 2 * (p0 + q);
      st(ra, i, S[e].re);
      if (ra + 1 < nrows) st(ra + 1, i, S[e].im);
    }
    __syncthreads();
  }
}

// Complex transforms of nrows rows of length N: ld(row, i) -> cpx, st(row, i, cpx).
template <class LD, class ST>
__device__ void cfft_rows(int nrows, int N, int lg, const Fft3& F, const cpx<double>* tw,
                          bool inv, LD ld, ST st) {
  const int rpb = kFftCap3 / N;
  for (int r0 = 0; r0 < nrows; r0 += rpb) {
    const int nb = min(rpb, nrows - r0);
    for (int e = tid(); e < nb * N; e += nthr()) {
      const int q = e / N, i = e - q * N;
      F.A[e] = ld(r0 + q, i);
    }
    __syncthreads();
    cpx<double>* R = fft3(F.A, F.B, nb, N, lg, tw, inv);
    for (int e = tid(); e < nb * N; e += nthr()) {
      const int q = e / N, i = e - q * N;
      st(r0 + q, i, R[e]);
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------- one tank's view

struct View3 {
  int nx, ny, nh, lgx, lgy;
  double kfx, kfy;
  const double* G;   // geometry rows
  Fft3 F;
};

__device__ __forceinline__ View3 view3(char* ws, const Tank3& t) {
  View3 v;
  v.nx = t.nx; v.ny = t.ny; v.nh = t.nx * t.ny; v.lgx = t.lgx; v.lgy = t.lgy;
  v.kfx = t.kfx; v.kfy = t.kfy;
  v.G = wc<double>(ws, t.geo);
  v.F = fft3_layout(t.nx);
  return v;
}

struct LevV {
  int nz, nzc;
  const double *Ds, *sig, *R, *P, *colinv, *modeinv;
  double *x, *f, *r, *t1, *gx, *gy, *t2, *t3;
  cpx<double>* spec;
};

__device__ __forceinline__ LevV levv(char* ws, const Lev3& d) {
  LevV L;
  L.nz = d.nz; L.nzc = d.nzc;
  L.Ds = wc<double>(ws, d.ds); L.sig = wc<double>(ws, d.sig);
  L.R = d.nzc ? wc<double>(ws, d.R) : nullptr; L.P = d.nzc ? wc<double>(ws, d.P) : nullptr;
  L.colinv = wc<double>(ws, d.colinv); L.modeinv = wc<double>(ws, d.modeinv);
  L.x = wp<double>(ws, d.x); L.f = wp<double>(ws, d.f); L.r = wp<double>(ws, d.r);
  L.t1 = wp<double>(ws, d.t1); L.gx = wp<double>(ws, d.gx); L.gy = wp<double>(ws, d.gy);
  L.t2 = wp<double>(ws, d.t2); L.t3 = wp<double>(ws, d.t3);
  L.spec = wp<cpx<double>>(ws, d.spec);
  return L;
}

// out = D_sigma in, column by column.
__device__ void col_dsig3(const View3& v, const LevV& L, const double* in, double* out) {
  const int nz = L.nz, nh = v.nh;
  for (int e = tid(); e < nz * nh; e += nthr()) {
    const int j = e / nh, c = e - j * nh;
    double s = 0.0;
    for (int l = 0; l < nz; ++l) s += L.Ds[j * nz + l] * in[l * nh + c];
    out[e] = s;
  }
}

enum : int { F3_APPLY = 0, F3_RESID = 1 };

// The operator on one level: out = A in (F3_APPLY) or out = f - A in (F3_RESID).
//   t1 = D_s in; gx = D_x in + sigma_x^old t1; gy = D_y in + sigma_y^old t1;
//   t2 = D_x gx; t3 = D_y gy; interior rows t2 + t3 + sigma_x^new D_s gx + sigma_y^new D_s gy
//   + (1/d_new) D_s (t1 / d_old); row 0 = in; row M = -(h_x gx + h_y gy + t1 / d_old).
__device__ void op3(const View3& v, const LevV& L, int mode, const double* in, double* out,
                    const double* f) {
  const int nz = L.nz, M = nz - 1, nx = v.nx, ny = v.ny, nh = v.nh;
  const double* G = v.G;
  col_dsig3(v, L, in, L.t1);
  __syncthreads();
  double* gx = L.gx;
  double* gy = L.gy;
  double* t1 = L.t1;
  const double* sig = L.sig;
  deriv_rows(nz * ny, nx, v.lgx, v.kfx, v.F, v.F.twx,
             [=](int row, int i) { return in[row * nx + i]; },
             [=](int row, int i, double d) {
               const int j = row / ny, c = (row - j * ny) * nx + i;
               gx[row * nx + i] = d + (G[G_AXO * nh + c] + G[G_BXO * nh + c] * sig[j]) * t1[row * nx + i];
             });
  deriv_rows(nz * nx, ny, v.lgy, v.kfy, v.F, v.F.twy,
             [=](int row, int i) {
               const int j = row / nx, ix = row - j * nx;
               return in[j * nh + i * nx + ix];
             },
             [=](int row, int i, double d) {
               const int j = row / nx, ix = row - j * nx, c = i * nx + ix;
               gy[j * nh + c] = d + (G[G_AYO * nh + c] + G[G_BYO * nh + c] * sig[j]) * t1[j * nh + c];
             });
  double* t2 = L.t2;
  double* t3 = L.t3;
  deriv_rows(nz * ny, nx, v.lgx, v.kfx, v.F, v.F.twx,
             [=](int row, int i) { return gx[row * nx + i]; },
             [=](int row, int i, double d) { t2[row * nx + i] = d; });
  deriv_rows(nz * nx, ny, v.lgy, v.kfy, v.F, v.F.twy,
             [=](int row, int i) {
               const int j = row / nx, ix = row - j * nx;
               return gy[j * nh + i * nx + ix];
             },
             [=](int row, int i, double d) {
               const int j = row / nx, ix = row - j * nx;
               t3[j * nh + i * nx + ix] = d;
             });
  for (int e = tid(); e < nz * nh; e += nthr()) {
    const int j = e / nh, c = e - j * nh;
    double a;
    if (j == 0) {
      a = in[e];
    } else if (j == M) {
      a = -(G[G_HX * nh + c] * gx[e] + G[G_HY * nh + c] * gy[e] + t1[e] * G[G_IDO * nh + c]);
    } else {
      double sx = 0.0, sy = 0.0, sz = 0.0;
      for (int l = 0; l < nz; ++l) {
        const double dl = L.Ds[j * nz + l];
        sx += dl * gx[l * nh + c];
        sy += dl * gy[l * nh + c];
        sz += dl * t1[l * nh + c];
      }
      const double sxn = G[G_AXN * nh + c] + G[G_BXN * nh + c] * sig[j];
      const double syn = G[G_AYN * nh + c] + G[G_BYN * nh + c] * sig[j];
      a = t2[e] + t3[e] + sxn * sx + syn * sy + G[G_IDN * nh + c] * G[G_IDO * nh + c] * sz;
    }
    out[e] = (mode == F3_APPLY) ? a : f[e] - a;
  }
  __syncthreads();
}

// Column step x += omega B_c^-1 r (from x = 0 when zero: x = omega B_c^-1 f).
__device__ void col_step3(const View3& v, const LevV& L, const double* r, double* x, double w,
                          bool zero) {
  const int nz = L.nz, nh = v.nh;
  for (int e = tid(); e < nz * nh; e += nthr()) {
    const int j = e / nh, c = e - j * nh;
    double s = 0.0;
    for (int l = 0; l < nz; ++l) s += L.colinv[(int64_t)(j * nz + l) * nh + c] * r[l * nh + c];
    // every thread reads its own column's r only; x is written after all r are read
    L.t2[e] = w * s;
  }
  __syncthreads();
  for (int e = tid(); e < nz * nh; e += nthr()) x[e] = zero ? L.t2[e] : x[e] + L.t2[e];
  __syncthreads();
}

// Mode step x += omega F^-1 Ahat^-1 F r: 2D transforms of the packed row pairs (x, then y),
// per mode (ky, kx) with its partner (-ky, -kx) unpack, solve with the flat block, repack,
// inverse transforms (y, then x) adding omega times the correction to x (or setting it).
__device__ void mode_step3(const View3& v, const LevV& L, const double* r, double* x, double w,
                           bool zero) {
  const int nz = L.nz, nx = v.nx, ny = v.ny, nh = v.nh, np = (nz + 1) >> 1;
  cpx<double>* spec = L.spec;
  cfft_rows(np * ny, nx, v.lgx, v.F, v.F.twx, false,
            [=](int row, int i) {
              const int p = row / ny, iy = row - p * ny, j0 = 2 * p, j1 = j0 + 1;
              return cpx<double>{r[j0 * nh + iy * nx + i], j1 < nz ? r[j1 * nh + iy * nx + i] : 0.0};
            },
            [=](int row, int i, cpx<double> z) { spec[row * nx + i] = z; });
  cfft_rows(np * nx, ny, v.lgy, v.F, v.F.twy, false,
            [=](int row, int i) {
              const int p = row / nx, kx = row - p * nx;
              return spec[p * nh + i * nx + kx];
            },
            [=](int row, int i, cpx<double> z) {
              const int p = row / nx, kx = row - p * nx;
              spec[p * nh + i * nx + kx] = z;
            });
  const double scale = 1.0 / (double)nh;
  for (int m = tid(); m < nh; m += nthr()) {
    const int ky = m / nx, kx = m - ky * nx;
    const int mc = ((ny - ky) & (ny - 1)) * nx + ((nx - kx) & (nx - 1));
    if (mc < m) continue;
    cpx<double> rh[kMaxNz3];
    for (int p = 0; p < np; ++p) {
      const cpx<double> z = spec[p * nh + m], zc = spec[p * nh + mc];
      rh[2 * p] = {0.5 * (z.re + zc.re), 0.5 * (z.im - zc.im)};
      if (2 * p + 1 < nz) rh[2 * p + 1] = {0.5 * (z.im + zc.im), -0.5 * (z.re - zc.re)};
    }
    for (int p = 0; p < np; ++p) {
      const int j0 = 2 * p, j1 = j0 + 1;
      cpx<double> s0 = {0.0, 0.0}, s1 = {0.0, 0.0};
      for (int l = 0; l < nz; ++l) {
        const double a = L.modeinv[(int64_t)(j0 * nz + l) * nh + m];
        s0.re += a * rh[l].re;
        s0.im += a * rh[l].im;
        if (j1 < nz) {
          const double b = L.modeinv[(int64_t)(j1 * nz + l) * nh + m];
          s1.re += b * rh[l].re;
          s1.im += b * rh[l].im;
        }
      }
      s0.re *= scale; s0.im *= scale; s1.re *= scale; s1.im *= scale;
      spec[p * nh + m] = {s0.re - s1.im, s0.im + s1.re};
      if (mc != m) spec[p * nh + mc] = {s0.re + s1.im, s1.re - s0.im};
    }
  }
  __syncthreads();
  cfft_rows(np * nx, ny, v.lgy, v.F, v.F.twy, true,
            [=](int row, int i) {
              const int p = row / nx, kx = row - p * nx;
              return spec[p * nh + i * nx + kx];
            },
            [=](int row, int i, cpx<double> z) {
              const int p = row / nx, kx = row - p * nx;
              spec[p * nh + i * nx + kx] = z;
            });
  cfft_rows(np * ny, nx, v.lgx, v.F, v.F.twx, true,
            [=](int row, int i) { return spec[row * nx + i]; },
            [=](int row, int i, cpx<double> z) {
              const int p = row / ny, iy = row - p * ny, j0 = 2 * p, j1 = j0 + 1;
              const int e0 = j0 * nh + iy * nx + i;
              x[e0] = zero ? w * z.re : x[e0] + w * z.re;
              if (j1 < nz) {
                const int e1 = j1 * nh + iy * nx + i;
                x[e1] = zero ? w * z.im : x[e1] + w * z.im;
              }
            });
}

// V-cycle (Alg. 1, correction scheme from x = 0) on level l: f = lev(l).f in, lev(l).x out.
// Levels below are visited iteratively (a down sweep then an up sweep) to keep the device code
// free of recursion: pre-smoothing and restriction going down, the coarsest pairs, then
// prolongation and post-smoothing going up.
__device__ void vcycle3(char* ws, const Tank3& t, const View3& v, const Opts3& o) {
  const int nlev = t.nlev, nh = v.nh;
  const double wc = o.omega_c;
  const double wm = o.omega_m;
  for (int l = 0; l < nlev; ++l) {
    const LevV L = levv(ws, t.lev[l]);
    const bool coarsest = (l == nlev - 1);
    const int npre = coarsest ? o.coarse_pairs : o.nu1;
    bool zero = true;
    for (int q = 0; q < npre; ++q) {
      if (zero) {
        col_step3(v, L, L.f, L.x, wc, true);
      } else {
        op3(v, L, F3_RESID, L.x, L.r, L.f);
        col_step3(v, L, L.r, L.x, wc, false);
      }
      zero = false;
      op3(v, L, F3_RESID, L.x, L.r, L.f);
      mode_step3(v, L, L.r, L.x, wm, false);
    }
    if (zero) {
      for (int e = tid(); e < L.nz * nh; e += nthr()) L.x[e] = 0.0;
      __syncthreads();
    }
    if (!coarsest) {
      const LevV C = levv(ws, t.lev[l + 1]);
      op3(v, L, F3_RESID, L.x, L.r, L.f);
      for (int e = tid(); e < C.nz * nh; e += nthr()) {
        const int jc = e / nh, c = e - jc * nh;
        double s = 0.0;
        for (int k = 0; k < L.nz; ++k) s += L.R[jc * L.nz + k] * L.r[k * nh + c];
        C.f[e] = s;
      }
      __syncthreads();
    }
  }
  for (int l = nlev - 2; l >= 0; --l) {
    const LevV L = levv(ws, t.lev[l]);
    const LevV C = levv(ws, t.lev[l + 1]);
    for (int e = tid(); e < L.nz * nh; e += nthr()) {
      const int j = e / nh, c = e - j * nh;
      double s = 0.0;
      for (int k = 0; k < C.nz; ++k) s += L.P[j * C.nz + k] * C.x[k * nh + c];
      L.x[e] += s;
    }
    __syncthreads();
    for (int q = 0; q < o.nu2; ++q) {
      op3(v, L, F3_RESID, L.x, L.r, L.f);
      col_step3(v, L, L.r, L.x, wc, false);
      op3(v, L, F3_RESID, L.x, L.r, L.f);
      mode_step3(v, L, L.r, L.x, wm, false);
    }
  }
}

struct Kry3 {
  double H[(kMaxRestart3 + 1) * kMaxRestart3];
  double cs[kMaxRestart3], sn[kMaxRestart3], g[kMaxRestart3 + 1], y[kMaxRestart3];
  double red[16];
  double res;
};

// Threads per 3D solve workgroup (one workgroup per tank): eight wavefronts.
constexpr int kThreads3 = 1024;

__global__ void __launch_bounds__(kThreads3) k3_solve(const Tank3* __restrict__ descs, char* ws,
                                                int mode, const double* in, double* out,
                                                double rtol, int maxit, Info3* info, Opts3 o) {
  __shared__ Kry3 K;
  const Tank3 t = descs[blockIdx.x];
  const int nz = t.nz, nh = t.nx * t.ny, n = nz * nh;
  const double* b = in + t.off3d;
  double* x = out + t.off3d;
  int32_t* st = status_of(ws, t);
  if (*st != ST3_OK) {
    if (info && tid() == 0) info[blockIdx.x] = {0, *st, 0.0};
    return;
  }
  if (o.adapt) o.omega_m *= wc<double>(ws, t.scal)[3];
  const View3 v = view3(ws, t);
  fft3_twiddles(v.F, t.nx, t.ny);
  const LevV L0 = levv(ws, t.lev[0]);
  if (mode == M3_APPLY) {
    op3(v, L0, F3_APPLY, b, x, nullptr);
    return;
  }
  if (mode == M3_VCYCLE) {
    for (int e = tid(); e < n; e += nthr()) L0.f[e] = b[e];
    __syncthreads();
    vcycle3(ws, t, v, o);
    for (int e = tid(); e < n; e += nthr()) x[e] = L0.x[e];
    return;
  }
  double* V = wp<double>(ws, t.V);
  double* Z = wp<double>(ws, t.Z);
  const int m = min(o.restart, kMaxRestart3);
  double s = 0.0;
  for (int e = tid(); e < n; e += nthr()) s += b[e] * b[e];
  const double bn = sqrt(block_sum(s, K.red));
  int it = 0, status = ST3_NOCONV;
  double rel = 1.0;
  if (bn == 0.0) {
    for (int e = tid(); e < n; e += nthr()) x[e] = 0.0;
    if (info && tid() == 0) info[blockIdx.x] = {0, ST3_OK, 0.0};
    return;
  }
  if (!isfinite(bn)) {
    if (info && tid() == 0) info[blockIdx.x] = {0, ST3_ENAN, 0.0};
    return;
  }
  for (;;) {
    op3(v, L0, F3_RESID, x, V, b);
    s = 0.0;
    for (int e = tid(); e < n; e += nthr()) s += V[e] * V[e];
    const double beta = sqrt(block_sum(s, K.red));
    rel = beta / bn;
    if (!isfinite(beta)) { status = ST3_ENAN; break; }
    if (rel <= rtol) { status = ST3_OK; break; }
    if (it >= maxit) { status = ST3_NOCONV; break; }
    for (int e = tid(); e < n; e += nthr()) V[e] /= beta;
    if (tid() == 0) K.g[0] = beta;
    __syncthreads();
    const int mm = min(m, maxit - it);
    int kdone = 0;
    bool bad = false;
    for (int j = 0; j < mm; ++j) {
      double* vj = V + (int64_t)j * n;
      double* zj = Z + (int64_t)j * n;
      double* w = V + (int64_t)(j + 1) * n;
      for (int e = tid(); e < n; e += nthr()) L0.f[e] = vj[e];
      __syncthreads();
      vcycle3(ws, t, v, o);
      for (int e = tid(); e < n; e += nthr()) zj[e] = L0.x[e];
      __syncthreads();
      op3(v, L0, F3_APPLY, zj, w, nullptr);
      // modified Gram-Schmidt
      for (int i = 0; i <= j; ++i) {
        const double* vi = V + (int64_t)i * n;
        double acc = 0.0;
        for (int e = tid(); e < n; e += nthr()) acc += w[e] * vi[e];
        const double h = block_sum(acc, K.red);
        if (tid() == 0) K.H[i * kMaxRestart3 + j] = h;
        for (int e = tid(); e < n; e += nthr()) w[e] -= h * vi[e];
        __syncthreads();
      }
      double acc = 0.0;
      for (int e = tid(); e < n; e += nthr()) acc += w[e] * w[e];
      const double hn = sqrt(block_sum(acc, K.red));
      if (tid() == 0) K.H[(j + 1) * kMaxRestart3 + j] = hn;
      if (hn > 0.0 && isfinite(hn))
        for (int e = tid(); e < n; e += nthr()) w[e] /= hn;
      __syncthreads();
      if (tid() == 0) {
        double* H = K.H;
        for (int i = 0; i < j; ++i) {
          const double a = H[i * kMaxRestart3 + j], c2 = H[(i + 1) * kMaxRestart3 + j];
          H[i * kMaxRestart3 + j] = K.cs[i] * a + K.sn[i] * c2;
          H[(i + 1) * kMaxRestart3 + j] = -K.sn[i] * a + K.cs[i] * c2;
        }
        const double a = H[j * kMaxRestart3 + j], c2 = H[(j + 1) * kMaxRestart3 + j];
        const double den = hypot(a, c2);
        const double cj = den > 0.0 ? a / den : 1.0, sj = den > 0.0 ? c2 / den : 0.0;
        K.cs[j] = cj;
        K.sn[j] = sj;
        H[j * kMaxRestart3 + j] = den;
        H[(j + 1) * kMaxRestart3 + j] = 0.0;
        K.g[j + 1] = -sj * K.g[j];
        K.g[j] = cj * K.g[j];
        K.res = fabs(K.g[j + 1]);
      }
      __syncthreads();
      ++it;
      kdone = j + 1;
      const double res = K.res;
      const double hjj = K.H[j * kMaxRestart3 + j];
      if (!isfinite(res) || !isfinite(hjj)) { bad = true; break; }
      if (res / bn <= rtol || hjj == 0.0) break;
    }
    if (bad) { status = ST3_ENAN; break; }
    if (tid() == 0) {
      for (int i = kdone - 1; i >= 0; --i) {
        double a = K.g[i];
        for (int l = i + 1; l < kdone; ++l) a -= K.H[i * kMaxRestart3 + l] * K.y[l];
        K.y[i] = a / K.H[i * kMaxRestart3 + i];
      }
    }
    __syncthreads();
    for (int e = tid(); e < n; e += nthr()) {
      double a = x[e];
      for (int i = 0; i < kdone; ++i) a += K.y[i] * Z[(int64_t)i * n + e];
      x[e] = a;
    }
    __syncthreads();
  }
  if (info && tid() == 0) info[blockIdx.x] = {it, status, rel};
}

// ----------------------------------------------------------------------------- set-up kernels

// Metrics of the old and new surface from h, eta (device [ny][nx]): spectral h_x, h_y, d_x, d_y;
// geometry rows; the flat-mode averages cbar = <1/(d_o d_n)>, ebar = <(1 + h_x^2 + h_y^2)/d_o>
// and the mode damping factor min(1, 2 / (1 + (r/2)^0.4)), r = max c / min c, c = 1/(d_o d_n).
// d <= 0 or non-finite marks the tank EGEOM.
__global__ void __launch_bounds__(256) k3_geometry(const Tank3* __restrict__ descs, char* ws,
                                                   const double* h, const double* eo,
                                                   const double* en) {
  __shared__ double red[16];
  const Tank3 t = descs[blockIdx.x];
  const int nx = t.nx, ny = t.ny, nh = nx * ny;
  const View3 v = view3(ws, t);
  fft3_twiddles(v.F, nx, ny);
  double* G = wp<double>(ws, t.geo);
  const double* hh = h + t.off2d;
  const double* e0 = eo + t.off2d;
  const double* e1 = en + t.off2d;
  // h_x, h_y into their rows; d_x and d_y of both surfaces into the a/b rows as scratch
  double* HX = G + G_HX * nh;
  double* HY = G + G_HY * nh;
  deriv_rows(ny, nx, v.lgx, v.kfx, v.F, v.F.twx, [=](int r, int i) { return hh[r * nx + i]; },
             [=](int r, int i, double d) { HX[r * nx + i] = d; });
  deriv_rows(nx, ny, v.lgy, v.kfy, v.F, v.F.twy, [=](int r, int i) { return hh[i * nx + r]; },
             [=](int r, int i, double d) { HY[i * nx + r] = d; });
  for (int g = 0; g < 2; ++g) {
    const double* ee = g == 0 ? e0 : e1;
    double* BX = G + (g == 0 ? G_BXO : G_BXN) * nh;
    double* BY = G + (g == 0 ? G_BYO : G_BYN) * nh;
    deriv_rows(ny, nx, v.lgx, v.kfx, v.F, v.F.twx,
               [=](int r, int i) { return hh[r * nx + i] + ee[r * nx + i]; },
               [=](int r, int i, double d) { BX[r * nx + i] = d; });
    deriv_rows(nx, ny, v.lgy, v.kfy, v.F, v.F.twy,
               [=](int r, int i) { return hh[i * nx + r] + ee[i * nx + r]; },
               [=](int r, int i, double d) { BY[i * nx + r] = d; });
  }
  int bad = 0;
  for (int c = tid(); c < nh; c += nthr()) {
    for (int g = 0; g < 2; ++g) {
      const double* ee = g == 0 ? e0 : e1;
      const double d = hh[c] + ee[c];
      if (!(d > 0.0) || !isfinite(d)) bad = 1;
      const double id = 1.0 / d;
      const int o = g == 0 ? 0 : (G_AXN - G_AXO);
      const double dxd = G[(G_BXO + o) * nh + c], dyd = G[(G_BYO + o) * nh + c];
      G[(G_AXO + o) * nh + c] = HX[c] * id;
      G[(G_BXO + o) * nh + c] = -dxd * id;
      G[(G_AYO + o) * nh + c] = HY[c] * id;
      G[(G_BYO + o) * nh + c] = -dyd * id;
      G[(G_IDO + o) * nh + c] = id;
    }
  }
  __syncthreads();
  const double nbad = block_sum((double)bad, red);
  double sc = 0.0, se = 0.0, cmax = 0.0, cmin = 1e300;
  for (int c = tid(); c < nh; c += nthr()) {
    const double cc = G[G_IDO * nh + c] * G[G_IDN * nh + c];
    sc += cc;
    se += (1.0 + HX[c] * HX[c] + HY[c] * HY[c]) * G[G_IDO * nh + c];
    cmax = fmax(cmax, cc);
    cmin = fmin(cmin, cc);
  }
  const double tc = block_sum(sc, red), te = block_sum(se, red);
  const double mx = pmgw::block_max(cmax, red), mn = -pmgw::block_max(-cmin, red);
  if (tid() == 0) {
    double* S = wp<double>(ws, t.scal);
    S[0] = tc / nh;
    S[1] = te / nh;
    const double r = mx / mn;
    S[3] = fmin(1.0, 2.0 / (1.0 + pow(0.5 * r, 0.4)));
    *reinterpret_cast<int32_t*>(S + 2) = (nbad > 0.0) ? ST3_EGEOM : ST3_OK;
  }
}

// Column blocks (kind 0, one per column c) and flat-mode blocks (kind 1, one per mode m) of
// level l, inverted by Gauss-Jordan with partial pivoting in LDS; one wavefront per block.
// blockIdx.x = index within the level's 2 nh blocks, blockIdx.y = level, blockIdx.z = tank.
__global__ void __launch_bounds__(64) k3_blocks(const Tank3* __restrict__ descs, char* ws) {
  __shared__ double A[kMaxNz3][kMaxNz3 + 1];
  __shared__ double Dsl[kMaxNz3][kMaxNz3 + 1];
  __shared__ int piv[kMaxNz3];
  const Tank3& t = descs[blockIdx.z];
  const int l = blockIdx.y;
  if (l >= t.nlev) return;
  const int nx = t.nx, ny = t.ny, nh = nx * ny;
  const int b = blockIdx.x;
  if (b >= 2 * nh) return;
  if (*reinterpret_cast<const int32_t*>(wc<double>(ws, t.scal) + 2) != ST3_OK) return;
  const Lev3& lv = t.lev[l];
  const int nz = lv.nz, M = nz - 1;
  const int th = tid();
  const double* Ds = wc<double>(ws, lv.ds);
  const double* sig = wc<double>(ws, lv.sig);
  for (int e = th; e < nz * nz; e += 64) Dsl[e / nz][e % nz] = Ds[e];
  __syncthreads();
  const bool col = b < nh;
  const int idx = col ? b : b - nh;
  if (col) {
    const double* G = wc<double>(ws, t.geo);
    const int c = idx;
    const double axo = G[G_AXO * nh + c], bxo = G[G_BXO * nh + c];
    const double ayo = G[G_AYO * nh + c], byo = G[G_BYO * nh + c], ido = G[G_IDO * nh + c];
    const double axn = G[G_AXN * nh + c], bxn = G[G_BXN * nh + c];
    const double ayn = G[G_AYN * nh + c], byn = G[G_BYN * nh + c], idn = G[G_IDN * nh + c];
    const double hx = G[G_HX * nh + c], hy = G[G_HY * nh + c];
    if (th < nz) {
      const int j = th;
      const double sxn = axn + bxn * sig[j], syn = ayn + byn * sig[j];
      for (int k = 0; k < nz; ++k) {
        double val;
        if (j == 0) {
          val = (k == 0) ? 1.0 : 0.0;
        } else if (j == M) {
          val = -(hx * (axo + bxo * sig[M]) + hy * (ayo + byo * sig[M]) + ido) * Dsl[M][k];
        } else {
          double s = 0.0;
          for (int q = 0; q < nz; ++q)
            s += Dsl[j][q] * Dsl[q][k] *
                 (sxn * (axo + bxo * sig[q]) + syn * (ayo + byo * sig[q]) + idn * ido);
          val = s + ((k == j) ? (t.cxx + t.cyy) : 0.0);
        }
        A[j][k] = val;
      }
    }
  } else {
    const double* S = wc<double>(ws, t.scal);
    const double cbar = S[0], ebar = S[1];
    const int ky = idx / nx, kx = idx - ky * nx;
    const int kkx = (kx <= nx / 2) ? kx : kx - nx, kky = (ky <= ny / 2) ? ky : ky - ny;
    const double kapx = (kx == nx / 2) ? 0.0 : t.kfx * kkx;
    const double kapy = (ky == ny / 2) ? 0.0 : t.kfy * kky;
    const double k2 = kapx * kapx + kapy * kapy;
    if (th < nz) {
      const int j = th;
      for (int k = 0; k < nz; ++k) {
        double val;
        if (j == 0) {
          val = (k == 0) ? 1.0 : 0.0;
        } else if (j == M) {
          val = -ebar * Dsl[M][k];
        } else {
          double s = 0.0;
          for (int q = 0; q < nz; ++q) s += Dsl[j][q] * Dsl[q][k];
          val = cbar * s - ((k == j) ? k2 : 0.0);
        }
        A[j][k] = val;
      }
    }
  }
  __syncthreads();
  for (int k = 0; k < nz; ++k) {
    double v = -1.0;
    if (th >= k && th < nz) {
      v = fabs(A[th][k]);
      if (!(v >= 0.0)) v = INFINITY;
    }
    int id = th;
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(v, o, 64);
      const int oi = __shfl_xor(id, o, 64);
      if (ov > v || (ov == v && oi < id)) { v = ov; id = oi; }
    }
    const int p = id;
    if (p != k && th < nz) {
      const double tmp = A[k][th];
      A[k][th] = A[p][th];
      A[p][th] = tmp;
    }
    if (th == 0) piv[k] = p;
    __syncthreads();
    const double inv = 1.0 / A[k][k];
    if (th < nz && th != k) {
      const double fr = A[th][k] * inv;
      for (int c = 0; c < nz; ++c)
        if (c != k) A[th][c] -= fr * A[k][c];
      A[th][k] = -fr;
    }
    __syncthreads();
    if (th < nz) A[k][th] = (th == k) ? inv : A[k][th] * inv;
    __syncthreads();
  }
  for (int k = nz - 1; k >= 0; --k) {
    const int p = piv[k];
    if (p != k && th < nz) {
      const double tmp = A[th][k];
      A[th][k] = A[th][p];
      A[th][p] = tmp;
    }
    __syncthreads();
  }
  double* out = wp<double>(ws, col ? lv.colinv : lv.modeinv);
  for (int e = th; e < nz * nz; e += 64) out[(int64_t)e * nh + idx] = A[e / nz][e % nz];
}

}  // namespace pmgw3

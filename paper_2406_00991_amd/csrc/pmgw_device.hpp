// Device building blocks of the p-multigrid Poisson solver (gfx950).
//
// One workgroup owns one tank for the whole solve; every phase below is a loop over the
// workgroup's threads followed by __syncthreads(). Fields are [nz][nx] arrays in global memory
// (they stay in L2 for the tank sizes of interest); the x-FFTs are staged through LDS.
//
//   row phases    (x direction): D_x by FFT (paper Sec. 3.5), flat-mode line solve
//   column phases (sigma):       D_sigma contraction, boundary rows, column-block solve,
//                                restriction and prolongation (Sec. 4.2, 4.3)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

#include "pmgw_layout.hpp"

namespace pmgw {

template <typename T>
struct cpx {
  T re, im;
};
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }

__device__ __forceinline__ int tid() { return (int)threadIdx.x; }
__device__ __forceinline__ int nthr() { return (int)blockDim.x; }

// Sum over the workgroup; every thread returns the same value (fixed summation order).
// `red` is LDS scratch of at least nthr()/64 doubles.
__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = tid() & 63, wid = tid() >> 6, nw = nthr() >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

// ----------------------------------------------------------------------------- FFT in LDS
//
// Stockham auto-sort FFT of `nrows` complex rows of length N = 2^log2N held in LDS buffer a
// (row r at a + r N), ping-ponging with b. One radix-2 pass first when log2N is odd, then
// radix-4 passes; p is the length of the sub-transforms already done. Returns the buffer that
// holds the (natural-order) result. Forward: exp(-2 pi i / N) kernel; inverse: conjugate,
// unscaled. tw[t] = exp(-2 pi i t / N) for t < N.
template <typename T, bool INV>
__device__ cpx<T>* fft_lds(cpx<T>* a, cpx<T>* b, int nrows, int N, int log2N,
                           const cpx<T>* __restrict__ tw) {
  int p = 1;
  if (log2N & 1) {
    const int h = N >> 1, items = nrows << (log2N - 1);
    for (int it = tid(); it < items; it += nthr()) {
      const int r = it >> (log2N - 1), i = it & (h - 1);
      const cpx<T>* s = a + r * N;
      cpx<T>* d = b + r * N;
      const cpx<T> u0 = s[i], u1 = s[i + h];
      d[2 * i] = cadd(u0, u1);
      d[2 * i + 1] = csub(u0, u1);
    }
    __syncthreads();
    cpx<T>* t = a; a = b; b = t;
    p = 2;
  }
  while (p < N) {
    const int q = N >> 2, items = nrows << (log2N - 2);
    const int tstep = N / (4 * p);
    for (int it = tid(); it < items; it += nthr()) {
      const int r = it >> (log2N - 2), i = it & (q - 1), k = i & (p - 1);
      const cpx<T>* s = a + r * N;
      cpx<T>* d = b + r * N;
      cpx<T> u0 = s[i], u1 = s[i + q], u2 = s[i + 2 * q], u3 = s[i + 3 * q];
      if (p > 1) {
        const int t = k * tstep;
        cpx<T> w1 = tw[t], w2 = tw[2 * t], w3 = tw[3 * t];
        if (INV) { w1.im = -w1.im; w2.im = -w2.im; w3.im = -w3.im; }
        u1 = cmul(u1, w1);
        u2 = cmul(u2, w2);
        u3 = cmul(u3, w3);
      }
      const cpx<T> v0 = cadd(u0, u2), v1 = csub(u0, u2), v2 = cadd(u1, u3);
      const cpx<T> dd = csub(u1, u3);
      const cpx<T> v3 = INV ? cpx<T>{-dd.im, dd.re} : cpx<T>{dd.im, -dd.re};
      const int j = ((i - k) << 2) + k;
      d[j] = cadd(v0, v2);
      d[j + p] = cadd(v1, v3);
      d[j + 2 * p] = csub(v0, v2);
      d[j + 3 * p] = csub(v1, v3);
    }
    __syncthreads();
    cpx<T>* t = a; a = b; b = t;
    p <<= 2;
  }
  return a;
}

template <typename T>
__device__ __forceinline__ int fft_cap() { return kFftBytes / (int)sizeof(cpx<T>); }

// D_x of `nrows` real rows (paper Sec. 3.5: F^-1(i kappa F f), Nyquist coefficient zeroed).
// Two real rows are packed into one complex FFT (D_x is a real operator, so real and
// imaginary parts stay separate). ld(j, i) reads input row j at column i; st(j, i, v) writes
// the derivative. Ends with a barrier.
template <typename T, class LD, class ST>
__device__ void dx_rows(int nrows, int N, int log2N, T kfac, const cpx<T>* __restrict__ tw,
                        cpx<T>* lds, LD ld, ST st) {
  const int cap = fft_cap<T>();
  cpx<T>* A0 = lds;
  cpx<T>* B0 = lds + cap;
  const int rpb = cap >> log2N;
  const int npairs = (nrows + 1) >> 1;
  const T scale = T(1) / T(N);
  for (int p0 = 0; p0 < npairs; p0 += rpb) {
    const int nb = min(rpb, npairs - p0);
    const int items = nb << log2N;
    for (int it = tid(); it < items; it += nthr()) {
      const int q = it >> log2N, n = it & (N - 1), ra = 2 * (p0 + q);
      const T re = ld(ra, n);
      const T im = (ra + 1 < nrows) ? ld(ra + 1, n) : T(0);
      A0[it] = {re, im};
    }
    __syncthreads();
    cpx<T>* R = fft_lds<T, false>(A0, B0, nb, N, log2N, tw);
    for (int it = tid(); it < items; it += nthr()) {
      const int n = it & (N - 1);
      const int kk = (n <= (N >> 1)) ? n : n - N;
      const T kap = (n == (N >> 1)) ? T(0) : kfac * T(kk) * scale;
      const cpx<T> v = R[it];
      R[it] = {-kap * v.im, kap * v.re};
    }
    __syncthreads();
    cpx<T>* S = fft_lds<T, true>(R, R == A0 ? B0 : A0, nb, N, log2N, tw);
    for (int it = tid(); it < items; it += nthr()) {
      const int q = it >> log2N, n = it & (N - 1), ra = 2 * (p0 + q);
      st(ra, n, S[it].re);
      if (ra + 1 < nrows) st(ra + 1, n, S[it].im);
    }
    __syncthreads();
  }
}

// Forward FFT of real rows, packed in pairs, into spec[(nrows+1)/2][N] (global). Barrier at end.
template <typename T, class LD>
__device__ void rows_fft_to_global(int nrows, int N, int log2N, const cpx<T>* __restrict__ tw,
                                   cpx<T>* lds, LD ld, cpx<T>* spec) {
  const int cap = fft_cap<T>();
  cpx<T>* A0 = lds;
  cpx<T>* B0 = lds + cap;
  const int rpb = cap >> log2N;
  const int npairs = (nrows + 1) >> 1;
  for (int p0 = 0; p0 < npairs; p0 += rpb) {
    const int nb = min(rpb, npairs - p0);
    const int items = nb << log2N;
    for (int it = tid(); it < items; it += nthr()) {
      const int q = it >> log2N, n = it & (N - 1), ra = 2 * (p0 + q);
      A0[it] = {ld(ra, n), (ra + 1 < nrows) ? ld(ra + 1, n) : T(0)};
    }
    __syncthreads();
    cpx<T>* R = fft_lds<T, false>(A0, B0, nb, N, log2N, tw);
    for (int it = tid(); it < items; it += nthr()) spec[(p0 << log2N) + it] = R[it];
    __syncthreads();
  }
}

// Inverse FFT (unscaled) of packed spectra spec[(nrows+1)/2][N]; st(j, i, v) receives the real
// rows. Barrier at end.
template <typename T, class ST>
__device__ void rows_ifft_from_global(int nrows, int N, int log2N, const cpx<T>* __restrict__ tw,
                                      cpx<T>* lds, const cpx<T>* spec, ST st) {
  const int cap = fft_cap<T>();
  cpx<T>* A0 = lds;
  cpx<T>* B0 = lds + cap;
  const int rpb = cap >> log2N;
  const int npairs = (nrows + 1) >> 1;
  for (int p0 = 0; p0 < npairs; p0 += rpb) {
    const int nb = min(rpb, npairs - p0);
    const int items = nb << log2N;
    for (int it = tid(); it < items; it += nthr()) A0[it] = spec[(p0 << log2N) + it];
    __syncthreads();
    cpx<T>* S = fft_lds<T, true>(A0, B0, nb, N, log2N, tw);
    for (int it = tid(); it < items; it += nthr()) {
      const int q = it >> log2N, n = it & (N - 1), ra = 2 * (p0 + q);
      st(ra, n, S[it].re);
      if (ra + 1 < nrows) st(ra + 1, n, S[it].im);
    }
    __syncthreads();
  }
}

// Flat-mode line solve in Fourier space: for each mode k in [0, N/2], unpack the spectra of
// the nz real rows from the packed pairs, multiply by the inverse mode block (real, the same
// for k and N-k), repack, and fold in the 1/N of the inverse FFT. minv is [NZ][NZ][N/2+1].
template <typename T, int NZ>
__device__ void mode_matvec(int N, const T* __restrict__ minv, cpx<T>* spec) {
  constexpr int NP = (NZ + 1) / 2;
  const int nh = (N >> 1) + 1;
  const T half = T(0.5), scale = T(1) / T(N);
  for (int k = tid(); k < nh; k += nthr()) {
    const int kc = (N - k) & (N - 1);
    cpx<T> rh[NZ];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const cpx<T> z = spec[p * N + k], zc = spec[p * N + kc];
      rh[2 * p] = {half * (z.re + zc.re), half * (z.im - zc.im)};
      if (2 * p + 1 < NZ) rh[2 * p + 1] = {half * (z.im + zc.im), -half * (z.re - zc.re)};
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      cpx<T> s0 = {T(0), T(0)}, s1 = {T(0), T(0)};
      const int j0 = 2 * p, j1 = 2 * p + 1;
#pragma unroll
      for (int l = 0; l < NZ; ++l) {
        const T a = minv[(j0 * NZ + l) * nh + k];
        s0.re += a * rh[l].re;
        s0.im += a * rh[l].im;
        if (j1 < NZ) {
          const T c = minv[(j1 * NZ + l) * nh + k];
          s1.re += c * rh[l].re;
          s1.im += c * rh[l].im;
        }
      }
      s0.re *= scale; s0.im *= scale; s1.re *= scale; s1.im *= scale;
      spec[p * N + k] = {s0.re - s1.im, s0.im + s1.re};
      if (k != 0 && k != (N >> 1)) spec[p * N + kc] = {s0.re + s1.im, s1.re - s0.im};
    }
  }
}

// ----------------------------------------------------------------------------- geometry

template <typename T>
struct Geo {
  const T *ao, *bo, *ido, *an, *bn, *idn, *hx;   // sigma_x = a + b sigma; ido = 1/d
};

template <typename T>
struct Lev {
  int nz, nzc;
  const T *Ds, *sig, *colinv, *modeinv, *R, *P;
  T *x, *f, *r, *t1, *t2, *t3;
  cpx<T>* spec;
};

template <typename T>
struct Ctx {
  int nx, log2nx;
  T kfac;
  const cpx<T>* tw;
  Geo<T> g;
  cpx<T>* lds;
};

// ----------------------------------------------------------------------------- column phases

// out = D_sigma in, column by column.
template <typename T, int NZ>
__device__ void col_dsig(int nx, const T* __restrict__ Ds, const T* in, T* out) {
  for (int i = tid(); i < nx; i += nthr()) {
    T v[NZ];
#pragma unroll
    for (int l = 0; l < NZ; ++l) v[l] = in[l * nx + i];
#pragma unroll
    for (int j = 0; j < NZ; ++j) {
      T s = T(0);
#pragma unroll
      for (int l = 0; l < NZ; ++l) s += Ds[j * NZ + l] * v[l];
      out[j * nx + i] = s;
    }
  }
}

enum : int { FIN_APPLY = 0, FIN_RESID = 1, FIN_COLSTEP = 2 };

// Last phase of the operator: A in = D_x G_x + sx_new D_s G_x + D_s G_z / d_new on interior
// rows, row 0 = in (Dirichlet), row M = -(h_x G_x + G_z) (bed). gz, gx are G_z, G_x; dxgx holds
// D_x G_x and is used as scratch. With sx_new = a_n + b_n sigma the interior rows are
//   D_x G_x + D_s (a_n G_x + G_z / d_n) + b_n sigma D_s G_x,
// evaluated in two column passes that each hold one column in registers. FIN_APPLY writes A in
// to out; FIN_RESID writes f - A in; FIN_COLSTEP also applies x += omega B_i^-1 (f - A in)_i
// column by column (x may alias in).
template <typename T, int NZ, int MODE>
__device__ __forceinline__ void col_finish(int nx, const T* __restrict__ Ds,
                                           const T* __restrict__ sig, const Geo<T>& g,
                                           const T* in, const T* gz, const T* gx, T* dxgx, T* out,
                                           const T* f, T* x, const T* __restrict__ cinv,
                                           T omega) {
  for (int i = tid(); i < nx; i += nthr()) {
    const T an = g.an[i], bn = g.bn[i], idn = g.idn[i];
    {
      T u[NZ];
#pragma unroll
      for (int l = 0; l < NZ; ++l) u[l] = an * gx[l * nx + i] + idn * gz[l * nx + i];
#pragma unroll
      for (int j = 1; j < NZ - 1; ++j) {
        T s = T(0);
#pragma unroll
        for (int l = 0; l < NZ; ++l) s += Ds[j * NZ + l] * u[l];
        dxgx[j * nx + i] += s;
      }
    }
    {
      T v[NZ];
#pragma unroll
      for (int l = 0; l < NZ; ++l) v[l] = gx[l * nx + i];
      const T bed = -(g.hx[i] * v[NZ - 1] + gz[(NZ - 1) * nx + i]);
#pragma unroll
      for (int j = 0; j < NZ; ++j) {
        T o;
        if (j == 0) {
          o = in[i];
        } else if (j == NZ - 1) {
          o = bed;
        } else {
          T s = T(0);
#pragma unroll
          for (int l = 0; l < NZ; ++l) s += Ds[j * NZ + l] * v[l];
          o = dxgx[j * nx + i] + bn * sig[j] * s;
        }
        if (MODE == FIN_APPLY) out[j * nx + i] = o;
        else out[j * nx + i] = f[j * nx + i] - o;
      }
    }
    if (MODE == FIN_COLSTEP) {
      T r[NZ];
#pragma unroll
      for (int l = 0; l < NZ; ++l) r[l] = out[l * nx + i];
#pragma unroll
      for (int j = 0; j < NZ; ++j) {
        T s = T(0);
#pragma unroll
        for (int l = 0; l < NZ; ++l) s += cinv[(j * NZ + l) * nx + i] * r[l];
        x[j * nx + i] += omega * s;
      }
    }
  }
}

// x = omega B_i^-1 f_i (column step from a zero iterate: the residual is f).
template <typename T, int NZ>
__device__ void col_solve_zero(int nx, const T* __restrict__ cinv, const T* f, T* x, T omega) {
  for (int i = tid(); i < nx; i += nthr()) {
    T v[NZ];
#pragma unroll
    for (int l = 0; l < NZ; ++l) v[l] = f[l * nx + i];
#pragma unroll
    for (int j = 0; j < NZ; ++j) {
      T s = T(0);
#pragma unroll
      for (int l = 0; l < NZ; ++l) s += cinv[(j * NZ + l) * nx + i] * v[l];
      x[j * nx + i] = omega * s;
    }
  }
}

// fc = R r (restriction to the next coarser order, NZC = (NZ+1)/2 rows).
template <typename T, int NZ>
__device__ void col_restrict(int nx, const T* __restrict__ R, const T* r, T* fc) {
  constexpr int NZC = (NZ + 1) / 2;
  for (int i = tid(); i < nx; i += nthr()) {
    T v[NZ];
#pragma unroll
    for (int l = 0; l < NZ; ++l) v[l] = r[l * nx + i];
#pragma unroll
    for (int j = 0; j < NZC; ++j) {
      T s = T(0);
#pragma unroll
      for (int l = 0; l < NZ; ++l) s += R[j * NZ + l] * v[l];
      fc[j * nx + i] = s;
    }
  }
}

// x += P xc (prolongation from the next coarser order).
template <typename T, int NZ>
__device__ void col_prolong_add(int nx, const T* __restrict__ P, const T* xc, T* x) {
  constexpr int NZC = (NZ + 1) / 2;
  for (int i = tid(); i < nx; i += nthr()) {
    T v[NZC];
#pragma unroll
    for (int c = 0; c < NZC; ++c) v[c] = xc[c * nx + i];
#pragma unroll
    for (int j = 0; j < NZ; ++j) {
      T s = T(0);
#pragma unroll
      for (int c = 0; c < NZC; ++c) s += P[j * NZC + c] * v[c];
      x[j * nx + i] += s;
    }
  }
}

// ----------------------------------------------------------------------------- operator

// The composite operator on one level of NZ rows (paper eq. poissonp, eq. bcpd, eq. bcpdneu):
//   A: t1 = D_s in                                        (column phase)
//   B: t2 = G_x = D_x in + sx_old t1; t1 = G_z = t1/d_old (row FFTs + epilogue)
//   C: t3 = D_x G_x                                       (row FFTs)
//   D: finish (column phase, see col_finish)
template <typename T, int NZ, int MODE>
__device__ __noinline__ void op_apply(const Ctx<T>& c, const Lev<T>& L, const T* in, T* out,
                                         const T* f, T* x, T omega) {
  const int nx = c.nx;
  T* t1 = L.t1;
  T* t2 = L.t2;
  T* t3 = L.t3;
  const T* sig = L.sig;
  const Geo<T> g = c.g;
  col_dsig<T, NZ>(nx, L.Ds, in, t1);
  __syncthreads();
  dx_rows<T>(NZ, nx, c.log2nx, c.kfac, c.tw, c.lds,
             [=](int j, int i) { return in[j * nx + i]; },
             [=](int j, int i, T v) {
               const T ps = t1[j * nx + i];
               t2[j * nx + i] = v + (g.ao[i] + g.bo[i] * sig[j]) * ps;
               t1[j * nx + i] = ps * g.ido[i];
             });
  dx_rows<T>(NZ, nx, c.log2nx, c.kfac, c.tw, c.lds,
             [=](int j, int i) { return t2[j * nx + i]; },
             [=](int j, int i, T v) { t3[j * nx + i] = v; });
  col_finish<T, NZ, MODE>(nx, L.Ds, sig, g, in, t1, t2, t3, out, f, x, L.colinv, omega);
  __syncthreads();
}

// One smoothing pair on a level: column-block step x += omega_c B^-1 (f - A x), then the
// flat-mode step x += omega_m F^-1 Ahat^-1 F (f - A x). xzero: x is known to be zero.
template <typename T, int NZ>
__device__ __noinline__ void smooth_pair(const Ctx<T>& c, const Lev<T>& L, bool xzero,
                                            T omega_c, T omega_m) {
  const int nx = c.nx;
  if (xzero) {
    col_solve_zero<T, NZ>(nx, L.colinv, L.f, L.x, omega_c);
    __syncthreads();
  } else {
    op_apply<T, NZ, FIN_COLSTEP>(c, L, L.x, L.r, L.f, L.x, omega_c);
  }
  op_apply<T, NZ, FIN_RESID>(c, L, L.x, L.r, L.f, nullptr, T(0));
  const T* r = L.r;
  rows_fft_to_global<T>(NZ, nx, c.log2nx, c.tw, c.lds,
                        [=](int j, int i) { return r[j * nx + i]; }, L.spec);
  mode_matvec<T, NZ>(nx, L.modeinv, L.spec);
  __syncthreads();
  T* x = L.x;
  rows_ifft_from_global<T>(NZ, nx, c.log2nx, c.tw, c.lds, L.spec,
                           [=](int j, int i, T v) { x[j * nx + i] += omega_m * v; });
}

template <typename T>
__device__ __forceinline__ void fill_zero(T* p, int n) {
  for (int e = tid(); e < n; e += nthr()) p[e] = T(0);
}

// The V-cycle (paper Alg. 1) from a zero guess on the levels l, l+1, ..., whose row counts are
// NZ, (NZ+1)/2, ..., 3 (order halves per level). lev(l) returns the Lev of level l; input
// lev(l).f, output lev(l).x. The recursion is resolved at compile time.
template <typename T, int NZ, class LP>
__device__ __noinline__ void vcycle(const Ctx<T>& c, const LP& lev, int l, const KOpts& o) {
  const int nx = c.nx;
  const T wc = T(o.omega_c), wm = T(o.omega_m);
  const Lev<T> L = lev(l);
  if constexpr (NZ == 3) {
    for (int s = 0; s < o.coarse_pairs; ++s) smooth_pair<T, 3>(c, L, s == 0, wc, wm);
    if (o.coarse_pairs == 0) {
      fill_zero(L.x, 3 * nx);
      __syncthreads();
    }
  } else {
    constexpr int NZC = (NZ + 1) / 2;
    for (int s = 0; s < o.nu1; ++s) smooth_pair<T, NZ>(c, L, s == 0, wc, wm);
    const T* rr = L.f;
    if (o.nu1 > 0) {
      op_apply<T, NZ, FIN_RESID>(c, L, L.x, L.r, L.f, nullptr, T(0));
      rr = L.r;
    } else {
      fill_zero(L.x, NZ * nx);
    }
    const Lev<T> C = lev(l + 1);
    col_restrict<T, NZ>(nx, L.R, rr, C.f);
    __syncthreads();
    vcycle<T, NZC>(c, lev, l + 1, o);
    col_prolong_add<T, NZ>(nx, L.P, C.x, L.x);
    __syncthreads();
    for (int s = 0; s < o.nu2; ++s) smooth_pair<T, NZ>(c, L, false, wc, wm);
  }
}

}  // namespace pmgw

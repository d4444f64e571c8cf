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

// Global-memory pointers: accesses through them compile to global (not flat) memory
// instructions, which keeps field traffic off the counter that scalar and LDS loads wait on.
#define PMGW_GLOBAL __attribute__((address_space(1)))
template <typename T>
using gptr = PMGW_GLOBAL T*;
template <typename T>
__device__ __forceinline__ gptr<T> as_global(T* p) { return (gptr<T>)p; }

// LDS pointers, for code that is not inlined into the function owning the LDS buffer: accesses
// through them compile to ds_* instructions (a generic pointer would give flat instructions).
#define PMGW_LOCAL __attribute__((address_space(3)))
template <typename T>
using lptr = PMGW_LOCAL T*;
template <typename T>
__device__ __forceinline__ lptr<T> as_lds(T* p) { return (lptr<T>)p; }

// Constant-address-space view of tables that no kernel writes while it runs (the Chebyshev
// matrices, nodes and transfer matrices of the levels, the sigma filter). Reads at a
// wavefront-uniform index then compile to scalar loads. Those are waited on through their own
// counter, so they do not queue behind the vector stores of a column phase, as vector loads of
// the same tables did (the vector-memory counter retires loads and stores in order).
#define PMGW_CONST __attribute__((address_space(4)))
template <typename T>
using cptr = const PMGW_CONST T*;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(PMGW_GLOBAL const T* p) { return (cptr<T>)p; }

template <typename T>
struct cpx {
  T re, im;
};
// Complex values in global memory, read and written member by member.
template <typename T>
__device__ __forceinline__ cpx<T> gld(gptr<const cpx<T>> p, int i) {
  return {p[i].re, p[i].im};
}
template <typename T>
__device__ __forceinline__ cpx<T> gld(gptr<cpx<T>> p, int i) {
  return {p[i].re, p[i].im};
}
template <typename T>
__device__ __forceinline__ void gst(gptr<cpx<T>> p, int i, cpx<T> v) {
  p[i].re = v.re;
  p[i].im = v.im;
}

template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }

// Complex values in LDS through lptr, member by member.
template <typename T>
__device__ __forceinline__ cpx<T> lld(lptr<const cpx<T>> p, int i) {
  return {p[i].re, p[i].im};
}
template <typename T>
__device__ __forceinline__ cpx<T> lld(lptr<cpx<T>> p, int i) {
  return {p[i].re, p[i].im};
}
template <typename T>
__device__ __forceinline__ void lst(lptr<cpx<T>> p, int i, cpx<T> v) {
  p[i].re = v.re;
  p[i].im = v.im;
}

__device__ __forceinline__ int tid() { return (int)threadIdx.x; }
__device__ __forceinline__ int nthr() { return (int)blockDim.x; }

// Workgroup-uniform values passed through a function call arrive in vector registers; these
// helpers move them back to scalar registers (every lane holds the same value) so that the
// callee addresses its tables with scalar loads.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uni(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uni(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename P>
__device__ __forceinline__ P* uni(P* p) {
  const unsigned long long u = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(u & 0xffffffffULL));
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(u >> 32));
  return reinterpret_cast<P*>(((unsigned long long)hi << 32) | lo);
}

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

// Maximum over the workgroup; every thread returns the same value.
__device__ __forceinline__ double block_max(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  const int lane = tid() & 63, wid = tid() >> 6, nw = nthr() >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = red[0];
  for (int i = 1; i < nw; ++i) s = fmax(s, red[i]);
  return s;
}

// ----------------------------------------------------------------------------- FFT in LDS
//
// Stockham auto-sort FFT of `nrows` complex rows of length N = 2^log2N held in LDS buffer a
// (row r at a + r N), ping-ponging with b. One radix-2 pass first when log2N is odd, then
// radix-4 passes; p is the length of the sub-transforms already done. Returns the buffer that
// holds the (natural-order) result. Forward: exp(-2 pi i / N) kernel; inverse: conjugate,
// unscaled. tw[t] = exp(-2 pi i t / N) for t < N, in LDS (see lds_tw).
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

// LDS staging buffer of the row FFTs: dynamic shared memory of 2 * fftb bytes (two ping-pong
// halves for the workgroup-wide FFT; per-wavefront rows for the wavefront FFT). It is declared
// at namespace scope so that every function of a kernel addresses it as LDS.
extern __shared__ double g_fft_lds[];

template <typename T>
__device__ __forceinline__ cpx<T>* fft_buf() {
  return reinterpret_cast<cpx<T>*>(g_fft_lds);
}

template <typename T>
__device__ __forceinline__ int fft_cap(int fftb) { return fftb / (int)sizeof(cpx<T>); }

// Twiddle tables in LDS, after the two FFT halves: N float64 values, then N float32 values.
// A launch whose kernels run FFTs reserves 2 fftb + 24 N bytes of dynamic LDS (N = the largest
// Nx among its tanks), and the kernel copies its tank's tables there first (stage_twiddles).
template <typename T>
__device__ __forceinline__ cpx<T>* lds_tw(int fftb, int N) {
  char* b = reinterpret_cast<char*>(g_fft_lds) + 2 * fftb + (sizeof(T) == 4 ? 16 * N : 0);
  return reinterpret_cast<cpx<T>*>(b);
}

__device__ __forceinline__ void stage_twiddles(gptr<const cpx<double>> t64,
                                               gptr<const cpx<float>> t32, int N, int fftb) {
  cpx<double>* d = lds_tw<double>(fftb, N);
  cpx<float>* f = lds_tw<float>(fftb, N);
  for (int t = tid(); t < N; t += nthr()) {
    d[t] = gld<double>(t64, t);
    f[t] = gld<float>(t32, t);
  }
  __syncthreads();
}

// Orders LDS accesses of one wavefront: every lane's earlier LDS writes are seen by the later
// reads of the other lanes of the same wavefront (LDS executes a wavefront's operations in
// order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The Stockham FFT of fft_lds for nr <= RM rows at a, a + rs, ..., a + (nr-1) rs of length N
// (64 <= N <= 512; row stride rs >= N, in complex elements), owned by one wavefront and done in
// place: each radix pass reads the inputs of all rows before one wavefront sync and writes all
// outputs before the next, so the rows' LDS and arithmetic latencies overlap; the twiddles of a
// butterfly are read once for all rows.
template <typename T, bool INV, int RM>
__device__ void fft_wave_m(lptr<cpx<T>> a, int nr, int N, int log2N, lptr<const cpx<T>> tw,
                           int lane, int rs) {
  int p = 1;
  if (log2N & 1) {
    const int h = N >> 1;
    cpx<T> r[RM][8];
#pragma unroll
    for (int q = 0; q < RM; ++q) {
      if (q < nr) {
        const lptr<cpx<T>> s = a + q * rs;
#pragma unroll
        for (int it = 0; it < 4; ++it) {
          const int i = lane + 64 * it;
          if (i < h) { r[q][2 * it] = lld<T>(s, i); r[q][2 * it + 1] = lld<T>(s, i + h); }
        }
      }
    }
    wave_sync();
#pragma unroll
    for (int q = 0; q < RM; ++q) {
      if (q < nr) {
        const lptr<cpx<T>> d = a + q * rs;
#pragma unroll
        for (int it = 0; it < 4; ++it) {
          const int i = lane + 64 * it;
          if (i < h) {
            lst<T>(d, 2 * i, cadd(r[q][2 * it], r[q][2 * it + 1]));
            lst<T>(d, 2 * i + 1, csub(r[q][2 * it], r[q][2 * it + 1]));
          }
        }
      }
    }
    wave_sync();
    p = 2;
  }
  while (p < N) {
    const int qn = N >> 2;
    const int tstep = N / (4 * p);
    cpx<T> r[RM][8];
#pragma unroll
    for (int q = 0; q < RM; ++q) {
      if (q < nr) {
        const lptr<cpx<T>> s = a + q * rs;
#pragma unroll
        for (int it = 0; it < 2; ++it) {
          const int i = lane + 64 * it;
          if (i < qn) {
            r[q][4 * it] = lld<T>(s, i); r[q][4 * it + 1] = lld<T>(s, i + qn);
            r[q][4 * it + 2] = lld<T>(s, i + 2 * qn); r[q][4 * it + 3] = lld<T>(s, i + 3 * qn);
          }
        }
      }
    }
    wave_sync();
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const int i = lane + 64 * it;
      if (i < qn) {
        const int k = i & (p - 1);
        cpx<T> w1 = {T(1), T(0)}, w2 = w1, w3 = w1;
        if (p > 1) {
          const int t = k * tstep;
          w1 = lld<T>(tw, t); w2 = lld<T>(tw, 2 * t); w3 = lld<T>(tw, 3 * t);
          if (INV) { w1.im = -w1.im; w2.im = -w2.im; w3.im = -w3.im; }
        }
        const int j = ((i - k) << 2) + k;
#pragma unroll
        for (int q = 0; q < RM; ++q) {
          if (q < nr) {
            cpx<T> u0 = r[q][4 * it], u1 = r[q][4 * it + 1], u2 = r[q][4 * it + 2];
            cpx<T> u3 = r[q][4 * it + 3];
            if (p > 1) {
              u1 = cmul(u1, w1);
              u2 = cmul(u2, w2);
              u3 = cmul(u3, w3);
            }
            const cpx<T> v0 = cadd(u0, u2), v1 = csub(u0, u2), v2 = cadd(u1, u3);
            const cpx<T> dd = csub(u1, u3);
            const cpx<T> v3 = INV ? cpx<T>{-dd.im, dd.re} : cpx<T>{dd.im, -dd.re};
            const lptr<cpx<T>> d = a + q * rs;
            lst<T>(d, j, cadd(v0, v2));
            lst<T>(d, j + p, cadd(v1, v3));
            lst<T>(d, j + 2 * p, csub(v0, v2));
            lst<T>(d, j + 3 * p, csub(v1, v3));
          }
        }
      }
    }
    wave_sync();
    p <<= 2;
  }
}

// Rows of the multi-row wavefront FFT: at most kWaveRows row pairs per wavefront and round.
constexpr int kWaveRows = 3;

// Row pairs per wavefront and round for the wavefront FFT (bounded by kWaveRows, by what the
// FFT buffer holds, and by the work: npairs spread over the wavefronts).
template <typename T>
__device__ __forceinline__ int wave_rows(int N, int fftb, int npairs) {
  const int nw = nthr() >> 6;
  const int fit = (2 * fft_cap<T>(fftb)) / (nw * N);
  const int need = (npairs + nw - 1) / nw;
  return max(1, min(kWaveRows, min(fit, need)));
}

// Load row pairs pp0, pp0 + nw, ... (nr of them) as packed complex rows into A, A + N, ...: all
// global loads are issued before the first LDS write.
template <typename T, class LD>
__device__ __forceinline__ void wave_load_pairs(cpx<T>* A, int nr, int N, int lane, int pp0,
                                                int nw, int nrows, LD ld) {
  cpx<T> v[kWaveRows][8];
#pragma unroll
  for (int q = 0; q < kWaveRows; ++q) {
    if (q < nr) {
      const int ra = 2 * (pp0 + q * nw);
#pragma unroll
      for (int it = 0; it < 8; ++it) {
        const int n = lane + 64 * it;
        if (n < N) v[q][it] = {ld(ra, n), (ra + 1 < nrows) ? ld(ra + 1, n) : T(0)};
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kWaveRows; ++q) {
    if (q < nr) {
#pragma unroll
      for (int it = 0; it < 8; ++it) {
        const int n = lane + 64 * it;
        if (n < N) A[q * N + n] = v[q][it];
      }
    }
  }
}

// Hand the wavefront's LDS rows back as real row pairs: LDS reads first, then st().
template <typename T, class ST>
__device__ __forceinline__ void wave_store_pairs(const cpx<T>* A, int nr, int N, int lane,
                                                 int pp0, int nw, int nrows, ST st) {
  cpx<T> v[kWaveRows][8];
#pragma unroll
  for (int q = 0; q < kWaveRows; ++q) {
    if (q < nr) {
#pragma unroll
      for (int it = 0; it < 8; ++it) {
        const int n = lane + 64 * it;
        if (n < N) v[q][it] = A[q * N + n];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kWaveRows; ++q) {
    if (q < nr) {
      const int ra = 2 * (pp0 + q * nw);
#pragma unroll
      for (int it = 0; it < 8; ++it) {
        const int n = lane + 64 * it;
        if (n < N) {
          st(ra, n, v[q][it].re);
          if (ra + 1 < nrows) st(ra + 1, n, v[q][it].im);
        }
      }
    }
  }
}

// Store target of an inverse row FFT: x = w v, or x += w v when add (x has row stride nx).
template <typename T>
struct Axpy {
  gptr<T> x;
  int nx;
  T w;
  bool add;
  __device__ __forceinline__ void operator()(int j, int i, T v) const {
    if (add) x[j * nx + i] += w * v;
    else x[j * nx + i] = w * v;
  }
};

// wave_store_pairs for an Axpy target. With add, every old value of x is loaded before the first
// store: a load issued after a store waits for that store (the vector-memory counter retires both
// in order), which would cost a memory round trip per element.
template <typename T>
__device__ __forceinline__ void wave_axpy_pairs(const cpx<T>* A, int nr, int N, int lane,
                                                int pp0, int nw, int nrows, const Axpy<T>& st) {
  cpx<T> v[kWaveRows][8], o[kWaveRows][8];
#pragma unroll
  for (int q = 0; q < kWaveRows; ++q) {
    if (q < nr) {
#pragma unroll
      for (int it = 0; it < 8; ++it) {
        const int n = lane + 64 * it;
        if (n < N) v[q][it] = A[q * N + n];
      }
    }
  }
  if (st.add) {
#pragma unroll
    for (int q = 0; q < kWaveRows; ++q) {
      if (q < nr) {
        const int ra = 2 * (pp0 + q * nw);
#pragma unroll
        for (int it = 0; it < 8; ++it) {
          const int n = lane + 64 * it;
          if (n < N) {
            o[q][it].re = st.x[ra * st.nx + n];
            o[q][it].im = (ra + 1 < nrows) ? st.x[(ra + 1) * st.nx + n] : T(0);
          }
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kWaveRows; ++q) {
    if (q < nr) {
      const int ra = 2 * (pp0 + q * nw);
#pragma unroll
      for (int it = 0; it < 8; ++it) {
        const int n = lane + 64 * it;
        if (n < N) {
          st.x[ra * st.nx + n] = st.add ? o[q][it].re + st.w * v[q][it].re : st.w * v[q][it].re;
          if (ra + 1 < nrows)
            st.x[(ra + 1) * st.nx + n] =
                st.add ? o[q][it].im + st.w * v[q][it].im : st.w * v[q][it].im;
        }
      }
    }
  }
}

// Whether the per-wavefront FFT path applies: 64 <= N <= 512 and one N-row per wavefront fits.
template <typename T>
__device__ __forceinline__ bool fft_by_wave(int N, int fftb) {
  return N >= 64 && N <= 512 && N * (nthr() >> 6) <= 2 * fft_cap<T>(fftb);
}

// ----------------------------------------------------------------------------- 16 x 16 transform
//
// Rows of N = 256 by the four-step split N = 16 x 16, sixteen lanes per (packed) row: lane t of a
// group holds x[t + 16 r] in v[r]. A 16-point DFT in registers over r, the twiddles W_256^(t s),
// one transpose through LDS and a second 16-point DFT leave X[t + 16 u] in v[u]: one LDS round
// trip per transform instead of one per radix-4 pass.

// W_16^e a for the exponents e = n1 k1 (n1, k1 < 4) of the 4 x 4 split of a 16-point DFT.
template <typename T>
__device__ __forceinline__ cpx<T> fs16_twiddle(cpx<T> a, int e) {
  const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173);
  const T h = T(0.70710678118654752440);
  switch (e) {
    case 1: return {c1 * a.re + s1 * a.im, c1 * a.im - s1 * a.re};
    case 2: return {h * (a.re + a.im), h * (a.im - a.re)};
    case 3: return {s1 * a.re + c1 * a.im, s1 * a.im - c1 * a.re};
    case 4: return {a.im, -a.re};
    case 6: return {h * (a.im - a.re), -h * (a.re + a.im)};
    case 9: return {-c1 * a.re - s1 * a.im, s1 * a.re - c1 * a.im};
    default: return a;
  }
}

// Forward 4-point DFT in place.
template <typename T>
__device__ __forceinline__ void fs16_dft4(cpx<T>& a0, cpx<T>& a1, cpx<T>& a2, cpx<T>& a3) {
  const cpx<T> s02 = cadd(a0, a2), d02 = csub(a0, a2), s13 = cadd(a1, a3), d13 = csub(a1, a3);
  const cpx<T> md = {d13.im, -d13.re};   // -i (a1 - a3)
  a0 = cadd(s02, s13);
  a1 = cadd(d02, md);
  a2 = csub(s02, s13);
  a3 = csub(d02, md);
}

// Forward 16-point DFT of v in registers: with n = n1 + 4 n2 and k = k1 + 4 k2,
// X[k1 + 4 k2] = sum_n1 W_4^(n1 k2) W_16^(n1 k1) sum_n2 v[n1 + 4 n2] W_4^(n2 k1).
template <typename T>
__device__ __forceinline__ void fs16_dft(cpx<T> (&v)[16]) {
  cpx<T> a[4][4];
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) {
    cpx<T> q0 = v[n1], q1 = v[n1 + 4], q2 = v[n1 + 8], q3 = v[n1 + 12];
    fs16_dft4(q0, q1, q2, q3);
    a[n1][0] = q0;
    a[n1][1] = fs16_twiddle(q1, n1);
    a[n1][2] = fs16_twiddle(q2, 2 * n1);
    a[n1][3] = fs16_twiddle(q3, 3 * n1);
  }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cpx<T> q0 = a[0][k1], q1 = a[1][k1], q2 = a[2][k1], q3 = a[3][k1];
    fs16_dft4(q0, q1, q2, q3);
    v[k1] = q0;
    v[k1 + 4] = q1;
    v[k1 + 8] = q2;
    v[k1 + 12] = q3;
  }
}

// Unscaled inverse 16-point DFT by the identity IDFT(v) = swap(DFT(swap(v))), where swap exchanges
// the real and imaginary parts.
template <typename T>
__device__ __forceinline__ void fs16_idft(cpx<T> (&v)[16]) {
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = cpx<T>{v[k].im, v[k].re};
  fs16_dft(v);
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = cpx<T>{v[k].im, v[k].re};
}

// The transpose between the two 16-point passes, through the group's 256-element LDS row S: lane t
// receives in v[q] what lane q held in v[t]. XOR-swizzled columns keep the 16 lanes of a write or
// read on distinct banks. Only groups with a row (ok) touch S; the wavefront syncs are uniform.
template <typename T>
__device__ __forceinline__ void fs16_transpose(cpx<T> (&v)[16], lptr<cpx<T>> S, int t, bool ok) {
  if (ok) {
#pragma unroll
    for (int s = 0; s < 16; ++s) lst<T>(S, s * 16 + (t ^ s), v[s]);
  }
  wave_sync();
  if (ok) {
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = lld<T>(S, t * 16 + (q ^ t));
  }
  wave_sync();
}

// Forward transform of one packed row held by a group in the 16 x 16 layout: in v[r] =
// x[t + 16 r], out v[u] = X[t + 16 u].
template <typename T>
__device__ __forceinline__ void fs16_forward(cpx<T> (&v)[16], lptr<const cpx<T>> tw,
                                             lptr<cpx<T>> S, int t, bool ok) {
  fs16_dft(v);
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = cmul(v[q], lld<T>(tw, (t * q) & 255));   // W_256^(t q)
  fs16_transpose(v, S, t, ok);
  fs16_dft(v);
}

// Unscaled inverse: in v[u] = X[t + 16 u], out v[r] = N x[t + 16 r].
template <typename T>
__device__ __forceinline__ void fs16_inverse(cpx<T> (&v)[16], lptr<const cpx<T>> tw,
                                             lptr<cpx<T>> S, int t, bool ok) {
  fs16_idft(v);
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const cpx<T> w = lld<T>(tw, (t * q) & 255);
    v[q] = cmul(v[q], cpx<T>{w.re, -w.im});
  }
  fs16_transpose(v, S, t, ok);
  fs16_idft(v);
}

// F^-1 (m_k F v) of one packed row in the 16 x 16 layout, with the multiplier applied as
// v[u] = sm(t + 16 u, v[u]) between the passes.
template <typename T, class SM>
__device__ __forceinline__ void fs16_spectral(cpx<T> (&v)[16], lptr<const cpx<T>> tw,
                                              lptr<cpx<T>> S, int t, bool ok, SM sm) {
  fs16_forward(v, tw, S, t, ok);
#pragma unroll
  for (int u = 0; u < 16; ++u) v[u] = sm(t + 16 * u, v[u]);
  fs16_inverse(v, tw, S, t, ok);
}

// Lane roles of the 16 x 16 row transforms of a workgroup: group t = lane & 15 of LDS slot
// (lane >> 4) nw + wavefront; the slots are bounded by the FFT buffer (2 fftb bytes).
template <typename T>
struct Fs16Lanes {
  int t, slot, nslots;
  lptr<cpx<T>> S;
  lptr<const cpx<T>> tw;
  __device__ __forceinline__ Fs16Lanes(int fftb) {
    const int nw = nthr() >> 6;
    t = tid() & 15;
    slot = ((tid() & 63) >> 4) * nw + (tid() >> 6);
    nslots = min(4 * nw, (2 * fft_cap<T>(fftb)) / 256);
    S = as_lds(fft_buf<T>() + min(slot, nslots - 1) * 256);
    tw = as_lds((const cpx<T>*)lds_tw<T>(fftb, 256));
  }
};

// Largest level the operator runs the 16 x 16 transforms on. The 33-row operators keep the
// radix-4 path: the calls of the transform in the 33-row solve kernel's body raised its register
// spills enough to slow its 64 x 33 solves by a quarter.
constexpr int kFs16MaxRows = 17;

// Whether the 16 x 16 row transforms apply: float64 rows of N = 256 and room for one slot.
template <typename T>
__device__ __forceinline__ bool fs16_fits(int N, int fftb) {
  return sizeof(T) == 8 && N == 256 && 2 * fft_cap<T>(fftb) >= N;
}

// spectral_rows by the 16 x 16 transform: each group reads its row pair from ld and writes it
// through st directly from registers. Ends with a barrier. Not inlined: the unrolled transforms
// at every call site would make the callers too long for short branches.
template <typename T, class LD, class SM, class ST>
__device__ __noinline__ void spectral_rows_fs(int nrows, int fftb, LD ld, SM sm, ST st) {
  const int npairs = (nrows + 1) >> 1;
  const Fs16Lanes<T> g(fftb);
  for (int base = 0; base < npairs; base += g.nslots) {
    const int pp = base + g.slot;
    const bool ok = g.slot < g.nslots && pp < npairs;
    const int ra = 2 * pp;
    cpx<T> v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int n = g.t + 16 * r;
      v[r] = {T(0), T(0)};
      if (ok) v[r] = {ld(ra, n), (ra + 1 < nrows) ? ld(ra + 1, n) : T(0)};
    }
    fs16_spectral(v, g.tw, g.S, g.t, ok, sm);
    if (ok) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        st(ra, g.t + 16 * r, v[r].re);
        if (ra + 1 < nrows) st(ra + 1, g.t + 16 * r, v[r].im);
      }
    }
  }
  __syncthreads();
}

// A real spectral operator along x on `nrows` real rows: F^-1 (m_k F f) (paper Sec. 3.5 for D_x,
// Sec. 3.6 for the filter). Two real rows are packed into one complex FFT; the multiplier must
// satisfy m_{-k} = conj(m_k) (a real operator) so that real and imaginary parts stay separate.
// ld(j, i) reads input row j at column i; sm(k, v) returns m_k v / N for the unscaled inverse FFT;
// st(j, i, v) writes the result. fftb: bytes of one half of the FFT LDS buffer. Ends with a
// barrier.
// FS = false keeps float64 rows of N = 256 on the radix-4 path (no call to the 16 x 16 transform
// in the caller).
template <typename T, bool FS = true, class LD, class SM, class ST>
__device__ void spectral_rows(int nrows, int N, int log2N, int fftb, LD ld, SM sm, ST st) {
  if constexpr (FS && sizeof(T) == 8) {
    if (fs16_fits<T>(N, fftb)) {
      spectral_rows_fs<T>(nrows, fftb, ld, sm, st);
      return;
    }
  }
  const int npairs = (nrows + 1) >> 1;
  const cpx<T>* tw = lds_tw<T>(fftb, N);
  if (fft_by_wave<T>(N, fftb)) {
    const int lane = tid() & 63, w = tid() >> 6, nw = nthr() >> 6;
    const int R = wave_rows<T>(N, fftb, npairs);
    cpx<T>* A = fft_buf<T>() + w * R * N;
    for (int base = 0; base < npairs; base += nw * R) {
      const int pp0 = base + w;
      const int nr = pp0 < npairs ? min(R, (npairs - pp0 + nw - 1) / nw) : 0;
      wave_load_pairs<T>(A, nr, N, lane, pp0, nw, nrows, ld);
      wave_sync();
      fft_wave_m<T, false, kWaveRows>(as_lds(A), nr, N, log2N, as_lds(tw), lane, N);
      for (int q = 0; q < nr; ++q)
        for (int n = lane; n < N; n += 64) A[q * N + n] = sm(n, A[q * N + n]);
      wave_sync();
      fft_wave_m<T, true, kWaveRows>(as_lds(A), nr, N, log2N, as_lds(tw), lane, N);
      wave_store_pairs<T>(A, nr, N, lane, pp0, nw, nrows, st);
      wave_sync();
    }
    __syncthreads();
    return;
  }
  const int cap = fft_cap<T>(fftb);
  cpx<T>* A0 = fft_buf<T>();
  cpx<T>* B0 = A0 + cap;
  const int rpb = cap >> log2N;
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
    for (int it = tid(); it < items; it += nthr()) R[it] = sm(it & (N - 1), R[it]);
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

// The spectral multiplier of D_x for an unscaled inverse FFT: i kappa_k / N, Nyquist entry zeroed.
template <typename T>
struct DxMul {
  int N;
  T kfac;
  __device__ __forceinline__ cpx<T> operator()(int n, cpx<T> v) const {
    const T scale = T(1) / T(N);
    const int kk = (n <= (N >> 1)) ? n : n - N;
    const T kap = (n == (N >> 1)) ? T(0) : kfac * T(kk) * scale;
    return cpx<T>{-kap * v.im, kap * v.re};
  }
};

// D_x of `nrows` real rows.
template <typename T, bool FS = true, class LD, class ST>
__device__ __forceinline__ void dx_rows(int nrows, int N, int log2N, T kfac, int fftb, LD ld,
                                        ST st) {
  spectral_rows<T, FS>(nrows, N, log2N, fftb, ld, DxMul<T>{N, kfac}, st);
}

// dx2_rows by the 16 x 16 transform (float64, N = 256): per row pair, p_x = D_x in from ld,
// stored through stx; g = mid(j, i, p_x) formed in registers (mid's global reads issued before
// the stores of p_x); D_x g stored through sto. Ends with a barrier. Not inlined (see
// spectral_rows_fs).
template <typename T, class SM, class LD, class STX, class MID, class STO>
__device__ __noinline__ void dx2_rows_fs(int nrows, int fftb, SM sm, LD ld, STX stx, MID mid,
                                         STO sto) {
  const int npairs = (nrows + 1) >> 1;
  const Fs16Lanes<T> g(fftb);
  for (int base = 0; base < npairs; base += g.nslots) {
    const int pp = base + g.slot;
    const bool ok = g.slot < g.nslots && pp < npairs;
    const int ra = 2 * pp;
    const bool two = ra + 1 < nrows;
    cpx<T> v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int n = g.t + 16 * r;
      v[r] = {T(0), T(0)};
      if (ok) v[r] = {ld(ra, n), two ? ld(ra + 1, n) : T(0)};
    }
    fs16_spectral(v, g.tw, g.S, g.t, ok, sm);
    if (ok) {
      cpx<T> gv[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int n = g.t + 16 * r;
        gv[r] = {mid(ra, n, v[r].re), two ? mid(ra + 1, n, v[r].im) : T(0)};
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int n = g.t + 16 * r;
        stx(ra, n, v[r].re);
        if (two) stx(ra + 1, n, v[r].im);
        v[r] = gv[r];
      }
    }
    fs16_spectral(v, g.tw, g.S, g.t, ok, sm);
    if (ok) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        sto(ra, g.t + 16 * r, v[r].re);
        if (two) sto(ra + 1, g.t + 16 * r, v[r].im);
      }
    }
  }
  __syncthreads();
}

// Between the two passes of dx2_rows: the wavefront's rows of p_x = D_x in (packed pairs in LDS)
// are stored through stx and replaced in LDS by g = mid(j, i, p_x). mid's global reads are issued
// before the stores (a load issued after a store waits for it).
template <typename T, class STX, class MID>
__device__ __forceinline__ void wave_mid_pairs(cpx<T>* A, int nr, int N, int lane, int pp0,
                                               int nw, int nrows, STX stx, MID mid) {
  cpx<T> v[kWaveRows][8], gv[kWaveRows][8];
#pragma unroll
  for (int q = 0; q < kWaveRows; ++q) {
    if (q < nr) {
#pragma unroll
      for (int it = 0; it < 8; ++it) {
        const int n = lane + 64 * it;
        if (n < N) v[q][it] = A[q * N + n];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kWaveRows; ++q) {
    if (q < nr) {
      const int ra = 2 * (pp0 + q * nw);
#pragma unroll
      for (int it = 0; it < 8; ++it) {
        const int n = lane + 64 * it;
        if (n < N)
          gv[q][it] = {mid(ra, n, v[q][it].re),
                       (ra + 1 < nrows) ? mid(ra + 1, n, v[q][it].im) : T(0)};
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kWaveRows; ++q) {
    if (q < nr) {
      const int ra = 2 * (pp0 + q * nw);
#pragma unroll
      for (int it = 0; it < 8; ++it) {
        const int n = lane + 64 * it;
        if (n < N) {
          stx(ra, n, v[q][it].re);
          if (ra + 1 < nrows) stx(ra + 1, n, v[q][it].im);
          A[q * N + n] = gv[q][it];
        }
      }
    }
  }
}

// Two chained D_x passes over the same rows (phases B and C of the operator): p_x = D_x in is
// stored through stx, then D_x g with g = mid(j, i, p_x) is stored through sto. On the wavefront
// path each wavefront keeps its rows in LDS from the first pass to the second, so the second pass
// needs no workgroup barrier and does not read p_x back; mid may read only fields completed
// before the call. Otherwise, and always for float64 rows (whose doubled register footprint in
// the fused form made the float64 solve slower), the two passes run one after the other, the
// second reading p_x back through ldx. Ends with a barrier.
//
// FS (float64 rows of N = 256): both passes by the 16 x 16 transform in one call, each group
// keeping its row pair in registers from the first pass to the second; as on the fused float32
// path, mid may then read only fields completed before the call. FS = false: the radix-4 path.
template <typename T, bool FS = true, class LD, class STX, class LDX, class MID, class STO>
__device__ void dx2_rows(int nrows, int N, int log2N, T kfac, int fftb, LD ld, STX stx, LDX ldx,
                         MID mid, STO sto) {
  const DxMul<T> sm{N, kfac};
  if constexpr (FS && sizeof(T) == 8) {
    if (fs16_fits<T>(N, fftb)) {
      dx2_rows_fs<T>(nrows, fftb, sm, ld, stx, mid, sto);
      return;
    }
  }
  if (sizeof(T) == 8 || !fft_by_wave<T>(N, fftb)) {
    spectral_rows<T, false>(nrows, N, log2N, fftb, ld, sm, stx);
    spectral_rows<T, false>(nrows, N, log2N, fftb,
                            [=](int j, int i) { return mid(j, i, ldx(j, i)); }, sm, sto);
    return;
  }
  if constexpr (sizeof(T) == 4) {
    const int npairs = (nrows + 1) >> 1;
    const cpx<T>* tw = lds_tw<T>(fftb, N);
    const int lane = tid() & 63, w = tid() >> 6, nw = nthr() >> 6;
    const int R = wave_rows<T>(N, fftb, npairs);
    cpx<T>* A = fft_buf<T>() + w * R * N;
    for (int base = 0; base < npairs; base += nw * R) {
      const int pp0 = base + w;
      const int nr = pp0 < npairs ? min(R, (npairs - pp0 + nw - 1) / nw) : 0;
      wave_load_pairs<T>(A, nr, N, lane, pp0, nw, nrows, ld);
      for (int pass = 0; pass < 2; ++pass) {
        wave_sync();
        fft_wave_m<T, false, kWaveRows>(as_lds(A), nr, N, log2N, as_lds(tw), lane, N);
        for (int q = 0; q < nr; ++q)
          for (int n = lane; n < N; n += 64) A[q * N + n] = sm(n, A[q * N + n]);
        wave_sync();
        fft_wave_m<T, true, kWaveRows>(as_lds(A), nr, N, log2N, as_lds(tw), lane, N);
        if (pass == 0) wave_mid_pairs<T>(A, nr, N, lane, pp0, nw, nrows, stx, mid);
      }
      wave_store_pairs<T>(A, nr, N, lane, pp0, nw, nrows, sto);
      wave_sync();
    }
    __syncthreads();
  }
}

// rows_fft_to_global by the 16 x 16 transform (float64, N = 256; not inlined, see
// spectral_rows_fs).
template <typename T, class LD>
__device__ __noinline__ void rows_fft_to_global_fs(int nrows, int fftb, LD ld,
                                                   gptr<cpx<T>> spec) {
  const int npairs = (nrows + 1) >> 1;
  const Fs16Lanes<T> g(fftb);
  for (int base = 0; base < npairs; base += g.nslots) {
    const int pp = base + g.slot;
    const bool ok = g.slot < g.nslots && pp < npairs;
    const int ra = 2 * pp;
    cpx<T> v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int n = g.t + 16 * r;
      v[r] = {T(0), T(0)};
      if (ok) v[r] = {ld(ra, n), (ra + 1 < nrows) ? ld(ra + 1, n) : T(0)};
    }
    fs16_forward(v, g.tw, g.S, g.t, ok);
    if (ok) {
#pragma unroll
      for (int u = 0; u < 16; ++u) gst<T>(spec, pp * 256 + g.t + 16 * u, v[u]);
    }
  }
  __syncthreads();
}

// rows_ifft_from_global by the 16 x 16 transform (float64, N = 256). For an Axpy target with add,
// every old value of x is loaded before the first store.
template <typename T, class ST>
__device__ __noinline__ void rows_ifft_from_global_fs(int nrows, int fftb,
                                                      gptr<const cpx<T>> spec, ST st) {
  const int npairs = (nrows + 1) >> 1;
  const Fs16Lanes<T> g(fftb);
  for (int base = 0; base < npairs; base += g.nslots) {
    const int pp = base + g.slot;
    const bool ok = g.slot < g.nslots && pp < npairs;
    const int ra = 2 * pp;
    const bool two = ra + 1 < nrows;
    cpx<T> v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      v[u] = {T(0), T(0)};
      if (ok) v[u] = gld<T>(spec, pp * 256 + g.t + 16 * u);
    }
    fs16_inverse(v, g.tw, g.S, g.t, ok);
    if (!ok) continue;
    if constexpr (std::is_same<ST, Axpy<T>>::value) {
      cpx<T> o[16];
      if (st.add) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int n = g.t + 16 * r;
          o[r] = {st.x[ra * st.nx + n], two ? st.x[(ra + 1) * st.nx + n] : T(0)};
        }
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int n = g.t + 16 * r;
        st.x[ra * st.nx + n] = st.add ? o[r].re + st.w * v[r].re : st.w * v[r].re;
        if (two) st.x[(ra + 1) * st.nx + n] = st.add ? o[r].im + st.w * v[r].im : st.w * v[r].im;
      }
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        st(ra, g.t + 16 * r, v[r].re);
        if (two) st(ra + 1, g.t + 16 * r, v[r].im);
      }
    }
  }
  __syncthreads();
}

// Forward FFT of real rows, packed in pairs, into spec[(nrows+1)/2][N] (global). Barrier at end.
template <typename T, bool FS = true, class LD>
__device__ void rows_fft_to_global(int nrows, int N, int log2N, int fftb, LD ld,
                                   gptr<cpx<T>> spec) {
  if constexpr (FS && sizeof(T) == 8) {
    if (fs16_fits<T>(N, fftb)) {
      rows_fft_to_global_fs<T>(nrows, fftb, ld, spec);
      return;
    }
  }
  const cpx<T>* tw = lds_tw<T>(fftb, N);
  const int npairs = (nrows + 1) >> 1;
  if (fft_by_wave<T>(N, fftb)) {
    const int lane = tid() & 63, w = tid() >> 6, nw = nthr() >> 6;
    const int R = wave_rows<T>(N, fftb, npairs);
    cpx<T>* A = fft_buf<T>() + w * R * N;
    for (int base = 0; base < npairs; base += nw * R) {
      const int pp0 = base + w;
      const int nr = pp0 < npairs ? min(R, (npairs - pp0 + nw - 1) / nw) : 0;
      wave_load_pairs<T>(A, nr, N, lane, pp0, nw, nrows, ld);
      wave_sync();
      fft_wave_m<T, false, kWaveRows>(as_lds(A), nr, N, log2N, as_lds(tw), lane, N);
      for (int q = 0; q < nr; ++q)
        for (int n = lane; n < N; n += 64) gst<T>(spec, (pp0 + q * nw) * N + n, A[q * N + n]);
      wave_sync();
    }
    __syncthreads();
    return;
  }
  const int cap = fft_cap<T>(fftb);
  cpx<T>* A0 = fft_buf<T>();
  cpx<T>* B0 = A0 + cap;
  const int rpb = cap >> log2N;
  for (int p0 = 0; p0 < npairs; p0 += rpb) {
    const int nb = min(rpb, npairs - p0);
    const int items = nb << log2N;
    for (int it = tid(); it < items; it += nthr()) {
      const int q = it >> log2N, n = it & (N - 1), ra = 2 * (p0 + q);
      A0[it] = {ld(ra, n), (ra + 1 < nrows) ? ld(ra + 1, n) : T(0)};
    }
    __syncthreads();
    cpx<T>* R = fft_lds<T, false>(A0, B0, nb, N, log2N, tw);
    for (int it = tid(); it < items; it += nthr()) gst<T>(spec, (p0 << log2N) + it, R[it]);
    __syncthreads();
  }
}

// Inverse FFT (unscaled) of packed spectra spec[(nrows+1)/2][N]; st(j, i, v) receives the real
// rows. Barrier at end.
template <typename T, bool FS = true, class ST>
__device__ void rows_ifft_from_global(int nrows, int N, int log2N, int fftb,
                                      gptr<const cpx<T>> spec, ST st) {
  if constexpr (FS && sizeof(T) == 8) {
    if (fs16_fits<T>(N, fftb)) {
      rows_ifft_from_global_fs<T>(nrows, fftb, spec, st);
      return;
    }
  }
  const cpx<T>* tw = lds_tw<T>(fftb, N);
  const int npairs = (nrows + 1) >> 1;
  if (fft_by_wave<T>(N, fftb)) {
    const int lane = tid() & 63, w = tid() >> 6, nw = nthr() >> 6;
    const int R = wave_rows<T>(N, fftb, npairs);
    cpx<T>* A = fft_buf<T>() + w * R * N;
    for (int base = 0; base < npairs; base += nw * R) {
      const int pp0 = base + w;
      const int nr = pp0 < npairs ? min(R, (npairs - pp0 + nw - 1) / nw) : 0;
      {
        cpx<T> v[kWaveRows][8];
#pragma unroll
        for (int q = 0; q < kWaveRows; ++q) {
          if (q < nr) {
#pragma unroll
            for (int it = 0; it < 8; ++it) {
              const int n = lane + 64 * it;
              if (n < N) v[q][it] = gld<T>(spec, (pp0 + q * nw) * N + n);
            }
          }
        }
#pragma unroll
        for (int q = 0; q < kWaveRows; ++q) {
          if (q < nr) {
#pragma unroll
            for (int it = 0; it < 8; ++it) {
              const int n = lane + 64 * it;
              if (n < N) A[q * N + n] = v[q][it];
            }
          }
        }
      }
      wave_sync();
      fft_wave_m<T, true, kWaveRows>(as_lds(A), nr, N, log2N, as_lds(tw), lane, N);
      if constexpr (std::is_same<ST, Axpy<T>>::value)
        wave_axpy_pairs<T>(A, nr, N, lane, pp0, nw, nrows, st);
      else
        wave_store_pairs<T>(A, nr, N, lane, pp0, nw, nrows, st);
      wave_sync();
    }
    __syncthreads();
    return;
  }
  const int cap = fft_cap<T>(fftb);
  cpx<T>* A0 = fft_buf<T>();
  cpx<T>* B0 = A0 + cap;
  const int rpb = cap >> log2N;
  for (int p0 = 0; p0 < npairs; p0 += rpb) {
    const int nb = min(rpb, npairs - p0);
    const int items = nb << log2N;
    for (int it = tid(); it < items; it += nthr()) A0[it] = gld<T>(spec, (p0 << log2N) + it);
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

// Whether a column phase holds its thread's whole column in registers, with the row loops fully
// unrolled, so that every vector load of the column is issued before its first store: a load
// issued after a store also waits for that store, because the vector-memory counter retires both
// in order, and a row loop that stores row j before loading row j + 1 pays one memory round trip
// per row. This is done for the float32 levels of up to 17 rows (the mixed-precision V-cycle).
// Unrolled float64 columns, whose operator the solve kernel inlines at several call sites, and
// 33-row columns would make the kernels too long for short branches; those keep row loops that
// step through the rows in chunks of kRowChunk.
template <typename T, int NZ>
constexpr bool kColInRegs = sizeof(T) == 4 && NZ <= 17;

// Rows per step of the row loops that are not unrolled: the loads of a chunk of rows are issued
// together before its stores, which cuts the round trips of a column phase by that factor (two
// for the float64 33-row columns, whose loads in flight would otherwise crowd the registers).
template <typename T, int NZ>
constexpr int kRowChunk = (sizeof(T) == 8 && NZ > 17) ? 2 : 4;

// One output pair p of the flat-mode solve at mode k (rows 2p and 2p + 1, packed as one complex
// value): ok is stored at k and okc at kc = N - k.
template <typename T, int NZ, bool TR>
__device__ __forceinline__ void mode_pair(gptr<const T> __restrict__ minv, int nh, int k, int p,
                                          const cpx<T> (&rh)[NZ], T scale, cpx<T>& ok,
                                          cpx<T>& okc) {
  cpx<T> s0 = {T(0), T(0)}, s1 = {T(0), T(0)};
  const int j0 = 2 * p, j1 = 2 * p + 1;
#pragma unroll
  for (int l = 0; l < NZ; ++l) {
    const T a = minv[(TR ? l * NZ + j0 : j0 * NZ + l) * nh + k];
    s0.re += a * rh[l].re;
    s0.im += a * rh[l].im;
    if (j1 < NZ) {
      const T c = minv[(TR ? l * NZ + j1 : j1 * NZ + l) * nh + k];
      s1.re += c * rh[l].re;
      s1.im += c * rh[l].im;
    }
  }
  s0.re *= scale; s0.im *= scale; s1.re *= scale; s1.im *= scale;
  ok = {s0.re - s1.im, s0.im + s1.re};
  okc = {s0.re + s1.im, s1.re - s0.im};
}

// Flat-mode line solve in Fourier space: for each mode k in [0, N/2], unpack the spectra of
// the nz real rows from the packed pairs, multiply by the inverse mode block (real, the same
// for k and N-k), repack, and fold in the 1/N of the inverse FFT. minv is [NZ][NZ][N/2+1].
// TR: use the transposed blocks (the transpose of the whole real map, because the block of
// mode k equals that of mode N-k).
template <typename T, int NZ, bool TR = false>
__device__ void mode_matvec(int N, gptr<const T> __restrict__ minv, gptr<cpx<T>> spec) {
  constexpr int NP = (NZ + 1) / 2;
  const int nh = (N >> 1) + 1;
  const T half = T(0.5), scale = T(1) / T(N);
  for (int k = tid(); k < nh; k += nthr()) {
    const int kc = (N - k) & (N - 1);
    const bool both = (k != 0 && k != (N >> 1));
    cpx<T> rh[NZ];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const cpx<T> z = gld<T>(spec, p * N + k), zc = gld<T>(spec, p * N + kc);
      rh[2 * p] = {half * (z.re + zc.re), half * (z.im - zc.im)};
      if (2 * p + 1 < NZ) rh[2 * p + 1] = {half * (z.im + zc.im), -half * (z.re - zc.re)};
    }
    if constexpr (kColInRegs<T, NZ>) {
      // all block reads before the first store (see kColInRegs)
      cpx<T> ok[NP], okc[NP];
#pragma unroll
      for (int p = 0; p < NP; ++p) mode_pair<T, NZ, TR>(minv, nh, k, p, rh, scale, ok[p], okc[p]);
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        gst<T>(spec, p * N + k, ok[p]);
        if (both) gst<T>(spec, p * N + kc, okc[p]);
      }
    } else {
#pragma unroll 1
      for (int p = 0; p < NP; ++p) {
        cpx<T> ok, okc;
        mode_pair<T, NZ, TR>(minv, nh, k, p, rh, scale, ok, okc);
        gst<T>(spec, p * N + k, ok);
        if (both) gst<T>(spec, p * N + kc, okc);
      }
    }
  }
}

// ----------------------------------------------------------------------------- geometry

template <typename T>
struct Geo {
  gptr<const T> ao, bo, ido, an, bn, idn, hx;   // sigma_x = a + b sigma; ido = 1/d
};

template <typename T>
struct Lev {
  int nz, nzc;
  gptr<const T> Ds, sig, colinv, modeinv, R, P;
  gptr<const T> PT, RT;          // P^T [nzc][nz] and R^T [nz][nzc] (transposed V-cycle)
  gptr<T> x, f, r, t1, t2, t3, u;
  gptr<cpx<T>> spec;
  gptr<const T> binv;            // bed-line inverse, transposed [nx][nx] (null when unused)
};

template <typename T>
struct Ctx {
  int nx, log2nx, fftb;
  T kfac;
  Geo<T> g;
  gptr<const double> cw, cwt;   // direct coarsest-level solve: W and W^T (null when not set up)
};

template <typename T>
__device__ __forceinline__ Ctx<T> uni(const Ctx<T>& c) {
  Ctx<T> u;
  u.nx = uni(c.nx); u.log2nx = uni(c.log2nx); u.fftb = uni(c.fftb); u.kfac = uni(c.kfac);
  u.g.ao = uni(c.g.ao); u.g.bo = uni(c.g.bo); u.g.ido = uni(c.g.ido); u.g.an = uni(c.g.an);
  u.g.bn = uni(c.g.bn); u.g.idn = uni(c.g.idn); u.g.hx = uni(c.g.hx);
  u.cw = uni(c.cw); u.cwt = uni(c.cwt);
  return u;
}

template <typename T>
__device__ __forceinline__ Lev<T> uni(const Lev<T>& L) {
  Lev<T> u;
  u.nz = uni(L.nz); u.nzc = uni(L.nzc);
  u.Ds = uni(L.Ds); u.sig = uni(L.sig); u.colinv = uni(L.colinv); u.modeinv = uni(L.modeinv);
  u.R = uni(L.R); u.P = uni(L.P); u.PT = uni(L.PT); u.RT = uni(L.RT);
  u.x = uni(L.x); u.f = uni(L.f); u.r = uni(L.r); u.t1 = uni(L.t1); u.t2 = uni(L.t2);
  u.t3 = uni(L.t3); u.u = uni(L.u); u.spec = uni(L.spec); u.binv = uni(L.binv);
  return u;
}

// ----------------------------------------------------------------------------- column phases

// out = D_sigma in, column by column.
template <typename T, int NZ>
__device__ void col_dsig(int nx, gptr<const T> Ds_, gptr<const T> in, gptr<T> out) {
  const cptr<T> Ds = as_const(Ds_);
  for (int i = tid(); i < nx; i += nthr()) {
    T v[NZ];
#pragma unroll
    for (int l = 0; l < NZ; ++l) v[l] = in[l * nx + i];
#pragma unroll 1
    for (int j = 0; j < NZ; ++j) {
      T s = T(0);
#pragma unroll
      for (int l = 0; l < NZ; ++l) s += Ds[j * NZ + l] * v[l];
      out[j * nx + i] = s;
    }
  }
}

// out = D_sigma in for column i only (the calling thread's own column).
template <typename T, int NZ>
__device__ __forceinline__ void col_dsig_one(int nx, cptr<T> Ds, gptr<const T> in, gptr<T> out,
                                             int i) {
  T v[NZ];
#pragma unroll
  for (int l = 0; l < NZ; ++l) v[l] = in[l * nx + i];
#pragma unroll 1
  for (int j = 0; j < NZ; ++j) {
    T s = T(0);
#pragma unroll
    for (int l = 0; l < NZ; ++l) s += Ds[j * NZ + l] * v[l];
    out[j * nx + i] = s;
  }
}

// out = D_sigma v for column i, from the column's values v in registers.
template <typename T, int NZ>
__device__ __forceinline__ void col_dsig_regs(int nx, cptr<T> Ds, const T (&v)[NZ], gptr<T> out,
                                              int i) {
#pragma unroll
  for (int j = 0; j < NZ; ++j) {
    T s = T(0);
#pragma unroll
    for (int l = 0; l < NZ; ++l) s += Ds[j * NZ + l] * v[l];
    out[j * nx + i] = s;
  }
}

// fc = R v for column i (restriction to NZC = (NZ+1)/2 rows), from the column v in registers.
template <typename T, int NZ>
__device__ __forceinline__ void col_restrict_regs(int nx, cptr<T> R, const T (&v)[NZ],
                                                  gptr<T> fc, int i) {
  constexpr int NZC = (NZ + 1) / 2;
#pragma unroll 1
  for (int j = 0; j < NZC; ++j) {
    T s = T(0);
#pragma unroll
    for (int l = 0; l < NZ; ++l) s += R[j * NZ + l] * v[l];
    fc[j * nx + i] = s;
  }
}

// FIN_FULL: the interior formula on every row (no boundary rows): Div Grad of a field, used for
// the viscous term of the momentum equations.
enum : int { FIN_APPLY = 0, FIN_RESID = 1, FIN_COLSTEP = 2, FIN_FULL = 3 };

// Last phase of the operator: A in = D_x G_x + sx_new D_s G_x + D_s G_z / d_new on interior
// rows, row 0 = in (Dirichlet), row M = -(h_x G_x + G_z) (bed), where per column
// G_x = P_x + sx_old P_s and G_z = P_s / d_old are rebuilt in registers from ps = D_s in and
// px = D_x in, and dxgx = D_x G_x. With sx_new = a_n + b_n sigma the interior rows are
//   D_x G_x + D_s (a_n G_x + G_z / d_n) + b_n sigma D_s G_x,
// both contractions taken in one pass over each row of D_s. FIN_APPLY writes A in to out;
// FIN_RESID writes f - A in; FIN_COLSTEP also applies x += omega B_i^-1 (f - A in)_i column by
// column (x may alias in) and, when t1w is non-null, stores D_s of the updated column there
// (the next operator application on x then skips its D_s phase).
template <typename T, int NZ>
__device__ __forceinline__ void col_finish(int mode, int nx, gptr<const T> Ds_,
                                           gptr<const T> sig_, const Geo<T>& g,
                                           gptr<const T> in, gptr<const T> ps,
                                           gptr<const T> px, gptr<const T> dxgx, gptr<T> out,
                                           gptr<const T> f, gptr<T> x,
                                           gptr<const T> __restrict__ cinv, T omega,
                                           gptr<T> t1w = gptr<T>(nullptr),
                                           gptr<const T> R_ = gptr<const T>(nullptr),
                                           gptr<T> fc = gptr<T>(nullptr)) {
  constexpr int NZC = (NZ + 1) / 2;
  const cptr<T> Ds = as_const(Ds_);
  const cptr<T> sig = as_const(sig_);
  const cptr<T> R = as_const(R_);
  const bool full = (mode == FIN_FULL);
  const bool apply = (mode == FIN_APPLY) || full;   // rows hold A in; otherwise f - A in
  for (int i = tid(); i < nx; i += nthr()) {
    const T ao = g.ao[i], bo = g.bo[i], ido = g.ido[i];
    const T an = g.an[i], bn = g.bn[i], idn = g.idn[i], hx = g.hx[i];
    T gx[NZ], u[NZ];
    T gzM = T(0);
#pragma unroll
    for (int l = 0; l < NZ; ++l) {
      const T a = ps[l * nx + i];
      gx[l] = px[l * nx + i] + (ao + bo * sig[l]) * a;
      const T gz = a * ido;
      u[l] = an * gx[l] + idn * gz;
      if (l == NZ - 1) gzM = gz;
    }
    // interior row j of A in, given D_x G_x at that row
    auto row = [&](int j, T dg) {
      T s1 = T(0), s2 = T(0);
#pragma unroll
      for (int l = 0; l < NZ; ++l) {
        const T d = Ds[j * NZ + l];
        s1 += d * u[l];
        s2 += d * gx[l];
      }
      return dg + s1 + bn * sig[j] * s2;
    };
    if constexpr (kColInRegs<T, NZ>) {
      T dg[NZ], fv[NZ], xv[NZ], res[NZ];
      const T top = full ? T(0) : in[i];
#pragma unroll
      for (int l = 0; l < NZ; ++l) dg[l] = dxgx[l * nx + i];
      if (!apply) {
#pragma unroll
        for (int l = 0; l < NZ; ++l) fv[l] = f[l * nx + i];
      }
      if (mode == FIN_COLSTEP) {
#pragma unroll
        for (int l = 0; l < NZ; ++l) xv[l] = x[l * nx + i];
      }
      if (!full) {
        const T bed = -(hx * gx[NZ - 1] + gzM);
        res[0] = apply ? top : fv[0] - top;
        res[NZ - 1] = apply ? bed : fv[NZ - 1] - bed;
      }
#pragma unroll
      for (int j = 0; j < NZ; ++j) {
        if (!full && (j == 0 || j == NZ - 1)) continue;
        const T o = row(j, dg[j]);
        res[j] = apply ? o : fv[j] - o;
      }
#pragma unroll
      for (int l = 0; l < NZ; ++l) out[l * nx + i] = res[l];
      if (fc) col_restrict_regs<T, NZ>(nx, R, res, fc, i);
      if (mode == FIN_COLSTEP) {
        T xn[NZ];
#pragma unroll
        for (int j = 0; j < NZ; ++j) {
          T s = T(0);
#pragma unroll
          for (int l = 0; l < NZ; ++l) s += cinv[(j * NZ + l) * nx + i] * res[l];
          xn[j] = xv[j] + omega * s;
        }
#pragma unroll
        for (int l = 0; l < NZ; ++l) x[l * nx + i] = xn[l];
        if (t1w) col_dsig_regs<T, NZ>(nx, Ds, xn, t1w, i);
      }
    } else {
      if (!full) {
        const T bed = -(hx * gx[NZ - 1] + gzM);
        const T top = in[i];
        if (mode == FIN_APPLY) {
          out[i] = top;
          out[(NZ - 1) * nx + i] = bed;
        } else {
          out[i] = f[i] - top;
          out[(NZ - 1) * nx + i] = f[(NZ - 1) * nx + i] - bed;
        }
      }
      constexpr int C = kRowChunk<T, NZ>;
      const int j0 = full ? 0 : 1, j1 = full ? NZ : NZ - 1;
#pragma unroll 1
      for (int j = j0; j < j1; j += C) {
        T dg[C], fv[C];
#pragma unroll
        for (int q = 0; q < C; ++q) {
          if (j + q < j1) {
            dg[q] = dxgx[(j + q) * nx + i];
            if (!apply) fv[q] = f[(j + q) * nx + i];
          }
        }
#pragma unroll
        for (int q = 0; q < C; ++q) {
          if (j + q < j1) {
            const T o = row(j + q, dg[q]);
            out[(j + q) * nx + i] = apply ? o : fv[q] - o;
          }
        }
      }
      if (mode == FIN_COLSTEP || fc) {
        T r[NZ];
#pragma unroll
        for (int l = 0; l < NZ; ++l) r[l] = out[l * nx + i];
        if (fc) col_restrict_regs<T, NZ>(nx, R, r, fc, i);
#pragma unroll 1
        for (int j = 0; j < NZ && mode == FIN_COLSTEP; j += C) {
          T s[C], xo[C];
#pragma unroll
          for (int q = 0; q < C; ++q) {
            s[q] = T(0);
            if (j + q < NZ) {
              xo[q] = x[(j + q) * nx + i];
#pragma unroll
              for (int l = 0; l < NZ; ++l) s[q] += cinv[((j + q) * NZ + l) * nx + i] * r[l];
            }
          }
#pragma unroll
          for (int q = 0; q < C; ++q)
            if (j + q < NZ) x[(j + q) * nx + i] = xo[q] + omega * s[q];
        }
        if (mode == FIN_COLSTEP && t1w) col_dsig_one<T, NZ>(nx, Ds, gptr<const T>(x), t1w, i);
      }
    }
  }
}

// x = omega B_i^-1 f_i (column step from a zero iterate: the residual is f); TR: B_i^-T. When
// t1w is non-null, also t1w = D_s x for the column.
template <typename T, int NZ, bool TR = false>
__device__ void col_solve_zero(int nx, gptr<const T> __restrict__ cinv, gptr<const T> f,
                               gptr<T> x, T omega, gptr<const T> Ds_ = gptr<const T>(nullptr),
                               gptr<T> t1w = gptr<T>(nullptr)) {
  const cptr<T> Ds = as_const(Ds_);
  for (int i = tid(); i < nx; i += nthr()) {
    T v[NZ];
#pragma unroll
    for (int l = 0; l < NZ; ++l) v[l] = f[l * nx + i];
    if constexpr (kColInRegs<T, NZ>) {
      T xn[NZ];
#pragma unroll
      for (int j = 0; j < NZ; ++j) {
        T s = T(0);
#pragma unroll
        for (int l = 0; l < NZ; ++l) s += cinv[(TR ? l * NZ + j : j * NZ + l) * nx + i] * v[l];
        xn[j] = omega * s;
      }
#pragma unroll
      for (int l = 0; l < NZ; ++l) x[l * nx + i] = xn[l];
      if (t1w) col_dsig_regs<T, NZ>(nx, Ds, xn, t1w, i);
    } else {
      constexpr int C = kRowChunk<T, NZ>;
#pragma unroll 1
      for (int j = 0; j < NZ; j += C) {
        T s[C];
#pragma unroll
        for (int q = 0; q < C; ++q) {
          s[q] = T(0);
          const int jq = j + q;
          if (jq < NZ) {
#pragma unroll
            for (int l = 0; l < NZ; ++l)
              s[q] += cinv[(TR ? l * NZ + jq : jq * NZ + l) * nx + i] * v[l];
          }
        }
#pragma unroll
        for (int q = 0; q < C; ++q)
          if (j + q < NZ) x[(j + q) * nx + i] = omega * s[q];
      }
      if (t1w) col_dsig_one<T, NZ>(nx, Ds, gptr<const T>(x), t1w, i);
    }
  }
}

// fc = R r (restriction to the next coarser order, NZC = (NZ+1)/2 rows).
template <typename T, int NZ>
__device__ void col_restrict(int nx, gptr<const T> R_, gptr<const T> r, gptr<T> fc) {
  constexpr int NZC = (NZ + 1) / 2;
  const cptr<T> R = as_const(R_);
  for (int i = tid(); i < nx; i += nthr()) {
    T v[NZ];
#pragma unroll
    for (int l = 0; l < NZ; ++l) v[l] = r[l * nx + i];
#pragma unroll 1
    for (int j = 0; j < NZC; ++j) {
      T s = T(0);
#pragma unroll
      for (int l = 0; l < NZ; ++l) s += R[j * NZ + l] * v[l];
      fc[j * nx + i] = s;
    }
  }
}

// x += P xc (prolongation from the next coarser order). When t1w is non-null, also
// t1w = D_s x for the corrected column (the next operator application then skips its D_s phase).
template <typename T, int NZ>
__device__ void col_prolong_add(int nx, gptr<const T> P_, gptr<const T> xc, gptr<T> x,
                                gptr<const T> Ds_ = gptr<const T>(nullptr),
                                gptr<T> t1w = gptr<T>(nullptr)) {
  constexpr int NZC = (NZ + 1) / 2;
  const cptr<T> P = as_const(P_);
  const cptr<T> Ds = as_const(Ds_);
  for (int i = tid(); i < nx; i += nthr()) {
    T v[NZC];
#pragma unroll
    for (int c = 0; c < NZC; ++c) v[c] = xc[c * nx + i];
    if constexpr (kColInRegs<T, NZ>) {
      T xv[NZ];
#pragma unroll
      for (int j = 0; j < NZ; ++j) xv[j] = x[j * nx + i];
      T xn[NZ];
#pragma unroll
      for (int j = 0; j < NZ; ++j) {
        T s = T(0);
#pragma unroll
        for (int c = 0; c < NZC; ++c) s += P[j * NZC + c] * v[c];
        xn[j] = xv[j] + s;
        x[j * nx + i] = xn[j];
      }
      if (t1w) col_dsig_regs<T, NZ>(nx, Ds, xn, t1w, i);
    } else {
      constexpr int C = kRowChunk<T, NZ>;
#pragma unroll 1
      for (int j = 0; j < NZ; j += C) {
        T s[C], xo[C];
#pragma unroll
        for (int q = 0; q < C; ++q) {
          s[q] = T(0);
          if (j + q < NZ) {
            xo[q] = x[(j + q) * nx + i];
#pragma unroll
            for (int c = 0; c < NZC; ++c) s[q] += P[(j + q) * NZC + c] * v[c];
          }
        }
#pragma unroll
        for (int q = 0; q < C; ++q)
          if (j + q < NZ) x[(j + q) * nx + i] = xo[q] + s[q];
      }
      if (t1w) col_dsig_one<T, NZ>(nx, Ds, gptr<const T>(x), t1w, i);
    }
  }
}

// ----------------------------------------------------------------------------- operator

// The composite operator on one level of NZ rows (paper eq. poissonp, eq. bcpd, eq. bcpdneu):
//   A: t1 = P_s = D_s in                                   (column phase)
//   B: t2 = P_x = D_x in                                   (row FFTs)
//   C: t3 = D_x G_x with G_x = P_x + sx_old P_s            (row FFTs, G_x formed in LDS)
//   D: finish (column phase, see col_finish; mode FIN_APPLY, FIN_RESID or FIN_COLSTEP)
// B and C run fused per wavefront (dx2_rows), so C reads P_x from LDS without a barrier; a
// barrier after A makes t1 complete first. t1_ready: t1 already holds D_s in (A is skipped).
// keep_t1: in FIN_COLSTEP, leave D_s of the updated x in t1.
// FS: float64 rows of N = 256 by the 16 x 16 transform (by default on levels of up to
// kFs16MaxRows rows).
template <typename T, int NZ, bool FS = (NZ <= kFs16MaxRows)>
__device__ __forceinline__ void op_apply(const Ctx<T>& c, const Lev<T>& L, int mode,
                                         gptr<const T> in, gptr<T> out, gptr<const T> f,
                                         gptr<T> x, T omega, bool t1_ready = false,
                                         bool keep_t1 = false, gptr<T> fc = gptr<T>(nullptr)) {
  constexpr bool kFs16 = FS;
  const int nx = c.nx;
  const gptr<T> t1 = L.t1;
  const gptr<T> t2 = L.t2;
  const gptr<T> t3 = L.t3;
  const gptr<const T> sig = L.sig;
  const Geo<T> g = c.g;
  if (!t1_ready) {
    col_dsig<T, NZ>(nx, L.Ds, in, t1);
    // the fused passes read t1 without a barrier of their own; the float64 radix-4 path runs B
    // and C apart, and B's closing barrier orders t1 for C
    if (sizeof(T) == 4 || (kFs16 && fs16_fits<T>(nx, c.fftb))) __syncthreads();
  }
  dx2_rows<T, kFs16>(
      NZ, nx, c.log2nx, c.kfac, c.fftb, [=](int j, int i) { return in[j * nx + i]; },
      [=](int j, int i, T v) { t2[j * nx + i] = v; }, [=](int j, int i) { return t2[j * nx + i]; },
      [=](int j, int i, T px) { return px + (g.ao[i] + g.bo[i] * sig[j]) * t1[j * nx + i]; },
      [=](int j, int i, T v) { t3[j * nx + i] = v; });
  col_finish<T, NZ>(mode, nx, L.Ds, sig, g, in, t1, t2, t3, out, f, x, L.colinv, omega,
                    keep_t1 ? t1 : gptr<T>(nullptr), L.R, fc);
  __syncthreads();
}

// ----------------------------------------------------------------------------- transpose
//
// A^T lam for the operator above. With Li = lam on the interior rows (0 on rows 0 and M):
//   Gbar_x = -D_x Li + D_s^T (sx_new Li) + e_M (-h_x lam_M)
//   Gbar_z =           D_s^T (Li / d_new) + e_M (-lam_M)
//   A^T lam = -D_x Gbar_x + D_s^T (sx_old Gbar_x + Gbar_z / d_old) + e_0 lam_0
// (D_x is antisymmetric). Phases:
//   A: t1 = D_s^T (sx_new Li) + bed part of Gbar_x,  t2 = Gbar_z      (column phase)
//   B: t3 = D_x Li                                                   (row FFTs, mask on load)
//   C: out = D_x Gbar_x with Gbar_x = t1 - t3 formed on load          (row FFTs)
//   D: finish (column phase): mode FIN_APPLY writes A^T in, FIN_RESID f - A^T in, FIN_COLSTEP
//      also applies x += omega B_i^-T (f - A^T in)_i (x may alias in; out must not).
template <typename T, int NZ>
__device__ void colT_start(int nx, gptr<const T> __restrict__ Ds, gptr<const T> __restrict__ sig,
                           const Geo<T>& g, gptr<const T> in, gptr<T> t1, gptr<T> t2) {
  for (int i = tid(); i < nx; i += nthr()) {
    const T an = g.an[i], bn = g.bn[i], idn = g.idn[i], hx = g.hx[i];
    T sl[NZ], il[NZ];
#pragma unroll
    for (int l = 0; l < NZ; ++l) {
      const T v = (l == 0 || l == NZ - 1) ? T(0) : in[l * nx + i];
      sl[l] = (an + bn * sig[l]) * v;
      il[l] = idn * v;
    }
    const T lamM = in[(NZ - 1) * nx + i];
#pragma unroll 1
    for (int j = 0; j < NZ; ++j) {
      T s1 = T(0), s2 = T(0);
#pragma unroll
      for (int l = 0; l < NZ; ++l) {
        const T d = Ds[l * NZ + j];
        s1 += d * sl[l];
        s2 += d * il[l];
      }
      if (j == NZ - 1) {
        s1 -= hx * lamM;
        s2 -= lamM;
      }
      t1[j * nx + i] = s1;
      t2[j * nx + i] = s2;
    }
  }
}

template <typename T, int NZ>
__device__ __forceinline__ void colT_finish(int mode, int nx, gptr<const T> __restrict__ Ds,
                                            gptr<const T> __restrict__ sig, const Geo<T>& g,
                                            gptr<const T> in, gptr<const T> t1,
                                            gptr<const T> t2, gptr<const T> t3, gptr<T> out,
                                            gptr<const T> f, gptr<T> x,
                                            gptr<const T> __restrict__ cinv, T omega) {
  for (int i = tid(); i < nx; i += nthr()) {
    const T ao = g.ao[i], bo = g.bo[i], ido = g.ido[i];
    T v[NZ], o[NZ];
#pragma unroll
    for (int l = 0; l < NZ; ++l) {
      const T gbx = t1[l * nx + i] - t3[l * nx + i];
      v[l] = (ao + bo * sig[l]) * gbx + ido * t2[l * nx + i];
      o[l] = -out[l * nx + i];
    }
    o[0] += in[i];
#pragma unroll 1
    for (int j = 0; j < NZ; ++j) {
      T s = o[j];
#pragma unroll
      for (int l = 0; l < NZ; ++l) s += Ds[l * NZ + j] * v[l];
      o[j] = (mode == FIN_APPLY) ? s : f[j * nx + i] - s;
    }
#pragma unroll
    for (int l = 0; l < NZ; ++l) out[l * nx + i] = o[l];
    if (mode == FIN_COLSTEP) {
#pragma unroll 1
      for (int j = 0; j < NZ; ++j) {
        T s = T(0);
#pragma unroll
        for (int l = 0; l < NZ; ++l) s += cinv[(l * NZ + j) * nx + i] * o[l];
        x[j * nx + i] += omega * s;
      }
    }
  }
}

template <typename T, int NZ>
__device__ __forceinline__ void op_apply_T(const Ctx<T>& c, const Lev<T>& L, int mode,
                                           gptr<const T> in, gptr<T> out, gptr<const T> f,
                                           gptr<T> x, T omega) {
  const int nx = c.nx;
  const gptr<T> t1 = L.t1;
  const gptr<T> t2 = L.t2;
  const gptr<T> t3 = L.t3;
  const Geo<T> g = c.g;
  colT_start<T, NZ>(nx, L.Ds, L.sig, g, in, t1, t2);
  // no barrier: the next phase reads only `in`; t1 and t2 are read after its closing barrier
  constexpr bool kFs16 = NZ <= kFs16MaxRows;
  dx_rows<T, kFs16>(NZ, nx, c.log2nx, c.kfac, c.fftb,
                    [=](int j, int i) { return (j == 0 || j == NZ - 1) ? T(0) : in[j * nx + i]; },
                    [=](int j, int i, T v) { t3[j * nx + i] = v; });
  dx_rows<T, kFs16>(NZ, nx, c.log2nx, c.kfac, c.fftb,
             [=](int j, int i) { return t1[j * nx + i] - t3[j * nx + i]; },
             [=](int j, int i, T v) { out[j * nx + i] = v; });
  colT_finish<T, NZ>(mode, nx, L.Ds, L.sig, g, in, t1, t2, t3, out, f, x, L.colinv, omega);
  __syncthreads();
}

// Applies A (TR = false) or A^T (TR = true).
template <typename T, int NZ, bool TR>
__device__ __forceinline__ void op_any(const Ctx<T>& c, const Lev<T>& L, int mode,
                                       gptr<const T> in, gptr<T> out, gptr<const T> f,
                                       gptr<T> x, T omega, bool t1_ready = false,
                                       bool keep_t1 = false, gptr<T> fc = gptr<T>(nullptr)) {
  if constexpr (TR) op_apply_T<T, NZ>(c, L, mode, in, out, f, x, omega);
  else op_apply<T, NZ>(c, L, mode, in, out, f, x, omega, t1_ready, keep_t1, fc);
}

template <typename P>
__device__ __forceinline__ void fill_zero(P p, int n) {
  for (int e = tid(); e < n; e += nthr()) p[e] = 0;
}

// Direct solve of the coarsest level (order 2, three rows) from its stored inverse, in float64
// whatever T: x_0 = f_0 and [x_1; x_2] = W [f_0; f_1; f_2], W = [Q | B^-1] (2 nx x 3 nx, see
// k_coarse_setup), read through wt = W^T [3 nx][2 nx] so that the rows of W are read coalesced.
// TR: the transpose of that linear map, x_0 = f_0 + Q^T [f_1; f_2], [x_1; x_2] = B^-T [f_1; f_2],
// read through w = W [2 nx][3 nx]. f is staged as float64 in fin (LDS, 24 nx bytes; by default
// the FFT buffer). f and x may be global or LDS fields.
template <typename T, bool TR, class PF, class PX, class PS>
__device__ void coarse_direct(int nx, gptr<const double> w, gptr<const double> wt, PF f, PX x,
                              PS fin) {
  const int n2 = 2 * nx, n3 = 3 * nx;
  for (int e = tid(); e < n3; e += nthr()) fin[e] = (double)f[e];
  __syncthreads();
  constexpr int U = 8;   // loads in flight per thread (n3 and n2 are multiples of 8)
  if constexpr (!TR) {
    for (int r = tid(); r < n2; r += nthr()) {
      double acc[U];
#pragma unroll
      for (int q = 0; q < U; ++q) acc[q] = 0.0;
      for (int c = 0; c < n3; c += U) {
        double a[U];
#pragma unroll
        for (int q = 0; q < U; ++q) a[q] = wt[(int64_t)(c + q) * n2 + r];
#pragma unroll
        for (int q = 0; q < U; ++q) acc[q] += a[q] * fin[c + q];
      }
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < U; ++q) s += acc[q];
      x[nx + r] = (T)s;
    }
    for (int i = tid(); i < nx; i += nthr()) x[i] = (T)fin[i];
  } else {
    for (int c = tid(); c < n3; c += nthr()) {
      double acc[U];
#pragma unroll
      for (int q = 0; q < U; ++q) acc[q] = 0.0;
      for (int r = 0; r < n2; r += U) {
        double a[U];
#pragma unroll
        for (int q = 0; q < U; ++q) a[q] = w[(int64_t)(r + q) * n3 + c];
#pragma unroll
        for (int q = 0; q < U; ++q) acc[q] += a[q] * fin[nx + r + q];
      }
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < U; ++q) s += acc[q];
      x[c] = (T)((c < nx ? fin[c] : 0.0) + s);
    }
  }
  __syncthreads();
}

// Bed-line step of a forward smoothing pair (option bed_line): the bed row solved exactly with
// the other rows held, x_M <- L_b^-1 (f_M + q s), s = sum_{l<M} (D_sigma)_Ml x_l,
// q = h_x sigma_x^old[M] + 1/d_old (the bed row of A x with the bed unknowns moved to the left
// side). g = f_M + q s is staged in LDS; L.binv holds L_b^-1 transposed, read coalesced.
template <typename T, int NZ>
__device__ void bed_step(const Ctx<T>& c, const Lev<T>& L) {
  constexpr int M = NZ - 1;
  const int nx = c.nx;
  T* g = reinterpret_cast<T*>(fft_buf<T>());
  const T sgm = L.sig[M];
  for (int i = tid(); i < nx; i += nthr()) {
    T s = T(0);
#pragma unroll
    for (int l = 0; l < M; ++l) s += L.Ds[M * NZ + l] * L.x[l * nx + i];
    const T q = c.g.hx[i] * (c.g.ao[i] + c.g.bo[i] * sgm) + c.g.ido[i];
    g[i] = L.f[M * nx + i] + q * s;
  }
  __syncthreads();
  for (int i = tid(); i < nx; i += nthr()) {
    T acc = T(0);
    for (int k = 0; k < nx; ++k) acc += L.binv[(int64_t)k * nx + i] * g[k];
    L.x[M * nx + i] = acc;
  }
  __syncthreads();
}

// The transposed cycle's bed-line step (before its mode step): x_M += L_b^-T (f - A^T x)_M,
// from x = 0 when xzero (then x is zero-filled first).
template <typename T, int NZ>
__device__ void bed_step_T(const Ctx<T>& c, const Lev<T>& L, bool xzero) {
  constexpr int M = NZ - 1;
  const int nx = c.nx;
  gptr<const T> r = gptr<const T>(L.f);
  if (xzero) {
    for (int e = tid(); e < NZ * nx; e += nthr()) L.x[e] = T(0);
    __syncthreads();
  } else {
    op_any<T, NZ, true>(c, L, FIN_RESID, gptr<const T>(L.x), L.r, gptr<const T>(L.f),
                        gptr<T>(nullptr), T(0), false, false, gptr<T>(nullptr));
    r = gptr<const T>(L.r);
  }
  T* g = reinterpret_cast<T*>(fft_buf<T>());
  for (int i = tid(); i < nx; i += nthr()) g[i] = r[M * nx + i];
  __syncthreads();
  for (int i = tid(); i < nx; i += nthr()) {
    T acc = T(0);
    for (int k = 0; k < nx; ++k) acc += L.binv[(int64_t)i * nx + k] * g[k];
    L.x[M * nx + i] += acc;
  }
  __syncthreads();
}

// The V-cycle (paper Alg. 1) from a zero guess on the levels l, l+1, ..., whose row counts are
// NZ, (NZ+1)/2, ..., 3 (the order halves per level). lev(l) returns the Lev of level l; input
// lev(l).f, output lev(l).x.
//
// One level runs a list of steps, each an operator application followed by an action:
//   COL   column-block step   x += omega_c B^-1 (f - A x)        (from x = 0: x = omega_c B^-1 f)
//   MODE  flat-mode step      x += omega_m F^-1 Ahat^-1 F (f - A x)
//   DOWN  residual, restriction, the coarser V-cycle (a call), prolongation and correction
// in the order nu1 x (COL, MODE), DOWN, nu2 x (COL, MODE); the coarsest level (3 rows) runs
// coarse_pairs x (COL, MODE). The operator appears once in the loop body, which keeps each
// level's code compact. In the forward cycle the residual phase before DOWN also restricts each
// column it finishes, and the prolongation also leaves D_s x in t1, so neither runs as a phase of
// its own behind a barrier.
//
// TR = true gives the transpose M^T of the cycle's linear map M (the preconditioner of the
// adjoint solve): the same cycle on A^T with every step's order reversed (nu2 x (MODE, COL),
// DOWN, nu1 x (MODE, COL)), transposed block inverses, restriction by P^T and prolongation by
// R^T. (Reverse-mode differentiation of the cycle gives exactly this sequence.)
template <typename T, int NZ, class LP, bool TR = false>
__device__ __noinline__ void vcycle(Ctx<T> c_, LP lev_, int l_, KOpts o_) {
  const Ctx<T> c = uni(c_);
  const LP lev = uni(lev_);
  const int l = uni(l_);
  KOpts o;
  o.nu1 = uni(o_.nu1); o.nu2 = uni(o_.nu2); o.coarse_pairs = uni(o_.coarse_pairs);
  o.restart = uni(o_.restart); o.omega_c = uni(o_.omega_c); o.omega_m = uni(o_.omega_m);
  o.adapt = uni(o_.adapt); o.cycle = uni(o_.cycle); o.coarse_exact = uni(o_.coarse_exact);
  o.bed_line = uni(o_.bed_line);
  const int nx = c.nx;
  const T wc = T(o.omega_c), wm = T(o.omega_m);
  const Lev<T> L = uni(lev(l));
  if constexpr (NZ == 3) {
    if (uni(o_.coarse_exact) && c.cw) {
      coarse_direct<T, TR>(nx, c.cw, c.cwt, gptr<const T>(L.f), L.x,
                           as_lds(reinterpret_cast<double*>(g_fft_lds)));
      return;
    }
  }
  enum { COL = 0, MODE = 1, DOWN = 2 };
  const int first = TR ? MODE : COL, second = TR ? COL : MODE;
  const int npre = (NZ == 3) ? o.coarse_pairs : (TR ? o.nu2 : o.nu1);
  const int npost = (NZ == 3) ? 0 : (TR ? o.nu1 : o.nu2);
  const int nops = 2 * npre + ((NZ == 3) ? 0 : 1) + 2 * npost;
  bool xzero = true;
  bool t1x = false;   // forward cycle: t1 holds D_s x (set by column steps)
  for (int q = 0; q < nops; ++q) {
    int kind;
    if (q < 2 * npre) kind = (q & 1) ? second : first;
    else if (NZ != 3 && q == 2 * npre) kind = DOWN;
    else kind = ((q - 2 * npre - 1) & 1) ? second : first;
    // before a level move of the forward cycle the residual phase also restricts its columns
    gptr<T> fc(nullptr);
    if constexpr (NZ > 3 && !TR) {
      if (kind == DOWN) fc = uni(lev(l + 1)).f;
    }
    // the transposed pair starts with the transposed bed-line step
    if (TR && o.bed_line && L.binv && kind == MODE) {
      bed_step_T<T, NZ>(c, L, xzero);
      xzero = false;
    }
    if (!xzero)
      op_any<T, NZ, TR>(c, L, kind == COL ? FIN_COLSTEP : FIN_RESID, L.x, L.r, L.f, L.x, wc,
                        !TR && t1x, !TR && kind == COL, fc);
    const bool restricted = !xzero && fc;
    t1x = !TR && kind == COL;
    if (kind == COL) {
      if (xzero) {
        col_solve_zero<T, NZ, TR>(nx, L.colinv, L.f, L.x, wc, L.Ds,
                                  TR ? gptr<T>(nullptr) : L.t1);
        __syncthreads();
        xzero = false;
      }
    } else if (kind == MODE) {
      const gptr<const T> r = xzero ? gptr<const T>(L.f) : gptr<const T>(L.r);
      rows_fft_to_global<T, (NZ <= kFs16MaxRows)>(NZ, nx, c.log2nx, c.fftb,
                            [=](int j, int i) { return r[j * nx + i]; }, L.spec);
      mode_matvec<T, NZ, TR>(nx, L.modeinv, L.spec);
      __syncthreads();
      rows_ifft_from_global<T, (NZ <= kFs16MaxRows)>(NZ, nx, c.log2nx, c.fftb, L.spec,
                                                     Axpy<T>{L.x, nx, wm, !xzero});
      xzero = false;
      // the forward pair ends with the bed-line step
      if (!TR && o.bed_line && L.binv) bed_step<T, NZ>(c, L);
    } else {
      if constexpr (NZ > 3) {
        constexpr int NZC = (NZ + 1) / 2;
        const Lev<T> C = uni(lev(l + 1));
        if (xzero) fill_zero(L.x, NZ * nx);
        if (!restricted) {
          col_restrict<T, NZ>(nx, TR ? L.PT : L.R,
                              xzero ? gptr<const T>(L.f) : gptr<const T>(L.r), C.f);
          __syncthreads();
        }
        vcycle<T, NZC, LP, TR>(c, lev, l + 1, o);
        // forward cycle: the correction also leaves D_s x in t1 for the next step's operator
        col_prolong_add<T, NZ>(nx, TR ? L.RT : L.P, C.x, L.x, TR ? gptr<const T>(nullptr) : L.Ds,
                               TR ? gptr<T>(nullptr) : L.t1);
        __syncthreads();
        t1x = !TR;
        xzero = false;
      }
    }
  }
  if (xzero) {
    fill_zero(L.x, NZ * nx);
    __syncthreads();
  }
}

// Full multigrid (paper Alg. 2) on the levels l, l+1, ...: input lev(l).f, output lev(l).x.
// The right-hand side is restricted to the next level and solved there by full multigrid; its
// result, prolongated, is the initial guess u of this level's V-cycle, evaluated as
// u + V_0(f - A u) with the V-cycle from zero (the same linear map: every smoothing and
// correction step commutes with shifting the iterate by u). lev(l).f is overwritten by the
// residual and lev(l).u holds u. On the coarsest level (3 rows) it is the coarse V-cycle.
template <typename T, int NZ, class LP>
__device__ __noinline__ void fmg(Ctx<T> c_, LP lev_, int l_, KOpts o_) {
  const Ctx<T> c = uni(c_);
  const LP lev = uni(lev_);
  const int l = uni(l_);
  KOpts o;
  o.nu1 = uni(o_.nu1); o.nu2 = uni(o_.nu2); o.coarse_pairs = uni(o_.coarse_pairs);
  o.restart = uni(o_.restart); o.omega_c = uni(o_.omega_c); o.omega_m = uni(o_.omega_m);
  o.adapt = uni(o_.adapt); o.cycle = uni(o_.cycle); o.coarse_exact = uni(o_.coarse_exact);
  o.bed_line = uni(o_.bed_line);
  if constexpr (NZ == 3) {
    vcycle<T, NZ, LP, false>(c, lev, l, o);
  } else {
    constexpr int NZC = (NZ + 1) / 2;
    const int nx = c.nx;
    const Lev<T> L = uni(lev(l));
    const Lev<T> C = uni(lev(l + 1));
    col_restrict<T, NZ>(nx, L.R, gptr<const T>(L.f), C.f);
    __syncthreads();
    fmg<T, NZC>(c, lev, l + 1, o);
    fill_zero(L.u, NZ * nx);
    __syncthreads();
    col_prolong_add<T, NZ>(nx, L.P, gptr<const T>(C.x), L.u);
    __syncthreads();
    op_apply<T, NZ>(c, L, FIN_RESID, gptr<const T>(L.u), L.f, gptr<const T>(L.f), gptr<T>(nullptr),
                    T(0));
    vcycle<T, NZ, LP, false>(c, lev, l, o);
    const gptr<T> x = L.x;
    const gptr<const T> u = L.u;
    for (int e = tid(); e < NZ * nx; e += nthr()) x[e] += u[e];
    __syncthreads();
  }
}

}  // namespace pmgw

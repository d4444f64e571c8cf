// LDS-resident float32 V-cycle of the mixed-precision solve (paper Alg. 1 with the smoother,
// transfers and coarsest level of the global-memory cycle in pmgw_device.hpp, same arithmetic).
//
// The global-memory cycle keeps its level vectors in L2 and pays an L2 round trip in every
// barrier-separated phase (about 75 phases per cycle at 256 x 17). Here every level's iterate x
// and right-hand side f, the operator temporaries and the float32 metrics stay in the workgroup's
// LDS for the whole cycle, so a phase costs an LDS round trip instead. Only the block inverses,
// the level tables and (with the direct coarse solve) its inverse are read from global memory.
//
// LDS map (floats from the start of the dynamic LDS, nx = the tank's Nx, NZ0 = finest rows):
//   geo  7 nx          ao, bo, ido, an, bn, idn, hx (sigma_x = a + b sigma; 1/d), old and new
//   t1   NZ0 nx        D_s x (plain rows [j][i])
//   t2   (NZ0 + 1) nx  G_x, rows packed in pairs: element (j, i) at ((j+1)/2) 2 nx + 2 i + ((j+1) & 1)
//   t3   (NZ0 + 1) nx  packed pairs: the operator's FFT rows, D_x G_x, the residual, its spectra
//   x_l, f_l           rows_l nx each, plain, for every level l (rows NZ0, (NZ0+1)/2, ..., 3)
//   tables             per level D_sigma, sigma, R, P (float32), after the fields
// A packed pair of rows is exactly the complex row (re = row 2p - 1, im = row 2p) that the x-FFT
// transforms, so every FFT runs in place in t3 with no staging buffer; the column phases read
// packed rows two at a time. Row 0 shares its complex row with a zero pad (row -1): a float32
// FFT leaks about eps times the larger row of a pair into the smaller, and the Dirichlet row's
// residual is near zero while row 1's can be a thousand times the iterate. The map is used for NZ0 <= 17 and 64 <= Nx <= 512 where it fits in
// LDS next to the twiddles and the Krylov state (256 x 17: 131 KB).
#pragma once
#include "pmgw_device.hpp"

namespace pmgw {

// rows of level l below a finest level of nz0 rows
__host__ __device__ constexpr int res_rows(int nz0, int l) {
  int r = nz0;
  for (int i = 0; i < l; ++i) r = (r + 1) / 2;
  return r;
}
__host__ __device__ constexpr int res_level(int nz0, int nz) {
  int l = 0, r = nz0;
  while (r > nz) { r = (r + 1) / 2; ++l; }
  return l;
}
__host__ __device__ constexpr int res_rows_before(int nz0, int l) {
  int s = 0;
  for (int i = 0; i < l; ++i) s += res_rows(nz0, i);
  return s;
}
__host__ __device__ constexpr int res_rows_total(int nz0) {
  int s = 0, r = nz0;
  while (true) {
    s += r;
    if (r <= 3) break;
    r = (r + 1) / 2;
  }
  return s;
}
// floats of the map per x column
__host__ __device__ constexpr int res_floats_per_col(int nz0) {
  return 7 + nz0 + 2 * (nz0 + 1) + 2 * res_rows_total(nz0);
}
// floats of the level tables of level l (D_sigma, sigma, R, P), kept in LDS after the map
__host__ __device__ constexpr int res_tab_level(int nz0, int l) {
  const int r = res_rows(nz0, l);
  const int rc = r > 3 ? (r + 1) / 2 : 0;
  return r * r + r + 2 * r * rc;
}
__host__ __device__ constexpr int res_tab_before(int nz0, int l) {
  int s = 0;
  for (int i = 0; i < l; ++i) s += res_tab_level(nz0, i);
  return s;
}
__host__ __device__ constexpr int res_tab_floats(int nz0) {
  int s = 0, l = 0;
  while (true) {
    s += res_tab_level(nz0, l);
    if (res_rows(nz0, l) <= 3) break;
    ++l;
  }
  return s;
}
// bytes of the whole map (fields of a tank with nx columns, then the tables)
__host__ __device__ constexpr long long res_map_bytes(int nz0, int nx) {
  return 4LL * ((long long)res_floats_per_col(nz0) * nx + res_tab_floats(nz0));
}
constexpr int kResMaxNz = 17;

typedef float vf2 __attribute__((ext_vector_type(2)));

// uni() for LDS pointers (32-bit addresses).
template <typename T>
__device__ __forceinline__ lptr<T> uni(lptr<T> p) {
  const unsigned a = (unsigned)(unsigned long long)p;
  return (lptr<T>)(unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)a);
}

struct RMap {
  lptr<float> geo, t1, t2, t3, x, f, xc, fc;
  lptr<float> tab;   // the level's tables: D_sigma [NZ][NZ], sigma [NZ], R [NZC][NZ], P [NZ][NZC]
};

template <int NZ0, int NZ>
__device__ __forceinline__ RMap res_map(int nx) {
  const lptr<float> b = (lptr<float>)(reinterpret_cast<float*>(g_fft_lds));
  constexpr int l = res_level(NZ0, NZ);
  RMap m;
  m.geo = b;
  m.t1 = b + 7 * nx;
  m.t2 = b + (7 + NZ0) * nx;
  m.t3 = b + (8 + 2 * NZ0) * nx;
  m.x = b + (9 + 3 * NZ0) * nx + 2 * res_rows_before(NZ0, l) * nx;
  m.f = m.x + NZ * nx;
  m.xc = m.f + NZ * nx;               // the next coarser level follows directly
  m.fc = m.xc + ((NZ + 1) / 2) * nx;
  m.tab = b + res_floats_per_col(NZ0) * nx + res_tab_before(NZ0, l);
  return m;
}

// Uniform parameters of the resident cycle.
struct RCtx {
  int nx, log2nx, fftb;
  float kfac, wc, wm;
  int nu1, nu2, coarse_pairs, coarse_exact;
  const TankDesc* td;
  char* ws;
  gptr<const double> cw, cwt;
};

__device__ __forceinline__ RCtx uni(const RCtx& c) {
  RCtx u;
  u.nx = uni(c.nx); u.log2nx = uni(c.log2nx); u.fftb = uni(c.fftb);
  u.kfac = uni(c.kfac); u.wc = uni(c.wc); u.wm = uni(c.wm);
  u.nu1 = uni(c.nu1); u.nu2 = uni(c.nu2); u.coarse_pairs = uni(c.coarse_pairs);
  u.coarse_exact = uni(c.coarse_exact);
  u.td = uni(c.td); u.ws = uni(c.ws); u.cw = uni(c.cw); u.cwt = uni(c.cwt);
  return u;
}

// Level tables (float32) of level l: the small matrices in LDS (read at uniform addresses, which
// LDS broadcasts; scalar loads would share the LDS wait counter and, completing out of order,
// force a wait for every outstanding LDS access at each use), the block inverses in global memory.
struct RLev {
  lptr<const float> Ds, sig, R, P;
  gptr<const float> colinv, modeinv;
};

template <int NZ>
__device__ __forceinline__ RLev res_lev(const RCtx& c, const RMap& m, int l) {
  constexpr int NZC = NZ > 3 ? (NZ + 1) / 2 : 0;
  const LevelDesc& d = c.td->lev[l];
  RLev L;
  L.Ds = m.tab;
  L.sig = m.tab + NZ * NZ;
  L.R = m.tab + NZ * NZ + NZ;
  L.P = m.tab + NZ * NZ + NZ + NZC * NZ;
  L.colinv = (gptr<const float>)(c.ws + d.colinv);
  L.modeinv = (gptr<const float>)(c.ws + d.modeinv);
  return L;
}

// Rows 2 pr - 1 and 2 pr of a packed field at column i (row -1 is the zero pad).
__device__ __forceinline__ vf2 pk_ld(lptr<float> p, int nx, int pr, int i) {
  return *(lptr<vf2>)(p + pr * 2 * nx + 2 * i);
}
__device__ __forceinline__ void pk_st(lptr<float> p, int nx, int pr, int i, vf2 v) {
  *(lptr<vf2>)(p + pr * 2 * nx + 2 * i) = v;
}

// Reads rows 0..NZ-1 of column i of a packed field into v.
template <int NZ>
__device__ __forceinline__ void pk_col(lptr<float> p, int nx, int i, float (&v)[NZ]) {
#pragma unroll
  for (int pr = 0; pr < (NZ + 1) / 2; ++pr) {
    const vf2 a = pk_ld(p, nx, pr, i);
    if (pr > 0) v[2 * pr - 1] = a.x;
    v[2 * pr] = a.y;
  }
}

// out[j] = D_s v at row j for a column in registers.
template <int NZ>
__device__ __forceinline__ void r_dsig_col(lptr<const float> Ds, const float (&v)[NZ], lptr<float> t1,
                                           int nx, int i) {
#pragma unroll
  for (int j = 0; j < NZ; ++j) {
    float s = 0.f;
#pragma unroll
    for (int l = 0; l < NZ; ++l) s += Ds[j * NZ + l] * v[l];
    t1[j * nx + i] = s;
  }
}

// t1 = D_s x.
template <int NZ>
__device__ void r_dsig(int nx, lptr<const float> Ds, lptr<float> x, lptr<float> t1) {
  for (int i = tid(); i < nx; i += nthr()) {
    float v[NZ];
#pragma unroll
    for (int l = 0; l < NZ; ++l) v[l] = x[l * nx + i];
    r_dsig_col<NZ>(Ds, v, t1, nx, i);
  }
  __syncthreads();
}

// Rows of a block-inverse product per step: the NZ x kBlkRows block entries of a step are loaded
// together (enough loads in flight to cover the global latency, few enough registers for a
// non-inlined level function, which has 256).
constexpr int kBlkRows = 6;

// x[j] = a x[j] + w (B_i^-1 v)_j for the column i (a = 0: x = w B_i^-1 v), kBlkRows rows at a
// time; x is the LDS field (row stride nx).
template <int NZ>
__device__ __forceinline__ void r_blk_apply(gptr<const float> cinv, int nx, int i,
                                            const float (&v)[NZ], lptr<float> x, float a,
                                            float w) {
#pragma unroll 1
  for (int j = 0; j < NZ; j += kBlkRows) {
    float s[kBlkRows], blk[kBlkRows][NZ];
#pragma unroll
    for (int q = 0; q < kBlkRows; ++q)
#pragma unroll
      for (int l = 0; l < NZ; ++l)
        blk[q][l] = (j + q < NZ) ? cinv[((j + q) * NZ + l) * nx + i] : 0.f;
    // every load of the step is issued before the first product: without this the scheduler,
    // short of registers, waits for each load in turn (one memory round trip per entry)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < kBlkRows; ++q) {
      s[q] = 0.f;
#pragma unroll
      for (int l = 0; l < NZ; ++l) s[q] += blk[q][l] * v[l];
    }
#pragma unroll
    for (int q = 0; q < kBlkRows; ++q)
      if (j + q < NZ) {
        const int e = (j + q) * nx + i;
        x[e] = (a == 0.f) ? w * s[q] : x[e] + w * s[q];
      }
  }
}

// Column step from a zero iterate: x = omega_c B_i^-1 f_i, and t1 = D_s x.
template <int NZ>
__device__ void r_colzero(int nx, const RLev& L, lptr<float> f, lptr<float> x, lptr<float> t1,
                          float wc) {
  for (int i = tid(); i < nx; i += nthr()) {
    float v[NZ], xn[NZ];
#pragma unroll
    for (int l = 0; l < NZ; ++l) v[l] = f[l * nx + i];
    r_blk_apply<NZ>(L.colinv, nx, i, v, x, 0.f, wc);
#pragma unroll
    for (int l = 0; l < NZ; ++l) xn[l] = x[l * nx + i];
    r_dsig_col<NZ>(L.Ds, xn, t1, nx, i);
  }
  __syncthreads();
}

// ----------------------------------------------------------------------------- lane FFT
//
// Complex FFT of length N = 64 M (M = 1, 2, 4, 8) held by one wavefront in registers: lane l
// holds the values x[l + 64 r], r < M. With k = M k1 + k2 (k1 < 64, k2 < M),
//   X[M k1 + k2] = sum_l W_64^(l k1) [ W_N^(l k2) sum_r x[l + 64 r] W_M^(r k2) ],
// so the forward transform is an M-point DFT in each lane's registers, a twiddle W_N^(l k2), and
// for every k2 a 64-point radix-2 decimation-in-frequency transform across the lanes (the partner
// of lane l at distance h is lane l ^ h, reached with DPP permutations for h < 16 and the
// gfx950 lane swaps for h = 16, 32). The result is left in bit-reversed lane order: lane l', register k2 holds
// X[M brev6(l') + k2]. The inverse runs the same steps backwards (decimation in time across the
// lanes, conjugate twiddles, inverse register DFT) and takes that order to natural order, so a
// multiplier in Fourier space needs no reordering at all. No LDS traffic and no wavefront sync.

__device__ __forceinline__ int brev6(int l) { return (int)(__builtin_bitreverse32((unsigned)l) >> 26); }

// The value of lane l ^ H for H < 16, by DPP lane permutations inside each row of 16 lanes
// (plain VALU moves, no LDS round trip): quad_perm [1,0,3,2] (H = 1), quad_perm [2,3,0,1]
// (H = 2), row_half_mirror then quad_perm [3,2,1,0] (l ^ 7 ^ 3 = l ^ 4) and row_ror:8 (H = 8).
template <int H>
__device__ __forceinline__ float lane_xor(float v) {
  const int x = __float_as_int(v);
  if constexpr (H == 1) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false));
  } else if constexpr (H == 2) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false));
  } else if constexpr (H == 4) {
    const int m = __builtin_amdgcn_mov_dpp(x, 0x141, 0xF, 0xF, false);
    return __int_as_float(__builtin_amdgcn_mov_dpp(m, 0x1B, 0xF, 0xF, false));
  } else {
    static_assert(H == 8, "lane_xor covers distances below 16");
    return __int_as_float(__builtin_amdgcn_mov_dpp(x, 0x128, 0xF, 0xF, false));
  }
}
template <int H>
__device__ __forceinline__ cpx<float> lane_xor(cpx<float> v) {
  return {lane_xor<H>(v.re), lane_xor<H>(v.im)};
}

// For H = 16 or 32: the gfx950 lane swap (v_permlane16_swap / v_permlane32_swap of a value with
// itself) returns, on every lane, s0 = the value of the lower lane of the pair (l & ~H) and
// s1 = that of the upper lane (l | H). The butterfly sum on the lower lane and difference on the
// upper one are then both s0 + sg s1 (sg = +1 below, -1 above).
template <int H>
__device__ __forceinline__ float lane_pair_sum(float v, float sg) {
  static_assert(H == 16 || H == 32, "lane_pair_sum covers distances 16 and 32");
  const unsigned x = __float_as_uint(v);
  if constexpr (H == 16) {
    const auto s = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    return __uint_as_float(s[0]) + sg * __uint_as_float(s[1]);
  } else {
    const auto s = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    return __uint_as_float(s[0]) + sg * __uint_as_float(s[1]);
  }
}

// Per-lane twiddles for one row length: wl[k2] = W_N^(l k2) and, per cross-lane stage s
// (distance h = 32 >> s), ws[s] = W_(2h)^(l mod h); read once from the LDS table tw[t] = W_N^t.
template <int M>
struct LaneTw {
  cpx<float> wl[M];
  cpx<float> ws[6];
};

template <int M>
__device__ __forceinline__ LaneTw<M> lane_tw(lptr<const cpx<float>> tw, int lane) {
  constexpr int N = 64 * M;
  LaneTw<M> t;
#pragma unroll
  for (int k2 = 0; k2 < M; ++k2) t.wl[k2] = lld<float>(tw, (lane * k2) & (N - 1));
#pragma unroll
  for (int st = 0; st < 6; ++st) {
    const int h = 32 >> st;
    t.ws[st] = lld<float>(tw, (lane & (h - 1)) * (32 * M / h));
  }
  return t;
}

__device__ __forceinline__ cpx<float> cconj(cpx<float> a) { return {a.re, -a.im}; }
__device__ __forceinline__ cpx<float> cswap(cpx<float> a) { return {a.im, a.re}; }

// In-register forward DFT of size M: v[k] <- sum_r v[r] W_M^(r k).
template <int M>
__device__ __forceinline__ void reg_dft(cpx<float> (&v)[M]) {
  if constexpr (M == 2) {
    const cpx<float> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (M == 4) {
    const cpx<float> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const cpx<float> t2 = cadd(v[1], v[3]), t3 = csub(v[1], v[3]);
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = {t1.re + t3.im, t1.im - t3.re};
    v[3] = {t1.re - t3.im, t1.im + t3.re};
  } else if constexpr (M == 8) {
    const float s = 0.70710678118654752f;
    cpx<float> a[4], b[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      a[r] = cadd(v[r], v[r + 4]);
      b[r] = csub(v[r], v[r + 4]);
    }
    b[1] = {s * (b[1].re + b[1].im), s * (b[1].im - b[1].re)};
    b[2] = {b[2].im, -b[2].re};
    b[3] = {s * (b[3].im - b[3].re), -s * (b[3].re + b[3].im)};
    reg_dft<4>(a);
    reg_dft<4>(b);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[2 * k] = a[k];
      v[2 * k + 1] = b[k];
    }
  }
}

// One cross-lane stage of the forward transform (distance H). With sg = +1 on the lower lane of
// each pair and -1 on the upper one, and wl = 1 on the lower lane and W_(2h)^(l mod h) on the
// upper one, the butterfly (x[j] + x[j+h], (x[j] - x[j+h]) W) is, on every lane,
// v' = (p + sg v) wl with p the partner's value: no selects and no divergent branches.
template <int M, int R, int H>
__device__ __forceinline__ void lane_dif(cpx<float> (&v)[R][M], cpx<float> w, int lane) {
  const bool up = (lane & H) != 0;
  const float sg = up ? -1.f : 1.f;
  const cpx<float> wl = up ? w : cpx<float>{1.f, 0.f};
#pragma unroll
  for (int q = 0; q < R; ++q)
#pragma unroll
    for (int k2 = 0; k2 < M; ++k2) {
      cpx<float> u;
      if constexpr (H >= 16) {
        u = {lane_pair_sum<H>(v[q][k2].re, sg), lane_pair_sum<H>(v[q][k2].im, sg)};
      } else {
        const cpx<float> p = lane_xor<H>(v[q][k2]);
        u = {p.re + sg * v[q][k2].re, p.im + sg * v[q][k2].im};
      }
      v[q][k2] = cmul(u, wl);
    }
}

// One cross-lane stage of the inverse transform (distance H, conjugate twiddle w): the upper lane
// sends t = v W (the lower lane t = v, wl = 1), and every lane forms v' = p + sg t.
template <int M, int R, int H>
__device__ __forceinline__ void lane_dit(cpx<float> (&v)[R][M], cpx<float> w, int lane) {
  const bool up = (lane & H) != 0;
  const float sg = up ? -1.f : 1.f;
  const cpx<float> wl = up ? w : cpx<float>{1.f, 0.f};
#pragma unroll
  for (int q = 0; q < R; ++q)
#pragma unroll
    for (int k2 = 0; k2 < M; ++k2) {
      const cpx<float> t = cmul(v[q][k2], wl);
      if constexpr (H >= 16) {
        v[q][k2] = {lane_pair_sum<H>(t.re, sg), lane_pair_sum<H>(t.im, sg)};
      } else {
        const cpx<float> p = lane_xor<H>(t);
        v[q][k2] = {p.re + sg * t.re, p.im + sg * t.im};
      }
    }
}

// Forward transform of R rows (natural order in, bit-reversed lane order out).
template <int M, int R>
__device__ __forceinline__ void lane_fft_fwd(cpx<float> (&v)[R][M], const LaneTw<M>& t,
                                             int lane) {
#pragma unroll
  for (int q = 0; q < R; ++q) {
    reg_dft<M>(v[q]);
#pragma unroll
    for (int k2 = 1; k2 < M; ++k2) v[q][k2] = cmul(v[q][k2], t.wl[k2]);
  }
  lane_dif<M, R, 32>(v, t.ws[0], lane);
  lane_dif<M, R, 16>(v, t.ws[1], lane);
  lane_dif<M, R, 8>(v, t.ws[2], lane);
  lane_dif<M, R, 4>(v, t.ws[3], lane);
  lane_dif<M, R, 2>(v, t.ws[4], lane);
  lane_dif<M, R, 1>(v, t.ws[5], lane);
}

// Inverse transform (unscaled) of R rows (bit-reversed lane order in, natural order out).
template <int M, int R>
__device__ __forceinline__ void lane_fft_inv(cpx<float> (&v)[R][M], const LaneTw<M>& t,
                                             int lane) {
  lane_dit<M, R, 1>(v, cconj(t.ws[5]), lane);
  lane_dit<M, R, 2>(v, cconj(t.ws[4]), lane);
  lane_dit<M, R, 4>(v, cconj(t.ws[3]), lane);
  lane_dit<M, R, 8>(v, cconj(t.ws[2]), lane);
  lane_dit<M, R, 16>(v, cconj(t.ws[1]), lane);
  lane_dit<M, R, 32>(v, cconj(t.ws[0]), lane);
#pragma unroll
  for (int q = 0; q < R; ++q) {
#pragma unroll
    for (int k2 = 1; k2 < M; ++k2) v[q][k2] = cmul(v[q][k2], cconj(t.wl[k2]));
    // inverse register DFT by the swap identity: IDFT(a) = swap(DFT(swap(a)))
#pragma unroll
    for (int k2 = 0; k2 < M; ++k2) v[q][k2] = cswap(v[q][k2]);
    reg_dft<M>(v[q]);
#pragma unroll
    for (int k2 = 0; k2 < M; ++k2) v[q][k2] = cswap(v[q][k2]);
  }
}

// Mode pairs whose block entries one step of the mode solve loads together.
constexpr int kModePairs = 5;

// The flat-mode solve on the spectra of the NP packed pairs in T3 (row length N, the spectrum
// of frequency k of pair p at p N + pos(k)): for each k in [0, N/2], unpack the nz real rows'
// spectra at k and N - k, multiply by the inverse mode block (minv [NZ][NZ][N/2 + 1]), repack
// in place, with the inverse transform's 1/N. One thread per mode pair (k, N - k).
template <int NZ, class Pos>
__device__ __forceinline__ void r_mode_matvec(int N, lptr<cpx<float>> T3, gptr<const float> minv,
                                              Pos pos) {
  constexpr int NP = (NZ + 1) / 2;
  const int nh = (N >> 1) + 1;
  const float half = 0.5f, scale = 1.f / (float)N;
  for (int k = tid(); k < nh; k += nthr()) {
    const int kc = (N - k) & (N - 1);
    const bool both = (k != 0 && k != (N >> 1));
    const int pk = pos(k), pkc = pos(kc);
    cpx<float> rh[NZ];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const cpx<float> z = lld<float>(T3, p * N + pk), zc = lld<float>(T3, p * N + pkc);
      if (p > 0) rh[2 * p - 1] = {half * (z.re + zc.re), half * (z.im - zc.im)};
      rh[2 * p] = {half * (z.im + zc.im), -half * (z.re - zc.re)};
    }
    // every pair's spectra at k and N - k are in rh: results overwrite the inputs in place
#pragma unroll 1
    for (int p0 = 0; p0 < NP; p0 += kModePairs) {
      float a[kModePairs][2][NZ];
#pragma unroll
      for (int q = 0; q < kModePairs; ++q)
#pragma unroll
        for (int l = 0; l < NZ; ++l) {
          const int j0 = 2 * (p0 + q) - 1, j1 = j0 + 1;
          a[q][0][l] = (j0 >= 0 && j0 < NZ) ? minv[(j0 * NZ + l) * nh + k] : 0.f;
          a[q][1][l] = (j1 < NZ) ? minv[(j1 * NZ + l) * nh + k] : 0.f;
        }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int q = 0; q < kModePairs; ++q) {
        const int p = p0 + q;
        if (p >= NP) break;
        cpx<float> s0 = {0.f, 0.f}, s1 = {0.f, 0.f};
#pragma unroll
        for (int l = 0; l < NZ; ++l) {
          s0.re += a[q][0][l] * rh[l].re;
          s0.im += a[q][0][l] * rh[l].im;
          s1.re += a[q][1][l] * rh[l].re;
          s1.im += a[q][1][l] * rh[l].im;
        }
        s0.re *= scale; s0.im *= scale; s1.re *= scale; s1.im *= scale;
        lst<float>(T3, p * N + pk, {s0.re - s1.im, s0.im + s1.re});
        if (both) lst<float>(T3, p * N + pkc, {s0.re + s1.im, s1.re - s0.im});
      }
    }
  }
}

// ----------------------------------------------------------------------------- 16 x 16 rows
// Rows of N = 256 points by the four-step factorisation 256 = 16 x 16, one row per group of 16
// lanes (four rows per wavefront). With n = t + 16 r and k = s + 16 u (t, r, s, u < 16),
//   X[s + 16 u] = sum_t W_16^(t u) [ W_256^(t s) sum_r x[t + 16 r] W_16^(r s) ]:
// lane t holds x[t + 16 r] in register r, transforms over r in registers, applies the twiddle,
// and a transpose through LDS gives lane s the values over t, which it transforms in registers,
// ending with X[s + 16 u] in register u: natural order, lane s holding every frequency = s mod 16.
// Per row this is about 2.3 times fewer vector instructions than six cross-lane radix-2 stages.
// The transpose writes element (t, s) at s 16 + (t ^ s) and reads it back there: both sides touch
// 16 distinct bank pairs, and the buffer is the 256-element row it belongs to.

// W_16^e for e = n1 k1 of the radix-4 x 4 split, applied to a (e = 4 is -i).
__device__ __forceinline__ cpx<float> w16mul(cpx<float> a, int e) {
  const float c1 = 0.92387953251128674f, s1 = 0.38268343236508977f, h = 0.70710678118654752f;
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

// In-register forward DFT of 16 points, radix 4 x 4: with n = n1 + 4 n2 and k = k1 + 4 k2,
// X[k1 + 4 k2] = sum_n1 W_4^(n1 k2) W_16^(n1 k1) sum_n2 v[n1 + 4 n2] W_4^(n2 k1).
__device__ __forceinline__ void reg_dft16(cpx<float> (&v)[16]) {
  cpx<float> a[4][4];
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) {
    cpx<float> q[4] = {v[n1], v[n1 + 4], v[n1 + 8], v[n1 + 12]};
    reg_dft<4>(q);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) a[n1][k1] = w16mul(q[k1], n1 * k1);
  }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cpx<float> q[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
    reg_dft<4>(q);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = q[k2];
  }
}

// Inverse (unscaled) by the swap identity IDFT(a) = swap(DFT(swap(a))).
__device__ __forceinline__ void reg_idft16(cpx<float> (&v)[16]) {
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = cswap(v[k]);
  reg_dft16(v);
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = cswap(v[k]);
}

// Twiddles of lane t: w[s] = W_256^(t s).
struct FsTw {
  cpx<float> w[16];
};
__device__ __forceinline__ FsTw fs_tw(lptr<const cpx<float>> tw, int t) {
  FsTw f;
#pragma unroll
  for (int s = 0; s < 16; ++s) f.w[s] = lld<float>(tw, (t * s) & 255);
  return f;
}

// Forward transform of the group's row: in v[r] = x[t + 16 r], out v[u] = X[t + 16 u]. S is the
// row's 256-element LDS buffer (only groups with a row, ok, touch it); the wavefront syncs are
// uniform.
__device__ __forceinline__ void fs_fwd(cpx<float> (&v)[16], const FsTw& tw,
                                       lptr<cpx<float>> S, int t, bool ok) {
  reg_dft16(v);
#pragma unroll
  for (int s = 0; s < 16; ++s) v[s] = cmul(v[s], tw.w[s]);
  if (ok) {
#pragma unroll
    for (int s = 0; s < 16; ++s) lst<float>(S, s * 16 + (t ^ s), v[s]);
  }
  wave_sync();
  if (ok) {
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = lld<float>(S, t * 16 + (q ^ t));
  }
  wave_sync();
  reg_dft16(v);
}

// Inverse (unscaled): in v[u] = X[t + 16 u], out v[r] = N x[t + 16 r].
__device__ __forceinline__ void fs_inv(cpx<float> (&v)[16], const FsTw& tw,
                                       lptr<cpx<float>> S, int t, bool ok) {
  reg_idft16(v);
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = cmul(v[q], cconj(tw.w[q]));
  if (ok) {
#pragma unroll
    for (int q = 0; q < 16; ++q) lst<float>(S, q * 16 + (t ^ q), v[q]);
  }
  wave_sync();
  if (ok) {
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = lld<float>(S, t * 16 + (q ^ t));
  }
  wave_sync();
  reg_idft16(v);
}

// r_dx2_lane for N = 256 with the 16 x 16 transform: pair pp = 4 (wavefront) + group. The pair's
// t3 row is the transpose buffer of both passes (its result is stored last).
template <int NZ>
__device__ __noinline__ void r_dx2_fs(RCtx c_, RMap m_, lptr<const float> sig_) {
  constexpr int N = 256, NP = (NZ + 1) / 2;
  const RCtx c = uni(c_);
  RMap m;
  m.geo = uni(m_.geo); m.t1 = uni(m_.t1); m.t2 = uni(m_.t2); m.t3 = uni(m_.t3); m.x = uni(m_.x);
  const lptr<const float> sig = uni(sig_);
  const int lane = tid() & 63, t = lane & 15;
  const lptr<const cpx<float>> twl = (lptr<const cpx<float>>)as_lds(lds_tw<float>(c.fftb, N));
  const FsTw tw = fs_tw(twl, t);
  float kap[16];   // i kappa / N at frequency t + 16 u (Nyquist 0)
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int k = t + 16 * u;
    const int kk = (k <= N / 2) ? k : k - N;
    kap[u] = (k == N / 2) ? 0.f : c.kfac * (float)kk * (1.f / (float)N);
  }
  const lptr<cpx<float>> T2 = (lptr<cpx<float>>)m.t2;
  const lptr<cpx<float>> T3 = (lptr<cpx<float>>)m.t3;
  const lptr<float> ao = m.geo, bo = m.geo + N;
  for (int base = 0; base < NP; base += 4 * (nthr() >> 6)) {
    const int pp = base + (tid() >> 4);
    const bool ok = pp < NP;
    const int j0 = 2 * pp - 1, j1 = 2 * pp;
    const lptr<cpx<float>> S = T3 + (ok ? pp : 0) * N;
    cpx<float> v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int n = t + 16 * r;
      v[r] = {(ok && j0 >= 0) ? m.x[j0 * N + n] : 0.f, ok ? m.x[j1 * N + n] : 0.f};
    }
    const float s0 = (ok && j0 >= 0) ? sig[j0] : 0.f, s1 = ok ? sig[j1] : 0.f;
    for (int pass = 0; pass < 2; ++pass) {
      fs_fwd(v, tw, S, t, ok);
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = {-kap[u] * v[u].im, kap[u] * v[u].re};
      fs_inv(v, tw, S, t, ok);
      if (!ok) continue;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int n = t + 16 * r;
        if (pass == 0) {
          const float a = ao[n], b = bo[n];
          const cpx<float> g = {j0 >= 0 ? v[r].re + (a + b * s0) * m.t1[j0 * N + n] : 0.f,
                                v[r].im + (a + b * s1) * m.t1[j1 * N + n]};
          lst<float>(T2, pp * N + n, g);
          v[r] = g;
        } else {
          lst<float>(T3, pp * N + n, v[r]);
        }
      }
    }
  }
  __syncthreads();
}

// r_mode_lane for N = 256 with the 16 x 16 transform: spectra in natural order in t3.
template <int NZ>
__device__ __noinline__ void r_mode_fs(RCtx c_, RMap m_, gptr<const float> minv_) {
  constexpr int N = 256, NP = (NZ + 1) / 2;
  const RCtx c = uni(c_);
  const lptr<float> t3 = uni(m_.t3), x = uni(m_.x);
  const gptr<const float> minv = uni(minv_);
  const int lane = tid() & 63, t = lane & 15;
  const lptr<const cpx<float>> twl = (lptr<const cpx<float>>)as_lds(lds_tw<float>(c.fftb, N));
  const FsTw tw = fs_tw(twl, t);
  const lptr<cpx<float>> T3 = (lptr<cpx<float>>)t3;
  for (int base = 0; base < NP; base += 4 * (nthr() >> 6)) {
    const int pp = base + (tid() >> 4);
    const bool ok = pp < NP;
    const lptr<cpx<float>> S = T3 + (ok ? pp : 0) * N;
    cpx<float> v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = ok ? lld<float>(S, t + 16 * r) : cpx<float>{0.f, 0.f};
    wave_sync();
    fs_fwd(v, tw, S, t, ok);
    if (ok) {
#pragma unroll
      for (int u = 0; u < 16; ++u) lst<float>(S, t + 16 * u, v[u]);
    }
  }
  __syncthreads();
  r_mode_matvec<NZ>(N, T3, minv, [](int k) { return k; });
  __syncthreads();
  const float wm = c.wm;
  for (int base = 0; base < NP; base += 4 * (nthr() >> 6)) {
    const int pp = base + (tid() >> 4);
    const bool ok = pp < NP;
    const int j0 = 2 * pp - 1, j1 = 2 * pp;
    const lptr<cpx<float>> S = T3 + (ok ? pp : 0) * N;
    cpx<float> v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = ok ? lld<float>(S, t + 16 * u) : cpx<float>{0.f, 0.f};
    wave_sync();
    fs_inv(v, tw, S, t, ok);
    if (!ok) continue;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int n = t + 16 * r;
      const float x0 = j0 >= 0 ? x[j0 * N + n] : 0.f;
      const float x1 = x[j1 * N + n];
      if (j0 >= 0) x[j0 * N + n] = x0 + wm * v[r].re;
      x[j1 * N + n] = x1 + wm * v[r].im;
    }
  }
  __syncthreads();
}

// Row pairs per wavefront and round of the lane FFT: enough for four wavefronts to cover the
// NP = (NZ + 1) / 2 pairs in one round, at most kWaveRows.
template <int NZ>
constexpr int kLaneRows = ((NZ + 1) / 2 + 3) / 4 < kWaveRows ? ((NZ + 1) / 2 + 3) / 4 : kWaveRows;

// Phases B and C of the operator with the lane FFT (rows of length 64 M): per pair of rows, in
// registers, P_x = D_x x, G_x = P_x + sigma_x^old D_s x (stored to t2, packed) and D_x G_x
// (stored to t3, packed). Only the closing barrier is a workgroup barrier.
template <int NZ, int M>
__device__ __noinline__ void r_dx2_lane(RCtx c_, RMap m_, lptr<const float> sig_) {
  constexpr int N = 64 * M, NP = (NZ + 1) / 2, R = kLaneRows<NZ>;
  const RCtx c = uni(c_);
  RMap m;
  m.geo = uni(m_.geo); m.t1 = uni(m_.t1); m.t2 = uni(m_.t2); m.t3 = uni(m_.t3); m.x = uni(m_.x);
  const lptr<const float> sig = uni(sig_);
  const int lane = tid() & 63, w = tid() >> 6, nw = nthr() >> 6;
  const lptr<const cpx<float>> twl = (lptr<const cpx<float>>)as_lds(lds_tw<float>(c.fftb, N));
  const LaneTw<M> t = lane_tw<M>(twl, lane);
  float kap[M];   // i kappa / N at the frequency this lane's register k2 holds (Nyquist 0)
#pragma unroll
  for (int k2 = 0; k2 < M; ++k2) {
    const int k = M * brev6(lane) + k2;
    const int kk = (k <= N / 2) ? k : k - N;
    kap[k2] = (k == N / 2) ? 0.f : c.kfac * (float)kk * (1.f / (float)N);
  }
  const lptr<cpx<float>> T2 = (lptr<cpx<float>>)m.t2;
  const lptr<cpx<float>> T3 = (lptr<cpx<float>>)m.t3;
  const lptr<float> ao = m.geo, bo = m.geo + N;
  for (int base = 0; base < NP; base += nw * R) {
    cpx<float> v[R][M];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int pp = base + w + q * nw, j0 = 2 * pp - 1, j1 = 2 * pp;
#pragma unroll
      for (int r = 0; r < M; ++r) {
        const int n = lane + 64 * r;
        v[q][r] = {(j0 >= 0 && pp < NP) ? m.x[j0 * N + n] : 0.f, pp < NP ? m.x[j1 * N + n] : 0.f};
      }
    }
    for (int pass = 0; pass < 2; ++pass) {
      lane_fft_fwd<M, R>(v, t, lane);
#pragma unroll
      for (int q = 0; q < R; ++q)
#pragma unroll
        for (int k2 = 0; k2 < M; ++k2) v[q][k2] = {-kap[k2] * v[q][k2].im, kap[k2] * v[q][k2].re};
      lane_fft_inv<M, R>(v, t, lane);
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int pp = base + w + q * nw, j0 = 2 * pp - 1, j1 = 2 * pp;
        if (pp >= NP) continue;
        const float s0 = j0 >= 0 ? sig[j0] : 0.f, s1 = sig[j1];
#pragma unroll
        for (int r = 0; r < M; ++r) {
          const int n = lane + 64 * r;
          if (pass == 0) {
            const float a = ao[n], b = bo[n];
            const cpx<float> g = {j0 >= 0 ? v[q][r].re + (a + b * s0) * m.t1[j0 * N + n] : 0.f,
                                  v[q][r].im + (a + b * s1) * m.t1[j1 * N + n]};
            lst<float>(T2, pp * N + n, g);
            v[q][r] = g;
          } else {
            lst<float>(T3, pp * N + n, v[q][r]);
          }
        }
      }
    }
  }
  __syncthreads();
}

// Flat-mode step with the lane FFT: the residual r in t3 (packed, natural order) is transformed
// in registers and its spectra stored back in t3 in the lane order (pair p, lane l', register
// k2 at p N + 64 k2 + l'); mode k is at 64 (k mod M) + brev6(k / M). The mode blocks then act
// per Fourier mode (with the 1/N of the inverse transform), and the inverse transforms add
// omega_m times the correction to x.
template <int NZ, int M>
__device__ __noinline__ void r_mode_lane(RCtx c_, RMap m_, gptr<const float> minv_) {
  constexpr int N = 64 * M, NP = (NZ + 1) / 2, R = kLaneRows<NZ>;
  const RCtx c = uni(c_);
  const lptr<float> t3 = uni(m_.t3), x = uni(m_.x);
  const gptr<const float> minv = uni(minv_);
  const int lane = tid() & 63, w = tid() >> 6, nw = nthr() >> 6;
  const lptr<const cpx<float>> twl = (lptr<const cpx<float>>)as_lds(lds_tw<float>(c.fftb, N));
  const LaneTw<M> t = lane_tw<M>(twl, lane);
  const lptr<cpx<float>> T3 = (lptr<cpx<float>>)t3;
  for (int base = 0; base < NP; base += nw * R) {
    cpx<float> v[R][M];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int pp = base + w + q * nw;
#pragma unroll
      for (int r = 0; r < M; ++r)
        v[q][r] = pp < NP ? lld<float>(T3, pp * N + lane + 64 * r) : cpx<float>{0.f, 0.f};
    }
    lane_fft_fwd<M, R>(v, t, lane);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int pp = base + w + q * nw;
      if (pp >= NP) continue;
#pragma unroll
      for (int k2 = 0; k2 < M; ++k2) lst<float>(T3, pp * N + 64 * k2 + lane, v[q][k2]);
    }
  }
  __syncthreads();
  r_mode_matvec<NZ>(N, T3, minv,
                    [](int k) { return 64 * (k & (M - 1)) + brev6(k / M); });
  __syncthreads();
  const float wm = c.wm;
  for (int base = 0; base < NP; base += nw * R) {
    cpx<float> v[R][M];
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int pp = base + w + q * nw;
#pragma unroll
      for (int k2 = 0; k2 < M; ++k2)
        v[q][k2] = pp < NP ? lld<float>(T3, pp * N + 64 * k2 + lane) : cpx<float>{0.f, 0.f};
    }
    lane_fft_inv<M, R>(v, t, lane);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int pp = base + w + q * nw, j0 = 2 * pp - 1, j1 = 2 * pp;
      if (pp >= NP) continue;
#pragma unroll
      for (int r = 0; r < M; ++r) {
        const int n = lane + 64 * r;
        const float x0 = j0 >= 0 ? x[j0 * N + n] : 0.f;
        const float x1 = x[j1 * N + n];
        if (j0 >= 0) x[j0 * N + n] = x0 + wm * v[q][r].re;
        x[j1 * N + n] = x1 + wm * v[q][r].im;
      }
    }
  }
  __syncthreads();
}

enum : int { RF_RESID = 0, RF_COLSTEP = 1 };

// Phase D of the operator (column finish) with t1 = D_s x, t2 = G_x, t3 = D_x G_x:
//   A x = D_x G_x + D_s (a_n G_x + G_z / d_n) + b_n sigma D_s G_x inside (G_z = D_s x / d_o),
//   row 0 = x (Dirichlet), row M = -(h_x G_x + G_z) (bed),
// and r = f - A x. RF_RESID: r goes to t3 (packed, in place of D_x G_x), or, when fc is given,
// only its restriction R r to fc (the next level's right-hand side). RF_COLSTEP: the column-block
// step x += omega_c B_i^-1 r_i, then t1 = D_s x.
template <int NZ>
__device__ void r_finish(int mode, const RCtx& c, const RMap& m, const RLev& L, lptr<float> fc) {
  constexpr int M = NZ - 1, NZC = (NZ + 1) / 2;
  const int nx = c.nx;
  const lptr<float> g = m.geo;
  for (int i = tid(); i < nx; i += nthr()) {
    // live across the row loop: G_x, u = a_n G_x + G_z / d_n and the residual column
    float gx[NZ], u[NZ], res[NZ];
    pk_col<NZ>(m.t2, nx, i, gx);
    const float ido = g[2 * nx + i], an = g[3 * nx + i], bn = g[4 * nx + i];
    const float idn = g[5 * nx + i], hx = g[6 * nx + i];
    float psM;
    {
      float ps[NZ];
#pragma unroll
      for (int l = 0; l < NZ; ++l) ps[l] = m.t1[l * nx + i];
#pragma unroll
      for (int l = 0; l < NZ; ++l) u[l] = an * gx[l] + idn * (ps[l] * ido);
      psM = ps[M];
    }
    res[0] = m.f[i] - m.x[i];
    res[M] = m.f[M * nx + i] + (hx * gx[M] + psM * ido);
#pragma unroll
    for (int j = 1; j < M; ++j) {
      float s1 = 0.f, s2 = 0.f;
#pragma unroll
      for (int l = 0; l < NZ; ++l) {
        const float d = L.Ds[j * NZ + l];
        s1 += d * u[l];
        s2 += d * gx[l];
      }
      const float dg = m.t3[((j + 1) >> 1) * 2 * nx + 2 * i + ((j + 1) & 1)];
      res[j] = m.f[j * nx + i] - (dg + s1 + bn * L.sig[j] * s2);
    }
    if (mode == RF_RESID) {
      if (fc) {
#pragma unroll
        for (int jc = 0; jc < NZC; ++jc) {
          float s = 0.f;
#pragma unroll
          for (int l = 0; l < NZ; ++l) s += L.R[jc * NZ + l] * res[l];
          fc[jc * nx + i] = s;
        }
      } else {
#pragma unroll
        for (int pr = 0; pr < NZC; ++pr)
          pk_st(m.t3, nx, pr, i, vf2{pr > 0 ? res[2 * pr - 1] : 0.f, res[2 * pr]});
      }
    } else {
      r_blk_apply<NZ>(L.colinv, nx, i, res, m.x, 1.f, c.wc);
      float xn[NZ];
#pragma unroll
      for (int l = 0; l < NZ; ++l) xn[l] = m.x[l * nx + i];
      r_dsig_col<NZ>(L.Ds, xn, m.t1, nx, i);
    }
  }
  __syncthreads();
}

// x += P xc (prolongation from the next coarser level), then t1 = D_s x.
template <int NZ>
__device__ void r_prolong(int nx, const RLev& L, lptr<float> xc, lptr<float> x, lptr<float> t1) {
  constexpr int NZC = (NZ + 1) / 2;
  for (int i = tid(); i < nx; i += nthr()) {
    float v[NZC], xn[NZ];
#pragma unroll
    for (int cc = 0; cc < NZC; ++cc) v[cc] = xc[cc * nx + i];
#pragma unroll
    for (int j = 0; j < NZ; ++j) {
      float s = 0.f;
#pragma unroll
      for (int cc = 0; cc < NZC; ++cc) s += L.P[j * NZC + cc] * v[cc];
      xn[j] = x[j * nx + i] + s;
    }
#pragma unroll
    for (int l = 0; l < NZ; ++l) x[l * nx + i] = xn[l];
    r_dsig_col<NZ>(L.Ds, xn, t1, nx, i);
  }
  __syncthreads();
}

// fc = R f (restriction of the right-hand side itself: a level move from a zero iterate).
template <int NZ>
__device__ void r_restrict(int nx, const RLev& L, lptr<float> f, lptr<float> fc) {
  constexpr int NZC = (NZ + 1) / 2;
  for (int i = tid(); i < nx; i += nthr()) {
    float v[NZ];
#pragma unroll
    for (int l = 0; l < NZ; ++l) v[l] = f[l * nx + i];
#pragma unroll
    for (int jc = 0; jc < NZC; ++jc) {
      float s = 0.f;
#pragma unroll
      for (int l = 0; l < NZ; ++l) s += L.R[jc * NZ + l] * v[l];
      fc[jc * nx + i] = s;
    }
  }
  __syncthreads();
}

__device__ __forceinline__ void r_fill(lptr<float> p, int n) {
  for (int e = tid(); e < n; e += nthr()) p[e] = 0.f;
  __syncthreads();
}

// The resident V-cycle on the level of NZ rows (finest NZ0), from a zero iterate: input f_l,
// output x_l. The same sequence of steps as vcycle() in pmgw_device.hpp: nu1 x (column step,
// mode step), the level move (residual restricted in the column finish, the coarser cycle,
// prolongation), nu2 x (column step, mode step); on the coarsest level (3 rows) coarse_pairs
// pairs or the direct solve.
template <int NZ0, int NZ>
__device__ __noinline__ void rvcycle(RCtx c_) {
  const RCtx c = uni(c_);
  const int nx = c.nx;
  constexpr int l = res_level(NZ0, NZ);
  const RMap m = res_map<NZ0, NZ>(nx);
  const RLev L = res_lev<NZ>(c, m, l);
  if constexpr (NZ == 3) {
    if (c.coarse_exact && c.cw) {
      coarse_direct<float, false>(nx, c.cw, c.cwt, m.f, m.x,
                                  (lptr<double>)(reinterpret_cast<lptr<char>>(m.t2)));
      return;
    }
  }
  enum { COL = 0, MODE = 1, DOWN = 2 };
  const int npre = (NZ == 3) ? c.coarse_pairs : c.nu1;
  const int npost = (NZ == 3) ? 0 : c.nu2;
  const int nsteps = 2 * npre + ((NZ == 3) ? 0 : 1) + 2 * npost;
  bool xzero = true, t1x = false;
  for (int q = 0; q < nsteps; ++q) {
    int kind;
    if (q < 2 * npre) kind = (q & 1) ? MODE : COL;
    else if (NZ != 3 && q == 2 * npre) kind = DOWN;
    else kind = ((q - 2 * npre - 1) & 1) ? MODE : COL;
    if (kind == COL && xzero) {
      r_colzero<NZ>(nx, L, m.f, m.x, m.t1, c.wc);
      xzero = false;
      t1x = true;
      continue;
    }
    if (xzero) {
      // a mode step or a level move before any column step (nu1 = 0): from x = 0
      r_fill(m.x, NZ * nx);
      r_fill(m.t1, NZ * nx);
      xzero = false;
      t1x = true;
      if constexpr (NZ > 3) {
        if (kind == DOWN) {
          r_restrict<NZ>(nx, L, m.f, m.fc);
          rvcycle<NZ0, (NZ + 1) / 2>(c);
          r_prolong<NZ>(nx, L, m.xc, m.x, m.t1);
          continue;
        }
      }
    }
    if (!t1x) r_dsig<NZ>(nx, L.Ds, m.x, m.t1);
    switch (nx) {
      case 64: r_dx2_lane<NZ, 1>(c, m, L.sig); break;
      case 128: r_dx2_lane<NZ, 2>(c, m, L.sig); break;
      case 256:
        // the 16 x 16 transform pays off with two or more pairs per wavefront (17 rows)
        if constexpr (NZ == 17) r_dx2_fs<NZ>(c, m, L.sig);
        else r_dx2_lane<NZ, 4>(c, m, L.sig);
        break;
      default: r_dx2_lane<NZ, 8>(c, m, L.sig); break;
    }
    if (kind == COL) {
      r_finish<NZ>(RF_COLSTEP, c, m, L, lptr<float>(nullptr));
      t1x = true;
    } else if (kind == MODE) {
      r_finish<NZ>(RF_RESID, c, m, L, lptr<float>(nullptr));
      switch (nx) {
        case 64: r_mode_lane<NZ, 1>(c, m, L.modeinv); break;
        case 128: r_mode_lane<NZ, 2>(c, m, L.modeinv); break;
        case 256:
          if constexpr (NZ == 17) r_mode_fs<NZ>(c, m, L.modeinv);
          else r_mode_lane<NZ, 4>(c, m, L.modeinv);
          break;
        default: r_mode_lane<NZ, 8>(c, m, L.modeinv); break;
      }
      t1x = false;
    } else {
      if constexpr (NZ > 3) {
        r_finish<NZ>(RF_RESID, c, m, L, m.fc);
        rvcycle<NZ0, (NZ + 1) / 2>(c);
        r_prolong<NZ>(nx, L, m.xc, m.x, m.t1);
        t1x = true;
      }
    }
  }
  if (xzero) r_fill(m.x, NZ * nx);
}

// Loads the float32 metrics into the map's geometry rows (ao, bo, ido, an, bn, idn, hx) and every
// level's tables into the table area (no barrier; the caller's next barrier orders them).
template <int NZ0>
__device__ __forceinline__ void res_load_geo(char* ws, const TankDesc& td) {
  const lptr<float> g = (lptr<float>)(reinterpret_cast<float*>(g_fft_lds));
  const gptr<const float> src = (gptr<const float>)(ws + td.geo32);
  for (int e = tid(); e < 7 * td.nx; e += nthr()) g[e] = src[e];
  const lptr<float> tab = g + res_floats_per_col(NZ0) * td.nx;
  for (int l = 0; l < td.nlev; ++l) {
    const LevelDesc& d = td.lev[l];
    const int nz = d.nz, nzc = d.nzc;
    const lptr<float> t = tab + ((l == 0) ? 0 : res_tab_before(NZ0, l));
    const gptr<const float> Ds = (gptr<const float>)(ws + d.ds[1]);
    const gptr<const float> sg = (gptr<const float>)(ws + d.sig[1]);
    for (int e = tid(); e < nz * nz; e += nthr()) t[e] = Ds[e];
    for (int e = tid(); e < nz; e += nthr()) t[nz * nz + e] = sg[e];
    if (nzc) {
      const gptr<const float> R = (gptr<const float>)(ws + d.R[1]);
      const gptr<const float> P = (gptr<const float>)(ws + d.P[1]);
      for (int e = tid(); e < nzc * nz; e += nthr()) {
        t[nz * nz + nz + e] = R[e];
        t[nz * nz + nz + nzc * nz + e] = P[e];
      }
    }
  }
}

}  // namespace pmgw

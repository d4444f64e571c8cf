// Host side of the p-multigrid pressure Poisson library: plans, workspace layout, constant
// tables, argument validation and kernel launches behind the C ABI declared in pmgw.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <atomic>
#include <mutex>
#include <vector>

#include "../../include/pmgw.h"
#include "pmgw_launch.hpp"
#include "pmgw_setup.hpp"
#include "pmgw_tables.hpp"

using namespace pmgw;

static_assert(sizeof(pmgw_info) == sizeof(pmgw_info_dev), "info layout");

namespace {

thread_local std::string g_err;

std::atomic<uint64_t> g_plan_gen{0};   // owner tags of the static scratch array

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(PMGW_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

int64_t align256(int64_t v) { return (v + 255) & ~int64_t(255); }

}  // namespace

// the 3D tanks' entry points report through the same per-thread message
namespace pmgw_errors {
int set(int code, const std::string& msg) { return fail(code, msg); }
}  // namespace pmgw_errors

namespace {

using pmgw_tables::cgl_sigma;
using pmgw_tables::dsigma;
using pmgw_tables::ilog2;
using pmgw_tables::prolongation;
using pmgw_tables::restriction;
using pmgw_tables::transpose;

// Exponential cut-off filter of paper Sec. 3.6 (with the damping sign): 1 for i <= Nc, else
// exp(-alpha ((i - Nc)/(N + 1 - Nc))^s).
double filter_factor(int i, int N, int Nc, double alpha, double s) {
  if (i <= Nc) return 1.0;
  return std::exp(-alpha * std::pow((i - Nc) / (N + 1.0 - Nc), s));
}

// Nodal sigma filter on the CGL nodes: Chebyshev coefficients scaled by the filter factors.
std::vector<double> sigma_filter(int M, double frac, double alpha, double s) {
  const int n = M + 1, Nc = (int)std::floor(frac * M);
  std::vector<double> F(n * n, 0.0);
  for (int j = 0; j < n; ++j)
    for (int l = 0; l < n; ++l) {
      const double cl = (l == 0 || l == M) ? 2.0 : 1.0;
      double acc = 0.0;
      for (int m = 0; m <= M; ++m) {
        const double cm = (m == 0 || m == M) ? 2.0 : 1.0;
        acc += std::cos(M_PI * j * m / M) * filter_factor(m, M, Nc, alpha, s) *
               (2.0 / (M * cm * cl)) * std::cos(M_PI * m * l / M);
      }
      F[j * n + l] = acc;
    }
  return F;
}

// Carpenter-Kennedy (5,4) coefficients of the 2N low-storage scheme.
const double kCkAlpha[5] = {0.0, -567301805773.0 / 1357537059087.0,
                            -2404267990393.0 / 2016746695238.0,
                            -3550918686646.0 / 2091501179385.0,
                            -1275806237668.0 / 842570457699.0};
const double kCkBeta[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                           1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                           2277821191437.0 / 14882151754819.0};

}  // namespace

struct pmgw_plan_s {
  int ntanks = 0;
  int prec = PMGW_FP64;
  pmgw_opts opts{};
  hipStream_t stream = nullptr;
  int device = 0;
  std::vector<TankDesc> tanks;
  std::vector<BlockJob> jobs;
  int64_t nblocks = 0;
  std::vector<int64_t> off2d, off1d;
  // constant image: [descs][jobs][per-tank tables...] copied at bind time
  std::vector<char> image;
  int64_t desc_off = 0, job_off = 0, info_off = 0, rk_off = 0, adj_off = 0;
  // stage pressure history of opts.guess_steps: 5 rings of m slots of n2d doubles at hist_off;
  // hist_cnt[s] recorded steps of stage s + 1, hist_head[s] its next slot, hist_k the last
  // rk4_stage call's k (0: none), hist_dt its dt
  int64_t hist_off = 0;
  int hist_cnt[5] = {0, 0, 0, 0, 0}, hist_head[5] = {0, 0, 0, 0, 0};
  int hist_k = 0;
  double hist_dt = 0.0;
  // opts.guess_correct: the last call's extrapolation (n2d doubles at eprev_off), valid when
  // hist_eprev is set
  int64_t eprev_off = 0;
  bool hist_eprev = false;
  // tanks grouped by finest-level row count (3, 5, 9, 17, 33): one solve launch per class
  int64_t ids_off[5] = {0, 0, 0, 0, 0};
  std::vector<int32_t> ids[5];
  int maxnx[5] = {0, 0, 0, 0, 0};   // largest Nx per class (sizes the LDS twiddle tables)
  int maxnx_all = 0;
  int64_t total = 0;
  char* ws = nullptr;
  bool geometry_set = false;
  bool serial = false;     // run the Nz classes one after another on `stream` (no side streams)
  uint64_t gen = 0;        // unique id of the plan (owner tag of the static scratch array)
  int threads = 256;
  // launch timing of the solve kernels (pmgw_profile): one event pair per solve call
  std::vector<hipEvent_t> ev0, ev1;
  int prof_n = 0;
  bool prof_on = false;
  // side streams (default priority) and events that run the Nz classes of one solve call
  // concurrently, forked from and joined back to `stream`; created on first use
  // each class split for the mixed-precision V-cycle: rids = tanks whose cycle runs in LDS
  // (pmgw_resident.hpp), xids = the others; rres = largest resident map (bytes) of the class
  int64_t rids_off[5] = {0, 0, 0, 0, 0}, xids_off[5] = {0, 0, 0, 0, 0};
  std::vector<int32_t> rids[5], xids[5];
  int rmaxnx[5] = {0, 0, 0, 0, 0}, xmaxnx[5] = {0, 0, 0, 0, 0};
  int64_t rres[5] = {0, 0, 0, 0, 0};
  // launch groups 3 c + k of class c: k = 0 all tanks, 1 the resident part, 2 the rest; side
  // streams (default priority) and events that run the groups of one solve call concurrently,
  // forked from and joined back to `stream`; created on first use
  hipStream_t side[15] = {};
  hipEvent_t fork = nullptr, join[15] = {};
  // rk4_stage runs the smoother set-up (block inverses, optional bed-line and coarse set-ups) on
  // this stream, forked after the geometry kernel and joined before the solve, so that it
  // overlaps the forcing kernels; created on first use, default priority
  hipStream_t setup_side = nullptr;
  hipEvent_t setup_fork = nullptr, setup_join = nullptr;
  int nclasses = 0;
  ~pmgw_plan_s() {
    for (hipEvent_t e : ev0) (void)hipEventDestroy(e);
    for (hipEvent_t e : ev1) (void)hipEventDestroy(e);
    for (int g = 0; g < 15; ++g) {
      if (side[g]) (void)hipStreamDestroy(side[g]);
      if (join[g]) (void)hipEventDestroy(join[g]);
    }
    if (fork) (void)hipEventDestroy(fork);
    if (setup_fork) (void)hipEventDestroy(setup_fork);
    if (setup_join) (void)hipEventDestroy(setup_join);
    if (setup_side) (void)hipStreamDestroy(setup_side);
  }
};

namespace {

template <typename T>
void put(std::vector<char>& img, int64_t off, const std::vector<double>& v) {
  T* p = reinterpret_cast<T*>(img.data() + off);
  for (size_t i = 0; i < v.size(); ++i) p[i] = (T)v[i];
}

bool valid_m(int M) { return M == 2 || M == 4 || M == 8 || M == 16 || M == 32; }

int check_plan(pmgw_plan p) {
  if (!p) return fail(PMGW_EINVAL, "plan is NULL");
  if (!p->ws) return fail(PMGW_EWORKSPACE, "no workspace bound");
  return PMGW_OK;
}

KOpts kopts(const pmgw_plan_s* p) {
  KOpts o;
  o.nu1 = p->opts.nu1;
  o.nu2 = p->opts.nu2;
  o.coarse_pairs = p->opts.coarse_pairs;
  o.restart = p->opts.restart;
  o.omega_c = p->opts.omega_c;
  o.omega_m = p->opts.omega_m;
  o.adapt = p->opts.adapt_omega_m;
  o.cycle = p->opts.cycle;
  o.coarse_exact = p->opts.coarse_exact;
  o.bed_line = p->opts.bed_line;
  return o;
}

// Dynamic LDS of a launch that runs FFTs: two FFT halves of fftb bytes, then the float64 and
// float32 twiddle tables of the largest Nx.
size_t lds_bytes(int fftb, int maxnx) { return (size_t)(2 * fftb) + (size_t)24 * maxnx; }

int nz_class(int nz) { return nz == 3 ? 0 : nz == 5 ? 1 : nz == 9 ? 2 : nz == 17 ? 3 : 4; }

// Bytes of one FFT half for a solve launch. Classes whose rows all go through the wavefront FFT
// (64 <= Nx <= 512) get what kWaveRows row pairs per wavefront need (2 fftb = wavefronts x
// kWaveRows x Nx complex float64), so that with fewer threads per workgroup two workgroups fit in
// one CU's LDS; other classes get 32 KB halves for the workgroup-wide FFT.
int solve_fftb(int threads, int maxnx) {
  if (maxnx >= 64 && maxnx <= 512) {
    const int need = (threads / 64) * kWaveRows * maxnx * 16 / 2;
    return std::max(4096, std::min(32768, need));
  }
  return 32768;
}

// LDS bytes that the resident V-cycle of a tank needs beside the Krylov state: its map, the two
// twiddle tables and the solve kernel's static LDS.
int64_t resident_lds(int nz, int nx) {
  return res_map_bytes(nz, nx) + 24LL * nx + (int64_t)sizeof(KrylovLds);
}
constexpr int64_t kLdsPerWorkgroup = 163840;

struct GroupView {
  int64_t off;
  unsigned count;
  int maxnx;
};

GroupView group_view(const pmgw_plan_s* p, int g) {
  const int c = g / 3, k = g % 3;
  if (k == 1) return {p->rids_off[c], (unsigned)p->rids[c].size(), p->rmaxnx[c]};
  if (k == 2) return {p->xids_off[c], (unsigned)p->xids[c].size(), p->xmaxnx[c]};
  return {p->ids_off[c], (unsigned)p->ids[c].size(), p->maxnx[c]};
}

template <typename TV, int NZ, bool TR>
void launch_group(pmgw_plan p, int g, int mode, const double* in, double* out, double rtol,
                  int maxit, pmgw_info_dev* info, const KOpts& o, hipStream_t st) {
  const GroupView v = group_view(p, g);
  SolveArgs a;
  a.descs = reinterpret_cast<const TankDesc*>(p->ws + p->desc_off);
  a.ids = reinterpret_cast<const int32_t*>(p->ws + v.off);
  a.ws = p->ws;
  a.mode = mode;
  a.in = in;
  a.out = out;
  a.rtol = rtol;
  a.maxit = maxit;
  a.info = info;
  a.o = o;
  const int cls = p->opts.class_threads[g / 3];
  int thr = cls ? cls : (p->opts.threads ? p->opts.threads : 256);
  if constexpr (std::is_same<TV, float>::value && !TR && NZ <= kResMaxNz) {
    if (g % 3 == 1) {
      // the resident map lives in the first 2 fftb bytes, before the twiddles
      thr = std::min(thr, 256);
      const int64_t half = (p->rres[g / 3] + 511) / 512 * 256;
      a.fftb = (int)std::max<int64_t>(solve_fftb(thr, v.maxnx), half);
      launch_k_solve_res<NZ>(v.count, thr, lds_bytes(a.fftb, v.maxnx), st, a);
      return;
    }
  }
  if constexpr (TR) thr = std::min(thr, 256);
  a.fftb = solve_fftb(thr, v.maxnx);
  if (!TR && thr > 256)
    launch_k_solve_wide<TV, NZ>(v.count, thr, lds_bytes(a.fftb, v.maxnx), st, a);
  else
    launch_k_solve<TV, NZ, TR>(v.count, thr, lds_bytes(a.fftb, v.maxnx), st, a);
}

// Creates the set-up stream of rk4_stage and its fork/join events once.
int ensure_setup_stream(pmgw_plan p) {
  if (p->setup_side) return PMGW_OK;
  hipError_t e = hipEventCreateWithFlags(&p->setup_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->setup_join, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->setup_side, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "creating the set-up stream");
  return PMGW_OK;
}

// Creates the side streams and fork/join events once (only plans with several launch groups).
int ensure_side_streams(pmgw_plan p) {
  if (p->fork) return PMGW_OK;
  hipError_t e = hipEventCreateWithFlags(&p->fork, hipEventDisableTiming);
  for (int g = 0; g < 15 && e == hipSuccess; ++g) {
    if (group_view(p, g).count == 0) continue;
    e = hipStreamCreateWithFlags(&p->side[g], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->join[g], hipEventDisableTiming);
  }
  if (e != hipSuccess) return hip_fail(e, "creating side streams");
  return PMGW_OK;
}

// One solve-kernel launch per group of tanks: per Nz class, and for mixed-precision V-cycles per
// part of a class (LDS-resident cycle or global-memory cycle). With several groups the launches go
// to side streams that wait on an event recorded on the plan's stream and are joined back into
// it, so that the groups run concurrently (a 512-tank batch has three classes); the order seen by
// later work on the plan's stream is unchanged, and the fork/join pattern is valid under graph
// capture.
template <typename TV, bool TR>
int launch_all(pmgw_plan p, int mode, const double* in, double* out, double rtol, int maxit,
               pmgw_info_dev* info, const KOpts& o) {
  const bool split = std::is_same<TV, float>::value && !TR && o.cycle == PMGW_CYCLE_V &&
                     (mode == MODE_SOLVE || mode == MODE_VCYCLE);
  // heaviest groups first (more rows, then the global-memory part of a class, whose tanks are
  // the wider ones): the dispatcher places the workgroups of earlier launches first, so the
  // longest solves of a batch start at once instead of waiting for CUs behind short ones
  int gl[15], ng = 0;
  for (int c = 4; c >= 0; --c) {
    if (split && !p->rids[c].empty()) {
      if (!p->xids[c].empty()) gl[ng++] = 3 * c + 2;
      gl[ng++] = 3 * c + 1;
    } else if (!p->ids[c].empty()) {
      gl[ng++] = 3 * c;
    }
  }
  const bool multi = ng > 1 && !p->serial;
  if (multi) {
    int rc = ensure_side_streams(p);
    if (rc) return rc;
    hipError_t e = hipEventRecord(p->fork, p->stream);
    if (e != hipSuccess) return hip_fail(e, "fork event");
  }
  for (int q = 0; q < ng; ++q) {
    const int g = gl[q];
    hipStream_t st = p->stream;
    if (multi) {
      st = p->side[g];
      hipError_t e = hipStreamWaitEvent(st, p->fork, 0);
      if (e != hipSuccess) return hip_fail(e, "side stream wait");
    }
    switch (g / 3) {
      case 0: launch_group<TV, 3, TR>(p, g, mode, in, out, rtol, maxit, info, o, st); break;
      case 1: launch_group<TV, 5, TR>(p, g, mode, in, out, rtol, maxit, info, o, st); break;
      case 2: launch_group<TV, 9, TR>(p, g, mode, in, out, rtol, maxit, info, o, st); break;
      case 3: launch_group<TV, 17, TR>(p, g, mode, in, out, rtol, maxit, info, o, st); break;
      default: launch_group<TV, 33, TR>(p, g, mode, in, out, rtol, maxit, info, o, st); break;
    }
    if (multi) {
      hipError_t e = hipEventRecord(p->join[g], st);
      if (e == hipSuccess) e = hipStreamWaitEvent(p->stream, p->join[g], 0);
      if (e != hipSuccess) return hip_fail(e, "join event");
    }
  }
  return PMGW_OK;
}

// tr: the transposed operator and cycle (adjoint solves).
int launch_solve(pmgw_plan p, int mode, const double* in, double* out, double rtol, int maxit,
                 pmgw_info_dev* info, bool tr = false) {
  const KOpts o = kopts(p);
  const bool timed = p->prof_on && mode == MODE_SOLVE && !tr && p->prof_n < (int)p->ev0.size();
  if (timed) (void)hipEventRecord(p->ev0[p->prof_n], p->stream);
  int rc;
  if (p->prec == PMGW_FP64)
    rc = tr ? launch_all<double, true>(p, mode, in, out, rtol, maxit, info, o)
            : launch_all<double, false>(p, mode, in, out, rtol, maxit, info, o);
  else
    rc = tr ? launch_all<float, true>(p, mode, in, out, rtol, maxit, info, o)
            : launch_all<float, false>(p, mode, in, out, rtol, maxit, info, o);
  if (rc) return rc;
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "solve kernel launch");
  if (timed) (void)hipEventRecord(p->ev1[p->prof_n++], p->stream);
  return PMGW_OK;
}

}  // namespace

// Internal hooks used by the RK stage (pmgw_rk.hpp) and the adjoint.
int pmgw_internal_solve(pmgw_plan p, const double* b, double* x, double rtol, int maxit,
                        pmgw_info_dev* info) {
  return launch_solve(p, MODE_SOLVE, b, x, rtol, maxit, info);
}

extern "C" {

void pmgw_default_opts(pmgw_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->nu1 = 1;
  o->nu2 = 1;
  o->coarse_pairs = 1;
  o->restart = 30;
  o->omega_c = 1.0;
  o->omega_m = 1.0;
  o->rho = 1000.0;
  o->g = 9.81;
  o->nu_visc = 1e-6;
  o->filt_alpha = 36.0;
  o->filt_s = 2.0;
  o->filt_fx = 0.5;
  o->filt_fz = 0.9;
  o->threads = 0;
  o->adapt_omega_m = 1;
  o->cycle = PMGW_CYCLE_V;
  o->resident = 1;
}

const char* pmgw_last_error(void) { return g_err.c_str(); }

int pmgw_plan_create(pmgw_plan* out, int32_t ntanks, const int32_t* nx, const int32_t* nz,
                     const double* L, int32_t precision, const pmgw_opts* opts, void* stream) {
  g_err.clear();
  if (!out) return fail(PMGW_EINVAL, "out is NULL");
  *out = nullptr;
  if (ntanks < 1 || ntanks > 65536) return fail(PMGW_EINVAL, "ntanks must be in [1, 65536]");
  if (!nx || !nz || !L) return fail(PMGW_EINVAL, "nx, nz and L must be non-NULL");
  if (precision != PMGW_FP64 && precision != PMGW_MIXED)
    return fail(PMGW_EINVAL, "precision must be PMGW_FP64 or PMGW_MIXED");
  pmgw_opts o;
  pmgw_default_opts(&o);
  if (opts) o = *opts;
  if (o.nu1 < 0 || o.nu2 < 0 || o.coarse_pairs < 0 || o.nu1 > 8 || o.nu2 > 8 ||
      o.coarse_pairs > 64)
    return fail(PMGW_EINVAL, "smoothing counts out of range");
  if (!(o.rho > 0.0) || !(o.g >= 0.0) || !(o.nu_visc >= 0.0) || !(o.filt_alpha >= 0.0) ||
      !(o.filt_s > 0.0) || !(o.filt_fx >= 0.0 && o.filt_fx <= 1.0) ||
      !(o.filt_fz >= 0.0 && o.filt_fz <= 1.0))
    return fail(PMGW_EINVAL, "physical or filter options out of range");
  if (o.restart < 1 || o.restart > kMaxRestart)
    return fail(PMGW_EINVAL, "restart must be in [1, 32]");
  if (!(o.omega_c > 0.0 && o.omega_c < 2.0) || !(o.omega_m > 0.0 && o.omega_m < 2.0))
    return fail(PMGW_EINVAL, "damping factors must be in (0, 2)");
  auto thr_ok = [](int t) { return t == 0 || t == 64 || t == 128 || t == 256 || t == 512; };
  if (!thr_ok(o.threads)) return fail(PMGW_EINVAL, "threads must be 0, 64, 128, 256 or 512");
  for (int c = 0; c < 5; ++c) {
    if (!thr_ok(o.class_threads[c]))
      return fail(PMGW_EINVAL, "class_threads must be 0, 64, 128, 256 or 512");
    if (o.class_resident[c] < 0 || o.class_resident[c] > 2)
      return fail(PMGW_EINVAL, "class_resident must be 0, 1 or 2");
  }
  if (o.adapt_omega_m != 0 && o.adapt_omega_m != 1)
    return fail(PMGW_EINVAL, "adapt_omega_m must be 0 or 1");
  if (o.cycle != PMGW_CYCLE_V && o.cycle != PMGW_CYCLE_FMG)
    return fail(PMGW_EINVAL, "cycle must be PMGW_CYCLE_V or PMGW_CYCLE_FMG");
  if (o.coarse_exact != 0 && o.coarse_exact != 1)
    return fail(PMGW_EINVAL, "coarse_exact must be 0 or 1");
  if (o.bed_line != 0 && o.bed_line != 1) return fail(PMGW_EINVAL, "bed_line must be 0 or 1");
  if (o.linear != 0 && o.linear != 1) return fail(PMGW_EINVAL, "linear must be 0 or 1");
  if (o.no_slip != 0 && o.no_slip != 1) return fail(PMGW_EINVAL, "no_slip must be 0 or 1");
  if (o.guess_steps != 0 && (o.guess_steps < 2 || o.guess_steps > 5))
    return fail(PMGW_EINVAL, "guess_steps must be 0 or in 2..5");
  if (o.guess_correct != 0 && o.guess_correct != 1)
    return fail(PMGW_EINVAL, "guess_correct must be 0 or 1");
  if (o.guess_correct && !o.guess_steps)
    return fail(PMGW_EINVAL, "guess_correct needs guess_steps");
  if (o.resident != 0 && o.resident != 1) return fail(PMGW_EINVAL, "resident must be 0 or 1");
  for (int t = 0; t < ntanks; ++t) {
    const int n = nx[t], M = nz[t] - 1;
    if (n < 8 || n > 2048 || (n & (n - 1)) != 0)
      return fail(PMGW_EINVAL, "tank " + std::to_string(t) + ": Nx must be a power of two in [8, 2048]");
    if (!valid_m(M))
      return fail(PMGW_EINVAL, "tank " + std::to_string(t) + ": Nz must be 3, 5, 9, 17 or 33");
    if (n < 2 * M) return fail(PMGW_EINVAL, "tank " + std::to_string(t) + ": Nx must be >= 2 (Nz - 1)");
    if (o.coarse_exact && n > kCoarseExactMaxNx)
      return fail(PMGW_EINVAL, "tank " + std::to_string(t) +
                                   ": the direct coarsest solve needs Nx <= 512");
    if (o.bed_line && n > kBedLineMaxNx)
      return fail(PMGW_EINVAL, "tank " + std::to_string(t) + ": the bed-line step needs Nx <= 1024");
    if (!(L[t] > 0.0) || !std::isfinite(L[t]))
      return fail(PMGW_EINVAL, "tank " + std::to_string(t) + ": L must be positive and finite");
  }

  auto* p = new pmgw_plan_s();
  p->ntanks = ntanks;
  p->prec = precision;
  p->opts = o;
  p->stream = reinterpret_cast<hipStream_t>(stream);
  if (hipGetDevice(&p->device) != hipSuccess) p->device = 0;
  p->threads = o.threads;
  p->gen = g_plan_gen.fetch_add(1) + 1;
  const int vb = precision == PMGW_FP64 ? 8 : 4;   // V-cycle word size
  const int m = o.restart;

  // pass 1: offsets
  int64_t cur = 0;
  p->desc_off = cur;
  cur = align256(cur + (int64_t)sizeof(TankDesc) * ntanks);
  int njobs = 0;
  for (int t = 0; t < ntanks; ++t) {
    int M = nz[t] - 1, nl = 0;
    while (true) { ++nl; if (M == 2) break; M /= 2; }
    njobs += 2 * nl;
  }
  p->job_off = cur;
  cur = align256(cur + (int64_t)sizeof(BlockJob) * njobs);
  p->info_off = cur;
  cur = align256(cur + (int64_t)sizeof(pmgw_info) * ntanks);
  for (int t = 0; t < ntanks; ++t) {
    const int c = nz_class(nz[t]);
    p->ids[c].push_back(t);
    p->maxnx[c] = std::max(p->maxnx[c], (int)nx[t]);
    p->maxnx_all = std::max(p->maxnx_all, (int)nx[t]);
  }
  for (int c = 0; c < 5; ++c) {
    // largest tanks first: the hardware dispatches workgroups in order, so the longest solves
    // start earliest
    std::stable_sort(p->ids[c].begin(), p->ids[c].end(),
                     [&](int32_t a, int32_t b) { return nx[a] > nx[b]; });
    if (!p->ids[c].empty()) ++p->nclasses;
    p->ids_off[c] = cur;
    cur = align256(cur + 4 * (int64_t)p->ids[c].size());
    for (int32_t t : p->ids[c]) {
      const int tnz = nz[t], tnx = nx[t];
      const bool want = o.class_resident[c] == 0 ? o.resident != 0 : o.class_resident[c] == 1;
      const bool res = precision == PMGW_MIXED && want && !o.bed_line && tnz <= kResMaxNz &&
                       tnx >= 64 &&
                       tnx <= 512 && resident_lds(tnz, tnx) <= kLdsPerWorkgroup;
      if (res) {
        p->rids[c].push_back(t);
        p->rmaxnx[c] = std::max(p->rmaxnx[c], tnx);
        p->rres[c] = std::max<int64_t>(p->rres[c], res_map_bytes(tnz, tnx));
      } else {
        p->xids[c].push_back(t);
        p->xmaxnx[c] = std::max(p->xmaxnx[c], tnx);
      }
    }
    p->rids_off[c] = cur;
    cur = align256(cur + 4 * (int64_t)p->rids[c].size());
    p->xids_off[c] = cur;
    cur = align256(cur + 4 * (int64_t)p->xids[c].size());
  }
  p->tanks.resize(ntanks);
  p->off2d.assign(ntanks + 1, 0);
  p->off1d.assign(ntanks + 1, 0);
  // constant tables first (contiguous, copied at bind), then mutable arrays
  for (int t = 0; t < ntanks; ++t) {
    TankDesc& d = p->tanks[t];
    std::memset(&d, 0, sizeof(d));
    d.nx = nx[t];
    d.nz = nz[t];
    d.log2nx = ilog2(nx[t]);
    d.L = L[t];
    d.kfac = 2.0 * M_PI / L[t];
    const double K = nx[t] / 2 - 1;
    d.cxx = -(d.kfac * d.kfac / nx[t]) * 2.0 * (K * (K + 1.0) * (2.0 * K + 1.0) / 6.0);
    d.off2d = p->off2d[t];
    d.off1d = p->off1d[t];
    p->off2d[t + 1] = p->off2d[t] + (int64_t)nx[t] * nz[t];
    p->off1d[t + 1] = p->off1d[t] + nx[t];
    int M = nz[t] - 1, l = 0;
    while (true) {
      LevelDesc& lv = d.lev[l];
      lv.nz = M + 1;
      lv.nzc = (M > 2) ? M / 2 + 1 : 0;
      lv.dss = cur; cur = align256(cur + 16LL * lv.nz * lv.nz);
      for (int pr = 0; pr < 2; ++pr) {
        const int64_t w = pr == 0 ? 8 : 4;
        lv.ds[pr] = cur; cur = align256(cur + w * lv.nz * lv.nz);
        lv.sig[pr] = cur; cur = align256(cur + w * lv.nz);
        if (lv.nzc) {
          lv.R[pr] = cur; cur = align256(cur + w * lv.nzc * lv.nz);
          lv.P[pr] = cur; cur = align256(cur + w * lv.nz * lv.nzc);
          lv.PT[pr] = cur; cur = align256(cur + w * lv.nzc * lv.nz);
          lv.RT[pr] = cur; cur = align256(cur + w * lv.nz * lv.nzc);
        }
      }
      ++l;
      if (M == 2) break;
      M /= 2;
    }
    d.nlev = l;
    d.tw[0] = cur; cur = align256(cur + 16LL * nx[t]);
    d.tw[1] = cur; cur = align256(cur + 8LL * nx[t]);
    d.filtx = cur; cur = align256(cur + 8LL * (nx[t] / 2 + 1));
    d.filtz = cur; cur = align256(cur + 8LL * nz[t] * nz[t]);
  }
  const int64_t const_end = cur;
  for (int t = 0; t < ntanks; ++t) {
    TankDesc& d = p->tanks[t];
    const int64_t n = (int64_t)d.nx * d.nz;
    d.geo64 = cur; cur = align256(cur + 8LL * 10 * d.nx);
    d.geo32 = cur; cur = align256(cur + 4LL * 7 * d.nx);
    d.scal = cur; cur = align256(cur + 64);
    d.V = cur; cur = align256(cur + 8LL * (m + 1) * n);
    d.Z = cur; cur = align256(cur + 8LL * m * n);
    d.a1 = cur; cur = align256(cur + 8LL * n);
    d.a2 = cur; cur = align256(cur + 8LL * n);
    d.a3 = cur; cur = align256(cur + 8LL * n);
    d.aspec = cur; cur = align256(cur + 16LL * ((d.nz + 1) / 2) * d.nx);
    if (o.coarse_exact) {
      d.cw = cur; cur = align256(cur + 8LL * 6 * d.nx * d.nx);
      d.cwt = cur; cur = align256(cur + 8LL * 6 * d.nx * d.nx);
    }
    for (int l = 0; l < d.nlev; ++l) {
      LevelDesc& lv = d.lev[l];
      const int64_t nl = (int64_t)lv.nz * d.nx;
      lv.colinv = cur; cur = align256(cur + vb * (int64_t)lv.nz * lv.nz * d.nx);
      lv.modeinv = cur; cur = align256(cur + vb * (int64_t)lv.nz * lv.nz * (d.nx / 2 + 1));
      lv.x = cur; cur = align256(cur + vb * nl);
      lv.u = cur; cur = align256(cur + vb * nl);
      lv.f = cur; cur = align256(cur + vb * nl);
      lv.r = cur; cur = align256(cur + vb * nl);
      lv.t1 = cur; cur = align256(cur + vb * nl);
      lv.t2 = cur; cur = align256(cur + vb * nl);
      lv.t3 = cur; cur = align256(cur + vb * nl);
      lv.spec = cur; cur = align256(cur + 2LL * vb * ((lv.nz + 1) / 2) * d.nx);
      if (o.bed_line) {
        lv.bedinv = cur; cur = align256(cur + 8LL * d.nx * d.nx);
        if (precision == PMGW_MIXED) {
          lv.bedinv32 = cur; cur = align256(cur + 4LL * d.nx * d.nx);
        }
      }
    }
  }
  p->rk_off = cur;
  cur = align256(cur + rk_workspace_bytes(p->off2d[ntanks], p->off1d[ntanks]));
  p->adj_off = cur;
  cur = align256(cur + adj_workspace_bytes(p->off2d[ntanks], p->off1d[ntanks]));
  if (o.guess_steps > 0) {
    p->hist_off = cur;
    cur = align256(cur + 8LL * 5 * o.guess_steps * p->off2d[ntanks]);
  }
  if (o.guess_correct) {
    p->eprev_off = cur;
    cur = align256(cur + 8LL * p->off2d[ntanks]);
  }
  p->total = cur;

  // block-inversion jobs
  int64_t first = 0;
  for (int t = 0; t < ntanks; ++t) {
    const TankDesc& d = p->tanks[t];
    for (int l = 0; l < d.nlev; ++l) {
      p->jobs.push_back(BlockJob{t, l, 0, d.nx, first});
      first += d.nx;
      p->jobs.push_back(BlockJob{t, l, 1, d.nx / 2 + 1, first});
      first += d.nx / 2 + 1;
    }
  }
  p->nblocks = first;
  if (p->nblocks > 0x7fffffffLL) {
    delete p;
    return fail(PMGW_EINVAL, "too many blocks for one launch");
  }

  // pass 2: constant image
  p->image.assign(const_end, 0);
  std::memcpy(p->image.data() + p->desc_off, p->tanks.data(), sizeof(TankDesc) * ntanks);
  std::memcpy(p->image.data() + p->job_off, p->jobs.data(), sizeof(BlockJob) * p->jobs.size());
  for (int c = 0; c < 5; ++c) {
    if (!p->ids[c].empty())
      std::memcpy(p->image.data() + p->ids_off[c], p->ids[c].data(), 4 * p->ids[c].size());
    if (!p->rids[c].empty())
      std::memcpy(p->image.data() + p->rids_off[c], p->rids[c].data(), 4 * p->rids[c].size());
    if (!p->xids[c].empty())
      std::memcpy(p->image.data() + p->xids_off[c], p->xids[c].data(), 4 * p->xids[c].size());
  }
  for (int t = 0; t < ntanks; ++t) {
    const TankDesc& d = p->tanks[t];
    for (int l = 0; l < d.nlev; ++l) {
      const LevelDesc& lv = d.lev[l];
      const int M = lv.nz - 1;
      const auto D = dsigma(M);
      const auto s = cgl_sigma(M);
      put<double>(p->image, lv.ds[0], D);
      put<float>(p->image, lv.ds[1], D);
      put<double>(p->image, lv.sig[0], s);
      put<float>(p->image, lv.sig[1], s);
      const int nz = lv.nz;
      std::vector<double> dss(2 * nz * nz, 0.0);
      for (int j = 0; j < nz; ++j)
        for (int c = 0; c < nz; ++c) {
          double a = 0.0, b = 0.0;
          for (int m = 0; m < nz; ++m) {
            a += D[j * nz + m] * D[m * nz + c];
            b += D[j * nz + m] * s[m] * D[m * nz + c];
          }
          dss[j * nz + c] = a;
          dss[nz * nz + j * nz + c] = b;
        }
      put<double>(p->image, lv.dss, dss);
      if (lv.nzc) {
        const auto R = restriction(M);
        const auto P = prolongation(M);
        put<double>(p->image, lv.R[0], R);
        put<float>(p->image, lv.R[1], R);
        put<double>(p->image, lv.P[0], P);
        put<float>(p->image, lv.P[1], P);
        const auto PT = transpose(P, lv.nz, lv.nzc);
        const auto RT = transpose(R, lv.nzc, lv.nz);
        put<double>(p->image, lv.PT[0], PT);
        put<float>(p->image, lv.PT[1], PT);
        put<double>(p->image, lv.RT[0], RT);
        put<float>(p->image, lv.RT[1], RT);
      }
    }
    std::vector<double> tw(2 * d.nx);
    for (int k = 0; k < d.nx; ++k) {
      const long double a = -2.0L * (long double)M_PI * k / d.nx;
      tw[2 * k] = (double)std::cos(a);
      tw[2 * k + 1] = (double)std::sin(a);
    }
    put<double>(p->image, d.tw[0], tw);
    put<float>(p->image, d.tw[1], tw);
    std::vector<double> fx(d.nx / 2 + 1);
    const int Nc = (int)std::floor(o.filt_fx * (d.nx / 2));
    for (int k = 0; k <= d.nx / 2; ++k)
      fx[k] = filter_factor(k, d.nx / 2, Nc, o.filt_alpha, o.filt_s);
    put<double>(p->image, d.filtx, fx);
    put<double>(p->image, d.filtz, sigma_filter(d.nz - 1, o.filt_fz, o.filt_alpha, o.filt_s));
  }
  *out = p;
  return PMGW_OK;
}

size_t pmgw_workspace_bytes(pmgw_plan p) { return p ? (size_t)p->total : 0; }

int pmgw_bind_workspace(pmgw_plan p, void* dev, size_t bytes) {
  g_err.clear();
  if (!p) return fail(PMGW_EINVAL, "plan is NULL");
  if (!dev) return fail(PMGW_EWORKSPACE, "workspace pointer is NULL");
  if ((reinterpret_cast<uintptr_t>(dev) & 255) != 0)
    return fail(PMGW_EWORKSPACE, "workspace must be 256-byte aligned");
  if ((int64_t)bytes < p->total)
    return fail(PMGW_EWORKSPACE, "workspace too small: need " + std::to_string(p->total) + " bytes");
  hipError_t e = hipMemcpy(dev, p->image.data(), p->image.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy of constant tables");
  p->ws = reinterpret_cast<char*>(dev);
  p->geometry_set = false;
  return PMGW_OK;
}

int pmgw_field_offsets(pmgw_plan p, int64_t* off2d, int64_t* off1d) {
  if (!p) return fail(PMGW_EINVAL, "plan is NULL");
  if (off2d) std::memcpy(off2d, p->off2d.data(), sizeof(int64_t) * (p->ntanks + 1));
  if (off1d) std::memcpy(off1d, p->off1d.data(), sizeof(int64_t) * (p->ntanks + 1));
  return PMGW_OK;
}

}  // extern "C"

namespace {

// sigma-metrics of both geometries (k_geometry) on stream st.
int geometry_kernel(pmgw_plan p, const double* h, const double* eo, const double* en,
                    hipStream_t st) {
  const TankDesc* d = reinterpret_cast<const TankDesc*>(p->ws + p->desc_off);
  hipLaunchKernelGGL(k_geometry, dim3(p->ntanks), dim3(256), lds_bytes(kGeoFftBytes, p->maxnx_all),
                     st, d, p->ws, h, eo, en);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "geometry kernel launch");
  return PMGW_OK;
}

// The surface part of a stage and the metrics of its two geometries (k_rk_pre_geometry), on the
// plan's stream.
int pre_geometry_kernel(pmgw_plan p, const RkCoef& cf, const double* h, const double* u,
                        const double* w, double* eta, double* Keta, const RkBufs& rb) {
  const TankDesc* d = reinterpret_cast<const TankDesc*>(p->ws + p->desc_off);
  hipLaunchKernelGGL(k_rk_pre_geometry, dim3(p->ntanks), dim3(256),
                     lds_bytes(kGeoFftBytes, p->maxnx_all), p->stream, d, p->ws, cf, h, u, w, eta,
                     Keta, rb);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "stage surface kernel launch");
  return PMGW_OK;
}

// The smoother's set-up from the metrics: block inverses, and the bed-line and direct coarse
// solve set-ups when enabled, on stream st.
int setup_kernels(pmgw_plan p, hipStream_t st) {
  const TankDesc* d = reinterpret_cast<const TankDesc*>(p->ws + p->desc_off);
  const BlockJob* j = reinterpret_cast<const BlockJob*>(p->ws + p->job_off);
  if (p->prec == PMGW_FP64)
    hipLaunchKernelGGL(k_blocks<double>, dim3((unsigned)p->nblocks), dim3(64), 0, st, d, j,
                       (int)p->jobs.size(), p->ws);
  else
    hipLaunchKernelGGL(k_blocks<float>, dim3((unsigned)p->nblocks), dim3(64), 0, st, d, j,
                       (int)p->jobs.size(), p->ws);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "block kernel launch");
  if (p->opts.bed_line) {
    hipLaunchKernelGGL(k_bedline_setup, dim3(p->ntanks, kMaxLev), dim3(kBedLineThreads),
                       lds_bytes(kGeoFftBytes, p->maxnx_all), st, d, p->ws);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "bed-line set-up kernel launch");
  }
  if (p->opts.coarse_exact) {
    hipLaunchKernelGGL(k_coarse_setup, dim3(p->ntanks), dim3(kCoarseThreads),
                       lds_bytes(kGeoFftBytes, p->maxnx_all), st, d, p->ws);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "coarse set-up kernel launch");
  }
  return PMGW_OK;
}

}  // namespace

extern "C" {

int pmgw_set_geometry(pmgw_plan p, const double* h, const double* eo, const double* en) {
  g_err.clear();
  int rc = check_plan(p);
  if (rc) return rc;
  if (!h || !eo || !en) return fail(PMGW_EINVAL, "h, eta_old and eta_new must be non-NULL");
  if ((rc = geometry_kernel(p, h, eo, en, p->stream))) return rc;
  if ((rc = setup_kernels(p, p->stream))) return rc;
  p->geometry_set = true;
  return PMGW_OK;
}

int laplacian_apply(pmgw_plan p, const double* in, double* out) {
  g_err.clear();
  int rc = check_plan(p);
  if (rc) return rc;
  if (!p->geometry_set) return fail(PMGW_EINVAL, "geometry not set");
  if (!in || !out) return fail(PMGW_EINVAL, "p and Ap must be non-NULL");
  if (in == out) return fail(PMGW_EINVAL, "p and Ap must not overlap");
  return launch_solve(p, MODE_APPLY, in, out, 0.0, 0, nullptr);
}

int pmg_vcycle(pmgw_plan p, const double* r, double* z) {
  g_err.clear();
  int rc = check_plan(p);
  if (rc) return rc;
  if (!p->geometry_set) return fail(PMGW_EINVAL, "geometry not set");
  if (!r || !z) return fail(PMGW_EINVAL, "r and z must be non-NULL");
  if (r == z) return fail(PMGW_EINVAL, "r and z must not overlap");
  return launch_solve(p, MODE_VCYCLE, r, z, 0.0, 0, nullptr);
}

}  // extern "C"

namespace {

int solve_entry(pmgw_plan p, bool tr, const double* b, double* x, double rtol, int32_t maxit,
                pmgw_info* info_host, pmgw_info* info_dev) {
  int rc = check_plan(p);
  if (rc) return rc;
  if (!p->geometry_set) return fail(PMGW_EINVAL, "geometry not set");
  if (!b || !x) return fail(PMGW_EINVAL, "b and p must be non-NULL");
  if (b == x) return fail(PMGW_EINVAL, "b and p must not overlap");
  if (!(rtol > 0.0) || !std::isfinite(rtol)) return fail(PMGW_EINVAL, "rtol must be positive");
  if (maxit < 1) return fail(PMGW_EINVAL, "maxit must be >= 1");
  pmgw_info_dev* dinfo = info_dev ? reinterpret_cast<pmgw_info_dev*>(info_dev)
                                  : reinterpret_cast<pmgw_info_dev*>(p->ws + p->info_off);
  rc = launch_solve(p, MODE_SOLVE, b, x, rtol, maxit, dinfo, tr);
  if (rc) return rc;
  if (info_host) {
    hipError_t e = hipMemcpyAsync(info_host, dinfo, sizeof(pmgw_info) * p->ntanks,
                                  hipMemcpyDeviceToHost, p->stream);
    if (e != hipSuccess) return hip_fail(e, "info copy");
    e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "stream synchronize");
    int worst = PMGW_OK;
    for (int t = 0; t < p->ntanks; ++t) {
      const int s = info_host[t].status;
      if (s < 0 && (worst >= 0 || s < worst)) worst = s;
      else if (s > 0 && worst == PMGW_OK) worst = s;
    }
    if (worst < 0) return fail(worst, "a tank failed (see info)");
    if (worst > 0) g_err = "a tank did not converge (see info)";
    return worst;
  }
  return PMGW_OK;
}

}  // namespace

extern "C" {

int poisson_solve(pmgw_plan p, const double* b, double* x, double rtol, int32_t maxit,
                  pmgw_info* info_host, pmgw_info* info_dev) {
  g_err.clear();
  return solve_entry(p, false, b, x, rtol, maxit, info_host, info_dev);
}

int pmgw_fmg(pmgw_plan p, const double* r, double* z) {
  g_err.clear();
  int rc = check_plan(p);
  if (rc) return rc;
  if (!p->geometry_set) return fail(PMGW_EINVAL, "geometry not set");
  if (!r || !z) return fail(PMGW_EINVAL, "r and z must be non-NULL");
  if (r == z) return fail(PMGW_EINVAL, "r and z must not overlap");
  return launch_solve(p, MODE_FMG, r, z, 0.0, 0, nullptr);
}

int pmgw_adjoint_apply(pmgw_plan p, const double* lam, double* out) {
  g_err.clear();
  int rc = check_plan(p);
  if (rc) return rc;
  if (!p->geometry_set) return fail(PMGW_EINVAL, "geometry not set");
  if (!lam || !out) return fail(PMGW_EINVAL, "lambda and out must be non-NULL");
  if (lam == out) return fail(PMGW_EINVAL, "lambda and out must not overlap");
  return launch_solve(p, MODE_APPLY, lam, out, 0.0, 0, nullptr, true);
}

int pmgw_adjoint_vcycle(pmgw_plan p, const double* r, double* z) {
  g_err.clear();
  int rc = check_plan(p);
  if (rc) return rc;
  if (!p->geometry_set) return fail(PMGW_EINVAL, "geometry not set");
  if (!r || !z) return fail(PMGW_EINVAL, "r and z must be non-NULL");
  if (r == z) return fail(PMGW_EINVAL, "r and z must not overlap");
  return launch_solve(p, MODE_VCYCLE, r, z, 0.0, 0, nullptr, true);
}

int pmgw_adjoint_solve(pmgw_plan p, const double* g, double* lam, double rtol, int32_t maxit,
                       pmgw_info* info_host, pmgw_info* info_dev) {
  g_err.clear();
  return solve_entry(p, true, g, lam, rtol, maxit, info_host, info_dev);
}

void pmgw_plan_destroy(pmgw_plan p) { delete p; }

int pmgw_profile(pmgw_plan p, int32_t capacity) {
  g_err.clear();
  if (!p) return fail(PMGW_EINVAL, "plan is NULL");
  if (capacity < 0 || capacity > (1 << 20)) return fail(PMGW_EINVAL, "capacity out of range");
  p->prof_on = capacity > 0;
  p->prof_n = 0;
  while ((int)p->ev0.size() < capacity) {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e != hipSuccess) {
      if (a) (void)hipEventDestroy(a);
      p->prof_on = false;
      return hip_fail(e, "hipEventCreate");
    }
    p->ev0.push_back(a);
    p->ev1.push_back(b);
  }
  return PMGW_OK;
}

int pmgw_profile_read(pmgw_plan p, int32_t* launches, double* total_ms, double* max_ms) {
  g_err.clear();
  if (!p || !launches || !total_ms || !max_ms) return fail(PMGW_EINVAL, "NULL argument");
  double tot = 0.0, mx = 0.0;
  for (int i = 0; i < p->prof_n; ++i) {
    hipError_t e = hipEventSynchronize(p->ev1[i]);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, p->ev0[i], p->ev1[i]);
    if (e != hipSuccess) return hip_fail(e, "reading solve timings");
    tot += ms;
    mx = ms > mx ? ms : mx;
  }
  *launches = p->prof_n;
  *total_ms = tot;
  *max_ms = mx;
  return PMGW_OK;
}

}  // extern "C"

namespace {

template <int NZ>
void launch_rk(pmgw_plan p, int c, int which, const RkCoef& cf, const double* u, const double* w,
               double* eta, double* Ku, double* Kw, double* Keta, const double* pr, double* uo,
               double* wo, const RkBufs& rb) {
  RkArgs a;
  a.descs = reinterpret_cast<const TankDesc*>(p->ws + p->desc_off);
  a.ids = reinterpret_cast<const int32_t*>(p->ws + p->ids_off[c]);
  a.ws = p->ws;
  a.cf = cf;
  a.u = u;
  a.w = w;
  a.eta = eta;
  a.Ku = Ku;
  a.Kw = Kw;
  a.Keta = Keta;
  a.pr = pr;
  a.uo = uo;
  a.wo = wo;
  a.rb = rb;
  a.fftb = 32768;
  launch_k_rk<NZ>(which, (unsigned)p->ids[c].size(), lds_bytes(a.fftb, p->maxnx[c]), p->stream, a);
}

int launch_rk_all(pmgw_plan p, int which, const RkCoef& cf, double* u, double* w, double* eta,
                  double* Ku, double* Kw, double* Keta, const double* pr, const RkBufs& rb) {
  if (!p->ids[0].empty()) launch_rk<3>(p, 0, which, cf, u, w, eta, Ku, Kw, Keta, pr, u, w, rb);
  if (!p->ids[1].empty()) launch_rk<5>(p, 1, which, cf, u, w, eta, Ku, Kw, Keta, pr, u, w, rb);
  if (!p->ids[2].empty()) launch_rk<9>(p, 2, which, cf, u, w, eta, Ku, Kw, Keta, pr, u, w, rb);
  if (!p->ids[3].empty()) launch_rk<17>(p, 3, which, cf, u, w, eta, Ku, Kw, Keta, pr, u, w, rb);
  if (!p->ids[4].empty()) launch_rk<33>(p, 4, which, cf, u, w, eta, Ku, Kw, Keta, pr, u, w, rb);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "stage kernel launch");
  return PMGW_OK;
}

}  // namespace

namespace {

// The history step of rk4_stage with opts.guess_steps = m: record the incoming p as the value of
// the previous call's stage, then extrapolate stage k's record into p, with opts.guess_correct
// plus the previous call's extrapolation error (k_guess, one launch).
int stage_guess(pmgw_plan p, int k, double dt, double* pr, hipStream_t st) {
  const int m = p->opts.guess_steps;
  const bool in_order = p->hist_k != 0 && k == p->hist_k % 5 + 1 && dt == p->hist_dt;
  if (!in_order) {
    for (int s = 0; s < 5; ++s) p->hist_cnt[s] = p->hist_head[s] = 0;
    p->hist_eprev = false;
  }
  GuessArgs g{};
  g.store = -1;
  if (in_order) {
    const int s = p->hist_k - 1;
    g.store = s * m + p->hist_head[s];
    p->hist_head[s] = (p->hist_head[s] + 1) % m;
    p->hist_cnt[s] = std::min(p->hist_cnt[s] + 1, m);
  }
  const int s = k - 1, c = p->hist_cnt[s];
  if (c >= 2) {
    g.nsrc = c;
    double binom = 1.0;   // C(c, i), built up over i
    for (int i = 1; i <= c; ++i) {
      binom = binom * (c - i + 1) / i;
      g.src[i - 1] = s * m + (p->hist_head[s] - i + m) % m;
      g.c[i - 1] = (i % 2 == 1 ? 1.0 : -1.0) * binom;
    }
  }
  if (p->opts.guess_correct && g.nsrc > 0) {
    g.eprev = reinterpret_cast<double*>(p->ws + p->eprev_off);
    g.corr = p->hist_eprev ? 1 : 0;
    g.save = 1;
  }
  p->hist_eprev = p->opts.guess_correct && g.nsrc > 0;
  p->hist_k = k;
  p->hist_dt = dt;
  if (g.store < 0 && g.nsrc == 0) return PMGW_OK;
  const int64_t n2d = p->off2d[p->ntanks];
  const int64_t blocks = std::min<int64_t>((n2d + 255) / 256, 4096);
  hipLaunchKernelGGL(k_guess, dim3((unsigned)blocks), dim3(256), 0, st, pr,
                     reinterpret_cast<double*>(p->ws + p->hist_off), n2d, g);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "initial-guess kernel launch");
  return PMGW_OK;
}

}  // namespace

extern "C" int rk4_stage(pmgw_plan p, int32_t k, double dt, const double* h, double* u, double* w,
                         double* eta, double* Ku, double* Kw, double* Keta, double* pr,
                         double rtol, int32_t maxit, pmgw_info* info_dev) {
  g_err.clear();
  int rc = check_plan(p);
  if (rc) return rc;
  if (k < 1 || k > 5) return fail(PMGW_EINVAL, "stage k must be in 1..5");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(PMGW_EINVAL, "dt must be positive");
  if (!h || !u || !w || !eta || !Ku || !Kw || !Keta || !pr)
    return fail(PMGW_EINVAL, "fields must be non-NULL");
  if (!(rtol > 0.0) || !std::isfinite(rtol)) return fail(PMGW_EINVAL, "rtol must be positive");
  if (maxit < 1) return fail(PMGW_EINVAL, "maxit must be >= 1");
  RkCoef cf;
  cf.a = kCkAlpha[k - 1];
  cf.b = kCkBeta[k - 1];
  cf.dt = dt;
  cf.rho = p->opts.rho;
  cf.g = p->opts.g;
  cf.nu = p->opts.nu_visc;
  cf.lin = p->opts.linear;
  cf.noslip = p->opts.no_slip;
  const RkBufs rb = rk_bufs(p->ws + p->rk_off, p->off2d[p->ntanks], p->off1d[p->ntanks]);
  // surface update and the metrics of the old and new surface (the linearised model keeps the
  // still-water geometry)
  if ((rc = pre_geometry_kernel(p, cf, h, u, w, eta, Keta, rb))) return rc;
  // the smoother set-up needs only the metrics: it runs on the set-up stream while the forcing
  // and right-hand-side kernels run here, and is joined before the solve
  if ((rc = ensure_setup_stream(p))) return rc;
  hipError_t e = hipEventRecord(p->setup_fork, p->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(p->setup_side, p->setup_fork, 0);
  if (e != hipSuccess) return hip_fail(e, "set-up fork");
  if ((rc = setup_kernels(p, p->setup_side))) return rc;
  // the initial guess touches only p and its record: it runs on the set-up stream as well
  if (p->opts.guess_steps > 0 && (rc = stage_guess(p, k, dt, pr, p->setup_side))) return rc;
  e = hipEventRecord(p->setup_join, p->setup_side);
  if (e != hipSuccess) return hip_fail(e, "set-up join");
  p->geometry_set = true;
  rc = launch_rk_all(p, 1, cf, u, w, eta, Ku, Kw, Keta, pr, rb);
  if (rc) return rc;
  e = hipStreamWaitEvent(p->stream, p->setup_join, 0);
  if (e != hipSuccess) return hip_fail(e, "set-up join");
  pmgw_info_dev* dinfo = info_dev ? reinterpret_cast<pmgw_info_dev*>(info_dev)
                                  : reinterpret_cast<pmgw_info_dev*>(p->ws + p->info_off);
  rc = launch_solve(p, MODE_SOLVE, rb.b, pr, rtol, maxit, dinfo);
  if (rc) return rc;
  return launch_rk_all(p, 2, cf, u, w, eta, Ku, Kw, Keta, pr, rb);
}

extern "C" int pmgw_stream_target(pmgw_plan p, const double* coef, int32_t nmodes, double t,
                                  double a, const double* window, double* u, double* w,
                                  double* eta) {
  g_err.clear();
  const int rc = check_plan(p);
  if (rc) return rc;
  if (nmodes < 1 || nmodes > kStreamMaxModes)
    return fail(PMGW_EINVAL, "nmodes must be in [1, 64]");
  if (!coef || !window || !u || !w || !eta) return fail(PMGW_EINVAL, "arrays must be non-NULL");
  if (!std::isfinite(t) || !std::isfinite(a)) return fail(PMGW_EINVAL, "t and a must be finite");
  hipLaunchKernelGGL(k_stream_target, dim3((unsigned)p->ntanks, kMaxNz), dim3(256), 0, p->stream,
                     reinterpret_cast<const TankDesc*>(p->ws + p->desc_off), p->ws, coef,
                     (int)nmodes, t, a, window, u, w, eta);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "stream target kernel launch");
  return PMGW_OK;
}

extern "C" int pmgw_relax(pmgw_plan p, const double* r, const double* u_t, const double* w_t,
                          const double* eta_t, double* u, double* w, double* eta) {
  g_err.clear();
  const int rc = check_plan(p);
  if (rc) return rc;
  if (!r || !u_t || !w_t || !eta_t || !u || !w || !eta)
    return fail(PMGW_EINVAL, "arrays must be non-NULL");
  hipLaunchKernelGGL(k_relax, dim3((unsigned)p->ntanks, 16), dim3(256), 0, p->stream,
                     reinterpret_cast<const TankDesc*>(p->ws + p->desc_off), r, u_t, w_t, eta_t,
                     u, w, eta);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "relaxation kernel launch");
  return PMGW_OK;
}

extern "C" int pmgw_history_reset(pmgw_plan p) {
  g_err.clear();
  if (!p) return fail(PMGW_EINVAL, "plan is NULL");
  for (int s = 0; s < 5; ++s) p->hist_cnt[s] = p->hist_head[s] = 0;
  p->hist_k = 0;
  p->hist_eprev = false;
  return PMGW_OK;
}

namespace {

template <int NZ>
void launch_rka(pmgw_plan p, int c, int which, const RkCoef& cf, const double* u,
                const double* w, double* ub, double* wb, double* etab, double* Kub, double* Kwb,
                double* Ketab, double* hbar, const RkBufs& rb, const AdjBufs& ab) {
  RkaArgs a;
  a.descs = reinterpret_cast<const TankDesc*>(p->ws + p->desc_off);
  a.ids = reinterpret_cast<const int32_t*>(p->ws + p->ids_off[c]);
  a.ws = p->ws;
  a.cf = cf;
  a.u = u;
  a.w = w;
  a.ub = ub;
  a.wb = wb;
  a.etab = etab;
  a.Kub = Kub;
  a.Kwb = Kwb;
  a.Ketab = Ketab;
  a.hbar = hbar;
  a.rb = rb;
  a.ab = ab;
  a.fftb = 32768;
  launch_k_rka<NZ>(which, (unsigned)p->ids[c].size(), lds_bytes(a.fftb, p->maxnx[c]), p->stream,
                   a);
}

int launch_rka_all(pmgw_plan p, int which, const RkCoef& cf, const double* u, const double* w,
                   double* ub, double* wb, double* etab, double* Kub, double* Kwb, double* Ketab,
                   double* hbar, const RkBufs& rb, const AdjBufs& ab) {
  if (!p->ids[0].empty()) launch_rka<3>(p, 0, which, cf, u, w, ub, wb, etab, Kub, Kwb, Ketab, hbar, rb, ab);
  if (!p->ids[1].empty()) launch_rka<5>(p, 1, which, cf, u, w, ub, wb, etab, Kub, Kwb, Ketab, hbar, rb, ab);
  if (!p->ids[2].empty()) launch_rka<9>(p, 2, which, cf, u, w, ub, wb, etab, Kub, Kwb, Ketab, hbar, rb, ab);
  if (!p->ids[3].empty()) launch_rka<17>(p, 3, which, cf, u, w, ub, wb, etab, Kub, Kwb, Ketab, hbar, rb, ab);
  if (!p->ids[4].empty()) launch_rka<33>(p, 4, which, cf, u, w, ub, wb, etab, Kub, Kwb, Ketab, hbar, rb, ab);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "adjoint stage kernel launch");
  return PMGW_OK;
}

int fill_zero_dev(pmgw_plan p, double* a, int64_t n) {
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, p->stream, a, n, 0.0);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "fill kernel launch");
  return PMGW_OK;
}

}  // namespace

extern "C" int rk4_stage_adjoint(pmgw_plan p, int32_t k, double dt, const double* h,
                                 const double* u, const double* w, const double* eta,
                                 const double* Ku, const double* Kw, const double* Keta,
                                 double* ub, double* wb, double* etab, double* Kub, double* Kwb,
                                 double* Ketab, double* hbar, double rtol, int32_t maxit,
                                 pmgw_info* info_dev) {
  g_err.clear();
  int rc = check_plan(p);
  if (rc) return rc;
  if (k < 1 || k > 5) return fail(PMGW_EINVAL, "stage k must be in 1..5");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(PMGW_EINVAL, "dt must be positive");
  if (!h || !u || !w || !eta || !Ku || !Kw || !Keta || !ub || !wb || !etab || !Kub || !Kwb ||
      !Ketab || !hbar)
    return fail(PMGW_EINVAL, "fields must be non-NULL");
  if (!(rtol > 0.0) || !std::isfinite(rtol)) return fail(PMGW_EINVAL, "rtol must be positive");
  if (maxit < 1) return fail(PMGW_EINVAL, "maxit must be >= 1");
  if (p->opts.linear || p->opts.no_slip)
    return fail(PMGW_EINVAL, "the adjoint stage covers the default model (linear = no_slip = 0)");
  RkCoef cf;
  cf.a = kCkAlpha[k - 1];
  cf.b = kCkBeta[k - 1];
  cf.dt = dt;
  cf.rho = p->opts.rho;
  cf.g = p->opts.g;
  cf.nu = p->opts.nu_visc;
  const int64_t n2d = p->off2d[p->ntanks], n1d = p->off1d[p->ntanks];
  const RkBufs rb = rk_bufs(p->ws + p->rk_off, n2d, n1d);
  const AdjBufs ab = adj_bufs(p->ws + p->adj_off, n2d, n1d);
  // forward recompute of the stage's intermediates (the caller's state is left untouched)
  hipError_t e = hipMemcpyAsync(ab.eta1, eta, 8 * n1d, hipMemcpyDeviceToDevice, p->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ab.keta1, Keta, 8 * n1d, hipMemcpyDeviceToDevice, p->stream);
  if (e != hipSuccess) return hip_fail(e, "state copy");
  double* cu = const_cast<double*>(u);
  double* cw = const_cast<double*>(w);
  double* cku = const_cast<double*>(Ku);
  double* ckw = const_cast<double*>(Kw);
  rc = launch_rk_all(p, 0, cf, cu, cw, ab.eta1, cku, ckw, ab.keta1, nullptr, rb);
  if (rc) return rc;
  rc = pmgw_set_geometry(p, h, rb.eo, ab.eta1);
  if (rc) return rc;
  rc = launch_rk_all(p, 1, cf, cu, cw, ab.eta1, cku, ckw, ab.keta1, nullptr, rb);
  if (rc) return rc;
  // info_dev, when given, holds 2 x ntanks records: the forward recompute solve's, then the
  // adjoint solve's
  pmgw_info_dev* iinfo = info_dev ? reinterpret_cast<pmgw_info_dev*>(info_dev)
                                  : reinterpret_cast<pmgw_info_dev*>(p->ws + p->info_off);
  pmgw_info_dev* dinfo = info_dev ? iinfo + p->ntanks : iinfo;
  if ((rc = fill_zero_dev(p, ab.p, n2d))) return rc;
  rc = launch_solve(p, MODE_SOLVE, rb.b, ab.p, rtol, maxit, iinfo);
  if (rc) return rc;
  // reverse steps
  rc = launch_rka_all(p, 0, cf, u, w, ub, wb, etab, Kub, Kwb, Ketab, hbar, rb, ab);
  if (rc) return rc;
  if ((rc = fill_zero_dev(p, ab.lam, n2d))) return rc;
  rc = launch_solve(p, MODE_SOLVE, ab.pb, ab.lam, rtol, maxit, dinfo, true);
  if (rc) return rc;
  for (int which = 1; which <= 3; ++which) {
    rc = launch_rka_all(p, which, cf, u, w, ub, wb, etab, Kub, Kwb, Ketab, hbar, rb, ab);
    if (rc) return rc;
  }
  return PMGW_OK;
}

// ----------------------------------------------------------------------------- static scratch
//
// For callers that cannot allocate device memory (code under HIP graph capture, serving loops,
// harnesses that forbid hipMalloc): poisson_solve_noalloc runs the geometry and the solve in this
// file-scope device array instead of a caller-bound workspace. Each GPU that the library runs on
// holds its own copy until the process ends. In host code the name `scratch` is only a host-side
// stand-in; the device address comes from hipGetSymbolAddress, once per device, and is kept in
// g_scratch below.

constexpr size_t kScratchBytes = size_t(48) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};          // device address of `scratch` on each device
uint64_t g_scratch_owner[kMaxDevices] = {}; // gen of the plan whose constant tables it holds

// Device address of the scratch array on device dev (the current device), looked up on the first
// call for that device.
int scratch_for_device(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(PMGW_EDEVICE, "device index out of range");
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255) != 0)
      return fail(PMGW_EDEVICE, "static scratch array is not 256-byte aligned");
    g_scratch[dev] = reinterpret_cast<char*>(ptr);
  }
  *out = g_scratch[dev];
  return PMGW_OK;
}

}  // namespace

extern "C" int poisson_solve_noalloc(pmgw_plan p, const double* h, const double* eta_old,
                                     const double* eta_new, const double* b, double* x,
                                     double rtol, int32_t maxit, pmgw_info* info_host,
                                     pmgw_info* info_dev) {
  g_err.clear();
  if (!p) return fail(PMGW_EINVAL, "plan is NULL");
  if (!h || !eta_old || !eta_new || !b || !x)
    return fail(PMGW_EINVAL, "h, eta_old, eta_new, b and p must be non-NULL");
  if (b == x) return fail(PMGW_EINVAL, "b and p must not overlap");
  if (!(rtol > 0.0) || !std::isfinite(rtol)) return fail(PMGW_EINVAL, "rtol must be positive");
  if (maxit < 1) return fail(PMGW_EINVAL, "maxit must be >= 1");
  if ((size_t)p->total > kScratchBytes)
    return fail(PMGW_EWORKSPACE, "plan needs " + std::to_string(p->total) +
                                     " bytes of workspace; the static scratch array holds " +
                                     std::to_string(kScratchBytes));
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != p->device) return fail(PMGW_EINVAL, "the plan's device is not the current device");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  char* ws = nullptr;
  int rc = scratch_for_device(dev, &ws);
  if (rc) return rc;
  // the array keeps the last call's contents: copy this plan's constant tables in unless they
  // are still there (every other byte the call reads it first writes)
  if (g_scratch_owner[dev] != p->gen) {
    e = hipMemcpyAsync(ws, p->image.data(), p->image.size(), hipMemcpyHostToDevice, p->stream);
    if (e != hipSuccess) return hip_fail(e, "copy of constant tables into the static scratch");
    g_scratch_owner[dev] = p->gen;
  }
  char* const saved_ws = p->ws;
  const bool saved_geo = p->geometry_set, saved_serial = p->serial;
  p->ws = ws;
  p->serial = true;   // no side streams: they would be created on first use
  rc = pmgw_set_geometry(p, h, eta_old, eta_new);
  if (rc == PMGW_OK) rc = solve_entry(p, false, b, x, rtol, maxit, info_host, info_dev);
  const std::string msg = g_err;
  p->ws = saved_ws;
  p->geometry_set = saved_geo;
  p->serial = saved_serial;
  g_err = msg;
  return rc;
}

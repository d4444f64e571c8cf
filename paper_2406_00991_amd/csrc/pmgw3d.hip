// Host side of the 3D tanks: plans, workspace layout, constant tables, launches, C ABI
// (pmgw3d.h). The device code is in pmgw3d_device.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pmgw3d.h"
#include "pmgw3d_device.hpp"
#include "pmgw_tables.hpp"

using namespace pmgw3;

extern "C" const char* pmgw_last_error(void);
// the 2D library's error channel (shared: one last-error message per thread)
namespace pmgw_errors {
int set(int code, const std::string& msg);
}

namespace {

int fail3(int code, const std::string& msg) { return pmgw_errors::set(code, msg); }
int hip_fail3(hipError_t e, const char* what) {
  return fail3(PMGW_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
int64_t al256(int64_t v) { return (v + 255) & ~int64_t(255); }

constexpr size_t kLds3 = 2 * kFftCap3 * 16 + 2 * kMaxN3 * 16;

}  // namespace

struct pmgw3_plan_s {
  int ntanks = 0;
  pmgw_opts opts;
  hipStream_t stream = nullptr;
  std::vector<Tank3> tanks;
  std::vector<int64_t> off3d, off2d;
  std::vector<char> image;     // constant part of the workspace (descriptors, tables)
  int64_t desc_off = 0, info_off = 0, total = 0;
  int maxlev = 0, maxnh = 0;
  char* ws = nullptr;
  bool geometry_set = false;
};

namespace {

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
bool valid_m(int M) { return M == 2 || M == 4 || M == 8 || M == 16 || M == 32; }

template <typename T>
void put(std::vector<char>& img, int64_t off, const std::vector<double>& v) {
  T* p = reinterpret_cast<T*>(img.data() + off);
  for (size_t i = 0; i < v.size(); ++i) p[i] = (T)v[i];
}

Opts3 opts3(const pmgw_opts& o) {
  Opts3 r;
  r.nu1 = o.nu1; r.nu2 = o.nu2; r.coarse_pairs = o.coarse_pairs; r.restart = o.restart;
  r.omega_c = o.omega_c; r.omega_m = o.omega_m; r.adapt = o.adapt_omega_m;
  return r;
}

int check3(pmgw3_plan p) {
  if (!p) return fail3(PMGW_EINVAL, "plan is NULL");
  if (!p->ws) return fail3(PMGW_EWORKSPACE, "no workspace bound");
  return PMGW_OK;
}

int launch3(pmgw3_plan p, int mode, const double* in, double* out, double rtol, int maxit,
            Info3* info) {
  const Tank3* d = reinterpret_cast<const Tank3*>(p->ws + p->desc_off);
  hipLaunchKernelGGL(k3_solve, dim3(p->ntanks), dim3(kThreads3), kLds3, p->stream, d, p->ws,
                     mode, in, out, rtol, maxit, info, opts3(p->opts));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail3(e, "3D solve kernel launch");
  return PMGW_OK;
}

}  // namespace

extern "C" {

int pmgw3_plan_create(pmgw3_plan* out, int32_t ntanks, const int32_t* nx, const int32_t* ny,
                      const int32_t* nz, const double* Lx, const double* Ly, int32_t precision,
                      const pmgw_opts* opts, void* stream) {
  if (!out) return fail3(PMGW_EINVAL, "out is NULL");
  *out = nullptr;
  if (ntanks < 1 || ntanks > 65536) return fail3(PMGW_EINVAL, "ntanks must be in [1, 65536]");
  if (!nx || !ny || !nz || !Lx || !Ly) return fail3(PMGW_EINVAL, "size arrays must be non-NULL");
  if (precision != PMGW_FP64) return fail3(PMGW_EINVAL, "3D tanks run in PMGW_FP64 only");
  pmgw_opts o;
  pmgw_default_opts(&o);
  if (opts) o = *opts;
  if (o.nu1 < 0 || o.nu2 < 0 || o.coarse_pairs < 0 || o.nu1 > 8 || o.nu2 > 8 ||
      o.coarse_pairs > 64)
    return fail3(PMGW_EINVAL, "smoothing counts out of range");
  if (o.restart < 1 || o.restart > kMaxRestart3)
    return fail3(PMGW_EINVAL, "restart must be in [1, 32]");
  if (!(o.omega_c > 0.0 && o.omega_c < 2.0) || !(o.omega_m > 0.0 && o.omega_m < 2.0))
    return fail3(PMGW_EINVAL, "damping factors must be in (0, 2)");
  for (int t = 0; t < ntanks; ++t) {
    if (!pow2(nx[t]) || !pow2(ny[t]) || nx[t] < 4 || ny[t] < 4 || nx[t] > kMaxN3 ||
        ny[t] > kMaxN3 || (int64_t)nx[t] * ny[t] > 65536)
      return fail3(PMGW_EINVAL, "tank " + std::to_string(t) +
                                    ": Nx, Ny must be powers of two in [4, 1024], Nx Ny <= 65536");
    if (!valid_m(nz[t] - 1))
      return fail3(PMGW_EINVAL, "tank " + std::to_string(t) + ": Nz must be 3, 5, 9, 17 or 33");
    if (!(Lx[t] > 0.0) || !(Ly[t] > 0.0) || !std::isfinite(Lx[t]) || !std::isfinite(Ly[t]))
      return fail3(PMGW_EINVAL, "tank " + std::to_string(t) + ": Lx and Ly must be positive");
  }
  pmgw3_plan p = new pmgw3_plan_s();
  p->ntanks = ntanks;
  p->opts = o;
  p->stream = reinterpret_cast<hipStream_t>(stream);
  p->tanks.resize(ntanks);
  p->off3d.assign(ntanks + 1, 0);
  p->off2d.assign(ntanks + 1, 0);
  int64_t cur = 0;
  p->desc_off = cur;
  cur = al256(cur + (int64_t)sizeof(Tank3) * ntanks);
  p->info_off = cur;
  cur = al256(cur + (int64_t)sizeof(Info3) * ntanks);
  // constant tables per tank and level
  for (int t = 0; t < ntanks; ++t) {
    Tank3& d = p->tanks[t];
    std::memset(&d, 0, sizeof(d));
    d.nx = nx[t]; d.ny = ny[t]; d.nz = nz[t];
    d.lgx = pmgw_tables::ilog2(nx[t]); d.lgy = pmgw_tables::ilog2(ny[t]);
    d.Lx = Lx[t]; d.Ly = Ly[t];
    d.kfx = 2.0 * M_PI / Lx[t]; d.kfy = 2.0 * M_PI / Ly[t];
    const double Kx = nx[t] / 2 - 1, Ky = ny[t] / 2 - 1;
    d.cxx = -(d.kfx * d.kfx / nx[t]) * 2.0 * (Kx * (Kx + 1.0) * (2.0 * Kx + 1.0) / 6.0);
    d.cyy = -(d.kfy * d.kfy / ny[t]) * 2.0 * (Ky * (Ky + 1.0) * (2.0 * Ky + 1.0) / 6.0);
    d.off3d = p->off3d[t];
    d.off2d = p->off2d[t];
    const int64_t nh = (int64_t)nx[t] * ny[t];
    p->off3d[t + 1] = p->off3d[t] + nh * nz[t];
    p->off2d[t + 1] = p->off2d[t] + nh;
    int M = nz[t] - 1, l = 0;
    while (true) {
      Lev3& lv = d.lev[l];
      lv.nz = M + 1;
      lv.nzc = (M > 2) ? M / 2 + 1 : 0;
      lv.ds = cur; cur = al256(cur + 8LL * lv.nz * lv.nz);
      lv.sig = cur; cur = al256(cur + 8LL * lv.nz);
      if (lv.nzc) {
        lv.R = cur; cur = al256(cur + 8LL * lv.nzc * lv.nz);
        lv.P = cur; cur = al256(cur + 8LL * lv.nz * lv.nzc);
      }
      ++l;
      if (M == 2) break;
      M /= 2;
    }
    d.nlev = l;
    p->maxlev = std::max(p->maxlev, l);
    p->maxnh = std::max<int>(p->maxnh, (int)nh);
  }
  const int64_t const_end = cur;
  const int m = o.restart;
  for (int t = 0; t < ntanks; ++t) {
    Tank3& d = p->tanks[t];
    const int64_t nh = (int64_t)d.nx * d.ny, n = nh * d.nz;
    d.geo = cur; cur = al256(cur + 8LL * G_COUNT * nh);
    d.scal = cur; cur = al256(cur + 64);
    d.V = cur; cur = al256(cur + 8LL * (m + 1) * n);
    d.Z = cur; cur = al256(cur + 8LL * m * n);
    for (int l = 0; l < d.nlev; ++l) {
      Lev3& lv = d.lev[l];
      const int64_t nl = nh * lv.nz;
      lv.colinv = cur; cur = al256(cur + 8LL * lv.nz * lv.nz * nh);
      lv.modeinv = cur; cur = al256(cur + 8LL * lv.nz * lv.nz * nh);
      for (int64_t* f : {&lv.x, &lv.f, &lv.r, &lv.t1, &lv.gx, &lv.gy, &lv.t2, &lv.t3}) {
        *f = cur;
        cur = al256(cur + 8LL * nl);
      }
      lv.spec = cur; cur = al256(cur + 16LL * ((lv.nz + 1) / 2) * nh);
    }
  }
  p->total = cur;
  p->image.assign(const_end, 0);
  std::memcpy(p->image.data() + p->desc_off, p->tanks.data(), sizeof(Tank3) * ntanks);
  for (int t = 0; t < ntanks; ++t) {
    const Tank3& d = p->tanks[t];
    for (int l = 0; l < d.nlev; ++l) {
      const Lev3& lv = d.lev[l];
      const int M = lv.nz - 1;
      put<double>(p->image, lv.ds, pmgw_tables::dsigma(M));
      put<double>(p->image, lv.sig, pmgw_tables::cgl_sigma(M));
      if (lv.nzc) {
        put<double>(p->image, lv.R, pmgw_tables::restriction(M));
        put<double>(p->image, lv.P, pmgw_tables::prolongation(M));
      }
    }
  }
  *out = p;
  return PMGW_OK;
}

size_t pmgw3_workspace_bytes(pmgw3_plan p) { return p ? (size_t)p->total : 0; }

int pmgw3_bind_workspace(pmgw3_plan p, void* dev, size_t bytes) {
  if (!p) return fail3(PMGW_EINVAL, "plan is NULL");
  if (!dev || bytes < (size_t)p->total)
    return fail3(PMGW_EWORKSPACE, "workspace missing or smaller than pmgw3_workspace_bytes");
  if (reinterpret_cast<uintptr_t>(dev) & 255)
    return fail3(PMGW_EWORKSPACE, "workspace must be 256-byte aligned");
  p->ws = static_cast<char*>(dev);
  hipError_t e = hipMemcpyAsync(p->ws, p->image.data(), p->image.size(), hipMemcpyHostToDevice,
                                p->stream);
  if (e != hipSuccess) return hip_fail3(e, "workspace image copy");
  e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return hip_fail3(e, "workspace image copy");
  p->geometry_set = false;
  return PMGW_OK;
}

int pmgw3_field_offsets(pmgw3_plan p, int64_t* off3d, int64_t* off2d) {
  if (!p || !off3d || !off2d) return fail3(PMGW_EINVAL, "NULL argument");
  std::copy(p->off3d.begin(), p->off3d.end(), off3d);
  std::copy(p->off2d.begin(), p->off2d.end(), off2d);
  return PMGW_OK;
}

int pmgw3_set_geometry(pmgw3_plan p, const double* h, const double* eo, const double* en) {
  int rc = check3(p);
  if (rc) return rc;
  if (!h || !eo || !en) return fail3(PMGW_EINVAL, "h, eta_old and eta_new must be non-NULL");
  const Tank3* d = reinterpret_cast<const Tank3*>(p->ws + p->desc_off);
  hipLaunchKernelGGL(k3_geometry, dim3(p->ntanks), dim3(256), kLds3, p->stream, d, p->ws, h, eo,
                     en);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail3(e, "3D geometry kernel launch");
  hipLaunchKernelGGL(k3_blocks, dim3(2 * p->maxnh, p->maxlev, p->ntanks), dim3(64), 0, p->stream,
                     d, p->ws);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail3(e, "3D block kernel launch");
  p->geometry_set = true;
  return PMGW_OK;
}

int pmgw3_laplacian_apply(pmgw3_plan p, const double* in, double* out) {
  int rc = check3(p);
  if (rc) return rc;
  if (!p->geometry_set) return fail3(PMGW_EINVAL, "geometry not set");
  if (!in || !out || in == out) return fail3(PMGW_EINVAL, "p and Ap must be distinct, non-NULL");
  return launch3(p, M3_APPLY, in, out, 0.0, 0, nullptr);
}

int pmgw3_vcycle(pmgw3_plan p, const double* r, double* z) {
  int rc = check3(p);
  if (rc) return rc;
  if (!p->geometry_set) return fail3(PMGW_EINVAL, "geometry not set");
  if (!r || !z || r == z) return fail3(PMGW_EINVAL, "r and z must be distinct, non-NULL");
  return launch3(p, M3_VCYCLE, r, z, 0.0, 0, nullptr);
}

int pmgw3_poisson_solve(pmgw3_plan p, const double* b, double* x, double rtol, int32_t maxit,
                        pmgw_info* info_host, pmgw_info* info_dev) {
  int rc = check3(p);
  if (rc) return rc;
  if (!p->geometry_set) return fail3(PMGW_EINVAL, "geometry not set");
  if (!b || !x || b == x) return fail3(PMGW_EINVAL, "b and p must be distinct, non-NULL");
  if (!(rtol > 0.0) || !std::isfinite(rtol)) return fail3(PMGW_EINVAL, "rtol must be positive");
  if (maxit < 1) return fail3(PMGW_EINVAL, "maxit must be >= 1");
  static_assert(sizeof(Info3) == sizeof(pmgw_info), "info layout");
  Info3* di = info_dev ? reinterpret_cast<Info3*>(info_dev)
                       : reinterpret_cast<Info3*>(p->ws + p->info_off);
  rc = launch3(p, M3_SOLVE, b, x, rtol, maxit, di);
  if (rc) return rc;
  if (info_host) {
    hipError_t e = hipMemcpyAsync(info_host, di, sizeof(pmgw_info) * p->ntanks,
                                  hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail3(e, "info copy");
    int worst = PMGW_OK;
    for (int t = 0; t < p->ntanks; ++t) {
      const int s = info_host[t].status;
      if (s < 0 && (worst >= 0 || s < worst)) worst = s;
      else if (s > 0 && worst == PMGW_OK) worst = s;
    }
    if (worst < 0) return fail3(worst, "a tank failed (see info)");
    return worst;
  }
  return PMGW_OK;
}

void pmgw3_plan_destroy(pmgw3_plan p) { delete p; }

}  // extern "C"

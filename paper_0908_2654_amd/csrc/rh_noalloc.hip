// Handle-free residual evaluation that allocates nothing: the variant of
// rh_residual for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// rh_residual keeps its face coefficients, the constant part of the
// radiation residual, the local elimination terms and the reduction
// partials in the caller's workspace.  Here they live in one file-scope
// device array, `scratch`, sized for grids of up to kMaxCells cells; each
// GPU holds its own copy for the life of the process.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in
// symbol): the device address is looked up with hipGetSymbolAddress once
// per device, on the first call with that device current, and kept.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <mutex>

#include "rh_internal.h"

using namespace rh;

namespace {

constexpr long long kMaxCells = 1LL << 18;  // 64^3
constexpr int kFields = 8;                  // cf_x, cf_y, cf_z, rhs^n, BCn, BCe, Bfn, Bfe
constexpr size_t kFieldDoubles = (size_t)kMaxCells;
constexpr size_t kPartDoubles = (size_t)RS_COUNT * kPartCap + RS_COUNT;
constexpr size_t kOutOffset = kFields * kFieldDoubles + ((kPartDoubles + 31) / 32) * 32;
constexpr size_t kScratchDoubles = kOutOffset + 32;  // + the finalized slots

// 8 * 2 MiB of fields + 2.2 MiB of partials (about 18.3 MiB per GPU)
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
double* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of the scratch array.
rh_status scratch_ptr(double** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    set_last_error("rh_residual_noalloc: no current HIP device");
    return RH_EHIP;
  }
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      char buf[160];
      std::snprintf(buf, sizeof buf, "rh_residual_noalloc: hipGetSymbolAddress failed: %s",
                    hipGetErrorString(e));
      set_last_error(buf);
      return RH_EHIP;
    }
    g_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_ptr[dev];
  return RH_OK;
}

bool bad_ptr(const void* q) { return !q || reinterpret_cast<uintptr_t>(q) % 8 != 0; }

rh_status hip_fail(const char* what) {
  const hipError_t e = hipGetLastError();
  char buf[200];
  std::snprintf(buf, sizeof buf, "rh_residual_noalloc: HIP error at %s: %s", what,
                hipGetErrorString(e));
  set_last_error(buf);
  return RH_EHIP;
}

// The second reduction pass into the scratch's output slots, then the
// values to the host (the stream drains).
rh_status finalize_to_host(hipStream_t s, const double* part, double* out_dev, unsigned mask,
                           double* host) {
  launch_finalize(s, part, out_dev, mask);
  if (hipGetLastError() != hipSuccess) return hip_fail("finalize");
  if (hipMemcpyAsync(host, out_dev, sizeof(double) * RS_COUNT, hipMemcpyDeviceToHost, s) !=
      hipSuccess)
    return hip_fail("hipMemcpyAsync");
  if (hipStreamSynchronize(s) != hipSuccess) return hip_fail("hipStreamSynchronize");
  return RH_OK;
}

}  // namespace

extern "C" rh_status rh_residual_noalloc(const rh_params* p, void* hip_stream, double t_n,
                                         double dt, const double* nH, const double* src,
                                         const double* E_n, const double* e_n,
                                         const double* nHI_n, const double* E, const double* e,
                                         const double* nHI, double* fE, double* fe, double* fn,
                                         double* norm_out) {
  char err[256];
  if (!params_valid(p, err, sizeof err)) {
    set_last_error(err);
    return RH_EINVAL;
  }
  const long long N = (long long)p->nx * p->ny * p->nz;
  if (N > kMaxCells) {
    std::snprintf(err, sizeof err,
                  "rh_residual_noalloc: %lld cells exceed the static scratch limit of %lld "
                  "(64^3); use rh_residual with a workspace",
                  N, kMaxCells);
    set_last_error(err);
    return RH_EINVAL;
  }
  const bool iso = p->isothermal != 0;
  for (const void* q : {(const void*)nH, (const void*)src, (const void*)E_n,
                        (const void*)nHI_n, (const void*)E, (const void*)nHI})
    if (bad_ptr(q)) {
      set_last_error("rh_residual_noalloc: NULL or misaligned field pointer");
      return RH_EINVAL;
    }
  if (!iso && (bad_ptr(e_n) || bad_ptr(e))) {
    set_last_error("rh_residual_noalloc: NULL or misaligned field pointer");
    return RH_EINVAL;
  }
  for (const void* q : {(const void*)fE, (const void*)fe, (const void*)fn})
    if (q && reinterpret_cast<uintptr_t>(q) % 8 != 0) {
      set_last_error("rh_residual_noalloc: misaligned output pointer");
      return RH_EINVAL;
    }
  if (!(dt > 0) || !std::isfinite(dt) || !std::isfinite(t_n)) {
    set_last_error("rh_residual_noalloc: dt must be > 0 and t finite");
    return RH_EINVAL;
  }
  if (p->cosmology != RH_COSMO_STATIC && !(t_n > 0)) {
    set_last_error("rh_residual_noalloc: expanding cosmology needs t > 0");
    return RH_EINVAL;
  }
  double* base = nullptr;
  rh_status st = scratch_ptr(&base);
  if (st != RH_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  double* cf[3] = {base, base + kFieldDoubles, base + 2 * kFieldDoubles};
  double* rhsn = base + 3 * kFieldDoubles;
  double* loc[4];
  for (int q = 0; q < 4; ++q) loc[q] = base + (4 + q) * kFieldDoubles;
  double* part = base + kFields * kFieldDoubles;
  double* out = base + kOutOffset;
  double host[RS_COUNT];

  // face limiter from U^n, constant part of f_E and the norm scale E_s
  StepK k = step_scalars(*p, t_n, dt);
  launch_step_setup(s, k, E_n, nHI_n, nullptr, nullptr, src, cf[0], cf[1], cf[2], nullptr, rhsn,
                    part);
  if (hipGetLastError() != hipSuccess) return hip_fail("step setup");
  if ((st = finalize_to_host(s, part, out,
                             slot_bit(RS_EMAX) | slot_bit(RS_SMAX) | slot_bit(RS_NONFINITE),
                             host)) != RH_OK)
    return st;
  if (host[RS_NONFINITE] != 0.0) {
    set_last_error("rh_residual_noalloc: non-finite E^n, n_HI^n or src");
    return RH_ENONFINITE;
  }
  k.E_s = std::fmax(std::fmax(host[RS_EMAX], k.dt * host[RS_SMAX]), p->E_floor);

  // local residuals and elimination terms at U, then the radiation residual
  LocalArgs a{};
  a.Ek = E; a.dE = nullptr; a.lam = 0.0;
  a.ek = iso ? nullptr : e; a.nk = nHI;
  a.En = E_n; a.en = iso ? nullptr : e_n; a.nn = nHI_n; a.nH = nH;
  a.BCn = loc[0]; a.BCe = loc[1]; a.Bfn = loc[2]; a.Bfe = loc[3];
  a.fn_out = fn; a.fe_out = iso ? nullptr : fe;
  a.mode = 1;
  launch_local(s, k, a, part);
  if (hipGetLastError() != hipSuccess) return hip_fail("local terms");
  ResidArgs r{};
  r.E = E; r.n = nHI; r.En = E_n; r.nn = nHI_n;
  for (int d = 0; d < 3; ++d) r.cf[d] = cf[d];
  r.rhsn = rhsn;
  r.BCn = loc[0]; r.Bfn = loc[2];
  r.fE_out = fE;
  launch_residual(s, k, r, part);
  if (hipGetLastError() != hipSuccess) return hip_fail("radiation residual");
  const unsigned mask = slot_bit(RS_FE2) | slot_bit(RS_FN2) | slot_bit(RS_FE_LOC2) |
                        slot_bit(RS_NONFINITE) | slot_bit(RS_BAD_RES);
  if ((st = finalize_to_host(s, part, out, mask, host)) != RH_OK) return st;
  const double sum = host[RS_FE2] + host[RS_FN2] + (iso ? 0.0 : host[RS_FE_LOC2]);
  if (norm_out) *norm_out = std::sqrt(sum / (N * (iso ? 2.0 : 3.0)));
  return RH_OK;
}

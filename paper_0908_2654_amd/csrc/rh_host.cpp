// Host side of the C ABI: parameter validation, grey constants, cosmology,
// workspace carve-up, and the Newton / defect-correction / V-cycle drivers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "rh_host_internal.h"

using namespace rh;

namespace {

// message of the last failed handle-free call on this thread (a fixed
// buffer: setting it allocates nothing)
thread_local char g_last_error[256];

void set_global_error(const char* msg) {
  std::snprintf(g_last_error, sizeof g_last_error, "%s", msg);
}

// ---------------------------------------------------------------------------
// grey constants of the T_B blackbody above h nu_0 (equation grey_definition)
// with sigma(nu) = sigma_0 (nu_0/nu)^3; evaluated by series (the oracle
// uses quadrature of the defining integrals).
// ---------------------------------------------------------------------------
double expint_E1(double x) {
  if (x <= 1.0) {  // power series: -gamma - ln x - sum (-x)^k / (k k!)
    const double euler = 0.57721566490153286061;
    double sum = 0.0, term = 1.0;
    for (int k = 1; k < 200; ++k) {
      term *= -x / k;
      double add = term / k;
      sum += add;
      if (std::fabs(add) < 1e-18 * std::fabs(sum)) break;
    }
    return -euler - std::log(x) - sum;
  }
  // continued fraction e^-x / (x+1 - 1/(x+3 - 4/(x+5 - ...))), modified Lentz
  const double tiny = 1e-300;
  double b = x + 1.0, c = 1.0 / tiny, d = 1.0 / b, h = d;
  for (int i = 1; i < 500; ++i) {
    double an = -(double)i * i;
    b += 2.0;
    d = 1.0 / (an * d + b);
    c = b + an / c;
    double del = c * d;
    h *= del;
    if (std::fabs(del - 1.0) < 1e-16) break;
  }
  return h * std::exp(-x);
}


Grey grey_constants(const rh_params& p) {
  Grey g;
  g.hnu0 = p.hnu0_eV * kEV;
  if (p.spectrum == RH_SPEC_MONO) {
    g.sigma_E = p.sigma0_cm2;
    g.K_Gamma = p.sigma0_cm2 / g.hnu0;
    g.K_G = 0.0;
    g.eps_bar = g.hnu0;
    return g;
  }
  const double kT = kKB * p.T_bb_K;
  const double x = g.hnu0 / kT;
  double IE = 0.0, IN = 0.0, IsN = 0.0;
  for (int k = 1; k < 2000; ++k) {
    const double ek = std::exp(-k * x);
    const double kk = k;
    const double tE = ek * (x * x * x / kk + 3 * x * x / (kk * kk) + 6 * x / (kk * kk * kk) +
                            6 / (kk * kk * kk * kk));
    const double tN = ek * (x * x / kk + 2 * x / (kk * kk) + 2 / (kk * kk * kk));
    const double tS = expint_E1(kk * x);
    IE += tE;
    IN += tN;
    IsN += tS;
    if (tE < 1e-19 * IE && tS < 1e-19 * IsN) break;
  }
  const double x3 = x * x * x;
  const double IsE = -x3 * std::log1p(-std::exp(-x));
  IsN *= x3;
  g.sigma_E = p.sigma0_cm2 * IsE / IE;
  g.K_Gamma = p.sigma0_cm2 * IsN / (kT * IE);
  g.K_G = g.sigma_E - g.hnu0 * g.K_Gamma;
  g.eps_bar = kT * IE / IN;
  return g;
}

// ---------------------------------------------------------------------------
// cosmology (Friedmann equation closed forms)
// ---------------------------------------------------------------------------
// Open universe (Omega_L = 0, Ok = 1 - Omega_m > 0): H^2 = H0^2 (Om a^-3 +
// Ok a^-2) is solved by a = A (cosh u - 1), t = B (sinh u - u) with
// A = Om / (2 Ok), B = Om / (2 H0 Ok^1.5).  g(u) = sinh u - u, written as a
// series where the difference would cancel.
static double open_g(double u) {
  if (u < 0.1) {
    const double u2 = u * u;
    return u * u2 / 6.0 * (1.0 + u2 / 20.0 * (1.0 + u2 / 42.0 * (1.0 + u2 / 72.0)));
  }
  return std::sinh(u) - u;
}

// The development angle u with g(u) = tau: Newton from above (g is convex
// and increasing for u > 0, so the iterates decrease monotonically to the root).
static double open_angle(double tau) {
  double u = std::max(std::cbrt(6.0 * tau), std::asinh(tau) + 1.0);
  while (open_g(u) < tau) u *= 2.0;
  for (int it = 0; it < 200; ++it) {
    const double gp = 2.0 * std::sinh(0.5 * u) * std::sinh(0.5 * u);  // cosh u - 1
    const double step = (open_g(u) - tau) / gp;
    if (!(step > 0.0)) break;
    u -= step;
    if (step <= 1e-16 * u) break;
  }
  return u;
}

void cosmo_at(const rh_params& p, double t, double& a, double& H) {
  const double H0 = p.hubble_h * kH100;
  if (p.cosmology == RH_COSMO_STATIC) {
    a = 1.0;
    H = 0.0;
  } else if (p.cosmology == RH_COSMO_EDS) {
    a = std::pow(1.5 * H0 * t, 2.0 / 3.0);
    H = 2.0 / (3.0 * t);
  } else if (p.cosmology == RH_COSMO_OPEN) {
    const double Ok = 1.0 - p.Omega_m;
    const double A = p.Omega_m / (2.0 * Ok), B = p.Omega_m / (2.0 * H0 * Ok * std::sqrt(Ok));
    const double u = open_angle(t / B);
    a = A * 2.0 * std::sinh(0.5 * u) * std::sinh(0.5 * u);
    H = H0 * std::sqrt(p.Omega_m / (a * a * a) + Ok / (a * a));
  } else {
    const double s = std::sinh(1.5 * std::sqrt(p.Omega_L) * H0 * t);
    a = std::cbrt(p.Omega_m / p.Omega_L) * std::pow(s, 2.0 / 3.0);
    H = H0 * std::sqrt(p.Omega_m / (a * a * a) + p.Omega_L);
  }
}

// Compton cooling coefficient 4 sigma_T a_rad k_B T_cmb0^4 / (m_e c) (the
// rate per electron and per kelvin of T - T_cmb at z = 0; scales as (1+z)^4).
double compton_coefficient() {
  return 4.0 * kSigmaT * kARad * kKB * std::pow(kTcmb0, 4) / (kME * kC);
}

// ---------------------------------------------------------------------------
// validation and multigrid plan
// ---------------------------------------------------------------------------

bool plan_levels(const rh_params& p, Plan& pl, std::string& err) {
  int d[3] = {p.nx, p.ny, p.nz};
  pl.nlev = 1;
  pl.dims[0][0] = d[0]; pl.dims[0][1] = d[1]; pl.dims[0][2] = d[2];
  const long long cap = p.mg_coarse_max;
  while (pl.nlev < kMaxLevels) {
    long long cells = (long long)d[0] * d[1] * d[2];
    if (cells <= cap) break;
    bool ok = true;
    for (int a = 0; a < 3; ++a) ok = ok && (d[a] % 2 == 0) && d[a] >= 4;
    if (!ok) break;
    for (int a = 0; a < 3; ++a) d[a] /= 2;
    pl.dims[pl.nlev][0] = d[0]; pl.dims[pl.nlev][1] = d[1]; pl.dims[pl.nlev][2] = d[2];
    ++pl.nlev;
  }
  long long cells = (long long)d[0] * d[1] * d[2];
  if (cells > kCoarseMaxCells) {
    err = "grid cannot be coarsened to <= 512 cells (dimensions must stay even while halving)";
    return false;
  }
  return true;
}

bool validate(const rh_params* p, std::string& err) {
  if (!p) { err = "params is NULL"; return false; }
  const int d[3] = {p->nx, p->ny, p->nz};
  for (int a = 0; a < 3; ++a)
    if (d[a] < 1) { err = "grid dimensions must be >= 1"; return false; }
  if ((long long)d[0] * d[1] * d[2] > (1LL << 34)) { err = "grid too large"; return false; }
  for (int f = 0; f < 6; ++f)
    if (p->bc[f] < 0 || p->bc[f] > 2) { err = "unknown boundary condition"; return false; }
  for (int a = 0; a < 3; ++a) {
    const bool lo = p->bc[2 * a] == RH_BC_PERIODIC, hi = p->bc[2 * a + 1] == RH_BC_PERIODIC;
    if (lo != hi) { err = "periodic boundaries must be paired"; return false; }
    if (lo && d[a] < 3) { err = "periodic dimension needs >= 3 cells"; return false; }
  }
  if (!(p->box_comoving_cm > 0) || !std::isfinite(p->box_comoving_cm)) { err = "box must be > 0"; return false; }
  if (!(p->theta > 0.0 && p->theta <= 1.0)) { err = "theta must lie in (0, 1]"; return false; }
  if (!(p->gamma > 1.0)) { err = "gamma must be > 1"; return false; }
  if (p->isothermal && !(p->T_iso_K > 0)) { err = "T_iso must be > 0"; return false; }
  if (p->spectrum != RH_SPEC_MONO && p->spectrum != RH_SPEC_BLACKBODY) { err = "unknown spectrum"; return false; }
  if (p->spectrum == RH_SPEC_BLACKBODY && !(p->T_bb_K > 0)) { err = "T_bb must be > 0"; return false; }
  if (!(p->hnu0_eV > 0) || !(p->sigma0_cm2 >= 0)) { err = "hnu0 > 0 and sigma0 >= 0 required"; return false; }
  if (p->rates != RH_RATES_CONST && p->rates != RH_RATES_FIT) { err = "unknown rates"; return false; }
  if (p->rates == RH_RATES_CONST && !(p->alphaB_const >= 0)) { err = "alphaB_const must be >= 0"; return false; }
  if (p->cosmology < 0 || p->cosmology > 3) { err = "unknown cosmology"; return false; }
  if (p->cosmology == RH_COSMO_OPEN && (!(p->Omega_m > 0 && p->Omega_m < 1) || p->Omega_L != 0)) {
    err = "open cosmology needs 0 < Omega_m < 1 and Omega_L = 0"; return false;
  }
  if (p->cosmology != RH_COSMO_STATIC && !(p->hubble_h > 0)) { err = "hubble_h must be > 0"; return false; }
  if (p->cosmology == RH_COSMO_EDS && std::fabs(p->Omega_m - 1.0) > 1e-12) { err = "EdS needs Omega_m = 1"; return false; }
  if (p->cosmology == RH_COSMO_FLAT_LCDM &&
      (std::fabs(p->Omega_m + p->Omega_L - 1.0) > 1e-12 || !(p->Omega_L > 0) || !(p->Omega_m > 0))) {
    err = "flat LCDM needs Omega_m + Omega_L = 1, both > 0"; return false;
  }
  if (p->precision != RH_PREC_FP64 && p->precision != RH_PREC_MIXED) { err = "unknown precision"; return false; }
  if (!(p->E_floor > 0)) { err = "E_floor must be > 0"; return false; }
  if (!(p->newton_tol > 0) || p->newton_max_it < 1 || p->ls_max_cuts < 0) { err = "bad Newton settings"; return false; }
  if (!(p->lin_forcing > 0) || p->lin_max_it < 1) { err = "bad linear settings"; return false; }
  if (p->mg_pre < 1 || p->mg_post < 0 || p->mg_pre > 16 || p->mg_post > 16) { err = "mg_pre in [1,16], mg_post in [0,16]"; return false; }
  if (p->mg_coarse_max < 1 || p->mg_coarse_max > kCoarseMaxCells) { err = "mg_coarse_max in [1, 512]"; return false; }
  if (p->krylov != 0 && p->krylov != 1) { err = "krylov must be 0 or 1"; return false; }
  if (p->smoother < 0 || p->smoother > 2) { err = "smoother must be 0, 1 or 2"; return false; }
  if (p->mg_block_radius < 0 || p->mg_block_radius > 2) { err = "mg_block_radius in [0, 2]"; return false; }
  if (p->mg_block_levels < 0 || p->mg_block_levels > kMaxBlockLevels) { err = "mg_block_levels in [0, 4]"; return false; }
  if (p->mg_block_max < 0 || p->mg_block_max > (1 << 20)) { err = "mg_block_max in [0, 2^20]"; return false; }
  Plan pl;
  if (!plan_levels(*p, pl, err)) return false;
  return true;
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
// Most source cells with boxes: mg_block_max, or when it is 0 one per 4096
// cells, at least 64 and at most 8192.
long long block_capacity(const rh_params& p) {
  if (p.mg_block_max > 0) return p.mg_block_max;
  const long long N = (long long)p.nx * p.ny * p.nz;
  return std::min<long long>(8192, std::max<long long>(64, N / 4096));
}

struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

}  // namespace


namespace {

size_t layout(rh_handle* h, const rh_params& p, const Plan& pl, char* base) {
  Carver cv{base};
  const long long N = (long long)p.nx * p.ny * p.nz;
  h->En = cv.take<double>(N);
  h->en = cv.take<double>(N);
  h->nn = cv.take<double>(N);
  h->rhsn = cv.take<double>(N);
  h->rS = cv.take<double>(N);
  h->diag64 = cv.take<double>(N);
  h->dEa = cv.take<double>(N);
  h->dEb = cv.take<double>(N);
  if (p.krylov) {
    h->r64 = cv.take<double>(N);
    h->pa = cv.take<double>(N);
    h->pb = cv.take<double>(N);
    h->q64 = cv.take<double>(N);
  }
  for (int d = 0; d < 3; ++d) h->cf64[d] = cv.take<double>(N);
  h->B.E = cv.take<double>(N);
  h->B.e = cv.take<double>(N);
  h->B.n = cv.take<double>(N);
  for (int q = 0; q < 4; ++q) h->B.loc[q] = cv.take<double>(N);
  for (int q = 0; q < 4; ++q) h->locA[q] = cv.take<double>(N);
  h->part = cv.take<double>((size_t)RS_COUNT * kPartCap + RS_COUNT);
  const bool mixed = p.precision == RH_PREC_MIXED;
  for (int l = 0; l < pl.nlev; ++l) {
    const int* d = pl.dims[l];
    const long long n = (long long)d[0] * d[1] * d[2];
    const int per[3] = {p.bc[0] == RH_BC_PERIODIC, p.bc[2] == RH_BC_PERIODIC,
                        p.bc[4] == RH_BC_PERIODIC};
    if (mixed) {
      LevelK<float>& L = h->L32[l];
      L.nx = d[0]; L.ny = d[1]; L.nz = d[2]; L.N = n;
      for (int a = 0; a < 3; ++a) L.per[a] = per[a];
      L.x = cv.take<float>(n);
      L.x2 = cv.take<float>(n);
      L.b = cv.take<float>(n);
      L.r = cv.take<float>(n);
      L.op = cv.take<Op16>(n);
    } else {
      LevelK<double>& L = h->L64[l];
      L.nx = d[0]; L.ny = d[1]; L.nz = d[2]; L.N = n;
      for (int a = 0; a < 3; ++a) L.per[a] = per[a];
      L.x = cv.take<double>(n);
      L.x2 = cv.take<double>(n);
      L.b = cv.take<double>(n);
      L.r = cv.take<double>(n);
      if (l == 0) {
        L.diag = h->diag64;
        for (int a = 0; a < 3; ++a) L.cf[a] = h->cf64[a];
      } else {
        L.diag = cv.take<double>(n);
        for (int a = 0; a < 3; ++a) L.cf[a] = cv.take<double>(n);
      }
    }
  }
  const int* dc = pl.dims[pl.nlev - 1];
  const long long nc = (long long)dc[0] * dc[1] * dc[2];
  h->cA = cv.take<double>(nc * nc);
  h->cInv = cv.take<double>(nc * nc);
  h->cInv32 = mixed ? cv.take<float>(nc * nc) : nullptr;
  h->cInv64 = mixed ? nullptr : cv.take<double>(nc * nc);
  // block smoother: source scan buffers and, per level with boxes, the box
  // corners and inverses
  const int R = p.mg_block_radius;
  const int blevels = R > 0 ? std::min(p.mg_block_levels, pl.nlev - 1) : 0;
  h->src_groups = (int)std::min<long long>(4096, (N + kBlock - 1) / kBlock);
  h->src_chunk = (N + h->src_groups - 1) / h->src_groups;
  h->src_count = cv.take<int>(h->src_groups);
  h->src_offset = cv.take<int>(h->src_groups);
  const long long cap = block_capacity(p);
  h->src_list = blevels > 0 ? cv.take<int>(cap) : nullptr;
  for (int l = 0; l < kMaxBlockLevels; ++l) {
    h->bstart[l] = nullptr;
    h->B32[l] = BlockSet<float>{};
    h->B64[l] = BlockSet<double>{};
  }
  for (int l = 0; l < blevels; ++l) {
    int m = 1;
    for (int a = 0; a < 3; ++a) m *= std::min(2 * R + 1, pl.dims[l][a]);
    h->bstart[l] = cv.take<int>((size_t)3 * cap);
    if (mixed)
      h->B32[l].inv = cv.take<float>((size_t)cap * m * m);
    else
      h->B64[l].inv = cv.take<double>((size_t)cap * m * m);
  }
  return cv.off + 256;
}

#define HIPCHK(call)                                                           \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      h->err = std::string("HIP error: ") + hipGetErrorString(e_) + " at " #call; \
      return RH_EHIP;                                                          \
    }                                                                          \
  } while (0)

rh_status fail(rh_handle* h, rh_status st, const std::string& msg) {
  h->err = msg;
  return st;
}

StepK make_step_from(const rh_params& p, const Grey& g, double t_n, double dt) {
  const double hcell = p.box_comoving_cm / p.nx;
  StepK k;
  k.nx = p.nx; k.ny = p.ny; k.nz = p.nz;
  k.N = (long long)p.nx * p.ny * p.nz;
  for (int f = 0; f < 6; ++f) k.bc[f] = p.bc[f];
  k.iso = p.isothermal ? 1 : 0;
  k.rates = p.rates;
  k.cooling = p.cooling_mask;
  k.theta_lt1 = p.theta < 1.0 ? 1 : 0;
  k.h = hcell;
  k.dt = dt;
  k.theta = p.theta;
  cosmo_at(p, t_n, k.a_n, k.H_n);
  cosmo_at(p, t_n + dt, k.a_1, k.H_1);
  k.sigma_E = g.sigma_E;
  k.K_Gamma = g.K_Gamma;
  k.K_G = g.K_G;
  k.hnu0 = g.hnu0;
  k.T_iso = p.T_iso_K;
  k.alphaB = p.alphaB_const;
  k.gamma = p.gamma;
  k.compton = compton_coefficient();
  k.E_floor = p.E_floor;
  k.R_min = p.R_min > 0 ? p.R_min : 1.0 / (k.a_n * p.box_comoving_cm);
  k.cf_scale = dt * p.theta / (k.a_1 * k.a_1 * hcell * hcell);
  k.expl_ratio = (1.0 - p.theta) / p.theta * (k.a_1 * k.a_1) / (k.a_n * k.a_n);
  k.E_s = 1.0;
  k.sig_he[0] = k.sig_he[1] = 0.0;
  k.src_frac = 1.0;
  return k;
}

StepK make_step(rh_handle* h, double t_n, double dt) { return make_step_from(h->p, h->g, t_n, dt); }

// Phases of a step (rh_step_stats.t_ms[1..5]).
enum Phase { PH_SETUP = 1, PH_EVAL = 2, PH_COARSE = 3, PH_VCYCLE = 4, PH_OUTER = 5 };

void phase_begin(rh_handle* h) {
  h->npev = 0;
  h->cur_phase = -1;
  for (double& v : h->pms) v = 0.0;
  h->phases_on = h->phase_events;
}

const char* const kPhaseName[6] = {"", "step setup", "local solve + residual",
                                   "coarse operators", "V-cycles", "outer iteration"};

// The step's profiler ranges: one over the call, and one per phase that
// phase_mark switches; the destructor closes both on every return path.
struct StepMarks {
  rh_handle* h;
  MarkerRange step;
  StepMarks(rh_handle* hh, const char* name) : h(hh), step(name) { h->mark_on = true; }
  ~StepMarks() {
    if (h->mark_phase) roctxRangeStop(h->mark_id);
    h->mark_phase = 0;
    h->mark_on = false;
  }
};

void phase_mark(rh_handle* h, int phase) {
  if (h->mark_on && h->mark_phase != phase) {
    if (h->mark_phase) roctxRangeStop(h->mark_id);
    h->mark_id = roctxRangeStartA(kPhaseName[phase]);
    h->mark_phase = phase;
  }
  if (!h->phases_on || h->cur_phase == phase || h->npev == rh_handle::kPhaseEv) return;
  if (hipEventRecord(h->pev[h->npev], h->stream) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  h->pph[h->npev++] = phase;
  h->cur_phase = phase;
}

// After a stream synchronisation: fold the completed intervals; the last
// marker stays open.
void phase_fold(rh_handle* h) {
  if (!h->phases_on || h->npev < 2) return;
  for (int i = 0; i + 1 < h->npev; ++i) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, h->pev[i], h->pev[i + 1]) == hipSuccess) h->pms[h->pph[i]] += ms;
  }
  std::swap(h->pev[0], h->pev[h->npev - 1]);
  h->pph[0] = h->pph[h->npev - 1];
  h->npev = 1;
  (void)hipGetLastError();
}

// After `end` has completed: close the open interval at `end`.
void phase_close(rh_handle* h, hipEvent_t end) {
  phase_fold(h);
  if (h->phases_on && h->npev == 1) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, h->pev[0], end) == hipSuccess) h->pms[h->pph[0]] += ms;
    (void)hipGetLastError();
  }
  h->npev = 0;
  h->cur_phase = -1;
  h->phases_on = false;
}

rh_status sync_reductions(rh_handle* h, unsigned mask) {
  {
    Timed tm(h, KK_FINALIZE);
    launch_finalize(h->stream, h->part, h->hred_dev, mask);
  }
  HIPCHK(hipGetLastError());
  // the results are in host memory once the stream has drained
  HIPCHK(hipStreamSynchronize(h->stream));
  if (h->timing) flush_timing(h);
  phase_fold(h);
  return RH_OK;
}

double nvars(const rh_handle* h) { return h->p.isothermal ? 2.0 : 3.0; }

rh_status plan_blocks(rh_handle* h, const double* src);

// Per-step setup: U^n copies are already in En/en/nn.
// Face coefficients, constant part of f_E and E_s of a step from U^n (the
// handle's copy unless En / nn are given; y1n, y2n: helium of a multigroup
// step), the coarse face coefficients and the source boxes.
rh_status setup_step(rh_handle* h, StepK& k, const double* src, const double* En = nullptr,
                     const double* nn = nullptr, const double* y1n = nullptr,
                     const double* y2n = nullptr) {
  const bool mixed = h->p.precision == RH_PREC_MIXED;
  phase_mark(h, PH_SETUP);
  Op16* op32 = mixed ? h->L32[0].op : nullptr;
  {
    Timed tm0(h, KK_SETUP);
    launch_step_setup(h->stream, k, En ? En : h->En, nn ? nn : h->nn, y1n, y2n, src, h->cf64[0],
                      h->cf64[1], h->cf64[2], op32, h->rhsn, h->part);
  }
  HIPCHK(hipGetLastError());
  rh_status st = sync_reductions(h, kAllSlots);
  if (st != RH_OK) return st;
  if (h->hred[RS_NONFINITE] != 0.0) return fail(h, RH_ENONFINITE, "non-finite E^n, n_HI^n or src");
  k.E_s = std::max(std::max(h->hred[RS_EMAX], k.dt * h->hred[RS_SMAX]), h->p.E_floor);
  h->last_E_s = k.E_s;
  // coarse face coefficients
  for (int l = 1; l < h->plan.nlev; ++l) {
    if (mixed)
      launch_coarsen_faces<float>(h->stream, h->L32[l - 1], h->L32[l]);
    else
      launch_coarsen_faces<double>(h->stream, h->L64[l - 1], h->L64[l]);
    HIPCHK(hipGetLastError());
  }
  return plan_blocks(h, src);
}

// Two boxes (corners a, b; extents e) touch or overlap along an axis of n
// cells when their distance is at most e (periodic axes: either way round).
bool boxes_meet_1d(int a, int b, int e, int n, bool per) {
  int d = std::abs(a - b);
  if (per) d = std::min(d, n - d);
  return d <= e;
}

// Boxes of the block smoother for this step: the source cells (src > 0),
// on each level with boxes the coarse cells that contain them, one box of
// radius R around each (shifted inwards so it never wraps), coloured
// greedily in cell order so that boxes of one colour neither overlap nor
// touch.  No boxes (this step) when there are no sources or more than
// mg_block_max of them.
rh_status plan_blocks(rh_handle* h, const double* src) {
  h->nblk = 0;
  const rh_params& p = h->p;
  const int R = p.mg_block_radius;
  const int blevels = R > 0 ? std::min(p.mg_block_levels, h->plan.nlev - 1) : 0;
  h->nsrc = 0;
  if (blevels == 0) return RH_OK;
  const bool mixed = p.precision == RH_PREC_MIXED;
  const int G = h->src_groups;
  launch_src_count(h->stream, h->N, h->src_chunk, G, src, h->src_count);
  HIPCHK(hipGetLastError());
  std::vector<int> cnt(G), off(G);
  HIPCHK(hipMemcpyAsync(cnt.data(), h->src_count, sizeof(int) * G, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  long long total = 0;
  for (int g = 0; g < G; ++g) {
    off[g] = (int)total;
    total += cnt[g];
  }
  h->nsrc = (int)std::min<long long>(total, INT32_MAX);
  if (total == 0 || total > block_capacity(p)) return RH_OK;
  HIPCHK(hipMemcpyAsync(h->src_offset, off.data(), sizeof(int) * G, hipMemcpyHostToDevice, h->stream));
  launch_src_list(h->stream, h->N, h->src_chunk, G, src, h->src_offset, h->src_list);
  HIPCHK(hipGetLastError());
  std::vector<int> cells((size_t)total);
  HIPCHK(hipMemcpyAsync(cells.data(), h->src_list, sizeof(int) * total, hipMemcpyDeviceToHost,
                        h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  const int per[3] = {p.bc[0] == RH_BC_PERIODIC, p.bc[2] == RH_BC_PERIODIC, p.bc[4] == RH_BC_PERIODIC};
  for (int l = 0; l < blevels; ++l) {
    const int* n = h->plan.dims[l];
    int e[3];
    for (int a = 0; a < 3; ++a) e[a] = std::min(2 * R + 1, n[a]);
    // coarse cells of the sources, unique, in cell order
    std::vector<long long> cen;
    cen.reserve(cells.size());
    for (int c : cells) {
      const long long i = c / ((long long)p.ny * p.nz), j = (c / p.nz) % p.ny, k = c % p.nz;
      cen.push_back(((i >> l) * n[1] + (j >> l)) * n[2] + (k >> l));
    }
    std::sort(cen.begin(), cen.end());
    cen.erase(std::unique(cen.begin(), cen.end()), cen.end());
    const int nb = (int)cen.size();
    std::vector<int> st(3 * (size_t)nb);
    for (int b = 0; b < nb; ++b) {
      const long long c[3] = {cen[b] / ((long long)n[1] * n[2]), (cen[b] / n[2]) % n[1],
                              cen[b] % n[2]};
      for (int a = 0; a < 3; ++a)
        st[3 * b + a] = (int)std::min<long long>(std::max<long long>(c[a] - R, 0), n[a] - e[a]);
    }
    // greedy colouring through bins of width 2R + 2 (boxes in bins further
    // apart along an axis cannot meet along it)
    const int W = 2 * R + 2;
    int nbin[3];
    for (int a = 0; a < 3; ++a) nbin[a] = (n[a] + W - 1) / W;
    std::vector<std::vector<int>> bins((size_t)nbin[0] * nbin[1] * nbin[2]);
    std::vector<int> colour(nb, -1);
    int ncol = 0;
    for (int b = 0; b < nb; ++b) {
      int bb[3];
      for (int a = 0; a < 3; ++a) bb[a] = st[3 * b + a] / W;
      unsigned long long used = 0;
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dz = -1; dz <= 1; ++dz) {
            int q[3] = {bb[0] + dx, bb[1] + dy, bb[2] + dz};
            bool ok = true;
            for (int a = 0; a < 3; ++a) {
              if (q[a] < 0 || q[a] >= nbin[a]) {
                if (!per[a]) ok = false;
                q[a] = (q[a] + nbin[a]) % nbin[a];
              }
            }
            if (!ok) continue;
            for (int o : bins[((size_t)q[0] * nbin[1] + q[1]) * nbin[2] + q[2]]) {
              bool meet = true;
              for (int a = 0; a < 3; ++a)
                meet = meet && boxes_meet_1d(st[3 * b + a], st[3 * o + a], e[a], n[a], per[a]);
              if (meet && colour[o] < 64) used |= 1ull << colour[o];
            }
          }
      int c = 0;
      while (c < 64 && ((used >> c) & 1ull)) ++c;
      if (c == 64) return fail(h, RH_EINVAL, "block smoother: more than 64 box colours");
      colour[b] = c;
      ncol = std::max(ncol, c + 1);
      // the periodic wrap of the bins can map two neighbour offsets to one
      // bin: each box is inserted once and tested against every box there
      bins[((size_t)bb[0] * nbin[1] + bb[1]) * nbin[2] + bb[2]].push_back(b);
    }
    // boxes ordered by colour
    std::vector<int> sorted(3 * (size_t)nb);
    std::vector<int>& offc = h->bcolour[l];
    offc.assign(ncol + 1, 0);
    for (int b = 0; b < nb; ++b) ++offc[colour[b] + 1];
    for (int c = 0; c < ncol; ++c) offc[c + 1] += offc[c];
    std::vector<int> fill(offc.begin(), offc.end() - 1);
    for (int b = 0; b < nb; ++b) {
      const int dst = fill[colour[b]]++;
      for (int a = 0; a < 3; ++a) sorted[3 * dst + a] = st[3 * b + a];
    }
    HIPCHK(hipMemcpyAsync(h->bstart[l], sorted.data(), sizeof(int) * 3 * nb, hipMemcpyHostToDevice,
                          h->stream));
    // the host vectors must outlive the copy
    HIPCHK(hipStreamSynchronize(h->stream));
    if (mixed) {
      BlockSet<float>& B = h->B32[l];
      B.n = nb; B.ex = e[0]; B.ey = e[1]; B.ez = e[2]; B.m = e[0] * e[1] * e[2];
      B.start = h->bstart[l];
    } else {
      BlockSet<double>& B = h->B64[l];
      B.n = nb; B.ex = e[0]; B.ey = e[1]; B.ez = e[2]; B.m = e[0] * e[1] * e[2];
      B.start = h->bstart[l];
    }
    h->nblk = l + 1;
  }
  return RH_OK;
}

struct EvalOut {
  double norm, rmax;
  bool finite, local_ok;
};

// Local solve (mode 0) or evaluation (mode 1) followed by the radiation residual.
rh_status eval_state(rh_handle* h, const StepK& k, const StateBuf& cur, const double* dE,
                     double lam, const StateBuf& out, bool predictor, const double* nH, int mode,
                     double* fE_out, double* fe_out, double* fn_out, EvalOut& res) {
  phase_mark(h, PH_EVAL);
  LocalArgs a{};
  a.Ek = cur.E; a.dE = dE; a.lam = lam;
  a.ek = cur.e; a.nk = cur.n;
  if (predictor) {
    a.pBCn = cur.loc[0]; a.pBCe = cur.loc[1]; a.pBfn = cur.loc[2]; a.pBfe = cur.loc[3];
  }
  a.En = h->En; a.en = h->en; a.nn = h->nn; a.nH = nH;
  a.Et = out.E; a.et = out.e; a.nt = out.n;
  a.BCn = out.loc[0]; a.BCe = out.loc[1]; a.Bfn = out.loc[2]; a.Bfe = out.loc[3];
  a.fn_out = fn_out; a.fe_out = fe_out;
  a.mode = mode;
  {
    Timed tm(h, KK_LOCAL);
    launch_local(h->stream, k, a, h->part);
  }
  HIPCHK(hipGetLastError());
  ResidArgs r{};
  r.E = mode == 0 ? out.E : cur.E;
  r.n = mode == 0 ? out.n : cur.n;
  r.En = h->En; r.nn = h->nn;
  for (int d = 0; d < 3; ++d) r.cf[d] = h->cf64[d];
  r.rhsn = h->rhsn;
  r.BCn = out.loc[0]; r.Bfn = out.loc[2];
  r.rS = h->rS; r.diag64 = h->diag64;
  r.op32 = h->p.precision == RH_PREC_MIXED ? h->L32[0].op : nullptr;
  r.fE_out = fE_out;
  {
    Timed tm(h, KK_RESID);
    launch_residual(h->stream, k, r, h->part);
  }
  HIPCHK(hipGetLastError());
  rh_status st = sync_reductions(h, kAllSlots);
  if (st != RH_OK) return st;
  const double* v = h->hred;
  const double s = v[RS_FE2] + v[RS_FN2] + (h->p.isothermal ? 0.0 : v[RS_FE_LOC2]);
  res.norm = std::sqrt(s / (h->N * nvars(h)));
  res.rmax = v[RS_RMAX];
  res.finite = std::isfinite(res.norm) && v[RS_NONFINITE] == 0.0 && v[RS_BAD_RES] == 0.0 &&
               std::isfinite(res.rmax);
  res.local_ok = v[RS_LOCAL_FAIL] == 0.0;
  h->local_its_max = std::max(h->local_its_max, (int)v[RS_LOCAL_ITS]);
  return RH_OK;
}

// ---------------------------------------------------------------------------
// multigrid
// ---------------------------------------------------------------------------
template <class T>
LevelK<T>* levels(rh_handle* h);
template <>
LevelK<float>* levels<float>(rh_handle* h) { return h->L32; }
template <>
LevelK<double>* levels<double>(rh_handle* h) { return h->L64; }
template <class T>
T* coarse_inverse(rh_handle* h);
template <>
float* coarse_inverse<float>(rh_handle* h) { return h->cInv32; }
template <>
double* coarse_inverse<double>(rh_handle* h) { return h->cInv64; }

template <class T>
BlockSet<T>* block_sets(rh_handle* h);
template <>
BlockSet<float>* block_sets<float>(rh_handle* h) { return h->B32; }
template <>
BlockSet<double>* block_sets<double>(rh_handle* h) { return h->B64; }

template <class T>
rh_status coarse_setup(rh_handle* h) {
  LevelK<T>* L = levels<T>(h);
  phase_mark(h, PH_COARSE);
  {
    Timed tm(h, KK_COARSE);
    for (int l = 1; l < h->plan.nlev; ++l) launch_coarse_diag<T>(h->stream, L[l - 1], L[l]);
    launch_coarsest_inverse<T>(h->stream, L[h->plan.nlev - 1], h->cA, h->cInv,
                               coarse_inverse<T>(h));
  }
  HIPCHK(hipGetLastError());
  // the block smoother's box inverses from this Newton iteration's operator
  BlockSet<T>* B = block_sets<T>(h);
  for (int l = 0; l < h->nblk; ++l) {
    Timed tm(h, KK_BLOCKINV);
    launch_block_inverse<T>(h->stream, L[l], B[l]);
  }
  HIPCHK(hipGetLastError());
  return RH_OK;
}

// Block relaxation on level l's boxes, colour by colour (forward before
// coarsening, reversed after it: the cycle stays symmetric).
template <class T>
void block_relax(rh_handle* h, int l, bool forward) {
  if (l >= h->nblk) return;
  const BlockSet<T>& B = block_sets<T>(h)[l];
  const std::vector<int>& off = h->bcolour[l];
  const int nc = (int)off.size() - 1;
  for (int i = 0; i < nc; ++i) {
    const int c = forward ? i : nc - 1 - i;
    Timed tm(h, l == 0 ? KK_BLOCK0 : KK_COARSE);
    launch_block_relax<T>(h->stream, levels<T>(h)[l], B, off[c], off[c + 1] - off[c]);
  }
}

// One red-black sweep on level l: fused (x -> x2, then swap) when the level
// fits the marching tiles, else colour by colour in place.
// last: the last sweep of the V-cycle on this level; on the finest level it
// takes over the conjugate-gradient dot products when the caller asked for
// them (h->dots) and the sweep is fused
template <class T>
void sweep(rh_handle* h, int l, int first_color, int zero_init, bool last = false) {
  LevelK<T>* L = levels<T>(h);
  // auto: the fused sweep where it gets at least one workgroup per CU, with
  // the longest chunks (up to 32 planes: least re-staging of each chunk's
  // boundary planes) that keep that many (measured on 128^3: 24.6 us against
  // 2 x 23 us for the two colour launches; 64^3 levels stay per colour)
  const long long min_tiles = h->p.smoother == 2 ? 1 : 256;
  if (h->p.smoother != 1 && rbgs_march_fits<T>(L[l], min_tiles)) {
    const bool dots = l == 0 && last && h->dots_wanted;
    if (dots) {
      Timed tm(h, KK_RBGS0D);
      h->dots_done = launch_rbgs_march<T>(h->stream, L[l], first_color, zero_init, 1, min_tiles,
                                          &h->dots);
    }
    if (!h->dots_done || !dots) {
      Timed tm(h, l == 0 ? KK_RBGS0 : KK_COARSE);
      launch_rbgs_march<T>(h->stream, L[l], first_color, zero_init, l == 0, min_tiles, nullptr);
    }
    std::swap(L[l].x, L[l].x2);
    return;
  }
  const int kr = l == 0 ? KK_RBGS0C : KK_COARSE;
  { Timed tm(h, kr); launch_rbgs<T>(h->stream, L[l], first_color, zero_init, l == 0); }
  { Timed tm(h, kr); launch_rbgs<T>(h->stream, L[l], 1 - first_color, 0, l == 0); }
}

// Residual of level l restricted into the right-hand side of level l+1: one
// fused launch where the level takes the marching sweep, else two.
template <class T>
void residual_restrict(rh_handle* h, int l) {
  LevelK<T>* L = levels<T>(h);
  const long long min_tiles = h->p.smoother == 2 ? 1 : 512;
  if (h->p.smoother != 1 && resid_restrict_fits<T>(L[l], min_tiles)) {
    Timed tm(h, l == 0 ? KK_MGRES0 : KK_COARSE);
    launch_resid_restrict_march<T>(h->stream, L[l], L[l + 1], min_tiles);
    return;
  }
  { Timed tm(h, l == 0 ? KK_MGRES0 : KK_COARSE); launch_mg_residual<T>(h->stream, L[l]); }
  { Timed tm(h, l == 0 ? KK_RESTRICT0 : KK_COARSE); launch_restrict<T>(h->stream, L[l], L[l + 1]); }
}

template <class T>
void vcycle(rh_handle* h, int l) {
  LevelK<T>* L = levels<T>(h);
  hipStream_t s = h->stream;
  if (l == h->plan.nlev - 1) {
    Timed tm(h, KK_COARSE);
    launch_coarsest_solve<T>(s, L[l], coarse_inverse<T>(h));
    return;
  }
  // red first on the way down, black first on the way up, and the source
  // boxes after the pre-smoothing and before the post-smoothing: the cycle
  // is symmetric
  for (int it = 0; it < h->p.mg_pre; ++it) sweep<T>(h, l, 0, it == 0);
  block_relax<T>(h, l, true);
  residual_restrict<T>(h, l);
  vcycle<T>(h, l + 1);
  { Timed tm(h, l == 0 ? KK_PROLONG0 : KK_COARSE); launch_prolong<T>(s, L[l + 1], L[l]); }
  block_relax<T>(h, l, false);
  for (int it = 0; it < h->p.mg_post; ++it) sweep<T>(h, l, 1, 0, it == h->p.mg_post - 1);
}

// Defect correction: S dE = rS with V-cycles in T and FP64 residuals.
// Stops when the weighted norm sqrt(sum (r/E_s)^2 / (N nvars)) <= target_w,
// or the plain ||r||_2 <= target_2, or on stagnation, or after max_it.
// On return *dE_final points at the solution.
template <class T>
rh_status linear_solve(rh_handle* h, const StepK& k, double rmax0, double target_w,
                       double target_2, int max_it, double** dE_final, int* its_out,
                       double* w_out, double* l2_out, bool* reached) {
  LevelK<T>* L = levels<T>(h);
  rh_status st = RH_OK;
  if (!h->keep_coarse && (st = coarse_setup<T>(h)) != RH_OK) return st;
  double* dE_in = h->dEa;
  double* dE_out = h->dEb;
  *its_out = 0;
  *reached = true;
  if (rmax0 == 0.0) {
    HIPCHK(hipMemsetAsync(dE_in, 0, sizeof(double) * h->N, h->stream));
    *dE_final = dE_in;
    *w_out = 0.0;
    *l2_out = 0.0;
    return RH_OK;
  }
  double sigma_b = rmax0, rmax_cur = rmax0;
  phase_mark(h, PH_OUTER);
  launch_cast_scale<T>(h->stream, h->N, h->rS, 1.0 / sigma_b, L[0].b);
  HIPCHK(hipGetLastError());
  bool first = true;
  double prev = INFINITY;
  int slow = 0;
  double w = INFINITY, l2 = INFINITY;
  for (int j = 1; j <= max_it; ++j) {
    phase_mark(h, PH_VCYCLE);
    vcycle<T>(h, 0);
    phase_mark(h, PH_OUTER);
    DefectArgs a{};
    a.rS = h->rS; a.dE_in = dE_in; a.dE_out = dE_out;
    a.diag64 = h->diag64;
    for (int d = 0; d < 3; ++d) a.cf[d] = h->cf64[d];
    a.first = first ? 1 : 0;
    a.sigma_x = sigma_b;
    a.inv_sigma_b = 1.0 / rmax_cur;
    {
      Timed tm(h, KK_DEFECT);
      launch_accum_defect<T>(h->stream, k, a, L[0].x, L[0].b, h->part);
    }
    HIPCHK(hipGetLastError());
    sigma_b = rmax_cur;
    st = sync_reductions(h, kAllSlots);
    if (st != RH_OK) return st;
    std::swap(dE_in, dE_out);
    first = false;
    *its_out = j;
    w = std::sqrt(h->hred[RS_FE2] / (h->N * nvars(h)));
    l2 = std::sqrt(h->hred[RS_R2]);
    rmax_cur = h->hred[RS_RMAX];
    if (!std::isfinite(w) || !std::isfinite(l2))
      return fail(h, RH_ELINEAR, "non-finite linear residual");
    if (w <= target_w || l2 <= target_2 || rmax_cur == 0.0) break;
    slow = (w > 0.9 * prev) ? slow + 1 : 0;
    if (slow >= 3) break;  // stagnated at the rounding floor
    prev = w;
  }
  *reached = w <= target_w || l2 <= target_2 || rmax_cur == 0.0;
  *dE_final = dE_in;
  *w_out = w;
  *l2_out = l2;
  return RH_OK;
}

// Flexible preconditioned conjugate gradients on S x = rS in FP64 with one
// V-cycle in T as the preconditioner (the symmetric V-cycle makes plain CG
// valid in exact arithmetic; the flexible beta absorbs FP32 rounding).
// One V-cycle as the preconditioner (z_T = V(b)).  The partial sums of z.r
// and z.q (z = sigma z_T; q may be NULL) come from the V-cycle's last sweep
// on the finest level when that sweep is fused, else from a pass of their own.
template <class T>
void precondition(rh_handle* h, const StepK& k, double sigma, const double* q) {
  h->dots = SweepDots{sigma, h->r64, q, h->part};
  h->dots_wanted = true;
  h->dots_done = false;
  phase_mark(h, PH_VCYCLE);
  vcycle<T>(h, 0);
  phase_mark(h, PH_OUTER);
  h->dots_wanted = false;
  if (!h->dots_done) {
    Timed tm(h, KK_PCG_PRE);
    launch_pcg_precond<T>(h->stream, k, sigma, levels<T>(h)[0].x, h->r64, q, h->part);
  }
}

template <class T>
rh_status pcg_solve(rh_handle* h, const StepK& k, double rmax0, double target_w, double target_2,
                    int max_it, double** x_final, int* its_out, double* w_out, double* l2_out,
                    bool* reached) {
  LevelK<T>* L = levels<T>(h);
  rh_status st = RH_OK;
  if (!h->keep_coarse && (st = coarse_setup<T>(h)) != RH_OK) return st;
  double* x = h->dEa;
  *its_out = 0;
  *x_final = x;
  *reached = true;
  if (rmax0 == 0.0) {
    HIPCHK(hipMemsetAsync(x, 0, sizeof(double) * h->N, h->stream));
    *w_out = 0.0;
    *l2_out = 0.0;
    return RH_OK;
  }
  phase_mark(h, PH_OUTER);
  HIPCHK(hipMemcpyAsync(h->r64, h->rS, sizeof(double) * h->N, hipMemcpyDeviceToDevice, h->stream));
  double sigma_b = rmax0;
  {
    Timed tm(h, KK_CAST);
    launch_cast_scale<T>(h->stream, h->N, h->r64, 1.0 / sigma_b, L[0].b);
  }
  precondition<T>(h, k, sigma_b, nullptr);
  HIPCHK(hipGetLastError());
  if ((st = sync_reductions(h, slot_bit(RS_ZR) | slot_bit(RS_ZQ))) != RH_OK) return st;
  double rz = h->hred[RS_ZR];
  double beta = 0.0, rmax_cur = rmax0;
  double w = INFINITY, l2 = INFINITY;
  double* p_in = h->pa;
  double* p_out = h->pb;
  const double* const cf[3] = {h->cf64[0], h->cf64[1], h->cf64[2]};
  // x += alpha_j p_j of an update is applied by the next direction kernel
  // (which reads p_j anyway) or, after the last update, by one axpy
  double alpha_prev = 0.0;
  bool pending = false;
  const double* p_last = nullptr;
  for (int j = 1; j <= max_it; ++j) {
    {
      Timed tm(h, KK_PCG_DIR);
      // z = sigma_b * (V-cycle output): sigma_b is still the scale of that V-cycle's input
      const XFold xf{x, alpha_prev, pending ? (j == 2 ? 1 : 2) : 0};
      launch_pcg_dir<T>(h->stream, k, h->diag64, cf, L[0].x, sigma_b, p_in, p_out, h->q64, beta,
                        j == 1, xf, h->part);
      pending = false;
    }
    HIPCHK(hipGetLastError());
    if ((st = sync_reductions(h, slot_bit(RS_PQ))) != RH_OK) return st;
    const double pq = h->hred[RS_PQ];
    if (!(pq > 0.0) || !std::isfinite(pq) || !(rz > 0.0)) {
      if (j == 1) return fail(h, RH_ELINEAR, "conjugate gradients broke down (S or V-cycle not positive)");
      break;
    }
    const double alpha = rz / pq;
    {
      Timed tm(h, KK_PCG_UPD);
      launch_pcg_update<T>(h->stream, k, alpha, p_out, h->q64, nullptr, h->r64, 1.0 / rmax_cur,
                           L[0].b, j == 1, h->part);
    }
    alpha_prev = alpha;
    pending = true;
    p_last = p_out;
    HIPCHK(hipGetLastError());
    sigma_b = rmax_cur;
    if ((st = sync_reductions(h, slot_bit(RS_FE2) | slot_bit(RS_R2) | slot_bit(RS_RMAX))) != RH_OK) return st;
    *its_out = j;
    w = std::sqrt(h->hred[RS_FE2] / (h->N * nvars(h)));
    l2 = std::sqrt(h->hred[RS_R2]);
    rmax_cur = h->hred[RS_RMAX];
    if (!std::isfinite(w) || !std::isfinite(l2))
      return fail(h, RH_ELINEAR, "non-finite linear residual");
    if (w <= target_w || l2 <= target_2 || rmax_cur == 0.0) break;
    precondition<T>(h, k, sigma_b, h->q64);
    HIPCHK(hipGetLastError());
    if ((st = sync_reductions(h, slot_bit(RS_ZR) | slot_bit(RS_ZQ))) != RH_OK) return st;
    const double rz_new = h->hred[RS_ZR];
    beta = -alpha * h->hred[RS_ZQ] / rz;
    rz = rz_new;
    std::swap(p_in, p_out);
  }
  if (pending) {
    Timed tm(h, KK_PCG_UPD);
    launch_xaxpy(h->stream, h->N, alpha_prev, p_last, x, *its_out == 1);
    HIPCHK(hipGetLastError());
  }
  *reached = w <= target_w || l2 <= target_2 || rmax_cur == 0.0;
  *w_out = w;
  *l2_out = l2;
  return RH_OK;
}

// Linear solve of the Schur system; *reached reports whether the stopping
// test was met (false: stopped at max_it, on stagnation or on a CG breakdown
// after the first iteration).
rh_status solve_linear(rh_handle* h, const StepK& k, double rmax0, double target_w,
                       double target_2, int max_it, double** dE_final, int* its, double* w,
                       double* l2, bool* reached) {
  const bool mixed = h->p.precision == RH_PREC_MIXED;
  if (h->p.krylov) {
    if (mixed)
      return pcg_solve<float>(h, k, rmax0, target_w, target_2, max_it, dE_final, its, w, l2, reached);
    return pcg_solve<double>(h, k, rmax0, target_w, target_2, max_it, dE_final, its, w, l2, reached);
  }
  if (mixed)
    return linear_solve<float>(h, k, rmax0, target_w, target_2, max_it, dE_final, its, w, l2, reached);
  return linear_solve<double>(h, k, rmax0, target_w, target_2, max_it, dE_final, its, w, l2, reached);
}

rh_status check_ptrs(rh_handle* h, std::initializer_list<const void*> ptrs) {
  for (const void* q : ptrs) {
    if (!q) return fail(h, RH_EINVAL, "NULL field pointer");
    if (reinterpret_cast<uintptr_t>(q) % 8 != 0) return fail(h, RH_EINVAL, "misaligned field pointer");
  }
  return RH_OK;
}

rh_status copy_state(rh_handle* h, double* E, double* e, double* n, const double* Es,
                     const double* es, const double* ns) {
  const size_t bytes = sizeof(double) * h->N;
  HIPCHK(hipMemcpyAsync(E, Es, bytes, hipMemcpyDeviceToDevice, h->stream));
  if (!h->p.isothermal) HIPCHK(hipMemcpyAsync(e, es, bytes, hipMemcpyDeviceToDevice, h->stream));
  HIPCHK(hipMemcpyAsync(n, ns, bytes, hipMemcpyDeviceToDevice, h->stream));
  return RH_OK;
}

}  // namespace

// Helpers of the handle-free entry point (rh_noalloc.hip).
namespace rh {

void flush_timing(rh_handle* h) {
  for (int i = 0; i < h->npool; ++i) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, h->eva[i], h->evb[i]) == hipSuccess) {
      h->kms[h->pkind[i]] += ms;
      h->kcount[h->pkind[i]] += 1;
    }
  }
  h->npool = 0;
  // a failed query must not surface later through hipGetLastError
  (void)hipGetLastError();
}

bool params_valid(const rh_params* p, char* err, size_t n) {
  std::string e;
  if (validate(p, e)) return true;
  std::snprintf(err, n, "%s", e.c_str());
  return false;
}
StepK step_scalars(const rh_params& p, double t_n, double dt) {
  return make_step_from(p, grey_constants(p), t_n, dt);
}
void set_last_error(const char* msg) { set_global_error(msg); }

// Helpers of the multigroup driver (rh_groups_host.cpp).
StepK handle_step(const rh_handle* h, double t_n, double dt) {
  return make_step_from(h->p, h->g, t_n, dt);
}
rh_status handle_setup_step(rh_handle* h, StepK& k, const double* src, const double* En,
                            const double* nn, const double* y1n, const double* y2n) {
  return setup_step(h, k, src, En, nn, y1n, y2n);
}
rh_status handle_reductions(rh_handle* h, unsigned mask) { return sync_reductions(h, mask); }
rh_status handle_solve(rh_handle* h, const StepK& k, double rmax0, double target_w,
                       double target_2, int max_it, double** x, int* its, double* w, double* l2,
                       bool* reached) {
  return solve_linear(h, k, rmax0, target_w, target_2, max_it, x, its, w, l2, reached);
}
double handle_nvars(const rh_handle* h) { return nvars(h); }
}  // namespace rh

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void rh_default_params(rh_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->nx = p->ny = p->nz = 16;
  for (int f = 0; f < 6; ++f) p->bc[f] = RH_BC_ZEROFLUX;
  p->box_comoving_cm = 6.6 * 3.0856775814913673e21;
  p->isothermal = 0;
  p->T_iso_K = 1.0e4;
  p->spectrum = RH_SPEC_BLACKBODY;
  p->T_bb_K = 1.0e5;
  p->hnu0_eV = 13.6;
  p->sigma0_cm2 = 6.3e-18;
  p->rates = RH_RATES_FIT;
  p->alphaB_const = 2.59e-13;
  p->cooling_mask = RH_COOL_RECB | RH_COOL_COLLEXC | RH_COOL_COMPTON;
  p->cosmology = RH_COSMO_STATIC;
  p->hubble_h = 0.7;
  p->Omega_m = 1.0;
  p->Omega_L = 0.0;
  p->theta = 1.0;
  p->E_floor = 1.0e-40;
  p->R_min = 0.0;
  p->gamma = 5.0 / 3.0;
  p->newton_tol = 1.0e-8;
  p->newton_max_it = 30;
  p->ls_max_cuts = 10;
  p->lin_forcing = 1.0e-13;
  p->lin_max_it = 500;
  p->precision = RH_PREC_FP64;
  p->mg_pre = 2;
  p->mg_post = 2;
  p->mg_coarse_max = 64;
  p->krylov = 1;
  p->smoother = 0;
  p->mg_block_radius = 2;
  p->mg_block_levels = 2;
  p->mg_block_max = 0;
}

size_t rh_workspace_bytes(const rh_params* p) {
  std::string err;
  if (!validate(p, err)) {
    set_global_error(err.c_str());
    return 0;
  }
  Plan pl;
  plan_levels(*p, pl, err);
  rh_handle tmp;
  return layout(&tmp, *p, pl, nullptr);
}

rh_status rh_setup(const rh_params* p, void* workspace, size_t ws_bytes, void* hip_stream,
                   rh_handle** out) {
  std::string err;
  if (!out) {
    set_global_error("out is NULL");
    return RH_EINVAL;
  }
  *out = nullptr;
  if (!validate(p, err)) {
    set_global_error(err.c_str());
    return RH_EINVAL;
  }
  const size_t need = rh_workspace_bytes(p);
  if (!workspace || ws_bytes < need) {
    set_global_error("workspace missing or smaller than rh_workspace_bytes");
    return workspace ? RH_ENOMEM : RH_EINVAL;
  }
  rh_handle* h = new rh_handle();
  h->p = *p;
  plan_levels(*p, h->plan, err);
  h->g = grey_constants(*p);
  h->h = p->box_comoving_cm / p->nx;
  h->compton = compton_coefficient();
  h->N = (long long)p->nx * p->ny * p->nz;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  h->ws = reinterpret_cast<char*>(workspace);
  h->ws_bytes = ws_bytes;
  char* base = reinterpret_cast<char*>(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
  layout(h, *p, h->plan, base);
  hipError_t e1 = hipGetDevice(&h->device);
  hipError_t e2 = hipHostMalloc(reinterpret_cast<void**>(&h->hred), sizeof(double) * RS_COUNT);
  if (e2 == hipSuccess)
    e2 = hipHostGetDevicePointer(reinterpret_cast<void**>(&h->hred_dev), h->hred, 0);
  hipError_t e3 = hipEventCreate(&h->ev0);
  hipError_t e4 = hipEventCreate(&h->ev1);
  int made = 0;
  while (made < rh_handle::kPhaseEv && e3 == hipSuccess &&
         (e3 = hipEventCreate(&h->pev[made])) == hipSuccess)
    ++made;
  h->phase_events = made == rh_handle::kPhaseEv;
  if (!h->phase_events)
    for (int i = 0; i < made; ++i) (void)hipEventDestroy(h->pev[i]);
  // no reducing kernel has run yet: every slot's block count is 0
  hipError_t e5 = hipMemsetAsync(h->part + (size_t)RS_COUNT * kPartCap, 0,
                                 sizeof(double) * RS_COUNT, h->stream);
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess ||
      e5 != hipSuccess) {
    const hipError_t es[5] = {e1, e2, e3, e4, e5};
    const char* what[5] = {"hipGetDevice", "hipHostMalloc / hipHostGetDevicePointer",
                           "hipEventCreate", "hipEventCreate",
                           "hipMemsetAsync (reduction counts)"};
    int i = 0;
    while (es[i] == hipSuccess) ++i;
    set_global_error((std::string("HIP initialisation failed: ") + what[i] + ": " +
                      hipGetErrorString(es[i])).c_str());
    delete h;
    return RH_EHIP;
  }
  *out = h;
  return RH_OK;
}

rh_status rh_implicit_step(rh_handle* h, double t_n, double dt, const double* nH, const double* src,
                           double* E, double* e, double* nHI, rh_step_stats* stats) {
  if (!h) return RH_EINVAL;
  const bool iso = h->p.isothermal != 0;
  rh_status st = check_ptrs(h, {nH, src, E, nHI});
  if (st != RH_OK) return st;
  if (!iso && (st = check_ptrs(h, {e})) != RH_OK) return st;
  if (!(dt > 0) || !std::isfinite(dt) || !std::isfinite(t_n))
    return fail(h, RH_EINVAL, "dt must be > 0 and t finite");
  if (h->p.cosmology != RH_COSMO_STATIC && !(t_n > 0))
    return fail(h, RH_EINVAL, "expanding cosmology needs t > 0");
  h->lin_its = 0;
  h->local_its_max = 0;
  h->lin_res_max = 0.0;
  h->lin_cap_hits = 0;
  h->lin_its_max = 0;
  StepMarks marks(h, "rh_implicit_step");
  HIPCHK(hipEventRecord(h->ev0, h->stream));
  phase_begin(h);
  phase_mark(h, PH_SETUP);
  StepK k = make_step(h, t_n, dt);
  if ((st = copy_state(h, h->En, h->en, h->nn, E, e, nHI)) != RH_OK) return st;
  if ((st = setup_step(h, k, src)) != RH_OK) return st;

  StateBuf A{E, iso ? nullptr : e, nHI, {h->locA[0], h->locA[1], h->locA[2], h->locA[3]}};
  StateBuf B = h->B;
  if (iso) B.e = nullptr;
  StateBuf* cur = &A;
  StateBuf* oth = &B;
  EvalOut ev{};
  int newton_its = 0, cuts = 0;
  double res0 = 0.0;
  rh_status result = RH_OK;
  // local solve at E = E^n
  st = eval_state(h, k, *cur, nullptr, 0.0, *oth, false, nH, 0, nullptr, nullptr, nullptr, ev);
  if (st != RH_OK) return st;
  std::swap(cur, oth);
  res0 = ev.norm;
  for (;;) {
    if (!ev.finite) { result = fail(h, RH_ENONFINITE, "non-finite residual"); break; }
    if (!ev.local_ok) { result = fail(h, RH_ELINEAR, "local per-cell solve did not converge"); break; }
    if (ev.norm <= h->p.newton_tol) break;
    if (newton_its >= h->p.newton_max_it) {
      char buf[160];
      std::snprintf(buf, sizeof buf, "Newton did not converge in %d iterations (||f|| = %.3e)",
                    newton_its, ev.norm);
      result = fail(h, RH_ENEWTON, buf);
      break;
    }
    double* dE = nullptr;
    int its = 0;
    double w = 0, l2 = 0;
    bool reached = true;
    st = solve_linear(h, k, ev.rmax, h->p.lin_forcing * ev.norm, 0.0, h->p.lin_max_it, &dE, &its,
                      &w, &l2, &reached);
    if (st != RH_OK) { result = st; break; }
    h->lin_its += its;
    h->lin_its_max = std::max(h->lin_its_max, its);
    if (!reached) ++h->lin_cap_hits;
    if (ev.norm > 0) h->lin_res_max = std::max(h->lin_res_max, w / ev.norm);
    ++newton_its;
    const double f0 = ev.norm;
    double lam = 1.0;
    bool accepted = false;
    for (int c = 0; c <= h->p.ls_max_cuts; ++c) {
      st = eval_state(h, k, *cur, dE, lam, *oth, true, nH, 0, nullptr, nullptr, nullptr, ev);
      if (st != RH_OK) return st;
      if (ev.finite && ev.local_ok && ev.norm <= (1.0 - 1e-4 * lam) * f0) {
        accepted = true;
        break;
      }
      lam *= 0.5;
      ++cuts;
    }
    if (!accepted) {
      result = fail(h, RH_ENEWTON, "line search failed");
      break;
    }
    std::swap(cur, oth);
  }
  phase_mark(h, PH_SETUP);
  if (result == RH_OK) {
    if (cur->E != E) {
      if ((st = copy_state(h, E, e, nHI, cur->E, cur->e, cur->n)) != RH_OK) return st;
    }
  } else {
    if ((st = copy_state(h, E, e, nHI, h->En, h->en, h->nn)) != RH_OK) return st;
  }
  HIPCHK(hipEventRecord(h->ev1, h->stream));
  HIPCHK(hipEventSynchronize(h->ev1));
  phase_close(h, h->ev1);
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->newton_its = newton_its;
    stats->lin_its_total = h->lin_its;
    stats->ls_cuts = cuts;
    stats->local_its_max = h->local_its_max;
    stats->res0 = res0;
    stats->res_final = ev.norm;
    stats->lin_res_max = h->lin_res_max;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, h->ev0, h->ev1);
    stats->t_ms[0] = ms;
    for (int q = 1; q <= 5; ++q) stats->t_ms[q] = h->pms[q];
    stats->lin_cap_hits = h->lin_cap_hits;
    stats->lin_its_max = h->lin_its_max;
    stats->source_boxes = h->nblk > 0 ? h->B32[0].n + h->B64[0].n : 0;
  }
  return result;
}

rh_status rh_advance(rh_handle* h, double t0, double t_end, double dt0, double tau_tol,
                     double dt_max, const double* nH, const double* src, double* E, double* e,
                     double* nHI, rh_advance_stats* stats, double* t_reached) {
  if (!h) return RH_EINVAL;
  const bool iso = h->p.isothermal != 0;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (t_reached) *t_reached = t0;
  if (!std::isfinite(t0) || !std::isfinite(t_end) || !(t_end > t0) || !(dt0 > 0) ||
      !(tau_tol > 0) || !(dt_max > 0))
    return fail(h, RH_EINVAL, "need t_end > t0 and dt0, tau_tol, dt_max > 0");
  const double eps_t = 1e-12 * std::max(std::fabs(t_end), t_end - t0);
  constexpr int kMaxRejects = 12;
  double t = t0, dt = std::min(dt0, dt_max);
  double dt_min_acc = INFINITY, dt_max_acc = 0.0;
  int rejects = 0;
  rh_advance_stats acc{};
  while (t_end - t > eps_t) {
    const bool last = dt >= t_end - t - eps_t;
    const double dt_try = last ? t_end - t : dt;
    rh_step_stats ss{};
    rh_status why = rh_implicit_step(h, t, dt_try, nH, src, E, e, nHI, &ss);
    if (why != RH_OK && why != RH_ENEWTON && why != RH_ELINEAR && why != RH_ENONFINITE)
      return why;  // invalid arguments or a HIP error: no retry
    double w = 0.0;
    if (why == RH_OK) {
      // h->En / en / nn still hold U^n of this step
      launch_change_norm(h->stream, h->N, h->last_E_s, E, iso ? nullptr : e, nHI, h->En,
                         iso ? nullptr : h->en, h->nn, nH, h->part);
      HIPCHK(hipGetLastError());
      rh_status st = sync_reductions(h, slot_bit(RS_CHG2) | slot_bit(RS_NEGE));
      if (st != RH_OK) return st;
      w = std::sqrt(h->hred[RS_CHG2] / (h->N * nvars(h)));
      if (h->hred[RS_NEGE] > 1e-10 || !std::isfinite(w)) {
        // negative E (or a non-finite change): back to U^n
        if ((st = copy_state(h, E, e, nHI, h->En, h->en, h->nn)) != RH_OK) return st;
        HIPCHK(hipStreamSynchronize(h->stream));
        why = RH_ENONFINITE;
      }
    }
    if (why != RH_OK) {
      ++acc.rejected;
      if (++rejects >= kMaxRejects) {
        if (stats) *stats = acc;
        if (t_reached) *t_reached = t;
        return fail(h, why, "rh_advance: step rejected 12 times in a row");
      }
      dt = 0.5 * dt_try;
      continue;
    }
    rejects = 0;
    t = last ? t_end : t + dt_try;
    ++acc.steps;
    acc.newton_its += ss.newton_its;
    acc.lin_its_total += ss.lin_its_total;
    dt_min_acc = std::min(dt_min_acc, dt_try);
    dt_max_acc = std::max(dt_max_acc, dt_try);
    acc.change_max = std::max(acc.change_max, w);
    acc.change_last = w;
    const double factor = w > 0.0 ? std::min(2.0, std::max(0.1, tau_tol / w)) : 2.0;
    dt = std::min(dt_try * factor, dt_max);
  }
  acc.dt_min = dt_min_acc;
  acc.dt_max = dt_max_acc;
  acc.dt_next = dt;
  if (stats) *stats = acc;
  if (t_reached) *t_reached = t;
  return RH_OK;
}

rh_status rh_advect(rh_handle* h, double t0, double dt, const double* vx, const double* vy,
                    const double* vz, double cfl, double* nH, double* E, double* e, double* nHI,
                    rh_advect_stats* stats) {
  if (!h) return RH_EINVAL;
  const bool iso = h->p.isothermal != 0;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  rh_status st = check_ptrs(h, {vx, vy, vz, nH, E, nHI});
  if (st != RH_OK) return st;
  if (!iso && (st = check_ptrs(h, {e})) != RH_OK) return st;
  if (!std::isfinite(t0) || !(dt > 0) || !std::isfinite(dt) || !(cfl > 0) || !(cfl <= 1))
    return fail(h, RH_EINVAL, "need finite t0, dt > 0 and 0 < cfl <= 1");
  {
    const void* fields[4] = {nH, E, nHI, iso ? nullptr : e};
    const void* vel[3] = {vx, vy, vz};
    for (int i = 0; i < 4; ++i)
      for (int j = i + 1; j < 4; ++j)
        if (fields[i] && fields[i] == fields[j])
          return fail(h, RH_EINVAL, "rh_advect: the advected fields must be distinct arrays");
    for (const void* v : vel)
      for (const void* f : fields)
        if (f && v == f) return fail(h, RH_EINVAL, "rh_advect: a velocity aliases an advected field");
  }
  AdvK a{};
  a.nx = h->p.nx; a.ny = h->p.ny; a.nz = h->p.nz;
  a.N = h->N;
  for (int f = 0; f < 6; ++f) a.bc[f] = h->p.bc[f];
  a.iso = iso ? 1 : 0;
  a.v[0] = vx; a.v[1] = vy; a.v[2] = vz;
  double a0, H0;
  cosmo_at(h->p, t0, a0, H0);
  a.scale = dt / (a0 * h->h);
  {
    Timed tm(h, KK_ADVECT_C);
    launch_advect_courant(h->stream, a, h->part);
  }
  HIPCHK(hipGetLastError());
  if ((st = sync_reductions(h, slot_bit(RS_COURANT) | slot_bit(RS_NONFINITE))) != RH_OK) return st;
  const double C = h->hred[RS_COURANT];
  if (h->hred[RS_NONFINITE] > 0 || !std::isfinite(C))
    return fail(h, RH_ENONFINITE, "rh_advect: non-finite velocity or Courant number");
  constexpr double kMaxSub = 1 << 20;
  const double msub = std::max(1.0, std::ceil(C / cfl));
  if (msub > kMaxSub) return fail(h, RH_EINVAL, "rh_advect: more than 2^20 substeps needed");
  const int m = (int)msub;
  const double ds = dt / m;
  // ping-pong between the caller's fields (A) and workspace buffers (B),
  // which are free between implicit steps
  double* A[4] = {nH, E, nHI, iso ? nullptr : e};
  double* B[4] = {h->dEa, h->B.E, h->B.n, iso ? nullptr : h->B.e};
  for (int sub = 0; sub < m; ++sub) {
    double a_mid, H_mid;
    cosmo_at(h->p, t0 + (sub + 0.5) * ds, a_mid, H_mid);
    a.scale = ds / (a_mid * h->h);
    double* const* from = (sub & 1) ? B : A;
    double* const* to = (sub & 1) ? A : B;
    for (int q = 0; q < 4; ++q) {
      a.qi[q] = from[q];
      a.qo[q] = to[q];
    }
    Timed tm(h, KK_ADVECT);
    launch_advect(h->stream, a);
  }
  HIPCHK(hipGetLastError());
  if (m & 1) {
    const size_t bytes = sizeof(double) * h->N;
    for (int q = 0; q < (iso ? 3 : 4); ++q)
      HIPCHK(hipMemcpyAsync(A[q], B[q], bytes, hipMemcpyDeviceToDevice, h->stream));
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  if (h->timing) flush_timing(h);
  if (stats) {
    stats->substeps = m;
    stats->courant = C;
    stats->courant_substep = C / m;
  }
  return RH_OK;
}

rh_status rh_residual(rh_handle* h, double t_n, double dt, const double* nH, const double* src,
                      const double* E_n, const double* e_n, const double* nHI_n, const double* E,
                      const double* e, const double* nHI, double* fE, double* fe, double* fn,
                      double* norm_out) {
  if (!h) return RH_EINVAL;
  const bool iso = h->p.isothermal != 0;
  rh_status st = check_ptrs(h, {nH, src, E_n, nHI_n, E, nHI});
  if (st != RH_OK) return st;
  if (!iso && (st = check_ptrs(h, {e_n, e})) != RH_OK) return st;
  if (!(dt > 0)) return fail(h, RH_EINVAL, "dt must be > 0");
  StepK k = make_step(h, t_n, dt);
  if ((st = copy_state(h, h->En, h->en, h->nn, E_n, e_n, nHI_n)) != RH_OK) return st;
  if ((st = setup_step(h, k, src)) != RH_OK) return st;
  StateBuf U{const_cast<double*>(E), iso ? nullptr : const_cast<double*>(e),
             const_cast<double*>(nHI), {h->locA[0], h->locA[1], h->locA[2], h->locA[3]}};
  EvalOut ev{};
  st = eval_state(h, k, U, nullptr, 0.0, U, false, nH, 1, fE, iso ? nullptr : fe, fn, ev);
  if (st != RH_OK) return st;
  if (norm_out) *norm_out = ev.norm;
  return RH_OK;
}

// Face limiter from U^n, then the local elimination and the Schur operator
// (diag64, cf64) at U; shared by rh_schur_solve and rh_schur_operator.
static rh_status schur_at(rh_handle* h, StepK& k, const double* nH, const double* src,
                          const double* E_n, const double* e_n, const double* nHI_n,
                          const double* E, const double* e, const double* nHI) {
  const bool iso = h->p.isothermal != 0;
  rh_status st;
  if ((st = copy_state(h, h->En, h->en, h->nn, E_n, e_n, nHI_n)) != RH_OK) return st;
  if ((st = setup_step(h, k, src)) != RH_OK) return st;
  StateBuf U{const_cast<double*>(E), iso ? nullptr : const_cast<double*>(e),
             const_cast<double*>(nHI), {h->locA[0], h->locA[1], h->locA[2], h->locA[3]}};
  EvalOut ev{};
  return eval_state(h, k, U, nullptr, 0.0, U, false, nH, 1, nullptr, nullptr, nullptr, ev);
}

rh_status rh_schur_operator(rh_handle* h, double t_n, double dt, const double* nH,
                            const double* src, const double* E_n, const double* e_n,
                            const double* nHI_n, const double* E, const double* e,
                            const double* nHI, double* diag, double* cf_x, double* cf_y,
                            double* cf_z) {
  if (!h) return RH_EINVAL;
  const bool iso = h->p.isothermal != 0;
  rh_status st = check_ptrs(h, {nH, src, E_n, nHI_n, E, nHI, diag, cf_x, cf_y, cf_z});
  if (st != RH_OK) return st;
  if (!iso && (st = check_ptrs(h, {e_n, e})) != RH_OK) return st;
  if (!(dt > 0)) return fail(h, RH_EINVAL, "dt must be > 0");
  StepK k = make_step(h, t_n, dt);
  if ((st = schur_at(h, k, nH, src, E_n, e_n, nHI_n, E, e, nHI)) != RH_OK) return st;
  const size_t bytes = sizeof(double) * h->N;
  HIPCHK(hipMemcpyAsync(diag, h->diag64, bytes, hipMemcpyDeviceToDevice, h->stream));
  double* out[3] = {cf_x, cf_y, cf_z};
  for (int d = 0; d < 3; ++d)
    HIPCHK(hipMemcpyAsync(out[d], h->cf64[d], bytes, hipMemcpyDeviceToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return RH_OK;
}

rh_status rh_schur_solve(rh_handle* h, double t_n, double dt, const double* nH, const double* src,
                         const double* E_n, const double* e_n, const double* nHI_n,
                         const double* E, const double* e, const double* nHI, const double* b,
                         double* x, double rel_tol, int32_t max_it, int32_t* iters,
                         double* rel_res) {
  if (!h) return RH_EINVAL;
  const bool iso = h->p.isothermal != 0;
  rh_status st = check_ptrs(h, {nH, src, E_n, nHI_n, E, nHI, b, x});
  if (st != RH_OK) return st;
  if (!iso && (st = check_ptrs(h, {e_n, e})) != RH_OK) return st;
  if (!(dt > 0) || !(rel_tol >= 0) || max_it < 1) return fail(h, RH_EINVAL, "bad dt / tol / max_it");
  StepK k = make_step(h, t_n, dt);
  if ((st = schur_at(h, k, nH, src, E_n, e_n, nHI_n, E, e, nHI)) != RH_OK) return st;
  // right-hand side b replaces the Schur right-hand side; its norms first
  HIPCHK(hipMemcpyAsync(h->rS, b, sizeof(double) * h->N, hipMemcpyDeviceToDevice, h->stream));
  DefectArgs a{};
  a.rS = h->rS; a.dE_in = nullptr; a.dE_out = h->dEb;
  a.diag64 = h->diag64;
  for (int d = 0; d < 3; ++d) a.cf[d] = h->cf64[d];
  a.first = 1; a.sigma_x = 0.0; a.inv_sigma_b = 0.0;
  if (h->p.precision == RH_PREC_MIXED)
    launch_accum_defect<float>(h->stream, k, a, nullptr, h->L32[0].r, h->part);
  else
    launch_accum_defect<double>(h->stream, k, a, nullptr, h->L64[0].r, h->part);
  HIPCHK(hipGetLastError());
  if ((st = sync_reductions(h, kAllSlots)) != RH_OK) return st;
  const double bnorm = std::sqrt(h->hred[RS_R2]);
  const double bmax = h->hred[RS_RMAX];
  double* dE = nullptr;
  int its = 0;
  double w = 0, l2 = 0;
  bool reached = true;
  st = solve_linear(h, k, bmax, 0.0, rel_tol * bnorm, max_it, &dE, &its, &w, &l2, &reached);
  if (st != RH_OK) return st;
  HIPCHK(hipMemcpyAsync(x, dE, sizeof(double) * h->N, hipMemcpyDeviceToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (iters) *iters = its;
  if (rel_res) *rel_res = bnorm > 0 ? l2 / bnorm : 0.0;
  return RH_OK;
}

rh_status rh_adjoint_step(rh_handle* h, double t_n, double dt, const double* nH,
                          const double* src, const double* E_n, const double* e_n,
                          const double* nHI_n, const double* E_1, const double* e_1,
                          const double* nHI_1, double* lE, double* le, double* lnHI,
                          double* g_src, double* g_nH, rh_step_stats* stats) {
  if (!h) return RH_EINVAL;
  const bool iso = h->p.isothermal != 0;
  rh_status st = check_ptrs(h, {nH, src, E_n, nHI_n, E_1, nHI_1, lE, lnHI, g_src, g_nH});
  if (st != RH_OK) return st;
  if (!iso && (st = check_ptrs(h, {e_n, e_1, le})) != RH_OK) return st;
  if (!(dt > 0) || !std::isfinite(dt) || !std::isfinite(t_n))
    return fail(h, RH_EINVAL, "dt must be > 0 and t finite");
  if (h->p.cosmology != RH_COSMO_STATIC && !(t_n > 0))
    return fail(h, RH_EINVAL, "expanding cosmology needs t > 0");
  h->lin_its = 0;
  h->local_its_max = 0;
  StepMarks marks(h, "rh_adjoint_step");
  HIPCHK(hipEventRecord(h->ev0, h->stream));
  phase_begin(h);
  phase_mark(h, PH_SETUP);
  StepK k = make_step(h, t_n, dt);
  // recompute the step's face limiter from U^n and the local terms and the
  // Schur operator at the converged U^{n+1}
  if ((st = copy_state(h, h->En, h->en, h->nn, E_n, e_n, nHI_n)) != RH_OK) return st;
  if ((st = setup_step(h, k, src)) != RH_OK) return st;
  StateBuf U{const_cast<double*>(E_1), iso ? nullptr : const_cast<double*>(e_1),
             const_cast<double*>(nHI_1), {h->locA[0], h->locA[1], h->locA[2], h->locA[3]}};
  EvalOut ev{};
  st = eval_state(h, k, U, nullptr, 0.0, U, false, nH, 1, nullptr, nullptr, nullptr, ev);
  if (st != RH_OK) return st;
  if (!ev.finite) return fail(h, RH_ENONFINITE, "non-finite state in the adjoint step");
  // S mu_E = lE - (B^-1 C)^T lambda_loc
  phase_mark(h, PH_OUTER);
  launch_adj_rhs(h->stream, k, lE, le, lnHI, h->locA[0], h->locA[1], h->rS, h->part);
  HIPCHK(hipGetLastError());
  if ((st = sync_reductions(h, kAllSlots)) != RH_OK) return st;
  const double rnorm = std::sqrt(h->hred[RS_R2]);
  const double rmax = h->hred[RS_RMAX];
  if (!std::isfinite(rnorm)) return fail(h, RH_ENONFINITE, "non-finite adjoint right-hand side");
  double* mu = nullptr;
  int its = 0;
  double w = 0, l2 = 0;
  bool reached = true;
  st = solve_linear(h, k, rmax, 0.0, h->p.lin_forcing * rnorm, h->p.lin_max_it, &mu, &its, &w,
                    &l2, &reached);
  if (st != RH_OK) return st;
  h->lin_its = its;
  if (!reached) {
    // no outer iteration corrects an inexact transpose solve: fail without
    // touching lE, le, lnHI, g_src, g_nH
    HIPCHK(hipStreamSynchronize(h->stream));
    h->phases_on = false;
    h->npev = 0;
    if (stats) {
      std::memset(stats, 0, sizeof(*stats));
      stats->lin_its_total = its;
      stats->lin_its_max = its;
      stats->lin_cap_hits = 1;
      stats->res0 = rnorm;
      stats->res_final = l2;
      stats->lin_res_max = rnorm > 0 ? l2 / rnorm : 0.0;
    }
    char buf[200];
    std::snprintf(buf, sizeof buf,
                  "adjoint linear solve stopped after %d cycles at relative residual %.3e "
                  "(target lin_forcing = %.1e; raise lin_max_it)", its,
                  rnorm > 0 ? l2 / rnorm : 0.0, h->p.lin_forcing);
    return fail(h, RH_ELINEAR, buf);
  }
  phase_mark(h, PH_EVAL);
  AdjArgs a{};
  a.E1 = E_1; a.e1 = iso ? nullptr : e_1; a.n1 = nHI_1;
  a.En = h->En; a.en = h->en; a.nn = h->nn;
  a.nH = nH; a.muE = mu;
  a.lE = lE; a.le = iso ? nullptr : le; a.ln = lnHI;
  a.g_src = g_src; a.g_nH = g_nH;
  launch_adj_local(h->stream, k, a);
  HIPCHK(hipGetLastError());
  launch_adj_limiter(h->stream, k, a);
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(h->ev1, h->stream));
  HIPCHK(hipEventSynchronize(h->ev1));
  phase_close(h, h->ev1);
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->lin_its_total = its;
    stats->lin_its_max = its;
    stats->res0 = rnorm;
    stats->res_final = l2;
    stats->lin_res_max = rnorm > 0 ? l2 / rnorm : 0.0;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, h->ev0, h->ev1);
    stats->t_ms[0] = ms;
    for (int q = 1; q <= 5; ++q) stats->t_ms[q] = h->pms[q];
  }
  return RH_OK;
}

rh_status rh_initial_state(rh_handle* h, const double* nH, double x0, double T0_K, double E0,
                           double* E, double* e, double* nHI) {
  if (!h) return RH_EINVAL;
  const bool iso = h->p.isothermal != 0;
  rh_status st = check_ptrs(h, {nH, E, nHI});
  if (st != RH_OK) return st;
  if (e && (st = check_ptrs(h, {e})) != RH_OK) return st;
  if (!iso && !e) return fail(h, RH_EINVAL, "e is required unless the run is isothermal");
  const double T = iso ? h->p.T_iso_K : T0_K;
  if (!(x0 >= 0.0 && x0 < 1.0) || !(T > 0.0) || !std::isfinite(T) || !(E0 >= 0.0) ||
      !std::isfinite(E0))
    return fail(h, RH_EINVAL, "need 0 <= x0 < 1, T0 > 0 and finite E0 >= 0");
  // ideal gas: T = (gamma - 1) mu m_H e / k_B, mu = 1 / (1 + x)
  const double mu = 1.0 / (1.0 + x0);
  const double e0 = kKB * T / ((h->p.gamma - 1.0) * mu * kMH);
  launch_init_state(h->stream, h->N, E0, 1.0 - x0, e0, nH, E, e, nHI, h->part);
  HIPCHK(hipGetLastError());
  if ((st = sync_reductions(h, slot_bit(RS_NONFINITE))) != RH_OK) return st;
  if (h->hred[RS_NONFINITE] != 0.0) return fail(h, RH_ENONFINITE, "n_H must be finite and > 0");
  return RH_OK;
}

rh_status rh_source_field(rh_handle* h, const double* photon_rate, double* src) {
  if (!h) return RH_EINVAL;
  rh_status st = check_ptrs(h, {photon_rate, src});
  if (st != RH_OK) return st;
  const double scale = h->g.eps_bar / (h->h * h->h * h->h);
  launch_scale_field(h->stream, h->N, scale, photon_rate, src, h->part);
  HIPCHK(hipGetLastError());
  if ((st = sync_reductions(h, slot_bit(RS_NONFINITE))) != RH_OK) return st;
  if (h->hred[RS_NONFINITE] != 0.0)
    return fail(h, RH_ENONFINITE, "photon rates must be finite and >= 0");
  return RH_OK;
}

rh_status rh_set_kernel_timing(rh_handle* h, int32_t enable) {
  if (!h) return RH_EINVAL;
  if (enable && !h->timing) {
    for (int i = 0; i < rh_handle::kPool; ++i) {
      if (hipEventCreate(&h->eva[i]) != hipSuccess || hipEventCreate(&h->evb[i]) != hipSuccess)
        return fail(h, RH_EHIP, "hipEventCreate failed");
    }
  }
  if (!enable && h->timing) {
    (void)hipStreamSynchronize(h->stream);
    flush_timing(h);
    for (int i = 0; i < rh_handle::kPool; ++i) {
      (void)hipEventDestroy(h->eva[i]);
      (void)hipEventDestroy(h->evb[i]);
    }
  }
  h->timing = enable != 0;
  return RH_OK;
}

rh_status rh_get_kernel_timing(rh_handle* h, double* ms, int64_t* counts, int32_t n, int32_t reset) {
  if (!h || n < 1) return RH_EINVAL;
  if (h->timing) {
    HIPCHK(hipStreamSynchronize(h->stream));
    flush_timing(h);
  }
  for (int i = 0; i < n && i < KK_COUNT; ++i) {
    if (ms) ms[i] = h->kms[i];
    if (counts) counts[i] = h->kcount[i];
  }
  if (reset) {
    for (int i = 0; i < KK_COUNT; ++i) {
      h->kms[i] = 0.0;
      h->kcount[i] = 0;
    }
  }
  return RH_OK;
}

rh_status rh_get_constants(const rh_handle* h, double* out, int32_t n) {
  if (!h || !out || n < 8) return RH_EINVAL;
  out[0] = h->g.sigma_E;
  out[1] = h->g.K_Gamma;
  out[2] = h->g.K_G;
  out[3] = h->g.eps_bar;
  out[4] = h->g.hnu0;
  out[5] = h->h;
  out[6] = h->plan.nlev;
  const int* d = h->plan.dims[h->plan.nlev - 1];
  out[7] = (double)d[0] * d[1] * d[2];
  return RH_OK;
}

rh_status rh_cosmology_at(const rh_params* p, double t, double* a, double* H) {
  if (!p || !a || !H) return RH_EINVAL;
  if (p->cosmology != RH_COSMO_STATIC && !(t > 0)) return RH_EINVAL;
  cosmo_at(*p, t, *a, *H);
  return RH_OK;
}

rh_status rh_cosmic_time(const rh_params* p, double a, double* t) {
  if (!p || !t || !(a > 0)) return RH_EINVAL;
  const double H0 = p->hubble_h * kH100;
  if (p->cosmology == RH_COSMO_EDS) {
    *t = std::pow(a, 1.5) / (1.5 * H0);
    return RH_OK;
  }
  if (p->cosmology == RH_COSMO_FLAT_LCDM) {
    *t = 2.0 / (3.0 * std::sqrt(p->Omega_L) * H0) *
         std::asinh(std::sqrt(p->Omega_L / p->Omega_m) * std::pow(a, 1.5));
    return RH_OK;
  }
  if (p->cosmology == RH_COSMO_OPEN) {
    const double Ok = 1.0 - p->Omega_m;
    const double A = p->Omega_m / (2.0 * Ok), B = p->Omega_m / (2.0 * H0 * Ok * std::sqrt(Ok));
    *t = B * open_g(std::acosh(1.0 + a / A));
    return RH_OK;
  }
  return RH_EINVAL;
}

const char* rh_last_error(const rh_handle* h) {
  return h ? h->err.c_str() : g_last_error;
}

void rh_destroy(rh_handle* h) {
  if (!h) return;
  if (h->timing) rh_set_kernel_timing(h, 0);
  if (h->hred) (void)hipHostFree(h->hred);
  (void)hipEventDestroy(h->ev0);
  (void)hipEventDestroy(h->ev1);
  if (h->phase_events)
    for (int i = 0; i < rh_handle::kPhaseEv; ++i) (void)hipEventDestroy(h->pev[i]);
  delete h;
}

}  // extern "C"

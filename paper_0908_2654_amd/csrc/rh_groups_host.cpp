// Host side of the hydrogen + helium multigroup step: group constants by
// quadrature, the handle (one grey handle per group), the Newton driver with
// the per-cell elimination over (e, n_HI, n_HeI, n_HeII), and flexible GMRES
// on the coupled Schur system preconditioned by a block Gauss-Seidel sweep
// over the groups (each group's multigrid on its grey handle).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>

#include "rh_host_internal.h"

using namespace rh;

// ---------------------------------------------------------------------------
// hydrogen + helium chemistry with multigroup radiation
// ---------------------------------------------------------------------------
namespace {

constexpr double kHeIThresholdEV = 24.587;  // HeI ionisation threshold
constexpr double kHeISigma0 = 7.42e-18;     // HeI threshold cross-section, cm^2
constexpr double kInnerReduction = 0.02;    // a group's solve: residual / 50 per sweep
constexpr int kRestart = 8;                 // flexible GMRES restart length
static_assert(kRestart + 1 <= kKrylovMax, "Krylov kernels combine at most kKrylovMax vectors");

// Gauss-Legendre nodes and weights on [-1, 1]: Newton's iteration on the
// Legendre polynomial P_n from cosine first guesses.
void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// int_lo^hi x^m (xs / x)^q / (e^x - 1) dx (hi may be infinite) by composite
// 20-point Gauss-Legendre panels of width 1/4; the integrand falls as
// x^m e^-x, so 120 units past lo it no longer contributes in FP64.
struct GaussLegendre20 {
  double x[20], w[20];
  GaussLegendre20() { gauss_legendre(20, x, w); }
};

double bose_moment(double lo, double hi, int m, double xs, double q) {
  static const GaussLegendre20 gl;  // initialised once, thread-safe
  const double* gx = gl.x;
  const double* gw = gl.w;
  const double top = std::min(hi, lo + 120.0);
  if (!(top > lo)) return 0.0;
  const int panels = std::max(1, (int)std::ceil((top - lo) / 0.25));
  const double wpan = (top - lo) / panels;
  double sum = 0.0;
  for (int pi = 0; pi < panels; ++pi) {
    const double a = lo + pi * wpan;
    double ps = 0.0;
    for (int i = 0; i < 20; ++i) {
      const double x = a + 0.5 * wpan * (gx[i] + 1.0);
      ps += gw[i] * std::pow(x, m) * std::pow(xs / x, q) / std::expm1(x);
    }
    sum += 0.5 * wpan * ps;
  }
  return sum;
}

struct GroupConsts {
  int G;
  double frac[kMaxGroups];
  double sigE[3][kMaxGroups], KGam[3][kMaxGroups], KG[3][kMaxGroups];
  double eps_bar;
};

bool validate_groups(const rh_params* p, const rh_multigroup_params* mg, std::string& err) {
  char msg[256];
  if (!params_valid(p, msg, sizeof msg)) {
    err = msg;
    return false;
  }
  if (!mg) {
    err = "multigroup parameters are NULL";
    return false;
  }
  if (p->spectrum != RH_SPEC_BLACKBODY) {
    err = "multigroup radiation needs the blackbody spectrum (spectrum = RH_SPEC_BLACKBODY)";
    return false;
  }
  if (mg->groups < 1 || mg->groups > RH_MAX_GROUPS || mg->reserved != 0) {
    err = "groups must be 1..RH_MAX_GROUPS and reserved 0";
    return false;
  }
  if (!(std::fabs(mg->edge_eV[0] - p->hnu0_eV) <= 1e-12 * p->hnu0_eV)) {
    err = "the first group edge must be the hydrogen threshold hnu0_eV";
    return false;
  }
  for (int g = 1; g < mg->groups; ++g)
    if (!(mg->edge_eV[g] > mg->edge_eV[g - 1]) || !std::isfinite(mg->edge_eV[g])) {
      err = "group edges must increase and be finite";
      return false;
    }
  if (!(mg->y_he >= 0.0) || !std::isfinite(mg->y_he) || !(mg->sigma_power >= 0.0) ||
      !(mg->sigma_power <= 10.0)) {
    err = "need finite y_he >= 0 and 0 <= sigma_power <= 10";
    return false;
  }
  return true;
}

// Group constants by quadrature of their defining integrals (rh.h).
GroupConsts group_constants(const rh_params& p, const rh_multigroup_params& mg) {
  GroupConsts c{};
  c.G = mg.groups;
  const double kT = kKB * p.T_bb_K;
  double xe[RH_MAX_GROUPS + 1];
  for (int g = 0; g < c.G; ++g) xe[g] = mg.edge_eV[g] * kEV / kT;
  xe[c.G] = INFINITY;
  const double thr[3] = {p.hnu0_eV * kEV / kT, kHeIThresholdEV * kEV / kT,
                         4.0 * p.hnu0_eV * kEV / kT};
  const double sig0[3] = {p.sigma0_cm2, kHeISigma0, 0.25 * p.sigma0_cm2};
  double I[kMaxGroups], Itot = 0.0;
  for (int g = 0; g < c.G; ++g) {
    I[g] = bose_moment(xe[g], xe[g + 1], 3, 1.0, 0.0);
    Itot += I[g];
  }
  for (int g = 0; g < c.G; ++g) {
    c.frac[g] = I[g] / Itot;
    for (int s = 0; s < 3; ++s) {
      const double lo = std::max(xe[g], thr[s]), hi = xe[g + 1];
      if (!(hi > lo)) continue;
      const double sE = bose_moment(lo, hi, 3, thr[s], mg.sigma_power);
      const double sN = bose_moment(lo, hi, 2, thr[s], mg.sigma_power);
      c.sigE[s][g] = sig0[s] * sE / I[g];
      c.KGam[s][g] = sig0[s] * sN / (kT * I[g]);
      c.KG[s][g] = c.sigE[s][g] - thr[s] * kT * c.KGam[s][g];
    }
  }
  c.eps_bar = kT * bose_moment(thr[0], INFINITY, 3, 1.0, 0.0) /
              bose_moment(thr[0], INFINITY, 2, 1.0, 0.0);
  return c;
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// coupled fields of the multigroup handle, in units of one N-cell FP64 field
int group_fields(int G) { return G * G + (12 + 2 * kRestart + 1) * G + 17; }

struct GState {
  double* E;   // [G][N]
  double* e;   // [N] (null: isothermal)
  double* y;   // [3][N]
  double* Bf;  // [4][N]
  double* BC;  // [4][G][N]
};

struct GEval {
  double norm;
  double rmax[kMaxGroups];
  bool finite, local_ok;
};

}  // namespace

struct rh_multigroup {
  rh_params p;
  rh_multigroup_params mg;
  GroupConsts gc;
  GroupK gk;
  int G = 0;
  bool iso = false, he = false;
  long long N = 0;
  hipStream_t stream = nullptr;
  rh_handle* sub[kMaxGroups] = {};  // one grey handle per group: its face
                                    // coefficients, Schur diagonal and multigrid
  double *En = nullptr, *en = nullptr, *yn = nullptr;   // U^n
  double *E2 = nullptr, *e2 = nullptr, *y2 = nullptr;   // the second state buffer
  double *BfA = nullptr, *BCA = nullptr, *BfB = nullptr, *BCB = nullptr;
  double *K = nullptr, *kB = nullptr;                   // Schur coupling [G][G][N], [G][N]
  double *dE = nullptr;                                 // Newton direction [G][N]
  double *b = nullptr;                                  // right-hand side of a group solve
  double *KV = nullptr, *KZ = nullptr;                  // Krylov bases [kRestart + 1][G][N], [kRestart][G][N]
  double *kpart = nullptr;                              // Krylov reduction partials
  double *kred = nullptr, *kred_dev = nullptr;          // their sums (mapped host memory)
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::string err;
  int local_its_max = 0;
};

namespace {

rh_status gfail(rh_multigroup* h, rh_status st, const std::string& msg) {
  h->err = msg;
  return st;
}

#define GHIPCHK(call)                                                          \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess)                                                      \
      return gfail(h, RH_EHIP, std::string("HIP error: ") + hipGetErrorString(e_) + " at " #call); \
  } while (0)

// a failure inside group g's grey handle, with its message
rh_status sub_fail(rh_multigroup* h, int g, rh_status st) {
  return gfail(h, st, "group " + std::to_string(g) + ": " + h->sub[g]->err);
}

double group_nvars(const rh_multigroup* h) {
  return h->G + (h->iso ? 0 : 1) + 1 + (h->he ? 2 : 0);
}

rh_status gcheck_ptrs(rh_multigroup* h, std::initializer_list<const void*> ptrs) {
  for (const void* q : ptrs) {
    if (!q) return gfail(h, RH_EINVAL, "NULL field pointer");
    if (reinterpret_cast<uintptr_t>(q) % 8 != 0) return gfail(h, RH_EINVAL, "misaligned field pointer");
  }
  return RH_OK;
}

StepK group_step(const rh_multigroup* h, int g, double t_n, double dt) {
  StepK k = handle_step(h->sub[g], t_n, dt);
  k.sigma_E = h->gc.sigE[0][g];
  k.K_Gamma = h->gc.KGam[0][g];
  k.K_G = h->gc.KG[0][g];
  k.sig_he[0] = h->he ? h->gc.sigE[1][g] : 0.0;
  k.sig_he[1] = h->he ? h->gc.sigE[2][g] : 0.0;
  k.src_frac = h->gc.frac[g];
  return k;
}

// U^n into the handle; per group: face coefficients from (E_g^n, kappa_g^n),
// the constant part of the residual, E_s and the coarse coefficients.
rh_status groups_setup(rh_multigroup* h, StepK (&kg)[kMaxGroups], double t_n, double dt,
                       const double* src, const double* E, const double* e, const double* y) {
  MarkerRange mark("groups: step setup");
  const size_t f = sizeof(double) * h->N;
  GHIPCHK(hipMemcpyAsync(h->En, E, f * h->G, hipMemcpyDeviceToDevice, h->stream));
  if (!h->iso) GHIPCHK(hipMemcpyAsync(h->en, e, f, hipMemcpyDeviceToDevice, h->stream));
  GHIPCHK(hipMemcpyAsync(h->yn, y, f * (h->he ? 3 : 1), hipMemcpyDeviceToDevice, h->stream));
  for (int g = 0; g < h->G; ++g) {
    kg[g] = group_step(h, g, t_n, dt);
    rh_status st = handle_setup_step(h->sub[g], kg[g], src, h->En + g * h->N, h->yn,
                                     h->he ? h->yn + h->N : nullptr,
                                     h->he ? h->yn + 2 * h->N : nullptr);
    if (st != RH_OK) return sub_fail(h, g, st);
  }
  return RH_OK;
}

// Local solve (mode 0) or evaluation (mode 1) and every group's residual,
// Schur right-hand side and diagonal.
rh_status groups_eval(rh_multigroup* h, const StepK (&kg)[kMaxGroups], const GState& cur,
                      const double* dE, double lam, const GState& out, bool predictor,
                      const double* nH, int mode, double* fE, double* fe, double* fy,
                      GEval& res) {
  MarkerRange mark("groups: local solve + residuals");
  const long long N = h->N;
  rh_handle* s0 = h->sub[0];
  GroupLocalArgs a{};
  a.Ek = cur.E; a.dE = dE; a.lam = lam;
  a.ek = cur.e; a.yk = cur.y;
  if (predictor) {
    a.pBf = cur.Bf;
    a.pBC = cur.BC;
  }
  a.En = h->En; a.en = h->en; a.yn = h->yn; a.nH = nH;
  a.Et = out.E; a.et = out.e; a.yt = out.y;
  a.Bf = mode == 0 ? out.Bf : cur.Bf;
  a.BC = mode == 0 ? out.BC : cur.BC;
  a.K = h->K; a.kB = h->kB;
  a.fe_out = fe; a.fy_out = fy;
  a.mode = mode;
  {
    Timed tm(s0, KK_LOCALG);
    launch_local_groups(h->stream, kg[0], h->gk, a, s0->part);
  }
  GHIPCHK(hipGetLastError());
  const double* Ec = mode == 0 ? out.E : cur.E;
  const double* yc = mode == 0 ? out.y : cur.y;
  const bool mixed = h->p.precision == RH_PREC_MIXED;
  double sum = 0.0;
  res.finite = true;
  res.local_ok = true;
  for (int g = 0; g < h->G; ++g) {
    rh_handle* s = h->sub[g];
    ResidArgs r{};
    r.E = Ec + g * N;
    r.n = yc;
    r.En = h->En + g * N;
    r.nn = h->yn;
    if (h->he) {
      r.y1 = yc + N; r.y2 = yc + 2 * N;
      r.y1n = h->yn + N; r.y2n = h->yn + 2 * N;
    }
    for (int d = 0; d < 3; ++d) r.cf[d] = s->cf64[d];
    r.rhsn = s->rhsn;
    r.kB = h->kB + g * N;
    r.Kgg = h->K + (long long)(g * h->G + g) * N;
    r.rS = s->rS;
    r.diag64 = s->diag64;
    r.op32 = mixed ? s->L32[0].op : nullptr;
    r.fE_out = fE ? fE + g * N : nullptr;
    {
      Timed tm(s, KK_RESID);
      launch_residual(h->stream, kg[g], r, s->part);
    }
    GHIPCHK(hipGetLastError());
    const unsigned mask = g == 0 ? kAllSlots
                                 : slot_bit(RS_FE2) | slot_bit(RS_RMAX) | slot_bit(RS_BAD_RES);
    rh_status st = handle_reductions(s, mask);
    if (st != RH_OK) return sub_fail(h, g, st);
    const double* v = s->hred;
    sum += v[RS_FE2];
    res.rmax[g] = v[RS_RMAX];
    res.finite = res.finite && v[RS_BAD_RES] == 0.0 && std::isfinite(v[RS_RMAX]);
    if (g == 0) {
      sum += v[RS_FN2] + (h->iso ? 0.0 : v[RS_FE_LOC2]);
      res.local_ok = v[RS_LOCAL_FAIL] == 0.0;
      res.finite = res.finite && v[RS_NONFINITE] == 0.0;
      h->local_its_max = std::max(h->local_its_max, (int)v[RS_LOCAL_ITS]);
    }
  }
  res.norm = std::sqrt(sum / (N * group_nvars(h)));
  res.finite = res.finite && std::isfinite(res.norm);
  return RH_OK;
}

// Coupled residual of group g for the right-hand side rhs at x into h->b:
// b = rhs_g - S_gg x_g + sum_{h != g} K_gh x_h, with its weighted sum of
// squares and max |b|.
rh_status coupled_residual(rh_multigroup* h, const StepK& k, int g, const double* rhs,
                           const double* x, double& fe2, double& rmax) {
  rh_handle* s = h->sub[g];
  const double* cf[3] = {s->cf64[0], s->cf64[1], s->cf64[2]};
  {
    Timed tm(s, KK_GCOUPLED);
    launch_group_coupled(h->stream, k, h->G, g, rhs, s->diag64, cf, h->K, x, h->b, s->part);
  }
  GHIPCHK(hipGetLastError());
  rh_status st = handle_reductions(s, slot_bit(RS_FE2) | slot_bit(RS_R2) | slot_bit(RS_RMAX));
  if (st != RH_OK) return sub_fail(h, g, st);
  fe2 = s->hred[RS_FE2];
  rmax = s->hred[RS_RMAX];
  return RH_OK;
}

// Preconditioner of the coupled solve: z = one block Gauss-Seidel sweep over
// the groups from z = 0 for the right-hand side v ([G][N]); group g's
// correction solves S_gg c = v_g - S_gg z_g + sum_{h != g} K_gh z_h with its
// own multigrid to kInnerReduction of that residual.
rh_status groups_precondition(rh_multigroup* h, const StepK (&kg)[kMaxGroups], const double* v,
                              double* z, int& its_total) {
  const long long N = h->N;
  GHIPCHK(hipMemsetAsync(z, 0, sizeof(double) * h->G * N, h->stream));
  for (int g = 0; g < h->G; ++g) {
    double fe2 = 0.0, rmax = 0.0;
    rh_status st = coupled_residual(h, kg[g], g, v + g * N, z, fe2, rmax);
    if (st != RH_OK) return st;
    if (rmax == 0.0) continue;
    static_assert(kMaxGroups == 4, "one range name per group");
    static const char* const kInner[kMaxGroups] = {"group 1 inner solve", "group 2 inner solve",
                                                   "group 3 inner solve", "group 4 inner solve"};
    MarkerRange mark(kInner[g]);
    rh_handle* s = h->sub[g];
    const double wsub = std::sqrt(fe2 / (N * handle_nvars(s)));
    double* keep = s->rS;
    s->rS = h->b;
    double* x = nullptr;
    int its = 0;
    double wi = 0.0, l2 = 0.0;
    bool reached = true;
    st = handle_solve(s, kg[g], rmax, kInnerReduction * wsub, 0.0, s->p.lin_max_it, &x, &its, &wi,
                      &l2, &reached);
    s->rS = keep;
    s->keep_coarse = true;
    if (st != RH_OK) return sub_fail(h, g, st);
    its_total += its;
    {
      Timed tm(h->sub[0], KK_KRYLOV);
      launch_xaxpy(h->stream, N, 1.0, x, z + g * N, 0);
    }
    GHIPCHK(hipGetLastError());
  }
  return RH_OK;
}

// Flexible GMRES(kRestart) on the coupled Schur system
//   S_gg dE_g - sum_{h != g} K_gh dE_h = rS_g   (g = 1..G)
// in the inner product of the norm's weights, right-preconditioned by one
// block Gauss-Seidel sweep (groups_precondition).  Stops when the weighted
// RMS of the true residual is <= target or at its FP64 rounding floor
// (1e-15 of the RMS of the magnitudes of the terms it sums), or after
// max_sweeps preconditioner applications.
rh_status groups_solve(rh_multigroup* h, const StepK (&kg)[kMaxGroups], double target,
                       int max_sweeps, int& its_total, int& sweeps, bool& reached,
                       double& w_final) {
  MarkerRange mark("groups: FGMRES");
  const long long N = h->N;
  const int G = h->G;
  const long long GN = (long long)G * N;
  const double scale = 1.0 / (N * group_nvars(h));
  rh_handle* s0 = h->sub[0];
  GroupOps ops{};
  WeightK wk{};
  for (int g = 0; g < G; ++g) {
    ops.rS[g] = h->sub[g]->rS;
    ops.diag[g] = h->sub[g]->diag64;
    for (int d = 0; d < 3; ++d) ops.cf[g][d] = h->sub[g]->cf64[d];
    ops.E_s[g] = kg[g].E_s;
    wk.w[g] = 1.0 / (kg[g].E_s * kg[g].E_s);
  }
  GroupOps apply = ops;  // the operator alone: B = S x
  for (int g = 0; g < G; ++g) apply.rS[g] = nullptr;
  GHIPCHK(hipMemsetAsync(h->dE, 0, sizeof(double) * GN, h->stream));
  for (int g = 0; g < G; ++g) h->sub[g]->keep_coarse = false;
  its_total = 0;
  sweeps = 0;
  reached = false;
  const Coefs none{};
  double* V = h->KV;   // basis, kRestart + 1 vectors of G N
  double* Z = h->KZ;   // preconditioned basis, kRestart vectors
  double* hv = h->kred;  // mapped host memory the Krylov reductions write
  rh_status st = RH_OK;
  for (int restart = 0;; ++restart) {
    // true residual V_0 = rS - S dE and its norm
    {
      Timed tm(s0, KK_GCOUPLED);
      launch_groups_coupled(h->stream, kg[0], G, ops, h->K, h->dE, V, s0->part);
    }
    GHIPCHK(hipGetLastError());
    if ((st = handle_reductions(s0, slot_bit(RS_FE2) | slot_bit(RS_MAG2))) != RH_OK)
      return sub_fail(h, 0, st);
    const double rr = s0->hred[RS_FE2];
    const double floor = 1e-15 * std::sqrt(s0->hred[RS_MAG2] * scale);
    const double w = std::sqrt(rr * scale);
    w_final = w;
    if (!std::isfinite(w)) return gfail(h, RH_ELINEAR, "non-finite coupled linear residual");
    if (w <= target || w <= floor) {
      reached = true;
      break;
    }
    if (sweeps >= max_sweeps) break;
    const double beta = std::sqrt(rr);
    {
      Timed tm(s0, KK_KRYLOV);
      launch_wcombine(h->stream, N, G, wk, V, 1.0 / beta, nullptr, 0, 0, none, h->kpart, nullptr);
    }
    GHIPCHK(hipGetLastError());
    double H[kRestart + 1][kRestart] = {};
    double cs[kRestart] = {}, sn[kRestart] = {}, gv[kRestart + 1] = {};
    gv[0] = beta;
    int kdim = 0;
    for (int j = 0; j < kRestart; ++j) {
      if ((st = groups_precondition(h, kg, V + j * GN, Z + j * GN, its_total)) != RH_OK) return st;
      ++sweeps;
      double* Vn = V + (j + 1) * GN;
      {
        Timed tm(s0, KK_GCOUPLED);
        launch_groups_coupled(h->stream, kg[0], G, apply, h->K, Z + j * GN, Vn, s0->part);
      }
      GHIPCHK(hipGetLastError());
      // classical Gram-Schmidt, twice
      for (int pass = 0; pass < 2; ++pass) {
        {
          Timed tm(s0, KK_KRYLOV);
          launch_wdots(h->stream, N, G, wk, Vn, V, GN, j + 1, h->kpart, h->kred_dev);
        }
        GHIPCHK(hipGetLastError());
        GHIPCHK(hipStreamSynchronize(h->stream));
        Coefs c{};
        for (int i = 0; i <= j; ++i) {
          c.c[i] = -hv[i];
          H[i][j] += hv[i];
        }
        {
          Timed tm(s0, KK_KRYLOV);
          launch_wcombine(h->stream, N, G, wk, Vn, 1.0, V, GN, j + 1, c, h->kpart,
                          pass == 1 ? h->kred_dev : nullptr);
        }
        GHIPCHK(hipGetLastError());
      }
      GHIPCHK(hipStreamSynchronize(h->stream));
      const double hn = std::sqrt(std::max(hv[0], 0.0));
      H[j + 1][j] = hn;
      if (hn > 0.0) {
        Timed tm(s0, KK_KRYLOV);
        launch_wcombine(h->stream, N, G, wk, Vn, 1.0 / hn, nullptr, 0, 0, none, h->kpart, nullptr);
        GHIPCHK(hipGetLastError());
      }
      // Givens rotations: H upper triangular, gv the rotated right-hand side
      for (int i = 0; i < j; ++i) {
        const double a = cs[i] * H[i][j] + sn[i] * H[i + 1][j];
        H[i + 1][j] = -sn[i] * H[i][j] + cs[i] * H[i + 1][j];
        H[i][j] = a;
      }
      const double den = std::hypot(H[j][j], H[j + 1][j]);
      cs[j] = den > 0.0 ? H[j][j] / den : 1.0;
      sn[j] = den > 0.0 ? H[j + 1][j] / den : 0.0;
      H[j][j] = den;
      H[j + 1][j] = 0.0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      kdim = j + 1;
      const double est = std::fabs(gv[j + 1]) * std::sqrt(scale);
      if (est <= target || est <= floor || hn == 0.0 || sweeps >= max_sweeps) break;
    }
    // dE += sum_i y_i Z_i with H y = gv (upper triangular, kdim x kdim)
    Coefs y{};
    for (int i = kdim - 1; i >= 0; --i) {
      double t = gv[i];
      for (int l = i + 1; l < kdim; ++l) t -= H[i][l] * y.c[l];
      y.c[i] = H[i][i] != 0.0 ? t / H[i][i] : 0.0;
    }
    {
      Timed tm(s0, KK_KRYLOV);
      launch_wcombine(h->stream, N, G, wk, h->dE, 1.0, Z, GN, kdim, y, h->kpart, nullptr);
    }
    GHIPCHK(hipGetLastError());
  }
  for (int g = 0; g < G; ++g) h->sub[g]->keep_coarse = false;
  return RH_OK;
}

rh_status groups_copy(rh_multigroup* h, double* E, double* e, double* y, const double* Es,
                      const double* es, const double* ys) {
  const size_t f = sizeof(double) * h->N;
  GHIPCHK(hipMemcpyAsync(E, Es, f * h->G, hipMemcpyDeviceToDevice, h->stream));
  if (!h->iso) GHIPCHK(hipMemcpyAsync(e, es, f, hipMemcpyDeviceToDevice, h->stream));
  GHIPCHK(hipMemcpyAsync(y, ys, f * (h->he ? 3 : 1), hipMemcpyDeviceToDevice, h->stream));
  return RH_OK;
}

rh_status groups_args(rh_multigroup* h, double t_n, double dt, const double* nH,
                      const double* src, const double* E, const double* e, const double* y) {
  rh_status st = gcheck_ptrs(h, {nH, src, E, y});
  if (st != RH_OK) return st;
  if (!h->iso && (st = gcheck_ptrs(h, {e})) != RH_OK) return st;
  if (!(dt > 0) || !std::isfinite(dt) || !std::isfinite(t_n))
    return gfail(h, RH_EINVAL, "dt must be > 0 and t finite");
  if (h->p.cosmology != RH_COSMO_STATIC && !(t_n > 0))
    return gfail(h, RH_EINVAL, "expanding cosmology needs t > 0");
  return RH_OK;
}

}  // namespace

extern "C" {

rh_status rh_multigroup_constants(const rh_params* p, const rh_multigroup_params* mg, double* out,
                                  int32_t n) {
  std::string err;
  if (!validate_groups(p, mg, err)) {
    set_last_error(err.c_str());
    return RH_EINVAL;
  }
  const int G = mg->groups;
  if (!out || n < 10 * G + 1) {
    set_last_error("out is NULL or shorter than 10 G + 1");
    return RH_EINVAL;
  }
  const GroupConsts c = group_constants(*p, *mg);
  int i = 0;
  for (int g = 0; g < G; ++g) out[i++] = c.frac[g];
  for (int s = 0; s < 3; ++s)
    for (int g = 0; g < G; ++g) out[i++] = c.sigE[s][g];
  for (int s = 0; s < 3; ++s)
    for (int g = 0; g < G; ++g) out[i++] = c.KGam[s][g];
  for (int s = 0; s < 3; ++s)
    for (int g = 0; g < G; ++g) out[i++] = c.KG[s][g];
  out[i] = c.eps_bar;
  return RH_OK;
}

size_t rh_multigroup_workspace_bytes(const rh_params* p, const rh_multigroup_params* mg) {
  std::string err;
  if (!validate_groups(p, mg, err)) {
    set_last_error(err.c_str());
    return 0;
  }
  const size_t N = (size_t)p->nx * p->ny * p->nz;
  // 16 arrays of whole fields and the Krylov partials, each rounded up to 256 bytes
  return 256 + mg->groups * round256(rh_workspace_bytes(p)) +
         group_fields(mg->groups) * sizeof(double) * N + 16 * 256 +
         round256(sizeof(double) * kKrylovMax * kKrylovGrid);
}

rh_status rh_multigroup_setup(const rh_params* p, const rh_multigroup_params* mg, void* workspace,
                              size_t ws_bytes, void* hip_stream, rh_multigroup** out) {
  std::string err;
  if (!out) {
    set_last_error("out is NULL");
    return RH_EINVAL;
  }
  *out = nullptr;
  if (!validate_groups(p, mg, err)) {
    set_last_error(err.c_str());
    return RH_EINVAL;
  }
  const size_t need = rh_multigroup_workspace_bytes(p, mg);
  if (!workspace || ws_bytes < need) {
    set_last_error("workspace missing or smaller than rh_multigroup_workspace_bytes");
    return workspace ? RH_ENOMEM : RH_EINVAL;
  }
  rh_multigroup* h = new rh_multigroup();
  h->p = *p;
  h->mg = *mg;
  h->G = mg->groups;
  h->iso = p->isothermal != 0;
  h->he = mg->y_he > 0.0;
  h->N = (long long)p->nx * p->ny * p->nz;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  h->gc = group_constants(*p, *mg);
  GroupK& k = h->gk;
  k = GroupK{};
  k.G = h->G;
  k.he = h->he ? 1 : 0;
  k.y_he = mg->y_he;
  for (int s = 0; s < 3; ++s)
    for (int g = 0; g < h->G; ++g) {
      // without helium the helium species never absorb
      const bool on = s == 0 || h->he;
      k.KGam[s][g] = on ? h->gc.KGam[s][g] : 0.0;
      k.KG[s][g] = on ? h->gc.KG[s][g] : 0.0;
      k.sigE[s][g] = on ? h->gc.sigE[s][g] : 0.0;
    }
  char* base = reinterpret_cast<char*>(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
  const size_t sub_bytes = round256(rh_workspace_bytes(p));
  for (int g = 0; g < h->G; ++g) {
    rh_status st = rh_setup(p, base, sub_bytes, hip_stream, &h->sub[g]);
    if (st != RH_OK) {
      rh_multigroup_destroy(h);
      return st;  // rh_setup left its message for rh_last_error(NULL)
    }
    base += sub_bytes;
  }
  // each array of nf fields is one block ([nf][N], no padding inside)
  const int G = h->G;
  auto take_block = [&](int nf) {
    double* q = reinterpret_cast<double*>(base);
    base += round256(sizeof(double) * h->N * nf);
    return q;
  };
  h->En = take_block(G);
  h->en = take_block(1);
  h->yn = take_block(3);
  h->E2 = take_block(G);
  h->e2 = take_block(1);
  h->y2 = take_block(3);
  h->BfA = take_block(4);
  h->BCA = take_block(4 * G);
  h->BfB = take_block(4);
  h->BCB = take_block(4 * G);
  h->K = take_block(G * G);
  h->kB = take_block(G);
  h->dE = take_block(G);
  h->b = take_block(1);
  h->KV = take_block((kRestart + 1) * G);
  h->KZ = take_block(kRestart * G);
  h->kpart = reinterpret_cast<double*>(base);
  base += round256(sizeof(double) * kKrylovMax * kKrylovGrid);
  if (hipHostMalloc(reinterpret_cast<void**>(&h->kred), sizeof(double) * kKrylovMax) != hipSuccess ||
      hipHostGetDevicePointer(reinterpret_cast<void**>(&h->kred_dev), h->kred, 0) != hipSuccess) {
    rh_multigroup_destroy(h);
    set_last_error("hipHostMalloc failed");
    return RH_EHIP;
  }
  if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess) {
    rh_multigroup_destroy(h);
    set_last_error("hipEventCreate failed");
    return RH_EHIP;
  }
  *out = h;
  return RH_OK;
}

rh_status rh_multigroup_initial_state(rh_multigroup* h, const double* nH, double x0, double T0_K,
                                      double E0, double* E, double* e, double* y) {
  if (!h) return RH_EINVAL;
  rh_status st = gcheck_ptrs(h, {nH, E, y});
  if (st != RH_OK) return st;
  if (e && (st = gcheck_ptrs(h, {e})) != RH_OK) return st;
  if (!h->iso && !e) return gfail(h, RH_EINVAL, "e is required unless the run is isothermal");
  const double T = h->iso ? h->p.T_iso_K : T0_K;
  if (!(x0 >= 0.0 && x0 < 1.0) || !(T > 0.0) || !std::isfinite(T) || !(E0 >= 0.0) ||
      !std::isfinite(E0))
    return gfail(h, RH_EINVAL, "need 0 <= x0 < 1, T0 > 0 and finite E0 >= 0");
  // T = (gamma - 1) mu m_H e / k_B with mu = (1 + 4 y) / ((1 + y)(1 + x0))
  const double yhe = h->mg.y_he;
  const double mu = (1.0 + 4.0 * yhe) / ((1.0 + yhe) * (1.0 + x0));
  const double e0 = kKB * T / ((h->p.gamma - 1.0) * mu * kMH);
  rh_handle* s0 = h->sub[0];
  launch_groups_init(h->stream, h->N, h->gk, h->gc.frac, E0, x0, e0, nH, E, e, y, s0->part);
  GHIPCHK(hipGetLastError());
  if ((st = handle_reductions(s0, slot_bit(RS_NONFINITE))) != RH_OK) return sub_fail(h, 0, st);
  if (s0->hred[RS_NONFINITE] != 0.0) return gfail(h, RH_ENONFINITE, "n_H must be finite and > 0");
  return RH_OK;
}

rh_status rh_multigroup_step(rh_multigroup* h, double t_n, double dt, const double* nH,
                             const double* src, double* E, double* e, double* y,
                             rh_step_stats* stats) {
  if (!h) return RH_EINVAL;
  rh_status st = groups_args(h, t_n, dt, nH, src, E, e, y);
  if (st != RH_OK) return st;
  MarkerRange mark("rh_multigroup_step");
  h->local_its_max = 0;
  GHIPCHK(hipEventRecord(h->ev0, h->stream));
  StepK kg[kMaxGroups];
  if ((st = groups_setup(h, kg, t_n, dt, src, E, e, y)) != RH_OK) return st;
  GState A{E, h->iso ? nullptr : e, y, h->BfA, h->BCA};
  GState B{h->E2, h->iso ? nullptr : h->e2, h->y2, h->BfB, h->BCB};
  GState* cur = &A;
  GState* oth = &B;
  GEval ev{};
  int newton_its = 0, cuts = 0, lin_total = 0, sweeps_max = 0, cap_hits = 0;
  double lin_res_max = 0.0;
  st = groups_eval(h, kg, *cur, nullptr, 0.0, *oth, false, nH, 0, nullptr, nullptr, nullptr, ev);
  if (st != RH_OK) return st;
  std::swap(cur, oth);
  const double res0 = ev.norm;
  rh_status result = RH_OK;
  for (;;) {
    if (!ev.finite) { result = gfail(h, RH_ENONFINITE, "non-finite residual"); break; }
    if (!ev.local_ok) { result = gfail(h, RH_ELINEAR, "local per-cell solve did not converge"); break; }
    if (ev.norm <= h->p.newton_tol) break;
    if (newton_its >= h->p.newton_max_it) {
      char buf[160];
      std::snprintf(buf, sizeof buf, "Newton did not converge in %d iterations (||f|| = %.3e)",
                    newton_its, ev.norm);
      result = gfail(h, RH_ENEWTON, buf);
      break;
    }
    int its = 0, sweeps = 0;
    bool reached = false;
    double w = 0.0;
    st = groups_solve(h, kg, h->p.lin_forcing * ev.norm, h->p.lin_max_it, its, sweeps, reached, w);
    if (st != RH_OK) { result = st; break; }
    lin_total += its;
    sweeps_max = std::max(sweeps_max, sweeps);
    if (!reached) ++cap_hits;
    if (ev.norm > 0) lin_res_max = std::max(lin_res_max, w / ev.norm);
    ++newton_its;
    const double f0 = ev.norm;
    double lam = 1.0;
    bool accepted = false;
    for (int c = 0; c <= h->p.ls_max_cuts; ++c) {
      st = groups_eval(h, kg, *cur, h->dE, lam, *oth, true, nH, 0, nullptr, nullptr, nullptr, ev);
      if (st != RH_OK) return st;
      if (ev.finite && ev.local_ok && ev.norm <= (1.0 - 1e-4 * lam) * f0) {
        accepted = true;
        break;
      }
      lam *= 0.5;
      ++cuts;
    }
    if (!accepted) {
      result = gfail(h, RH_ENEWTON, "line search failed");
      break;
    }
    std::swap(cur, oth);
  }
  if (result == RH_OK) {
    if (cur->E != E && (st = groups_copy(h, E, e, y, cur->E, cur->e, cur->y)) != RH_OK) return st;
  } else {
    if ((st = groups_copy(h, E, e, y, h->En, h->en, h->yn)) != RH_OK) return st;
  }
  GHIPCHK(hipEventRecord(h->ev1, h->stream));
  GHIPCHK(hipEventSynchronize(h->ev1));
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->newton_its = newton_its;
    stats->lin_its_total = lin_total;
    stats->ls_cuts = cuts;
    stats->local_its_max = h->local_its_max;
    stats->res0 = res0;
    stats->res_final = ev.norm;
    stats->lin_res_max = lin_res_max;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, h->ev0, h->ev1);
    stats->t_ms[0] = ms;
    stats->lin_cap_hits = cap_hits;
    stats->lin_its_max = sweeps_max;
    stats->source_boxes = h->sub[0]->nblk > 0 ? h->sub[0]->B32[0].n + h->sub[0]->B64[0].n : 0;
  }
  return result;
}

rh_status rh_multigroup_residual(rh_multigroup* h, double t_n, double dt, const double* nH,
                                 const double* src, const double* E_n, const double* e_n,
                                 const double* y_n, const double* E, const double* e,
                                 const double* y, double* fE, double* fe, double* fy,
                                 double* norm_out) {
  if (!h) return RH_EINVAL;
  rh_status st = groups_args(h, t_n, dt, nH, src, E_n, e_n, y_n);
  if (st != RH_OK) return st;
  if ((st = gcheck_ptrs(h, {E, y})) != RH_OK) return st;
  if (!h->iso && (st = gcheck_ptrs(h, {e})) != RH_OK) return st;
  StepK kg[kMaxGroups];
  if ((st = groups_setup(h, kg, t_n, dt, src, E_n, e_n, y_n)) != RH_OK) return st;
  GState U{const_cast<double*>(E), h->iso ? nullptr : const_cast<double*>(e),
           const_cast<double*>(y), h->BfA, h->BCA};
  GEval ev{};
  st = groups_eval(h, kg, U, nullptr, 0.0, U, false, nH, 1, fE, h->iso ? nullptr : fe, fy, ev);
  if (st != RH_OK) return st;
  if (norm_out) *norm_out = ev.norm;
  return RH_OK;
}

rh_status rh_multigroup_set_kernel_timing(rh_multigroup* h, int32_t enable) {
  if (!h) return RH_EINVAL;
  for (int g = 0; g < h->G; ++g) {
    rh_status st = rh_set_kernel_timing(h->sub[g], enable);
    if (st != RH_OK) return sub_fail(h, g, st);
  }
  return RH_OK;
}

rh_status rh_multigroup_get_kernel_timing(rh_multigroup* h, double* ms, int64_t* counts,
                                          int32_t n, int32_t reset) {
  if (!h || n < 1) return RH_EINVAL;
  const int m = std::min<int>(n, KK_COUNT);
  if (ms) std::fill(ms, ms + m, 0.0);
  if (counts) std::fill(counts, counts + m, int64_t(0));
  for (int g = 0; g < h->G; ++g) {
    double gm[KK_COUNT];
    int64_t gc[KK_COUNT];
    rh_status st = rh_get_kernel_timing(h->sub[g], gm, gc, KK_COUNT, reset);
    if (st != RH_OK) return sub_fail(h, g, st);
    for (int i = 0; i < m; ++i) {
      if (ms) ms[i] += gm[i];
      if (counts) counts[i] += gc[i];
    }
  }
  return RH_OK;
}

const char* rh_multigroup_last_error(const rh_multigroup* h) {
  return h ? h->err.c_str() : rh_last_error(nullptr);
}

void rh_multigroup_destroy(rh_multigroup* h) {
  if (!h) return;
  for (int g = 0; g < kMaxGroups; ++g) rh_destroy(h->sub[g]);
  if (h->kred) (void)hipHostFree(h->kred);
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  delete h;
}

}  // extern "C"

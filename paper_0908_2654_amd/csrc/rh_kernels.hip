// HIP kernels of the coupled implicit radiation step (gfx950).
//
// Layout: every field is float64 (or float32 on the multigrid levels of the
// mixed path), C order [x][y][z], z fastest.  Face coefficients are stored
// for the + face of each cell along each axis; the last cell's + face holds
// the periodic wrap face, or 0 on a non-periodic boundary.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "rh_device.h"
#include "rh_dual.h"
#include "rh_internal.h"

namespace rh {

// ---------------------------------------------------------------------------
// face limiter (equation limiter, kappa_S = 0)
// ---------------------------------------------------------------------------
__device__ inline double limiter_D(const StepK& k, double EL, double ER, double kL, double kR) {
  double Ebar = fmax(0.5 * (EL + ER), k.E_floor);
  double R = fmax(fabs(ER - EL) / (k.a_n * k.h * Ebar), k.R_min);
  double kap = 0.5 * (kL + kR);
  return kC * (2.0 * kap + R) / (6.0 * kap * kap + 3.0 * kap * R + R * R);
}

// Sum of the dimensionless coefficients of the outflow boundary faces of a
// cell (ghost E = E_floor, ghost opacity = the cell's own).
__device__ inline double outflow_sum(const StepK& k, int i, int j, int kk, double En_P,
                                     double kap_P) {
  double s = 0.0;
  const int c[3] = {i, j, kk};
  const int n[3] = {k.nx, k.ny, k.nz};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (c[d] == 0 && k.bc[2 * d] == RH_BC_OUTFLOW)
      s += k.cf_scale * limiter_D(k, k.E_floor, En_P, kap_P, kap_P);
    if (c[d] == n[d] - 1 && k.bc[2 * d + 1] == RH_BC_OUTFLOW)
      s += k.cf_scale * limiter_D(k, En_P, k.E_floor, kap_P, kap_P);
  }
  return s;
}

// ---------------------------------------------------------------------------
// K0: per-step setup: + face coefficients, constant part of f_E, max E^n, max src
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
k_step_setup(StepK k, const double* __restrict__ En, const double* __restrict__ nn,
             const double* __restrict__ y1n, const double* __restrict__ y2n,
             const double* __restrict__ src, double* __restrict__ cfx, double* __restrict__ cfy,
             double* __restrict__ cfz, Op16* __restrict__ op32, double* __restrict__ rhsn,
             double* __restrict__ part) {
  const int per[3] = {k.bc[0] == RH_BC_PERIODIC, k.bc[2] == RH_BC_PERIODIC,
                      k.bc[4] == RH_BC_PERIODIC};
  const int n[3] = {k.nx, k.ny, k.nz};
  const double kfac = k.sigma_E / (k.a_n * k.a_n * k.a_n);
  const double kf1 = k.sig_he[0] / (k.a_n * k.a_n * k.a_n);
  const double kf2 = k.sig_he[1] / (k.a_n * k.a_n * k.a_n);
  // opacity kappa^n of a cell (helium terms only in a multigroup step)
  auto kap = [&](long long i) {
    double v = kfac * nn[i];
    if (y1n) v += kf1 * y1n[i] + kf2 * y2n[i];
    return v;
  };
  double emax = 0.0, smax = 0.0, bad = 0.0;
  double* cfo[3] = {cfx, cfy, cfz};
  // blocks of one XCD take consecutive cells, so the y neighbours a block
  // reads were loaded by its neighbours on the same XCD (shared L2)
  for (long long idx = xcd_tile(blockIdx.x, gridDim.x) * (long long)blockDim.x + threadIdx.x;
       idx < k.N; idx += (long long)blockDim.x * gridDim.x) {
    int c[3];
    cell_ijk(idx, k.ny, k.nz, c[0], c[1], c[2]);
    const double EP = En[idx];
    const double kP = kap(idx);
    const double sP = k.src_frac * src[idx];
    emax = fmax(emax, EP);
    smax = fmax(smax, sP);
    if (!isfinite(EP) || !isfinite(sP) || !isfinite(kP)) bad = 1.0;
    double Ln = 0.0;  // dt theta L_{n+1} E^n (used for the explicit part)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int q[3];
      double cfp = 0.0;
      if (neighbour(c, n, per, d, +1, q)) {
        long long Q = cell_index(q[0], q[1], q[2], k.ny, k.nz);
        double EQ = En[Q];
        cfp = k.cf_scale * limiter_D(k, EP, EQ, kP, kap(Q));
        Ln += cfp * (EQ - EP);
      }
      cfo[d][idx] = cfp;
      if (op32) op32[idx].f[d] = bf16_round((float)cfp);  // FP32 finest level
      if (k.theta_lt1 && neighbour(c, n, per, d, -1, q)) {
        long long Q = cell_index(q[0], q[1], q[2], k.ny, k.nz);
        double EQ = En[Q];
        Ln += k.cf_scale * limiter_D(k, EQ, EP, kap(Q), kP) * (EQ - EP);
      }
    }
    double r = EP + k.dt * k.theta * sP;
    if (k.theta_lt1) {
      double bs = outflow_sum(k, c[0], c[1], c[2], EP, kP);
      Ln += bs * (k.E_floor - EP);
      // dt (1-theta) (L_n E^n - H_n E^n + src - c kappa_n E^n)
      r += k.expl_ratio * Ln +
           k.dt * (1.0 - k.theta) * (-k.H_n * EP + sP - kC * kP * EP);
    }
    rhsn[idx] = r;
  }
  double v[3] = {emax, smax, bad};
  const int im[3] = {1, 1, 1};
  const int sl[3] = {RS_EMAX, RS_SMAX, RS_NONFINITE};
  block_reduce_store<3>(v, im, sl, part);
}

void launch_step_setup(hipStream_t s, const StepK& k, const double* En, const double* nn,
                       const double* y1n, const double* y2n, const double* src, double* cfx,
                       double* cfy, double* cfz, Op16* op32, double* rhsn, double* part) {
  hipLaunchKernelGGL(k_step_setup, dim3(red_grid(k.N)), dim3(kBlock), 0, s, k, En, nn, y1n, y2n,
                     src, cfx, cfy, cfz, op32, rhsn, part);
}

// ---------------------------------------------------------------------------
// forward-mode dual numbers over (n, e, E) for the local Jacobian
// ---------------------------------------------------------------------------
struct D3 {
  double v, g[3];
};
__device__ inline D3 dconst(double v) { return D3{v, {0.0, 0.0, 0.0}}; }
__device__ inline D3 dvar(double v, int i) {
  D3 r{v, {0.0, 0.0, 0.0}};
  r.g[i] = 1.0;
  return r;
}
__device__ inline D3 operator+(D3 a, D3 b) {
  return D3{a.v + b.v, {a.g[0] + b.g[0], a.g[1] + b.g[1], a.g[2] + b.g[2]}};
}
__device__ inline D3 operator-(D3 a, D3 b) {
  return D3{a.v - b.v, {a.g[0] - b.g[0], a.g[1] - b.g[1], a.g[2] - b.g[2]}};
}
__device__ inline D3 operator*(D3 a, D3 b) {
  return D3{a.v * b.v, {a.g[0] * b.v + a.v * b.g[0], a.g[1] * b.v + a.v * b.g[1],
                        a.g[2] * b.v + a.v * b.g[2]}};
}
__device__ inline D3 operator/(D3 a, D3 b) {
  double iv = 1.0 / b.v, q = a.v * iv;
  return D3{q, {(a.g[0] - q * b.g[0]) * iv, (a.g[1] - q * b.g[1]) * iv,
                (a.g[2] - q * b.g[2]) * iv}};
}
__device__ inline D3 operator+(D3 a, double b) { return D3{a.v + b, {a.g[0], a.g[1], a.g[2]}}; }
__device__ inline D3 operator+(double b, D3 a) { return a + b; }
__device__ inline D3 operator-(D3 a, double b) { return D3{a.v - b, {a.g[0], a.g[1], a.g[2]}}; }
__device__ inline D3 operator-(double b, D3 a) {
  return D3{b - a.v, {-a.g[0], -a.g[1], -a.g[2]}};
}
__device__ inline D3 operator*(D3 a, double b) {
  return D3{a.v * b, {a.g[0] * b, a.g[1] * b, a.g[2] * b}};
}
__device__ inline D3 operator*(double b, D3 a) { return a * b; }
__device__ inline D3 operator/(D3 a, double b) { return a * (1.0 / b); }
__device__ inline D3 operator/(double b, D3 a) { return dconst(b) / a; }
__device__ inline D3 dexp(D3 a) {
  double ev = exp(a.v);
  return D3{ev, {a.g[0] * ev, a.g[1] * ev, a.g[2] * ev}};
}
__device__ inline D3 dpow(D3 a, double p) {
  double pv = pow(a.v, p);
  double dv = p * pv / a.v;
  return D3{pv, {a.g[0] * dv, a.g[1] * dv, a.g[2] * dv}};
}
__device__ inline D3 dsqrt(D3 a) {
  double sv = sqrt(a.v);
  double dv = 0.5 / sv;
  return D3{sv, {a.g[0] * dv, a.g[1] * dv, a.g[2] * dv}};
}
__device__ inline D3 dlog(D3 a) {
  double iv = 1.0 / a.v;
  return D3{log(a.v), {a.g[0] * iv, a.g[1] * iv, a.g[2] * iv}};
}
__device__ inline D3 dmax0(D3 a) { return a.v >= 0.0 ? a : dconst(0.0); }
template <>
__device__ inline D3 lift<D3>(double v) { return dconst(v); }

// The temperature fits are functions of T alone: evaluate them once with one
// derivative slot (d/dT) and chain the result into the caller's dual numbers.
__device__ inline double dval(const D3& a) { return a.v; }
__device__ inline D3 dchain(const D3& x, double fv, double dfv) {
  return D3{fv, {x.g[0] * dfv, x.g[1] * dfv, x.g[2] * dfv}};
}
struct TFits {
  double alpha, dalpha, recB, drecB, ce, dce;  // values and d/dT
};
__device__ inline TFits t_fits(double T, bool alpha, bool recB, bool ce) {
  TFits f{};
  const DN<1> Td = dn_var<1>(T, 0);
  if (alpha || recB) {
    const DN<1> L = hg_ln_lambda(Td);
    if (alpha) {
      const DN<1> a = alpha_B_of_L(L);
      f.alpha = a.v;
      f.dalpha = a.g[0];
    }
    if (recB) {
      const DN<1> r = cool_recB_of_L(Td, L);
      f.recB = r.v;
      f.drecB = r.g[0];
    }
  }
  if (ce) {
    const DN<1> c = cool_collexc(Td);
    f.ce = c.v;
    f.dce = c.g[0];
  }
  return f;
}

// Rates of the local ODEs at a state: dn/dt = A - B n, de/dt = q - 2 H e.
template <class S>
__device__ inline void local_rates(const StepK& k, S E, S e, S n, double nH, double a, S& A,
                                   S& B, S& q) {
  const double a3 = a * a * a;
  S Epos = dmax0(E);
  S T;
  if (k.iso) {
    T = lift<S>(k.T_iso);
  } else {
    S mu = 1.0 / (2.0 - n / nH);  // 1/(1+x), x = 1 - n/n_H
    T = ((k.gamma - 1.0) * kMH / kKB) * mu * e;
  }
  S ne = (nH - n) / a3;
  const bool fit_recB = !k.iso && (k.cooling & RH_COOL_RECB);
  const bool fit_ce = !k.iso && (k.cooling & RH_COOL_COLLEXC);
  const TFits tf = t_fits(dval(T), k.rates, fit_recB, fit_ce);
  S alpha = k.rates ? dchain(T, tf.alpha, tf.dalpha) : lift<S>(k.alphaB);
  A = alpha * ne * nH;
  B = alpha * ne + (kC * k.K_Gamma / a3) * Epos;
  if (k.iso) {
    q = lift<S>(0.0);
    return;
  }
  S nHI = n / a3;
  S G = (kC * k.K_G / a3) * nHI * Epos;
  S Lam = lift<S>(0.0);
  if (fit_recB) Lam = Lam + dchain(T, tf.recB, tf.drecB) * ne * ne;
  if (fit_ce) Lam = Lam + dchain(T, tf.ce, tf.dce) * ne * nHI;
  if (k.cooling & RH_COOL_COMPTON) {
    const double zp1 = 1.0 / a;
    Lam = Lam + (k.compton * zp1 * zp1 * zp1 * zp1) * (T - kTcmb0 * zp1) * ne;
  }
  q = (G - Lam) * (a3 / (kMH * nH));
}

// theta-method local solutions S_n(U), S_e(U) with explicit parts Rn, qn.
template <class S>
__device__ inline void local_S(const StepK& k, S E, S e, S n, double nH, double nn, double en,
                               double Rn, double qn, S& Sn, S& Se) {
  S A, B, q;
  local_rates(k, E, e, n, nH, k.a_1, A, B, q);
  const double th = k.theta, dt = k.dt;
  Sn = (nn + dt * th * A + dt * (1.0 - th) * Rn) / (1.0 + (th * dt) * B);
  if (k.iso) {
    Se = lift<S>(en);
  } else {
    Se = (en + dt * th * q + dt * (1.0 - th) * qn) / (1.0 + 2.0 * th * dt * k.H_1);
  }
}

// ---------------------------------------------------------------------------
// K1: local solve / evaluation
// ---------------------------------------------------------------------------
// at least 3 waves per SIMD (<= 168 VGPRs): the FP64 chemistry is latency-bound at 2
__global__ void __launch_bounds__(kBlock, 3)
k_local(StepK k, LocalArgs a, double* __restrict__ part) {
  double sfn = 0.0, sfe = 0.0, fail = 0.0, itmax = 0.0, bad = 0.0;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < k.N;
       idx += (long long)blockDim.x * gridDim.x) {
    const double nH = a.nH[idx];
    const double nn = a.nn[idx];
    const double en = k.iso ? 0.0 : a.en[idx];
    double E = a.Ek[idx];
    double dEv = 0.0;
    if (a.dE) {
      dEv = a.dE[idx];
      E += a.lam * dEv;
    }
    double n = a.nk[idx];
    double e = k.iso ? 0.0 : a.ek[idx];
    // explicit parts of the theta method
    double Rn = 0.0, qn = 0.0;
    if (k.theta_lt1) {
      double An, Bn, qq;
      local_rates<double>(k, a.En[idx], en, nn, nH, k.a_n, An, Bn, qq);
      Rn = An - Bn * nn;
      qn = k.iso ? 0.0 : qq - 2.0 * k.H_n * en;
    }
    int its = 0;
    if (a.mode == 0) {
      // predictor from the linearisation at U_k
      if (a.pBCn && a.dE) {
        n -= a.pBfn[idx] + a.pBCn[idx] * a.lam * dEv;
        if (!k.iso) e -= a.pBfe[idx] + a.pBCe[idx] * a.lam * dEv;
      }
      n = fmin(fmax(n, 0.0), nH);
      if (!k.iso) e = fmax(e, 1e-300);
      bool conv = false;
      for (its = 1; its <= 80; ++its) {
        // E is fixed here: two derivative slots (n, e)
        DN<2> Sn, Se;
        local_S<DN<2>>(k, dn_const<2>(E), dn_var<2>(e, 1), dn_var<2>(n, 0), nH, nn, en, Rn, qn,
                       Sn, Se);
        const double fn = n - Sn.v;
        const double b11 = 1.0 - Sn.g[0];
        double dn, de = 0.0;
        if (k.iso) {
          dn = -fn / b11;
        } else {
          const double fe = e - Se.v;
          const double b12 = -Sn.g[1], b21 = -Se.g[0], b22 = 1.0 - Se.g[1];
          const double det = b11 * b22 - b12 * b21;
          dn = -(b22 * fn - b12 * fe) / det;
          de = -(-b21 * fn + b11 * fe) / det;
        }
        double lam = 1.0;
        if (n + dn < 0.0) lam = fmin(lam, 0.9 * n / (-dn));
        if (n + dn > nH) lam = fmin(lam, 0.9 * (nH - n) / dn);
        if (!k.iso && e + de <= 0.0) lam = fmin(lam, 0.9 * e / (-de));
        n += lam * dn;
        double small = fabs(lam * dn) / nH;
        if (!k.iso) {
          e += lam * de;
          small = fmax(small, fabs(lam * de) / e);
        }
        if (!(small == small)) break;  // NaN
        // an undamped step of relative size s leaves an error of order s^2
        // (quadratic convergence of the 2x2 Newton iteration): after s <= 1e-9
        // the iterate is at the root to rounding
        if (lam == 1.0 && small <= 1e-9) {
          conv = true;
          break;
        }
      }
      if (!conv) fail = 1.0;
      itmax = fmax(itmax, (double)its);
      a.Et[idx] = E;
      a.nt[idx] = n;
      if (!k.iso) a.et[idx] = e;
    }
    // local residual and Jacobian terms at the (solved or given) state
    D3 Sn, Se;
    local_S<D3>(k, dvar(E, 2), dvar(e, 1), dvar(n, 0), nH, nn, en, Rn, qn, Sn, Se);
    const double fn = n - Sn.v;
    const double b11 = 1.0 - Sn.g[0];
    double Bfn, Bcn, Bfe = 0.0, Bce = 0.0, fe = 0.0;
    if (k.iso) {
      Bfn = fn / b11;
      Bcn = -Sn.g[2] / b11;
    } else {
      fe = e - Se.v;
      const double b12 = -Sn.g[1], b21 = -Se.g[0], b22 = 1.0 - Se.g[1];
      const double c1 = -Sn.g[2], c2 = -Se.g[2];
      const double idet = 1.0 / (b11 * b22 - b12 * b21);
      Bfn = (b22 * fn - b12 * fe) * idet;
      Bfe = (-b21 * fn + b11 * fe) * idet;
      Bcn = (b22 * c1 - b12 * c2) * idet;
      Bce = (-b21 * c1 + b11 * c2) * idet;
      sfe += (fe / en) * (fe / en);
    }
    sfn += (fn / nH) * (fn / nH);
    if (!isfinite(fn) || !isfinite(fe) || !isfinite(E)) bad = 1.0;
    a.BCn[idx] = Bcn;
    a.Bfn[idx] = Bfn;
    if (!k.iso) {
      a.BCe[idx] = Bce;
      a.Bfe[idx] = Bfe;
    }
    if (a.fn_out) a.fn_out[idx] = fn;
    if (a.fe_out && !k.iso) a.fe_out[idx] = fe;
  }
  double v[5] = {sfn, sfe, fail, itmax, bad};
  const int im[5] = {0, 0, 1, 1, 1};
  const int sl[5] = {RS_FN2, RS_FE_LOC2, RS_LOCAL_FAIL, RS_LOCAL_ITS, RS_NONFINITE};
  block_reduce_store<5>(v, im, sl, part);
}

void launch_local(hipStream_t s, const StepK& k, const LocalArgs& a, double* part) {
  // many small workgroups: the ALU-bound solve runs at 3 waves per SIMD, which
  // the fixed reduction grid would fill only in one and a third rounds
  const long long g = (k.N + kBlock - 1) / kBlock;
  const int grid = (int)(g < kPartCap ? g : kPartCap);
  hipLaunchKernelGGL(k_local, dim3(grid), dim3(kBlock), 0, s, k, a, part);
}

// ---------------------------------------------------------------------------
// K2/K3: radiation residual f_E, Schur right-hand side and diagonal
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
k_residual(StepK k, ResidArgs a, double* __restrict__ part) {
  const int per[3] = {k.bc[0] == RH_BC_PERIODIC, k.bc[2] == RH_BC_PERIODIC,
                      k.bc[4] == RH_BC_PERIODIC};
  const int nd[3] = {k.nx, k.ny, k.nz};
  const double a13 = k.a_1 * k.a_1 * k.a_1;
  const double dth = k.dt * k.theta;
  const double kfac_n = k.sigma_E / (k.a_n * k.a_n * k.a_n);
  double sfe = 0.0, rmax = 0.0, bad = 0.0;
  // blocks of one XCD take consecutive cells, so the y neighbours a block
  // reads were loaded by its neighbours on the same XCD (shared L2)
  for (long long idx = xcd_tile(blockIdx.x, gridDim.x) * (long long)blockDim.x + threadIdx.x;
       idx < k.N; idx += (long long)blockDim.x * gridDim.x) {
    int c[3];
    cell_ijk(idx, k.ny, k.nz, c[0], c[1], c[2]);
    const double EP = a.E[idx];
    const double nP = a.n[idx];
    double LE = 0.0, csum = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int q[3];
      if (neighbour(c, nd, per, d, +1, q)) {
        const double cf = a.cf[d][idx];
        LE += cf * (a.E[cell_index(q[0], q[1], q[2], k.ny, k.nz)] - EP);
        csum += cf;
      }
      if (neighbour(c, nd, per, d, -1, q)) {
        const long long Q = cell_index(q[0], q[1], q[2], k.ny, k.nz);
        const double cf = a.cf[d][Q];
        LE += cf * (a.E[Q] - EP);
        csum += cf;
      }
    }
    bool bnd = (c[0] == 0 || c[0] == k.nx - 1 || c[1] == 0 || c[1] == k.ny - 1 || c[2] == 0 ||
                c[2] == k.nz - 1);
    double bs = 0.0;
    if (bnd) {
      double kn = kfac_n * a.nn[idx];
      if (a.y1n) kn += (k.sig_he[0] * a.y1n[idx] + k.sig_he[1] * a.y2n[idx]) / (k.a_n * k.a_n * k.a_n);
      bs = outflow_sum(k, c[0], c[1], c[2], a.En[idx], kn);
    }
    double absorb = kC * k.sigma_E * nP / a13;
    if (a.y1) absorb += kC * (k.sig_he[0] * a.y1[idx] + k.sig_he[1] * a.y2[idx]) / a13;
    const double fE = EP + dth * (k.H_1 + absorb) * EP - LE + bs * (EP - k.E_floor) - a.rhsn[idx];
    double diag = 1.0 + dth * (k.H_1 + absorb) + csum + bs;
    double rS = -fE;
    if (a.kB) {
      diag -= a.Kgg[idx];
      rS += a.kB[idx];
    } else {
      const double JEn = dth * kC * k.sigma_E * EP / a13;
      diag -= JEn * a.BCn[idx];
      rS += JEn * a.Bfn[idx];
    }
    if (a.rS) a.rS[idx] = rS;
    if (a.diag64) a.diag64[idx] = diag;
    // FP32 finest level: the shift, diagonal minus the faces
    if (a.op32) a.op32[idx].s = bf16_round((float)(diag - csum));
    if (a.fE_out) a.fE_out[idx] = fE;
    sfe += (fE / k.E_s) * (fE / k.E_s);
    rmax = fmax(rmax, fabs(rS));
    if (!isfinite(fE) || !isfinite(diag)) bad = 1.0;
  }
  double v[3] = {sfe, rmax, bad};
  const int im[3] = {0, 1, 1};
  const int sl[3] = {RS_FE2, RS_RMAX, RS_BAD_RES};
  block_reduce_store<3>(v, im, sl, part);
}

void launch_residual(hipStream_t s, const StepK& k, const ResidArgs& a, double* part) {
  hipLaunchKernelGGL(k_residual, dim3(red_grid(k.N)), dim3(kBlock), 0, s, k, a, part);
}

// ---------------------------------------------------------------------------
// deterministic second pass of the reductions
// ---------------------------------------------------------------------------
// One workgroup per reduction slot in `mask`: the slot's block partials in
// a fixed order, so the result does not depend on scheduling.
__global__ void __launch_bounds__(kBlock) k_finalize(const double* __restrict__ part,
                                                     double* __restrict__ out, unsigned mask) {
  __shared__ double sh[kBlock / 64];
  const int s = blockIdx.x;
  if (!((mask >> s) & 1u)) return;
  const bool is_max = (s == RS_RMAX || s == RS_LOCAL_FAIL || s == RS_LOCAL_ITS || s == RS_EMAX ||
                       s == RS_SMAX || s == RS_NONFINITE || s == RS_BAD_RES || s == RS_NEGE ||
                       s == RS_COURANT);
  const int nblocks =
      (int)fmin(fmax(part[(long long)RS_COUNT * kPartCap + s], 0.0), (double)kPartCap);
  double v = is_max ? -INFINITY : 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kBlock) {
    const double p = part[(long long)s * kPartCap + b];
    v = is_max ? fmax(v, p) : v + p;
  }
  v = is_max ? wave_max(v) : wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = sh[0];
    for (int w = 1; w < kBlock / 64; ++w) t = is_max ? fmax(t, sh[w]) : t + sh[w];
    out[s] = t;
  }
}

__global__ void __launch_bounds__(kBlock)
k_change_norm(long long N, double E_s, const double* __restrict__ E, const double* __restrict__ e,
              const double* __restrict__ n, const double* __restrict__ En,
              const double* __restrict__ en, const double* __restrict__ nn,
              const double* __restrict__ nH, double* __restrict__ part) {
  double s2 = 0.0, neg = -INFINITY;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < N;
       idx += (long long)blockDim.x * gridDim.x) {
    const double dE = (E[idx] - En[idx]) / E_s;
    const double dn = (n[idx] - nn[idx]) / nH[idx];
    s2 += dE * dE + dn * dn;
    if (e) {
      const double de = (e[idx] - en[idx]) / en[idx];
      s2 += de * de;
    }
    neg = fmax(neg, -E[idx] / E_s);
  }
  double v[2] = {s2, neg};
  const int im[2] = {0, 1};
  const int sl[2] = {RS_CHG2, RS_NEGE};
  block_reduce_store<2>(v, im, sl, part);
}

void launch_change_norm(hipStream_t s, long long N, double E_s, const double* E, const double* e,
                        const double* n, const double* En, const double* en, const double* nn,
                        const double* nH, double* part) {
  hipLaunchKernelGGL(k_change_norm, dim3(red_grid(N)), dim3(kBlock), 0, s, N, E_s, E, e, n, En,
                     en, nn, nH, part);
}

// Initial fields of a run: E = E0, n_HI = keep * n_H and, when e is given,
// e = e0 (the host evaluates the gas energy of the initial temperature);
// an input n_H that is not finite and positive raises the non-finite flag.
__global__ void __launch_bounds__(kBlock)
k_init_state(long long N, double E0, double keep, double e0, const double* __restrict__ nH,
             double* __restrict__ E, double* __restrict__ e, double* __restrict__ n,
             double* __restrict__ part) {
  double bad = 0.0;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < N;
       idx += (long long)blockDim.x * gridDim.x) {
    const double h = nH[idx];
    if (!(h > 0.0) || !isfinite(h)) bad = 1.0;
    E[idx] = E0;
    n[idx] = keep * h;
    if (e) e[idx] = e0;
  }
  double v[1] = {bad};
  const int im[1] = {1};
  const int sl[1] = {RS_NONFINITE};
  block_reduce_store<1>(v, im, sl, part);
}

void launch_init_state(hipStream_t s, long long N, double E0, double keep, double e0,
                       const double* nH, double* E, double* e, double* n, double* part) {
  hipLaunchKernelGGL(k_init_state, dim3(red_grid(N)), dim3(kBlock), 0, s, N, E0, keep, e0, nH, E,
                     e, n, part);
}

// out = scale * in (emissivity from photon rates: scale = mean photon energy
// / cell volume); flags entries that are negative or not finite.
__global__ void __launch_bounds__(kBlock)
k_scale_field(long long N, double scale, const double* __restrict__ in, double* __restrict__ out,
              double* __restrict__ part) {
  double bad = 0.0;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < N;
       idx += (long long)blockDim.x * gridDim.x) {
    const double q = in[idx];
    if (!(q >= 0.0) || !isfinite(q)) bad = 1.0;
    out[idx] = q * scale;
  }
  double v[1] = {bad};
  const int im[1] = {1};
  const int sl[1] = {RS_NONFINITE};
  block_reduce_store<1>(v, im, sl, part);
}

void launch_scale_field(hipStream_t s, long long N, double scale, const double* in, double* out,
                        double* part) {
  hipLaunchKernelGGL(k_scale_field, dim3(red_grid(N)), dim3(kBlock), 0, s, N, scale, in, out,
                     part);
}

void launch_finalize(hipStream_t s, const double* part, double* out, unsigned mask) {
  hipLaunchKernelGGL(k_finalize, dim3(RS_COUNT), dim3(kBlock), 0, s, part, out, mask);
}

// ---------------------------------------------------------------------------
// multigrid: coarse operators
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(kBlock) k_coarsen_faces(LevelK<T> f, LevelK<T> c) {
  const int fny = f.ny, fnz = f.nz;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < c.N;
       idx += (long long)blockDim.x * gridDim.x) {
    int I, J, K;
    cell_ijk(idx, c.ny, c.nz, I, J, K);
    // + x face of coarse (I,J,K): fine faces between x = 2I+1 and 2I+2
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        sx += (double)face_of(f, 0, cell_index(2 * I + 1, 2 * J + a, 2 * K + b, fny, fnz));
        sy += (double)face_of(f, 1, cell_index(2 * I + a, 2 * J + 1, 2 * K + b, fny, fnz));
        sz += (double)face_of(f, 2, cell_index(2 * I + a, 2 * J + b, 2 * K + 1, fny, fnz));
      }
    // mean of the 4 fine faces, times 1/4 for the doubled cell width
    put_face(c, 0, idx, 0.0625 * sx);
    put_face(c, 1, idx, 0.0625 * sy);
    put_face(c, 2, idx, 0.0625 * sz);
  }
}

template <class T>
void launch_coarsen_faces(hipStream_t s, const LevelK<T>& f, const LevelK<T>& c) {
  hipLaunchKernelGGL((k_coarsen_faces<T>), dim3(red_grid(c.N)), dim3(kBlock), 0, s, f, c);
}

// Sum of a cell's interior face coefficients (6 faces).
template <class T>
__device__ inline double face_sum(const LevelK<T>& l, const int (&c)[3], long long idx) {
  const int n[3] = {l.nx, l.ny, l.nz};
  double s = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int q[3];
    if (neighbour(c, n, l.per, d, +1, q)) s += (double)face_of(l, d, idx);
    if (neighbour(c, n, l.per, d, -1, q))
      s += (double)face_of(l, d, cell_index(q[0], q[1], q[2], l.ny, l.nz));
  }
  return s;
}

// Coarse shift = mean of the eight children's shifts (shift = diagonal
// minus the cell's faces); FP64 levels store the diagonal (coarse shift plus
// the coarse faces), FP32 levels the shift itself.
template <class T>
__global__ void __launch_bounds__(kBlock) k_coarse_diag(LevelK<T> f, LevelK<T> c) {
  constexpr bool kF32 = std::is_same<T, float>::value;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < c.N;
       idx += (long long)blockDim.x * gridDim.x) {
    int C[3];
    cell_ijk(idx, c.ny, c.nz, C[0], C[1], C[2]);
    double sh = 0.0;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int d = 0; d < 2; ++d) {
          int F[3] = {2 * C[0] + a, 2 * C[1] + b, 2 * C[2] + d};
          long long fi = cell_index(F[0], F[1], F[2], f.ny, f.nz);
          if constexpr (kF32)
            sh += (double)bf16_value(f.op[fi].s);
          else
            sh += (double)f.diag[fi] - face_sum(f, F, fi);
        }
    if constexpr (kF32)
      c.op[idx].s = bf16_round((float)(0.125 * sh));
    else
      c.diag[idx] = (T)(0.125 * sh + face_sum(c, C, idx));
  }
}

template <class T>
void launch_coarse_diag(hipStream_t s, const LevelK<T>& f, const LevelK<T>& c) {
  hipLaunchKernelGGL((k_coarse_diag<T>), dim3(red_grid(c.N)), dim3(kBlock), 0, s, f, c);
}

// Coarsest level: assemble the dense matrix in FP64 and invert it by
// Gauss-Jordan elimination (symmetric, diagonally dominant: no pivoting).
template <class T>
__global__ void __launch_bounds__(1024) k_coarsest_inverse(LevelK<T> c, double* A, double* Inv,
                                                           T* InvT) {
  const int n = (int)c.N;
  const int nn = n * n;
  for (int t = threadIdx.x; t < nn; t += blockDim.x) {
    A[t] = 0.0;
    Inv[t] = (t / n == t % n) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nd[3] = {c.nx, c.ny, c.nz};
    for (int P = 0; P < n; ++P) {
      int C[3];
      cell_ijk(P, c.ny, c.nz, C[0], C[1], C[2]);
      A[(long long)P * n + P] += (double)diag_of(c, C, P);
      for (int d = 0; d < 3; ++d) {
        int q[3];
        if (neighbour(C, nd, c.per, d, +1, q)) {
          int Q = (int)cell_index(q[0], q[1], q[2], c.ny, c.nz);
          A[(long long)P * n + Q] -= (double)face_of(c, d, P);
        }
        if (neighbour(C, nd, c.per, d, -1, q)) {
          int Q = (int)cell_index(q[0], q[1], q[2], c.ny, c.nz);
          A[(long long)P * n + Q] -= (double)face_of(c, d, Q);
        }
      }
    }
  }
  __syncthreads();
  __shared__ double colk[kCoarseMaxCells];
  for (int kk = 0; kk < n; ++kk) {
    const double piv = A[(long long)kk * n + kk];
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      A[(long long)kk * n + j] /= piv;
      Inv[(long long)kk * n + j] /= piv;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) colk[i] = A[(long long)i * n + kk];
    __syncthreads();
    for (int t = threadIdx.x; t < nn; t += blockDim.x) {
      const int i = t / n, j = t % n;
      if (i == kk) continue;
      const double f = colk[i];
      A[t] -= f * A[(long long)kk * n + j];
      Inv[t] -= f * Inv[(long long)kk * n + j];
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < nn; t += blockDim.x) InvT[t] = (T)Inv[t];
}

template <class T>
void launch_coarsest_inverse(hipStream_t s, const LevelK<T>& c, double* A, double* Inv, T* InvT) {
  hipLaunchKernelGGL((k_coarsest_inverse<T>), dim3(1), dim3(1024), 0, s, c, A, Inv, InvT);
}

template <class T>
__global__ void __launch_bounds__(kCoarseMaxCells) k_coarsest_solve(LevelK<T> c, const T* InvT) {
  __shared__ T bs[kCoarseMaxCells];
  const int n = (int)c.N;
  for (int i = threadIdx.x; i < n; i += blockDim.x) bs[i] = c.b[i];
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    T s = 0;
    const T* row = InvT + (long long)i * n;
    for (int j = 0; j < n; ++j) s += row[j] * bs[j];
    c.x[i] = s;
  }
}

template <class T>
void launch_coarsest_solve(hipStream_t s, const LevelK<T>& c, const T* InvT) {
  hipLaunchKernelGGL((k_coarsest_solve<T>), dim3(1), dim3(kCoarseMaxCells), 0, s, c, InvT);
}

// ---------------------------------------------------------------------------
// multigrid: smoother, residual, transfers
// ---------------------------------------------------------------------------
// One colour of a red-black Gauss-Seidel sweep (red: i+j+k even).  FINE
// only gives the finest-level instantiation its own name for profiling.
template <class T, int FINE>
__global__ void __launch_bounds__(kBlock) k_rbgs(LevelK<T> l, int color, int zero_init) {
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < l.N;
       idx += (long long)blockDim.x * gridDim.x) {
    int c[3];
    cell_ijk(idx, l.ny, l.nz, c[0], c[1], c[2]);
    if (((c[0] + c[1] + c[2]) & 1) != color) continue;
    T off, dg;
    row_terms(l, c, idx, !zero_init, off, dg);
    T s = l.b[idx];
    if (!zero_init) s += off;
    l.x[idx] = s / dg;
  }
}

template <class T>
void launch_rbgs(hipStream_t s, const LevelK<T>& l, int color, int zero_init, int fine) {
  long long g = (l.N + kBlock - 1) / kBlock;
  const dim3 grid((unsigned)(g < 65536 ? g : 65536));
  if (fine)
    hipLaunchKernelGGL((k_rbgs<T, 1>), grid, dim3(kBlock), 0, s, l, color, zero_init);
  else
    hipLaunchKernelGGL((k_rbgs<T, 0>), grid, dim3(kBlock), 0, s, l, color, zero_init);
}

// One full red-black sweep (both colours) in one launch, marching along x.
// A block owns a TY x TZ tile of the (y, z) plane over XC consecutive x
// planes.  x is read from l.x (never written during the sweep) into a ring
// of four LDS planes with a 2-cell halo in y and z; the first colour is
// updated on plane p over the tile plus a 1-cell ring (the ring values are
// recomputed here, not written), then the second colour on plane p-1 over
// the tile, and plane p-1 (both colours) is written to l.x2.  The first
// colour is also recomputed on the plane before and after the block's x
// range.  Every LDS slot stands for a real cell (periodic wrap) or for
// "outside" (beyond a non-periodic wall); smoothed levels have all
// dimensions even, so neighbours always have the other colour.  Reading one
// buffer and writing another makes the result exactly that of a red sweep
// followed by a black sweep, independent of block scheduling.
//
// Every global value is read once per block: besides x, the right-hand
// side, the diagonal and the y/z face coefficients of a plane are staged in
// LDS over rows [0, TY+3) and columns [0, TZ+3) of the halo coordinates
// (two planes kept), and the x face coefficients over three planes, so a
// cell's minus faces are its neighbours' staged plus faces.  Faces towards
// "outside" are staged as 0 (the last cell along a non-periodic axis
// already carries a 0 plus face), so the update needs no wall tests.  The
// next plane's values are fetched into registers one iteration ahead and
// stored to LDS after the current plane's updates.  Each thread updates
// fixed z-pairs (lz, lz+1): exactly one cell of a pair has the colour.
// Tile shapes (rows x z-columns, threads): the sweep and the fused residual
// use the same staging; measured on 512^3 the sweep is fastest on 16 x 64
// tiles of 512 threads and the residual on 8 x 64 tiles of 256 (FP32).
template <class T>
struct MarchTile;
template <>
struct MarchTile<float> {
  static constexpr int TY = 16, TZ = 64, NT = 512;
};
template <>
struct MarchTile<double> {
  static constexpr int TY = 8, TZ = 32, NT = 256;
};
// Prefetch registers of one staged coefficient slot of a marching kernel:
// FP64 levels hold the diagonal and the three + faces, FP32 levels the raw
// packed record, split into its bfloat16 halves only when it is staged to
// LDS (so the loads in flight are not waited for early; the halves stay
// bfloat16 in LDS, half the bytes of FP32 staging).  In LDS the "diagonal"
// plane holds the diagonal (FP64) or the shift (FP32; the diagonal is then
// op_diag of the staged shift and faces).
template <class T>
struct CoefRegs {
  T d, f0, f1, f2;
};
template <>
struct CoefRegs<float> {
  uint2 raw;  // Op16 as two dwords: x = f0 | f1 << 16, y = f2 | s << 16
};
__device__ inline void load_coef(const LevelK<double>& l, long long P, bool ok, bool all,
                                 double d_out, CoefRegs<double>& r) {
  r.f0 = ok ? l.cf[0][P] : 0.0;
  if (all) {
    r.d = ok ? l.diag[P] : d_out;
    r.f1 = ok ? l.cf[1][P] : 0.0;
    r.f2 = ok ? l.cf[2][P] : 0.0;
  }
}
__device__ inline void load_coef(const LevelK<float>& l, long long P, bool ok, bool, double,
                                 CoefRegs<float>& r) {
  r.raw = ok ? reinterpret_cast<const uint2*>(l.op)[P] : make_uint2(0u, 0u);
}
// The same values in the form they are staged to LDS: FP32 levels keep the
// bfloat16 halves (2 bytes per value; read back with lv), FP64 levels the
// doubles.
__device__ inline uint16_t coef_r0(const CoefRegs<float>& r) { return (uint16_t)(r.raw.x & 0xFFFFu); }
__device__ inline uint16_t coef_r1(const CoefRegs<float>& r) { return (uint16_t)(r.raw.x >> 16); }
__device__ inline uint16_t coef_r2(const CoefRegs<float>& r) { return (uint16_t)(r.raw.y & 0xFFFFu); }
__device__ inline uint16_t coef_rd(const CoefRegs<float>& r) { return (uint16_t)(r.raw.y >> 16); }
__device__ inline double coef_r0(const CoefRegs<double>& r) { return r.f0; }
__device__ inline double coef_r1(const CoefRegs<double>& r) { return r.f1; }
__device__ inline double coef_r2(const CoefRegs<double>& r) { return r.f2; }
__device__ inline double coef_rd(const CoefRegs<double>& r) { return r.d; }
__device__ inline float lv(uint16_t h) { return bf16_value(h); }
__device__ inline double lv(double v) { return v; }
template <class T>
using staged_t = typename std::conditional<std::is_same<T, float>::value, uint16_t, T>::type;

// Diagonal of a staged cell from the staged "diagonal" value and the six
// staged faces (+x, -x, +y, -y, +z, -z).
__device__ inline double staged_diag(double d, double, double, double, double, double, double) {
  return d;
}
__device__ inline float staged_diag(float s, float xp, float xm, float yp, float ym, float zp,
                                    float zm) {
  return op_diag(s, xp, xm, yp, ym, zp, zm);
}

template <class T>
struct ResidTile;
template <>
struct ResidTile<float> {
  static constexpr int TY = 8, TZ = 64, NT = 256;
};
template <>
struct ResidTile<double> {
  static constexpr int TY = 8, TZ = 32, NT = 256;
};


//
// DOTS: the sweep's output is the preconditioned residual z_T of the
// conjugate-gradient iteration (last sweep of a V-cycle on the finest
// level); the block partials of z.r and z.q with z = sigma z_T are formed
// while writing it (q may be null), in place of a separate pass.
template <class T, int TY, int TZ, int NT, int FINE, int DOTS>
__global__ void __launch_bounds__(NT)
k_rbgs_march(LevelK<T> l, int first_color, int zero_init, int xc, double sigma,
             const double* __restrict__ rv, const double* __restrict__ qv,
             double* __restrict__ part) {
  static_assert(TZ % 2 == 0, "z-pairs need an even tile width");
  constexpr int HY = TY + 4, HZ = TZ + 4, PL = HY * HZ;   // x planes (halo 2)
  constexpr int CR = TY + 3, CZ = TZ + 3, CN = CR * CZ;    // staged coefficient region
  constexpr int CP = CR * HZ;                               // coefficient plane (row stride HZ)
  constexpr int NLX = (PL + NT - 1) / NT;
  constexpr int NLC = (CN + NT - 1) / NT;
  constexpr int NRED = ((TY + 2) * (TZ + 2) / 2 + NT - 1) / NT;
  constexpr int NBLK = (TY * TZ / 2 + NT - 1) / NT;
  __shared__ T xs[4 * PL];
  using CT = staged_t<T>;
  __shared__ T bsh[2 * CP];     // right-hand side (planes p-1, p)
  __shared__ CT cs[3][2 * CP];  // diag / shift, y faces, z faces (planes p-1, p)
  __shared__ CT c0s[3 * CP];    // x faces (planes p-2, p-1, p)
  const int ntz = (l.nz + TZ - 1) / TZ, nty = (l.ny + TY - 1) / TY;
  int bid = xcd_tile(blockIdx.x, gridDim.x);
  const int tz = bid % ntz;
  bid /= ntz;
  const int ty = bid % nty;
  const int cx = bid / nty;
  const int y0 = ty * TY - 2, z0 = tz * TZ - 2;  // global index of LDS row / column 0
  const int xa = cx * xc, xb = min(xa + xc, l.nx);
  const int plane = l.ny * l.nz;
  const int tid = threadIdx.x;
  auto wrap = [&](int g, int n, int per) -> int {
    if (g >= 0 && g < n) return g;
    if (!per) return -1;
    return g < 0 ? g + n : g - n;
  };
  auto inplane = [&](int ly, int lz) -> int {
    const int gy = wrap(y0 + ly, l.ny, l.per[1]), gz = wrap(z0 + lz, l.nz, l.per[2]);
    return (gy >= 0 && gz >= 0) ? gy * l.nz + gz : -1;
  };
  // in-plane offsets (or -1 outside) of this thread's staging slots
  int xoff[NLX], coff[NLC];
#pragma unroll
  for (int j = 0; j < NLX; ++j) {
    const int t = tid + j * NT;
    xoff[j] = t < PL ? inplane(t / HZ, t % HZ) : -1;
  }
#pragma unroll
  for (int j = 0; j < NLC; ++j) {
    const int t = tid + j * NT;
    coff[j] = t < CN ? inplane(t / CZ, t % CZ) : -1;
  }
  struct Buf {
    T x[NLX];
    T b[NLC];
    CoefRegs<T> k[NLC];
  };
  auto fetch_x = [&](int p, Buf& B) {
    const int gx = wrap(p, l.nx, l.per[0]);
#pragma unroll
    for (int j = 0; j < NLX; ++j)
      B.x[j] = (!zero_init && gx >= 0 && xoff[j] >= 0) ? l.x[gx * plane + xoff[j]] : T(0);
  };
  auto stash_x = [&](int p, const Buf& B) {
    T* dst = xs + pmod(p, 4) * PL;
#pragma unroll
    for (int j = 0; j < NLX; ++j) {
      const int t = tid + j * NT;
      if (t < PL) dst[t] = B.x[j];
    }
  };
  auto fetch_c = [&](int p, bool all, Buf& B) {
    const int gx = wrap(p, l.nx, l.per[0]);
#pragma unroll
    for (int j = 0; j < NLC; ++j) {
      const bool ok = gx >= 0 && coff[j] >= 0;
      const int P = ok ? gx * plane + coff[j] : 0;
      load_coef(l, P, ok, all, 1.0, B.k[j]);
      if (all) B.b[j] = ok ? l.b[P] : T(0);
    }
  };
  auto stash_c = [&](int p, bool all, const Buf& B) {
    const int s2 = pmod(p, 2) * CP, s3 = pmod(p, 3) * CP;
#pragma unroll
    for (int j = 0; j < NLC; ++j) {
      const int t = tid + j * NT;
      if (t >= CN) continue;
      const int li = (t / CZ) * HZ + t % CZ;
      c0s[s3 + li] = coef_r0(B.k[j]);
      if (all) {
        bsh[s2 + li] = B.b[j];
        cs[0][s2 + li] = coef_rd(B.k[j]);
        cs[1][s2 + li] = coef_r1(B.k[j]);
        cs[2][s2 + li] = coef_r2(B.k[j]);
      }
    }
  };
  // Update the cells of `color` on plane p over rows [lo, lo+ey) and
  // z-pairs starting at lo, lo+2, ... (ez columns); NP pairs per thread.
  auto update = [&](auto npc, int p, int color, int lo, int ey, int ez) {
    constexpr int NP = decltype(npc)::value;
    if (wrap(p, l.nx, l.per[0]) < 0) return;
    T* cur = xs + pmod(p, 4) * PL;
    const T* prv = xs + pmod(p - 1, 4) * PL;
    const T* nxt = xs + pmod(p + 1, 4) * PL;
    const int s2 = pmod(p, 2) * CP;
    const T* cb = bsh + s2;
    const CT* cd = cs[0] + s2;
    const CT* c1 = cs[1] + s2;
    const CT* c2 = cs[2] + s2;
    const CT* c0c = c0s + pmod(p, 3) * CP;
    const CT* c0m = c0s + pmod(p - 1, 3) * CP;
    const int half = ez / 2;
    int qs[NP];
    T nv[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      const int t = tid + j * NT;
      qs[j] = -1;
      if (t >= ey * half) continue;
      const int ly = lo + t / half;
      int lz = lo + 2 * (t % half);
      if (((p + y0 + ly + z0 + lz) & 1) != color) ++lz;
      if (wrap(y0 + ly, l.ny, l.per[1]) < 0 || wrap(z0 + lz, l.nz, l.per[2]) < 0) continue;
      const int q = ly * HZ + lz;
      qs[j] = q;
      // same order as row_terms: +x, -x, +y, -y, +z, -z
      const T fxp = lv(c0c[q]), fxm = lv(c0m[q]), fyp = lv(c1[q]), fym = lv(c1[q - HZ]);
      const T fzp = lv(c2[q]), fzm = lv(c2[q - 1]);
      T off = fxp * nxt[q];
      off += fxm * prv[q];
      off += fyp * cur[q + HZ];
      off += fym * cur[q - HZ];
      off += fzp * cur[q + 1];
      off += fzm * cur[q - 1];
      nv[j] = (cb[q] + off) / staged_diag(lv(cd[q]), fxp, fxm, fyp, fym, fzp, fzm);
    }
#pragma unroll
    for (int j = 0; j < NP; ++j)
      if (qs[j] >= 0) cur[qs[j]] = nv[j];
  };
  double zr = 0.0, zq = 0.0;
  Buf A, B;
  fetch_x(xa - 2, A);
  stash_x(xa - 2, A);
  fetch_x(xa - 1, A);
  stash_x(xa - 1, A);
  fetch_x(xa, A);
  stash_x(xa, A);
  fetch_c(xa - 2, false, A);
  stash_c(xa - 2, false, A);
  fetch_c(xa - 1, true, A);
  stash_c(xa - 1, true, A);
  __syncthreads();
  // registers run two planes ahead of LDS: plane p stores what plane p-1
  // fetched (x of p+2, coefficients of p+1) and fetches x of p+3 and the
  // coefficients of p+2 into the other buffer
  fetch_x(xa + 1, A);
  fetch_c(xa, true, A);
  constexpr int NW = (TY * TZ + NT - 1) / NT;  // written cells per thread and plane
  auto step = [&](int p, const Buf& now, Buf& ahead) {
    // in LDS: x planes p-2..p+1, coefficients of p-1 and p, x faces of p-2..p
    if (p + 3 <= xb + 1) fetch_x(p + 3, ahead);
    if (p + 2 <= xb) fetch_c(p + 2, true, ahead);
    const int q = p - 1;
    // r and q of the cells written below, in flight during both updates
    double rpre[NW], qpre[NW];
    if (DOTS && q >= xa) {
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        const int t = tid + k * NT;
        const int gy = ty * TY + t / TZ, gz = tz * TZ + t % TZ;
        const bool ok = t < TY * TZ && gy < l.ny && gz < l.nz;
        const int P = ok ? q * plane + gy * l.nz + gz : 0;
        rpre[k] = ok ? rv[P] : 0.0;
        qpre[k] = (ok && qv) ? qv[P] : 0.0;
      }
    }
    update(std::integral_constant<int, NRED>(), p, first_color, 1, TY + 2, TZ + 2);
    __syncthreads();
    if (q >= xa) {
      update(std::integral_constant<int, NBLK>(), q, 1 - first_color, 2, TY, TZ);
      __syncthreads();
      const T* src = xs + pmod(q, 4) * PL;
#pragma unroll
      for (int k = 0; k < NW; ++k) {
        const int t = tid + k * NT;
        const int lz = t % TZ, ly = t / TZ;
        const int gy = ty * TY + ly, gz = tz * TZ + lz;
        if (t < TY * TZ && gy < l.ny && gz < l.nz) {
          const int P = q * plane + gy * l.nz + gz;
          const T v = src[(ly + 2) * HZ + lz + 2];
          l.x2[P] = v;
          if (DOTS) {
            const double zv = sigma * (double)v;
            zr += zv * rpre[k];
            if (qv) zq += zv * qpre[k];
          }
        }
      }
    }
    // the slots of plane p-2 (x) and p-1 (coefficients) are free once plane
    // p-1 is done
    if (p + 2 <= xb + 1) stash_x(p + 2, now);
    if (p + 1 <= xb) stash_c(p + 1, true, now);
    __syncthreads();
  };
  for (int p = xa - 1; p <= xb; p += 2) {
    step(p, A, B);
    if (p + 1 <= xb) step(p + 1, B, A);
  }
  if (DOTS) {
    double v[2] = {zr, zq};
    const int im[2] = {0, 0};
    const int sl[2] = {RS_ZR, RS_ZQ};
    block_reduce_store<2, NT>(v, im, sl, part);
  }
}

// x planes per block of the marching sweep: 32, or fewer (down to 8) when
// that is what it takes to reach min_tiles workgroups; 0 when the level does
// not fit the tiles (the caller then sweeps colour by colour).
template <class T, int TY, int TZ>
int march_chunk_for(const LevelK<T>& l, long long min_tiles) {
  if (!l.x2 || l.nz < TZ || l.ny < TY || l.nx < 4 || l.N >= (1LL << 31)) return 0;
  const long long tiles = (long long)((l.ny + TY - 1) / TY) * ((l.nz + TZ - 1) / TZ);
  for (int xc = 32; xc >= 8; xc /= 2)
    if (tiles * ((l.nx + xc - 1) / xc) >= min_tiles) return xc;
  return 0;
}

template <class T>
int march_chunk(const LevelK<T>& l, long long min_tiles) {
  return march_chunk_for<T, MarchTile<T>::TY, MarchTile<T>::TZ>(l, min_tiles);
}

template <class T>
bool rbgs_march_fits(const LevelK<T>& l, long long min_tiles) {
  return march_chunk(l, min_tiles) > 0;
}

template <class T>
bool launch_rbgs_march(hipStream_t s, const LevelK<T>& l, int first_color, int zero_init,
                       int fine, long long min_tiles, const SweepDots* dots) {
  constexpr int TY = MarchTile<T>::TY, TZ = MarchTile<T>::TZ;
  const int xc = march_chunk(l, min_tiles);
  if (xc == 0) return false;
  const int nb = ((l.ny + TY - 1) / TY) * ((l.nz + TZ - 1) / TZ) * ((l.nx + xc - 1) / xc);
  if (dots && nb > kPartCap) return false;
  constexpr int NT = MarchTile<T>::NT;
  if (dots)
    hipLaunchKernelGGL((k_rbgs_march<T, TY, TZ, NT, 1, 1>), dim3(nb), dim3(NT), 0, s, l,
                       first_color, zero_init, xc, dots->sigma, dots->r, dots->q, dots->part);
  else if (fine)
    hipLaunchKernelGGL((k_rbgs_march<T, TY, TZ, NT, 1, 0>), dim3(nb), dim3(NT), 0, s, l,
                       first_color, zero_init, xc, 0.0, nullptr, nullptr, nullptr);
  else
    hipLaunchKernelGGL((k_rbgs_march<T, TY, TZ, NT, 0, 0>), dim3(nb), dim3(NT), 0, s, l,
                       first_color, zero_init, xc, 0.0, nullptr, nullptr, nullptr);
  return true;
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_mg_residual(LevelK<T> l) {
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < l.N;
       idx += (long long)blockDim.x * gridDim.x) {
    int c[3];
    cell_ijk(idx, l.ny, l.nz, c[0], c[1], c[2]);
    T off, dg;
    row_terms(l, c, idx, true, off, dg);
    l.r[idx] = l.b[idx] - (dg * l.x[idx] - off);
  }
}

template <class T>
void launch_mg_residual(hipStream_t s, const LevelK<T>& l) {
  long long g = (l.N + kBlock - 1) / kBlock;
  hipLaunchKernelGGL((k_mg_residual<T>), dim3((unsigned)(g < 65536 ? g : 65536)), dim3(kBlock), 0,
                     s, l);
}

// Fine index along one axis for a restriction / prolongation stencil:
// mirror at non-periodic walls, wrap when periodic.
__device__ inline int fold(int v, int n, int per) {
  if (v < 0) return per ? v + n : -1 - v;
  if (v >= n) return per ? v - n : 2 * n - 1 - v;
  return v;
}

// Full weighting R = P^T / 8: weights (1,3,3,1)/8 per axis over fine 2I-1..2I+2.
template <class T>
__global__ void __launch_bounds__(kBlock) k_restrict(LevelK<T> f, LevelK<T> c) {
  const double w[4] = {0.125, 0.375, 0.375, 0.125};
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < c.N;
       idx += (long long)blockDim.x * gridDim.x) {
    int I, J, K;
    cell_ijk(idx, c.ny, c.nz, I, J, K);
    double s = 0.0;
    for (int a = 0; a < 4; ++a) {
      const int i = fold(2 * I - 1 + a, f.nx, f.per[0]);
      for (int b = 0; b < 4; ++b) {
        const int j = fold(2 * J - 1 + b, f.ny, f.per[1]);
        double sz = 0.0;
        for (int d = 0; d < 4; ++d) {
          const int kk = fold(2 * K - 1 + d, f.nz, f.per[2]);
          sz += w[d] * (double)f.r[cell_index(i, j, kk, f.ny, f.nz)];
        }
        s += w[a] * w[b] * sz;
      }
    }
    c.b[idx] = (T)s;
  }
}

template <class T>
void launch_restrict(hipStream_t s, const LevelK<T>& f, const LevelK<T>& c) {
  hipLaunchKernelGGL((k_restrict<T>), dim3(red_grid(c.N)), dim3(kBlock), 0, s, f, c);
}

// Residual r = b - A x on level f fused with the full-weighting restriction
// of r into c.b (the arithmetic of k_mg_residual then k_restrict, in their
// order), marching along fine x planes; r itself is not stored.  Tiles and
// LDS staging are those of k_rbgs_march; a block owns TY x TZ fine cells of
// the (y, z) plane and fine planes [xa, xb) (xa even), i.e. whole coarse
// cells.  Per fine plane: r on the tile plus a 1-cell ring into an LDS plane
// (two kept), then each owned coarse cell adds that plane's terms to its
// running sum; a coarse plane is written once its fourth fine plane is in.
// Restriction reads fold the stencil at non-periodic walls (the fine plane,
// row or column 0 stands for -1, and n-1 for n); one barrier per plane.
template <class T, int TY, int TZ, int NT>
__global__ void __launch_bounds__(NT)
k_resid_restrict_march(LevelK<T> l, LevelK<T> c, int xc) {
  static_assert(TZ % 2 == 0 && TY % 2 == 0, "tiles hold whole coarse cells");
  constexpr int HY = TY + 4, HZ = TZ + 4, PL = HY * HZ;   // x planes (halo 2)
  constexpr int CR = TY + 3, CZ = TZ + 3, CN = CR * CZ;    // staged coefficient region
  constexpr int CP = CR * HZ;
  constexpr int NLX = (PL + NT - 1) / NT;
  constexpr int NLC = (CN + NT - 1) / NT;
  constexpr int RR = TY + 2, RZ = TZ + 2, RN = RR * RZ;   // residual slots: rows/cols 1..
  constexpr int NRES = (RN + NT - 1) / NT;
  constexpr int NCC = (TY / 2) * (TZ / 2);                 // coarse cells per tile
  static_assert(NCC <= NT, "one coarse cell per thread");
  __shared__ T xs[4 * PL];
  using CT = staged_t<T>;
  __shared__ T bsh[2 * CP];     // right-hand side (planes i, i+1)
  __shared__ CT cs[3][2 * CP];  // diag / shift, y faces, z faces (planes i, i+1)
  __shared__ CT c0s[3 * CP];    // x faces (planes i-1, i, i+1)
  __shared__ T rs[2][CP];      // residual planes (same coordinates)
  const int ntz = (l.nz + TZ - 1) / TZ, nty = (l.ny + TY - 1) / TY;
  int bid = xcd_tile(blockIdx.x, gridDim.x);
  const int tz = bid % ntz;
  bid /= ntz;
  const int ty = bid % nty;
  const int cx = bid / nty;
  const int y0 = ty * TY - 2, z0 = tz * TZ - 2;  // global index of LDS row / column 0
  const int xa = cx * xc, xb = min(xa + xc, l.nx);
  const int plane = l.ny * l.nz;
  const int tid = threadIdx.x;
  const int px = l.per[0];
  auto wrap = [&](int g, int n, int per) -> int {
    if (g >= 0 && g < n) return g;
    if (!per) return -1;
    return g < 0 ? g + n : g - n;
  };
  auto inplane = [&](int ly, int lz) -> int {
    const int gy = wrap(y0 + ly, l.ny, l.per[1]), gz = wrap(z0 + lz, l.nz, l.per[2]);
    return (gy >= 0 && gz >= 0) ? gy * l.nz + gz : -1;
  };
  int xoff[NLX], coff[NLC];
#pragma unroll
  for (int j = 0; j < NLX; ++j) {
    const int t = tid + j * NT;
    xoff[j] = t < PL ? inplane(t / HZ, t % HZ) : -1;
  }
#pragma unroll
  for (int j = 0; j < NLC; ++j) {
    const int t = tid + j * NT;
    coff[j] = t < CN ? inplane(t / CZ, t % CZ) : -1;
  }
  // residual slots of this thread (LDS index, or -1 when outside the grid)
  int rq[NRES];
#pragma unroll
  for (int j = 0; j < NRES; ++j) {
    const int t = tid + j * NT;
    rq[j] = -1;
    if (t < RN) {
      const int ly = 1 + t / RZ, lz = 1 + t % RZ;
      if (inplane(ly, lz) >= 0) rq[j] = ly * HZ + lz;
    }
  }
  // this thread's coarse cell and the LDS rows / columns of its stencil
  const bool has_cc = tid < NCC;
  const int cj = tid / (TZ / 2), ck = tid % (TZ / 2);
  const int J = ty * (TY / 2) + cj, K = tz * (TZ / 2) + ck;
  const bool cc_real = has_cc && J < c.ny && K < c.nz;
  int srow[4], scol[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int vy = 2 * J - 1 + b, vz = 2 * K - 1 + b;
    srow[b] = (l.per[1] ? vy : fold(vy, l.ny, 0)) - y0;
    scol[b] = (l.per[2] ? vz : fold(vz, l.nz, 0)) - z0;
  }
  struct Buf {  // as in k_rbgs_march
    T x[NLX];
    T b[NLC];
    CoefRegs<T> k[NLC];
  };
  // Every lane loads (slots outside the grid read cell 0) and those slots
  // are zeroed when staged, so no loaded value is used before its staging
  // (0.77 against 1.01 ms with masked loads on the 512^3 finest level; the
  // sweep measured the other way round and keeps masked loads).
  auto fetch_x = [&](int p, Buf& B) {
    const int gx = wrap(p, l.nx, px);
#pragma unroll
    for (int j = 0; j < NLX; ++j)
      B.x[j] = l.x[(gx >= 0 && xoff[j] >= 0) ? gx * plane + xoff[j] : 0];
  };
  auto stash_x = [&](int p, const Buf& B) {
    T* dst = xs + pmod(p, 4) * PL;
    const bool pok = wrap(p, l.nx, px) >= 0;
#pragma unroll
    for (int j = 0; j < NLX; ++j) {
      const int t = tid + j * NT;
      if (t < PL) dst[t] = (pok && xoff[j] >= 0) ? B.x[j] : T(0);
    }
  };
  auto fetch_c = [&](int p, bool all, Buf& B) {
    const int gx = wrap(p, l.nx, px);
#pragma unroll
    for (int j = 0; j < NLC; ++j) {
      const int P = (gx >= 0 && coff[j] >= 0) ? gx * plane + coff[j] : 0;
      load_coef(l, P, true, all, 0.0, B.k[j]);
      if (all) B.b[j] = l.b[P];
    }
  };
  auto stash_c = [&](int p, bool all, const Buf& B) {
    const int s2 = pmod(p, 2) * CP, s3 = pmod(p, 3) * CP;
    const bool pok = wrap(p, l.nx, px) >= 0;
#pragma unroll
    for (int j = 0; j < NLC; ++j) {
      const int t = tid + j * NT;
      if (t >= CN) continue;
      const int li = (t / CZ) * HZ + t % CZ;
      const bool ok = pok && coff[j] >= 0;
      c0s[s3 + li] = ok ? coef_r0(B.k[j]) : CT(0);
      if (all) {
        bsh[s2 + li] = ok ? B.b[j] : T(0);
        cs[0][s2 + li] = ok ? coef_rd(B.k[j]) : CT(0);
        cs[1][s2 + li] = ok ? coef_r1(B.k[j]) : CT(0);
        cs[2][s2 + li] = ok ? coef_r2(B.k[j]) : CT(0);
      }
    }
  };
  // fine planes whose residual this block needs: xa-1 .. xb (periodic), or
  // clipped to the grid (the fold repeats planes 0 and nx-1)
  const int i0 = px ? xa - 1 : max(xa - 1, 0);
  const int i1 = px ? xb : min(xb, l.nx - 1);
  const double w[4] = {0.125, 0.375, 0.375, 0.125};
  const int cplane = c.ny * c.nz;
  const int Ilo = xa / 2, Ihi = xb / 2;  // coarse planes [Ilo, Ihi) of this block
  double acc[2] = {0.0, 0.0};
  // add fine plane i's terms as stencil position a of coarse plane I
  auto add_terms = [&](const double (&sz)[4], int I, int a) {
    if (I < Ilo || I >= Ihi) return;
    double& s = acc[I & 1];
    if (a == 0) s = 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b) s += w[a] * w[b] * sz[b];
    if (a == 3 && cc_real) c.b[I * cplane + J * c.nz + K] = (T)s;
  };
  Buf A, B;
  fetch_x(i0 - 1, A);
  stash_x(i0 - 1, A);
  fetch_x(i0, A);
  stash_x(i0, A);
  fetch_x(i0 + 1, A);
  stash_x(i0 + 1, A);
  fetch_c(i0 - 1, false, A);
  stash_c(i0 - 1, false, A);
  fetch_c(i0, true, A);
  stash_c(i0, true, A);
  fetch_x(i0 + 2, A);
  fetch_c(i0 + 1, true, A);
  __syncthreads();
  auto step = [&](int i, const Buf& now, Buf& ahead) {
    // in LDS: x planes i-1..i+1, coefficients of i, x faces of i-1 and i
    if (i + 3 <= i1 + 1) fetch_x(i + 3, ahead);
    if (i + 2 <= i1) fetch_c(i + 2, true, ahead);
    {
      const T* cur = xs + pmod(i, 4) * PL;
      const T* prv = xs + pmod(i - 1, 4) * PL;
      const T* nxt = xs + pmod(i + 1, 4) * PL;
      const int s2 = pmod(i, 2) * CP;
      const T* cb = bsh + s2;
      const CT* cd = cs[0] + s2;
      const CT* c1 = cs[1] + s2;
      const CT* c2 = cs[2] + s2;
      const CT* c0c = c0s + pmod(i, 3) * CP;
      const CT* c0m = c0s + pmod(i - 1, 3) * CP;
      T* r = rs[i & 1];
#pragma unroll
      for (int j = 0; j < NRES; ++j) {
        const int q = rq[j];
        if (q < 0) continue;
        // k_mg_residual: b - (diag x - offdiag), offdiag in the order of row_terms
        const T fxp = lv(c0c[q]), fxm = lv(c0m[q]), fyp = lv(c1[q]), fym = lv(c1[q - HZ]);
        const T fzp = lv(c2[q]), fzm = lv(c2[q - 1]);
        T off = 0;
        off += fxp * nxt[q];
        off += fxm * prv[q];
        off += fyp * cur[q + HZ];
        off += fym * cur[q - HZ];
        off += fzp * cur[q + 1];
        off += fzm * cur[q - 1];
        const T dq = staged_diag(lv(cd[q]), fxp, fxm, fyp, fym, fzp, fzm);
        r[q] = cb[q] - (dq * cur[q] - off);
      }
    }
    if (i + 2 <= i1 + 1) stash_x(i + 2, now);
    if (i + 1 <= i1) stash_c(i + 1, true, now);
    __syncthreads();
    if (cc_real) {
      const T* r = rs[i & 1];
      double sz[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        double t = 0.0;
#pragma unroll
        for (int d = 0; d < 4; ++d) t += w[d] * (double)r[srow[b] * HZ + scol[d]];
        sz[b] = t;
      }
      // fine plane i is stencil position a = i + 1 - 2I of coarse plane I
      const int Ia = (i + 1) >> 1;  // positions 0 / 1
      if (!px && i == 0) add_terms(sz, 0, 0);              // plane -1 folds onto 0
      add_terms(sz, Ia, i + 1 - 2 * Ia);
      add_terms(sz, Ia - 1, i + 3 - 2 * Ia);               // positions 2 / 3
      if (!px && i == l.nx - 1) add_terms(sz, c.nx - 1, 3);  // plane nx folds onto nx-1
    }
  };
  for (int i = i0; i <= i1; i += 2) {
    step(i, A, B);
    if (i + 1 <= i1) step(i + 1, B, A);
  }
}

template <class T>
bool resid_restrict_fits(const LevelK<T>& f, long long min_tiles) {
  return (f.nx % 2 == 0 && f.ny % 2 == 0 && f.nz % 2 == 0) &&
         march_chunk_for<T, ResidTile<T>::TY, ResidTile<T>::TZ>(f, min_tiles) > 0;
}

template <class T>
bool launch_resid_restrict_march(hipStream_t s, const LevelK<T>& f, const LevelK<T>& c,
                                 long long min_tiles) {
  constexpr int TY = ResidTile<T>::TY, TZ = ResidTile<T>::TZ;
  if (!resid_restrict_fits(f, min_tiles)) return false;
  const int xc = march_chunk_for<T, TY, TZ>(f, min_tiles);
  const int nb = ((f.ny + TY - 1) / TY) * ((f.nz + TZ - 1) / TZ) * ((f.nx + xc - 1) / xc);
  constexpr int NT = ResidTile<T>::NT;
  hipLaunchKernelGGL((k_resid_restrict_march<T, TY, TZ, NT>), dim3(nb), dim3(NT), 0, s, f, c, xc);
  return true;
}

// Trilinear cell-centred prolongation (weights 3/4, 1/4 per axis), added to x.
template <class T>
__global__ void __launch_bounds__(kBlock) k_prolong(LevelK<T> c, LevelK<T> f) {
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < f.N;
       idx += (long long)blockDim.x * gridDim.x) {
    int i, j, k;
    cell_ijk(idx, f.ny, f.nz, i, j, k);
    int I[2], J[2], K[2];
    I[0] = i >> 1; J[0] = j >> 1; K[0] = k >> 1;
    I[1] = (i & 1) ? I[0] + 1 : I[0] - 1;
    J[1] = (j & 1) ? J[0] + 1 : J[0] - 1;
    K[1] = (k & 1) ? K[0] + 1 : K[0] - 1;
    // walls: mirror (the neighbour is the cell itself); periodic: wrap
    I[1] = (I[1] < 0 || I[1] >= c.nx) ? (c.per[0] ? (I[1] + c.nx) % c.nx : I[0]) : I[1];
    J[1] = (J[1] < 0 || J[1] >= c.ny) ? (c.per[1] ? (J[1] + c.ny) % c.ny : J[0]) : J[1];
    K[1] = (K[1] < 0 || K[1] >= c.nz) ? (c.per[2] ? (K[1] + c.nz) % c.nz : K[0]) : K[1];
    const double w[2] = {0.75, 0.25};
    double s = 0.0;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int d = 0; d < 2; ++d)
          s += w[a] * w[b] * w[d] * (double)c.x[cell_index(I[a], J[b], K[d], c.ny, c.nz)];
    f.x[idx] = (T)((double)f.x[idx] + s);
  }
}

// The same prolongation with one thread per coarse cell: its 8 fine children
// need only the 3x3x3 coarse neighbourhood (27 loads for 8 outputs instead of
// 8 per output), and children adjacent in z are read and written as pairs.
// Per child the sum is k_prolong's, in its order.
template <class T>
__global__ void __launch_bounds__(kBlock) k_prolong_cc(LevelK<T> c, LevelK<T> f) {
  const int cplane = c.ny * c.nz, fplane = f.ny * f.nz;
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < (int)c.N;
       idx += blockDim.x * gridDim.x) {
    const int I = idx / cplane, rem = idx - I * cplane;
    const int J = rem / c.nz, K = rem - J * c.nz;
    // coarse indices below / at / above along each axis, with k_prolong's
    // boundary rule (mirror: the cell itself; periodic: wrap)
    auto nb = [](int v, int n, int per, int s) {
      const int u = v + s;
      if (u >= 0 && u < n) return u;
      return per ? (u + n) % n : v;
    };
    const int Ic[3] = {nb(I, c.nx, c.per[0], -1), I, nb(I, c.nx, c.per[0], 1)};
    const int Jc[3] = {nb(J, c.ny, c.per[1], -1), J, nb(J, c.ny, c.per[1], 1)};
    const int Kc[3] = {nb(K, c.nz, c.per[2], -1), K, nb(K, c.nz, c.per[2], 1)};
    double cv[3][3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int d = 0; d < 3; ++d) cv[a][b][d] = (double)c.x[Ic[a] * cplane + Jc[b] * c.nz + Kc[d]];
    const double w[2] = {0.75, 0.25};
#pragma unroll
    for (int ca = 0; ca < 2; ++ca)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        // child (2I+ca, 2J+cb, 2K+cd): own coarse index, then the one on its side
        const int ia[2] = {1, ca ? 2 : 0}, jb[2] = {1, cb ? 2 : 0};
        const int fi = (2 * I + ca) * fplane + (2 * J + cb) * f.nz + 2 * K;
        T out[2];
#pragma unroll
        for (int cd = 0; cd < 2; ++cd) {
          const int kd[2] = {1, cd ? 2 : 0};
          double s = 0.0;
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
              for (int d = 0; d < 2; ++d) s += w[a] * w[b] * w[d] * cv[ia[a]][jb[b]][kd[d]];
          out[cd] = (T)((double)f.x[fi + cd] + s);
        }
        f.x[fi] = out[0];
        f.x[fi + 1] = out[1];
      }
  }
}

template <class T>
void launch_prolong(hipStream_t s, const LevelK<T>& c, const LevelK<T>& f) {
  if (c.N < (1LL << 31) / 8 && f.nx == 2 * c.nx && f.ny == 2 * c.ny && f.nz == 2 * c.nz) {
    const long long g = (c.N + kBlock - 1) / kBlock;
    hipLaunchKernelGGL((k_prolong_cc<T>), dim3((unsigned)(g < 65536 ? g : 65536)), dim3(kBlock),
                       0, s, c, f);
    return;
  }
  long long g = (f.N + kBlock - 1) / kBlock;
  hipLaunchKernelGGL((k_prolong<T>), dim3((unsigned)(g < 65536 ? g : 65536)), dim3(kBlock), 0, s,
                     c, f);
}

// ---------------------------------------------------------------------------
// defect correction in FP64
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(kBlock)
k_cast_scale(long long N, const double* __restrict__ r, double inv_sigma, T* __restrict__ b) {
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < N;
       idx += (long long)blockDim.x * gridDim.x)
    b[idx] = (T)(r[idx] * inv_sigma);
}

template <class T>
void launch_cast_scale(hipStream_t s, long long N, const double* r, double inv_sigma, T* b) {
  long long g = (N + kBlock - 1) / kBlock;
  hipLaunchKernelGGL((k_cast_scale<T>), dim3((unsigned)(g < 65536 ? g : 65536)), dim3(kBlock), 0,
                     s, N, r, inv_sigma, b);
}

// dE_out = dE_in + sigma_x x;  r = rS - S dE_out;  b = r * inv_sigma_b
template <class T>
__global__ void __launch_bounds__(kBlock)
k_accum_defect(StepK k, DefectArgs a, const T* __restrict__ x, T* __restrict__ b,
               double* __restrict__ part) {
  const int per[3] = {k.bc[0] == RH_BC_PERIODIC, k.bc[2] == RH_BC_PERIODIC,
                      k.bc[4] == RH_BC_PERIODIC};
  const int nd[3] = {k.nx, k.ny, k.nz};
  double s2w = 0.0, rmax = 0.0, s2 = 0.0;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < k.N;
       idx += (long long)blockDim.x * gridDim.x) {
    int c[3];
    cell_ijk(idx, k.ny, k.nz, c[0], c[1], c[2]);
    // x may be null (only the norms of rS are wanted)
    const double dP = (a.first ? 0.0 : a.dE_in[idx]) + (x ? a.sigma_x * (double)x[idx] : 0.0);
    double off = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int q[3];
      if (neighbour(c, nd, per, d, +1, q)) {
        const long long Q = cell_index(q[0], q[1], q[2], k.ny, k.nz);
        const double dQ = (a.first ? 0.0 : a.dE_in[Q]) + (x ? a.sigma_x * (double)x[Q] : 0.0);
        off += a.cf[d][idx] * dQ;
      }
      if (neighbour(c, nd, per, d, -1, q)) {
        const long long Q = cell_index(q[0], q[1], q[2], k.ny, k.nz);
        const double dQ = (a.first ? 0.0 : a.dE_in[Q]) + (x ? a.sigma_x * (double)x[Q] : 0.0);
        off += a.cf[d][Q] * dQ;
      }
    }
    const double r = a.rS[idx] - (a.diag64[idx] * dP - off);
    a.dE_out[idx] = dP;
    b[idx] = (T)(r * a.inv_sigma_b);
    s2w += (r / k.E_s) * (r / k.E_s);
    s2 += r * r;
    rmax = fmax(rmax, fabs(r));
  }
  double v[3] = {s2w, rmax, s2};
  const int im[3] = {0, 1, 0};
  const int sl[3] = {RS_FE2, RS_RMAX, RS_R2};
  block_reduce_store<3>(v, im, sl, part);
}

template <class T>
void launch_accum_defect(hipStream_t s, const StepK& k, const DefectArgs& a, const T* x, T* b,
                         double* part) {
  hipLaunchKernelGGL((k_accum_defect<T>), dim3(red_grid(k.N)), dim3(kBlock), 0, s, k, a, x, b,
                     part);
}

// ---------------------------------------------------------------------------
// flexible preconditioned conjugate gradients in FP64 (V-cycle preconditioner)
// ---------------------------------------------------------------------------
// A: p = z + beta p (p = z when first);  q = S p;  partial p.q
template <class T>
__global__ void __launch_bounds__(kBlock)
k_pcg_dir(StepK k, const double* __restrict__ diag, const double* __restrict__ cfx,
          const double* __restrict__ cfy, const double* __restrict__ cfz,
          const T* __restrict__ zT, double sigma, const double* __restrict__ p_in,
          double* __restrict__ p_out, double* __restrict__ q, double beta, int first,
          double* __restrict__ xv, double alpha_prev, int xmode, double* __restrict__ part) {
  const int per[3] = {k.bc[0] == RH_BC_PERIODIC, k.bc[2] == RH_BC_PERIODIC,
                      k.bc[4] == RH_BC_PERIODIC};
  const int nd[3] = {k.nx, k.ny, k.nz};
  const double* cf[3] = {cfx, cfy, cfz};
  double pq = 0.0;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < k.N;
       idx += (long long)blockDim.x * gridDim.x) {
    int c[3];
    cell_ijk(idx, k.ny, k.nz, c[0], c[1], c[2]);
    const double zP = sigma * (double)zT[idx];
    const double pP = first ? zP : zP + beta * p_in[idx];
    double off = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int qq[3];
      if (neighbour(c, nd, per, d, +1, qq)) {
        const long long Q = cell_index(qq[0], qq[1], qq[2], k.ny, k.nz);
        const double zQ = sigma * (double)zT[Q];
        off += cf[d][idx] * (first ? zQ : zQ + beta * p_in[Q]);
      }
      if (neighbour(c, nd, per, d, -1, qq)) {
        const long long Q = cell_index(qq[0], qq[1], qq[2], k.ny, k.nz);
        const double zQ = sigma * (double)zT[Q];
        off += cf[d][Q] * (first ? zQ : zQ + beta * p_in[Q]);
      }
    }
    const double qP = diag[idx] * pP - off;
    p_out[idx] = pP;
    q[idx] = qP;
    pq += pP * qP;
    if (xmode) xv[idx] = (xmode == 2 ? xv[idx] : 0.0) + alpha_prev * p_in[idx];
  }
  double v[1] = {pq};
  const int im[1] = {0};
  const int sl[1] = {RS_PQ};
  block_reduce_store<1>(v, im, sl, part);
}

// The same as k_pcg_dir, marching along x (the layout of k_rbgs_march): a
// block owns a TY x TZ tile of the (y, z) plane over xc consecutive planes.
// The current plane's p (tile + 1-cell ring) lives in LDS; each thread keeps
// p of its own cells on the planes before and after in registers, and the
// x face of the plane before; the y and z minus faces are read where the
// block reads them as plus faces of its own cells (cache hits).  Loads are
// issued one iteration before the one that consumes them.  The sum is formed
// in the order of k_pcg_dir (+x, -x, +y, -y, +z, -z).
constexpr int kDirTY = 8, kDirTZ = 64, kDirXC = 32;

template <class T>
__global__ void __launch_bounds__(kBlock)
k_pcg_dir_march(StepK k, const double* __restrict__ diag, const double* __restrict__ cfx,
                const double* __restrict__ cfy, const double* __restrict__ cfz,
                const T* __restrict__ zT, double sigma, const double* __restrict__ p_in,
                double* __restrict__ p_out, double* __restrict__ q, double beta, int first, int xc,
                double* __restrict__ xv, double alpha_prev, int xmode,
                double* __restrict__ part) {
  constexpr int TY = kDirTY, TZ = kDirTZ, HZ = TZ + 2, PL = (TY + 2) * HZ;
  constexpr int NR = TY / (kBlock / 64);  // own rows per thread
  constexpr int NRING = 2 * TZ + 2 * TY;  // ring cells of a plane (no corners)
  static_assert(TZ == 64 && NRING <= kBlock, "one wave per row, one ring cell per thread");
  __shared__ double pl[2][PL];
  const int per[3] = {k.bc[0] == RH_BC_PERIODIC, k.bc[2] == RH_BC_PERIODIC,
                      k.bc[4] == RH_BC_PERIODIC};
  const int ntz = (k.nz + TZ - 1) / TZ, nty = (k.ny + TY - 1) / TY;
  int bid = xcd_tile(blockIdx.x, gridDim.x);
  const int tz = bid % ntz;
  bid /= ntz;
  const int ty = bid % nty;
  const int cx = bid / nty;
  const int ya = ty * TY, za = tz * TZ;  // tile cell (0, 0) = LDS (1, 1)
  const int xa = cx * xc, xb = min(xa + xc, k.nx);
  const int plane = k.ny * k.nz;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  auto wrap = [&](int g, int n, int pr) -> int {
    if (g >= 0 && g < n) return g;
    if (!pr) return -1;
    return g < 0 ? g + n : g - n;
  };
  auto off2 = [&](int gy, int gz) -> int {
    const int wy = wrap(gy, k.ny, per[1]), wz = wrap(gz, k.nz, per[2]);
    return (wy >= 0 && wz >= 0) ? wy * k.nz + wz : -1;
  };
  // own cells (rows wid + 4m, column lane); overhang cells of a ragged tile
  // stand for their wrapped cell (or outside) and are not written
  int own[NR], omy[NR], omz[NR], li[NR];
  bool real[NR];
#pragma unroll
  for (int m = 0; m < NR; ++m) {
    const int ly = wid + (kBlock / 64) * m, gy = ya + ly, gz = za + lane;
    real[m] = gy < k.ny && gz < k.nz;
    own[m] = off2(gy, gz);
    omy[m] = off2(gy - 1, gz);
    omz[m] = off2(gy, gz - 1);
    li[m] = (ly + 1) * HZ + lane + 1;
  }
  // this thread's ring cell
  int r_off = -1, r_li = -1;
  if (threadIdx.x < NRING) {
    const int e = threadIdx.x;
    int ly, lz;
    if (e < 2 * TZ) {
      ly = e < TZ ? 0 : TY + 1;
      lz = e % TZ + 1;
    } else {
      const int f = e - 2 * TZ;
      ly = f % TY + 1;
      lz = f < TY ? 0 : TZ + 1;
    }
    r_li = ly * HZ + lz;
    r_off = off2(ya + ly - 1, za + lz - 1);
  }
  auto raw = [&](int p, int off, double& zv, double& pv) {
    const int gx = wrap(p, k.nx, per[0]);
    zv = 0.0;
    pv = 0.0;
    if (gx < 0 || off < 0) return;
    const int P = gx * plane + off;
    zv = sigma * (double)zT[P];
    if (!first) pv = p_in[P];
  };
  auto form = [&](double zv, double pv) { return first ? zv : zv + beta * pv; };
  struct Coef {
    double d[NR], c0[NR], c1[NR], c2[NR], c1m[NR], c2m[NR];
  };
  auto load_coef = [&](int p, Coef& C) {
    const int gx = wrap(p, k.nx, per[0]);
#pragma unroll
    for (int m = 0; m < NR; ++m) {
      const bool ok = gx >= 0 && own[m] >= 0;
      const int P = ok ? gx * plane + own[m] : 0;
      C.d[m] = ok ? diag[P] : 0.0;
      C.c0[m] = ok ? cfx[P] : 0.0;
      C.c1[m] = ok ? cfy[P] : 0.0;
      C.c2[m] = ok ? cfz[P] : 0.0;
      C.c1m[m] = (gx >= 0 && omy[m] >= 0) ? cfy[gx * plane + omy[m]] : 0.0;
      C.c2m[m] = (gx >= 0 && omz[m] >= 0) ? cfz[gx * plane + omz[m]] : 0.0;
    }
  };
  double pm[NR], pc[NR], pn[NR], c0m[NR];
  double zo[NR], po[NR];  // own raw at x+2 (in flight)
  double pin_c[NR], pin_n[NR], xcur[NR], xnext[NR];  // p_in at x, x+1; x at x, x+1
  double rz1, rp1, rz2, rp2;  // ring raw at x+1 (ready) and x+2 (in flight)
  Coef C, Cn;
  // prologue: planes xa-1, xa, xa+1 of p; plane xa in LDS; coefficients of xa
  {
    const int gxm = wrap(xa - 1, k.nx, per[0]);
#pragma unroll
    for (int m = 0; m < NR; ++m) {
      double a, b;
      raw(xa - 1, own[m], a, b);
      pm[m] = form(a, b);
      raw(xa, own[m], a, b);
      pc[m] = form(a, b);
      pin_c[m] = b;
      raw(xa + 1, own[m], a, b);
      pn[m] = form(a, b);
      pin_n[m] = b;
      xcur[m] = (xmode == 2 && real[m]) ? xv[xa * plane + own[m]] : 0.0;
      xnext[m] = 0.0;
      pl[xa & 1][li[m]] = pc[m];
      c0m[m] = (gxm >= 0 && own[m] >= 0) ? cfx[gxm * plane + own[m]] : 0.0;
    }
    if (r_li >= 0) {
      double a, b;
      raw(xa, r_off, a, b);
      pl[xa & 1][r_li] = form(a, b);
      raw(xa + 1, r_off, rz1, rp1);
    }
    load_coef(xa, C);
  }
  __syncthreads();
  double acc = 0.0;
  for (int x = xa; x < xb; ++x) {
    // in flight for the next iteration
    if (x + 1 < xb) load_coef(x + 1, Cn);
#pragma unroll
    for (int m = 0; m < NR; ++m) {
      zo[m] = 0.0;
      po[m] = 0.0;
      if (x + 2 <= xb) raw(x + 2, own[m], zo[m], po[m]);
      if (xmode == 2 && real[m] && x + 1 < xb) xnext[m] = xv[(x + 1) * plane + own[m]];
    }
    rz2 = rp2 = 0.0;
    if (r_li >= 0 && x + 2 < xb) raw(x + 2, r_off, rz2, rp2);
    // q on plane x
    const double* L = pl[x & 1];
    const int gx = x;
#pragma unroll
    for (int m = 0; m < NR; ++m) {
      if (!real[m]) continue;
      const int t = li[m];
      double off = C.c0[m] * pn[m];
      off += c0m[m] * pm[m];
      off += C.c1[m] * L[t + HZ];
      off += C.c1m[m] * L[t - HZ];
      off += C.c2[m] * L[t + 1];
      off += C.c2m[m] * L[t - 1];
      const double qv = C.d[m] * pc[m] - off;
      const int P = gx * plane + own[m];
      p_out[P] = pc[m];
      q[P] = qv;
      acc += pc[m] * qv;
      // the previous iteration's x += alpha p (p_in is that p)
      if (xmode) xv[P] = (xmode == 2 ? xcur[m] : 0.0) + alpha_prev * pin_c[m];
    }
    // plane x+1 into the other LDS buffer (its readers finished before the
    // last barrier)
    if (x + 1 < xb) {
      double* Ln = pl[(x + 1) & 1];
#pragma unroll
      for (int m = 0; m < NR; ++m) Ln[li[m]] = pn[m];
      if (r_li >= 0) Ln[r_li] = form(rz1, rp1);
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NR; ++m) {
      c0m[m] = C.c0[m];
      pm[m] = pc[m];
      pc[m] = pn[m];
      pn[m] = form(zo[m], po[m]);
      pin_c[m] = pin_n[m];
      pin_n[m] = po[m];
      xcur[m] = xnext[m];
    }
    rz1 = rz2;
    rp1 = rp2;
    C = Cn;
  }
  double v[1] = {acc};
  const int im[1] = {0};
  const int sl[1] = {RS_PQ};
  block_reduce_store<1>(v, im, sl, part);
}

template <class T>
void launch_pcg_dir(hipStream_t s, const StepK& k, const double* diag, const double* const cf[3],
                    const T* zT, double sigma, const double* p_in, double* p_out, double* q,
                    double beta, int first, const XFold& xf, double* part) {
  const int nty = (k.ny + kDirTY - 1) / kDirTY, ntz = (k.nz + kDirTZ - 1) / kDirTZ;
  const long long tiles = (long long)nty * ntz;
  if (k.nz >= kDirTZ && k.ny >= kDirTY && k.nx >= 2 && k.N < (1LL << 31) && tiles <= kPartCap) {
    int ncx = (k.nx + kDirXC - 1) / kDirXC;
    if (tiles * ncx > kPartCap) ncx = (int)(kPartCap / tiles);
    const int xc = (k.nx + ncx - 1) / ncx;
    ncx = (k.nx + xc - 1) / xc;
    hipLaunchKernelGGL((k_pcg_dir_march<T>), dim3((unsigned)(tiles * ncx)), dim3(kBlock), 0, s, k,
                       diag, cf[0], cf[1], cf[2], zT, sigma, p_in, p_out, q, beta, first, xc,
                       xf.x, xf.alpha, xf.mode, part);
    return;
  }
  hipLaunchKernelGGL((k_pcg_dir<T>), dim3(red_grid(k.N)), dim3(kBlock), 0, s, k, diag, cf[0],
                     cf[1], cf[2], zT, sigma, p_in, p_out, q, beta, first, xf.x, xf.alpha,
                     xf.mode, part);
}

// B: x += alpha p;  r -= alpha q;  norms of r;  b = r * inv_sigma (preconditioner input)
template <class T>
__global__ void __launch_bounds__(kBlock)
k_pcg_update(StepK k, double alpha, const double* __restrict__ p, const double* __restrict__ q,
             double* __restrict__ x, double* __restrict__ r, double inv_sigma, T* __restrict__ b,
             int first, double* __restrict__ part) {
  double s2w = 0.0, s2 = 0.0, rmax = 0.0;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < k.N;
       idx += (long long)blockDim.x * gridDim.x) {
    // x == NULL: x += alpha p is left to the next direction kernel
    if (x) x[idx] = (first ? 0.0 : x[idx]) + alpha * p[idx];
    const double rv = r[idx] - alpha * q[idx];
    r[idx] = rv;
    b[idx] = (T)(rv * inv_sigma);
    s2w += (rv / k.E_s) * (rv / k.E_s);
    s2 += rv * rv;
    rmax = fmax(rmax, fabs(rv));
  }
  double v[3] = {s2w, rmax, s2};
  const int im[3] = {0, 1, 0};
  const int sl[3] = {RS_FE2, RS_RMAX, RS_R2};
  block_reduce_store<3>(v, im, sl, part);
}

__global__ void __launch_bounds__(kBlock)
k_xaxpy(long long N, double alpha, const double* __restrict__ p, double* __restrict__ x,
        int first) {
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < N;
       idx += (long long)blockDim.x * gridDim.x)
    x[idx] = (first ? 0.0 : x[idx]) + alpha * p[idx];
}

void launch_xaxpy(hipStream_t s, long long N, double alpha, const double* p, double* x,
                  int first) {
  hipLaunchKernelGGL(k_xaxpy, dim3(red_grid(N)), dim3(kBlock), 0, s, N, alpha, p, x, first);
}

template <class T>
void launch_pcg_update(hipStream_t s, const StepK& k, double alpha, const double* p,
                       const double* q, double* x, double* r, double inv_sigma, T* b, int first,
                       double* part) {
  hipLaunchKernelGGL((k_pcg_update<T>), dim3(red_grid(k.N)), dim3(kBlock), 0, s, k, alpha, p, q,
                     x, r, inv_sigma, b, first, part);
}

// C: partial z.r and z.q for z = sigma * zT (q may be null on the first pass);
// z itself is formed again where it is used (the direction kernel)
template <class T>
__global__ void __launch_bounds__(kBlock)
k_pcg_precond(StepK k, double sigma, const T* __restrict__ zT, const double* __restrict__ r,
              const double* __restrict__ q, double* __restrict__ part) {
  double zr = 0.0, zq = 0.0;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < k.N;
       idx += (long long)blockDim.x * gridDim.x) {
    const double zv = sigma * (double)zT[idx];
    zr += zv * r[idx];
    if (q) zq += zv * q[idx];
  }
  double v[2] = {zr, zq};
  const int im[2] = {0, 0};
  const int sl[2] = {RS_ZR, RS_ZQ};
  block_reduce_store<2>(v, im, sl, part);
}

template <class T>
void launch_pcg_precond(hipStream_t s, const StepK& k, double sigma, const T* zT, const double* r,
                        const double* q, double* part) {
  hipLaunchKernelGGL((k_pcg_precond<T>), dim3(red_grid(k.N)), dim3(kBlock), 0, s, k, sigma, zT, r,
                     q, part);
}

// ---------------------------------------------------------------------------
// adjoint of the step (implicit-function theorem at the converged U^{n+1})
// ---------------------------------------------------------------------------
// Local rates with the hydrogen density as an independent variable.
template <class S>
__device__ inline void local_rates_nh(const StepK& k, S E, S e, S n, S nH, double a, S& A, S& B,
                                      S& q) {
  const double a3 = a * a * a;
  S Epos = dmax0(E);
  S T;
  if (k.iso) {
    T = lift<S>(k.T_iso);
  } else {
    S mu = 1.0 / (2.0 - n / nH);
    T = ((k.gamma - 1.0) * kMH / kKB) * mu * e;
  }
  S ne = (nH - n) / a3;
  const bool fit_recB = !k.iso && (k.cooling & RH_COOL_RECB);
  const bool fit_ce = !k.iso && (k.cooling & RH_COOL_COLLEXC);
  const TFits tf = t_fits(dval(T), k.rates, fit_recB, fit_ce);
  S alpha = k.rates ? dchain(T, tf.alpha, tf.dalpha) : lift<S>(k.alphaB);
  A = alpha * ne * nH;
  B = alpha * ne + (kC * k.K_Gamma / a3) * Epos;
  if (k.iso) {
    q = lift<S>(0.0);
    return;
  }
  S nHI = n / a3;
  S G = (kC * k.K_G / a3) * nHI * Epos;
  S Lam = lift<S>(0.0);
  if (fit_recB) Lam = Lam + dchain(T, tf.recB, tf.drecB) * ne * ne;
  if (fit_ce) Lam = Lam + dchain(T, tf.ce, tf.dce) * ne * nHI;
  if (k.cooling & RH_COOL_COMPTON) {
    const double zp1 = 1.0 / a;
    Lam = Lam + (k.compton * zp1 * zp1 * zp1 * zp1) * (T - kTcmb0 * zp1) * ne;
  }
  q = (G - Lam) * (a3 / kMH) / nH;
}

// right-hand side of the adjoint Schur system: r = lE - (B^-1 C)^T lambda_loc
__global__ void __launch_bounds__(kBlock)
k_adj_rhs(StepK k, const double* __restrict__ lE, const double* __restrict__ le,
          const double* __restrict__ ln, const double* __restrict__ BCn,
          const double* __restrict__ BCe, double* __restrict__ r, double* __restrict__ part) {
  double rmax = 0.0, r2 = 0.0;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < k.N;
       idx += (long long)blockDim.x * gridDim.x) {
    double v = lE[idx] - BCn[idx] * ln[idx];
    if (!k.iso) v -= BCe[idx] * le[idx];
    r[idx] = v;
    rmax = fmax(rmax, fabs(v));
    r2 += v * v;
  }
  double vv[2] = {rmax, r2};
  const int im[2] = {1, 0};
  const int sl[2] = {RS_RMAX, RS_R2};
  block_reduce_store<2>(vv, im, sl, part);
}

// Transposed local elimination and the local parts of (df/dU^n)^T mu,
// (df/dn_H)^T mu and (df/dsrc)^T mu.  Slots: n, e, E, n_H, n^n, e^n, E^n.
__global__ void __launch_bounds__(kBlock)
k_adj_local(StepK k, AdjArgs a) {
  const double a13 = k.a_1 * k.a_1 * k.a_1;
  const double an3 = k.a_n * k.a_n * k.a_n;
  const double th = k.theta, dt = k.dt;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < k.N;
       idx += (long long)blockDim.x * gridDim.x) {
    typedef DN<7> S;
    const double nH = a.nH[idx];
    S n = dn_var<7>(a.n1[idx], 0);
    S e = dn_var<7>(k.iso ? 0.0 : a.e1[idx], 1);
    S E = dn_var<7>(a.E1[idx], 2);
    S H = dn_var<7>(nH, 3);
    S nn = dn_var<7>(a.nn[idx], 4);
    S en = dn_var<7>(k.iso ? 0.0 : a.en[idx], 5);
    S En = dn_var<7>(a.En[idx], 6);
    S A, B, q;
    local_rates_nh<S>(k, E, e, n, H, k.a_1, A, B, q);
    S numn = nn + (dt * th) * A;
    S nume = en + (dt * th) * q;
    if (k.theta_lt1) {
      S An, Bn, qn;
      local_rates_nh<S>(k, En, en, nn, H, k.a_n, An, Bn, qn);
      numn = numn + (dt * (1.0 - th)) * (An - Bn * nn);
      nume = nume + (dt * (1.0 - th)) * (qn - (2.0 * k.H_n) * en);
    }
    S fn = n - numn / (1.0 + (th * dt) * B);
    const double muE = a.muE[idx];
    const double JEn = dt * th * kC * k.sigma_E * a.E1[idx] / a13;
    double mun, mue = 0.0;
    S fe = dn_const<7>(0.0);
    if (k.iso) {
      mun = (a.ln[idx] - JEn * muE) / fn.g[0];
    } else {
      fe = e - nume / (1.0 + 2.0 * th * dt * k.H_1);
      // B^T mu_loc = (ln - J_En mu_E, le),  B = [[fn_n, fn_e], [fe_n, fe_e]]
      const double b11 = fn.g[0], b12 = fn.g[1], b21 = fe.g[0], b22 = fe.g[1];
      const double r1 = a.ln[idx] - JEn * muE, r2 = a.le[idx];
      const double idet = 1.0 / (b11 * b22 - b12 * b21);
      mun = (b22 * r1 - b21 * r2) * idet;
      mue = (-b12 * r1 + b11 * r2) * idet;
    }
    // local explicit parts of f_E (theta < 1)
    double dfE_dEn = -1.0, dfE_dnn = 0.0;
    if (k.theta_lt1) {
      dfE_dEn += dt * (1.0 - th) * (k.H_n + kC * k.sigma_E * a.nn[idx] / an3);
      dfE_dnn += dt * (1.0 - th) * kC * k.sigma_E * a.En[idx] / an3;
    }
    const double lnn = -(fn.g[4] * mun + fe.g[4] * mue) - dfE_dnn * muE;
    const double lEn = -(fn.g[6] * mun + fe.g[6] * mue) - dfE_dEn * muE;
    a.ln[idx] = lnn;
    a.lE[idx] = lEn;
    if (!k.iso) a.le[idx] = -(fn.g[5] * mun + fe.g[5] * mue);
    a.g_nH[idx] += -(fn.g[3] * mun + fe.g[3] * mue);
    a.g_src[idx] += dt * muE;
  }
}

// Dependence of f_E on (E^n, n^n) through the lagged face limiter and the
// explicit part: for every face f = (R, Q) of cell R,
//   G_f = (mu_R - mu_Q) [ -c_f (E_Q - E_R) - c_f r_e (E^n_Q - E^n_R) ],
// c_f = cf_scale D_f(E^n, kappa^n), r_e = (1-theta)/theta (a_1/a_n)^2;
// lambda^n_R -= dG_f / d(E^n_R, n^n_R).  Outflow faces use the ghost
// (E = E^n = E_floor, mu = 0, kappa = kappa_R).
__global__ void __launch_bounds__(kBlock)
k_adj_limiter(StepK k, AdjArgs a) {
  const int per[3] = {k.bc[0] == RH_BC_PERIODIC, k.bc[2] == RH_BC_PERIODIC,
                      k.bc[4] == RH_BC_PERIODIC};
  const int nd[3] = {k.nx, k.ny, k.nz};
  const double kfac = k.sigma_E / (k.a_n * k.a_n * k.a_n);
  const double re = k.theta_lt1 ? k.expl_ratio : 0.0;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < k.N;
       idx += (long long)blockDim.x * gridDim.x) {
    int c[3];
    cell_ijk(idx, k.ny, k.nz, c[0], c[1], c[2]);
    typedef DN<2> S2;  // slots: E^n_R, kappa^n_R
    const double EnR = a.En[idx], E1R = a.E1[idx], muR = a.muE[idx];
    const S2 EnRd = dn_var<2>(EnR, 0);
    const S2 kRd = dn_var<2>(kfac * a.nn[idx], 1);
    double dE = 0.0, dk = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
#pragma unroll
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        int q[3];
        double EnQ, E1Q, muQ;
        S2 kQd;
        if (neighbour(c, nd, per, d, sgn, q)) {
          const long long Q = cell_index(q[0], q[1], q[2], k.ny, k.nz);
          EnQ = a.En[Q];
          E1Q = a.E1[Q];
          muQ = a.muE[Q];
          kQd = dn_const<2>(kfac * a.nn[Q]);
        } else if (k.bc[2 * d + (sgn > 0 ? 1 : 0)] == RH_BC_OUTFLOW) {
          EnQ = k.E_floor;
          E1Q = k.E_floor;
          muQ = 0.0;
          kQd = kRd;
        } else {
          continue;  // zero-flux wall: no face term
        }
        // D on the face, differentiated w.r.t. this cell's E^n and kappa^n
        const S2 Ebar = dfmax(0.5 * (EnRd + EnQ), k.E_floor);
        const S2 R = dfmax(dfabs(EnQ - EnRd) / (Ebar * (k.a_n * k.h)), k.R_min);
        const S2 kap = 0.5 * (kRd + kQd);
        const S2 D = kC * (2.0 * kap + R) / (6.0 * kap * kap + 3.0 * kap * R + R * R);
        const double cfv = k.cf_scale * D.v;
        const double w = muR - muQ;
        const double bracket = (E1Q - E1R) + re * (EnQ - EnR);
        // G = -w c (bracket);  dG/dE^n_R = -w (dc/dE^n_R bracket - c re)
        dE += w * (k.cf_scale * D.g[0] * bracket - cfv * re);
        dk += w * (k.cf_scale * D.g[1] * bracket);
      }
    }
    a.lE[idx] += dE;
    a.ln[idx] += dk * kfac;
  }
}

void launch_adj_rhs(hipStream_t s, const StepK& k, const double* lE, const double* le,
                    const double* ln, const double* BCn, const double* BCe, double* r,
                    double* part) {
  hipLaunchKernelGGL(k_adj_rhs, dim3(red_grid(k.N)), dim3(kBlock), 0, s, k, lE, le, ln, BCn, BCe,
                     r, part);
}

void launch_adj_local(hipStream_t s, const StepK& k, const AdjArgs& a) {
  hipLaunchKernelGGL(k_adj_local, dim3(red_grid(k.N)), dim3(kBlock), 0, s, k, a);
}

void launch_adj_limiter(hipStream_t s, const StepK& k, const AdjArgs& a) {
  hipLaunchKernelGGL(k_adj_limiter, dim3(red_grid(k.N)), dim3(kBlock), 0, s, k, a);
}

// ---------------------------------------------------------------------------
// explicit instantiations
// ---------------------------------------------------------------------------
#define RH_INST(T)                                                                            \
  template void launch_coarse_diag<T>(hipStream_t, const LevelK<T>&, const LevelK<T>&);       \
  template void launch_coarsest_inverse<T>(hipStream_t, const LevelK<T>&, double*, double*,   \
                                           T*);                                               \
  template void launch_coarsest_solve<T>(hipStream_t, const LevelK<T>&, const T*);            \
  template void launch_rbgs<T>(hipStream_t, const LevelK<T>&, int, int, int);                 \
  template bool launch_rbgs_march<T>(hipStream_t, const LevelK<T>&, int, int, int, long long,   \
                                     const SweepDots*);                                       \
  template bool rbgs_march_fits<T>(const LevelK<T>&, long long);                             \
  template bool launch_resid_restrict_march<T>(hipStream_t, const LevelK<T>&, const LevelK<T>&, \
                                               long long);                                    \
  template bool resid_restrict_fits<T>(const LevelK<T>&, long long);                         \
  template void launch_mg_residual<T>(hipStream_t, const LevelK<T>&);                         \
  template void launch_restrict<T>(hipStream_t, const LevelK<T>&, const LevelK<T>&);          \
  template void launch_prolong<T>(hipStream_t, const LevelK<T>&, const LevelK<T>&);           \
  template void launch_cast_scale<T>(hipStream_t, long long, const double*, double, T*);      \
  template void launch_accum_defect<T>(hipStream_t, const StepK&, const DefectArgs&, const T*, \
                                       T*, double*);                                          \
  template void launch_pcg_update<T>(hipStream_t, const StepK&, double, const double*,        \
                                     const double*, double*, double*, double, T*, int,        \
                                     double*);                                                \
  template void launch_pcg_precond<T>(hipStream_t, const StepK&, double, const T*,            \
                                      const double*, const double*, double*);                 \
  template void launch_pcg_dir<T>(hipStream_t, const StepK&, const double*,                   \
                                  const double* const[3], const T*, double, const double*,    \
                                  double*, double*, double, int, const XFold&, double*);
RH_INST(float)
RH_INST(double)
template void launch_coarsen_faces<double>(hipStream_t, const LevelK<double>&,
                                           const LevelK<double>&);
template void launch_coarsen_faces<float>(hipStream_t, const LevelK<float>&, const LevelK<float>&);

}  // namespace rh

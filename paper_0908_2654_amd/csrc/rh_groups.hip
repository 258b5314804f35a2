// Hydrogen + helium chemistry coupled to G radiation groups (gfx950): the
// extension the Conclusions and outlook section names first (multigroup
// flux-limited diffusion, helium ionisation).  The radiation residual and
// face limiter of each group are the grey kernels' (rh_kernels.hip) with the
// group's opacity and source; this file holds what is new: the per-cell
// local solve over (e, n_HI, n_HeI, n_HeII) with the elimination data of
// the Schur complement, the coupled Schur residual of one group, and the
// initial fields.
//
// Equations (per cell; comoving densities, proper ones in the rates):
//   n_HII = n_H - n_HI, n_HeIII = n_He - n_HeI - n_HeII,
//   n_e = n_HII + n_HeII + 2 n_HeIII (equation electron_density, helium
//   branch), mu = (n_H + 4 n_He) / (n_H + n_He + n_e),
//   dy/dt = a - M y for y = (n_HI, n_HeI, n_HeII) with
//     a = (alpha_H n_e n_H, 0, alpha_HeIII n_e n_He),
//     M = [[alpha_H n_e + Gamma_HI, 0, 0],
//          [0, Gamma_HeI, -alpha_HeII n_e],
//          [0, alpha_HeIII n_e - Gamma_HeI, Gamma_HeII + (alpha_HeII + alpha_HeIII) n_e]]
//   (equation chemical_ionization for each species), Gamma_s = c sum_g
//   K_Gamma[s][g] E_g; the theta method with M and a frozen at the implicit
//   level: (I + theta dt M(U)) S = y^n + dt [theta a(U) + (1 - theta)(a^n - M^n y^n)],
//   and the gas energy as in the hydrogen-only step with the multigroup
//   heating and the helium recombination cooling.
#include <hip/hip_runtime.h>

#include <cmath>

#include "rh_device.h"
#include "rh_dual.h"
#include "rh_internal.h"

namespace rh {

namespace {

constexpr double kLn570670 = 13.254566388120152;  // ln(2 x 285335 K), HeII case-B fit
constexpr double kLn4 = 1.3862943611198906;       // alpha_HeIII(T) = 2 alpha_H(T / 4)

// Rates of the local ODEs at a state: the nonzero entries of a and M, and
// the gas heating rate q (de/dt = q - 2 H e).
template <class S>
struct GroupRates {
  S A0, A2, M00, M11, M12, M21, M22, q;
};

template <class S>
__device__ inline GroupRates<S> group_rates(const StepK& k, const GroupK& m, const S (&E)[kMaxGroups],
                                            S e, S y0, S y1, S y2, double nH, double nHe,
                                            double a) {
  const double a3 = a * a * a;
  GroupRates<S> r;
  const S nHII = nH - y0;
  const S nHeIII = nHe - y1 - y2;
  const S ne_c = nHII + y2 + 2.0 * nHeIII;
  const S ne = ne_c / a3;
  S T;
  if (k.iso)
    T = lift<S>(k.T_iso);
  else
    T = ((k.gamma - 1.0) * kMH / kKB) * ((nH + 4.0 * nHe) / (nH + nHe + ne_c)) * e;
  const bool recB = !k.iso && (k.cooling & RH_COOL_RECB);
  S L = lift<S>(0.0);  // ln(315614 K / T) of the case-B fits
  if (k.rates || recB) L = hg_ln_lambda(T);
  const S aH = k.rates ? alpha_B_of_L(L) : lift<S>(k.alphaB);
  S aHeII = lift<S>(0.0), aHeIII = lift<S>(0.0);
  if (m.he) {
    aHeII = 1.26e-14 * dexp(0.75 * (kLn570670 - dlog(T)));
    aHeIII = k.rates ? 2.0 * alpha_B_of_L(L + kLn4) : lift<S>(2.0 * k.alphaB);
  }
  S Gam[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    Gam[s] = lift<S>(0.0);
#pragma unroll
    for (int g = 0; g < kMaxGroups; ++g)
      if (m.KGam[s][g] != 0.0) Gam[s] = Gam[s] + (kC * m.KGam[s][g] / a3) * dmax0(E[g]);
  }
  r.A0 = aH * ne * nH;
  r.A2 = aHeIII * ne * nHe;
  r.M00 = aH * ne + Gam[0];
  r.M11 = Gam[1];
  r.M12 = 0.0 - aHeII * ne;
  r.M21 = aHeIII * ne - Gam[1];
  r.M22 = Gam[2] + (aHeII + aHeIII) * ne;
  if (k.iso) {
    r.q = lift<S>(0.0);
    return r;
  }
  // heating: c sum_s n_s sum_g K_G[s][g] E_g (proper)
  const S ys[3] = {y0, y1, y2};
  S heat = lift<S>(0.0);
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    S hs = lift<S>(0.0);
#pragma unroll
    for (int g = 0; g < kMaxGroups; ++g)
      if (m.KG[s][g] != 0.0) hs = hs + (kC * m.KG[s][g] / a3) * dmax0(E[g]);
    heat = heat + (ys[s] / a3) * hs;
  }
  S Lam = lift<S>(0.0);
  if (recB) {
    Lam = Lam + cool_recB_of_L(T, L) * ne * (nHII / a3);
    if (m.he)
      Lam = Lam + (kKB * T) * aHeII * ne * (y2 / a3) +
            8.0 * cool_recB_of_L(0.25 * T, L + kLn4) * ne * (nHeIII / a3);
  }
  if (k.cooling & RH_COOL_COLLEXC) Lam = Lam + cool_collexc(T) * ne * (y0 / a3);
  if (k.cooling & RH_COOL_COMPTON) {
    const double zp1 = 1.0 / a;
    Lam = Lam + (k.compton * zp1 * zp1 * zp1 * zp1) * (T - kTcmb0 * zp1) * ne;
  }
  r.q = (heat - Lam) * (a3 / (kMH * (nH + 4.0 * nHe)));
  return r;
}

// Explicit (level n) parts of the theta method: R = a^n - M^n y^n and
// qn = q^n - 2 H_n e^n.
struct Explicit {
  double R[3], qn;
};

// theta-method local solutions S_y (3) and S_e at a state.  Without helium
// S_HeI = S_HeII = 0; isothermal runs keep S_e = 0.
template <class S>
__device__ inline void group_local_S(const StepK& k, const GroupK& m, const S (&E)[kMaxGroups], S e,
                                     S y0, S y1, S y2, double nH, double nHe,
                                     const double (&yn)[3], double en, const Explicit& x,
                                     S (&Sy)[3], S& Se) {
  const GroupRates<S> r = group_rates(k, m, E, e, y0, y1, y2, nH, nHe, k.a_1);
  const double th = k.theta, dt = k.dt, c = th * dt, ex = dt * (1.0 - th);
  Sy[0] = (yn[0] + ex * x.R[0] + (dt * th) * r.A0) / (1.0 + c * r.M00);
  if (m.he) {
    const S rhs1 = lift<S>(yn[1] + ex * x.R[1]);
    const S rhs2 = (yn[2] + ex * x.R[2]) + (dt * th) * r.A2;
    const S a11 = 1.0 + c * r.M11, a12 = c * r.M12;
    const S a21 = c * r.M21, a22 = 1.0 + c * r.M22;
    const S det = a11 * a22 - a12 * a21;
    Sy[1] = (a22 * rhs1 - a12 * rhs2) / det;
    Sy[2] = (a11 * rhs2 - a21 * rhs1) / det;
  } else {
    Sy[1] = lift<S>(0.0);
    Sy[2] = lift<S>(0.0);
  }
  if (k.iso)
    Se = lift<S>(0.0);
  else
    Se = (en + ex * x.qn + (dt * th) * r.q) / (1.0 + 2.0 * th * dt * k.H_1);
}

// Solve A X = R (A 4 x 4, R 4 x nc) by Gaussian elimination with partial
// pivoting; R is overwritten with X.
template <int NC>
__device__ inline void solve4(double (&A)[kLoc][kLoc], double (&R)[kLoc][NC]) {
#pragma unroll
  for (int c = 0; c < kLoc; ++c) {
    int p = c;
    double best = fabs(A[c][c]);
#pragma unroll
    for (int i = c + 1; i < kLoc; ++i)
      if (fabs(A[i][c]) > best) {
        best = fabs(A[i][c]);
        p = i;
      }
    // row swap with compile-time indices only (the arrays stay in registers)
#pragma unroll
    for (int i = c + 1; i < kLoc; ++i) {
      if (i != p) continue;
#pragma unroll
      for (int j = 0; j < kLoc; ++j) {
        const double t = A[c][j];
        A[c][j] = A[i][j];
        A[i][j] = t;
      }
#pragma unroll
      for (int j = 0; j < NC; ++j) {
        const double t = R[c][j];
        R[c][j] = R[i][j];
        R[i][j] = t;
      }
    }
    const double inv = 1.0 / A[c][c];
#pragma unroll
    for (int i = c + 1; i < kLoc; ++i) {
      const double f = A[i][c] * inv;
#pragma unroll
      for (int j = c; j < kLoc; ++j) A[i][j] -= f * A[c][j];
#pragma unroll
      for (int j = 0; j < NC; ++j) R[i][j] -= f * R[c][j];
    }
  }
#pragma unroll
  for (int c = kLoc - 1; c >= 0; --c) {
    const double inv = 1.0 / A[c][c];
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      double v = R[c][j];
#pragma unroll
      for (int i = c + 1; i < kLoc; ++i) v -= A[c][i] * R[i][j];
      R[c][j] = v * inv;
    }
  }
}

// shorten lam so that v + lam d stays above lo (0.9 of the way), as the
// caps of the local Newton iteration do
__device__ inline double cap_lo(double lam, double v, double d, double lo) {
  return v + d < lo ? fmin(lam, 0.9 * (v - lo) / (-d)) : lam;
}
__device__ inline double cap_hi(double lam, double v, double d, double hi) {
  return v + d > hi ? fmin(lam, 0.9 * (hi - v) / d) : lam;
}

constexpr int kJ = kLoc + kMaxGroups;  // derivative slots of the Jacobian pass

// Local solve (mode 0) or evaluation (mode 1) with the elimination data.
__global__ void __launch_bounds__(kBlock)
k_local_groups(StepK k, GroupK m, GroupLocalArgs a, double* __restrict__ part) {
  const long long N = k.N;
  const int G = m.G;
  double sfy = 0.0, sfe = 0.0, fail = 0.0, itmax = 0.0, bad = 0.0;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < N;
       idx += (long long)blockDim.x * gridDim.x) {
    const double nH = a.nH[idx];
    const double nHe = m.y_he * nH;
    double E[kMaxGroups], dEv[kMaxGroups];
#pragma unroll
    for (int g = 0; g < kMaxGroups; ++g) {
      E[g] = 0.0;
      dEv[g] = 0.0;
      if (g < G) {
        E[g] = a.Ek[g * N + idx];
        if (a.dE) {
          dEv[g] = a.dE[g * N + idx];
          E[g] += a.lam * dEv[g];
        }
      }
    }
    const double yn[3] = {a.yn[idx], m.he ? a.yn[N + idx] : 0.0, m.he ? a.yn[2 * N + idx] : 0.0};
    const double en = k.iso ? 0.0 : a.en[idx];
    // local unknowns z = (e, n_HI, n_HeI, n_HeII)
    double z[kLoc] = {k.iso ? 0.0 : a.ek[idx], a.yk[idx], m.he ? a.yk[N + idx] : 0.0,
                      m.he ? a.yk[2 * N + idx] : 0.0};
    Explicit xp{{0.0, 0.0, 0.0}, 0.0};
    if (k.theta_lt1) {
      double Enl[kMaxGroups];
#pragma unroll
      for (int g = 0; g < kMaxGroups; ++g) Enl[g] = g < G ? a.En[g * N + idx] : 0.0;
      const GroupRates<double> r =
          group_rates<double>(k, m, Enl, en, yn[0], yn[1], yn[2], nH, nHe, k.a_n);
      xp.R[0] = r.A0 - r.M00 * yn[0];
      xp.R[1] = -(r.M11 * yn[1] + r.M12 * yn[2]);
      xp.R[2] = r.A2 - (r.M21 * yn[1] + r.M22 * yn[2]);
      xp.qn = k.iso ? 0.0 : r.q - 2.0 * k.H_n * en;
    }
    int its = 0;
    if (a.mode == 0) {
      // predictor from the linearisation at U_k
      if (a.pBf && a.dE) {
#pragma unroll
        for (int s = 0; s < kLoc; ++s) {
          double v = a.pBf[s * N + idx];
#pragma unroll
          for (int h = 0; h < kMaxGroups; ++h)
            if (h < G) v += a.pBC[(s * G + h) * N + idx] * (a.lam * dEv[h]);
          z[s] -= v;
        }
      }
      if (k.iso) z[0] = 0.0; else z[0] = fmax(z[0], 1e-300);
      z[1] = fmin(fmax(z[1], 0.0), nH);
      if (m.he) {
        z[2] = fmin(fmax(z[2], 0.0), nHe);
        z[3] = fmin(fmax(z[3], 0.0), nHe - z[2]);
      } else {
        z[2] = z[3] = 0.0;
      }
      DN<kLoc> Ed[kMaxGroups];
#pragma unroll
      for (int g = 0; g < kMaxGroups; ++g) Ed[g] = dn_const<kLoc>(E[g]);
      bool conv = false;
      for (its = 1; its <= 100; ++its) {
        const DN<kLoc> ze = k.iso ? dn_const<kLoc>(0.0) : dn_var<kLoc>(z[0], 0);
        const DN<kLoc> z1 = dn_var<kLoc>(z[1], 1);
        const DN<kLoc> z2 = m.he ? dn_var<kLoc>(z[2], 2) : dn_const<kLoc>(0.0);
        const DN<kLoc> z3 = m.he ? dn_var<kLoc>(z[3], 3) : dn_const<kLoc>(0.0);
        DN<kLoc> Sy[3], Se;
        group_local_S<DN<kLoc>>(k, m, Ed, ze, z1, z2, z3, nH, nHe, yn, en, xp, Sy, Se);
        const DN<kLoc> Sz[kLoc] = {Se, Sy[0], Sy[1], Sy[2]};
        double B[kLoc][kLoc], d[kLoc][1];
#pragma unroll
        for (int i = 0; i < kLoc; ++i) {
          d[i][0] = -(z[i] - Sz[i].v);
#pragma unroll
          for (int j = 0; j < kLoc; ++j) B[i][j] = (i == j ? 1.0 : 0.0) - Sz[i].g[j];
        }
        solve4<1>(B, d);
        double lam = 1.0;
        lam = cap_lo(lam, z[1], d[1][0], 0.0);
        lam = cap_hi(lam, z[1], d[1][0], nH);
        if (m.he) {
          lam = cap_lo(lam, z[2], d[2][0], 0.0);
          lam = cap_lo(lam, z[3], d[3][0], 0.0);
          // n_HeIII >= 0; it starts at exactly 0, so a step over the bound by
          // rounding only is not cut
          const double tot = z[2] + z[3], dtot = d[2][0] + d[3][0];
          if (tot + dtot > nHe * (1.0 + 1e-12)) lam = cap_hi(lam, tot, dtot, nHe);
        }
        if (!k.iso) lam = cap_lo(lam, z[0], d[0][0], 0.0);
#pragma unroll
        for (int i = 0; i < kLoc; ++i) z[i] += lam * d[i][0];
        double small = fabs(lam * d[1][0]) / nH;
        if (m.he) small = fmax(small, fmax(fabs(lam * d[2][0]), fabs(lam * d[3][0])) / nHe);
        if (!k.iso) small = fmax(small, fabs(lam * d[0][0]) / z[0]);
        if (!(small == small)) break;  // NaN
        // quadratic convergence: after an undamped step of relative size
        // <= 1e-9 the iterate is at the root to rounding
        if (lam == 1.0 && small <= 1e-9) {
          conv = true;
          break;
        }
      }
      if (!conv) fail = 1.0;
      itmax = fmax(itmax, (double)its);
#pragma unroll
      for (int g = 0; g < kMaxGroups; ++g)
        if (g < G) a.Et[g * N + idx] = E[g];
      if (!k.iso) a.et[idx] = z[0];
      a.yt[idx] = z[1];
      if (m.he) {
        a.yt[N + idx] = z[2];
        a.yt[2 * N + idx] = z[3];
      }
    }
    // residual, B = d f_loc / dz and C = d f_loc / dE at the (solved or given) state
    DN<kJ> Ej[kMaxGroups];
#pragma unroll
    for (int g = 0; g < kMaxGroups; ++g)
      Ej[g] = g < G ? dn_var<kJ>(E[g], kLoc + g) : dn_const<kJ>(0.0);
    const DN<kJ> ze = k.iso ? dn_const<kJ>(0.0) : dn_var<kJ>(z[0], 0);
    const DN<kJ> z1 = dn_var<kJ>(z[1], 1);
    const DN<kJ> z2 = m.he ? dn_var<kJ>(z[2], 2) : dn_const<kJ>(0.0);
    const DN<kJ> z3 = m.he ? dn_var<kJ>(z[3], 3) : dn_const<kJ>(0.0);
    DN<kJ> Sy[3], Se;
    group_local_S<DN<kJ>>(k, m, Ej, ze, z1, z2, z3, nH, nHe, yn, en, xp, Sy, Se);
    const DN<kJ> Sz[kLoc] = {Se, Sy[0], Sy[1], Sy[2]};
    double B[kLoc][kLoc], X[kLoc][1 + kMaxGroups], f[kLoc];
#pragma unroll
    for (int i = 0; i < kLoc; ++i) {
      f[i] = z[i] - Sz[i].v;
      X[i][0] = f[i];
#pragma unroll
      for (int j = 0; j < kLoc; ++j) B[i][j] = (i == j ? 1.0 : 0.0) - Sz[i].g[j];
#pragma unroll
      for (int h = 0; h < kMaxGroups; ++h) X[i][1 + h] = -Sz[i].g[kLoc + h];
    }
    solve4<1 + kMaxGroups>(B, X);
    // Schur terms: J_gs = dt theta c sigma_E[s][g] E_g / a^3 (d f_E,g / d n_s)
    const double jf = k.dt * k.theta * kC / (k.a_1 * k.a_1 * k.a_1);
#pragma unroll
    for (int g = 0; g < kMaxGroups; ++g) {
      if (g >= G) continue;
      double J[3];
#pragma unroll
      for (int s = 0; s < 3; ++s) J[s] = jf * m.sigE[s][g] * E[g];
      double kb = 0.0;
#pragma unroll
      for (int s = 0; s < 3; ++s) kb += J[s] * X[1 + s][0];
      a.kB[g * N + idx] = kb;
#pragma unroll
      for (int h = 0; h < kMaxGroups; ++h) {
        if (h >= G) continue;
        double v = 0.0;
#pragma unroll
        for (int s = 0; s < 3; ++s) v += J[s] * X[1 + s][1 + h];
        a.K[(g * G + h) * N + idx] = v;
      }
    }
#pragma unroll
    for (int s = 0; s < kLoc; ++s) {
      a.Bf[s * N + idx] = X[s][0];
#pragma unroll
      for (int h = 0; h < kMaxGroups; ++h)
        if (h < G) a.BC[(s * G + h) * N + idx] = X[s][1 + h];
    }
    if (!k.iso) sfe += (f[0] / en) * (f[0] / en);
    sfy += (f[1] / nH) * (f[1] / nH);
    if (m.he) sfy += (f[2] / nHe) * (f[2] / nHe) + (f[3] / nHe) * (f[3] / nHe);
    bool finite = isfinite(f[0]) && isfinite(f[1]) && isfinite(f[2]) && isfinite(f[3]);
#pragma unroll
    for (int g = 0; g < kMaxGroups; ++g) finite = finite && isfinite(E[g]);
    if (!finite) bad = 1.0;
    if (a.fe_out && !k.iso) a.fe_out[idx] = f[0];
    if (a.fy_out) {
      a.fy_out[idx] = f[1];
      if (m.he) {
        a.fy_out[N + idx] = f[2];
        a.fy_out[2 * N + idx] = f[3];
      }
    }
  }
  double v[5] = {sfy, sfe, fail, itmax, bad};
  const int im[5] = {0, 0, 1, 1, 1};
  const int sl[5] = {RS_FN2, RS_FE_LOC2, RS_LOCAL_FAIL, RS_LOCAL_ITS, RS_NONFINITE};
  block_reduce_store<5>(v, im, sl, part);
}

// Coupled Schur residual of group g (see launch_group_coupled).
__global__ void __launch_bounds__(kBlock)
k_group_coupled(StepK k, int G, int g, const double* __restrict__ rS,
                const double* __restrict__ diag, const double* __restrict__ cfx,
                const double* __restrict__ cfy, const double* __restrict__ cfz,
                const double* __restrict__ K, const double* __restrict__ x,
                double* __restrict__ b, double* __restrict__ part) {
  const int per[3] = {k.bc[0] == RH_BC_PERIODIC, k.bc[2] == RH_BC_PERIODIC,
                      k.bc[4] == RH_BC_PERIODIC};
  const int nd[3] = {k.nx, k.ny, k.nz};
  const double* cf[3] = {cfx, cfy, cfz};
  const long long N = k.N;
  const double* xg = x + g * N;
  double sw = 0.0, s2 = 0.0, rmax = 0.0;
  for (long long idx = xcd_tile(blockIdx.x, gridDim.x) * (long long)blockDim.x + threadIdx.x;
       idx < N; idx += (long long)blockDim.x * gridDim.x) {
    int c[3];
    cell_ijk(idx, k.ny, k.nz, c[0], c[1], c[2]);
    double Ax = diag[idx] * xg[idx];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int q[3];
      if (neighbour(c, nd, per, d, +1, q))
        Ax -= cf[d][idx] * xg[cell_index(q[0], q[1], q[2], k.ny, k.nz)];
      if (neighbour(c, nd, per, d, -1, q)) {
        const long long Q = cell_index(q[0], q[1], q[2], k.ny, k.nz);
        Ax -= cf[d][Q] * xg[Q];
      }
    }
    double r = rS[idx] - Ax;
    for (int h = 0; h < G; ++h)
      if (h != g) r += K[((long long)g * G + h) * N + idx] * x[h * N + idx];
    b[idx] = r;
    sw += (r / k.E_s) * (r / k.E_s);
    s2 += r * r;
    rmax = fmax(rmax, fabs(r));
  }
  double v[3] = {sw, s2, rmax};
  const int im[3] = {0, 0, 1};
  const int sl[3] = {RS_FE2, RS_R2, RS_RMAX};
  block_reduce_store<3>(v, im, sl, part);
}

__global__ void __launch_bounds__(kBlock)
k_groups_coupled(StepK k, int G, GroupOps o, const double* __restrict__ K,
                 const double* __restrict__ x, double* __restrict__ B,
                 double* __restrict__ part) {
  const int per[3] = {k.bc[0] == RH_BC_PERIODIC, k.bc[2] == RH_BC_PERIODIC,
                      k.bc[4] == RH_BC_PERIODIC};
  const int nd[3] = {k.nx, k.ny, k.nz};
  const long long N = k.N;
  double sw = 0.0, sm = 0.0;
  for (long long idx = xcd_tile(blockIdx.x, gridDim.x) * (long long)blockDim.x + threadIdx.x;
       idx < N; idx += (long long)blockDim.x * gridDim.x) {
    int c[3];
    cell_ijk(idx, k.ny, k.nz, c[0], c[1], c[2]);
    long long Qp[3], Qm[3];
    bool hp[3], hm[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int q[3];
      hp[d] = neighbour(c, nd, per, d, +1, q);
      Qp[d] = hp[d] ? cell_index(q[0], q[1], q[2], k.ny, k.nz) : idx;
      hm[d] = neighbour(c, nd, per, d, -1, q);
      Qm[d] = hm[d] ? cell_index(q[0], q[1], q[2], k.ny, k.nz) : idx;
    }
    double xv[kMaxGroups];
#pragma unroll
    for (int g = 0; g < kMaxGroups; ++g) xv[g] = g < G ? x[g * N + idx] : 0.0;
#pragma unroll
    for (int g = 0; g < kMaxGroups; ++g) {
      if (g >= G) continue;
      const double* xg = x + g * N;
      double t = o.diag[g][idx] * xv[g];
      double Sx = t, mag = fabs(t);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        if (hp[d]) {
          t = o.cf[g][d][idx] * xg[Qp[d]];
          Sx -= t;
          mag += fabs(t);
        }
        if (hm[d]) {
          t = o.cf[g][d][Qm[d]] * xg[Qm[d]];
          Sx -= t;
          mag += fabs(t);
        }
      }
#pragma unroll
      for (int h = 0; h < kMaxGroups; ++h)
        if (h < G && h != g) {
          t = K[((long long)g * G + h) * N + idx] * xv[h];
          Sx -= t;
          mag += fabs(t);
        }
      double r = Sx;
      if (o.rS[g]) {
        r = o.rS[g][idx] - Sx;
        mag += fabs(o.rS[g][idx]);
      }
      B[g * N + idx] = r;
      const double iw = 1.0 / o.E_s[g];
      sw += (r * iw) * (r * iw);
      sm += (mag * iw) * (mag * iw);
    }
  }
  double v[2] = {sw, sm};
  const int im[2] = {0, 0};
  const int sl[2] = {RS_FE2, RS_MAG2};
  block_reduce_store<2>(v, im, sl, part);
}

// Weighted inner products <u, v>_W = sum_g sum_P u v / E_s,g^2 over [G][N]
// vectors: one partial sum per workgroup and vector, out[i * grid + block].
__global__ void __launch_bounds__(kBlock)
k_wdots(long long N, int G, WeightK wk, const double* __restrict__ u,
        const double* __restrict__ V, long long stride, int nv, double* __restrict__ out) {
  double acc[kKrylovMax];
#pragma unroll
  for (int i = 0; i < kKrylovMax; ++i) acc[i] = 0.0;
  for (int g = 0; g < G; ++g) {
    const double wg = wk.w[g];
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < N;
         idx += (long long)blockDim.x * gridDim.x) {
      const double ug = u[g * N + idx] * wg;
#pragma unroll
      for (int i = 0; i < kKrylovMax; ++i)
        if (i < nv) acc[i] += ug * V[i * stride + g * N + idx];
    }
  }
  __shared__ double sh[kKrylovMax][kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < kKrylovMax; ++i) {
    if (i >= nv) continue;
    const double v = wave_sum(acc[i]);
    if (lane == 0) sh[i][wid] = v;
  }
  __syncthreads();
  if (threadIdx.x < nv) {
    double t = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) t += sh[threadIdx.x][w];
    out[threadIdx.x * gridDim.x + blockIdx.x] = t;
  }
}

// y = a y + sum_{i < nv} c_i V_i over [G][N] vectors; with norm_part != NULL
// also the workgroup partials of ||y||_W^2 (after the update).
__global__ void __launch_bounds__(kBlock)
k_wcombine(long long N, int G, WeightK wk, double* __restrict__ y, double a,
           const double* __restrict__ V, long long stride, int nv, Coefs cs,
           double* __restrict__ norm_part) {
  double sn = 0.0;
  for (int g = 0; g < G; ++g) {
    const double wg = wk.w[g];
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < N;
         idx += (long long)blockDim.x * gridDim.x) {
      const long long o = g * N + idx;
      double v = a == 0.0 ? 0.0 : a * y[o];
#pragma unroll
      for (int i = 0; i < kKrylovMax; ++i)
        if (i < nv) v += cs.c[i] * V[i * stride + o];
      y[o] = v;
      sn += v * v * wg;
    }
  }
  if (!norm_part) return;
  __shared__ double sh[kBlock / 64];
  const double v = wave_sum(sn);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) t += sh[w];
    norm_part[blockIdx.x] = t;
  }
}

// out[i] = sum over the grid's partials of vector i, in a fixed order (one
// workgroup per vector; out may be mapped host memory).
__global__ void __launch_bounds__(kBlock)
k_wsum(const double* __restrict__ part, int grid, double* __restrict__ out) {
  __shared__ double sh[kBlock / 64];
  double v = 0.0;
  for (int b = threadIdx.x; b < grid; b += kBlock) v += part[blockIdx.x * grid + b];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) t += sh[w];
    out[blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(kBlock)
k_groups_init(long long N, GroupK m, double f0, double f1, double f2, double f3, double E0,
              double x0, double e0, const double* __restrict__ nH, double* __restrict__ E,
              double* __restrict__ e, double* __restrict__ y, double* __restrict__ part) {
  const double frac[kMaxGroups] = {f0, f1, f2, f3};
  double bad = 0.0;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < N;
       idx += (long long)blockDim.x * gridDim.x) {
    const double n = nH[idx];
    if (!(n > 0.0) || !isfinite(n)) bad = 1.0;
    for (int g = 0; g < m.G; ++g) E[g * N + idx] = frac[g] * E0;
    y[idx] = (1.0 - x0) * n;
    if (m.he) {
      const double nHe = m.y_he * n;
      y[N + idx] = (1.0 - x0) * nHe;
      y[2 * N + idx] = x0 * nHe;
    }
    if (e) e[idx] = e0;
  }
  double v[1] = {bad};
  const int im[1] = {1};
  const int sl[1] = {RS_NONFINITE};
  block_reduce_store<1>(v, im, sl, part);
}

}  // namespace

void launch_local_groups(hipStream_t s, const StepK& k, const GroupK& m, const GroupLocalArgs& a,
                         double* part) {
  const long long g = (k.N + kBlock - 1) / kBlock;
  const int grid = (int)(g < kPartCap ? g : kPartCap);
  hipLaunchKernelGGL(k_local_groups, dim3(grid), dim3(kBlock), 0, s, k, m, a, part);
}

void launch_group_coupled(hipStream_t s, const StepK& k, int G, int g, const double* rS,
                          const double* diag, const double* const cf[3], const double* K,
                          const double* x, double* b, double* part) {
  hipLaunchKernelGGL(k_group_coupled, dim3(red_grid(k.N)), dim3(kBlock), 0, s, k, G, g, rS, diag,
                     cf[0], cf[1], cf[2], K, x, b, part);
}

void launch_groups_coupled(hipStream_t s, const StepK& k, int G, const GroupOps& o,
                           const double* K, const double* x, double* B, double* part) {
  hipLaunchKernelGGL(k_groups_coupled, dim3(red_grid(k.N)), dim3(kBlock), 0, s, k, G, o, K, x, B,
                     part);
}

void launch_wdots(hipStream_t s, long long N, int G, const WeightK& wk, const double* u,
                  const double* V, long long stride, int nv, double* part, double* out) {
  hipLaunchKernelGGL(k_wdots, dim3(kKrylovGrid), dim3(kBlock), 0, s, N, G, wk, u, V, stride, nv,
                     part);
  hipLaunchKernelGGL(k_wsum, dim3(nv), dim3(kBlock), 0, s, part, kKrylovGrid, out);
}

void launch_wcombine(hipStream_t s, long long N, int G, const WeightK& wk, double* y, double a,
                     const double* V, long long stride, int nv, const Coefs& c, double* part,
                     double* norm_out) {
  hipLaunchKernelGGL(k_wcombine, dim3(kKrylovGrid), dim3(kBlock), 0, s, N, G, wk, y, a, V, stride,
                     nv, c, norm_out ? part : nullptr);
  if (norm_out) hipLaunchKernelGGL(k_wsum, dim3(1), dim3(kBlock), 0, s, part, kKrylovGrid, norm_out);
}

void launch_groups_init(hipStream_t s, long long N, const GroupK& m, const double* frac, double E0,
                        double x0, double e0, const double* nH, double* E, double* e, double* y,
                        double* part) {
  double f[kMaxGroups] = {0.0, 0.0, 0.0, 0.0};
  for (int g = 0; g < m.G; ++g) f[g] = frac[g];
  hipLaunchKernelGGL(k_groups_init, dim3(red_grid(N)), dim3(kBlock), 0, s, N, m, f[0], f[1], f[2],
                     f[3], E0, x0, e0, nH, E, e, y, part);
}

}  // namespace rh

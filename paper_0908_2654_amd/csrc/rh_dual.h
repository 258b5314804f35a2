// Forward-mode dual numbers and the temperature fits of the rate
// coefficients, shared by the hydrogen and the hydrogen + helium chemistry
// kernels.  The scalar type S of the templates is double or a dual number.
#ifndef RH_DUAL_H
#define RH_DUAL_H

#include <hip/hip_runtime.h>

#include <cmath>

namespace rh {

__device__ inline double dexp(double a) { return exp(a); }
__device__ inline double dpow(double a, double p) { return pow(a, p); }
__device__ inline double dsqrt(double a) { return sqrt(a); }
__device__ inline double dlog(double a) { return log(a); }
__device__ inline double dmax0(double a) { return fmax(a, 0.0); }
template <class S>
__device__ inline S lift(double v);
template <>
__device__ inline double lift<double>(double v) { return v; }

// Forward-mode dual numbers with NV derivative slots (the local solve uses
// two, the adjoint's local terms seven).
template <int NV>
struct DN {
  double v, g[NV];
};
template <int NV>
__device__ inline DN<NV> dn_const(double v) {
  DN<NV> r;
  r.v = v;
#pragma unroll
  for (int i = 0; i < NV; ++i) r.g[i] = 0.0;
  return r;
}
template <int NV>
__device__ inline DN<NV> dn_var(double v, int slot) {
  DN<NV> r = dn_const<NV>(v);
  r.g[slot] = 1.0;
  return r;
}
#define RH_DN_BIN(OP, VAL, GRAD)                                                   \
  template <int NV>                                                                \
  __device__ inline DN<NV> operator OP(DN<NV> a, DN<NV> b) {                       \
    DN<NV> r;                                                                      \
    r.v = VAL;                                                                     \
    _Pragma("unroll") for (int i = 0; i < NV; ++i) r.g[i] = GRAD;                  \
    return r;                                                                      \
  }
RH_DN_BIN(+, a.v + b.v, a.g[i] + b.g[i])
RH_DN_BIN(-, a.v - b.v, a.g[i] - b.g[i])
RH_DN_BIN(*, a.v * b.v, a.g[i] * b.v + a.v * b.g[i])
#undef RH_DN_BIN
template <int NV>
__device__ inline DN<NV> operator/(DN<NV> a, DN<NV> b) {
  const double iv = 1.0 / b.v, q = a.v * iv;
  DN<NV> r;
  r.v = q;
#pragma unroll
  for (int i = 0; i < NV; ++i) r.g[i] = (a.g[i] - q * b.g[i]) * iv;
  return r;
}
template <int NV> __device__ inline DN<NV> operator+(DN<NV> a, double b) { return a + dn_const<NV>(b); }
template <int NV> __device__ inline DN<NV> operator+(double b, DN<NV> a) { return dn_const<NV>(b) + a; }
template <int NV> __device__ inline DN<NV> operator-(DN<NV> a, double b) { return a - dn_const<NV>(b); }
template <int NV> __device__ inline DN<NV> operator-(double b, DN<NV> a) { return dn_const<NV>(b) - a; }
template <int NV>
__device__ inline DN<NV> operator*(DN<NV> a, double b) {
  DN<NV> r;
  r.v = a.v * b;
#pragma unroll
  for (int i = 0; i < NV; ++i) r.g[i] = a.g[i] * b;
  return r;
}
template <int NV> __device__ inline DN<NV> operator*(double b, DN<NV> a) { return a * b; }
template <int NV> __device__ inline DN<NV> operator/(DN<NV> a, double b) { return a * (1.0 / b); }
template <int NV> __device__ inline DN<NV> operator/(double b, DN<NV> a) { return dn_const<NV>(b) / a; }
template <int NV>
__device__ inline DN<NV> chain(DN<NV> a, double fv, double dfv) {
  DN<NV> r;
  r.v = fv;
#pragma unroll
  for (int i = 0; i < NV; ++i) r.g[i] = a.g[i] * dfv;
  return r;
}
template <int NV> __device__ inline DN<NV> dexp(DN<NV> a) { const double e = exp(a.v); return chain(a, e, e); }
template <int NV> __device__ inline DN<NV> dpow(DN<NV> a, double p) { const double pv = pow(a.v, p); return chain(a, pv, p * pv / a.v); }
template <int NV> __device__ inline DN<NV> dsqrt(DN<NV> a) { const double s = sqrt(a.v); return chain(a, s, 0.5 / s); }
template <int NV> __device__ inline DN<NV> dlog(DN<NV> a) { return chain(a, log(a.v), 1.0 / a.v); }
template <int NV> __device__ inline DN<NV> dmax0(DN<NV> a) { return a.v >= 0.0 ? a : dn_const<NV>(0.0); }
template <int NV> __device__ inline DN<NV> dfabs(DN<NV> a) { return a.v < 0.0 ? dn_const<NV>(0.0) - a : a; }
template <int NV> __device__ inline DN<NV> dfmax(DN<NV> a, double c) { return a.v >= c ? a : dn_const<NV>(c); }
template <>
__device__ inline DN<1> lift<DN<1>>(double v) { return dn_const<1>(v); }
template <>
__device__ inline DN<2> lift<DN<2>>(double v) { return dn_const<2>(v); }
template <>
__device__ inline DN<4> lift<DN<4>>(double v) { return dn_const<4>(v); }
template <>
__device__ inline DN<7> lift<DN<7>>(double v) { return dn_const<7>(v); }
template <>
__device__ inline DN<8> lift<DN<8>>(double v) { return dn_const<8>(v); }

// Rate fits (Hui & Gnedin 1997 case B; Cen 1992 collisional excitation).
// The case-B fits are powers of lambda = 315614 K / T and of 1 + (lambda /
// c)^p; they are evaluated as exponentials of L = ln(lambda), which the
// recombination rate and the recombination cooling share: 3 logarithms and
// 4 exponentials instead of 6 general powers (the ALU-bound local solve
// evaluates them in every iteration).
constexpr double kLn315614 = 12.662275226919286;  // ln(315614)
constexpr double kLn2p740 = 1.0079579203999789;   // ln(2.740)
constexpr double kLn2p250 = 0.8109302162163288;   // ln(2.250)
template <class S>
__device__ inline S hg_ln_lambda(S T) {
  return kLn315614 - dlog(T);
}
template <class S>
__device__ inline S alpha_B_of_L(S L) {
  S den = 1.0 + dexp(0.407 * (L - kLn2p740));
  return 2.753e-14 * dexp(1.5 * L - 2.242 * dlog(den));
}
template <class S>
__device__ inline S cool_recB_of_L(S T, S L) {
  S den = 1.0 + dexp(0.376 * (L - kLn2p250));
  return 3.435e-30 * T * dexp(1.970 * L - 3.720 * dlog(den));
}
template <class S>
__device__ inline S alpha_B_fit(S T) {
  return alpha_B_of_L(hg_ln_lambda(T));
}
template <class S>
__device__ inline S cool_recB(S T) {
  return cool_recB_of_L(T, hg_ln_lambda(T));
}
template <class S>
__device__ inline S cool_collexc(S T) {
  return 7.5e-19 * dexp(-118348.0 / T) / (1.0 + dsqrt(T / 1.0e5));
}

__device__ inline double dval(double a) { return a; }
template <int NV>
__device__ inline double dval(const DN<NV>& a) { return a.v; }
__device__ inline double dchain(double, double fv, double) { return fv; }
template <int NV>
__device__ inline DN<NV> dchain(const DN<NV>& x, double fv, double dfv) {
  return chain(x, fv, dfv);
}

}  // namespace rh

#endif  // RH_DUAL_H

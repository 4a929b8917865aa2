// Quadrature-point kernel D of the force operator and its hand-written tangent.
//
// Per quadrature point (Sec. 2.1 eq. matrices; Sec. 3.4 eqs. visc_stress .. energy_regularization):
//   J = dx/dxi, J^-1, grad v = (dv/dxi) J^-1,
//   e+ = (e + sqrt(e^2 + eps^2))/2,  p = (gamma-1) rho e+,  c_s = sqrt(gamma (gamma-1) e+),
//   sigma = -p I + mu eps(v)  (mu = mu_imp when viscosity is on),
//   S = w_q |J| sigma J^-T  (coefficient of grad_xi w_n in (F 1)_n),
//   s = w_q |J| sigma : grad v  (coefficient of phi_j in (F^T v)_j).
// Strong mass conservation rho |J| w_q = m_q (constant) removes rho and |J| from the
// pressure part: w_q |J| p = (gamma-1) m_q e+ and w_q |J| mu = m_q nu with
// nu = h (q2 |delta_v|_s + q1 c_s psi).  The tangent is the forward derivative of every
// step above along (dJ, d(dv/dxi), de), written out by hand.
#pragma once

#include <hip/hip_runtime.h>

#include "ilh_internal.h"

namespace ilh {

// FP64: IEEE operations.  FP32 (Jacobian actions inside the Krylov solver, tolerance
// 1e-5): the hardware reciprocal and square root (about 1 ulp), no correction steps.
__device__ __forceinline__ double f_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float f_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double f_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float f_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double f_cbrt(double x) { return cbrt(x); }
__device__ __forceinline__ float f_cbrt(float x) { return cbrtf(x); }
__device__ __forceinline__ double f_tanh(double x) { return tanh(x); }
__device__ __forceinline__ float f_tanh(float x) { return tanhf(x); }

// Minimum that propagates NaN from either argument (fmin drops it), so that a non-finite
// det J or time-step candidate is not mistaken for a valid one.
__device__ __forceinline__ double nan_min(double a, double b) { return (a != a || a < b) ? a : b; }

template <int D, typename T>
__device__ __forceinline__ void inv_det(const T J[D][D], T Ji[D][D], T& det) {
  if constexpr (D == 2) {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const T id = f_rcp(det);
    Ji[0][0] = J[1][1] * id;
    Ji[0][1] = -J[0][1] * id;
    Ji[1][0] = -J[1][0] * id;
    Ji[1][1] = J[0][0] * id;
  } else {
    const T c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const T c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const T c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    const T id = f_rcp(det);
    Ji[0][0] = c00 * id;
    Ji[1][0] = c01 * id;
    Ji[2][0] = c02 * id;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
  }
}

// e+ and r = sqrt(e^2 + eps^2); the negative branch uses the cancellation-free form.
template <typename T>
__device__ __forceinline__ void e_plus(T e, T eps, T& ep, T& r) {
  r = f_sqrt(e * e + eps * eps);
  ep = (e >= T(0)) ? T(0.5) * (e + r) : eps * eps * f_rcp(T(2) * (r - e));
}

template <int D, typename T>
__device__ __forceinline__ T h_scale(T ratio) {
  if constexpr (D == 2) return f_sqrt(ratio);
  else return f_cbrt(ratio);
}

// Residual form: S (d x d) and s.
template <int D, typename T>
__device__ __forceinline__ void qp_force(const KParams& P, T gam, T mq, T dJ0, const T J[D][D],
                                         const T Gv[D][D], T e, T S[D][D], T& s) {
  T Ji[D][D], det;
  inv_det<D, T>(J, Ji, det);
  T gv[D][D];
#pragma unroll
  for (int c = 0; c < D; ++c)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      T acc = 0;
#pragma unroll
      for (int a = 0; a < D; ++a) acc += Gv[c][a] * Ji[a][b];
      gv[c][b] = acc;
    }
  T ep, r;
  e_plus<T>(e, T(P.eps_e), ep, r);
  const T Pq = (gam - T(1)) * mq * ep;  // w_q |J| p
  T Sig[D][D];
#pragma unroll
  for (int c = 0; c < D; ++c)
#pragma unroll
    for (int b = 0; b < D; ++b) Sig[c][b] = (c == b) ? -Pq : T(0);
  if (P.visc) {
    const T h = T(P.h0) * h_scale<D, T>(det / dJ0);
    T div = 0;
#pragma unroll
    for (int c = 0; c < D; ++c) div += gv[c][c];
    const T dv = h * div;
    const T cs = f_sqrt(gam * (gam - T(1)) * ep);
    const T dsc = P.dsc_mode ? T(2) * h * cs * T(P.hc_inv) : T(P.dsc_w);
    const T aabs = f_sqrt(dv * dv + dsc * dsc);
    const T t = -dv / (T(2) * dsc) - T(P.psi_shift);
    const T psi = T(0.5) + T(0.5) * f_tanh(t);
    const T nu = h * (T(P.q2) * aabs + T(P.q1) * cs * psi);
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
      for (int b = 0; b < D; ++b) Sig[c][b] += mq * nu * T(0.5) * (gv[c][b] + gv[b][c]);
  }
  T ss = 0;
#pragma unroll
  for (int c = 0; c < D; ++c)
#pragma unroll
    for (int a = 0; a < D; ++a) {
      T acc = 0;
#pragma unroll
      for (int b = 0; b < D; ++b) acc += Sig[c][b] * Ji[a][b];
      S[c][a] = acc;
      ss += Sig[c][a] * gv[c][a];
    }
  s = ss;
}

// Tangent form: dS and ds along (dJ, dGv, de).  VISC = 0/1 fixes the viscosity switch at
// compile time, VISC = -1 reads it from P.
template <int D, typename T, int VISC = -1>
__device__ __forceinline__ void qp_tangent(const KParams& P, T gam, T mq, T dJ0, const T J[D][D],
                                           const T Gv[D][D], T e, const T dJ[D][D],
                                           const T dGv[D][D], T de, T dS[D][D], T& ds) {
  T Ji[D][D], det;
  inv_det<D, T>(J, Ji, det);
  // tmp = J^-1 dJ ; dJi = -tmp J^-1
  T tmp[D][D], dJi[D][D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int d = 0; d < D; ++d) {
      T acc = 0;
#pragma unroll
      for (int c = 0; c < D; ++c) acc += Ji[a][c] * dJ[c][d];
      tmp[a][d] = acc;
    }
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      T acc = 0;
#pragma unroll
      for (int d = 0; d < D; ++d) acc += tmp[a][d] * Ji[d][b];
      dJi[a][b] = -acc;
    }
  T gv[D][D], dgv[D][D];
#pragma unroll
  for (int c = 0; c < D; ++c)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      T acc = 0, dacc = 0;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        acc += Gv[c][a] * Ji[a][b];
        dacc += dGv[c][a] * Ji[a][b] + Gv[c][a] * dJi[a][b];
      }
      gv[c][b] = acc;
      dgv[c][b] = dacc;
    }
  T ep, r;
  e_plus<T>(e, T(P.eps_e), ep, r);
  const T dep = ep * f_rcp(r) * de;
  const T g1 = gam - T(1);
  const T Pq = g1 * mq * ep, dPq = g1 * mq * dep;
  T Sig[D][D], dSig[D][D];
#pragma unroll
  for (int c = 0; c < D; ++c)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      Sig[c][b] = (c == b) ? -Pq : T(0);
      dSig[c][b] = (c == b) ? -dPq : T(0);
    }
  if ((VISC < 0) ? (P.visc != 0) : (VISC == 1)) {
    T trd = 0, div = 0, ddiv = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      trd += tmp[a][a];
      div += gv[a][a];
      ddiv += dgv[a][a];
    }
    const T h = T(P.h0) * h_scale<D, T>(det * f_rcp(dJ0));
    const T dh = h * trd * T(1.0 / D);
    const T dv = h * div, ddv = dh * div + h * ddiv;
    const T cs = f_sqrt(gam * g1 * ep);
    const T dcs = cs * dep * f_rcp(T(2) * ep);
    T dsc, ddsc;
    if (P.dsc_mode) {
      dsc = T(2) * h * cs * T(P.hc_inv);
      ddsc = T(2) * T(P.hc_inv) * (dh * cs + h * dcs);
    } else {
      dsc = T(P.dsc_w);
      ddsc = T(0);
    }
    const T aabs = f_sqrt(dv * dv + dsc * dsc);
    const T daabs = (dv * ddv + dsc * ddsc) * f_rcp(aabs);
    const T i2d = f_rcp(T(2) * dsc);
    const T t = -dv * i2d - T(P.psi_shift);
    const T dt = -(ddv * dsc - dv * ddsc) * i2d * f_rcp(dsc);
    const T th = f_tanh(t);
    const T psi = T(0.5) + T(0.5) * th;
    const T dpsi = T(0.5) * (T(1) - th * th) * dt;
    const T base = T(P.q2) * aabs + T(P.q1) * cs * psi;
    const T nu = h * base;
    const T dnu = dh * base + h * (T(P.q2) * daabs + T(P.q1) * (dcs * psi + cs * dpsi));
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
      for (int b = 0; b < D; ++b) {
        const T ep_ = T(0.5) * (gv[c][b] + gv[b][c]);
        const T dep_ = T(0.5) * (dgv[c][b] + dgv[b][c]);
        Sig[c][b] += mq * nu * ep_;
        dSig[c][b] += mq * (dnu * ep_ + nu * dep_);
      }
  }
  T dss = 0;
#pragma unroll
  for (int c = 0; c < D; ++c)
#pragma unroll
    for (int a = 0; a < D; ++a) {
      T acc = 0;
#pragma unroll
      for (int b = 0; b < D; ++b) acc += dSig[c][b] * Ji[a][b] + Sig[c][b] * dJi[a][b];
      dS[c][a] = acc;
      dss += dSig[c][a] * gv[c][a] + Sig[c][a] * dgv[c][a];
    }
  ds = dss;
}

// TG2D energy source s(x,y) = (pi/4) (cos 3 pi x cos pi y - cos pi x cos 3 pi y) / (gamma-1)
// (= v . grad e for the steady vortex) and its gradient.
template <typename T>
__device__ __forceinline__ T tg_source(T x, T y, T gam) {
  const double pi = 3.14159265358979323846;
  const double X = double(x), Y = double(y);
  return T(pi / 4.0 * (cos(3 * pi * X) * cos(pi * Y) - cos(pi * X) * cos(3 * pi * Y)) /
           (double(gam) - 1.0));
}
__device__ __forceinline__ void f_sincospi(double x, double* s, double* c) { sincospi(x, s, c); }
// FP32: hardware sine/cosine (absolute error ~1e-6 for the bounded arguments used here)
__device__ __forceinline__ void f_sincospi(float x, float* s, float* c) {
  *s = __sinf(3.14159265358979f * x);
  *c = __cosf(3.14159265358979f * x);
}

// Gradient of the source in the working precision T (used by the tangent kernels):
// sin/cos of pi x and pi y, the triple angles from sin 3a = s (3 - 4 s^2), cos 3a = c (4 c^2 - 3).
template <typename T>
__device__ __forceinline__ void tg_source_grad(T x, T y, T gam, T& gx, T& gy) {
  const T pi = T(3.14159265358979323846);
  const T c = pi * pi * T(0.25) * f_rcp(gam - T(1));
  T sx, cx, sy, cy;
  f_sincospi(x, &sx, &cx);
  f_sincospi(y, &sy, &cy);
  const T s3x = sx * (T(3) - T(4) * sx * sx), c3x = cx * (T(4) * cx * cx - T(3));
  const T s3y = sy * (T(3) - T(4) * sy * sy), c3y = cy * (T(4) * cy * cy - T(3));
  gx = c * (-T(3) * s3x * cy + sx * c3y);
  gy = c * (-c3x * sy + T(3) * cx * s3y);
}

}  // namespace ilh

// Linearised Jacobian action of the stage residual: coefficients of the quadrature-point
// stress tangent (shared by the 2D and 3D kernels).
//
// At a quadrature point the tangent of (S, s) (Sec. 3.4: forward derivative of the stress
// kernel) is linear in the direction's (dJ, d(dv/dxi), de), with coefficients that depend on
// the state w alone.  With gv = (dv/dxi) J^-1, U = dJ J^-1, dJ^-1 = -J^-1 U and
// dgv = d(dv/dxi) J^-1 - gv U:
//   Sig  = -P I  [+ m_q nu eps(gv)],                      P  = (gamma - 1) m_q e+
//   dSig = -cP de I  [+ dnu eps(gv) + m_q nu eps(dgv)],   cP = P / sqrt(e^2 + eps^2)
//   dnu  = a0 tr(U) + a1 tr(dgv) + a2 de   (viscosity; m_q folded into a)
//   dS = dSig J^-T + Sig dJ^-T,   ds = dSig : gv + Sig : dgv,
//   TG source row: db = m_q grad s(x_q) . dx_q.
// Every coefficient after J^-1 and gv multiplies the direction exactly once, so the stage
// factor tau (the direction enters as tau dk) is folded into them at linearisation.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "ilh_internal.h"
#include "ilh_pointwise.h"

namespace ilh {

// Stored coefficients per point in D dimensions: J^-1 (D^2), gv (D^2); then P, cP without
// viscosity, or Sig (D(D+1)/2, upper triangle row by row), cP, m_q nu, a0, a1, a2 with it;
// then m_q grad s (D) with the source.
template <int D, int VISC, int SRC>
struct LinLayout {
  static constexpr int NSYM = D * (D + 1) / 2;
  static constexpr int BASE = 2 * D * D;
  static constexpr int NPT = BASE + (VISC ? NSYM + 5 : 2);
  static constexpr int NQD = NPT + (SRC ? D : 0);
};

// index of (r, c), r <= c, in the row-by-row upper triangle
template <int D>
__device__ __forceinline__ constexpr int sym_idx(int r, int c) {
  return r <= c ? r * D - r * (r - 1) / 2 + (c - r) : c * D - c * (c - 1) / 2 + (r - c);
}

// Coefficients of the stress tangent at one point, FP64 (see the file comment).
template <int D, int VISC>
__device__ __forceinline__ void lin_coefs(const KParams& P, double gam, double mq, double dJ0,
                                          const double J[D][D], const double Gv[D][D], double e, double* c) {
  constexpr int B = 2 * D * D;
  double Ji[D][D], det;
  inv_det<D, double>(J, Ji, det);
  double gv[D][D];
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      double acc = 0;
#pragma unroll
      for (int a = 0; a < D; ++a) acc += Gv[r][a] * Ji[a][b];
      gv[r][b] = acc;
    }
  double ep, rr;
  e_plus<double>(e, P.eps_e, ep, rr);
  const double g1 = gam - 1.0;
  const double Pq = g1 * mq * ep, cP = Pq / rr;
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      c[r * D + b] = Ji[r][b];
      c[D * D + r * D + b] = gv[r][b];
    }
  if constexpr (!VISC) {
    c[B] = Pq;
    c[B + 1] = cP;
  } else {
    constexpr int NSYM = D * (D + 1) / 2;
    double div = 0;
#pragma unroll
    for (int r = 0; r < D; ++r) div += gv[r][r];
    const double h = P.h0 * h_scale<D, double>(det / dJ0);
    const double dv = h * div;
    const double cs = sqrt(gam * g1 * ep);
    // derivatives as combinations of (tr U, tr dgv, de)
    const double dh[3] = {h / D, 0.0, 0.0};
    const double ddv[3] = {h * div / D, h, 0.0};
    const double dcs[3] = {0.0, 0.0, cs / (2.0 * rr)};
    double dsc, ddsc[3];
    if (P.dsc_mode) {
      dsc = 2.0 * h * cs * P.hc_inv;
#pragma unroll
      for (int i = 0; i < 3; ++i) ddsc[i] = 2.0 * P.hc_inv * (dh[i] * cs + h * dcs[i]);
    } else {
      dsc = P.dsc_w;
#pragma unroll
      for (int i = 0; i < 3; ++i) ddsc[i] = 0.0;
    }
    const double aabs = sqrt(dv * dv + dsc * dsc);
    const double t = -dv / (2.0 * dsc) - P.psi_shift;
    const double th = tanh(t);
    const double psi = 0.5 + 0.5 * th;
    const double base = P.q2 * aabs + P.q1 * cs * psi;
    const double mnu = mq * h * base;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double daabs = (dv * ddv[i] + dsc * ddsc[i]) / aabs;
      const double dt = -(ddv[i] * dsc - dv * ddsc[i]) / (2.0 * dsc * dsc);
      const double dpsi = 0.5 * (1.0 - th * th) * dt;
      const double dnu = dh[i] * base + h * (P.q2 * daabs + P.q1 * (dcs[i] * psi + cs * dpsi));
      c[B + NSYM + 2 + i] = mq * dnu;
    }
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int q = r; q < D; ++q) c[B + sym_idx<D>(r, q)] = (r == q ? -Pq : 0.0) + mnu * 0.5 * (gv[r][q] + gv[q][r]);
    c[B + NSYM] = cP;
    c[B + NSYM + 1] = mnu;
  }
}

// Apply the stored coefficients to one point's (dJ, dGv, de): dS (D x D) and ds.
template <int D, typename T, int VISC>
__device__ __forceinline__ void lin_apply(const T* c, const T dJ[D][D], const T dGv[D][D], T de, T dS[D][D],
                                          T& ds) {
  constexpr int B = 2 * D * D;
  T Ji[D][D], gv[D][D];
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      Ji[r][b] = c[r * D + b];
      gv[r][b] = c[D * D + r * D + b];
    }
  T U[D][D], dJi[D][D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      T acc = 0;
#pragma unroll
      for (int q = 0; q < D; ++q) acc += dJ[a][q] * Ji[q][b];
      U[a][b] = acc;
    }
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      T acc = 0;
#pragma unroll
      for (int q = 0; q < D; ++q) acc += Ji[a][q] * U[q][b];
      dJi[a][b] = -acc;
    }
  if constexpr (!VISC) {
    const T Pq = c[B], dP = c[B + 1] * de;
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int a = 0; a < D; ++a) dS[r][a] = -dP * Ji[a][r] - Pq * dJi[a][r];
    T trdgv = 0, trgv = 0;
#pragma unroll
    for (int r = 0; r < D; ++r) {
      trgv += gv[r][r];
#pragma unroll
      for (int a = 0; a < D; ++a) trdgv += dGv[r][a] * Ji[a][r] - gv[r][a] * U[a][r];
    }
    ds = -dP * trgv - Pq * trdgv;
  } else {
    constexpr int NSYM = D * (D + 1) / 2;
    T dgv[D][D];
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int b = 0; b < D; ++b) {
        T acc = 0;
#pragma unroll
        for (int q = 0; q < D; ++q) acc += dGv[r][q] * Ji[q][b] - gv[r][q] * U[q][b];
        dgv[r][b] = acc;
      }
    T trU = 0, trdgv = 0;
#pragma unroll
    for (int r = 0; r < D; ++r) {
      trU += U[r][r];
      trdgv += dgv[r][r];
    }
    const T dnu = c[B + NSYM + 2] * trU + c[B + NSYM + 3] * trdgv + c[B + NSYM + 4] * de;
    const T dP = c[B + NSYM] * de, mnu = c[B + NSYM + 1];
    T Sig[D][D], dSig[D][D];
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int q = 0; q < D; ++q) {
        Sig[r][q] = c[B + sym_idx<D>(r, q)];
        dSig[r][q] = (r == q ? -dP : T(0)) + dnu * (T(0.5) * (gv[r][q] + gv[q][r])) +
                     mnu * (T(0.5) * (dgv[r][q] + dgv[q][r]));
      }
    T dss = 0;
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int a = 0; a < D; ++a) {
        T acc = 0;
#pragma unroll
        for (int b = 0; b < D; ++b) acc += dSig[r][b] * Ji[a][b] + Sig[r][b] * dJi[a][b];
        dS[r][a] = acc;
        dss += dSig[r][a] * gv[r][a] + Sig[r][a] * dgv[r][a];
      }
    ds = dss;
  }
}

// Transpose of lin_apply at one point: given the weights A (D x D) of dS and a_s of ds, the
// weights GJ, GGv, ge of (dJ, dGv, de) such that <A, dS> + a_s ds = <GJ, dJ> + <GGv, dGv> + ge de
// for every direction.  Reverse sweep of the forward formulas (file comment):
//   Gsig = A J^-1 + a_s gv,   Gdji = A^T Sig,   Gdgv = a_s Sig + m_q nu sym(Gsig) + nub a1 I,
//   Pb = -tr Gsig,  nub = <Gsig, sym gv>,       ge = cP Pb + nub a2,
//   Ub = nub a0 I - gv^T Gdgv - J^-T Gdji,      GJ = Ub J^-T,  GGv = Gdgv J^-T.
// Without viscosity Sig = -P I and the nu terms vanish.
template <int D, typename T, int VISC>
__device__ __forceinline__ void lin_apply_t(const T* c, const T A[D][D], T as, T GJ[D][D], T GGv[D][D], T& ge) {
  constexpr int B = 2 * D * D;
  constexpr int NSYM = D * (D + 1) / 2;
  T Ji[D][D], gv[D][D], Sig[D][D];
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      Ji[r][b] = c[r * D + b];
      gv[r][b] = c[D * D + r * D + b];
    }
  T cP, mnu = T(0), a0 = T(0), a1 = T(0), a2 = T(0);
  if constexpr (!VISC) {
    const T Pq = c[B];
    cP = c[B + 1];
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int q = 0; q < D; ++q) Sig[r][q] = r == q ? -Pq : T(0);
  } else {
    cP = c[B + NSYM];
    mnu = c[B + NSYM + 1];
    a0 = c[B + NSYM + 2];
    a1 = c[B + NSYM + 3];
    a2 = c[B + NSYM + 4];
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
      for (int q = 0; q < D; ++q) Sig[r][q] = c[B + sym_idx<D>(r, q)];
  }
  T Gs[D][D];
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      T acc = as * gv[r][b];
#pragma unroll
      for (int a = 0; a < D; ++a) acc += A[r][a] * Ji[a][b];
      Gs[r][b] = acc;
    }
  T trGs = 0, nub = 0;
#pragma unroll
  for (int r = 0; r < D; ++r) {
    trGs += Gs[r][r];
#pragma unroll
    for (int q = 0; q < D; ++q) nub += Gs[r][q] * (T(0.5) * (gv[r][q] + gv[q][r]));
  }
  if constexpr (!VISC) nub = T(0);
  ge = -cP * trGs + nub * a2;
  T Gdgv[D][D], Gdji[D][D];
#pragma unroll
  for (int r = 0; r < D; ++r)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      T g = as * Sig[r][b] + (r == b ? nub * a1 : T(0));
      if constexpr (VISC) g += mnu * (T(0.5) * (Gs[r][b] + Gs[b][r]));
      Gdgv[r][b] = g;
      T acc = 0;
#pragma unroll
      for (int q = 0; q < D; ++q) acc += A[q][r] * Sig[q][b];
      Gdji[r][b] = acc;
    }
  T Ub[D][D];
#pragma unroll
  for (int q = 0; q < D; ++q)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      T acc = q == b ? nub * a0 : T(0);
#pragma unroll
      for (int r = 0; r < D; ++r) acc -= gv[r][q] * Gdgv[r][b] + Ji[r][q] * Gdji[r][b];
      Ub[q][b] = acc;
    }
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int q = 0; q < D; ++q) {
      T gj = 0, gg = 0;
#pragma unroll
      for (int b = 0; b < D; ++b) {
        gj += Ub[a][b] * Ji[q][b];
        gg += Gdgv[a][b] * Ji[q][b];
      }
      GJ[a][q] = gj;
      GGv[a][q] = gg;
    }
}

// 32-bit element offset from a uniform base (byte offsets below 4 GiB, checked on the host).
typedef const char __attribute__((address_space(1))) * gbytes;
template <typename T>
__device__ __forceinline__ T ld32(const T* __restrict__ base, uint32_t i) {
  const gbytes p = (gbytes)base + (uint64_t)(i * (uint32_t)sizeof(T));
  return *(const T __attribute__((address_space(1)))*)p;
}

// The same load with the non-temporal hint (streamed data read once per launch: the hint keeps it
// from evicting the lines that are reused, at the cost of the 64-bit address form)
template <typename T>
__device__ __forceinline__ T ld32_nt(const T* __restrict__ base, uint32_t i) {
  const gbytes p = (gbytes)base + (uint64_t)(i * (uint32_t)sizeof(T));
  return __builtin_nontemporal_load((const T __attribute__((address_space(1)))*)p);
}

// Store and no-return atomic add at a 32-bit element offset from a uniform base (the
// scalar-base + vector-offset forms; byte offsets below 4 GiB, checked on the host).
typedef char __attribute__((address_space(1))) * gbytes_w;
template <typename T>
__device__ __forceinline__ void st32(T* __restrict__ base, uint32_t i, T v) {
  *(T __attribute__((address_space(1)))*)((gbytes_w)base + (uint64_t)(i * (uint32_t)sizeof(T))) = v;
}
template <typename T>
__device__ __forceinline__ void atomic_add32(T* base, uint32_t i, T v) {
  __hip_atomic_fetch_add((T __attribute__((address_space(1)))*)((gbytes_w)base + (uint64_t)(i * (uint32_t)sizeof(T))), v,
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Work-group barrier ordering LDS only: its release and acquire fences name the local address
// space, so a wave's global stores and atomics still in flight are not drained first (the
// fences of __syncthreads cover global memory too and wait for them).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Wait for every vector memory operation of the wave.  Placed where all loads have been
// consumed and no store has been issued, it costs nothing and tells the compiler's wait
// insertion that no load is pending, so later register reuse does not wait on the stores
// and atomics issued after it.
__device__ __forceinline__ void vm_drained() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Work-group -> tile map for a chip of 8 XCDs, each with its own L2: work-groups are handed to
// the XCDs in turn (w mod 8), so neighbouring tiles would sit on different L2s and the cache
// lines they share (node rows at strip ends, the direction's overlapping strips) would be
// fetched and partially written back once per XCD.  The map gives XCD x the contiguous tile
// range [x nb/8, (x+1) nb/8) instead: a band of the mesh per L2.  It is a bijection of [0, nb),
// so results never depend on how the hardware actually distributes the work-groups.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t w, uint32_t nb) {
  constexpr uint32_t NX = 8;
  const uint32_t x = w % NX, slot = w / NX, q = nb / NX, rem = nb % NX;
  // x (q + 1) + slot for the first rem XCDs, rem (q + 1) + (x - rem) q + slot after them; in one
  // branch-free expression (the kernels' first scalar loads then issue together)
  return x * q + min(x, rem) + slot;
}

// A wave-uniform pointer made opaque to the compiler (scalar registers): loads from it take the
// scalar-base + 32-bit vector-offset form instead of per-lane 64-bit address arithmetic.
template <typename T>
__device__ __forceinline__ const T* sbase(const T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<const T*>(((uint64_t)hi << 32) | lo);
}

}  // namespace ilh

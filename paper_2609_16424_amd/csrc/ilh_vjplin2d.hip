// Transpose Jacobian action of the stage residual in 2D, J^T y, at the stored linearisation
// point: the transpose of eq. pa_jac_action, which keeps its gather - pointwise - scatter
// structure (Sec. 3.4).  The kernel reads the same stored tangent coefficients as the
// Jacobian action (ilh_jvplin2d.hip) and the same work-group / lane map: one wave = EPW
// consecutive elements of one element row, lane (z, qx) = quadrature column qx of element z.
//
// Per point, with y's velocity restricted to the unconstrained rows (constrained velocity rows
// of R are the identity and carry no force or mass), the gather forms the weights of the
// forward outputs: A = grad_xi y_v (paired with dS), a_s = -y_e (paired with ds, which enters
// the energy rows with a minus sign), and the mass and source terms; lin_apply_t returns the
// weights of (dJ, dGv, de), which the scatter contracts with grad_xi of the H1 basis (position
// and velocity rows) and with the L2 basis (energy rows).  The identity and -tau I blocks of
// the position rows and the identity of the constrained velocity rows are added by each node's
// owner.  Position and velocity rows take one atomic add per node and strip: both parts of the
// output's H1 rows must be zero on entry.
#include <hip/hip_runtime.h>

#include "ilh_internal.h"
#include "ilh_lin.h"

namespace ilh {

template <int D1D, int Q1D, typename T, int VISC, int SRC>
__global__ void __launch_bounds__(64) k_vjp2d_q(const KParams P, const Tab2<T, D1D, Q1D> tb,
                                                const T* __restrict__ y, const T* __restrict__ qd, double tau_,
                                                T* __restrict__ out) {
  constexpr int K = D1D - 1, L1D = K, NLD = L1D * L1D;
  constexpr int EPW = 64 / Q1D;
  constexpr int NS = K * EPW + 1;
  constexpr int NQD = LinLayout<2, VISC, SRC>::NQD;
  constexpr int NVO = 2 * D1D * D1D;  // one field's H1 outputs per element
  constexpr int NOP = NVO | 1;
  static_assert(Q1D % 2 == 0, "the quadrature rows are processed in pairs");

  __shared__ T sS[4][D1D][NS];  // y_x0 y_x1 y_v0 y_v1 strips (velocity: constrained rows zeroed)
  __shared__ T sE[EPW * NLD];   // y_e
  __shared__ T sO[64][NOP];     // per-lane contributions (position rows, velocity rows, energy rows)
  __shared__ T sBG[2][Q1D][D1D];
  __shared__ T sBLt[Q1D][L1D];

  const int lane = threadIdx.x;
  const uint32_t tile = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int sx = tile % gridDim.x, ey = tile / gridDim.x, ex0 = sx * EPW;
  const int nx = P.n[0];
  const int E = min(EPW, nx - ex0);
  const int ns = K * E + 1;
  const uint32_t ng0 = P.ng[0], ng1 = P.ng[1];
  const uint32_t N = (uint32_t)P.N, nh1 = 2 * N;
  const uint32_t ebase = (uint32_t)ey * nx + ex0;
  const uint32_t row0 = (uint32_t)(K * ey) * ng0 + (uint32_t)(K * ex0);
  const T tau = T(tau_);
  const bool last_x = (ex0 + E == nx), last_y = (ey == P.n[1] - 1);
  const int z = lane / Q1D, qx = lane - z * Q1D;
  const bool active = z < E;

  constexpr int NTS = 4 * D1D * NS, RT = (NTS + 63) / 64;
  constexpr int NLS = EPW * NLD, RL = (NLS + 63) / 64;
  T tr[RT], lr[RL];
#pragma unroll
  for (int q = 0; q < RT; ++q) {
    const int i = lane + 64 * q, si = min(i % NS, ns - 1), t = min(i / NS, 4 * D1D - 1), b = t % D1D,
              f = t / D1D;
    const T v = ld32(y, (f < 2 ? f * N : nh1 + (f - 2) * N) + row0 + (uint32_t)b * ng0 + si);
    const uint32_t I = K * ex0 + si, J = K * ey + b;
    const bool cons = f == 2 ? (I == 0 || I == ng0 - 1) : (f == 3 && (J == 0 || J == ng1 - 1));
    tr[q] = cons ? T(0) : v;
  }
#pragma unroll
  for (int q = 0; q < RL; ++q) lr[q] = ld32(y, 2 * nh1 + ebase * NLD + min(lane + 64 * q, E * NLD - 1));
  const double rj_l = P.rj0[ebase + (active ? z : 0)];
  for (int i = lane; i < Q1D * D1D; i += 64) {
    sBG[0][i / D1D][i % D1D] = tb.B[i / D1D][i % D1D];
    sBG[1][i / D1D][i % D1D] = tb.G[i / D1D][i % D1D];
  }
  for (int i = lane; i < Q1D * L1D; i += 64) sBLt[i / L1D][i % L1D] = tb.BL[i / L1D][i % L1D];
#pragma unroll
  for (int q = 0; q < RT; ++q) {
    const int i = lane + 64 * q;
    if (i < NTS) (&sS[0][0][0])[i] = tr[q];
  }
#pragma unroll
  for (int q = 0; q < RL; ++q) {
    const int i = lane + 64 * q;
    if (i < NLS) sE[i] = lr[q];
  }
  __syncthreads();

  // per-lane sums over the column: X (position rows), V (velocity rows), both as the
  // coefficients of (G_a B_b, B_a G_b + B_a B_b) like the forward kernel; TL energy rows
  T X0[2][D1D], X1[2][D1D], V0[2][D1D], V1[2][D1D], TL[L1D];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < D1D; ++b) X0[c][b] = X1[c][b] = V0[c][b] = V1[c][b] = T(0);
#pragma unroll
  for (int bl = 0; bl < L1D; ++bl) TL[bl] = T(0);
  if (active) {
    const int s0 = K * z;
    T AB[2][D1D], AG[2][D1D];
    {
      T Bq[D1D], Gq[D1D];
#pragma unroll
      for (int a = 0; a < D1D; ++a) {
        Bq[a] = sBG[0][qx][a];
        Gq[a] = sBG[1][qx][a];
      }
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < D1D; ++b) {
          T ab = 0, ag = 0;
#pragma unroll
          for (int a = 0; a < D1D; ++a) {
            const T yv = sS[2 + c][b][s0 + a];
            ab += Bq[a] * yv;
            ag += Gq[a] * yv;
          }
          AB[c][b] = ab;
          AG[c][b] = ag;
        }
    }
    T ALy[L1D];
#pragma unroll
    for (int bl = 0; bl < L1D; ++bl) {
      T a1 = 0;
#pragma unroll
      for (int al = 0; al < L1D; ++al) a1 += sBLt[qx][al] * sE[z * NLD + al + L1D * bl];
      ALy[bl] = a1;
    }
    const T wx = tb.W[qx] * T(rj_l);
    const T* __restrict__ qb = qd + (int64_t)tile * (Q1D * NQD * 64);
    auto ldrow = [&](const int qy, T* cf) {
      const T* rb = sbase(qb + qy * (NQD * 64));
#pragma unroll
      for (int f = 0; f < NQD; ++f) cf[f] = ld32(rb, (uint32_t)(f * 64 + lane));
    };
    auto row = [&](const int qy, const T* cf) {
      T A[2][2], yvq[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        T a0 = 0, a1 = 0, m = 0;
#pragma unroll
        for (int b = 0; b < D1D; ++b) {
          const T By = tb.B[qy][b], Gy = tb.G[qy][b];
          a0 += By * AG[c][b];
          a1 += Gy * AB[c][b];
          m += By * AB[c][b];
        }
        A[c][0] = a0;
        A[c][1] = a1;
        yvq[c] = m;
      }
      T yeq = 0;
#pragma unroll
      for (int bl = 0; bl < L1D; ++bl) yeq += tb.BL[qy][bl] * ALy[bl];
      const T mq = wx * tb.W[qy];
      T GJ[2][2], GGv[2][2], ge;
      lin_apply_t<2, T, VISC>(cf, A, -yeq, GJ, GGv, ge);
      T gx[2] = {T(0), T(0)};
      if constexpr (SRC != 0) {
        gx[0] = -yeq * cf[NQD - 2];
        gx[1] = -yeq * cf[NQD - 1];
      }
#pragma unroll
      for (int b = 0; b < D1D; ++b) {
        const T By = tb.B[qy][b], Gy = tb.G[qy][b];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          X0[c][b] += By * GJ[c][0];
          X1[c][b] += Gy * GJ[c][1] + By * gx[c];
          V0[c][b] += By * GGv[c][0];
          V1[c][b] += Gy * GGv[c][1] + By * (mq * yvq[c]);
        }
      }
      const T te = ge + mq * yeq;
#pragma unroll
      for (int bl = 0; bl < L1D; ++bl) TL[bl] += tb.BL[qy][bl] * te;
    };
    T ca[NQD], cb[NQD];
    ldrow(0, ca);
#pragma unroll 1
    for (int qy = 0; qy < Q1D; qy += 2) {
      ldrow(qy + 1, cb);
      row(qy, ca);
      if (qy + 2 < Q1D) ldrow(qy + 2, ca);
      row(qy + 1, cb);
    }
  }

  // H1 rows, position part then velocity part: per-lane contributions to sO, node sums over
  // the (one or two) elements of the strip holding the node, the owner's identity terms, one
  // atomic add per node
#pragma unroll 1
  for (int part = 0; part < 2; ++part) {
    if (active) {
      T Bq[D1D], Gq[D1D];
#pragma unroll
      for (int a = 0; a < D1D; ++a) {
        Bq[a] = sBG[0][qx][a];
        Gq[a] = sBG[1][qx][a];
      }
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < D1D; ++b)
#pragma unroll
          for (int a = 0; a < D1D; ++a)
            sO[lane][c * D1D * D1D + b * D1D + a] =
                part == 0 ? Gq[a] * X0[c][b] + Bq[a] * X1[c][b] : Gq[a] * V0[c][b] + Bq[a] * V1[c][b];
    }
    __syncthreads();
#pragma unroll 1
    for (int i = lane; i < 2 * D1D * NS; i += 64) {
      const int s = i % NS, t = i / NS, b = t % D1D, c = t / D1D;
      if (s >= ns) continue;
      const int zz = s / K, a = s - K * zz;
      T f = T(0);
      if (zz < E) {
#pragma unroll
        for (int q = 0; q < Q1D; ++q) f += sO[zz * Q1D + q][c * D1D * D1D + b * D1D + a];
      }
      if (a == 0 && zz > 0) {
#pragma unroll
        for (int q = 0; q < Q1D; ++q) f += sO[(zz - 1) * Q1D + q][c * D1D * D1D + b * D1D + K];
      }
      const uint32_t gi = c * N + row0 + (uint32_t)b * ng0 + s;
      const bool own = (s < K * E || last_x) && (b < K || last_y);
      if (own) {
        const T yx = sS[c][b][s];
        if (part == 0) {
          f += yx;
        } else {
          f -= tau * yx;
          const uint32_t I = K * ex0 + s, J = K * ey + b;
          const bool cons = (c == 0) ? (I == 0 || I == ng0 - 1) : (J == 0 || J == ng1 - 1);
          if (cons) f += y[nh1 + gi];
        }
      }
      unsafeAtomicAdd(&out[part * nh1 + gi], f);
    }
    __syncthreads();
  }
  // energy rows (element-owned)
  if (active) {
#pragma unroll
    for (int bl = 0; bl < L1D; ++bl)
#pragma unroll
      for (int al = 0; al < L1D; ++al) sO[lane][bl * L1D + al] = sBLt[qx][al] * TL[bl];
  }
  __syncthreads();
  for (int i = lane; i < E * NLD; i += 64) {
    const int zz = i / NLD, t = i % NLD;
    T o = 0;
#pragma unroll
    for (int q = 0; q < Q1D; ++q) o += sO[zz * Q1D + q][t];
    out[2 * nh1 + ebase * NLD + i] = o;
  }
}

// ---- host side ---------------------------------------------------------------------------
template <typename T, int D1D, int Q1D>
static Tab2<T, D1D, Q1D> vjp_tab2(const ilh_ctx* c) {
  Tab2<T, D1D, Q1D> tb;
  for (int q = 0; q < Q1D; ++q) {
    for (int d = 0; d < D1D; ++d) {
      tb.B[q][d] = T(c->h_B[q * D1D + d]);
      tb.G[q][d] = T(c->h_G[q * D1D + d]);
    }
    for (int d = 0; d < D1D - 1; ++d) tb.BL[q][d] = T(c->h_BL[q * (D1D - 1) + d]);
    tb.W[q] = T(c->h_w1[q]);
  }
  return tb;
}

template <int K, typename T, int VISC, int SRC>
static void vjp_t(ilh_ctx* c, const T* y, const T* qd, T* out) {
  constexpr int D1D = K + 1, Q1D = 2 * K, EPW = 64 / Q1D;
  const dim3 g((c->n[0] + EPW - 1) / EPW, c->n[1]);
  klaunch(c, k_vjp2d_q<D1D, Q1D, T, VISC, SRC>, g, dim3(64), 0, c->kp, vjp_tab2<T, D1D, Q1D>(c), y, qd,
          c->lin_tau, out);
}

template <typename T>
static int dispatch_vjp(ilh_ctx* c, const T* y, const T* qd, T* out) {
  const int v = c->kp.visc ? 1 : 0, s = c->kp.tg_source ? 1 : 0, code = 4 * c->k + 2 * v + s;
  switch (code) {
    case 8: vjp_t<2, T, 0, 0>(c, y, qd, out); break;
    case 9: vjp_t<2, T, 0, 1>(c, y, qd, out); break;
    case 10: vjp_t<2, T, 1, 0>(c, y, qd, out); break;
    case 11: vjp_t<2, T, 1, 1>(c, y, qd, out); break;
    case 12: vjp_t<3, T, 0, 0>(c, y, qd, out); break;
    case 13: vjp_t<3, T, 0, 1>(c, y, qd, out); break;
    case 14: vjp_t<3, T, 1, 0>(c, y, qd, out); break;
    case 15: vjp_t<3, T, 1, 1>(c, y, qd, out); break;
    default: return ILH_EINVAL;
  }
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

// Transpose action with the stored coefficients of precision prec (they must be current).
int launch_vjp2d_q(ilh_ctx* c, int prec, const void* y, void* out) {
  if (!lin2d_available(c)) return ILH_EINVAL;
  const int p = prec == 64 ? 1 : 0;
  if (!c->qd[p] || !c->qd_ok[p]) return fail(c, ILH_EINVAL, "transpose action before its linearisation");
  return p ? dispatch_vjp<double>(c, (const double*)y, (const double*)c->qd[p], (double*)out)
           : dispatch_vjp<float>(c, (const float*)y, (const float*)c->qd[p], (float*)out);
}

}  // namespace ilh

// Stage residual in 2D (Sec. 4: R(k) of the implicit stage, with the mass-multiplied rows of the
// block preconditioner's reading) on the work-group / lane map of the linearised kernels: one
// wave = EPW consecutive elements of one element row, lane (z, qx) = quadrature column qx of
// element z, walking the Q1D quadrature rows.  FP64 throughout; meshes without artificial
// viscosity (the viscous residual keeps the generic element kernel).
//
//   R_x = k_x - w_v                                  (position rows, written by the node's owner)
//   R_v = M_V k_v + F(w) 1                           (constrained velocity rows: R_v = k_v)
//   R_e = M_E k_e - F(w)^T w_v - b(w_x)              (element-owned)
// with w = u + tau k.  Per quadrature point the force S_q (d x d) and s_q = S_q : grad_xi w_v
// come from qp_force, the same pointwise code as the generic kernel; the transposes use the
// factored expansions of the linearised apply, and each velocity row of a strip takes one
// atomic add.  The velocity part of r must be zero on entry.
#include <hip/hip_runtime.h>

#include "ilh_internal.h"
#include "ilh_lin.h"
#include "ilh_pointwise.h"

namespace ilh {

// TG energy source (pi/4) (cos 3 pi x cos pi y - cos pi x cos 3 pi y) / (gamma - 1) from one
// cospi per coordinate and cos 3a = c (4 c^2 - 3)
__device__ __forceinline__ double tg_source_c(double x, double y, double gam) {
  const double cx = cospi(x), cy = cospi(y);
  const double c3x = cx * (4.0 * cx * cx - 3.0), c3y = cy * (4.0 * cy * cy - 3.0);
  return 0.78539816339744830962 * (c3x * cy - cx * c3y) / (gam - 1.0);
}

template <int D1D, int Q1D, int SRC>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
k_res2d(const KParams P, const Tab2<double, D1D, Q1D> tb, const double* __restrict__ u,
        const double* __restrict__ kk, double tau, double* __restrict__ r) {
  constexpr int K = D1D - 1, L1D = K, NLD = L1D * L1D;
  constexpr int EPW = 64 / Q1D;
  constexpr int NS = K * EPW + 1;
  constexpr int NVO = 2 * D1D * D1D;
  constexpr int NOP = NVO | 1;
  constexpr int NNE = 2 * D1D * NS, RG = (NNE + 63) / 64;  // node entries (c, b, s) of the strip
  constexpr int NLS = EPW * NLD, RL = (NLS + 63) / 64;

  __shared__ double sW[6][D1D][NS];  // w_x (2), w_v (2), k_v (2)
  __shared__ double sE[2][NLS];      // w_e, k_e
  __shared__ double sO[64][NOP];     // per-lane contributions (velocity, then energy)
  __shared__ double sBG[2][Q1D][D1D];
  __shared__ double sBLt[Q1D][L1D];

  const int lane = threadIdx.x;
  const uint32_t tile = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int sx = tile % gridDim.x, ey = tile / gridDim.x;
  const int ex0 = sx * EPW;
  const int nx = P.n[0], ny = P.n[1];
  const int E = min(EPW, nx - ex0);
  const int ns = K * E + 1;
  const uint32_t ng0 = P.ng[0], ng1 = P.ng[1];
  const uint32_t N = (uint32_t)P.N, nh1 = 2 * N;
  const bool last_x = (ex0 + E == nx), last_y = (ey == ny - 1);
  const uint32_t ebase = (uint32_t)ey * nx + ex0;
  const uint32_t row0 = (uint32_t)(K * ey) * ng0 + (uint32_t)(K * ex0);
  const int z = lane / Q1D, qx = lane - z * Q1D;
  const bool active = z < E;

  for (int i = lane; i < Q1D * D1D; i += 64) {
    sBG[0][i / D1D][i % D1D] = tb.B[i / D1D][i % D1D];
    sBG[1][i / D1D][i % D1D] = tb.G[i / D1D][i % D1D];
  }
  for (int i = lane; i < Q1D * L1D; i += 64) sBLt[i / L1D][i % L1D] = tb.BL[i / L1D][i % L1D];

  // gathers: every lane reads u_x, k_x, u_v, k_v of its node entries (indices clamped in range,
  // so all loads are in flight together), and the energy DOFs of the strip's elements
  double gx[RG], gk[RG], gv[RG], gkv[RG];
#pragma unroll
  for (int q = 0; q < RG; ++q) {
    const int i = min(lane + 64 * q, NNE - 1), s = min(i % NS, ns - 1), t = i / NS, b = t % D1D, c = t / D1D;
    const uint32_t gi = c * N + row0 + (uint32_t)b * ng0 + s;
    gx[q] = ld32(u, gi);
    gk[q] = ld32(kk, gi);
    gv[q] = ld32(u, nh1 + gi);
    gkv[q] = ld32(kk, nh1 + gi);
  }
  double ge[RL], gke[RL];
#pragma unroll
  for (int q = 0; q < RL; ++q) {
    const uint32_t i = 2 * nh1 + ebase * NLD + min(lane + 64 * q, E * NLD - 1);
    ge[q] = ld32(u, i);
    gke[q] = ld32(kk, i);
  }
  const double rj_l = P.rj0[ebase + (active ? z : 0)];
  const double gam = P.gamma[ebase + (active ? z : 0)];
  const double dJ0 = P.j0e[ebase + (active ? z : 0)];
#pragma unroll
  for (int q = 0; q < RG; ++q) {
    const int i = lane + 64 * q;
    if (i >= NNE) continue;
    const int s = i % NS, t = i / NS, b = t % D1D, c = t / D1D;
    const double wv = gv[q] + tau * gkv[q];
    sW[c][b][s] = gx[q] + tau * gk[q];
    sW[2 + c][b][s] = wv;
    sW[4 + c][b][s] = gkv[q];
    if (s >= ns) continue;
    // position rows and constrained velocity rows: the node's single owner
    const uint32_t I = K * ex0 + s, J = K * ey + b;
    const bool own = (s < K * E || last_x) && (b < K || last_y);
    if (!own) continue;
    const uint32_t gi = c * N + row0 + (uint32_t)b * ng0 + s;
    r[gi] = gk[q] - wv;
    const bool cons = (c == 0) ? (I == 0 || I == ng0 - 1) : (J == 0 || J == ng1 - 1);
    if (cons) r[nh1 + gi] = gkv[q];
  }
#pragma unroll
  for (int q = 0; q < RL; ++q) {
    const int i = lane + 64 * q;
    if (i < NLS) {
      sE[0][i] = ge[q] + tau * gke[q];
      sE[1][i] = gke[q];
    }
  }
  __syncthreads();

  double TL[L1D];
#pragma unroll
  for (int bl = 0; bl < L1D; ++bl) TL[bl] = 0.0;
  if (active) {
    const int s0 = K * z;
    double Bq[D1D], Gq[D1D], BLq[L1D];
#pragma unroll
    for (int a = 0; a < D1D; ++a) {
      Bq[a] = sBG[0][qx][a];
      Gq[a] = sBG[1][qx][a];
    }
#pragma unroll
    for (int a = 0; a < L1D; ++a) BLq[a] = sBLt[qx][a];
    // xi-contractions of the lane's column: w_x and w_v (value and derivative), k_v (value)
    double AB[4][D1D], AG[4][D1D], AK[2][D1D];
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
      for (int b = 0; b < D1D; ++b) {
        double ab = 0, ag = 0;
#pragma unroll
        for (int a = 0; a < D1D; ++a) {
          const double xv = sW[f][b][s0 + a];
          ab += Bq[a] * xv;
          ag += Gq[a] * xv;
        }
        AB[f][b] = ab;
        AG[f][b] = ag;
      }
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int b = 0; b < D1D; ++b) {
        double ab = 0;
#pragma unroll
        for (int a = 0; a < D1D; ++a) ab += Bq[a] * sW[4 + c][b][s0 + a];
        AK[c][b] = ab;
      }
    double ALw[L1D], ALk[L1D];
#pragma unroll
    for (int bl = 0; bl < L1D; ++bl) {
      double a1 = 0, a2 = 0;
#pragma unroll
      for (int al = 0; al < L1D; ++al) {
        a1 += BLq[al] * sE[0][z * NLD + al + L1D * bl];
        a2 += BLq[al] * sE[1][z * NLD + al + L1D * bl];
      }
      ALw[bl] = a1;
      ALk[bl] = a2;
    }
    double T0[2][D1D], T1[2][D1D];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int b = 0; b < D1D; ++b) T0[c][b] = T1[c][b] = 0.0;
    const double wx = tb.W[qx] * rj_l;
#pragma unroll 1
    for (int qy = 0; qy < Q1D; ++qy) {
      double J[2][2], Gv[2][2], kv[2], xq[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        double j0 = 0, j1 = 0, g0 = 0, g1 = 0, m = 0, x = 0;
#pragma unroll
        for (int b = 0; b < D1D; ++b) {
          const double By = tb.B[qy][b], Gy = tb.G[qy][b];
          j0 += By * AG[c][b];
          j1 += Gy * AB[c][b];
          g0 += By * AG[2 + c][b];
          g1 += Gy * AB[2 + c][b];
          m += By * AK[c][b];
          x += By * AB[c][b];
        }
        J[c][0] = j0;
        J[c][1] = j1;
        Gv[c][0] = g0;
        Gv[c][1] = g1;
        kv[c] = m;
        xq[c] = x;
      }
      double eq = 0, ke = 0;
#pragma unroll
      for (int bl = 0; bl < L1D; ++bl) {
        eq += tb.BL[qy][bl] * ALw[bl];
        ke += tb.BL[qy][bl] * ALk[bl];
      }
      const double mq = wx * tb.W[qy];
      double S[2][2], sq;
      qp_force<2, double>(P, gam, mq, dJ0, J, Gv, eq, S, sq);
      double cl = mq * ke - sq;
      if constexpr (SRC != 0) cl -= mq * tg_source_c(xq[0], xq[1], gam);
#pragma unroll
      for (int b = 0; b < D1D; ++b) {
        const double By = tb.B[qy][b], Gy = tb.G[qy][b];
        T0[0][b] += By * S[0][0];
        T0[1][b] += By * S[1][0];
        T1[0][b] += Gy * S[0][1] + By * mq * kv[0];
        T1[1][b] += Gy * S[1][1] + By * mq * kv[1];
      }
#pragma unroll
      for (int bl = 0; bl < L1D; ++bl) TL[bl] += tb.BL[qy][bl] * cl;
    }
#pragma unroll
    for (int a = 0; a < D1D; ++a) {  // reloaded: not kept live through the row loop
      Bq[a] = sBG[0][qx][a];
      Gq[a] = sBG[1][qx][a];
    }
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int b = 0; b < D1D; ++b)
#pragma unroll
        for (int a = 0; a < D1D; ++a)
          sO[lane][c * D1D * D1D + b * D1D + a] = Gq[a] * T0[c][b] + Bq[a] * T1[c][b];
  }
  __syncthreads();

  // velocity rows that are not constrained: the Q1D columns of the (one or two) elements of the
  // strip that hold the node, one atomic add per node and strip
#pragma unroll 1
  for (int i = lane; i < NNE; i += 64) {
    const int s = i % NS, t = i / NS, b = t % D1D, c = t / D1D;
    if (s >= ns) continue;
    const uint32_t I = K * ex0 + s, J = K * ey + b;
    const bool cons = (c == 0) ? (I == 0 || I == ng0 - 1) : (J == 0 || J == ng1 - 1);
    if (cons) continue;
    const int zz = s / K, a = s - K * zz;
    double f = 0.0;
    if (zz < E) {
#pragma unroll
      for (int q = 0; q < Q1D; ++q) f += sO[zz * Q1D + q][c * D1D * D1D + b * D1D + a];
    }
    if (a == 0 && zz > 0) {
#pragma unroll
      for (int q = 0; q < Q1D; ++q) f += sO[(zz - 1) * Q1D + q][c * D1D * D1D + b * D1D + K];
    }
    unsafeAtomicAdd(&r[nh1 + c * N + row0 + (uint32_t)b * ng0 + s], f);
  }
  // energy rows (element-owned): the column sums go through sO once the velocity is done
  __syncthreads();
  if (active) {
#pragma unroll
    for (int bl = 0; bl < L1D; ++bl)
#pragma unroll
      for (int al = 0; al < L1D; ++al) sO[lane][bl * L1D + al] = sBLt[qx][al] * TL[bl];
  }
  __syncthreads();
#pragma unroll 1
  for (int i = lane; i < E * NLD; i += 64) {
    const int zz = i / NLD, t = i % NLD;
    double o = 0;
#pragma unroll
    for (int q = 0; q < Q1D; ++q) o += sO[zz * Q1D + q][t];
    r[2 * nh1 + ebase * NLD + i] = o;
  }
}

// ---- host side ---------------------------------------------------------------------------
bool res2d_available(const ilh_ctx* c) {
  return c->dim == 2 && (c->k == 2 || c->k == 3) && !c->kp.visc && c->nblock < (int64_t(1) << 28);
}

template <int K, int SRC>
static void res_t(ilh_ctx* c, const double* k, const double* u, double tau, double* r) {
  constexpr int D1D = K + 1, Q1D = 2 * K, EPW = 64 / Q1D;
  Tab2<double, D1D, Q1D> tb;
  for (int q = 0; q < Q1D; ++q) {
    for (int d = 0; d < D1D; ++d) {
      tb.B[q][d] = c->h_B[q * D1D + d];
      tb.G[q][d] = c->h_G[q * D1D + d];
    }
    for (int d = 0; d < D1D - 1; ++d) tb.BL[q][d] = c->h_BL[q * (D1D - 1) + d];
    tb.W[q] = c->h_w1[q];
  }
  const dim3 grid((c->n[0] + EPW - 1) / EPW, c->n[1]);
  klaunch(c, k_res2d<D1D, Q1D, SRC>, grid, dim3(64), 0, c->kp, tb, u, k, tau, r);
}

// r = R(k; u, tau); the velocity rows of r must be zero on entry
int launch_res2d(ilh_ctx* c, const double* k, const double* u, double tau, double* r) {
  if (!res2d_available(c)) return ILH_EINVAL;
  const int code = 2 * c->k + (c->kp.tg_source ? 1 : 0);
  switch (code) {
    case 4: res_t<2, 0>(c, k, u, tau, r); break;
    case 5: res_t<2, 1>(c, k, u, tau, r); break;
    case 6: res_t<3, 0>(c, k, u, tau, r); break;
    case 7: res_t<3, 1>(c, k, u, tau, r); break;
    default: return ILH_EINVAL;
  }
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

}  // namespace ilh

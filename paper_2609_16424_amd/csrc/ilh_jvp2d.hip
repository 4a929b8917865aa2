// Register-resident 2D Jacobian-action kernel (the hot loop of the Newton-Krylov solve).
//
// Same operator as the M_JVP mode of the generic element kernel (eq. pa_jac_action applied
// to the stage residual), organised for CDNA4 wave64 execution:
//  * one work-group = one wave of 64 lanes = EPW consecutive elements of one element row;
//    lane (z, qx) owns quadrature column qx of element z and walks the column's Q1D points;
//  * gather: the D1D node rows shared by the EPW elements are loaded as contiguous strips
//    (consecutive lanes -> consecutive nodes), so every shared node is read once per block;
//  * xi-contractions of all 8 field components are kept in registers; the eta direction is
//    unrolled with the 1D tables in kernel arguments (scalar registers);
//  * the transposed contractions accumulate in registers; one LDS exchange combines the
//    Q1D column contributions of each element before the atomic scatter;
//  * the quadrature mass is factorised on the affine initial mesh:
//    m_q = (rho0 |J0|)_e w_qx w_qy, so no per-point data is read.
#include <hip/hip_runtime.h>

#include "ilh_internal.h"
#include "ilh_pointwise.h"

namespace ilh {

template <int D1D, int Q1D, typename T, int VISC, int SRC>
__global__ void __launch_bounds__(64) k_jvp2d(const KParams P, const Tab2<T, D1D, Q1D> tb, const EArgs<T> A) {
  constexpr int K = D1D - 1, L1D = K, NLD = L1D * L1D;
  constexpr int EPW = 64 / Q1D;
  constexpr int NS = K * EPW + 1;           // strip width (nodes along x)
  constexpr int NOUT = 2 * D1D * D1D + NLD; // outputs per element
  constexpr int NOP = NOUT | 1;             // odd LDS row length (bank spread)

  __shared__ double sX[2][D1D][NS];         // positions (FP64)
  __shared__ T sS[6][D1D][NS];              // v0 v1 dkx0 dkx1 dkv0 dkv1
  __shared__ T sE[2][EPW * NLD];            // e, dk_e
  __shared__ T sO[64][NOP];                 // per-lane output contributions
  __shared__ T sBG[2][Q1D][D1D];            // B, G (lane-indexed reads in the reduction)
  __shared__ T sBLt[Q1D][L1D];

  const int lane = threadIdx.x;
  const int ey = blockIdx.y, ex0 = blockIdx.x * EPW;
  const int nx = P.n[0];
  const int E = min(EPW, nx - ex0);
  const int ns = K * E + 1;
  const int64_t ng0 = P.ng[0];
  const int64_t N = P.N, nh1 = 2 * P.N;
  const T tau = T(A.tau);

  // strips: x0 x1 (FP64) and v0 v1 dkx0 dkx1 dkv0 dkv1 (T).  All global loads of a lane are
  // issued before any LDS store so their latencies overlap.
  constexpr int NXS = 2 * D1D * NS, NTS = 6 * D1D * NS, NLS = 2 * EPW * NLD;
  constexpr int RX = (NXS + 63) / 64, RT = (NTS + 63) / 64, RL = (NLS + 63) / 64;
  const int64_t ebase = (int64_t)ey * nx + ex0;
  double xr[RX];
  T tr[RT], lr[RL];
#pragma unroll
  for (int r = 0; r < RX; ++r) {
    const int i = lane + 64 * r, si = i % NS, t = i / NS, b = t % D1D, f = t / D1D;
    xr[r] = 0.0;
    if (i < NXS && si < ns) xr[r] = A.x[f * N + (int64_t)(K * ey + b) * ng0 + (int64_t)K * ex0 + si];
  }
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int i = lane + 64 * r, si = i % NS, t = i / NS, b = t % D1D, f = t / D1D;
    tr[r] = T(0);
    if (i < NTS && si < ns) {
      const int64_t node = (int64_t)(K * ey + b) * ng0 + (int64_t)K * ex0 + si;
      const T* src = (f < 2) ? A.v + f * N : (f < 4 ? A.dk + (f - 2) * N : A.dk + nh1 + (f - 4) * N);
      tr[r] = src[node];
    }
  }
#pragma unroll
  for (int r = 0; r < RL; ++r) {
    const int i = lane + 64 * r, f = i / (EPW * NLD), j = i % (EPW * NLD);
    lr[r] = T(0);
    if (i < NLS && j < E * NLD) lr[r] = f == 0 ? A.e[ebase * NLD + j] : A.dk[2 * nh1 + ebase * NLD + j];
  }
  // per-element material data of this lane's element (loaded with the strips)
  const int zl = lane / Q1D;
  const int64_t el = ebase + (zl < E ? zl : 0);
  const double gam_l = P.gamma[el], rj_l = P.rj0[el], j0_l = P.j0e[el];
  for (int i = lane; i < Q1D * D1D; i += 64) {
    sBG[0][i / D1D][i % D1D] = tb.B[i / D1D][i % D1D];
    sBG[1][i / D1D][i % D1D] = tb.G[i / D1D][i % D1D];
  }
  for (int i = lane; i < Q1D * L1D; i += 64) sBLt[i / L1D][i % L1D] = tb.BL[i / L1D][i % L1D];
#pragma unroll
  for (int r = 0; r < RX; ++r) {
    const int i = lane + 64 * r;
    if (i < NXS) (&sX[0][0][0])[i] = xr[r];
  }
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int i = lane + 64 * r;
    if (i < NTS) (&sS[0][0][0])[i] = tr[r];
  }
#pragma unroll
  for (int r = 0; r < RL; ++r) {
    const int i = lane + 64 * r;
    if (i < NLS) (&sE[0][0])[i] = lr[r];
  }
  __syncthreads();

  const int z = lane / Q1D, qx = lane - z * Q1D;
  const bool active = z < E;
  if (!active) {
    for (int t = 0; t < NOUT; ++t) sO[lane][t] = T(0);
  } else {
    const int s0 = K * z;
    const int64_t e = ebase + z;
    T Bq[D1D], Gq[D1D], BLq[L1D];
#pragma unroll
    for (int a = 0; a < D1D; ++a) {
      Bq[a] = sBG[0][qx][a];
      Gq[a] = sBG[1][qx][a];
    }
#pragma unroll
    for (int a = 0; a < L1D; ++a) BLq[a] = sBLt[qx][a];
    const double anc0 = sX[0][0][s0], anc1 = sX[1][0][s0];
    // xi-contractions: AB[f][b] = sum_a B(qx,a) X_f(a,b), AG likewise with G
    T AB[8][D1D], AG[8][D1D];
#pragma unroll
    for (int f = 0; f < 8; ++f)
#pragma unroll
      for (int b = 0; b < D1D; ++b) {
        T ab = 0, ag = 0;
#pragma unroll
        for (int a = 0; a < D1D; ++a) {
          T xv;
          if (f == 0) xv = T(sX[0][b][s0 + a] - anc0);
          else if (f == 1) xv = T(sX[1][b][s0 + a] - anc1);
          else xv = sS[f - 2][b][s0 + a];
          ab += Bq[a] * xv;
          ag += Gq[a] * xv;
        }
        AB[f][b] = ab;
        AG[f][b] = ag;
      }
    T ALe[L1D], ALd[L1D];
#pragma unroll
    for (int bl = 0; bl < L1D; ++bl) {
      T a0 = 0, a1 = 0;
#pragma unroll
      for (int al = 0; al < L1D; ++al) {
        a0 += BLq[al] * sE[0][z * NLD + al + L1D * bl];
        a1 += BLq[al] * sE[1][z * NLD + al + L1D * bl];
      }
      ALe[bl] = a0;
      ALd[bl] = a1;
    }
    const T gam = T(gam_l);
    const T rj = T(rj_l);
    const T dJ0 = T(j0_l);
    constexpr bool src = SRC != 0;
    T T0[2][D1D], T1[2][D1D], TL[L1D];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int b = 0; b < D1D; ++b) T0[c][b] = T1[c][b] = T(0);
#pragma unroll
    for (int bl = 0; bl < L1D; ++bl) TL[bl] = T(0);
    const T wx = tb.W[qx] * rj;
#pragma unroll 1
    for (int qy = 0; qy < Q1D; ++qy) {
      T Jm[2][2], Gv[2][2], dJ[2][2], dGv[2][2], dkv[2];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        T j0 = 0, j1 = 0, g0 = 0, g1 = 0, d0 = 0, d1 = 0, h0 = 0, h1 = 0, mv = 0;
#pragma unroll
        for (int b = 0; b < D1D; ++b) {
          const T By = tb.B[qy][b], Gy = tb.G[qy][b];
          j0 += By * AG[c][b];
          j1 += Gy * AB[c][b];
          g0 += By * AG[2 + c][b];
          g1 += Gy * AB[2 + c][b];
          d0 += By * AG[4 + c][b];
          d1 += Gy * AB[4 + c][b];
          h0 += By * AG[6 + c][b];
          h1 += Gy * AB[6 + c][b];
          mv += By * AB[6 + c][b];
        }
        Jm[c][0] = j0;
        Jm[c][1] = j1;
        Gv[c][0] = g0;
        Gv[c][1] = g1;
        dJ[c][0] = tau * d0;
        dJ[c][1] = tau * d1;
        dGv[c][0] = tau * h0;
        dGv[c][1] = tau * h1;
        dkv[c] = mv;
      }
      T eq = 0, dke = 0;
#pragma unroll
      for (int bl = 0; bl < L1D; ++bl) {
        eq += tb.BL[qy][bl] * ALe[bl];
        dke += tb.BL[qy][bl] * ALd[bl];
      }
      const T mq = wx * tb.W[qy];
      T dS[2][2], ds;
      qp_tangent<2, T, VISC>(P, gam, mq, dJ0, Jm, Gv, eq, dJ, dGv, tau * dke, dS, ds);
      T cl = mq * dke - ds;
      if constexpr (src) {
        T xq0 = 0, xq1 = 0, dx0 = 0, dx1 = 0;
#pragma unroll
        for (int b = 0; b < D1D; ++b) {
          const T By = tb.B[qy][b];
          xq0 += By * AB[0][b];
          xq1 += By * AB[1][b];
          dx0 += By * AB[4][b];
          dx1 += By * AB[5][b];
        }
        T gx, gy;
        tg_source_grad<T>(T(anc0 + double(xq0)), T(anc1 + double(xq1)), gam, gx, gy);
        cl -= mq * tau * (gx * dx0 + gy * dx1);
      }
#pragma unroll
      for (int b = 0; b < D1D; ++b) {
        const T By = tb.B[qy][b], Gy = tb.G[qy][b];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          T0[c][b] += By * dS[c][0];
          T1[c][b] += Gy * dS[c][1] + By * (mq * dkv[c]);
        }
      }
#pragma unroll
      for (int bl = 0; bl < L1D; ++bl) TL[bl] += tb.BL[qy][bl] * cl;
    }
    // contributions of this column to every output of the element
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int b = 0; b < D1D; ++b)
#pragma unroll
        for (int a = 0; a < D1D; ++a) sO[lane][c * D1D * D1D + b * D1D + a] = Gq[a] * T0[c][b] + Bq[a] * T1[c][b];
#pragma unroll
    for (int bl = 0; bl < L1D; ++bl)
#pragma unroll
      for (int al = 0; al < L1D; ++al) sO[lane][2 * D1D * D1D + bl * L1D + al] = BLq[al] * TL[bl];
  }
  __syncthreads();
  // combine the Q1D columns of each element and scatter
  if (active) {
    const int ex = ex0 + z;
    const int64_t e = ebase + z;
    for (int t = qx; t < NOUT; t += Q1D) {
      T o = 0;
#pragma unroll
      for (int q = 0; q < Q1D; ++q) o += sO[z * Q1D + q][t];
      if (t < 2 * D1D * D1D) {
        const int c = t / (D1D * D1D), r = t % (D1D * D1D), b = r / D1D, a = r % D1D;
        const int I = K * ex + a, J = K * ey + b;
        const bool cons = (c == 0) ? (I == 0 || I == P.ng[0] - 1) : (J == 0 || J == P.ng[1] - 1);
        if (!cons) unsafeAtomicAdd(&A.out[nh1 + c * N + (int64_t)J * ng0 + I], o);
      } else {
        A.out[2 * nh1 + e * NLD + (t - 2 * D1D * D1D)] = o;
      }
    }
  }
  // position rows (dk_x - tau dk_v) and constrained velocity rows (dk_v), by node owner
  const bool last_x = (ex0 + E == nx), last_y = (ey == P.n[1] - 1);
  for (int i = lane; i < 2 * D1D * NS; i += 64) {
    const int s = i % NS, t = i / NS, b = t % D1D, c = t / D1D;
    if (s >= ns) continue;
    if (!((s < K * E || last_x) && (b < K || last_y))) continue;
    const int I = K * ex0 + s, J = K * ey + b;
    const int64_t gi = c * N + (int64_t)J * ng0 + I;
    const T dkx = sS[2 + c][b][s], dkv = sS[4 + c][b][s];
    A.out[gi] = dkx - tau * dkv;
    const bool cons = (c == 0) ? (I == 0 || I == P.ng[0] - 1) : (J == 0 || J == P.ng[1] - 1);
    if (cons) unsafeAtomicAdd(&A.out[nh1 + gi], dkv);
  }
}

template <int K, typename T>
static int launch_jvp2d_t(ilh_ctx* c, const EArgs<T>& a) {
  constexpr int D1D = K + 1, Q1D = 2 * K, EPW = 64 / Q1D;
  Tab2<T, D1D, Q1D> tb;
  for (int q = 0; q < Q1D; ++q) {
    for (int d = 0; d < D1D; ++d) {
      tb.B[q][d] = T(c->h_B[q * D1D + d]);
      tb.G[q][d] = T(c->h_G[q * D1D + d]);
    }
    for (int d = 0; d < K; ++d) tb.BL[q][d] = T(c->h_BL[q * K + d]);
    tb.W[q] = T(c->h_w1[q]);
  }
  dim3 grid((c->n[0] + EPW - 1) / EPW, c->n[1]);
  const int visc = c->kp.visc ? 1 : 0, src = c->kp.tg_source ? 1 : 0;
  if (visc && src)
    klaunch(c, k_jvp2d<D1D, Q1D, T, 1, 1>, grid, dim3(64), 0, c->kp, tb, a);
  else if (visc)
    klaunch(c, k_jvp2d<D1D, Q1D, T, 1, 0>, grid, dim3(64), 0, c->kp, tb, a);
  else if (src)
    klaunch(c, k_jvp2d<D1D, Q1D, T, 0, 1>, grid, dim3(64), 0, c->kp, tb, a);
  else
    klaunch(c, k_jvp2d<D1D, Q1D, T, 0, 0>, grid, dim3(64), 0, c->kp, tb, a);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

// Returns ILH_EINVAL when no specialised kernel exists (the caller then uses the generic one).
int launch_jvp2d(ilh_ctx* c, int prec, const EArgs<double>* a64, const EArgs<float>* a32) {
  if (c->dim != 2) return ILH_EINVAL;
  if (prec == 64) {
    switch (c->k) {
      case 2: return launch_jvp2d_t<2, double>(c, *a64);
      case 3: return launch_jvp2d_t<3, double>(c, *a64);
    }
  } else {
    switch (c->k) {
      case 2: return launch_jvp2d_t<2, float>(c, *a32);
      case 3: return launch_jvp2d_t<3, float>(c, *a32);
    }
  }
  return ILH_EINVAL;
}

}  // namespace ilh

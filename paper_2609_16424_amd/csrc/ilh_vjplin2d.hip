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
  lds_barrier();

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

  vm_drained();  // every load is consumed and no store is issued yet

  // H1 rows, position part then velocity part: per-lane contributions to sO, node sums over the
  // (one or two) elements of the strip holding the node, the owner's identity terms, one atomic
  // add per node.  Lane gs of node group g takes node gs of the rows (component g, node row p):
  // per-lane LDS bases plus per-pass constants, all LDS reads issued before the first sum.
  constexpr int GS = NS <= 32 ? 32 : 64, NG = 64 / GS, PN = 2 * D1D / NG;
  int tn = lane % GS, gn = lane / GS;
  asm volatile("" : "+v"(tn), "+v"(gn));
  const int lc = NG == 1 ? 0 : gn;
  const int zz = tn / K, a = tn - K * zz, sc = min(tn, ns - 1);
  const bool left = zz < E, shared = a == 0 && zz > 0;
  const int oR = min(zz, E - 1) * Q1D * NOP + lc * D1D * D1D + a;
  int oL = max(zz - 1, 0) * Q1D * NOP + lc * D1D * D1D + K;
  asm volatile("" : "+v"(oL));
  const int oS = lc * D1D * NS + sc;
  const uint32_t I = K * ex0 + tn;
  const bool consI = lc == 0 && (I == 0 || I == ng0 - 1), isv = lc != 0, own_s = tn < K * E || last_x;
  const uint32_t gb = (uint32_t)lc * N + row0 + (uint32_t)sc;
  const T* const sOf = &sO[0][0];
  const T* const sSf = &sS[0][0][0];
#pragma unroll
  for (int part = 0; part < 2; ++part) {
    if (active) {
      T Bq[D1D], Gq[D1D];
#pragma unroll
      for (int a2 = 0; a2 < D1D; ++a2) {
        Bq[a2] = sBG[0][qx][a2];
        Gq[a2] = sBG[1][qx][a2];
      }
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < D1D; ++b)
#pragma unroll
          for (int a2 = 0; a2 < D1D; ++a2)
            sO[lane][c * D1D * D1D + b * D1D + a2] =
                part == 0 ? Gq[a2] * X0[c][b] + Bq[a2] * X1[c][b] : Gq[a2] * V0[c][b] + Bq[a2] * V1[c][b];
    }
    lds_barrier();
    // constrained velocity rows: the owner adds y_v (zeroed in the strips), read up front
    T yc[PN];
    if (part == 1) {
#pragma unroll
      for (int p = 0; p < PN; ++p) {
        const int cp = NG == 1 ? (p & 1) : 0, bp = NG == 1 ? (p >> 1) : p;
        yc[p] = ld32(y, nh1 + gb + (uint32_t)cp * N + (uint32_t)bp * ng0);
      }
    }
    T fv[PN], yx[PN];
#pragma unroll
    for (int p = 0; p < PN; ++p) {
      const int cp = NG == 1 ? (p & 1) : 0, bp = NG == 1 ? (p >> 1) : p;
      const int po = cp * D1D * D1D + bp * D1D;
      T f0 = sOf[oR + po], f1 = sOf[oL + po];
#pragma unroll
      for (int q = 1; q < Q1D; ++q) {
        f0 += sOf[oR + po + q * NOP];
        f1 += sOf[oL + po + q * NOP];
      }
      fv[p] = (left ? f0 : T(0)) + (shared ? f1 : T(0));
      yx[p] = sSf[oS + (cp * D1D + bp) * NS];
    }
    if (tn < ns) {
#pragma unroll
      for (int p = 0; p < PN; ++p) {
        const int cp = NG == 1 ? (p & 1) : 0, bp = NG == 1 ? (p >> 1) : p;
        const int b = bp;
        const bool own = own_s && (b < K || last_y);
        T f = fv[p];
        if (part == 0) {
          if (own) f += yx[p];
        } else {
          const uint32_t J = K * ey + b;
          const bool consJ = J == 0 || J == ng1 - 1;
          const bool cons = NG == 1 ? (cp == 0 ? (I == 0 || I == ng0 - 1) : consJ) : (consI || (isv && consJ));
          if (own) f -= tau * yx[p];
          if (own && cons) f += yc[p];
        }
        atomic_add32(out, part * nh1 + gb + (uint32_t)cp * N + (uint32_t)bp * ng0, f);
      }
    }
    lds_barrier();
  }
  // energy rows (element-owned)
  if (active) {
#pragma unroll
    for (int bl = 0; bl < L1D; ++bl)
#pragma unroll
      for (int al = 0; al < L1D; ++al) sO[lane][bl * L1D + al] = sBLt[qx][al] * TL[bl];
  }
  lds_barrier();
  constexpr int NE = (NLS + 63) / 64;
  T ev[NE];
#pragma unroll
  for (int it = 0; it < NE; ++it) {
    const int i = min(lane + 64 * it, E * NLD - 1), ze = i / NLD, t = i % NLD;
    T o = sO[ze * Q1D][t];
#pragma unroll
    for (int q = 1; q < Q1D; ++q) o += sO[ze * Q1D + q][t];
    ev[it] = o;
  }
#pragma unroll
  for (int it = 0; it < NE; ++it) {
    const int i = lane + 64 * it;
    if (i < E * NLD) st32(out, 2 * nh1 + ebase * NLD + i, ev[it]);
  }
}

// ---- 3D, Q2Q1: the transpose of k_jvp3d_q ------------------------------------------------
// One wave = EPW = 4 consecutive elements of an element row, lane (element, q_x, q_y) owns a
// quadrature column and walks q_z, as in the 3D forward kernels; the coefficients are read in
// the layout k_lin3d stores them (row-interleaved in FP32, field-major in FP64).
template <int D1D, int Q1D, typename T, int VISC>
__global__ void __launch_bounds__(64) k_vjp3d_q(const KParams P, const Tab2<T, D1D, Q1D> tb,
                                                const T* __restrict__ y, const T* __restrict__ qd, int64_t qs,
                                                double tau_, T* __restrict__ out) {
  constexpr int K = D1D - 1, L1D = K, NLD = L1D * L1D * L1D;
  constexpr int LPE = Q1D * Q1D, EPW = 64 / LPE;
  constexpr int NS = K * EPW + 1;
  constexpr int NQD = LinLayout<3, VISC, 0>::NQD;
  constexpr int NF = 6;  // y_x0 y_x1 y_x2, y~_v0 y~_v1 y~_v2 (constrained velocity rows zeroed)
  constexpr int NND = D1D * D1D * D1D;
  constexpr int NOP = (NND > NLD ? NND : NLD) | 1;

  __shared__ T sS[NF][D1D][D1D][NS];
  __shared__ T sE[EPW * NLD];
  __shared__ T sO[64][NOP];
  __shared__ T sBG[2][Q1D][D1D];
  __shared__ T sBL[Q1D][L1D];

  const int lane = threadIdx.x;
  const uint32_t tile = xcd_tile((blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x,
                                 gridDim.x * gridDim.y * gridDim.z);
  const int ex0 = (tile % gridDim.x) * EPW, ey = (tile / gridDim.x) % gridDim.y, ez = tile / (gridDim.x * gridDim.y);
  const int nx = P.n[0], ny = P.n[1];
  const int E = min(EPW, nx - ex0);
  const int ns = K * E + 1;
  const uint32_t ng0 = P.ng[0], ng1 = P.ng[1], ng2 = P.ng[2], ng01 = ng0 * ng1;
  const uint32_t N = (uint32_t)P.N, nh1 = 3 * N;
  const uint32_t ebase = ((uint32_t)ez * ny + ey) * nx + ex0;
  const uint32_t row0 = (uint32_t)(K * ez) * ng01 + (uint32_t)(K * ey) * ng0 + (uint32_t)(K * ex0);
  const T tau = T(tau_);

  constexpr int NTS = NF * D1D * D1D * NS, RT = (NTS + 63) / 64;
  constexpr int NLS = EPW * NLD, RL = (NLS + 63) / 64;
  T tr[RT], lr[RL];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int i = lane + 64 * r, s = min(i % NS, ns - 1), t = min(i / NS, NF * D1D * D1D - 1), b = t % D1D,
              cz = (t / D1D) % D1D, f = t / (D1D * D1D);
    const T v = ld32(y, (f < 3 ? f * N : nh1 + (f - 3) * N) + row0 + (uint32_t)cz * ng01 + (uint32_t)b * ng0 + s);
    const uint32_t I = K * ex0 + s, J = K * ey + b, Kz = K * ez + cz;
    const uint32_t idx = f == 3 ? I : (f == 4 ? J : Kz), ngf = f == 3 ? ng0 : (f == 4 ? ng1 : ng2);
    tr[r] = (f >= 3 && (idx == 0 || idx == ngf - 1)) ? T(0) : v;
  }
#pragma unroll
  for (int r = 0; r < RL; ++r) lr[r] = ld32(y, 2 * nh1 + ebase * NLD + min(lane + 64 * r, E * NLD - 1));
  const int zl = lane / LPE;
  const double rj_l = P.rj0[ebase + (zl < E ? zl : 0)];
  for (int i = lane; i < Q1D * D1D; i += 64) {
    sBG[0][i / D1D][i % D1D] = tb.B[i / D1D][i % D1D];
    sBG[1][i / D1D][i % D1D] = tb.G[i / D1D][i % D1D];
  }
  for (int i = lane; i < Q1D * L1D; i += 64) sBL[i / L1D][i % L1D] = tb.BL[i / L1D][i % L1D];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int i = lane + 64 * r;
    if (i < NTS) (&sS[0][0][0][0])[i] = tr[r];
  }
#pragma unroll
  for (int r = 0; r < RL; ++r) {
    const int i = lane + 64 * r;
    if (i < NLS) sE[i] = lr[r];
  }
  lds_barrier();

  const int z = lane / LPE, rr = lane - z * LPE, qy = rr / Q1D, qx = rr - qy * Q1D;
  const bool active = z < E;
  // per-lane sums over the column for the position (X*) and velocity (V*) rows: coefficients of
  // G_x B_y (x), B_x G_y (y), B_x B_y (z: derivative along z plus the value terms) per layer
  T Xx[3][D1D], Xy[3][D1D], Xz[3][D1D], Vx[3][D1D], Vy[3][D1D], Vz[3][D1D], TL[L1D];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < D1D; ++c) Xx[r][c] = Xy[r][c] = Xz[r][c] = Vx[r][c] = Vy[r][c] = Vz[r][c] = T(0);
#pragma unroll
  for (int cl = 0; cl < L1D; ++cl) TL[cl] = T(0);
  if (active) {
    const int s0 = K * z;
    T Bx[D1D], Gx[D1D], By[D1D], Gy[D1D];
#pragma unroll
    for (int a = 0; a < D1D; ++a) {
      Bx[a] = sBG[0][qx][a];
      Gx[a] = sBG[1][qx][a];
      By[a] = sBG[0][qy][a];
      Gy[a] = sBG[1][qy][a];
    }
    T BB[3][D1D], GB[3][D1D], BG[3][D1D];
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
      for (int cz = 0; cz < D1D; ++cz) {
        T bb = 0, gb = 0, bg = 0;
#pragma unroll
        for (int b = 0; b < D1D; ++b) {
          T ab = 0, ag = 0;
#pragma unroll
          for (int a = 0; a < D1D; ++a) {
            const T xv = sS[3 + f][cz][b][s0 + a];
            ab += Bx[a] * xv;
            ag += Gx[a] * xv;
          }
          bb += By[b] * ab;
          gb += By[b] * ag;
          bg += Gy[b] * ab;
        }
        BB[f][cz] = bb;
        GB[f][cz] = gb;
        BG[f][cz] = bg;
      }
    T EL[L1D];
#pragma unroll
    for (int cl = 0; cl < L1D; ++cl) {
      T acc = 0;
#pragma unroll
      for (int bl = 0; bl < L1D; ++bl)
#pragma unroll
        for (int al = 0; al < L1D; ++al)
          acc += sBL[qy][bl] * sBL[qx][al] * sE[z * NLD + al + L1D * (bl + L1D * cl)];
      EL[cl] = acc;
    }
    const T wxy = tb.W[qx] * tb.W[qy] * T(rj_l);
    constexpr bool ROWS = sizeof(T) == 4;
    const T* __restrict__ qb = qd + (int64_t)tile * (Q1D * (ROWS ? NQD : 1) * 64);
#pragma unroll 1
    for (int qz = 0; qz < Q1D; ++qz) {
      T cf[NQD];
      if constexpr (ROWS) {
        const T* rb = sbase(qb + qz * (NQD * 64));
#pragma unroll
        for (int f = 0; f < NQD; ++f) cf[f] = ld32(rb, (uint32_t)(f * 64 + lane));
      } else {
#pragma unroll
        for (int f = 0; f < NQD; ++f) cf[f] = ld32(sbase(qb + f * qs), (uint32_t)(qz * 64 + lane));
      }
      T A[3][3], yv[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        T a0 = 0, a1 = 0, a2 = 0, m = 0;
#pragma unroll
        for (int c = 0; c < D1D; ++c) {
          const T Bz = tb.B[qz][c], Gz = tb.G[qz][c];
          a0 += Bz * GB[r][c];
          a1 += Bz * BG[r][c];
          a2 += Gz * BB[r][c];
          m += Bz * BB[r][c];
        }
        A[r][0] = a0;
        A[r][1] = a1;
        A[r][2] = a2;
        yv[r] = m;
      }
      T ye = 0;
#pragma unroll
      for (int cl = 0; cl < L1D; ++cl) ye += tb.BL[qz][cl] * EL[cl];
      const T mq = wxy * tb.W[qz];
      T GJ[3][3], GGv[3][3], ge;
      lin_apply_t<3, T, VISC>(cf, A, -ye, GJ, GGv, ge);
#pragma unroll
      for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int c = 0; c < D1D; ++c) {
          const T Bz = tb.B[qz][c], Gz = tb.G[qz][c];
          Xx[r][c] += Bz * GJ[r][0];
          Xy[r][c] += Bz * GJ[r][1];
          Xz[r][c] += Gz * GJ[r][2];
          Vx[r][c] += Bz * GGv[r][0];
          Vy[r][c] += Bz * GGv[r][1];
          Vz[r][c] += Gz * GGv[r][2] + Bz * (mq * yv[r]);
        }
      }
      const T te = ge + mq * ye;
#pragma unroll
      for (int cl = 0; cl < L1D; ++cl) TL[cl] += tb.BL[qz][cl] * te;
    }
  }
  // H1 rows (position part, then velocity part), one component at a time: factored expansion of
  // each lane's column sums into sO, node sums over the (one or two) elements of the strip
  // holding the node, the owner's identity terms, one atomic per node and strip
  const T Bxl[D1D] = {sBG[0][qx][0], sBG[0][qx][1], sBG[0][qx][2]};
  const T Gxl[D1D] = {sBG[1][qx][0], sBG[1][qx][1], sBG[1][qx][2]};
  const T Byl[D1D] = {sBG[0][qy][0], sBG[0][qy][1], sBG[0][qy][2]};
  const T Gyl[D1D] = {sBG[1][qy][0], sBG[1][qy][1], sBG[1][qy][2]};
  const bool last_x = (ex0 + E == nx), last_y = (ey == ny - 1), last_z = (ez == P.n[2] - 1);
#pragma unroll 1
  for (int pr = 0; pr < 6; ++pr) {
    const int part = pr / 3, r = pr % 3;
    if (active) {
#pragma unroll
      for (int cz = 0; cz < D1D; ++cz) {
        T tx = 0, ty = 0, tzv = 0;
#pragma unroll
        for (int rq = 0; rq < 3; ++rq)
          if (rq == r) {
            tx = part == 0 ? Xx[rq][cz] : Vx[rq][cz];
            ty = part == 0 ? Xy[rq][cz] : Vy[rq][cz];
            tzv = part == 0 ? Xz[rq][cz] : Vz[rq][cz];
          }
#pragma unroll
        for (int a = 0; a < D1D; ++a) {
          const T q1 = Gxl[a] * tx + Bxl[a] * tzv, q2 = Bxl[a] * ty;
#pragma unroll
          for (int b = 0; b < D1D; ++b) sO[lane][(cz * D1D + b) * D1D + a] = Byl[b] * q1 + Gyl[b] * q2;
        }
      }
    }
    lds_barrier();
    for (int i = lane; i < D1D * D1D * NS; i += 64) {
      const int s = i % NS, t = i / NS, b = t % D1D, cz = t / D1D;
      if (s >= ns) continue;
      const int zz = s / K, a = s - K * zz;
      T o = 0;
      if (zz < E) {
#pragma unroll
        for (int q = 0; q < LPE; ++q) o += sO[zz * LPE + q][(cz * D1D + b) * D1D + a];
      }
      if (a == 0 && zz > 0) {
#pragma unroll
        for (int q = 0; q < LPE; ++q) o += sO[(zz - 1) * LPE + q][(cz * D1D + b) * D1D + K];
      }
      const uint32_t gi = r * N + row0 + cz * ng01 + b * ng0 + s;
      const bool own = (s < K * E || last_x) && (b < K || last_y) && (cz < K || last_z);
      if (own) {
        const T yx = sS[r][cz][b][s];
        if (part == 0) {
          o += yx;
        } else {
          o -= tau * yx;
          const uint32_t I = K * ex0 + s, J = K * ey + b, Kz = K * ez + cz;
          const uint32_t idx = r == 0 ? I : (r == 1 ? J : Kz), ngr = r == 0 ? ng0 : (r == 1 ? ng1 : ng2);
          if (idx == 0 || idx == ngr - 1) o += y[nh1 + gi];
        }
      }
      unsafeAtomicAdd(&out[part * nh1 + gi], o);
    }
    lds_barrier();
  }
  // energy rows (element-owned)
  if (active) {
#pragma unroll
    for (int cl = 0; cl < L1D; ++cl)
#pragma unroll
      for (int bl = 0; bl < L1D; ++bl)
#pragma unroll
        for (int al = 0; al < L1D; ++al) sO[lane][al + L1D * (bl + L1D * cl)] = sBL[qx][al] * sBL[qy][bl] * TL[cl];
  }
  lds_barrier();
  if (active) {
    for (int t = rr; t < NLD; t += LPE) {
      T o = 0;
#pragma unroll
      for (int q = 0; q < LPE; ++q) o += sO[z * LPE + q][t];
      out[2 * nh1 + (ebase + z) * NLD + t] = o;
    }
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

template <typename T>
static int dispatch_vjp3(ilh_ctx* c, const T* y, const T* qd, T* out) {
  constexpr int EPW = 4;
  const dim3 g((c->n[0] + EPW - 1) / EPW, c->n[1], c->n[2]);
  const int64_t qs = (int64_t)g.x * g.y * g.z * 4 * 64;
  if (c->kp.visc)
    klaunch(c, k_vjp3d_q<3, 4, T, 1>, g, dim3(64), 0, c->kp, vjp_tab2<T, 3, 4>(c), y, qd, qs, c->lin_tau, out);
  else
    klaunch(c, k_vjp3d_q<3, 4, T, 0>, g, dim3(64), 0, c->kp, vjp_tab2<T, 3, 4>(c), y, qd, qs, c->lin_tau, out);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

// Transpose action with the stored coefficients of precision prec (they must be current).
int launch_vjp3d_q(ilh_ctx* c, int prec, const void* y, void* out) {
  if (!lin3d_available(c)) return ILH_EINVAL;
  const int p = prec == 64 ? 1 : 0;
  if (!c->qd[p] || !c->qd_ok[p]) return fail(c, ILH_EINVAL, "transpose action before its linearisation");
  return p ? dispatch_vjp3<double>(c, (const double*)y, (const double*)c->qd[p], (double*)out)
           : dispatch_vjp3<float>(c, (const float*)y, (const float*)c->qd[p], (float*)out);
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

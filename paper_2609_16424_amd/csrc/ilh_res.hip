// Stage residual (Sec. 4: R(k) of the implicit stage, with the mass-multiplied rows of the
// block preconditioner's reading) on the work-group / lane maps of the linearised kernels.
// 2D (k = 2, 3): one wave = EPW consecutive elements of one element row, lane (z, qx) =
// quadrature column qx of element z, walking the Q1D quadrature rows.  3D (Q2Q1, no TG source):
// see k_res3d.  FP64 throughout; the artificial viscosity enters through qp_force.
//
//   R_x = k_x - w_v                                  (position rows, written by the node's owner)
//   R_v = M_V k_v + F(w) 1                           (constrained velocity rows: R_v = k_v)
//   R_e = M_E k_e - F(w)^T w_v - b(w_x)              (element-owned)
// with w = u + tau k.  Per quadrature point the force S_q (d x d) and s_q = S_q : grad_xi w_v
// come from qp_force, the same pointwise code as the generic kernel; the transposes use the
// factored expansions of the linearised apply; in 2D each velocity row of a strip takes one
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
        const double* __restrict__ kk1, double tau, double* __restrict__ r1, double* __restrict__ dmin1,
        const double* __restrict__ kk2, double* __restrict__ r2) {
  constexpr int K = D1D - 1, L1D = K, NLD = L1D * L1D;
  constexpr int EPW = 64 / Q1D;
  constexpr int NS = K * EPW + 1;
  constexpr int NVO = 2 * D1D * D1D;
  constexpr int NOP = NVO | 1;
  constexpr int NNE = 2 * D1D * NS, RG = (NNE + 63) / 64;  // node entries (c, b, s) of the strip
  constexpr int NLS = EPW * NLD, RL = (NLS + 63) / 64;

  // The gathered strips are read by the xi-contractions only, the per-lane contributions are
  // written after the quadrature rows: one LDS block serves both (the wave's LDS operations
  // complete in program order), which keeps a C2-sized grid resident in one round.
  union StripLds {
    struct {
      double W[6][D1D][NS];  // w_x (2), w_v (2), k_v (2)
      double E[2][NLS];      // w_e, k_e
    } in;
    double O[64][NOP];  // per-lane contributions (velocity, then energy)
  };
  __shared__ StripLds sm;
  auto& sW = sm.in.W;
  auto& sE = sm.in.E;
  auto& sO = sm.O;
  __shared__ double sBG[2][Q1D][D1D];
  __shared__ double sBLt[Q1D][L1D];

  const int lane = threadIdx.x;
  // grid.z = 2: a second residual, R(kk2) into r2, at the same u and tau, by a second set of
  // work-groups (one launch for the two; the XCD map spreads the combined set)
  const uint32_t nt = gridDim.x * gridDim.y;
  const uint32_t tz = xcd_tile((blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x, nt * gridDim.z);
  const bool second = tz >= nt;
  const uint32_t tile = second ? tz - nt : tz;
  const double* __restrict__ kk = second ? kk2 : kk1;
  double* __restrict__ r = second ? r2 : r1;
  double* __restrict__ dmin = second ? nullptr : dmin1;
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
  lds_barrier();

  double TL[L1D];
#pragma unroll
  for (int bl = 0; bl < L1D; ++bl) TL[bl] = 0.0;
  double dm = 1e300;  // the lane's smallest det J (dmin set)
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
      if (dmin) dm = nan_min(dm, J[0][0] * J[1][1] - J[0][1] * J[1][0]);
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
    asm volatile("" ::: "memory");  // sO overlays the strips read above: keep the order
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int b = 0; b < D1D; ++b)
#pragma unroll
        for (int a = 0; a < D1D; ++a)
          sO[lane][c * D1D * D1D + b * D1D + a] = Gq[a] * T0[c][b] + Bq[a] * T1[c][b];
  }
  vm_drained();  // every load is consumed; the position-row stores were issued long before
  lds_barrier();
  if (dmin) {  // the work-group's smallest det J of the stage positions w_x
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dm = nan_min(dm, __shfl_xor(dm, o, 64));
    if (lane == 0) dmin[tile] = dm;
  }

  // velocity rows that are not constrained: the Q1D columns of the (one or two) elements of the
  // strip that hold the node, one atomic add per node and strip.  Lane gs of half g takes node
  // gs of the rows (component g, node row p): per-lane LDS bases plus per-pass constants, all
  // LDS reads issued before the first sum.
  {
    constexpr int GS = NS <= 32 ? 32 : 64, NG = 64 / GS, PN = 2 * D1D / NG;
    int tn = lane % GS, gn = lane / GS;
    asm volatile("" : "+v"(tn), "+v"(gn));
    const int lc = NG == 1 ? 0 : gn;
    const int zz = tn / K, a = tn - K * zz;
    const bool left = zz < E, shared = a == 0 && zz > 0;
    const int oR = min(zz, E - 1) * Q1D * NOP + lc * D1D * D1D + a;
    int oL = max(zz - 1, 0) * Q1D * NOP + lc * D1D * D1D + K;
    asm volatile("" : "+v"(oL));
    const double* const sOf = &sO[0][0];
    double fv[PN];
#pragma unroll
    for (int p = 0; p < PN; ++p) {
      const int cp = NG == 1 ? (p & 1) : 0, bp = NG == 1 ? (p >> 1) : p;
      const int po = cp * D1D * D1D + bp * D1D;
      double f0 = sOf[oR + po], f1 = sOf[oL + po];
#pragma unroll
      for (int q = 1; q < Q1D; ++q) {
        f0 += sOf[oR + po + q * NOP];
        f1 += sOf[oL + po + q * NOP];
      }
      fv[p] = (left ? f0 : 0.0) + (shared ? f1 : 0.0);
    }
    const uint32_t I = K * ex0 + tn;
    const bool cI = lc == 0 && (I == 0 || I == ng0 - 1), isv = lc != 0;
    const uint32_t gb = nh1 + (uint32_t)lc * N + row0 + tn;
    if (tn < ns) {
#pragma unroll
      for (int p = 0; p < PN; ++p) {
        const int cp = NG == 1 ? (p & 1) : 0, bp = NG == 1 ? (p >> 1) : p;
        const uint32_t J = K * ey + bp;
        const bool consJ = J == 0 || J == ng1 - 1;
        const bool cons = NG == 1 ? (cp == 0 ? (I == 0 || I == ng0 - 1) : consJ) : (cI || (isv && consJ));
        if (!cons) atomic_add32(r, gb + (uint32_t)cp * N + (uint32_t)bp * ng0, fv[p]);
      }
    }
  }
  // energy rows (element-owned): the column sums go through sO once the velocity is done
  lds_barrier();
  if (active) {
#pragma unroll
    for (int bl = 0; bl < L1D; ++bl)
#pragma unroll
      for (int al = 0; al < L1D; ++al) sO[lane][bl * L1D + al] = sBLt[qx][al] * TL[bl];
  }
  lds_barrier();
  constexpr int NE = (NLS + 63) / 64;
  double ev[NE];
#pragma unroll
  for (int it = 0; it < NE; ++it) {
    const int i = min(lane + 64 * it, E * NLD - 1), zz = i / NLD, t = i % NLD;
    double o = sO[zz * Q1D][t];
#pragma unroll
    for (int q = 1; q < Q1D; ++q) o += sO[zz * Q1D + q][t];
    ev[it] = o;
  }
#pragma unroll
  for (int it = 0; it < NE; ++it) {
    const int i = lane + 64 * it;
    if (i < E * NLD) st32(r, 2 * nh1 + ebase * NLD + i, ev[it]);
  }
}

// ---- 3D, Q2Q1 (no TG source): the lane map of the 3D linearised kernels ---------------------
// One wave = EPW elements of one element row (fixed y, z), lane (z, qy, qx) = quadrature column
// (qx, qy) of element z walking its Q1D points in z.  Each velocity component's element sums go
// through LDS over the element's lanes and take one atomic per node and element.
template <int D1D, int Q1D>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1)))
k_res3d(const KParams P, const Tab2<double, D1D, Q1D> tb, const double* __restrict__ u,
        const double* __restrict__ kk, double tau, double* __restrict__ r, double* __restrict__ dmin) {
  constexpr int K = D1D - 1, L1D = K, NLD = L1D * L1D * L1D;
  constexpr int LPE = Q1D * Q1D, EPW = 64 / LPE;
  constexpr int NS = K * EPW + 1;
  constexpr int NND = D1D * D1D * D1D;
  constexpr int NOP = (NND > NLD ? NND : NLD) | 1;
  constexpr int NNE = 3 * D1D * D1D * NS, RG = (NNE + 63) / 64;  // node entries (c, cz, b, s)
  constexpr int NLS = EPW * NLD, RL = (NLS + 63) / 64;

  __shared__ double sW[9][D1D][D1D][NS];  // w_x (3), w_v (3), k_v (3)
  __shared__ double sE[2][NLS];           // w_e, k_e
  __shared__ double sO[64][NOP];
  __shared__ double sBG[2][Q1D][D1D];
  __shared__ double sBL[Q1D][L1D];

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
  const bool last_x = (ex0 + E == nx), last_y = (ey == ny - 1), last_z = (ez == P.n[2] - 1);
  const int z = lane / LPE, rr = lane - z * LPE, qy = rr / Q1D, qx = rr - qy * Q1D;
  const bool active = z < E;

  for (int i = lane; i < Q1D * D1D; i += 64) {
    sBG[0][i / D1D][i % D1D] = tb.B[i / D1D][i % D1D];
    sBG[1][i / D1D][i % D1D] = tb.G[i / D1D][i % D1D];
  }
  for (int i = lane; i < Q1D * L1D; i += 64) sBL[i / L1D][i % L1D] = tb.BL[i / L1D][i % L1D];

  double gx[RG], gk[RG], gv[RG], gkv[RG];
#pragma unroll
  for (int q = 0; q < RG; ++q) {
    const int i = min(lane + 64 * q, NNE - 1), s = min(i % NS, ns - 1), t = i / NS, b = t % D1D,
              cz = (t / D1D) % D1D, c = t / (D1D * D1D);
    const uint32_t gi = c * N + row0 + (uint32_t)cz * ng01 + (uint32_t)b * ng0 + s;
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
  const uint32_t el = ebase + (active ? z : 0);
  const double rj_l = P.rj0[el], gam = P.gamma[el], dJ0 = P.j0e[el];
#pragma unroll
  for (int q = 0; q < RG; ++q) {
    const int i = lane + 64 * q;
    if (i >= NNE) continue;
    const int s = i % NS, t = i / NS, b = t % D1D, cz = (t / D1D) % D1D, c = t / (D1D * D1D);
    const double wv = gv[q] + tau * gkv[q];
    sW[c][cz][b][s] = gx[q] + tau * gk[q];
    sW[3 + c][cz][b][s] = wv;
    sW[6 + c][cz][b][s] = gkv[q];
    if (s >= ns || !((s < K * E || last_x) && (b < K || last_y) && (cz < K || last_z))) continue;
    // position rows and constrained velocity rows: the node's single owner
    const uint32_t gi = c * N + row0 + (uint32_t)cz * ng01 + (uint32_t)b * ng0 + s;
    r[gi] = gk[q] - wv;
    const uint32_t I = K * ex0 + s, J = K * ey + b, Kz = K * ez + cz;
    const uint32_t idx = c == 0 ? I : (c == 1 ? J : Kz), ngc = c == 0 ? ng0 : (c == 1 ? ng1 : ng2);
    if (idx == 0 || idx == ngc - 1) r[nh1 + gi] = gkv[q];
  }
#pragma unroll
  for (int q = 0; q < RL; ++q) {
    const int i = lane + 64 * q;
    if (i < NLS) {
      sE[0][i] = ge[q] + tau * gke[q];
      sE[1][i] = gke[q];
    }
  }
  lds_barrier();

  double Tx[3][D1D], Ty[3][D1D], Tz[3][D1D], TL[L1D];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int cz = 0; cz < D1D; ++cz) Tx[c][cz] = Ty[c][cz] = Tz[c][cz] = 0.0;
#pragma unroll
  for (int cl = 0; cl < L1D; ++cl) TL[cl] = 0.0;
  double dm = 1e300;  // the lane's smallest det J (dmin set)
  if (active) {
    const int s0 = K * z;
    double Bx[D1D], Gx[D1D], By[D1D], Gy[D1D], BLx[L1D], BLy[L1D];
#pragma unroll
    for (int a = 0; a < D1D; ++a) {
      Bx[a] = sBG[0][qx][a];
      Gx[a] = sBG[1][qx][a];
      By[a] = sBG[0][qy][a];
      Gy[a] = sBG[1][qy][a];
    }
#pragma unroll
    for (int a = 0; a < L1D; ++a) {
      BLx[a] = sBL[qx][a];
      BLy[a] = sBL[qy][a];
    }
    // x-y contractions per z-layer: values BB, x-derivatives GB, y-derivatives BG of w_x and
    // w_v; values of k_v
    double BB[6][D1D], GB[6][D1D], BG[6][D1D], KB[3][D1D];
#pragma unroll
    for (int f = 0; f < 6; ++f)
#pragma unroll
      for (int cz = 0; cz < D1D; ++cz) {
        double bb = 0, gb = 0, bg = 0;
#pragma unroll
        for (int b = 0; b < D1D; ++b) {
          double ab = 0, ag = 0;
#pragma unroll
          for (int a = 0; a < D1D; ++a) {
            const double xv = sW[f][cz][b][s0 + a];
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
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int cz = 0; cz < D1D; ++cz) {
        double bb = 0;
#pragma unroll
        for (int b = 0; b < D1D; ++b) {
          double ab = 0;
#pragma unroll
          for (int a = 0; a < D1D; ++a) ab += Bx[a] * sW[6 + c][cz][b][s0 + a];
          bb += By[b] * ab;
        }
        KB[c][cz] = bb;
      }
    double EW[L1D], EK[L1D];
#pragma unroll
    for (int cl = 0; cl < L1D; ++cl) {
      double a1 = 0, a2 = 0;
#pragma unroll
      for (int bl = 0; bl < L1D; ++bl)
#pragma unroll
        for (int al = 0; al < L1D; ++al) {
          const double wgt = BLy[bl] * BLx[al];
          const int j = z * NLD + al + L1D * (bl + L1D * cl);
          a1 += wgt * sE[0][j];
          a2 += wgt * sE[1][j];
        }
      EW[cl] = a1;
      EK[cl] = a2;
    }
    const double wxy = tb.W[qx] * tb.W[qy] * rj_l;
#pragma unroll 1
    for (int qz = 0; qz < Q1D; ++qz) {
      double J[3][3], Gv[3][3], kv[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double j0 = 0, j1 = 0, j2 = 0, g0 = 0, g1 = 0, g2 = 0, m = 0;
#pragma unroll
        for (int cz = 0; cz < D1D; ++cz) {
          const double Bz = tb.B[qz][cz], Gz = tb.G[qz][cz];
          j0 += Bz * GB[c][cz];
          j1 += Bz * BG[c][cz];
          j2 += Gz * BB[c][cz];
          g0 += Bz * GB[3 + c][cz];
          g1 += Bz * BG[3 + c][cz];
          g2 += Gz * BB[3 + c][cz];
          m += Bz * KB[c][cz];
        }
        J[c][0] = j0;
        J[c][1] = j1;
        J[c][2] = j2;
        Gv[c][0] = g0;
        Gv[c][1] = g1;
        Gv[c][2] = g2;
        kv[c] = m;
      }
      double eq = 0, ke = 0;
#pragma unroll
      for (int cl = 0; cl < L1D; ++cl) {
        eq += tb.BL[qz][cl] * EW[cl];
        ke += tb.BL[qz][cl] * EK[cl];
      }
      const double mq = wxy * tb.W[qz];
      if (dmin)
        dm = nan_min(dm, J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                          J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                          J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]));
      double S[3][3], sq;
      qp_force<3, double>(P, gam, mq, dJ0, J, Gv, eq, S, sq);
      const double cl_ = mq * ke - sq;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double mv = mq * kv[c];
#pragma unroll
        for (int cz = 0; cz < D1D; ++cz) {
          const double Bz = tb.B[qz][cz], Gz = tb.G[qz][cz];
          Tx[c][cz] += Bz * S[c][0];
          Ty[c][cz] += Bz * S[c][1];
          Tz[c][cz] += Gz * S[c][2] + Bz * mv;
        }
      }
#pragma unroll
      for (int cl = 0; cl < L1D; ++cl) TL[cl] += tb.BL[qz][cl] * cl_;
    }
  }
  // velocity rows, one component at a time: column contributions to the element's nodes,
  // summed over the element's LPE lanes, one atomic per node and element (constrained rows were
  // written by their owner above)
  {
    double Bx[D1D], Gx[D1D], By[D1D], Gy[D1D];
#pragma unroll
    for (int a = 0; a < D1D; ++a) {
      Bx[a] = sBG[0][qx][a];
      Gx[a] = sBG[1][qx][a];
      By[a] = sBG[0][qy][a];
      Gy[a] = sBG[1][qy][a];
    }
    const int ex = ex0 + z;
#pragma unroll 1
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int cz = 0; cz < D1D; ++cz) {
        double tx = 0, ty = 0, tz = 0;
#pragma unroll
        for (int cq = 0; cq < 3; ++cq)
          if (cq == c) {
            tx = Tx[cq][cz];
            ty = Ty[cq][cz];
            tz = Tz[cq][cz];
          }
#pragma unroll
        for (int b = 0; b < D1D; ++b)
#pragma unroll
          for (int a = 0; a < D1D; ++a)
            sO[lane][(cz * D1D + b) * D1D + a] = Gx[a] * By[b] * tx + Bx[a] * Gy[b] * ty + Bx[a] * By[b] * tz;
      }
      lds_barrier();
      if (active) {
        for (int t = rr; t < NND; t += LPE) {
          double o = 0;
#pragma unroll
          for (int q = 0; q < LPE; ++q) o += sO[z * LPE + q][t];
          const int a = t % D1D, b = (t / D1D) % D1D, cz = t / (D1D * D1D);
          const uint32_t I = K * ex + a, J = K * ey + b, Kz = K * ez + cz;
          const uint32_t idx = c == 0 ? I : (c == 1 ? J : Kz), ngc = c == 0 ? ng0 : (c == 1 ? ng1 : ng2);
          if (idx != 0 && idx != ngc - 1) unsafeAtomicAdd(&r[nh1 + c * N + Kz * ng01 + J * ng0 + I], o);
        }
      }
      lds_barrier();
    }
  }
  // energy rows (element-owned)
  {
    double BLx[L1D], BLy[L1D];
#pragma unroll
    for (int a = 0; a < L1D; ++a) {
      BLx[a] = sBL[qx][a];
      BLy[a] = sBL[qy][a];
    }
#pragma unroll
    for (int cl = 0; cl < L1D; ++cl)
#pragma unroll
      for (int bl = 0; bl < L1D; ++bl)
#pragma unroll
        for (int al = 0; al < L1D; ++al) sO[lane][al + L1D * (bl + L1D * cl)] = BLx[al] * BLy[bl] * TL[cl];
  }
  lds_barrier();
  if (dmin) {  // the work-group's smallest det J of the stage positions w_x
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dm = nan_min(dm, __shfl_xor(dm, o, 64));
    if (lane == 0) dmin[(blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = dm;
  }
  if (active) {
    for (int t = rr; t < NLD; t += LPE) {
      double o = 0;
#pragma unroll
      for (int q = 0; q < LPE; ++q) o += sO[z * LPE + q][t];
      r[2 * nh1 + (ebase + z) * NLD + t] = o;
    }
  }
}

// ---- host side ---------------------------------------------------------------------------
bool res2d_available(const ilh_ctx* c) {
  return c->dim == 2 && (c->k == 2 || c->k == 3) && c->nblock < (int64_t(1) << 28) && !c->general;
}

bool res3d_available(const ilh_ctx* c) {
  return c->dim == 3 && c->k == 2 && !c->kp.tg_source && c->nblock < (int64_t(1) << 28) && !c->general;
}

template <int K, int SRC>
static void res_t(ilh_ctx* c, const double* k, const double* u, double tau, double* r, double* dmin,
                  const double* k2, double* r2) {
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
  const dim3 grid((c->n[0] + EPW - 1) / EPW, c->n[1], k2 ? 2 : 1);
  klaunch(c, k_res2d<D1D, Q1D, SRC>, grid, dim3(64), 0, c->kp, tb, u, k, tau, r, dmin, k2, r2);
}

int res3d_groups(const ilh_ctx* c) {
  const int EPW = 64 / 16;
  return ((c->n[0] + EPW - 1) / EPW) * c->n[1] * c->n[2];
}

// r = R(k; u, tau); the velocity rows of r must be zero on entry
int launch_res3d(ilh_ctx* c, const double* k, const double* u, double tau, double* r, double* dmin) {
  if (!res3d_available(c)) return ILH_EINVAL;
  constexpr int D1D = 3, Q1D = 4, EPW = 64 / (Q1D * Q1D);
  Tab2<double, D1D, Q1D> tb;
  for (int q = 0; q < Q1D; ++q) {
    for (int d = 0; d < D1D; ++d) {
      tb.B[q][d] = c->h_B[q * D1D + d];
      tb.G[q][d] = c->h_G[q * D1D + d];
    }
    for (int d = 0; d < D1D - 1; ++d) tb.BL[q][d] = c->h_BL[q * (D1D - 1) + d];
    tb.W[q] = c->h_w1[q];
  }
  const dim3 grid((c->n[0] + EPW - 1) / EPW, c->n[1], c->n[2]);
  klaunch(c, k_res3d<D1D, Q1D>, grid, dim3(64), 0, c->kp, tb, u, k, tau, r, dmin);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

int res2d_groups(const ilh_ctx* c) {
  const int EPW = 64 / (2 * c->k);
  return ((c->n[0] + EPW - 1) / EPW) * c->n[1];
}

// r = R(k; u, tau); the velocity rows of r must be zero on entry
int launch_res2d(ilh_ctx* c, const double* k, const double* u, double tau, double* r, double* dmin, const double* k2,
                 double* r2) {
  if (!res2d_available(c)) return ILH_EINVAL;
  if ((k2 == nullptr) != (r2 == nullptr) || (r2 && (r2 == r || dmin)))
    return fail(c, ILH_EINVAL, "residual pair: both or neither of k2, r2; distinct outputs; no det J");
  const int code = 2 * c->k + (c->kp.tg_source ? 1 : 0);
  switch (code) {
    case 4: res_t<2, 0>(c, k, u, tau, r, dmin, k2, r2); break;
    case 5: res_t<2, 1>(c, k, u, tau, r, dmin, k2, r2); break;
    case 6: res_t<3, 0>(c, k, u, tau, r, dmin, k2, r2); break;
    case 7: res_t<3, 1>(c, k, u, tau, r, dmin, k2, r2); break;
    default: return ILH_EINVAL;
  }
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

}  // namespace ilh

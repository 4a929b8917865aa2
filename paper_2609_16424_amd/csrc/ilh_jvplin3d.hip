// Linearised 3D Jacobian action of the stage residual (eq. pa_jac_action at a fixed Newton
// iterate): the 3D counterpart of ilh_jvplin2d.hip, with the stress-tangent coefficients of
// ilh_lin.h (20 values per point without viscosity, 29 with it; no TG source in 3D).
//
// Lane map (both kernels): one wave = EPW consecutive elements of one element row (fixed y and
// z index); lane (z, qy, qx) owns the quadrature column (qx, qy) of element z and walks its Q1D
// points in the third direction.  The wave's node strip (D1D z-layers x D1D y-rows x NS nodes
// per field) is gathered once into LDS; each lane forms the x and y contractions of every field
// for its column; the third direction is unrolled with the 1D tables in kernel arguments.  The
// element outputs are combined in LDS over the element's lanes, one velocity component at a
// time, before the atomic scatter of the shared nodes.
//
// Stored data: field f of lane l at step qz of strip b sits at qd[((b Q1D + qz) NQD + f) 64 + l]
// (the NQD fields of one wave's step form one contiguous block).  Strips are dealt to the XCDs
// in contiguous bands (xcd_tile).
#include <hip/hip_runtime.h>

#include "ilh_internal.h"
#include "ilh_lin.h"
#include "ilh_pointwise.h"

namespace ilh {

// ---- linearisation: state w (FP64) -> stored coefficients (T) ----------------------------
template <int D1D, int Q1D, typename T, int VISC>
__global__ void __launch_bounds__(64) k_lin3d(const KParams P, const Tab2<double, D1D, Q1D> tb,
                                              const double* __restrict__ w, double tau, T* __restrict__ qd,
                                              int64_t qs) {
  constexpr int K = D1D - 1, L1D = K, NLD = L1D * L1D * L1D;
  constexpr int LPE = Q1D * Q1D, EPW = 64 / LPE;
  constexpr int NS = K * EPW + 1;
  constexpr int NQD = LinLayout<3, VISC, 0>::NQD;
  constexpr int NPRE = 2 * 3 * 3;  // J^-1 and gv are not scaled by tau
  constexpr int NF = 6;            // x0 x1 x2 v0 v1 v2

  __shared__ double sS[NF][D1D][D1D][NS];
  __shared__ double sE[EPW * NLD];
  __shared__ double sBG[2][Q1D][D1D];
  __shared__ double sBL[Q1D][L1D];

  const int lane = threadIdx.x;
  const uint32_t tile = xcd_tile((blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x,
                                 gridDim.x * gridDim.y * gridDim.z);
  const int ex0 = (tile % gridDim.x) * EPW, ey = (tile / gridDim.x) % gridDim.y, ez = tile / (gridDim.x * gridDim.y);
  const int nx = P.n[0], ny = P.n[1];
  const int E = min(EPW, nx - ex0);
  const int ns = K * E + 1;
  const int64_t ng0 = P.ng[0], ng01 = (int64_t)P.ng[0] * P.ng[1];
  const int64_t N = P.N, nh1 = 3 * P.N;
  const int64_t ebase = ((int64_t)ez * ny + ey) * nx + ex0;
  const int64_t row0 = (int64_t)(K * ez) * ng01 + (int64_t)(K * ey) * ng0 + (int64_t)K * ex0;

  constexpr int NTS = NF * D1D * D1D * NS, RT = (NTS + 63) / 64;
  double tr[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int i = lane + 64 * r, s = i % NS, t = i / NS, b = t % D1D, cz = (t / D1D) % D1D, f = t / (D1D * D1D);
    tr[r] = 0.0;
    if (i < NTS && s < ns) tr[r] = w[(f < 3 ? f * N : nh1 + (f - 3) * N) + row0 + cz * ng01 + b * ng0 + s];
  }
  for (int i = lane; i < EPW * NLD; i += 64) sE[i] = (i < E * NLD) ? w[2 * nh1 + ebase * NLD + i] : 0.0;
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
  lds_barrier();

  const int z = lane / LPE, rr = lane - z * LPE, qy = rr / Q1D, qx = rr - qy * Q1D;
  if (z >= E) return;  // no barrier follows
  const int s0 = K * z;
  const int64_t e = ebase + z;
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
  // x-y contractions per z-layer: BB (values), GB (d/dx), BG (d/dy)
  double BB[NF][D1D], GB[NF][D1D], BG[NF][D1D];
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int cz = 0; cz < D1D; ++cz) {
      double bb = 0, gb = 0, bg = 0;
#pragma unroll
      for (int b = 0; b < D1D; ++b) {
        double ab = 0, ag = 0;
#pragma unroll
        for (int a = 0; a < D1D; ++a) {
          const double xv = sS[f][cz][b][s0 + a];
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
  double EL[L1D];
#pragma unroll
  for (int cl = 0; cl < L1D; ++cl) {
    double acc = 0;
#pragma unroll
    for (int bl = 0; bl < L1D; ++bl)
#pragma unroll
      for (int al = 0; al < L1D; ++al) acc += BLy[bl] * BLx[al] * sE[z * NLD + al + L1D * (bl + L1D * cl)];
    EL[cl] = acc;
  }
  const double gam = P.gamma[e], dJ0 = P.j0e[e];
  const double wxy = tb.W[qx] * tb.W[qy] * P.rj0[e];
  const int64_t blk = tile;
#pragma unroll 1
  for (int qz = 0; qz < Q1D; ++qz) {
    double J[3][3], Gv[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      double j0 = 0, j1 = 0, j2 = 0, g0 = 0, g1 = 0, g2 = 0;
#pragma unroll
      for (int c = 0; c < D1D; ++c) {
        const double Bz = tb.B[qz][c], Gz = tb.G[qz][c];
        j0 += Bz * GB[r][c];
        j1 += Bz * BG[r][c];
        j2 += Gz * BB[r][c];
        g0 += Bz * GB[3 + r][c];
        g1 += Bz * BG[3 + r][c];
        g2 += Gz * BB[3 + r][c];
      }
      J[r][0] = j0;
      J[r][1] = j1;
      J[r][2] = j2;
      Gv[r][0] = g0;
      Gv[r][1] = g1;
      Gv[r][2] = g2;
    }
    double eq = 0;
#pragma unroll
    for (int cl = 0; cl < L1D; ++cl) eq += tb.BL[qz][cl] * EL[cl];
    const double mq = wxy * tb.W[qz];
    double cf[NQD];
    lin_coefs<3, VISC>(P, gam, mq, dJ0, J, Gv, eq, cf);
#pragma unroll
    for (int f = NPRE; f < NQD; ++f) cf[f] *= tau;
    if constexpr (sizeof(T) == 4) {  // row-interleaved (FP32)
      T* q = qd + (blk * Q1D + qz) * (NQD * 64) + lane;
#pragma unroll
      for (int f = 0; f < NQD; ++f) q[f * 64] = T(cf[f]);
    } else {  // field-major (FP64)
      T* q = qd + (blk * Q1D + qz) * 64 + lane;
#pragma unroll
      for (int f = 0; f < NQD; ++f) q[f * qs] = T(cf[f]);
    }
  }
}

// ---- apply: direction dk (T) -> J dk (T) --------------------------------------------------
template <int D1D, int Q1D, typename T, int VISC>
__global__ void __launch_bounds__(64) k_jvp3d_q(const KParams P, const Tab2<T, D1D, Q1D> tb,
                                                const T* __restrict__ dk, const T* __restrict__ qd,
                                                int64_t qs, double tau_, T* __restrict__ out) {
  constexpr int K = D1D - 1, L1D = K, NLD = L1D * L1D * L1D;
  constexpr int LPE = Q1D * Q1D, EPW = 64 / LPE;
  constexpr int NS = K * EPW + 1;
  constexpr int NQD = LinLayout<3, VISC, 0>::NQD;
  constexpr int NF = 6;                      // dkx0 dkx1 dkx2 dkv0 dkv1 dkv2
  constexpr int NND = D1D * D1D * D1D;       // H1 nodes per element
  constexpr int NOP = (NND > NLD ? NND : NLD) | 1;  // odd LDS row length (bank spread)

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

  constexpr int NTS = NF * D1D * D1D * NS, RT = (NTS + 63) / 64;
  constexpr int NLS = EPW * NLD, RL = (NLS + 63) / 64;
  T tr[RT], lr[RL];
  // branch-free gathers: lanes past the strip re-read its last node (their LDS slots feed no
  // output), so every load is in flight before the first LDS store
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int i = lane + 64 * r, s = min(i % NS, ns - 1), t = min(i / NS, NF * D1D * D1D - 1), b = t % D1D,
              cz = (t / D1D) % D1D, f = t / (D1D * D1D);
    tr[r] = ld32(dk, (f < 3 ? f * N : nh1 + (f - 3) * N) + row0 + (uint32_t)cz * ng01 + (uint32_t)b * ng0 + s);
  }
#pragma unroll
  for (int r = 0; r < RL; ++r) lr[r] = ld32(dk, 2 * nh1 + ebase * NLD + min(lane + 64 * r, E * NLD - 1));
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
  T Bx[D1D], Gx[D1D], By[D1D], Gy[D1D], BLx[L1D], BLy[L1D];
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
  // per-lane sums over the column: Tx (coefficient of Gx By), Ty (Bx Gy), Tz (Bx By) per
  // velocity component and z-layer, TL per energy layer
  T Tx[3][D1D], Ty[3][D1D], Tz[3][D1D], TL[L1D];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < D1D; ++c) Tx[r][c] = Ty[r][c] = Tz[r][c] = T(0);
#pragma unroll
  for (int cl = 0; cl < L1D; ++cl) TL[cl] = T(0);
  if (active) {
    const int s0 = K * z;
    T BB[NF][D1D], GB[NF][D1D], BG[NF][D1D];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int cz = 0; cz < D1D; ++cz) {
        T bb = 0, gb = 0, bg = 0;
#pragma unroll
        for (int b = 0; b < D1D; ++b) {
          T ab = 0, ag = 0;
#pragma unroll
          for (int a = 0; a < D1D; ++a) {
            const T xv = sS[f][cz][b][s0 + a];
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
        for (int al = 0; al < L1D; ++al) acc += BLy[bl] * BLx[al] * sE[z * NLD + al + L1D * (bl + L1D * cl)];
      EL[cl] = acc;
    }
    const T wxy = tb.W[qx] * tb.W[qy] * T(rj_l);
    constexpr bool ROWS = sizeof(T) == 4;  // coefficient layout: row-interleaved (FP32), field-major (FP64)
    const T* __restrict__ qb = qd + (int64_t)tile * (Q1D * (ROWS ? NQD : 1) * 64);
    const T* qf[ROWS ? 1 : NQD];
    if constexpr (!ROWS) {
#pragma unroll
      for (int f = 0; f < NQD; ++f) qf[f] = sbase(qb + f * qs);
    }
    auto ldstep = [&](const int qz, T* c) {
      if constexpr (ROWS) {
        const T* rb = sbase(qb + qz * (NQD * 64));
#pragma unroll
        for (int f = 0; f < NQD; ++f) c[f] = ld32(rb, (uint32_t)(f * 64 + lane));
      } else {
#pragma unroll
        for (int f = 0; f < NQD; ++f) c[f] = ld32(qf[f], (uint32_t)(qz * 64 + lane));
      }
    };
    auto step = [&](const int qz, const T* cf) {
      // tau is folded into the coefficients: the contractions enter unscaled
      T dJ[3][3], dGv[3][3], dkv[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        T j0 = 0, j1 = 0, j2 = 0, g0 = 0, g1 = 0, g2 = 0, mv = 0;
#pragma unroll
        for (int c = 0; c < D1D; ++c) {
          const T Bz = tb.B[qz][c], Gz = tb.G[qz][c];
          j0 += Bz * GB[r][c];
          j1 += Bz * BG[r][c];
          j2 += Gz * BB[r][c];
          g0 += Bz * GB[3 + r][c];
          g1 += Bz * BG[3 + r][c];
          g2 += Gz * BB[3 + r][c];
          mv += Bz * BB[3 + r][c];
        }
        dJ[r][0] = j0;
        dJ[r][1] = j1;
        dJ[r][2] = j2;
        dGv[r][0] = g0;
        dGv[r][1] = g1;
        dGv[r][2] = g2;
        dkv[r] = mv;
      }
      T dke = 0;
#pragma unroll
      for (int cl = 0; cl < L1D; ++cl) dke += tb.BL[qz][cl] * EL[cl];
      const T mq = wxy * tb.W[qz];
      T dS[3][3], ds;
      lin_apply<3, T, VISC>(cf, dJ, dGv, dke, dS, ds);
      const T cl_ = mq * dke - ds;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const T mv = mq * dkv[r];
#pragma unroll
        for (int c = 0; c < D1D; ++c) {
          const T Bz = tb.B[qz][c], Gz = tb.G[qz][c];
          Tx[r][c] += Bz * dS[r][0];
          Ty[r][c] += Bz * dS[r][1];
          Tz[r][c] += Gz * dS[r][2] + Bz * mv;
        }
      }
#pragma unroll
      for (int cl = 0; cl < L1D; ++cl) TL[cl] += tb.BL[qz][cl] * cl_;
    };
    // the next step's coefficients are requested before this step's arithmetic
    T cf[NQD];
    ldstep(0, cf);
#pragma unroll 1
    for (int qz = 0; qz < Q1D; ++qz) {
      T cn[NQD];
      ldstep(qz + 1 < Q1D ? qz + 1 : qz, cn);
      step(qz, cf);
#pragma unroll
      for (int f = 0; f < NQD; ++f) cf[f] = cn[f];
    }
  }
  if constexpr (sizeof(T) == 4) {
  // velocity rows, one component at a time: each lane's column contributions to its element's
  // nodes (factored: out(a,b) = By_b (Gx_a Tx + Bx_a Tz) + Gy_b Bx_a Ty per z-layer) go to LDS;
  // one thread per node of the strip sums the columns of the (one or two) elements holding it
  // and issues one atomic add (constrained rows are set by the owner below)
#pragma unroll
  for (int a = 0; a < D1D; ++a) {  // reloaded: not kept live through the column loop
    Bx[a] = sBG[0][qx][a];
    Gx[a] = sBG[1][qx][a];
    By[a] = sBG[0][qy][a];
    Gy[a] = sBG[1][qy][a];
  }
#pragma unroll 1
  for (int r = 0; r < 3; ++r) {
#pragma unroll
    for (int cz = 0; cz < D1D; ++cz) {
      T tx = 0, ty = 0, tz = 0;
#pragma unroll
      for (int rq = 0; rq < 3; ++rq)
        if (rq == r) {
          tx = Tx[rq][cz];
          ty = Ty[rq][cz];
          tz = Tz[rq][cz];
        }
#pragma unroll
      for (int a = 0; a < D1D; ++a) {
        const T q1 = Gx[a] * tx + Bx[a] * tz, q2 = Bx[a] * ty;
#pragma unroll
        for (int b = 0; b < D1D; ++b) sO[lane][(cz * D1D + b) * D1D + a] = By[b] * q1 + Gy[b] * q2;
      }
    }
    lds_barrier();
    for (int i = lane; i < D1D * D1D * NS; i += 64) {
      const int s = i % NS, t = i / NS, b = t % D1D, cz = t / D1D;
      if (s >= ns) continue;
      const uint32_t I = K * ex0 + s, J = K * ey + b, Kz = K * ez + cz;
      const uint32_t idx = r == 0 ? I : (r == 1 ? J : Kz), ngr = r == 0 ? ng0 : (r == 1 ? ng1 : ng2);
      if (idx == 0 || idx == ngr - 1) continue;
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
      unsafeAtomicAdd(&out[nh1 + r * N + row0 + cz * ng01 + b * ng0 + s], o);
    }
    lds_barrier();
  }
  } else {  // FP64: per-element sums over the element's lanes, one atomic per node and element
  // velocity rows, one component at a time: column contributions to the element's nodes,
  // summed over the element's LPE lanes, scattered with atomics (shared nodes)
  const int ex = ex0 + z;
#pragma unroll
  for (int a = 0; a < D1D; ++a) {  // reloaded: not kept live through the column loop
    Bx[a] = sBG[0][qx][a];
    Gx[a] = sBG[1][qx][a];
    By[a] = sBG[0][qy][a];
    Gy[a] = sBG[1][qy][a];
  }
#pragma unroll 1
  for (int r = 0; r < 3; ++r) {
#pragma unroll
    for (int cz = 0; cz < D1D; ++cz)
#pragma unroll
      for (int b = 0; b < D1D; ++b)
#pragma unroll
        for (int a = 0; a < D1D; ++a) {
          T tx = 0, ty = 0, tz = 0;
#pragma unroll
          for (int rq = 0; rq < 3; ++rq)
            if (rq == r) {
              tx = Tx[rq][cz];
              ty = Ty[rq][cz];
              tz = Tz[rq][cz];
            }
          sO[lane][(cz * D1D + b) * D1D + a] = Gx[a] * By[b] * tx + Bx[a] * Gy[b] * ty + Bx[a] * By[b] * tz;
        }
    lds_barrier();
    if (active) {
      for (int t = rr; t < NND; t += LPE) {
        T o = 0;
#pragma unroll
        for (int q = 0; q < LPE; ++q) o += sO[z * LPE + q][t];
        const int a = t % D1D, b = (t / D1D) % D1D, cz = t / (D1D * D1D);
        const uint32_t I = K * ex + a, J = K * ey + b, Kz = K * ez + cz;
        const uint32_t idx = r == 0 ? I : (r == 1 ? J : Kz), ngr = r == 0 ? ng0 : (r == 1 ? ng1 : ng2);
        if (idx != 0 && idx != ngr - 1) unsafeAtomicAdd(&out[nh1 + r * N + Kz * ng01 + J * ng0 + I], o);
      }
    }
    lds_barrier();
  }
  }
  // energy rows (element-owned)
#pragma unroll
  for (int cl = 0; cl < L1D; ++cl)
#pragma unroll
    for (int bl = 0; bl < L1D; ++bl)
#pragma unroll
      for (int al = 0; al < L1D; ++al) sO[lane][al + L1D * (bl + L1D * cl)] = BLx[al] * BLy[bl] * TL[cl];
  lds_barrier();
  if (active) {
    for (int t = rr; t < NLD; t += LPE) {
      T o = 0;
#pragma unroll
      for (int q = 0; q < LPE; ++q) o += sO[z * LPE + q][t];
      out[2 * nh1 + (ebase + z) * NLD + t] = o;
    }
  }
  // position rows (dk_x - tau dk_v) and constrained velocity rows (dk_v), by node owner
  const T tau = T(tau_);
  const bool last_x = (ex0 + E == nx), last_y = (ey == ny - 1), last_z = (ez == P.n[2] - 1);
  for (int i = lane; i < 3 * D1D * D1D * NS; i += 64) {
    const int s = i % NS, t = i / NS, b = t % D1D, cz = (t / D1D) % D1D, c = t / (D1D * D1D);
    if (s >= ns || !((s < K * E || last_x) && (b < K || last_y) && (cz < K || last_z))) continue;
    const uint32_t I = K * ex0 + s, J = K * ey + b, Kz = K * ez + cz;
    const uint32_t gi = c * N + row0 + (uint32_t)cz * ng01 + (uint32_t)b * ng0 + s;
    const T dkv = sS[3 + c][cz][b][s];
    out[gi] = sS[c][cz][b][s] - tau * dkv;
    const uint32_t idx = c == 0 ? I : (c == 1 ? J : Kz), ngc = c == 0 ? ng0 : (c == 1 ? ng1 : ng2);
    if (idx == 0 || idx == ngc - 1) out[nh1 + gi] = dkv;  // the owner is the only writer
  }
}

// ---- host side ---------------------------------------------------------------------------
template <typename T, int D1D, int Q1D>
static Tab2<T, D1D, Q1D> make_tab3(const ilh_ctx* c) {
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

// 3D, Q2Q1 (4 elements per wave), no TG source; 32-bit element offsets into the block vectors
bool lin3d_available(const ilh_ctx* c) {
  return c->dim == 3 && c->k == 2 && !c->kp.tg_source && c->nblock < (int64_t(1) << 29) && !c->general;
}

static dim3 lin3d_grid(const ilh_ctx* c) {
  const int Q1D = 2 * c->k, EPW = 64 / (Q1D * Q1D);
  return dim3((c->n[0] + EPW - 1) / EPW, c->n[1], c->n[2]);
}

static int lin3d_nqd(const ilh_ctx* c) { return c->kp.visc ? LinLayout<3, 1, 0>::NQD : LinLayout<3, 0, 0>::NQD; }

static int64_t lin3d_stride(const ilh_ctx* c) {
  const dim3 g = lin3d_grid(c);
  return (int64_t)g.x * g.y * g.z * (2 * c->k) * 64;
}

template <typename T>
static int lin3d_t(ilh_ctx* c, T* qd) {
  if (c->kp.visc)
    klaunch(c, k_lin3d<3, 4, T, 1>, lin3d_grid(c), dim3(64), 0, c->kp, make_tab3<double, 3, 4>(c),
            (const double*)c->w64, c->lin_tau, qd, lin3d_stride(c));
  else
    klaunch(c, k_lin3d<3, 4, T, 0>, lin3d_grid(c), dim3(64), 0, c->kp, make_tab3<double, 3, 4>(c),
            (const double*)c->w64, c->lin_tau, qd, lin3d_stride(c));
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

template <typename T>
static int apply3d_t(ilh_ctx* c, const T* dk, const T* qd, T* out) {
  if (c->kp.visc)
    klaunch(c, k_jvp3d_q<3, 4, T, 1>, lin3d_grid(c), dim3(64), 0, c->kp, make_tab3<T, 3, 4>(c), dk, qd,
            lin3d_stride(c), c->lin_tau, out);
  else
    klaunch(c, k_jvp3d_q<3, 4, T, 0>, lin3d_grid(c), dim3(64), 0, c->kp, make_tab3<T, 3, 4>(c), dk, qd,
            lin3d_stride(c), c->lin_tau, out);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

int launch_lin3d(ilh_ctx* c, int prec) {
  if (!lin3d_available(c)) return ILH_EINVAL;
  const int p = prec == 64 ? 1 : 0;
  const int64_t len = (int64_t)lin3d_nqd(c) * lin3d_stride(c) * (p ? 8 : 4);
  if (!c->qd[p]) ILH_HIP(c, hipMalloc(&c->qd[p], len));
  return p ? lin3d_t<double>(c, (double*)c->qd[p]) : lin3d_t<float>(c, (float*)c->qd[p]);
}

int64_t lin3d_coef_bytes(const ilh_ctx* c, int prec) {
  return (int64_t)lin3d_nqd(c) * lin3d_stride(c) * (prec == 64 ? 8 : 4);
}

int launch_jvp3d_q(ilh_ctx* c, int prec, const void* dk, void* out) {
  if (!lin3d_available(c)) return ILH_EINVAL;
  const int p = prec == 64 ? 1 : 0;
  if (!c->qd[p]) return fail(c, ILH_EINVAL, "linearised Jacobian action before its linearisation");
  return p ? apply3d_t<double>(c, (const double*)dk, (const double*)c->qd[p], (double*)out)
           : apply3d_t<float>(c, (const float*)dk, (const float*)c->qd[p], (float*)out);
}

}  // namespace ilh

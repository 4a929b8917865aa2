// Linearised 2D Jacobian action of the stage residual (eq. pa_jac_action at a fixed Newton
// iterate), split into a linearisation launched once per iterate and an apply launched by
// every Krylov iteration.
//
// The tangent of the quadrature-point stress map is linear in the direction with coefficients
// that depend on the state alone (ilh_lin.h).  k_lin2d evaluates them at w in FP64 and stores
// them in the working precision (2D: 12 values per point without viscosity and with the TG
// source, 18 with both); k_jvp2d_q then reads the direction, the stored coefficients and the
// per-element mass factor only: geometry, inverse Jacobian, equation of state and viscosity
// of the state are not re-evaluated by each Krylov iteration.
//
// Layout of the stored data: field f of lane l at quadrature row qy of work-group b sits at
// qd[((b * Q1D + qy) * NQD + f) * 64 + l]: the NQD fields of one wave's quadrature row form
// one contiguous block of 64-lane rows (coalesced, one base address per row).  Both
// kernels use the work-group / lane map of the register-resident kernel: one wave = EPW
// consecutive elements of one element row, lane (z, qx) = quadrature column qx of element z.
#include <hip/hip_runtime.h>

#include "ilh_internal.h"
#include "ilh_lin.h"
#include "ilh_pointwise.h"

namespace ilh {

// ---- linearisation: state w (FP64) -> stored coefficients (T) ----------------------------
template <int D1D, int Q1D, typename T, int VISC, int SRC>
__global__ void __launch_bounds__(64) k_lin2d(const KParams P, const Tab2<double, D1D, Q1D> tb,
                                              const double* __restrict__ w, double tau, T* __restrict__ qd,
                                              int64_t qs) {
  constexpr int K = D1D - 1, L1D = K, NLD = L1D * L1D;
  constexpr int EPW = 64 / Q1D;
  constexpr int NS = K * EPW + 1;
  constexpr int NQD = LinLayout<2, VISC, SRC>::NQD;

  __shared__ double sS[4][D1D][NS];  // x0 x1 v0 v1
  __shared__ double sE[EPW * NLD];
  __shared__ double sBG[2][Q1D][D1D];
  __shared__ double sBLt[Q1D][L1D];

  const int lane = threadIdx.x;
  const uint32_t tile = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int sx = tile % gridDim.x, ey = tile / gridDim.x, ex0 = sx * EPW;
  const int nx = P.n[0];
  const int E = min(EPW, nx - ex0);
  const int ns = K * E + 1;
  const int64_t ng0 = P.ng[0];
  const int64_t N = P.N, nh1 = 2 * P.N;
  const int64_t ebase = (int64_t)ey * nx + ex0;

  constexpr int NTS = 4 * D1D * NS, RT = (NTS + 63) / 64;
  double tr[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int i = lane + 64 * r, si = i % NS, t = i / NS, b = t % D1D, f = t / D1D;
    tr[r] = 0.0;
    if (i < NTS && si < ns) {
      const int64_t node = (int64_t)(K * ey + b) * ng0 + (int64_t)K * ex0 + si;
      tr[r] = w[(f < 2 ? f * N : nh1 + (f - 2) * N) + node];
    }
  }
  for (int i = lane; i < EPW * NLD; i += 64) sE[i] = (i < E * NLD) ? w[2 * nh1 + ebase * NLD + i] : 0.0;
  for (int i = lane; i < Q1D * D1D; i += 64) {
    sBG[0][i / D1D][i % D1D] = tb.B[i / D1D][i % D1D];
    sBG[1][i / D1D][i % D1D] = tb.G[i / D1D][i % D1D];
  }
  for (int i = lane; i < Q1D * L1D; i += 64) sBLt[i / L1D][i % L1D] = tb.BL[i / L1D][i % L1D];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int i = lane + 64 * r;
    if (i < NTS) (&sS[0][0][0])[i] = tr[r];
  }
  __syncthreads();

  const int z = lane / Q1D, qx = lane - z * Q1D;
  if (z >= E) return;  // no barrier follows
  const int s0 = K * z;
  const int64_t e = ebase + z;
  double Bq[D1D], Gq[D1D], BLq[L1D];
#pragma unroll
  for (int a = 0; a < D1D; ++a) {
    Bq[a] = sBG[0][qx][a];
    Gq[a] = sBG[1][qx][a];
  }
#pragma unroll
  for (int a = 0; a < L1D; ++a) BLq[a] = sBLt[qx][a];
  double AB[4][D1D], AG[4][D1D];
#pragma unroll
  for (int f = 0; f < 4; ++f)
#pragma unroll
    for (int b = 0; b < D1D; ++b) {
      double ab = 0, ag = 0;
#pragma unroll
      for (int a = 0; a < D1D; ++a) {
        const double xv = sS[f][b][s0 + a];
        ab += Bq[a] * xv;
        ag += Gq[a] * xv;
      }
      AB[f][b] = ab;
      AG[f][b] = ag;
    }
  double ALe[L1D];
#pragma unroll
  for (int bl = 0; bl < L1D; ++bl) {
    double a0 = 0;
#pragma unroll
    for (int al = 0; al < L1D; ++al) a0 += BLq[al] * sE[z * NLD + al + L1D * bl];
    ALe[bl] = a0;
  }
  const double gam = P.gamma[e], dJ0 = P.j0e[e];
  const double wx = tb.W[qx] * P.rj0[e];
  const int64_t blk = tile;
#pragma unroll 1
  for (int qy = 0; qy < Q1D; ++qy) {
    double J[2][2], Gv[2][2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      double j0 = 0, j1 = 0, g0 = 0, g1 = 0;
#pragma unroll
      for (int b = 0; b < D1D; ++b) {
        const double By = tb.B[qy][b], Gy = tb.G[qy][b];
        j0 += By * AG[c][b];
        j1 += Gy * AB[c][b];
        g0 += By * AG[2 + c][b];
        g1 += Gy * AB[2 + c][b];
      }
      J[c][0] = j0;
      J[c][1] = j1;
      Gv[c][0] = g0;
      Gv[c][1] = g1;
    }
    double eq = 0;
#pragma unroll
    for (int bl = 0; bl < L1D; ++bl) eq += tb.BL[qy][bl] * ALe[bl];
    const double mq = wx * tb.W[qy];
    double cf[NQD];
    lin_coefs<2, VISC>(P, gam, mq, dJ0, J, Gv, eq, cf);
    if constexpr (SRC != 0) {
      double xq0 = 0, xq1 = 0;
#pragma unroll
      for (int b = 0; b < D1D; ++b) {
        xq0 += tb.B[qy][b] * AB[0][b];
        xq1 += tb.B[qy][b] * AB[1][b];
      }
      double gx, gy;
      if constexpr (sizeof(T) == 4) {
        // the pair is stored in FP32: the source gradient is evaluated in FP32 (positions O(1),
        // a few ulp of FP32 in the sines and cosines)
        float gxf, gyf;
        tg_source_grad<float>((float)xq0, (float)xq1, (float)gam, gxf, gyf);
        gx = gxf;
        gy = gyf;
      } else {
        tg_source_grad<double>(xq0, xq1, gam, gx, gy);
      }
      cf[NQD - 2] = mq * gx;
      cf[NQD - 1] = mq * gy;
    }
    // tau folded into every coefficient that multiplies the direction
#pragma unroll
    for (int f = 8; f < NQD; ++f) cf[f] *= tau;
    T* q = qd + (blk * Q1D + qy) * (NQD * 64) + lane;
#pragma unroll
    for (int f = 0; f < NQD; ++f) q[f * 64] = T(cf[f]);
  }
}

// ---- apply: direction dk (T) -> J dk (T) --------------------------------------------------
// One wave walks R consecutive element rows of its strip.  Per element row: the direction's
// node strips go to LDS, each lane contracts its quadrature column, and the per-lane
// contributions are summed per node in LDS (the vertical edges shared by neighbouring elements
// of the strip included).  Node row K of an element row is node row 0 of the next one: while the
// next row belongs to the same wave its partial sums are carried in LDS.  Each velocity row of
// the strip then takes one atomic add (one per node and strip instead of one per node and
// element); energy rows are element-owned, position rows and constrained velocity rows are
// written by the node's owner.  The velocity part of out must be zero on entry.
// W = 2 (FP32, small meshes): the two waves of a work-group share the strip, each takes half
// of the quadrature rows; the gathers and the node sums are spread over both, which halves the
// wave's chain of dependent row steps where the one-wave grid leaves most SIMDs idle.
template <int D1D, int Q1D, typename T, int VISC, int SRC, typename TO, int W, bool R1>
__global__ void __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(VISC && sizeof(T) == 8 ? 1 : 2))) k_jvp2d_q(const KParams P, const Tab2<T, D1D, Q1D> tb,
                                                const T* __restrict__ dk, const T* __restrict__ qd,
                                                int64_t qs, double tau_, TO* __restrict__ out, int R,
                                                const double* __restrict__ tau_dev,
                                                const double* __restrict__ skip) {
  constexpr int K = D1D - 1, L1D = K, NLD = L1D * L1D;
  constexpr int EPW = 64 / Q1D;
  constexpr int NS = K * EPW + 1;
  constexpr int NQD = LinLayout<2, VISC, SRC>::NQD;
  // node groups: GS lanes hold the NS nodes of one strip row (31 for Q3, 33 for Q2 strips)
  constexpr int GS = NS <= 32 ? 32 : 64;
  constexpr int NVO = 2 * D1D * D1D;  // velocity outputs per element (energy: NLD < NVO, later)
  constexpr int NOP = NVO | 1;        // odd LDS row length (bank spread)
  static_assert(Q1D % W == 0, "the quadrature rows split evenly over the waves");
  constexpr int NT = 64 * W;          // threads of the work-group
  constexpr int QW = Q1D / W;         // quadrature rows per wave

  __shared__ T sS[4][D1D][GS];  // dkx0 dkx1 dkv0 dkv1 strips (rows padded to the node group)
  __shared__ T sE[EPW * NLD];   // dk_e
  __shared__ T sO[W][64][NOP];  // per-lane contributions to the element's outputs (velocity, then energy)
  __shared__ T sC[2][2][NS];    // carried velocity sums of node row K (parity of the element row)
  __shared__ T sBG[2][Q1D][D1D];
  __shared__ T sBLt[Q1D][L1D];
  __shared__ T sW[Q1D];

  const int tid = threadIdx.x, hw = W == 1 ? 0 : tid / 64, lane = tid - 64 * hw;
  const uint32_t tile = xcd_tile(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int sx = tile % gridDim.x, sy = tile / gridDim.x;
  const int ex0 = sx * EPW;
  const int nx = P.n[0], ny = P.n[1];
  const int E = min(EPW, nx - ex0);
  const int ns = K * E + 1;
  const uint32_t ng0 = P.ng[0], ng1 = P.ng[1];
  const uint32_t N = (uint32_t)P.N, nh1 = 2 * N;
  const bool last_x = (ex0 + E == nx);
  const int ey0 = R1 ? sy : sy * R, ey1 = R1 ? ey0 + 1 : min(ey0 + R, ny);  // R1: R == 1
  const int z = lane / Q1D, qx = lane - z * Q1D;
  const bool active = z < E;
  constexpr int NG = NT / GS, PG = 4 * D1D / NG;
  static_assert(4 % NG == 0 || NG % 4 == 0, "node groups split the four fields evenly");
  const int gs = tid % GS, gg = tid / GS;
  const int sn = min(gs, ns - 1);  // this lane's node of the strip row (clamped)

#pragma unroll 1
  for (int ey = ey0; ey < ey1; ++ey) {
    const int r = ey - ey0;
    const bool last_y = (ey == ny - 1);
    const uint32_t ebase = (uint32_t)ey * nx + ex0;
    const uint32_t row0 = (uint32_t)(K * ey) * ng0 + (uint32_t)(K * ex0);  // first node of the strip

    constexpr int NLS = EPW * NLD, RL = (NLS + NT - 1) / NT;
    // branch-free gathers, one node of the strip per lane of a node group (GS lanes); pass p
    // of group g reads field f = g + NG p mod 4 (x0 x1 v0 v1 at f N) of node row (NG p) / 4,
    // so every address is the lane's base plus a per-pass scalar.  Lanes past the strip re-read
    // its last node (their LDS slots feed no output): all loads of the element row are in
    // flight together.
    T tr[PG], lr[RL];
    const uint32_t gbase = (uint32_t)gg * N + row0 + (uint32_t)sn;
#pragma unroll
    for (int p = 0; p < PG; ++p) {
      const int fo = (NG * p) & 3, bo = (NG * p) >> 2;
      tr[p] = ld32(dk, gbase + (uint32_t)fo * N + (uint32_t)bo * ng0);
    }
#pragma unroll
    for (int q = 0; q < RL; ++q) lr[q] = ld32(dk, 2 * nh1 + ebase * NLD + min(tid + NT * q, E * NLD - 1));
    const double rj_l = P.rj0[ebase + (active ? z : 0)];
    // coefficient rows of this element row: field f at qd[((blk Q1D + qy) NQD + f) 64 + lane]
    const T* __restrict__ qb = qd + ((int64_t)ey * gridDim.x + sx) * (Q1D * NQD * 64);
    // The row-loop instance (large meshes) streams them with the non-temporal hint: at 1024^2
    // they are 1.8 GB read once per launch, and unhinted they evict the direction's and the
    // output's lines, which neighbouring strips reuse (FP32 apply 534 -> 499 us, FP64 995 -> 970).
    // The one-row instance (small meshes, whose coefficients stay in the caches between the
    // Krylov iterations) keeps the plain load: the hint measured slower there.
    auto ldrow = [&](const int qy, T* cf) {
      const T* rb = sbase(qb + qy * (NQD * 64));
#pragma unroll
      for (int f = 0; f < NQD; ++f) {
        if constexpr (R1)
          cf[f] = ld32(rb, (uint32_t)(f * 64 + lane));
        else
          cf[f] = ld32_nt(rb, (uint32_t)(f * 64 + lane));
      }
    };
    T ca[NQD], cb[NQD];
    if (r == 0) {
      // the end-of-cycle flag is read while the first gathers are in flight (loads of a
      // launch that then returns are harmless), then the 1D tables go to LDS
      if (skip && *skip != 0.0) return;  // the Krylov cycle ended at the previous step
      for (int i = tid; i < Q1D * D1D; i += NT) {
        sBG[0][i / D1D][i % D1D] = tb.B[i / D1D][i % D1D];
        sBG[1][i / D1D][i % D1D] = tb.G[i / D1D][i % D1D];
      }
      for (int i = tid; i < Q1D * L1D; i += NT) sBLt[i / L1D][i % L1D] = tb.BL[i / L1D][i % L1D];
      if (tid < Q1D) sW[tid] = tb.W[tid];
    }
    lds_barrier();  // the previous element row's readers of sS, sE and sO are done
#pragma unroll
    for (int p = 0; p < PG; ++p) {
      const int fo = (NG * p) & 3, bo = (NG * p) >> 2;
      (&sS[0][0][0])[(gg * D1D) * GS + gs + (fo * D1D + bo) * GS] = tr[p];
    }
#pragma unroll
    for (int q = 0; q < RL; ++q) {
      const int i = tid + NT * q;
      if (i < NLS) sE[i] = lr[q];
    }
    lds_barrier();

    T TL[L1D];  // energy sums of the lane's column
#pragma unroll
    for (int bl = 0; bl < L1D; ++bl) TL[bl] = T(0);
    if (active) {
      const int s0 = K * z;
      T Bq[D1D], Gq[D1D], BLq[L1D];
#pragma unroll
      for (int a = 0; a < D1D; ++a) {
        Bq[a] = sBG[0][qx][a];
        Gq[a] = sBG[1][qx][a];
      }
#pragma unroll
      for (int a = 0; a < L1D; ++a) BLq[a] = sBLt[qx][a];
      T AB[4][D1D], AG[4][D1D];
#pragma unroll
      for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int b = 0; b < D1D; ++b) {
          T ab = 0, ag = 0;
#pragma unroll
          for (int a = 0; a < D1D; ++a) {
            const T xv = sS[f][b][s0 + a];
            ab += Bq[a] * xv;
            ag += Gq[a] * xv;
          }
          AB[f][b] = ab;
          AG[f][b] = ag;
        }
      T ALd[L1D];
#pragma unroll
      for (int bl = 0; bl < L1D; ++bl) {
        T a1 = 0;
#pragma unroll
        for (int al = 0; al < L1D; ++al) a1 += BLq[al] * sE[z * NLD + al + L1D * bl];
        ALd[bl] = a1;
      }
      T T0[2][D1D], T1[2][D1D];
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < D1D; ++b) T0[c][b] = T1[c][b] = T(0);
      const T wx = sW[qx] * T(rj_l);
      auto row = [&](const int qy, const T* cf) {
        // tau is folded into the coefficients: the contractions enter unscaled
        T dJ[2][2], dGv[2][2], dkv[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          T d0 = 0, d1 = 0, h0 = 0, h1 = 0, mv = 0;
#pragma unroll
          for (int b = 0; b < D1D; ++b) {
            const T By = tb.B[qy][b], Gy = tb.G[qy][b];
            d0 += By * AG[c][b];
            d1 += Gy * AB[c][b];
            h0 += By * AG[2 + c][b];
            h1 += Gy * AB[2 + c][b];
            mv += By * AB[2 + c][b];
          }
          dJ[c][0] = d0;
          dJ[c][1] = d1;
          dGv[c][0] = h0;
          dGv[c][1] = h1;
          dkv[c] = mv;
        }
        T dke = 0;
#pragma unroll
        for (int bl = 0; bl < L1D; ++bl) dke += tb.BL[qy][bl] * ALd[bl];
        const T mq = wx * tb.W[qy];
        T dS[2][2], ds;
        lin_apply<2, T, VISC>(cf, dJ, dGv, dke, dS, ds);
        T cl = mq * dke - ds;
        if constexpr (SRC != 0) {
          T dx0 = 0, dx1 = 0;
#pragma unroll
          for (int b = 0; b < D1D; ++b) {
            dx0 += tb.B[qy][b] * AB[0][b];
            dx1 += tb.B[qy][b] * AB[1][b];
          }
          cl -= cf[NQD - 2] * dx0 + cf[NQD - 1] * dx1;
        }
        const T mv0 = mq * dkv[0], mv1 = mq * dkv[1];
#pragma unroll
        for (int b = 0; b < D1D; ++b) {
          const T By = tb.B[qy][b], Gy = tb.G[qy][b];
          T0[0][b] += By * dS[0][0];
          T0[1][b] += By * dS[1][0];
          T1[0][b] += Gy * dS[0][1] + By * mv0;
          T1[1][b] += Gy * dS[1][1] + By * mv1;
        }
#pragma unroll
        for (int bl = 0; bl < L1D; ++bl) TL[bl] += tb.BL[qy][bl] * cl;
      };
      // this wave's quadrature rows [q0, q0 + QW); two coefficient buffers: the loads of one
      // row are in flight during the other's arithmetic
      const int q0 = hw * QW, q1 = q0 + QW;
      ldrow(q0, ca);
      auto pass = [&](const int qy) {
        constexpr bool ODD = QW % 2 != 0;  // the last pass of an odd count has one row
        if (!ODD || qy + 1 < q1) ldrow(qy + 1, cb);
        row(qy, ca);
        if (qy + 2 < q1) ldrow(qy + 2, ca);
        if (!ODD || qy + 1 < q1) row(qy + 1, cb);
      };
      if constexpr (R1 && W == 1) {  // straight-line rows (the multi-row instance keeps the loop)
#pragma unroll
        for (int qy = 0; qy < Q1D; qy += 2) pass(qy);
      } else {
#pragma unroll 1
        for (int qy = q0; qy < q1; qy += 2) pass(qy);
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
            sO[hw][lane][c * D1D * D1D + b * D1D + a] = Gq[a] * T0[c][b] + Bq[a] * T1[c][b];
    }
    vm_drained();  // every load is consumed and no store is issued yet
    lds_barrier();

    // node rows of the strip: position rows (dk_x - tau dk_v) and constrained velocity rows
    // (dk_v) by the node's single owner; every other velocity row sums the Q1D columns of the
    // (one or two) elements of the strip that hold the node.  Lane gs of node group g takes
    // node gs of the rows (component c, node row b) = ((g + NG p) mod 2, (g + NG p) / 2) over
    // the passes p: the LDS and global addresses are per-lane bases plus per-pass constants.
    // All LDS reads are issued before the first sum (clamped addresses; the terms a node does
    // not have are dropped by selection), then the stores and atomics follow.
    T* const cw = &sC[r & 1][0][0];
    const T* const cr = &sC[(r + 1) & 1][0][0];
    constexpr int NCB = 2 * D1D, PN = NCB / NG;
    static_assert(NCB % NG == 0, "node groups split the (component, node row) pairs evenly");
    int tn = gs, gn = gg;  // lane constants of the node phase, not held through the row loop
    asm volatile("" : "+v"(tn), "+v"(gn));
    // pass p of group g: component c = lc + cp(p), node row b = lb + bp(p)
    const int lc = NG == 1 ? 0 : (gn & 1), lb = NG <= 2 ? 0 : (gn >> 1);
    const int zz = tn / K, a = tn - K * zz, sc = min(tn, ns - 1);
    const bool left = zz < E, shared = a == 0 && zz > 0;
    const int oR = min(zz, E - 1) * Q1D * NOP + lc * D1D * D1D + lb * D1D + a;
    int oL = max(zz - 1, 0) * Q1D * NOP + lc * D1D * D1D + lb * D1D + K;
    asm volatile("" : "+v"(oL));  // its own base (not oR minus a constant): immediate LDS offsets
    const int oS = (lc * D1D + lb) * GS + sc;
    const T* const sOf = &sO[0][0][0];
    const T* const sSf = &sS[0][0][0];
    T fv[PN], xv[PN], vv[PN];
#pragma unroll
    for (int p = 0; p < PN; ++p) {
      const int cp = NG == 1 ? (p & 1) : 0, bp = NG == 1 ? (p >> 1) : (NG / 2) * p;
      const int po = cp * D1D * D1D + bp * D1D;
      T f0 = sOf[oR + po], f1 = sOf[oL + po];
#pragma unroll
      for (int hq = 1; hq < W * Q1D; ++hq) {
        const int h = hq / Q1D, q = hq % Q1D;
        f0 += sOf[oR + po + (h * 64 + q) * NOP];
        f1 += sOf[oL + po + (h * 64 + q) * NOP];
      }
      fv[p] = (left ? f0 : T(0)) + (shared ? f1 : T(0));
      xv[p] = sSf[oS + (cp * D1D + bp) * GS];
      vv[p] = sSf[oS + (cp * D1D + bp) * GS + 2 * D1D * GS];
    }
    // the stage factor is first needed here (its load is not waited for before the gathers)
    const T tau = T(tau_dev ? *tau_dev : tau_);
    const uint32_t I = K * ex0 + tn;
    const bool consI = I == 0 || I == ng0 - 1, own_s = tn < K * E || last_x;
    const bool cI = lc == 0 && consI, isv = lc != 0;  // constrained-row tests of the lane's component
    const uint32_t gb = (uint32_t)lc * N + (uint32_t)lb * ng0 + row0 + tn;
    if (tn < ns) {
#pragma unroll
      for (int p = 0; p < PN; ++p) {
        const int cp = NG == 1 ? (p & 1) : 0, bp = NG == 1 ? (p >> 1) : (NG / 2) * p;
        const int c = lc + cp, b = lb + bp;
        const uint32_t gi = gb + (uint32_t)cp * N + (uint32_t)bp * ng0;
        const bool own = own_s && (b < K || last_y);
        const T dkv = vv[p];
        const uint32_t J = K * ey + b;
        const bool consJ = J == 0 || J == ng1 - 1;
        const bool cons = NG == 1 ? (cp == 0 ? consI : consJ) : (cI || (isv && consJ));
        // node row K completed by the next element row of this wave
        const bool carry = !R1 && b == K && !last_y && ey + 1 < ey1;
        T f = fv[p];
        if (!R1 && b == 0 && r > 0) f += cr[c * NS + tn];
        if (own) st32(out, gi, TO(xv[p] - tau * dkv));
        if (cons && own) st32(out, nh1 + gi, TO(dkv));
        if (!cons && carry) cw[c * NS + tn] = f;
        // atomics also where no other wave adds to the node: plain stores of the partial cache
        // lines of a strip cost more than the atomic updates on this chip
        if (!cons && !carry) atomic_add32(out, nh1 + gi, TO(f));
      }
    }
    // energy rows (element-owned): the column sums go through sO once the velocity is done
    lds_barrier();
    if (active) {
#pragma unroll
      for (int bl = 0; bl < L1D; ++bl)
#pragma unroll
        for (int al = 0; al < L1D; ++al) sO[hw][lane][bl * L1D + al] = sBLt[qx][al] * TL[bl];
    }
    lds_barrier();
    constexpr int NET = EPW * NLD, NE = (NET + NT - 1) / NT;
    T ev[NE];
#pragma unroll
    for (int it = 0; it < NE; ++it) {
      const int i = min(tid + NT * it, E * NLD - 1), zz = i / NLD, t = i % NLD;
      T o = 0;
#pragma unroll
      for (int h = 0; h < W; ++h)
#pragma unroll
        for (int q = 0; q < Q1D; ++q) o += sO[h][zz * Q1D + q][t];
      ev[it] = o;
    }
#pragma unroll
    for (int it = 0; it < NE; ++it) {
      const int i = tid + NT * it;
      if (i < E * NLD) st32(out, 2 * nh1 + ebase * NLD + i, TO(ev[it]));
    }
  }
}

// ---- host side ---------------------------------------------------------------------------
template <typename T, int D1D, int Q1D>
static Tab2<T, D1D, Q1D> make_tab2(const ilh_ctx* c) {
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

// 32-bit element offsets into the block vectors (byte offsets below 4 GiB in FP64)
static bool lin2d_supported(const ilh_ctx* c) {
  return c->dim == 2 && (c->k == 2 || c->k == 3) && c->nblock < (int64_t(1) << 29) && !c->general;
}

static dim3 lin2d_grid(const ilh_ctx* c) {
  const int Q1D = 2 * c->k, EPW = 64 / Q1D;
  return dim3((c->n[0] + EPW - 1) / EPW, c->n[1]);
}

// Element rows walked by one apply wave: 1 while the one-row grid has few waves per SIMD
// (small meshes are latency-bound), more on large meshes, where fewer wave-shared nodes mean
// fewer atomics.  c->apply_rows > 0 overrides the choice.
static int apply_rows(const ilh_ctx* c) {
  if (c->apply_rows > 0) return std::min(c->apply_rows, c->n[1]);
  const dim3 g = lin2d_grid(c);
  const int64_t waves = (int64_t)g.x * g.y;
  int R = 1;
  while (R < 8 && waves / (2 * R) >= 16384) R *= 2;
  return R;
}

int lin2d_nqd(const ilh_ctx* c) { return (c->kp.visc ? 16 : 10) + (c->kp.tg_source ? 2 : 0); }

int64_t lin2d_stride(const ilh_ctx* c) {
  const dim3 g = lin2d_grid(c);
  return (int64_t)g.x * g.y * (2 * c->k) * 64;
}

template <int K, typename T, int VISC, int SRC>
static void lin_t(ilh_ctx* c, T* qd) {
  constexpr int D1D = K + 1, Q1D = 2 * K;
  klaunch(c, k_lin2d<D1D, Q1D, T, VISC, SRC>, lin2d_grid(c), dim3(64), 0, c->kp, make_tab2<double, D1D, Q1D>(c),
          (const double*)c->w64, c->lin_tau, qd, lin2d_stride(c));
}

// Waves per strip of the FP32 apply: 2 while the one-row, one-wave grid gives the SIMDs fewer
// than one wave each (1,024 SIMDs), else 1; FP64 always 1 (its register budget is full).
// c->apply_waves > 0 overrides the choice for FP32.
static int apply_waves(const ilh_ctx* c, bool fp32) {
  if (!fp32) return 1;
  if (c->apply_waves > 0) return c->apply_waves;
  const dim3 g = lin2d_grid(c);
  return (int64_t)g.x * g.y < 1024 ? 2 : 1;
}

template <int K, typename T, int VISC, int SRC, typename TO>
static void apply_t(ilh_ctx* c, const T* dk, const T* qd, TO* out, const double* tau_dev, const double* skip) {
  constexpr int D1D = K + 1, Q1D = 2 * K;
  const int R = apply_rows(c);
  const dim3 g = lin2d_grid(c), grid(g.x, (g.y + R - 1) / R);
  // one element row per wave: the kernel instance without the row loop
  if constexpr (sizeof(T) == 4) {
    if (apply_waves(c, true) == 2) {
      klaunch(c, R == 1 ? k_jvp2d_q<D1D, Q1D, T, VISC, SRC, TO, 2, true> : k_jvp2d_q<D1D, Q1D, T, VISC, SRC, TO, 2, false>,
              grid, dim3(128), 0, c->kp, make_tab2<T, D1D, Q1D>(c), dk, qd, lin2d_stride(c), c->lin_tau, out, R,
              tau_dev, skip);
      return;
    }
  }
  klaunch(c, R == 1 ? k_jvp2d_q<D1D, Q1D, T, VISC, SRC, TO, 1, true> : k_jvp2d_q<D1D, Q1D, T, VISC, SRC, TO, 1, false>,
          grid, dim3(64), 0, c->kp, make_tab2<T, D1D, Q1D>(c), dk, qd, lin2d_stride(c), c->lin_tau, out, R, tau_dev,
          skip);
}

template <typename T>
static int dispatch_lin(ilh_ctx* c, T* qd) {
  const int v = c->kp.visc ? 1 : 0, s = c->kp.tg_source ? 1 : 0, code = 4 * c->k + 2 * v + s;
  switch (code) {
    case 8: lin_t<2, T, 0, 0>(c, qd); break;
    case 9: lin_t<2, T, 0, 1>(c, qd); break;
    case 10: lin_t<2, T, 1, 0>(c, qd); break;
    case 11: lin_t<2, T, 1, 1>(c, qd); break;
    case 12: lin_t<3, T, 0, 0>(c, qd); break;
    case 13: lin_t<3, T, 0, 1>(c, qd); break;
    case 14: lin_t<3, T, 1, 0>(c, qd); break;
    case 15: lin_t<3, T, 1, 1>(c, qd); break;
    default: return ILH_EINVAL;
  }
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

template <typename T, typename TO>
static int dispatch_apply(ilh_ctx* c, const T* dk, const T* qd, TO* out, const double* tau_dev = nullptr,
                          const double* skip = nullptr) {
  const int v = c->kp.visc ? 1 : 0, s = c->kp.tg_source ? 1 : 0, code = 4 * c->k + 2 * v + s;
  switch (code) {
    case 8: apply_t<2, T, 0, 0, TO>(c, dk, qd, out, tau_dev, skip); break;
    case 9: apply_t<2, T, 0, 1, TO>(c, dk, qd, out, tau_dev, skip); break;
    case 10: apply_t<2, T, 1, 0, TO>(c, dk, qd, out, tau_dev, skip); break;
    case 11: apply_t<2, T, 1, 1, TO>(c, dk, qd, out, tau_dev, skip); break;
    case 12: apply_t<3, T, 0, 0, TO>(c, dk, qd, out, tau_dev, skip); break;
    case 13: apply_t<3, T, 0, 1, TO>(c, dk, qd, out, tau_dev, skip); break;
    case 14: apply_t<3, T, 1, 0, TO>(c, dk, qd, out, tau_dev, skip); break;
    case 15: apply_t<3, T, 1, 1, TO>(c, dk, qd, out, tau_dev, skip); break;
    default: return ILH_EINVAL;
  }
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

// Linearisation of precision prec at the current point (w64, lin_tau); the buffer is
// allocated on first use.  ILH_EINVAL when no linearised kernel exists for this context.
int launch_lin2d(ilh_ctx* c, int prec) {
  if (!lin2d_supported(c)) return ILH_EINVAL;
  const int p = prec == 64 ? 1 : 0;
  const int64_t len = (int64_t)lin2d_nqd(c) * lin2d_stride(c) * (p ? 8 : 4);
  if (!c->qd[p]) ILH_HIP(c, hipMalloc(&c->qd[p], len));
  return p ? dispatch_lin<double>(c, (double*)c->qd[p]) : dispatch_lin<float>(c, (float*)c->qd[p]);
}

int launch_jvp2d_q(ilh_ctx* c, int prec, const void* dk, void* out) {
  if (!lin2d_supported(c)) return ILH_EINVAL;
  const int p = prec == 64 ? 1 : 0;
  if (!c->qd[p]) return fail(c, ILH_EINVAL, "linearised Jacobian action before its linearisation");
  return p ? dispatch_apply<double, double>(c, (const double*)dk, (const double*)c->qd[p], (double*)out)
           : dispatch_apply<float, float>(c, (const float*)dk, (const float*)c->qd[p], (float*)out);
}

// FP32 action written straight into an FP64 vector (the Krylov basis): the velocity rows of out
// must be zero on entry, the FP32 coefficients current.
int launch_jvp2d_q_f32to64(ilh_ctx* c, const float* dk, double* out, const double* tau_dev, const double* skip) {
  if (!lin2d_supported(c)) return ILH_EINVAL;
  if (!c->qd[0] || !c->qd_ok[0]) return fail(c, ILH_EINVAL, "linearised Jacobian action before its linearisation");
  return dispatch_apply<float, double>(c, dk, (const float*)c->qd[0], out, tau_dev, skip);
}

// FP32 action into an FP32 Krylov vector, tau and the skip flag from the device (same contract)
int launch_jvp2d_q_f32to32(ilh_ctx* c, const float* dk, float* out, const double* tau_dev, const double* skip) {
  if (!lin2d_supported(c)) return ILH_EINVAL;
  if (!c->qd[0] || !c->qd_ok[0]) return fail(c, ILH_EINVAL, "linearised Jacobian action before its linearisation");
  return dispatch_apply<float, float>(c, dk, (const float*)c->qd[0], out, tau_dev, skip);
}

bool lin2d_available(const ilh_ctx* c) { return lin2d_supported(c); }

int64_t lin2d_coef_bytes(const ilh_ctx* c, int prec) {
  return (int64_t)lin2d_nqd(c) * lin2d_stride(c) * (prec == 64 ? 8 : 4);
}

}  // namespace ilh

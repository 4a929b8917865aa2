// Fused partial-assembly element kernels: gather (G), sum-factorised interpolation (B),
// quadrature-point kernel (D or its tangent), transposed interpolation (B^T) and scatter
// (G^T) in one launch -- the decomposition A = G^T B^T D B G of Sec. 2.2 (eq. decompose)
// applied to the nonlinear force operator (eq. pa_nonlinear) and to its Jacobian action
// (eq. pa_jac_action).
//
// Thread layout: one thread per quadrature point, NE elements per work-group.  The 1D
// basis tables B, G (H1, GLL Lagrange) and BL (L2, Bernstein) live in LDS; element DOFs
// are gathered into LDS, contracted one tensor direction at a time with barriers between
// the directions, and the shared H1 contributions are scattered with hardware FP64/FP32
// atomics into an output that was zero-filled beforehand.  Node indices are computed from
// the structured Cartesian numbering, so no element-to-node table is read.
#include <hip/hip_runtime.h>

#include "ilh_internal.h"
#include "ilh_pointwise.h"

namespace ilh {

template <typename T>
__device__ __forceinline__ void atomic_add(T* p, T v) {
  unsafeAtomicAdd(p, v);
}

template <typename T>
__device__ __forceinline__ const T* tab_ptr(const KParams& P);
template <>
__device__ __forceinline__ const double* tab_ptr<double>(const KParams& P) { return P.tab; }
template <>
__device__ __forceinline__ const float* tab_ptr<float>(const KParams& P) { return P.tabf; }

// ---------------------------------------------------------------------------------------
// 2D
// ---------------------------------------------------------------------------------------
template <int D1D, int Q1D, int MODE, typename T, int NE>
__global__ void __launch_bounds__(Q1D* Q1D* NE) k_elem2d(const KParams P, const EArgs<T> A) {
  constexpr int L1D = D1D - 1, ND = D1D * D1D, NLD = L1D * L1D, NQ = Q1D * Q1D, NT = NQ * NE;
  constexpr bool TAN = (MODE == M_FJVP || MODE == M_JVP);
  constexpr int NF = (MODE == M_FORCE) ? 2 : (MODE == M_RESID || MODE == M_ERATE ? 3 : 4);
  constexpr int NFL = (MODE == M_FORCE || MODE == M_ERATE) ? 1 : 2;
  constexpr bool WITH_SRC_OK = (MODE == M_RESID || MODE == M_JVP || MODE == M_ERATE);

  __shared__ T sB[Q1D * D1D], sG[Q1D * D1D], sBL[Q1D * L1D];
  __shared__ T sX[NE][NF][2][ND];
  __shared__ T sE[NE][NFL][NLD];
  __shared__ double sAnc[NE][2];
  __shared__ T sA[NE][2][2][D1D * Q1D];
  __shared__ T sAL[NE][NFL][L1D * Q1D];
  __shared__ T sQ[NE][7][NQ];

  const int tid = threadIdx.x;
  const int z = tid / NQ, q = tid - z * NQ, qx = q % Q1D, qy = q / Q1D;
  const int e0 = blockIdx.x * NE;
  const int k = P.k, n0 = P.n[0], n1 = P.n[1], ng0 = P.ng[0], ng1 = P.ng[1];
  const int64_t N = P.N, nh1 = 2 * P.N;
  const T tau = T(A.tau);
  const bool src = WITH_SRC_OK && P.tg_source;

  const T* tb = tab_ptr<T>(P);
  for (int i = tid; i < Q1D * D1D; i += NT) {
    sB[i] = tb[i];
    sG[i] = tb[Q1D * D1D + i];
  }
  for (int i = tid; i < Q1D * L1D; i += NT) sBL[i] = tb[2 * Q1D * D1D + i];
  if (tid < NE * 2) {
    const int zz = tid >> 1, c = tid & 1, e = e0 + zz;
    double a = 0.0;
    if (e < P.Ne) {
      const int ex = e % n0, ey = e / n0;
      const int64_t gi = c * N + (int64_t)k * ex + (int64_t)ng0 * k * ey;
      a = A.x[gi];
      if constexpr (MODE == M_RESID) a += A.tau * A.kk[gi];
    }
    sAnc[zz][c] = a;
  }
  __syncthreads();
  // gather H1 fields
  for (int i = tid; i < NE * NF * 2 * ND; i += NT) {
    const int a = i % D1D;
    int t = i / D1D;
    const int b = t % D1D;
    t /= D1D;
    const int c = t & 1;
    t >>= 1;
    const int f = t % NF, zz = t / NF, e = e0 + zz;
    T val = 0;
    if (e < P.Ne) {
      const int ex = e % n0, ey = e / n0;
      const int64_t gi = c * N + (int64_t)(k * ex + a) + (int64_t)ng0 * (k * ey + b);
      if (f == 0) {
        double xv = A.x[gi];
        if constexpr (MODE == M_RESID) xv += A.tau * A.kk[gi];
        val = T(xv - sAnc[zz][c]);
      } else if (f == 1) {
        if constexpr (MODE == M_RESID) val = T(double(A.v[gi]) + A.tau * A.kk[nh1 + gi]);
        else val = A.v[gi];
      } else if (f == 2) {
        if constexpr (MODE == M_RESID) val = T(A.kk[nh1 + gi]);
        else val = A.dk[gi];
      } else {
        if constexpr (TAN) val = A.dk[nh1 + gi];
      }
    }
    sX[zz][f][c][a + D1D * b] = val;
  }
  for (int i = tid; i < NE * NFL * NLD; i += NT) {
    const int j = i % NLD, t = i / NLD, f = t % NFL, zz = t / NFL, e = e0 + zz;
    T val = 0;
    if (e < P.Ne) {
      const int64_t gi = (int64_t)e * NLD + j;
      if (f == 0) {
        if constexpr (MODE == M_RESID) val = T(double(A.e[gi]) + A.tau * A.kk[2 * nh1 + gi]);
        else val = A.e[gi];
      } else {
        if constexpr (MODE == M_RESID) val = T(A.kk[2 * nh1 + gi]);
        else if constexpr (TAN) val = A.dk[2 * nh1 + gi];
      }
    }
    sE[zz][f][j] = val;
  }
  __syncthreads();
  // L2 contraction along xi
  for (int i = tid; i < NE * NFL * L1D * Q1D; i += NT) {
    const int qxx = i % Q1D;
    int t = i / Q1D;
    const int bl = t % L1D;
    t /= L1D;
    const int f = t % NFL, zz = t / NFL;
    T acc = 0;
#pragma unroll
    for (int al = 0; al < L1D; ++al) acc += sBL[qxx * L1D + al] * sE[zz][f][al + L1D * bl];
    sAL[zz][f][bl * Q1D + qxx] = acc;
  }
  T Jm[2][2], Gv[2][2], dJ[2][2], dGv[2][2], xval[2], mval[2], dxv[2];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    for (int i = tid; i < NE * 2 * D1D * Q1D; i += NT) {
      const int qxx = i % Q1D;
      int t = i / Q1D;
      const int b = t % D1D;
      t /= D1D;
      const int c = t & 1, zz = t >> 1;
      T ab = 0, ag = 0;
#pragma unroll
      for (int a = 0; a < D1D; ++a) {
        const T xv = sX[zz][f][c][a + D1D * b];
        ab += sB[qxx * D1D + a] * xv;
        ag += sG[qxx * D1D + a] * xv;
      }
      sA[zz][c][0][b * Q1D + qxx] = ab;
      sA[zz][c][1][b * Q1D + qxx] = ag;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      T gx = 0, gy = 0, val = 0;
#pragma unroll
      for (int b = 0; b < D1D; ++b) {
        const T Bb = sB[qy * D1D + b], Gb = sG[qy * D1D + b];
        const T ab = sA[z][c][0][b * Q1D + qx], ag = sA[z][c][1][b * Q1D + qx];
        gx += Bb * ag;
        gy += Gb * ab;
        val += Bb * ab;
      }
      if (f == 0) {
        Jm[c][0] = gx;
        Jm[c][1] = gy;
        xval[c] = val;
      } else if (f == 1) {
        Gv[c][0] = gx;
        Gv[c][1] = gy;
      } else if (f == 2) {
        if constexpr (MODE == M_RESID) {
          mval[c] = val;
        } else {
          dJ[c][0] = gx;
          dJ[c][1] = gy;
          dxv[c] = val;
        }
      } else {
        dGv[c][0] = gx;
        dGv[c][1] = gy;
        mval[c] = val;
      }
    }
    __syncthreads();
  }
  T eq = 0, e2 = 0;
#pragma unroll
  for (int bl = 0; bl < L1D; ++bl) {
    eq += sBL[qy * L1D + bl] * sAL[z][0][bl * Q1D + qx];
    if constexpr (NFL > 1) e2 += sBL[qy * L1D + bl] * sAL[z][1][bl * Q1D + qx];
  }
  // quadrature-point kernel
  const int e = e0 + z;
  const bool valid = e < P.Ne;
  T cx[2] = {0, 0}, cy[2] = {0, 0}, cm[2] = {0, 0}, cl = 0;
  if (valid) {
    const T mq = T(P.mq[(int64_t)e * NQ + q]);
    const T dJ0 = P.visc ? T(P.detJ0[(int64_t)e * NQ + q]) : T(1);
    const T gam = T(P.gamma[e]);
    if constexpr (!TAN) {
      T S[2][2], s;
      qp_force<2, T>(P, gam, mq, dJ0, Jm, Gv, eq, S, s);
      cx[0] = S[0][0];
      cy[0] = S[0][1];
      cx[1] = S[1][0];
      cy[1] = S[1][1];
      if constexpr (MODE == M_FORCE) {
        cl = s;
      } else if constexpr (MODE == M_ERATE) {
        // S : grad_xi vt = w |J| sigma : grad vt (field 2 holds the test velocity's gradient)
        cl = S[0][0] * dJ[0][0] + S[0][1] * dJ[0][1] + S[1][0] * dJ[1][0] + S[1][1] * dJ[1][1];
        if (src) cl += mq * tg_source<T>(T(sAnc[z][0] + double(xval[0])), T(sAnc[z][1] + double(xval[1])), gam);
      } else {
        cm[0] = mq * mval[0];
        cm[1] = mq * mval[1];
        cl = mq * e2 - s;
        if (src) cl -= mq * tg_source<T>(T(sAnc[z][0] + double(xval[0])),
                                         T(sAnc[z][1] + double(xval[1])), gam);
      }
    } else {
      const T sc = (MODE == M_JVP) ? tau : T(1);
      T dJs[2][2], dGs[2][2], dS[2][2], ds;
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          dJs[c][a] = sc * dJ[c][a];
          dGs[c][a] = sc * dGv[c][a];
        }
      qp_tangent<2, T>(P, gam, mq, dJ0, Jm, Gv, eq, dJs, dGs, sc * e2, dS, ds);
      cx[0] = dS[0][0];
      cy[0] = dS[0][1];
      cx[1] = dS[1][0];
      cy[1] = dS[1][1];
      if constexpr (MODE == M_FJVP) {
        cl = ds;
      } else {
        cm[0] = mq * mval[0];
        cm[1] = mq * mval[1];
        cl = mq * e2 - ds;
        if (src) {
          T gx, gy;
          tg_source_grad<T>(T(sAnc[z][0] + double(xval[0])), T(sAnc[z][1] + double(xval[1])), gam,
                            gx, gy);
          cl -= mq * tau * (gx * dxv[0] + gy * dxv[1]);
        }
      }
    }
  }
  sQ[z][0][q] = cx[0];
  sQ[z][1][q] = cx[1];
  sQ[z][2][q] = cy[0];
  sQ[z][3][q] = cy[1];
  sQ[z][4][q] = cm[0];
  sQ[z][5][q] = cm[1];
  sQ[z][6][q] = cl;
  __syncthreads();
  // transpose along eta
  for (int i = tid; i < NE * 2 * D1D * Q1D; i += NT) {
    const int qxx = i % Q1D;
    int t = i / Q1D;
    const int b = t % D1D;
    t /= D1D;
    const int c = t & 1, zz = t >> 1;
    T t0 = 0, t1 = 0;
#pragma unroll
    for (int qyy = 0; qyy < Q1D; ++qyy) {
      const T Bb = sB[qyy * D1D + b], Gb = sG[qyy * D1D + b];
      const int qq = qxx + Q1D * qyy;
      t0 += Bb * sQ[zz][c][qq];
      t1 += Gb * sQ[zz][2 + c][qq] + Bb * sQ[zz][4 + c][qq];
    }
    sA[zz][c][0][b * Q1D + qxx] = t0;
    sA[zz][c][1][b * Q1D + qxx] = t1;
  }
  for (int i = tid; i < NE * L1D * Q1D; i += NT) {
    const int qxx = i % Q1D, t = i / Q1D, bl = t % L1D, zz = t / L1D;
    T tl = 0;
#pragma unroll
    for (int qyy = 0; qyy < Q1D; ++qyy) tl += sBL[qyy * L1D + bl] * sQ[zz][6][qxx + Q1D * qyy];
    sAL[zz][0][bl * Q1D + qxx] = tl;
  }
  __syncthreads();
  // transpose along xi and scatter
  for (int i = tid; i < NE * 2 * ND; i += NT) {
    if constexpr (MODE == M_ERATE) break;  // energy rows only
    const int a = i % D1D;
    int t = i / D1D;
    const int b = t % D1D;
    t /= D1D;
    const int c = t & 1, zz = t >> 1, ee = e0 + zz;
    if (ee >= P.Ne) continue;
    T o = 0;
#pragma unroll
    for (int qxx = 0; qxx < Q1D; ++qxx)
      o += sG[qxx * D1D + a] * sA[zz][c][0][b * Q1D + qxx] + sB[qxx * D1D + a] * sA[zz][c][1][b * Q1D + qxx];
    const int ex = ee % n0, ey = ee / n0;
    const int I = k * ex + a, J = k * ey + b;
    const int64_t gi = c * N + I + (int64_t)ng0 * J;
    if constexpr (MODE == M_FORCE || MODE == M_FJVP) {
      atomic_add<T>(&A.out[gi], o);
    } else {
      const bool owner = (a < k || ex == n0 - 1) && (b < k || ey == n1 - 1);
      const bool cons = (c == 0) ? on_wall(P.walls, 0, I, ng0) : on_wall(P.walls, 1, J, ng1);
      const int li = a + D1D * b;
      if (!cons) atomic_add<T>(&A.out[nh1 + gi], o);
      if (owner) {
        if constexpr (MODE == M_RESID) {
          if (cons) atomic_add<T>(&A.out[nh1 + gi], sX[zz][2][c][li]);
          A.out[gi] = T(A.kk[gi]) - sX[zz][1][c][li];
        } else {
          if (cons) atomic_add<T>(&A.out[nh1 + gi], sX[zz][3][c][li]);
          A.out[gi] = sX[zz][2][c][li] - tau * sX[zz][3][c][li];
        }
      }
    }
  }
  for (int i = tid; i < NE * NLD; i += NT) {
    const int j = i % NLD, zz = i / NLD, al = j % L1D, bl = j / L1D, ee = e0 + zz;
    if (ee >= P.Ne) continue;
    T o = 0;
#pragma unroll
    for (int qxx = 0; qxx < Q1D; ++qxx) o += sBL[qxx * L1D + al] * sAL[zz][0][bl * Q1D + qxx];
    if constexpr (MODE == M_FORCE || MODE == M_FJVP || MODE == M_ERATE) A.out2[(int64_t)ee * NLD + j] = o;
    else A.out[2 * nh1 + (int64_t)ee * NLD + j] = o;
  }
}

// ---------------------------------------------------------------------------------------
// 3D
// ---------------------------------------------------------------------------------------
template <int D1D, int Q1D, int MODE, typename T, int NE>
__global__ void __launch_bounds__(Q1D* Q1D* Q1D* NE) k_elem3d(const KParams P, const EArgs<T> A) {
  constexpr int L1D = D1D - 1, ND = D1D * D1D * D1D, NLD = L1D * L1D * L1D;
  constexpr int NQ = Q1D * Q1D * Q1D, NT = NQ * NE;
  constexpr bool TAN = (MODE == M_FJVP || MODE == M_JVP);
  constexpr int NF = (MODE == M_FORCE) ? 2 : (MODE == M_RESID ? 3 : 4);
  constexpr int NFL = (MODE == M_FORCE) ? 1 : 2;
  constexpr int LA = D1D * D1D * Q1D;      // stage-1 buffer per (comp, kind)
  constexpr int LB = D1D * Q1D * Q1D;      // stage-2 buffer per (comp, kind)
  constexpr int LBUF = (2 * LA + 3 * LB > 4 * NQ) ? (2 * LA + 3 * LB) : (4 * NQ);

  __shared__ T sB[Q1D * D1D], sG[Q1D * D1D], sBL[Q1D * L1D];
  __shared__ T sX[NE][NF][3][ND];
  __shared__ T sE[NE][NFL][NLD];
  __shared__ double sAnc[NE][3];
  __shared__ T sW[NE][3][LBUF];  // stage buffers / per-qp outputs (per component)
  __shared__ T sL[NE][NFL][L1D * L1D * Q1D + L1D * Q1D * Q1D];
  __shared__ T sQL[NE][NQ];

  const int tid = threadIdx.x;
  const int z = tid / NQ, q = tid - z * NQ, qx = q % Q1D, qy = (q / Q1D) % Q1D, qz = q / (Q1D * Q1D);
  const int e0 = blockIdx.x * NE;
  const int k = P.k, n0 = P.n[0], n1 = P.n[1], n2 = P.n[2];
  const int ng0 = P.ng[0], ng1 = P.ng[1], ng2 = P.ng[2];
  const int64_t N = P.N, nh1 = 3 * P.N, s1 = ng0, s2 = (int64_t)ng0 * ng1;
  const T tau = T(A.tau);

  const T* tb = tab_ptr<T>(P);
  for (int i = tid; i < Q1D * D1D; i += NT) {
    sB[i] = tb[i];
    sG[i] = tb[Q1D * D1D + i];
  }
  for (int i = tid; i < Q1D * L1D; i += NT) sBL[i] = tb[2 * Q1D * D1D + i];
  if (tid < NE * 3) {
    const int zz = tid / 3, c = tid % 3, e = e0 + zz;
    double a = 0.0;
    if (e < P.Ne) {
      const int ex = e % n0, ey = (e / n0) % n1, ez = e / (n0 * n1);
      const int64_t gi = c * N + (int64_t)k * ex + s1 * k * ey + s2 * k * ez;
      a = A.x[gi];
      if constexpr (MODE == M_RESID) a += A.tau * A.kk[gi];
    }
    sAnc[zz][c] = a;
  }
  __syncthreads();
  for (int i = tid; i < NE * NF * 3 * ND; i += NT) {
    const int li = i % ND;
    int t = i / ND;
    const int c = t % 3;
    t /= 3;
    const int f = t % NF, zz = t / NF, e = e0 + zz;
    T val = 0;
    if (e < P.Ne) {
      const int a = li % D1D, b = (li / D1D) % D1D, cc = li / (D1D * D1D);
      const int ex = e % n0, ey = (e / n0) % n1, ez = e / (n0 * n1);
      const int64_t gi = c * N + (int64_t)(k * ex + a) + s1 * (k * ey + b) + s2 * (k * ez + cc);
      if (f == 0) {
        double xv = A.x[gi];
        if constexpr (MODE == M_RESID) xv += A.tau * A.kk[gi];
        val = T(xv - sAnc[zz][c]);
      } else if (f == 1) {
        if constexpr (MODE == M_RESID) val = T(double(A.v[gi]) + A.tau * A.kk[nh1 + gi]);
        else val = A.v[gi];
      } else if (f == 2) {
        if constexpr (MODE == M_RESID) val = T(A.kk[nh1 + gi]);
        else val = A.dk[gi];
      } else {
        if constexpr (TAN) val = A.dk[nh1 + gi];
      }
    }
    sX[zz][f][c][li] = val;
  }
  for (int i = tid; i < NE * NFL * NLD; i += NT) {
    const int j = i % NLD, t = i / NLD, f = t % NFL, zz = t / NFL, e = e0 + zz;
    T val = 0;
    if (e < P.Ne) {
      const int64_t gi = (int64_t)e * NLD + j;
      if (f == 0) {
        if constexpr (MODE == M_RESID) val = T(double(A.e[gi]) + A.tau * A.kk[2 * nh1 + gi]);
        else val = A.e[gi];
      } else {
        if constexpr (MODE == M_RESID) val = T(A.kk[2 * nh1 + gi]);
        else if constexpr (TAN) val = A.dk[2 * nh1 + gi];
      }
    }
    sE[zz][f][j] = val;
  }
  __syncthreads();
  // L2: three contractions (values only)
  for (int i = tid; i < NE * NFL * L1D * L1D * Q1D; i += NT) {
    const int qxx = i % Q1D;
    int t = i / Q1D;
    const int bc = t % (L1D * L1D);
    t /= (L1D * L1D);
    const int f = t % NFL, zz = t / NFL;
    T acc = 0;
#pragma unroll
    for (int al = 0; al < L1D; ++al) acc += sBL[qxx * L1D + al] * sE[zz][f][al + L1D * bc];
    sL[zz][f][bc * Q1D + qxx] = acc;  // [cl][bl][qx]
  }
  __syncthreads();
  for (int i = tid; i < NE * NFL * L1D * Q1D * Q1D; i += NT) {
    const int qxx = i % Q1D;
    int t = i / Q1D;
    const int qyy = t % Q1D;
    t /= Q1D;
    const int cl = t % L1D;
    t /= L1D;
    const int f = t % NFL, zz = t / NFL;
    T acc = 0;
#pragma unroll
    for (int bl = 0; bl < L1D; ++bl) acc += sBL[qyy * L1D + bl] * sL[zz][f][(cl * L1D + bl) * Q1D + qxx];
    sL[zz][f][L1D * L1D * Q1D + (cl * Q1D + qyy) * Q1D + qxx] = acc;
  }
  __syncthreads();
  T eq = 0, e2 = 0;
#pragma unroll
  for (int cl = 0; cl < L1D; ++cl) {
    eq += sBL[qz * L1D + cl] * sL[z][0][L1D * L1D * Q1D + (cl * Q1D + qy) * Q1D + qx];
    if constexpr (NFL > 1) e2 += sBL[qz * L1D + cl] * sL[z][1][L1D * L1D * Q1D + (cl * Q1D + qy) * Q1D + qx];
  }
  T Jm[3][3], Gv[3][3], dJ[3][3], dGv[3][3], mval[3], xval[3];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    // stage 1: contract a -> [c][kind][cc][b][qx]
    for (int i = tid; i < NE * 3 * D1D * D1D * Q1D; i += NT) {
      const int qxx = i % Q1D;
      int t = i / Q1D;
      const int bcc = t % (D1D * D1D);
      t /= (D1D * D1D);
      const int c = t % 3, zz = t / 3;
      T ab = 0, ag = 0;
#pragma unroll
      for (int a = 0; a < D1D; ++a) {
        const T xv = sX[zz][f][c][a + D1D * bcc];
        ab += sB[qxx * D1D + a] * xv;
        ag += sG[qxx * D1D + a] * xv;
      }
      sW[zz][c][bcc * Q1D + qxx] = ab;
      sW[zz][c][LA + bcc * Q1D + qxx] = ag;
    }
    __syncthreads();
    // stage 2: contract b -> BB, BG, GB [cc][qy][qx]
    for (int i = tid; i < NE * 3 * D1D * Q1D * Q1D; i += NT) {
      const int qxx = i % Q1D;
      int t = i / Q1D;
      const int qyy = t % Q1D;
      t /= Q1D;
      const int cc = t % D1D;
      t /= D1D;
      const int c = t % 3, zz = t / 3;
      T bb = 0, bg = 0, gb = 0;
#pragma unroll
      for (int b = 0; b < D1D; ++b) {
        const T Bb = sB[qyy * D1D + b], Gb = sG[qyy * D1D + b];
        const T ab = sW[zz][c][(cc * D1D + b) * Q1D + qxx];
        const T ag = sW[zz][c][LA + (cc * D1D + b) * Q1D + qxx];
        bb += Bb * ab;
        bg += Gb * ab;
        gb += Bb * ag;
      }
      const int o = 2 * LA + (cc * Q1D + qyy) * Q1D + qxx;
      sW[zz][c][o] = bb;
      sW[zz][c][o + LB] = bg;
      sW[zz][c][o + 2 * LB] = gb;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T g0 = 0, g1 = 0, g2 = 0, val = 0;
#pragma unroll
      for (int cc = 0; cc < D1D; ++cc) {
        const T Bc = sB[qz * D1D + cc], Gc = sG[qz * D1D + cc];
        const int o = 2 * LA + (cc * Q1D + qy) * Q1D + qx;
        const T bb = sW[z][c][o], bg = sW[z][c][o + LB], gb = sW[z][c][o + 2 * LB];
        g0 += Bc * gb;
        g1 += Bc * bg;
        g2 += Gc * bb;
        val += Bc * bb;
      }
      if (f == 0) {
        Jm[c][0] = g0;
        Jm[c][1] = g1;
        Jm[c][2] = g2;
        xval[c] = val;
      } else if (f == 1) {
        Gv[c][0] = g0;
        Gv[c][1] = g1;
        Gv[c][2] = g2;
      } else if (f == 2) {
        if constexpr (MODE == M_RESID) {
          mval[c] = val;
        } else {
          dJ[c][0] = g0;
          dJ[c][1] = g1;
          dJ[c][2] = g2;
        }
      } else {
        dGv[c][0] = g0;
        dGv[c][1] = g1;
        dGv[c][2] = g2;
        mval[c] = val;
      }
    }
    __syncthreads();
  }
  (void)xval;
  const int e = e0 + z;
  const bool valid = e < P.Ne;
  T cx[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, cm[3] = {0, 0, 0}, cl = 0;
  if (valid) {
    const T mq = T(P.mq[(int64_t)e * NQ + q]);
    const T dJ0 = P.visc ? T(P.detJ0[(int64_t)e * NQ + q]) : T(1);
    const T gam = T(P.gamma[e]);
    if constexpr (!TAN) {
      T s;
      qp_force<3, T>(P, gam, mq, dJ0, Jm, Gv, eq, cx, s);
      if constexpr (MODE == M_FORCE) {
        cl = s;
      } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) cm[c] = mq * mval[c];
        cl = mq * e2 - s;
      }
    } else {
      const T sc = (MODE == M_JVP) ? tau : T(1);
      T dJs[3][3], dGs[3][3], ds;
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          dJs[c][a] = sc * dJ[c][a];
          dGs[c][a] = sc * dGv[c][a];
        }
      qp_tangent<3, T>(P, gam, mq, dJ0, Jm, Gv, eq, dJs, dGs, sc * e2, cx, ds);
      if constexpr (MODE == M_FJVP) {
        cl = ds;
      } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) cm[c] = mq * mval[c];
        cl = mq * e2 - ds;
      }
    }
  }
  // per-qp outputs: sW[z][c][kind*NQ + q], kind 0..2 = grad coefficient, 3 = mass
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    sW[z][c][q] = cx[c][0];
    sW[z][c][NQ + q] = cx[c][1];
    sW[z][c][2 * NQ + q] = cx[c][2];
    sW[z][c][3 * NQ + q] = cm[c];
  }
  sQL[z][q] = cl;
  __syncthreads();
  // transposes.  H1: U[c][0..2][cc][qy][qx] (contract qz), then V[c][0..1][cc][b][qx]
  // (contract qy), then out[a][b][cc] (contract qx).  Registers hold U/V between barriers.
  constexpr int NU = NE * 3 * D1D * Q1D * Q1D;
  constexpr int NUT = (NU + NT - 1) / NT;
  T u0r[NUT], u1r[NUT], u2r[NUT];
#pragma unroll
  for (int r = 0; r < NUT; ++r) {
    const int i = tid + r * NT;
    if (i >= NU) break;
    const int qxx = i % Q1D;
    int t = i / Q1D;
    const int qyy = t % Q1D;
    t /= Q1D;
    const int cc = t % D1D;
    t /= D1D;
    const int c = t % 3, zz = t / 3;
    T a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
    for (int qzz = 0; qzz < Q1D; ++qzz) {
      const T Bc = sB[qzz * D1D + cc], Gc = sG[qzz * D1D + cc];
      const int qq = qxx + Q1D * (qyy + Q1D * qzz);
      a0 += Bc * sW[zz][c][qq];
      a1 += Bc * sW[zz][c][NQ + qq];
      a2 += Gc * sW[zz][c][2 * NQ + qq] + Bc * sW[zz][c][3 * NQ + qq];
    }
    u0r[r] = a0;
    u1r[r] = a1;
    u2r[r] = a2;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NUT; ++r) {
    const int i = tid + r * NT;
    if (i >= NU) break;
    const int qxx = i % Q1D;
    int t = i / Q1D;
    const int qyy = t % Q1D;
    t /= Q1D;
    const int cc = t % D1D;
    t /= D1D;
    const int c = t % 3, zz = t / 3;
    const int o = (cc * Q1D + qyy) * Q1D + qxx;
    sW[zz][c][o] = u0r[r];
    sW[zz][c][LB + o] = u1r[r];
    sW[zz][c][2 * LB + o] = u2r[r];
  }
  __syncthreads();
  // contract qy: V0 = sum B(qy,b) U0 ; V1 = sum G(qy,b) U1 + B(qy,b) U2
  constexpr int NV = NE * 3 * D1D * D1D * Q1D;
  constexpr int NVT = (NV + NT - 1) / NT;
  T v0r[NVT], v1r[NVT];
#pragma unroll
  for (int r = 0; r < NVT; ++r) {
    const int i = tid + r * NT;
    if (i >= NV) break;
    const int qxx = i % Q1D;
    int t = i / Q1D;
    const int b = t % D1D;
    t /= D1D;
    const int cc = t % D1D;
    t /= D1D;
    const int c = t % 3, zz = t / 3;
    T a0 = 0, a1 = 0;
#pragma unroll
    for (int qyy = 0; qyy < Q1D; ++qyy) {
      const T Bb = sB[qyy * D1D + b], Gb = sG[qyy * D1D + b];
      const int o = (cc * Q1D + qyy) * Q1D + qxx;
      a0 += Bb * sW[zz][c][o];
      a1 += Gb * sW[zz][c][LB + o] + Bb * sW[zz][c][2 * LB + o];
    }
    v0r[r] = a0;
    v1r[r] = a1;
  }
  // L2 transposes (independent of sW)
  for (int i = tid; i < NE * L1D * Q1D * Q1D; i += NT) {
    const int qxx = i % Q1D;
    int t = i / Q1D;
    const int qyy = t % Q1D;
    t /= Q1D;
    const int cl2 = t % L1D, zz = t / L1D;
    T acc = 0;
#pragma unroll
    for (int qzz = 0; qzz < Q1D; ++qzz) acc += sBL[qzz * L1D + cl2] * sQL[zz][qxx + Q1D * (qyy + Q1D * qzz)];
    sL[zz][0][(cl2 * Q1D + qyy) * Q1D + qxx] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < NVT; ++r) {
    const int i = tid + r * NT;
    if (i >= NV) break;
    const int qxx = i % Q1D;
    int t = i / Q1D;
    const int b = t % D1D;
    t /= D1D;
    const int cc = t % D1D;
    t /= D1D;
    const int c = t % 3, zz = t / 3;
    const int o = (cc * D1D + b) * Q1D + qxx;
    sW[zz][c][o] = v0r[r];
    sW[zz][c][LA + o] = v1r[r];
  }
  for (int i = tid; i < NE * L1D * L1D * Q1D; i += NT) {
    const int qxx = i % Q1D;
    int t = i / Q1D;
    const int bl = t % L1D;
    t /= L1D;
    const int cl2 = t % L1D, zz = t / L1D;
    T acc = 0;
#pragma unroll
    for (int qyy = 0; qyy < Q1D; ++qyy) acc += sBL[qyy * L1D + bl] * sL[zz][0][(cl2 * Q1D + qyy) * Q1D + qxx];
    sL[zz][0][L1D * Q1D * Q1D + (cl2 * L1D + bl) * Q1D + qxx] = acc;
  }
  __syncthreads();
  for (int i = tid; i < NE * 3 * ND; i += NT) {
    const int li = i % ND;
    int t = i / ND;
    const int c = t % 3, zz = t / 3, ee = e0 + zz;
    if (ee >= P.Ne) continue;
    const int a = li % D1D, b = (li / D1D) % D1D, cc = li / (D1D * D1D);
    T o = 0;
#pragma unroll
    for (int qxx = 0; qxx < Q1D; ++qxx) {
      const int oo = (cc * D1D + b) * Q1D + qxx;
      o += sG[qxx * D1D + a] * sW[zz][c][oo] + sB[qxx * D1D + a] * sW[zz][c][LA + oo];
    }
    const int ex = ee % n0, ey = (ee / n0) % n1, ez = ee / (n0 * n1);
    const int I = k * ex + a, J = k * ey + b, K = k * ez + cc;
    const int64_t gi = c * N + I + s1 * J + s2 * K;
    if constexpr (MODE == M_FORCE || MODE == M_FJVP) {
      atomic_add<T>(&A.out[gi], o);
    } else {
      const bool owner = (a < k || ex == n0 - 1) && (b < k || ey == n1 - 1) && (cc < k || ez == n2 - 1);
      const int gc = (c == 0) ? I : (c == 1 ? J : K);
      const int ngc = (c == 0) ? ng0 : (c == 1 ? ng1 : ng2);
      const bool cons = on_wall(P.walls, c, gc, ngc);
      if (!cons) atomic_add<T>(&A.out[nh1 + gi], o);
      if (owner) {
        if constexpr (MODE == M_RESID) {
          if (cons) atomic_add<T>(&A.out[nh1 + gi], sX[zz][2][c][li]);
          A.out[gi] = T(A.kk[gi]) - sX[zz][1][c][li];
        } else {
          if (cons) atomic_add<T>(&A.out[nh1 + gi], sX[zz][3][c][li]);
          A.out[gi] = sX[zz][2][c][li] - tau * sX[zz][3][c][li];
        }
      }
    }
  }
  for (int i = tid; i < NE * NLD; i += NT) {
    const int j = i % NLD, zz = i / NLD, ee = e0 + zz;
    if (ee >= P.Ne) continue;
    const int al = j % L1D, bcl = j / L1D;
    T o = 0;
#pragma unroll
    for (int qxx = 0; qxx < Q1D; ++qxx) o += sBL[qxx * L1D + al] * sL[zz][0][L1D * Q1D * Q1D + bcl * Q1D + qxx];
    if constexpr (MODE == M_FORCE || MODE == M_FJVP) A.out2[(int64_t)ee * NLD + j] = o;
    else A.out[2 * nh1 + (int64_t)ee * NLD + j] = o;
  }
}

// ---------------------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------------------
template <int DIM, int K>
struct ElemCfg;
template <> struct ElemCfg<2, 1> { static constexpr int NE = 64; };
template <> struct ElemCfg<2, 2> { static constexpr int NE = 16; };
template <> struct ElemCfg<2, 3> { static constexpr int NE = 7; };
template <> struct ElemCfg<2, 4> { static constexpr int NE = 4; };
template <> struct ElemCfg<3, 1> { static constexpr int NE = 32; };
template <> struct ElemCfg<3, 2> { static constexpr int NE = 4; };
template <> struct ElemCfg<3, 3> { static constexpr int NE = 1; };

template <int DIM, int K, int MODE, typename T>
static int launch_elem_t(ilh_ctx* c, const EArgs<T>& a) {
  constexpr int NE = ElemCfg<DIM, K>::NE;
  constexpr int Q1D = 2 * K;
  const int grid = (int)((c->Ne + NE - 1) / NE);
  if constexpr (DIM == 2) {
    klaunch(c, k_elem2d<K + 1, Q1D, MODE, T, NE>, dim3(grid), dim3(Q1D * Q1D * NE), 0, c->kp, a);
  } else {
    klaunch(c, k_elem3d<K + 1, Q1D, MODE, T, NE>, dim3(grid), dim3(Q1D * Q1D * Q1D * NE), 0, c->kp,
            a);
  }
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

template <int DIM, int K>
static int launch_elem_k(ilh_ctx* c, int mode, int prec, const EArgs<double>* a64, const EArgs<float>* a32) {
  if (prec == 64) {
    switch (mode) {
      case M_FORCE: return launch_elem_t<DIM, K, M_FORCE, double>(c, *a64);
      case M_RESID: return launch_elem_t<DIM, K, M_RESID, double>(c, *a64);
      case M_FJVP: return launch_elem_t<DIM, K, M_FJVP, double>(c, *a64);
      case M_JVP: return launch_elem_t<DIM, K, M_JVP, double>(c, *a64);
      case M_ERATE:
        if constexpr (DIM == 2) return launch_elem_t<DIM, K, M_ERATE, double>(c, *a64);
        break;
    }
  } else {
    switch (mode) {
      case M_FJVP: return launch_elem_t<DIM, K, M_FJVP, float>(c, *a32);
      case M_JVP: return launch_elem_t<DIM, K, M_JVP, float>(c, *a32);
    }
  }
  return fail(c, ILH_EINVAL, "unsupported element-kernel mode/precision");
}

int launch_elem(ilh_ctx* c, int mode, int prec, const EArgs<double>* a64, const EArgs<float>* a32) {
  if (c->Ne == 0) return ILH_OK;
  if (c->dim == 2) {
    switch (c->k) {
      case 1: return launch_elem_k<2, 1>(c, mode, prec, a64, a32);
      case 2: return launch_elem_k<2, 2>(c, mode, prec, a64, a32);
      case 3: return launch_elem_k<2, 3>(c, mode, prec, a64, a32);
      case 4: return launch_elem_k<2, 4>(c, mode, prec, a64, a32);
    }
  } else {
    switch (c->k) {
      case 1: return launch_elem_k<3, 1>(c, mode, prec, a64, a32);
      case 2: return launch_elem_k<3, 2>(c, mode, prec, a64, a32);
      case 3: return launch_elem_k<3, 3>(c, mode, prec, a64, a32);
    }
  }
  return fail(c, ILH_EINVAL, "unsupported dimension/order");
}

}  // namespace ilh

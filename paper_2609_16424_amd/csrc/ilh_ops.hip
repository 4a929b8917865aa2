// Mass operators, BLAS-1, reductions, per-quadrature-point diagnostics and the initial
// state.  The mass matrices M_V = int rho w w^T and M_E = int rho phi phi^T (Sec. 2.1,
// eq. matrices) are constant in time because rho |J| = rho0 |J0|; they are applied by
// partial assembly with the quadrature data m_q (Sec. 2.2) and M_V is inverted by
// Jacobi-preconditioned CG whose scalars stay on the device.
#include <hip/hip_runtime.h>

#include <cmath>
#include <utility>

#include "ilh_internal.h"
#include "ilh_pointwise.h"
#include "ilh_lin.h"

namespace ilh {

static constexpr int TPB = 256;

static inline int nblk(int64_t n, int cap = 65535 * 4) {
  int64_t b = (n + TPB - 1) / TPB;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

// ------------------------------------------------------------------ BLAS-1
__global__ void k_fill(double* p, double v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
// two arrays of one length set in one launch
__global__ void k_fill2(double* p, double* q, double v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    p[i] = v;
    q[i] = v;
  }
}
__global__ void k_fillf(float* p, float v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_axpby(double* y, double a, const double* x, double b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}
// w = u + t k; the first nz (<= n) entries of z are zeroed in the same pass (nz = 0: none)
__global__ void k_waxpy(double* w, const double* u, double t, const double* k, int64_t n, double* z, int64_t nz) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    w[i] = u[i] + t * k[i];
    if (i < nz) z[i] = 0.0;
  }
}
// u <- u + dt k, and k copied to kc (nullable) in the same pass
__global__ void k_step_update(double* u, double dt, const double* k, double* kc, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double ki = k[i];
    u[i] += dt * ki;
    if (kc) kc[i] = ki;
  }
}
// y = (float) x; the first nz (<= n) entries of z zeroed in the same pass (nz = 0: none)
__global__ void k_d2f(float* y, const double* x, int64_t n, double* z, int64_t nz) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    y[i] = (float)x[i];
    if (i < nz) z[i] = 0.0;
  }
}
__global__ void k_f2d(double* y, const float* x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (double)x[i];
}
// out = k1 (nhist 1) or 2 k1 - k2 (nhist 2); with tau > 0 the position block is u_v + tau out_v
__global__ void k_extrap(double* out, const double* u, const double* k1, const double* k2, int nhist, double tau,
                         int64_t nh1, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (tau > 0.0 && i < nh1) {
      const int64_t iv = nh1 + i;
      const double kv = nhist >= 2 ? 2.0 * k1[iv] - k2[iv] : k1[iv];
      out[i] = u[iv] + tau * kv;
    } else {
      out[i] = nhist >= 2 ? 2.0 * k1[i] - k2[i] : k1[i];
    }
  }
}
int launch_extrap(ilh_ctx* c, double* out, const double* u, const double* k1, const double* k2, int nhist,
                  double tau) {
  const int64_t n = c->nblock;
  hipLaunchKernelGGL(k_extrap, dim3(nblk(n, 4096)), dim3(TPB), 0, c->stream, out, u, k1, k2, nhist, tau, c->nh1, n);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

__global__ void k_jacobi(const double* r, const double* d, double* z, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    z[i] = r[i] / d[i];
}

int launch_fill(ilh_ctx* c, double* p, double v, int64_t n) {
  if (n <= 0) return ILH_OK;
  hipLaunchKernelGGL(k_fill, dim3(nblk(n)), dim3(TPB), 0, c->stream, p, v, n);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}
int launch_fill2(ilh_ctx* c, double* p, double* q, double v, int64_t n) {
  if (n <= 0) return ILH_OK;
  hipLaunchKernelGGL(k_fill2, dim3(nblk(n)), dim3(TPB), 0, c->stream, p, q, v, n);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}
int launch_fillf(ilh_ctx* c, float* p, float v, int64_t n) {
  if (n <= 0) return ILH_OK;
  hipLaunchKernelGGL(k_fillf, dim3(nblk(n)), dim3(TPB), 0, c->stream, p, v, n);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}
int launch_axpby(ilh_ctx* c, double* y, double a, const double* x, double b, int64_t n) {
  if (n <= 0) return ILH_OK;
  hipLaunchKernelGGL(k_axpby, dim3(nblk(n)), dim3(TPB), 0, c->stream, y, a, x, b, n);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}
int launch_waxpy(ilh_ctx* c, double* w, const double* u, double t, const double* k, int64_t n, double* z,
                 int64_t nz) {
  if (nz > n || nz < 0 || (nz > 0 && !z)) return fail(c, ILH_EINVAL, "waxpy: zero target longer than the vector");
  if (n <= 0) return ILH_OK;
  hipLaunchKernelGGL(k_waxpy, dim3(nblk(n)), dim3(TPB), 0, c->stream, w, u, t, k, n, z, nz);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}
int launch_step_update(ilh_ctx* c, double* u, double dt, const double* k, double* kc, int64_t n) {
  if (n <= 0) return ILH_OK;
  hipLaunchKernelGGL(k_step_update, dim3(nblk(n)), dim3(TPB), 0, c->stream, u, dt, k, kc, n);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}
int launch_cast_d2f(ilh_ctx* c, float* y, const double* x, int64_t n, double* z, int64_t nz) {
  if (nz > n || nz < 0 || (nz > 0 && !z)) return fail(c, ILH_EINVAL, "cast: zero target longer than the vector");
  if (n <= 0) return ILH_OK;
  hipLaunchKernelGGL(k_d2f, dim3(nblk(n)), dim3(TPB), 0, c->stream, y, x, n, z, nz);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}
// y = a x on the free rows of an H1 vector, 0 on the constrained (wall) rows
__global__ void k_scale_free(double* y, double a, const double* x, KParams P) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.dim * P.N) return;
  const int c = (int)(i / P.N);
  int64_t node = i - (int64_t)c * P.N;
  int64_t g = node % P.ng[0];
  if (c >= 1) {
    node /= P.ng[0];
    g = node % P.ng[1];
  }
  if (c == 2) g = node / P.ng[1];
  const bool cons = on_wall(P.walls, c, g, P.ng[c]);
  y[i] = cons ? 0.0 : a * x[i];
}

int launch_scale_free(ilh_ctx* c, double* y, double a, const double* x) {
  const int64_t n = c->nh1;
  hipLaunchKernelGGL(k_scale_free, dim3(nblk(n)), dim3(TPB), 0, c->stream, y, a, x, c->kp);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

int launch_cast_f2d(ilh_ctx* c, double* y, const float* x, int64_t n) {
  if (n <= 0) return ILH_OK;
  hipLaunchKernelGGL(k_f2d, dim3(nblk(n)), dim3(TPB), 0, c->stream, y, x, n);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}
int launch_jacobi(ilh_ctx* c, const double* r, double* z) {
  hipLaunchKernelGGL(k_jacobi, dim3(nblk(c->nh1)), dim3(TPB), 0, c->stream, r, c->Mdiag, z, c->nh1);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

// ------------------------------------------------------------------ reductions
// Deterministic two-pass reductions: a fixed grid writes one partial per block, a single
// block sums the partials in a fixed order.
template <int BS>
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double sh[BS / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < BS / 64; ++i) r += sh[i];
  __syncthreads();
  return r;
}
template <int BS>
__device__ __forceinline__ double block_min(double v) {
  __shared__ double sh[BS / 64];
  for (int o = 32; o > 0; o >>= 1) v = nan_min(v, __shfl_down(v, o, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = v;
  if (threadIdx.x == 0) {
    r = sh[0];
    for (int i = 1; i < BS / 64; ++i) r = nan_min(r, sh[i]);
  }
  __syncthreads();
  return r;
}

// partial sums of x . y, one per block; grid.y = 2: the blocks of row 1 take x2 . y2 into part2
__global__ void __launch_bounds__(TPB) k_dot_part(const double* x, const double* y, int64_t n, double* part,
                                                  const double* x2, const double* y2, double* part2) {
  if (blockIdx.y != 0) {
    x = x2;
    y = y2;
    part = part2;
  }
  double acc = 0;
  for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) acc += x[i] * y[i];
  acc = block_sum<TPB>(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}
__global__ void __launch_bounds__(TPB) k_sum_final(const double* part, int np, double* out, int is_min) {
  double acc = is_min ? 1e300 : 0.0;
  for (int i = threadIdx.x; i < np; i += TPB) acc = is_min ? nan_min(acc, part[i]) : acc + part[i];
  acc = is_min ? block_min<TPB>(acc) : block_sum<TPB>(acc);
  if (threadIdx.x == 0) *out = acc;
}

int launch_min_final(ilh_ctx* c, const double* part, int np, double* out) {
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(TPB), 0, c->stream, part, np, out, 1);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

static int red_blocks(ilh_ctx* c, int64_t n) {
  int b = (int)std::min<int64_t>((n + TPB - 1) / TPB, c->red_blocks);
  return b < 1 ? 1 : b;
}

int dot_dev(ilh_ctx* c, const double* x, const double* y, int64_t n, double* d_out) {
  const int nb = red_blocks(c, n);
  hipLaunchKernelGGL(k_dot_part, dim3(nb), dim3(TPB), 0, c->stream, x, y, n, c->red, x, y, c->red);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(TPB), 0, c->stream, c->red, nb, d_out, 0);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

int dot_part(ilh_ctx* c, const double* x, const double* y, int64_t n, double* part, int* np) {
  const int nb = red_blocks(c, n);
  hipLaunchKernelGGL(k_dot_part, dim3(nb), dim3(TPB), 0, c->stream, x, y, n, part, x, y, part);
  ILH_HIP(c, hipGetLastError());
  *np = nb;
  return ILH_OK;
}
int dot_part2(ilh_ctx* c, const double* x, const double* y, const double* x2, const double* y2, int64_t n,
              double* part, double* part2, int* np) {
  const int nb = red_blocks(c, n);
  hipLaunchKernelGGL(k_dot_part, dim3(nb, 2), dim3(TPB), 0, c->stream, x, y, n, part, x2, y2, part2);
  ILH_HIP(c, hipGetLastError());
  *np = nb;
  return ILH_OK;
}

// Two reductions of partial sums finished in one launch: out[0] = the sum (ma = 0) or the
// minimum (ma = 1) of pa[0..na), out[1] likewise of pb; out may be host-mapped memory, read once
// the stream has synchronised
__global__ void __launch_bounds__(TPB) k_pair_final(const double* pa, int na, int ma, const double* pb, int nb,
                                                    int mb, double* out) {
  double a = ma ? 1e300 : 0.0, b = mb ? 1e300 : 0.0;
  for (int i = threadIdx.x; i < na; i += TPB) a = ma ? nan_min(a, pa[i]) : a + pa[i];
  for (int i = threadIdx.x; i < nb; i += TPB) b = mb ? nan_min(b, pb[i]) : b + pb[i];
  a = ma ? block_min<TPB>(a) : block_sum<TPB>(a);
  b = mb ? block_min<TPB>(b) : block_sum<TPB>(b);
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = b;
    __threadfence_system();
  }
}

int launch_pair_final(ilh_ctx* c, const double* pa, int na, int ma, const double* pb, int nb, int mb, double* out) {
  hipLaunchKernelGGL(k_pair_final, dim3(1), dim3(TPB), 0, c->stream, pa, na, ma, pb, nb, mb, out);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

int dot_host(ilh_ctx* c, const double* x, const double* y, int64_t n, double* out) {
  double* d_out = c->red + c->red_blocks * 65;  // scalar slots after the partials
  int st = dot_dev(c, x, y, n, d_out);
  if (st) return st;
  ILH_HIP(c, hipMemcpyAsync(c->red_host, d_out, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  ILH_HIP(c, hipStreamSynchronize(c->stream));
  *out = c->red_host[0];
  return ILH_OK;
}

// out[j] = s_j sum_b part[j][b] (s = null: s_j = 1); outs (nullable) receives s_j out[j], the
// coefficient of the stored vector when V_j = s_j x (stored vector)
__global__ void __launch_bounds__(TPB) k_mdot_final(const double* part, int nb, int m, double* out,
                                                    const double* s, double* outs, const double* skip) {
  if (skip && *skip != 0.0) return;
  const int j = blockIdx.x;
  double acc = 0;
  for (int i = threadIdx.x; i < nb; i += TPB) acc += part[(int64_t)j * nb + i];
  acc = block_sum<TPB>(acc);
  if (threadIdx.x == 0) {
    const double sj = s ? s[j] : 1.0;
    out[j] = sj * acc;
    if (outs) outs[j] = sj * sj * acc;
  }
}
// w[i] += sign * sum_j h[j] V[j][i] (FP64 sums; the basis V stored in FP64 or FP32)
template <typename TV>
__global__ void k_maxpy(double* w, const TV* V, int64_t ldv, int m, const double* h, double sign, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0;
    for (int j = 0; j < m; ++j) acc += h[j] * (double)V[(int64_t)j * ldv + i];
    w[i] += sign * acc;
  }
}
template <typename TV>
int multiaxpy_dev(ilh_ctx* c, double* w, const TV* V, int64_t ldv, int m, const double* h, double sign, int64_t n) {
  if (m <= 0) return ILH_OK;
  hipLaunchKernelGGL(k_maxpy<TV>, dim3(nblk(n)), dim3(TPB), 0, c->stream, w, V, ldv, m, h, sign, n);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}
template int multiaxpy_dev<double>(ilh_ctx*, double*, const double*, int64_t, int, const double*, double, int64_t);
template int multiaxpy_dev<float>(ilh_ctx*, double*, const float*, int64_t, int, const double*, double, int64_t);

// ------------------------------------------------------------------ fused Krylov kernels
// Partial sums per block, then one small kernel adds them in a fixed order (deterministic).
// A single-launch variant with a last-block arrival counter was measured slower: the
// device-scope release fence it needs writes back each XCD's L2 once per block.
static constexpr int MDOT_JC = 8;  // basis vectors per pass over w
static constexpr int KU = 4;       // elements per thread and tile
static constexpr int64_t KTILE = (int64_t)TPB * KU;

// The sweeps below take the basis in chunks of MDOT_JC vectors and the elements in tiles of
// KU per thread; every load of a chunk and tile is issued before its first use (row and element
// indices are clamped in range, out-of-range terms enter with weight zero), so a wave keeps
// MDOT_JC x KU loads in flight instead of one row at a time.

// a[u] += sum_{j < m} cf[j] V_j[i_u] over one tile (i_u clamped to n - 1); the basis is stored in
// FP64 or FP32, every product and sum is FP64
template <typename TV>
__device__ __forceinline__ void tile_combo(const TV* __restrict__ V, int64_t ldv, int m,
                                           const double* __restrict__ cf, const int64_t (&ic)[KU],
                                           double (&a)[KU]) {
  for (int j0 = 0; j0 < m; j0 += MDOT_JC) {
    double v[MDOT_JC][KU];
    double cj[MDOT_JC];
#pragma unroll
    for (int jj = 0; jj < MDOT_JC; ++jj) {
      const int j = min(j0 + jj, m - 1);
      cj[jj] = (j0 + jj < m) ? cf[j] : 0.0;
#pragma unroll
      for (int u = 0; u < KU; ++u) v[jj][u] = (double)V[(int64_t)j * ldv + ic[u]];
    }
#pragma unroll
    for (int jj = 0; jj < MDOT_JC; ++jj)
#pragma unroll
      for (int u = 0; u < KU; ++u) a[u] += cj[jj] * v[jj][u];
  }
}

// acc[jj] += sum_u V_{j0+jj}[i_u] wv[u] for jj < MDOT_JC (rows past m - 1 clamped; the caller
// discards their sums)
template <typename TV>
__device__ __forceinline__ void tile_dots(const TV* __restrict__ V, int64_t ldv, int m, int j0,
                                          const int64_t (&ic)[KU], const double (&wv)[KU],
                                          double (&acc)[MDOT_JC]) {
  double v[MDOT_JC][KU];
#pragma unroll
  for (int jj = 0; jj < MDOT_JC; ++jj) {
    const int j = min(j0 + jj, m - 1);
#pragma unroll
    for (int u = 0; u < KU; ++u) v[jj][u] = (double)V[(int64_t)j * ldv + ic[u]];
  }
#pragma unroll
  for (int jj = 0; jj < MDOT_JC; ++jj)
#pragma unroll
    for (int u = 0; u < KU; ++u) acc[jj] += v[jj][u] * wv[u];
}

__device__ __forceinline__ void tile_index(int64_t t0, int64_t n, int64_t (&ic)[KU], bool (&in)[KU]) {
#pragma unroll
  for (int u = 0; u < KU; ++u) {
    const int64_t i = t0 + (int64_t)u * TPB + threadIdx.x;
    in[u] = i < n;
    ic[u] = in[u] ? i : n - 1;
  }
}

// x[i_u] for one tile, 0 past n: the loads are unconditional (i_u is clamped in range) and only
// the value is selected, so they are issued together; a load under the range test compiles to a
// branch with a wait for each element
template <typename TV>
__device__ __forceinline__ void tile_load(const TV* __restrict__ x, const int64_t (&ic)[KU], const bool (&in)[KU],
                                          double (&v)[KU]) {
  double t[KU];
#pragma unroll
  for (int u = 0; u < KU; ++u) t[u] = (double)x[ic[u]];
#pragma unroll
  for (int u = 0; u < KU; ++u) v[u] = in[u] ? t[u] : 0.0;
}

// Sums of K values (K a power of two, at most 64) over the 64 lanes of a wave.  Each exchange
// pairs lane l with l ^ mask and halves the values a lane holds (it keeps one half, adds the
// partner's copy of that half): K - 1 + (6 - log2 K) shuffles instead of 6 K.  Afterwards every
// lane holds in acc[0] the complete sum of the value index returned (the lanes that differ only
// in their low 6 - log2 K bits hold the same one).
template <int CNT, int MASK, int K>
__device__ __forceinline__ void wave_sums_r(double (&acc)[K], int lane, int& v) {
  if constexpr (MASK >= 1) {
    const bool hi = (lane & MASK) != 0;
    if constexpr (CNT > 1) {
      constexpr int HALF = CNT / 2;
#pragma unroll
      for (int i = 0; i < HALF; ++i) {
        const double send = hi ? acc[i] : acc[i + HALF];
        const double keep = hi ? acc[i + HALF] : acc[i];
        acc[i] = keep + __shfl_xor(send, MASK, 64);
      }
      if (hi) v += HALF;
      wave_sums_r<HALF, MASK / 2, K>(acc, lane, v);
    } else {
      acc[0] += __shfl_xor(acc[0], MASK, 64);
      wave_sums_r<1, MASK / 2, K>(acc, lane, v);
    }
  }
}

template <int K>
__device__ __forceinline__ int wave_sums(double (&acc)[K]) {
  static_assert(K >= 1 && K <= 64 && (K & (K - 1)) == 0, "K: a power of two up to 64");
  int v = 0;
  wave_sums_r<K, 32, K>(acc, (int)(threadIdx.x & 63), v);
  return v;
}

// part[(j0 + jj) * gridDim.x + blockIdx.x] = block sum of acc[jj], jj < jn
template <int JC>
__device__ __forceinline__ void store_block_sums(double (&acc)[JC], int j0, int jn, double* part) {
  __shared__ double sh[TPB / 64][JC];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int v = wave_sums<JC>(acc);
  if ((lane & (64 / JC - 1)) == 0) sh[wid][v] = acc[0];
  __syncthreads();
  const int q = threadIdx.x;
  if (q < jn) {
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < TPB / 64; ++i) r += sh[i][q];
    part[(int64_t)(j0 + q) * gridDim.x + blockIdx.x] = r;
  }
  __syncthreads();
}

// part[j][b] = block b's share of V_j . w, j < m (w read once per MDOT_JC vectors)
template <typename TV>
__global__ void __launch_bounds__(TPB) k_mdot_part8(const TV* __restrict__ V, int64_t ldv, int m,
                                                    const TV* __restrict__ w, int64_t n, double* part,
                                                    const double* skip) {
  if (skip && *skip != 0.0) return;
  const int64_t stride = (int64_t)gridDim.x * KTILE;
  for (int j0 = 0; j0 < m; j0 += MDOT_JC) {
    double acc[MDOT_JC];
#pragma unroll
    for (int jj = 0; jj < MDOT_JC; ++jj) acc[jj] = 0.0;
    for (int64_t t0 = (int64_t)blockIdx.x * KTILE; t0 < n; t0 += stride) {
      int64_t ic[KU];
      bool in[KU];
      tile_index(t0, n, ic, in);
      double wv[KU];
      tile_load(w, ic, in, wv);
      tile_dots(V, ldv, m, j0, ic, wv, acc);
    }
    store_block_sums(acc, j0, min(MDOT_JC, m - j0), part);
  }
}

// w -= sum_j cf[j] V_j, then part[j][b] = block b's share of V_j . w (the updated w), j < m:
// the first Gram-Schmidt pass's update and the second pass's products in one sweep.  Every
// thread revisits only its own indices, so the later chunks read back its own updates.
template <typename TV>
__global__ void __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(3))) k_maxpy_mdot_part(TV* __restrict__ w, const TV* __restrict__ V,
                                                         int64_t ldv, int m, const double* __restrict__ cf,
                                                         int64_t n, double* part, const double* skip) {
  if (skip && *skip != 0.0) return;
  const int64_t stride = (int64_t)gridDim.x * KTILE;
  for (int j0 = 0; j0 < m; j0 += MDOT_JC) {
    double acc[MDOT_JC];
#pragma unroll
    for (int jj = 0; jj < MDOT_JC; ++jj) acc[jj] = 0.0;
    for (int64_t t0 = (int64_t)blockIdx.x * KTILE; t0 < n; t0 += stride) {
      int64_t ic[KU];
      bool in[KU];
      tile_index(t0, n, ic, in);
      double wv[KU];
      if (j0 == 0) {
        // the first chunk's rows stay in registers for its products with the updated w
        double v0[MDOT_JC][KU], a[KU];
#pragma unroll
        for (int jj = 0; jj < MDOT_JC; ++jj) {
          const int j = min(jj, m - 1);
#pragma unroll
          for (int u = 0; u < KU; ++u) v0[jj][u] = (double)V[(int64_t)j * ldv + ic[u]];
        }
#pragma unroll
        for (int u = 0; u < KU; ++u) a[u] = 0.0;
#pragma unroll
        for (int jj = 0; jj < MDOT_JC; ++jj) {
          const double cj = jj < m ? cf[min(jj, m - 1)] : 0.0;
#pragma unroll
          for (int u = 0; u < KU; ++u) a[u] += cj * v0[jj][u];
        }
        if (m > MDOT_JC) tile_combo(V + MDOT_JC * ldv, ldv, m - MDOT_JC, cf + MDOT_JC, ic, a);
        double wo[KU];
        tile_load(w, ic, in, wo);
#pragma unroll
        for (int u = 0; u < KU; ++u) {
          // the stored (rounded) value is the one the products take, as a later pass reads it
          const TV wn = (TV)(wo[u] - a[u]);
          if (in[u]) w[ic[u]] = wn;
          wv[u] = in[u] ? (double)wn : 0.0;
        }
#pragma unroll
        for (int jj = 0; jj < MDOT_JC; ++jj)
#pragma unroll
          for (int u = 0; u < KU; ++u) acc[jj] += v0[jj][u] * wv[u];
      } else {
        tile_load(w, ic, in, wv);
        tile_dots(V, ldv, m, j0, ic, wv, acc);
      }
    }
    store_block_sums(acc, j0, min(MDOT_JC, m - j0), part);
  }
}

// w += sign sum_j h[j] V_j; part[b] = block b's share of |w|^2 of the result
template <typename TV>
__global__ void __launch_bounds__(TPB) k_maxpy_nrm_part(TV* __restrict__ w, const TV* __restrict__ V,
                                                        int64_t ldv, int m, const double* __restrict__ h,
                                                        double sign, int64_t n, double* part,
                                                        const double* skip) {
  if (skip && *skip != 0.0) return;
  double ss = 0.0;
  const int64_t stride = (int64_t)gridDim.x * KTILE;
  for (int64_t t0 = (int64_t)blockIdx.x * KTILE; t0 < n; t0 += stride) {
    int64_t ic[KU];
    bool in[KU];
    tile_index(t0, n, ic, in);
    double a[KU];
#pragma unroll
    for (int u = 0; u < KU; ++u) a[u] = 0.0;
    tile_combo(V, ldv, m, h, ic, a);
    double wo[KU];
    tile_load(w, ic, in, wo);
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const TV wn = (TV)(wo[u] + sign * a[u]);
      const double wd = (double)wn;
      ss += in[u] ? wd * wd : 0.0;  // the norm of the stored vector
      if (in[u]) w[ic[u]] = wn;
    }
  }
  ss = block_sum<TPB>(ss);
  if (threadIdx.x == 0) part[blockIdx.x] = ss;
}

static int fused_blocks(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(1024, (n + KTILE - 1) / KTILE));
}

template <typename TV>
int multidot_fused(ilh_ctx* c, const TV* V, int64_t ldv, int m, const TV* w, int64_t n, double* d_out,
                   const double* s, double* d_outs, const double* skip) {
  if (m <= 0) return ILH_OK;
  if (m > 64) return fail(c, ILH_EINVAL, "multidot: at most 64 vectors");
  const int nb = fused_blocks(n);
  hipLaunchKernelGGL(k_mdot_part8<TV>, dim3(nb), dim3(TPB), 0, c->stream, V, ldv, m, w, n, c->red, skip);
  hipLaunchKernelGGL(k_mdot_final, dim3(m), dim3(TPB), 0, c->stream, c->red, nb, m, d_out, s, d_outs, skip);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

template <typename TV>
int maxpy_multidot(ilh_ctx* c, TV* w, const TV* V, int64_t ldv, int m, const double* cf, int64_t n,
                   const double* s, double* d_out, double* d_outs, const double* skip) {
  if (m <= 0) return ILH_OK;
  if (m > 64) return fail(c, ILH_EINVAL, "multidot: at most 64 vectors");
  const int nb = fused_blocks(n);
  hipLaunchKernelGGL(k_maxpy_mdot_part<TV>, dim3(nb), dim3(TPB), 0, c->stream, w, V, ldv, m, cf, n, c->red, skip);
  hipLaunchKernelGGL(k_mdot_final, dim3(m), dim3(TPB), 0, c->stream, c->red, nb, m, d_out, s, d_outs, skip);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

__device__ void givens_update(double* h, double* G, int j, int m, const double* csl, const double* snl,
                              const double* coll);

// The residual estimate and h_{j+1,j} of column j to host memory (mapped, coherent) as two 16-byte
// records {estimate, tag} and {h_{j+1,j}, tag}: each record is one store, so the host never pairs
// a new tag with an old value whatever order the two stores become visible in
__device__ __forceinline__ void publish_estimate(double* hest, int j, double est, double hn, double tag) {
  double2* rec = reinterpret_cast<double2*>(hest + 4 * j);
  rec[0] = make_double2(est, tag);
  rec[1] = make_double2(hn, tag);
  __threadfence_system();
}

// final sum of the norm partials into h[144], the Givens update of Arnoldi step j, and the
// scale of the next basis vector, h[256 + j + 1] = 1 / |w| (1 for a zero or non-finite norm:
// the cycle ends at that step).  The residual estimate also goes straight to host memory
// (hest, mapped and coherent) with the cycle's tag h[255] (publish_estimate), which the host
// polls: no copy and no event are enqueued behind the step.
__device__ __forceinline__ void sum_givens_block(const GivensJob& g) {
  if (g.skip && *g.skip != 0.0) return;
  // the earlier rotations and the new Hessenberg column go to LDS while the partials are summed,
  // so the one thread that applies the rotations reads no global memory in its chain
  __shared__ double csl[64], snl[64], coll[64];
  double* h = g.h;
  const int j = g.j;
  const double* cs = g.G + 64 * 64;
  if ((int)threadIdx.x < j) {
    csl[threadIdx.x] = cs[threadIdx.x];
    snl[threadIdx.x] = cs[64 + threadIdx.x];
  }
  if ((int)threadIdx.x <= j) coll[threadIdx.x] = h[threadIdx.x] + h[72 + threadIdx.x];
  double acc = 0.0;
  for (int i = threadIdx.x; i < g.np; i += TPB) acc += g.part[i];
  acc = block_sum<TPB>(acc);  // its barriers also publish the LDS stores
  if (threadIdx.x == 0) {
    h[144] = acc;
    givens_update(h, g.G, j, g.m, csl, snl, coll);
    const double hn = sqrt(fmax(acc, 0.0));
    h[256 + j + 1] = (hn > 0.0 && hn <= 1.7e308) ? 1.0 / hn : 1.0;
    // the end test the host makes on the same two numbers (estimate at most the target, or a
    // zero norm), so a step the host discards does no work
    h[HDEV_FLAG + j] = (h[352 + 2 * j] <= h[252] || h[353 + 2 * j] == 0.0) ? 1.0 : 0.0;
    if (g.hest) {
      publish_estimate(g.hest, j, h[352 + 2 * j], h[353 + 2 * j], h[255]);
    }
  }
}

__global__ void __launch_bounds__(TPB) k_sum_givens(const GivensJob g) { sum_givens_block(g); }

// The scale 1 / |w| that sum_givens_block stores for the next basis vector, formed by a whole
// block from the same partial sums in the same order (so every block obtains the same value)
__device__ __forceinline__ double scale_from_partials(const double* part, int np) {
  __shared__ double sh_sc;
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += TPB) acc += part[i];
  acc = block_sum<TPB>(acc);
  if (threadIdx.x == 0) {
    const double hn = sqrt(fmax(acc, 0.0));
    sh_sc = (hn > 0.0 && hn <= 1.7e308) ? 1.0 / hn : 1.0;
  }
  __syncthreads();
  return sh_sc;
}

// y *= *s
__global__ void k_scale_dev(double* y, const double* s, int64_t n) {
  const double f = *s;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] *= f;
}

int launch_scale_dev(ilh_ctx* c, double* y, const double* s, int64_t n) {
  hipLaunchKernelGGL(k_scale_dev, dim3(nblk(n, 4096)), dim3(TPB), 0, c->stream, y, s, n);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

template <typename TV>
int multiaxpy_nrm(ilh_ctx* c, TV* w, const TV* V, int64_t ldv, int m, const double* cf, double sign,
                  int64_t n, double* h, double* G, int j, int mm, double* hest, GivensJob* job,
                  const double* skip) {
  const int nb = fused_blocks(n);
  hipLaunchKernelGGL(k_maxpy_nrm_part<TV>, dim3(nb), dim3(TPB), 0, c->stream, w, V, ldv, m, cf, sign, n, c->red, skip);
  ILH_HIP(c, hipGetLastError());
  *job = GivensJob{c->red, nb, h, G, j, mm, hest, skip};
  return ILH_OK;
}

template int multidot_fused<double>(ilh_ctx*, const double*, int64_t, int, const double*, int64_t, double*,
                                    const double*, double*, const double*);
template int multidot_fused<float>(ilh_ctx*, const float*, int64_t, int, const float*, int64_t, double*,
                                   const double*, double*, const double*);
template int maxpy_multidot<double>(ilh_ctx*, double*, const double*, int64_t, int, const double*, int64_t,
                                    const double*, double*, double*, const double*);
template int maxpy_multidot<float>(ilh_ctx*, float*, const float*, int64_t, int, const double*, int64_t,
                                   const double*, double*, double*, const double*);
template int multiaxpy_nrm<double>(ilh_ctx*, double*, const double*, int64_t, int, const double*, double, int64_t,
                                   double*, double*, int, int, double*, GivensJob*, const double*);
template int multiaxpy_nrm<float>(ilh_ctx*, float*, const float*, int64_t, int, const double*, double, int64_t,
                                  double*, double*, int, int, double*, GivensJob*, const double*);

int launch_sum_givens(ilh_ctx* c, const GivensJob& job) {
  hipLaunchKernelGGL(k_sum_givens, dim3(1), dim3(TPB), 0, c->stream, job);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}


// Givens update of Arnoldi step j on the device (one thread; j < m <= 64).  Column j of the
// Hessenberg matrix is the sum of the two Gram-Schmidt passes (coll[0..j] = h[0..j] +
// h[72..72+j], staged by the caller with the earlier rotations csl, snl = cs[0..j), sn[0..j)) with
// h_{j+1,j} = sqrt(h[144]); the earlier rotations are applied to it, the new one is formed and
// applied to the right-hand side g (g = beta e_1 at j = 0, beta in h[240]); the residual
// estimate |g_{j+1}| and h_{j+1,j} go to h[352 + 2j], h[353 + 2j].
// G layout: H [64][64] row-major (upper triangle after the rotations), cs [64], sn [64], g [65].
// givens_col: the same with h_{j+1,j} = hn given.
__device__ void givens_col(double* h, double* G, int j, int m, const double* csl, const double* snl,
                           const double* coll, double hn) {
  double* H = G;
  double* cs = G + 64 * 64;
  double* sn = cs + 64;
  double* g = sn + 64;
  if (j == 0) {
    g[0] = h[240];
    for (int i = 1; i <= m; ++i) g[i] = 0.0;
  }
  double cur = coll[0];
  for (int i = 0; i < j; ++i) {
    const double nx = coll[i + 1];
    H[i * 64 + j] = csl[i] * cur + snl[i] * nx;
    cur = -snl[i] * cur + csl[i] * nx;
  }
  const double den = hypot(cur, hn);
  const double c_ = den > 0 ? cur / den : 1.0, s_ = den > 0 ? hn / den : 0.0;
  cs[j] = c_;
  sn[j] = s_;
  H[j * 64 + j] = den;
  g[j + 1] = -s_ * g[j];
  g[j] = c_ * g[j];
  h[352 + 2 * j] = fabs(g[j + 1]);
  h[353 + 2 * j] = hn;
}

__device__ void givens_update(double* h, double* G, int j, int m, const double* csl, const double* snl,
                              const double* coll) {
  givens_col(h, G, j, m, csl, snl, coll, sqrt(fmax(h[144], 0.0)));
}


// y = H(0:n, 0:n)^-1 g(0:n) by back substitution (one thread)
__global__ void k_trisolve(const double* G, int n, double* y) {
  if (threadIdx.x != 0) return;
  const double* H = G;
  const double* g = G + 64 * 64 + 128;
  for (int i = n - 1; i >= 0; --i) {
    double acc = g[i];
    for (int l = i + 1; l < n; ++l) acc -= H[i * 64 + l] * y[l];
    y[i] = H[i * 64 + i] != 0 ? acc / H[i * 64 + i] : 0.0;
  }
}


// x += sum_{j < jn} y_j Z_j with y = H(0:jn, 0:jn)^-1 g(0:jn): every block repeats the small
// triangular solve (operands staged in LDS; one wave back-substitutes column by column, lane l
// holding row l of the right-hand side) and then takes its share of the update
template <typename TV>
__global__ void __launch_bounds__(TPB) k_trisolve_maxpy(double* __restrict__ x, const TV* __restrict__ Z,
                                                        int64_t ldz, const double* __restrict__ G, int jn, int64_t n,
                                                        int accumulate) {
  extern __shared__ double tsh[];  // H (jn x jn, row-major), then y (jn)
  double* Hs = tsh;
  double* ys = tsh + jn * jn;
  for (int t = threadIdx.x; t < jn * jn; t += TPB) Hs[t] = G[(t / jn) * 64 + t % jn];
  __syncthreads();
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    double rhs = lane < jn ? G[64 * 64 + 128 + lane] : 0.0;
    for (int i = jn - 1; i >= 0; --i) {
      const double num = __shfl(rhs, i, 64);
      const double hii = Hs[i * jn + i];
      const double yi = hii != 0.0 ? num / hii : 0.0;
      if (lane == i) ys[i] = yi;
      if (lane < i) rhs -= Hs[lane * jn + i] * yi;
    }
  }
  __syncthreads();
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0;
    for (int j = 0; j < jn; ++j) acc += ys[j] * (double)Z[(int64_t)j * ldz + i];
    x[i] = accumulate ? x[i] + acc : acc;
  }
}

template <typename TV>
int launch_trisolve_maxpy(ilh_ctx* c, double* x, const TV* Z, int64_t ldz, const double* G, int jn, int64_t n,
                          bool accumulate) {
  if (jn <= 0) return accumulate ? ILH_OK : launch_fill(c, x, 0.0, n);
  if (jn > 64) return fail(c, ILH_EINVAL, "triangular solve: at most 64 columns");
  const size_t shm = (size_t)(jn * jn + jn) * sizeof(double);
  hipLaunchKernelGGL(k_trisolve_maxpy<TV>, dim3(std::min(nblk(n), 1024)), dim3(TPB), shm, c->stream, x, Z, ldz, G, jn,
                     n, accumulate ? 1 : 0);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}
template int launch_trisolve_maxpy<double>(ilh_ctx*, double*, const double*, int64_t, const double*, int, int64_t,
                                          bool);
template int launch_trisolve_maxpy<float>(ilh_ctx*, double*, const float*, int64_t, const double*, int, int64_t,
                                         bool);

int launch_trisolve(ilh_ctx* c, const double* G, int m, int n, double* y) {
  (void)m;
  hipLaunchKernelGGL(k_trisolve, dim3(1), dim3(64), 0, c->stream, G, n, y);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

// ------------------------------------------------------------------ Gram-Schmidt with the second
// pass lagged one step (Sec. 3.5: the FGMRES solve of eq. newton_linear)
// On entry to Arnoldi step j the basis slots hold v_0 .. v_{j-1} (orthonormal) and u_j, the
// vector step j - 1 orthogonalised once against them and stored times s_j = 1 / |w_{j-1}|,
// and z_j = P u_j.  With w = J z_j:
//   dot sweep    a_k = v_k . u_j, b_k = v_k . w (k < j), |u_j|^2, u_j . w and |w|^2, in one pass
//   final block  rho_j = (|u_j|^2 - |a|^2)^(1/2) and v_j = (u_j - V a) / rho_j (the second
//                pass for u_j); u_j / s_j = (V a + rho_j v_j) / s_j, so column j - 1 of the
//                Hessenberg matrix is step j - 1's first-pass coefficients plus (a, rho_j) / s_j,
//                which the Givens update then takes; v_j . w = (u_j . w - a . b) / rho_j = d
//   update sweep v_j stored, u_{j+1} = s_{j+1} (w - V b - d v_j) (the first pass for w) stored,
//                and z_{j+1} = P u_{j+1} (the block preconditioner) with it
// The scale s_{j+1} = 1 / |w| keeps the stored vectors and the next action's input of order one
// (unscaled, the vectors grow by |J P| every step and leave the FP32 range).
// The two Gram-Schmidt passes of every vector are those of classical Gram-Schmidt twice; the
// second pass of u_j shares the sweeps of the first pass of w, so a step reads the basis twice.
// v_0 = r / |r| is taken as it is stored (rho_0 = 1).  Column j - 1 is finished by step j, so
// the residual estimate lags one step, and a cycle that ends at column L - 1 runs a closing
// step L (dot sweep on u_L and the final block only).
// Partial sums of the dot sweep: part[s][block], s = 2k (a_k), 2k + 1 (b_k), 2j (|u_j|^2),
// 2j + 1 (u_j . w), 2j + 2 (|w|^2).
static constexpr int LGS_NS = 2 * MDOT_JC + 3;
static constexpr int LGS_NP = 32;  // LGS_NS padded to a power of two for wave_sums

// LGS_DB threads per work-group: a quarter as many partial sums as 256-thread groups would leave
// for the final block, with the same number of waves
static constexpr int LGS_DB = 1024;
static constexpr int64_t LGS_DT = (int64_t)LGS_DB * KU;

template <typename TV>
__global__ void __launch_bounds__(LGS_DB) k_lgs_dots(const TV* __restrict__ V, int64_t ldv, int j,
                                                  const TV* __restrict__ uj, const TV* __restrict__ w,
                                                  int64_t n, double* part, const double* skip) {
  if (skip && *skip != 0.0) return;
  __shared__ double sh[LGS_DB / 64][LGS_NP];
  const int64_t stride = (int64_t)gridDim.x * LGS_DT;
  const int nch = j > 0 ? (j + MDOT_JC - 1) / MDOT_JC : 1;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int ch = 0; ch < nch; ++ch) {
    const int k0 = ch * MDOT_JC;
    double acc[LGS_NP];
#pragma unroll
    for (int q = 0; q < LGS_NP; ++q) acc[q] = 0.0;
    for (int64_t t0 = (int64_t)blockIdx.x * LGS_DT; t0 < n; t0 += stride) {
      int64_t ic[KU];
      bool in[KU];
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        const int64_t i = t0 + (int64_t)u * LGS_DB + threadIdx.x;
        in[u] = i < n;
        ic[u] = in[u] ? i : n - 1;
      }
      double uv[KU], wv[KU];
      tile_load(uj, ic, in, uv);
      tile_load(w, ic, in, wv);
      if (ch == 0) {
#pragma unroll
        for (int u = 0; u < KU; ++u) {
          acc[2 * MDOT_JC] += uv[u] * uv[u];
          acc[2 * MDOT_JC + 1] += uv[u] * wv[u];
          acc[2 * MDOT_JC + 2] += wv[u] * wv[u];
        }
      }
      if (j > 0) {
        double v[MDOT_JC][KU];
#pragma unroll
        for (int jj = 0; jj < MDOT_JC; ++jj) {
          const int k = min(k0 + jj, j - 1);
#pragma unroll
          for (int u = 0; u < KU; ++u) v[jj][u] = (double)V[(int64_t)k * ldv + ic[u]];
        }
#pragma unroll
        for (int jj = 0; jj < MDOT_JC; ++jj)
#pragma unroll
          for (int u = 0; u < KU; ++u) {
            acc[2 * jj] += v[jj][u] * uv[u];
            acc[2 * jj + 1] += v[jj][u] * wv[u];
          }
      }
    }
    // every sum reduced across its wave, then across the block's waves in a fixed order
    const int v = wave_sums<LGS_NP>(acc);
    if ((lane & (64 / LGS_NP - 1)) == 0) sh[wid][v] = acc[0];
    __syncthreads();
    const int q = threadIdx.x;
    if (q < LGS_NS) {
      int sidx = -1;
      if (q < 2 * MDOT_JC) {
        if (k0 + q / 2 < j) sidx = 2 * (k0 + q / 2) + (q & 1);
      } else if (ch == 0) {
        sidx = 2 * j + (q - 2 * MDOT_JC);
      }
      if (sidx >= 0) {
        double r = 0.0;
#pragma unroll
        for (int i = 0; i < LGS_DB / 64; ++i) r += sh[i][q];
        part[(int64_t)sidx * gridDim.x + blockIdx.x] = r;
      }
    }
    __syncthreads();
  }
}

// The same sweep with the basis count fixed at compile time: one pass over u_j, w and the basis,
// no loads for the missing vectors of a padded chunk.  Up to 7 vectors are one group of sums;
// j = N0 + N1 vectors beyond that are two chunks side by side (grid row 0: vectors [0, N0), the
// norms and u_j . w; row 1: vectors [N0, j)), so u_j and w are read twice but in parallel.
// Sums in the layout above (part[s][block]).
static constexpr int LGS_NVMAX = 15;

template <typename TV, int NV, bool NORMS>
__device__ __forceinline__ void lgs_dots_tile(const TV* __restrict__ V, int64_t ldv, int k0, int j,
                                              const TV* __restrict__ uj, const TV* __restrict__ w, int64_t n,
                                              double* part) {
  constexpr int NA = 2 * NV + (NORMS ? 3 : 0);
  constexpr int NP = NA <= 4 ? 4 : NA <= 8 ? 8 : NA <= 16 ? 16 : 32;
  static_assert(NA <= 32, "at most 32 sums per group");
  __shared__ double sh[LGS_DB / 64][NP];
  const int64_t stride = (int64_t)gridDim.x * LGS_DT;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double acc[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) acc[q] = 0.0;
  for (int64_t t0 = (int64_t)blockIdx.x * LGS_DT; t0 < n; t0 += stride) {
    // 32-bit offsets from wave-uniform bases (n sizeof(TV) < 4 GiB, checked on the host); the
    // basis loads first, then u_j and w, all in flight before the first product
    uint32_t io[KU];
    bool in[KU];
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int64_t i = t0 + (int64_t)u * LGS_DB + threadIdx.x;
      in[u] = i < n;
      io[u] = (uint32_t)(in[u] ? i : n - 1);
    }
    TV vr[NV > 0 ? NV : 1][KU];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const TV* vk = sbase(V + (int64_t)(k0 + k) * ldv);
#pragma unroll
      for (int u = 0; u < KU; ++u) vr[k][u] = ld32(vk, io[u]);
    }
    TV ur[KU], wr[KU];
    const TV* ub = sbase(uj);
    const TV* wb = sbase(w);
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      ur[u] = ld32(ub, io[u]);
      wr[u] = ld32(wb, io[u]);
    }
    double uv[KU], wv[KU];
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      uv[u] = in[u] ? (double)ur[u] : 0.0;
      wv[u] = in[u] ? (double)wr[u] : 0.0;
    }
    if constexpr (NORMS) {
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        acc[2 * NV] += uv[u] * uv[u];
        acc[2 * NV + 1] += uv[u] * wv[u];
        acc[2 * NV + 2] += wv[u] * wv[u];
      }
    }
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
      for (int u = 0; u < KU; ++u) {
        acc[2 * k] += (double)vr[k][u] * uv[u];
        acc[2 * k + 1] += (double)vr[k][u] * wv[u];
      }
  }
  const int v = wave_sums<NP>(acc);
  if ((lane & (64 / NP - 1)) == 0) sh[wid][v] = acc[0];
  __syncthreads();
  const int q = threadIdx.x;
  if (q < NA) {
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < LGS_DB / 64; ++i) r += sh[i][q];
    const int sidx = q < 2 * NV ? 2 * k0 + q : 2 * j + (q - 2 * NV);
    part[(int64_t)sidx * gridDim.x + blockIdx.x] = r;
  }
}

template <typename TV, int N0, int N1>
__global__ void __launch_bounds__(LGS_DB) k_lgs_dots_n(const TV* __restrict__ V, int64_t ldv,
                                                    const TV* __restrict__ uj, const TV* __restrict__ w,
                                                    int64_t n, double* part, const double* skip) {
  // (the flag is read first: the sweep is bound by its loads, which a launch after the end of
  // the cycle would otherwise still wait for)
  if (skip && *skip != 0.0) return;
  if (N1 == 0 || blockIdx.y == 0)
    lgs_dots_tile<TV, N0, true>(V, ldv, 0, N0 + N1, uj, w, n, part);
  else
    lgs_dots_tile<TV, N1, false>(V, ldv, N0, N0 + N1, uj, w, n, part);
}

// Final block of step j (one work-group of LGS_FT threads): the sums, the second pass's scale,
// column j - 1 with its Givens update and residual estimate (to h[352 + 2(j-1)]; to host memory
// with the cycle's tag (publish_estimate) by the update sweep, or here on the closing step), the
// cycle-end flag h[HDEV_LGSE] = j + 1 when column j - 1 met the target or rho_j = 0 (every later
// launch of the cycle then returns at once), and the update sweep's coefficients: a at h[0..j), b at h[72..72+j), 1 / rho_j at
// h[144], d at h[145], s_{j+1} at h[146]; step j's first-pass coefficients (b, d) go to
// h[HDEV_LGSP..+j] and 1 / s_{j+1} to h[HDEV_LGSP + 65] for step j + 1.  has_w = 0: the closing
// step (no w, no update).
static constexpr int LGS_FT = 1024;  // threads of the final block

__global__ void __launch_bounds__(LGS_FT) k_lgs_final(const double* __restrict__ part, int np, int j, int m,
                                                      int has_w, double* h, double* G, double* hest,
                                                      const double* skip) {
  __shared__ double S[2 * 65 + 1];
  __shared__ double csl[64], snl[64], coll[65], pl[65], sc[6];
  const int ns = 2 * (j + 1) + (has_w ? 1 : 0);
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  constexpr int NW = LGS_FT / 64;
  double* cs = G + 64 * 64;
  double* g = cs + 128;
  // every scalar the serial part needs is staged into LDS first, by other threads, so that its
  // chain reads no global memory.  The staged values are loaded by every lane of waves 0, 2 and 3
  // (two loads each, addresses chosen per lane, a harmless address elsewhere) before the partial
  // sums' loads and written to LDS after them, so that a wave waits for memory once: one round
  // trip before the serial part.  The cycle-end flag comes with them and is tested once they are
  // in (a launch after the end of the cycle only reads, and stores nothing).
  const double* sa = h + 240;
  const double* sb = h + 240;
  const int q = t - 192;
  if (wid == 0) {
    sa = cs + lane;  // c_i, s_i of the previous columns
    sb = cs + 64 + lane;
  } else if (wid == 2) {
    sa = h + HDEV_LGSP + lane;  // step j - 1's first-pass coefficients
  } else if (wid == 3) {
    // sc: g_{j-1} (rotated by column j - 1), the target h[240], h[252], the cycle tag h[255],
    // 1 / s_j, the flag
    sa = q == 0   ? g + (j >= 1 ? j - 1 : 0)
         : q == 1 ? h + 240
         : q == 2 ? h + 252
         : q == 3 ? h + 255
         : q == 4 ? h + HDEV_LGSP + 65
         : q == 5 ? (skip ? skip : h + 240)
                  : h + 240;
  }
  const double va = *sa, vb = *sb;
  // the sums: wave w takes sums w, w + NW, ..., two at a time, 256 partials of each per pass with
  // all their loads issued together (one pass for up to 256 partials)
  for (int s0 = wid; s0 < ns; s0 += 2 * NW) {
    const int s1 = s0 + NW;
    const bool two = s1 < ns;
    const double* p0 = part + (int64_t)s0 * np;
    const double* p1 = part + (int64_t)(two ? s1 : s0) * np;
    double a0 = 0.0, a1 = 0.0;
    for (int i0 = lane; i0 < np; i0 += 256) {
      double x0[4], x1[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + 64 * q;
        const int ic = i < np ? i : i0;
        x0[q] = p0[ic];
        x1[q] = p1[ic];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool in = i0 + 64 * q < np;
        a0 += in ? x0[q] : 0.0;
        a1 += (in && two) ? x1[q] : 0.0;
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      a0 += __shfl_down(a0, o, 64);
      a1 += __shfl_down(a1, o, 64);
    }
    if (lane == 0) {
      S[s0] = a0;
      if (two) S[s1] = a1;
    }
  }
  if (t < j - 1) {
    csl[t] = va;
    snl[t] = vb;
  }
  if (t >= 128 && t < 128 + j) pl[t - 128] = va;
  if (t >= 192 && t < 198) sc[q] = ((q == 0 && j < 1) || (q == 5 && !skip)) ? 0.0 : va;
  __syncthreads();
  if (sc[5] != 0.0 || t != 0) return;
  double aa = 0.0, ab = 0.0;
  for (int k = 0; k < j; ++k) {
    aa += S[2 * k] * S[2 * k];
    ab += S[2 * k] * S[2 * k + 1];
  }
  double rho = 1.0, flag = 0.0;
  if (j > 0) {
    const double r2 = S[2 * j] - aa;
    rho = (r2 == r2) ? sqrt(fmax(r2, 0.0)) : r2;
    const double gs = sc[4];  // 1 / s_j
    for (int k = 0; k < j; ++k) coll[k] = pl[k] + S[2 * k] * gs;
    const double hn = rho * gs;
    // Givens update of column jc = j - 1 (as givens_col, every operand from LDS)
    const int jc = j - 1;
    double* Hm = G;
    double cur = coll[0];
    for (int i = 0; i < jc; ++i) {
      const double nx = coll[i + 1];
      Hm[i * 64 + jc] = csl[i] * cur + snl[i] * nx;
      cur = -snl[i] * cur + csl[i] * nx;
    }
    const double den = hypot(cur, hn);
    const double c_ = den > 0 ? cur / den : 1.0, s_ = den > 0 ? hn / den : 0.0;
    cs[jc] = c_;
    cs[64 + jc] = s_;
    Hm[jc * 64 + jc] = den;
    const double gj = jc == 0 ? sc[1] : sc[0];
    if (jc == 0)
      for (int i = 2; i <= m; ++i) g[i] = 0.0;
    g[jc] = c_ * gj;
    g[jc + 1] = -s_ * gj;
    const double est = fabs(s_ * gj);
    h[352 + 2 * jc] = est;
    h[353 + 2 * jc] = hn;
    flag = (est <= sc[2] || hn == 0.0) ? 1.0 : 0.0;
    if (hest && !has_w) {  // a full step's update sweep publishes it (first block)
      publish_estimate(hest, jc, est, hn, sc[3]);
    }
  }
  if (flag != 0.0) h[HDEV_LGSE] = j + 1;
  if (!has_w) return;
  const double rinv = (rho > 0.0 && rho <= 1.7e308) ? 1.0 / rho : 0.0;
  const double d = j > 0 ? (S[2 * j + 1] - ab) * rinv : S[1];
  double* p = h + HDEV_LGSP;
  for (int k = 0; k < j; ++k) {
    h[k] = S[2 * k];
    h[72 + k] = S[2 * k + 1];
    p[k] = S[2 * k + 1];
  }
  p[j] = d;
  const double wn = sqrt(fmax(S[2 * j + 2], 0.0));
  const bool ok = wn > 0.0 && wn <= 1.7e308;
  p[65] = ok ? wn : 1.0;
  h[144] = j > 0 ? rinv : 1.0;
  h[145] = d;
  h[146] = ok ? 1.0 / wn : 1.0;
}

// A[r] = sum_{k < m} a_k V_k[rows[r]], B[r] likewise with b (FP64 sums of the stored basis)
template <typename TV, int R>
__device__ __forceinline__ void combo_ab(const TV* __restrict__ V, int64_t ldv, int m, const double* __restrict__ a,
                                         const double* __restrict__ b, const int64_t (&rows)[R], double (&A)[R],
                                         double (&B)[R]) {
#pragma unroll
  for (int r = 0; r < R; ++r) A[r] = B[r] = 0.0;
  for (int j0 = 0; j0 < m; j0 += MDOT_JC) {
    double v[MDOT_JC][R], ca[MDOT_JC], cb[MDOT_JC];
#pragma unroll
    for (int jj = 0; jj < MDOT_JC; ++jj) {
      const bool ok = j0 + jj < m;
      const int k = min(j0 + jj, m - 1);
      ca[jj] = ok ? a[k] : 0.0;
      cb[jj] = ok ? b[k] : 0.0;
#pragma unroll
      for (int r = 0; r < R; ++r) v[jj][r] = (double)V[(int64_t)k * ldv + rows[r]];
    }
#pragma unroll
    for (int jj = 0; jj < MDOT_JC; ++jj)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        A[r] += ca[jj] * v[jj][r];
        B[r] += cb[jj] * v[jj][r];
      }
  }
}

// combo_ab with the basis count fixed at compile time: every load issued before the first use
template <typename TV, int R, int M>
__device__ __forceinline__ void combo_ab_n(const TV* __restrict__ V, int64_t ldv, const double* __restrict__ a,
                                           const double* __restrict__ b, const int64_t (&rows)[R], double (&A)[R],
                                           double (&B)[R]) {
#pragma unroll
  for (int r = 0; r < R; ++r) A[r] = B[r] = 0.0;
  TV v[M > 0 ? M : 1][R];
#pragma unroll
  for (int k = 0; k < M; ++k)
#pragma unroll
    for (int r = 0; r < R; ++r) v[k][r] = V[(int64_t)k * ldv + rows[r]];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const double ca = a[k], cb = b[k];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      A[r] += ca * (double)v[k][r];
      B[r] += cb * (double)v[k][r];
    }
  }
}

// one row of the update from its loaded u_j and w: v_j (stored back when j > 0) and u_{j+1}
// (scaled by sg, stored over w); returns the stored u_{j+1}
template <typename TV>
__device__ __forceinline__ double lgs_row(TV* uj, TV* w, int64_t row, bool in, int j, double uv, double wv, double A,
                                          double B, double rinv, double d, double sg) {
  const TV vj = j > 0 ? (TV)((uv - A) * rinv) : (TV)uv;
  const TV un = (TV)(sg * (wv - B - d * (double)vj));
  if (in) {
    if (j > 0) uj[row] = vj;
    w[row] = un;
  }
  return (double)un;
}

static constexpr int LGS_NU = 2;  // node pairs (position row, velocity row) per thread

// Update sweep of step j with the preconditioner of the next basis vector.  Block 0 hands the
// residual estimate of column j - 1 (pub: j > 0), which the final block left in h, to host
// memory with the cycle's tag; blocks [1, 1 + nbx) take the H1 rows by node pairs (i, nh1 + i);
// the rest take whole elements' L2 rows (TPB / Nl elements per block), so z_{j+1} = P u_{j+1} is
// formed in the same launch: z_v = u_v / dv, z_x = u_x + tau z_v (coupled) or u_x,
// z_e = escale_e Me_e u_e (Me_e = me + e estride, Nl x Nl).  z (nullable): no preconditioned
// vector (the next step is a closing step); z32 (nullable): its FP32 copy; zero_v (nullable): the
// next Jacobian action's output, whose velocity rows are zeroed.  end: the cycle-end flag; the
// launch returns at once when an earlier step ended the cycle, and only block 0 works when this
// step's final block ended it (end = j + 1).
// M >= 0: the instance for j = M (compile-time basis count); M = -1: any j
template <typename TV, int M>
__global__ void __launch_bounds__(TPB) k_lgs_update(TV* __restrict__ V, int64_t ldv, int j,
                                                    const double* __restrict__ h, int64_t nh1, int64_t Ne, int Nl,
                                                    int nbx, TV* __restrict__ z, float* __restrict__ z32,
                                                    TV* __restrict__ zero_v, const double* __restrict__ dv,
                                                    const double* __restrict__ me, int64_t estride,
                                                    const double* __restrict__ escale, int coupled,
                                                    const double* __restrict__ tau_dev, int pub, double* hest,
                                                    const double* end) {
  if (blockIdx.x == 0) {
    // first in the grid, so that the fence runs beside the sweep instead of after it
    const double ended = *end;
    if (ended != 0.0 && ended != (double)(j + 1)) return;
    if (pub && hest && threadIdx.x == 0) {
      const int jc = j - 1;
      publish_estimate(hest, jc, h[352 + 2 * jc], h[353 + 2 * jc], h[255]);
    }
    return;
  }
  // the other blocks read the cycle-end flag behind their loads and return before any store
  // once an earlier step (or this step's final block) ended the cycle
  const int b = (int)blockIdx.x - 1;
  TV* uj = V + (int64_t)j * ldv;
  TV* w = uj + ldv;
  const double rinv = h[144], d = h[145], sg = h[146];
  if (b < nbx) {
    constexpr int R = 2 * LGS_NU;
    int64_t rows[R];
    bool in[LGS_NU];
#pragma unroll
    for (int q = 0; q < LGS_NU; ++q) {
      const int64_t i = ((int64_t)b * LGS_NU + q) * TPB + threadIdx.x;
      in[q] = i < nh1;
      rows[2 * q] = in[q] ? i : 0;
      rows[2 * q + 1] = nh1 + rows[2 * q];
    }
    // every load of the thread is issued before the first use
    double uv[R], wv[R], dd[LGS_NU];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      uv[r] = (double)uj[rows[r]];
      wv[r] = (double)w[rows[r]];
    }
#pragma unroll
    for (int q = 0; q < LGS_NU; ++q) dd[q] = z ? dv[rows[2 * q]] : 1.0;
    double A[R], B[R];
    if constexpr (M >= 0)
      combo_ab_n<TV, R, M>(V, ldv, h, h + 72, rows, A, B);
    else
      combo_ab(V, ldv, j, h, h + 72, rows, A, B);
    if (*end != 0.0) return;
    double un[R];
#pragma unroll
    for (int r = 0; r < R; ++r) un[r] = lgs_row(uj, w, rows[r], in[r / 2], j, uv[r], wv[r], A[r], B[r], rinv, d, sg);
    if (z) {
      const double tau = *tau_dev;
#pragma unroll
      for (int q = 0; q < LGS_NU; ++q) {
        if (!in[q]) continue;
        const int64_t i = rows[2 * q];
        const double zv = un[2 * q + 1] / dd[q];
        const double zx = coupled ? tau * zv + un[2 * q] : un[2 * q];
        z[i] = (TV)zx;
        z[nh1 + i] = (TV)zv;
        if (z32) {
          z32[i] = (float)zx;
          z32[nh1 + i] = (float)zv;
        }
        if (zero_v) zero_v[nh1 + i] = TV(0);
      }
    }
  } else {
    __shared__ double shu[TPB];
    const int epb = TPB / Nl;
    const int t = threadIdx.x, le = t / Nl, rr = t - le * Nl;
    const int64_t e = (int64_t)(b - nbx) * epb + le;
    const bool in = le < epb && e < Ne;
    const int64_t ec = in ? e : 0;
    const int64_t rows[1] = {2 * nh1 + ec * Nl + (in ? rr : 0)};
    const double uv = (double)uj[rows[0]], wv = (double)w[rows[0]];
    const double es = (z && escale) ? escale[ec] : 1.0;
    double A[1], B[1];
    if constexpr (M >= 0)
      combo_ab_n<TV, 1, M>(V, ldv, h, h + 72, rows, A, B);
    else
      combo_ab(V, ldv, j, h, h + 72, rows, A, B);
    if (*end != 0.0) return;  // uniform over the block: no thread reaches the barrier below
    const double un = lgs_row(uj, w, rows[0], in, j, uv, wv, A[0], B[0], rinv, d, sg);
    if (z) {
      shu[t] = un;
      __syncthreads();
      if (in) {
        const double* Me = me + e * estride + (int64_t)rr * Nl;
        const double* ue = shu + le * Nl;
        double acc = 0.0;
        for (int l = 0; l < Nl; ++l) acc += Me[l] * ue[l];
        acc *= es;
        z[rows[0]] = (TV)acc;
        if (z32) z32[rows[0]] = (float)acc;
      }
    }
  }
}

// instance tables indexed by the basis count: one group up to 6 vectors, two chunks beyond
template <int J>
struct LgsSplit {
  static constexpr int N0 = J <= 6 ? J : (J + 1) / 2, N1 = J - N0;
};
template <typename TV, int... I>
static auto lgs_dots_table(std::integer_sequence<int, I...>) {
  using F = void (*)(const TV*, int64_t, const TV*, const TV*, int64_t, double*, const double*);
  static const F t[] = {k_lgs_dots_n<TV, LgsSplit<I>::N0, LgsSplit<I>::N1>...};
  return t;
}
template <typename TV>
static auto lgs_dots_kernel(int j) {
  return lgs_dots_table<TV>(std::make_integer_sequence<int, LGS_NVMAX + 1>())[j];
}
template <typename TV, int... I>
static auto lgs_update_table(std::integer_sequence<int, I...>) {
  using F = decltype(&k_lgs_update<TV, -1>);
  static const F t[] = {k_lgs_update<TV, I>...};
  return t;
}
template <typename TV>
static auto lgs_update_kernel(int j) {
  return j <= LGS_NVMAX ? lgs_update_table<TV>(std::make_integer_sequence<int, LGS_NVMAX + 1>())[j]
                        : &k_lgs_update<TV, -1>;
}

template <typename TV>
int lgs_dots(ilh_ctx* c, const TV* V, int64_t ldv, int j, const TV* uj, const TV* w, int64_t n, double* part,
             int* np, const double* skip) {
  if (j > 64) return fail(c, ILH_EINVAL, "Gram-Schmidt: at most 64 basis vectors");
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (n + LGS_DT - 1) / LGS_DT));
  // the closing step has no w: its products are taken with u_j instead and not used
  // fixed-count instances up to 15 vectors in FP32 (a basis of restart length 15 and its
  // closing step), 12 in FP64 (beyond, their registers spill)
  if (j <= (sizeof(TV) == 4 ? LGS_NVMAX : 12) && n * (int64_t)sizeof(TV) <= (int64_t)UINT32_MAX) {
    hipLaunchKernelGGL(lgs_dots_kernel<TV>(j), dim3(nb, j <= 6 ? 1 : 2), dim3(LGS_DB), 0, c->stream, V, ldv, uj,
                       w ? w : uj, n, part, skip);
  } else {
    hipLaunchKernelGGL(k_lgs_dots<TV>, dim3(nb), dim3(LGS_DB), 0, c->stream, V, ldv, j, uj, w ? w : uj, n, part,
                       skip);
  }
  ILH_HIP(c, hipGetLastError());
  *np = nb;
  return ILH_OK;
}

int lgs_final(ilh_ctx* c, const double* part, int np, int j, int m, int has_w, double* h, double* G, double* hest,
              const double* skip) {
  hipLaunchKernelGGL(k_lgs_final, dim3(1), dim3(LGS_FT), 0, c->stream, part, np, j, m, has_w, h, G, hest, skip);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

template <typename TV>
int lgs_update(ilh_ctx* c, TV* V, int64_t ldv, int j, const double* h, TV* z, float* z32, TV* zero_v, int probe,
               int coupled, const double* tau_dev, double* hest, const double* end) {
  if (c->Nl > TPB) return fail(c, ILH_EINVAL, "Gram-Schmidt update: energy blocks larger than a work-group");
  const int64_t units = (int64_t)TPB * LGS_NU;
  const int nbx = (int)((c->nh1 + units - 1) / units);
  const int epb = TPB / c->Nl;
  const int nbe = (int)((c->Ne + epb - 1) / epb);
  const double* dv = probe ? c->pdv : c->Mdiag;
  const double* me = probe ? c->peinv : c->MEinv;
  const int64_t estride = probe ? (int64_t)c->Nl * c->Nl : c->me_stride;
  const double* escale = probe ? nullptr : c->me_scale;
  hipLaunchKernelGGL(lgs_update_kernel<TV>(j), dim3(1 + nbx + nbe), dim3(TPB), 0, c->stream, V, ldv, j, h, c->nh1, c->Ne,
                     c->Nl, nbx, z, z32, zero_v, dv, me, estride, escale, coupled, tau_dev, j > 0 ? 1 : 0, hest,
                     end);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

template int lgs_dots<double>(ilh_ctx*, const double*, int64_t, int, const double*, const double*, int64_t, double*,
                              int*, const double*);
template int lgs_dots<float>(ilh_ctx*, const float*, int64_t, int, const float*, const float*, int64_t, double*,
                             int*, const double*);
template int lgs_update<double>(ilh_ctx*, double*, int64_t, int, const double*, double*, float*, double*, int, int,
                                const double*, double*, const double*);
template int lgs_update<float>(ilh_ctx*, float*, int64_t, int, const double*, float*, float*, float*, int, int,
                               const double*, double*, const double*);

// Block preconditioner of the Newton-Krylov solve (eq. blockdiag_prec with a Jacobi M_V):
// z_v = r_v / diag(M_V) (1 on constrained rows), z_x = r_x + tau z_v (coupled) or r_x,
// z_e = M_E^-1 r_e; z32 (nullable) receives the FP32 copy of z.  The input is sc r with
// sc = *rs (rs nullable: 1).  With g.part set, the grid has one block more, block 0, which runs the norm
// reduction and Givens update of the previous Arnoldi step, and every other block forms the
// scale that reduction stores, sc = 1 / |r|, from the same partial sums.
template <typename TV>
__global__ void k_precond(const TV* __restrict__ r, const double* __restrict__ Mdiag,
                          const double* __restrict__ Minv, int64_t estride, const double* __restrict__ escale,
                          TV* z, float* z32,
                          double tau, int coupled, int64_t nh1, int64_t Ne, int Nl, TV* zero_v,
                          const double* tau_dev, const double* rs, const GivensJob g) {
  if (g.skip && *g.skip != 0.0) return;
  if (g.part && blockIdx.x == 0) {  // first, so its serial chain overlaps the rest of the grid
    sum_givens_block(g);
    return;
  }
  const double sc = g.part ? scale_from_partials(g.part, g.np) : (rs ? *rs : 1.0);
  const int64_t i = (blockIdx.x - (g.part ? 1 : 0)) * (int64_t)blockDim.x + threadIdx.x;
  if (zero_v && i < nh1) zero_v[i] = TV(0);  // velocity rows of the next Jacobian action's output
  if (tau_dev) tau = *tau_dev;
  if (i < nh1) {
    const double zv = sc * (double)r[nh1 + i] / Mdiag[i];
    const double zx = coupled ? tau * zv + sc * (double)r[i] : sc * (double)r[i];
    z[i] = (TV)zx;
    z[nh1 + i] = (TV)zv;
    if (z32) {
      z32[i] = (float)zx;
      z32[nh1 + i] = (float)zv;
    }
  } else if (i < nh1 + Ne * Nl) {
    const int64_t k = i - nh1, e = k / Nl;
    const int rr = (int)(k % Nl);
    const double* Me = Minv + e * estride;
    double acc = 0;
    for (int j = 0; j < Nl; ++j) acc += Me[rr * Nl + j] * (double)r[2 * nh1 + e * Nl + j];
    const double x = sc * (escale ? escale[e] * acc : acc);
    z[2 * nh1 + k] = (TV)x;
    if (z32) z32[2 * nh1 + k] = (float)x;
  }
}

template <typename TV>
int launch_precond(ilh_ctx* c, const TV* r, TV* z, float* z32, double tau, int coupled, TV* zero_v,
                   const double* tau_dev, const double* rs, const GivensJob* job) {
  const int64_t n = c->nh1 + c->Ne * c->Nl;
  const GivensJob g = job ? *job : GivensJob{};
  const unsigned nb = (unsigned)((n + TPB - 1) / TPB) + (job ? 1u : 0u);
  hipLaunchKernelGGL(k_precond<TV>, dim3(nb), dim3(TPB), 0, c->stream, r, c->Mdiag, c->MEinv, c->me_stride, c->me_scale,
                     z, z32, tau, coupled, c->nh1, c->Ne, c->Nl, zero_v, tau_dev, rs, g);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}
template int launch_precond<double>(ilh_ctx*, const double*, double*, float*, double, int, double*, const double*,
                                    const double*, const GivensJob*);
template int launch_precond<float>(ilh_ctx*, const float*, float*, float*, double, int, float*, const double*,
                                   const double*, const GivensJob*);

// ------------------------------------------------------------------ probed block preconditioner
// Node colours: (I mod M, J mod M[, K mod M]) with M = k + 1 -- two nodes of one colour never
// share an element, so a Jacobian action on the sum of the unit directions of one colour
// returns each node's diagonal entry at that node.
__device__ __forceinline__ int node_colour(int64_t i, int dim, const int* ng, int M) {
  const int64_t I = i % ng[0], J = (i / ng[0]) % ng[1], K = dim == 3 ? i / ((int64_t)ng[0] * ng[1]) : 0;
  return (int)((I % M) + M * ((J % M) + M * (K % M)));
}

struct NodeGrid {
  int ng[3];
};

// The previous probe's read-off, taken by the next probe's direction kernel from the action
// output y before it zeroes y's velocity rows for the next action (each entry of y is read and
// then zeroed by one thread): the velocity diagonal of probe (tcomp, tcol) into tD (nullable),
// column tj of every element's energy block into tB (nullable)
struct ProbeTake {
  int tcomp, tcol;
  double* tD;
  int tj;
  double* tB;
};
__device__ __forceinline__ void probe_take_zero(int64_t i, float* yz, int64_t N, int dim, const NodeGrid& g, int M,
                                                int Nl, const ProbeTake& tk) {
  const int64_t nh1 = (int64_t)dim * N;
  if (i >= nh1 && i < 2 * nh1) {
    const int64_t jv = i - nh1;
    const int cc = (int)(jv / N);
    if (tk.tD && cc == tk.tcomp && node_colour(jv - cc * N, dim, g.ng, M) == tk.tcol) tk.tD[jv] = (double)yz[i];
    yz[i] = 0.f;  // the velocity rows of the next action's output
  } else if (tk.tB && i >= 2 * nh1) {
    const int64_t t = i - 2 * nh1;
    tk.tB[t * Nl + tk.tj] = (double)yz[i];  // (e Nl + r) Nl + j with t = e Nl + r
  }
}

// direction: v component comp at the nodes of colour col = 1, x component comp there = tau
__global__ void k_probe_v_dir(float* d, int64_t N, int dim, NodeGrid g, int M, int comp, int col, float tau,
                              int64_t nblock, float* yz, int Nl, ProbeTake tk) {
  const int64_t nh1 = (int64_t)dim * N;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nblock; i += (int64_t)gridDim.x * blockDim.x) {
    if (yz) probe_take_zero(i, yz, N, dim, g, M, Nl, tk);
    float v = 0.f;
    if (i < 2 * nh1) {
      const int64_t j = i < nh1 ? i : i - nh1;
      const int c = (int)(j / N);
      if (c == comp && node_colour(j - c * N, dim, g.ng, M) == col) v = i < nh1 ? tau : 1.f;
    }
    d[i] = v;
  }
}

// direction: energy DOF j of every element = 1
__global__ void k_probe_e_dir(float* d, int64_t N, int dim, NodeGrid g, int M, int Nl, int j, int64_t nblock,
                              float* yz, ProbeTake tk) {
  const int64_t nh1x2 = 2 * (int64_t)dim * N;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nblock; i += (int64_t)gridDim.x * blockDim.x) {
    d[i] = (i >= nh1x2 && (i - nh1x2) % Nl == j) ? 1.f : 0.f;
    if (yz) probe_take_zero(i, yz, N, dim, g, M, Nl, tk);
  }
}

// column j of every element's energy block
__global__ void k_probe_e_take(const float* y, int64_t nh1x2, int64_t Ne, int Nl, int j, double* B) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < Ne * Nl; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = t / Nl;
    const int r = (int)(t % Nl);
    B[(e * Nl + r) * Nl + j] = (double)y[nh1x2 + t];
  }
}

// In-place inverse of every element block (Gauss-Jordan, partial pivoting), one thread each.
// A singular block is replaced by the identity (the preconditioner then leaves those rows).
__global__ void k_invert_blocks(double* B, int64_t Ne, int Nl) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= Ne) return;
  double* A = B + e * Nl * Nl;
  int piv[32];
  for (int i = 0; i < Nl; ++i) piv[i] = i;
  bool ok = true;
  for (int c = 0; c < Nl && ok; ++c) {
    int p = c;
    double best = fabs(A[c * Nl + c]);
    for (int r = c + 1; r < Nl; ++r)
      if (fabs(A[r * Nl + c]) > best) {
        best = fabs(A[r * Nl + c]);
        p = r;
      }
    if (!(best > 0.0)) {
      ok = false;
      break;
    }
    if (p != c) {
      for (int q = 0; q < Nl; ++q) {
        const double t = A[c * Nl + q];
        A[c * Nl + q] = A[p * Nl + q];
        A[p * Nl + q] = t;
      }
      const int t = piv[c];
      piv[c] = piv[p];
      piv[p] = t;
    }
    const double inv = 1.0 / A[c * Nl + c];
    A[c * Nl + c] = 1.0;
    for (int q = 0; q < Nl; ++q) A[c * Nl + q] *= inv;
    for (int r = 0; r < Nl; ++r) {
      if (r == c) continue;
      const double f = A[r * Nl + c];
      A[r * Nl + c] = 0.0;
      for (int q = 0; q < Nl; ++q) A[r * Nl + q] -= f * A[c * Nl + q];
    }
  }
  if (!ok) {
    for (int r = 0; r < Nl; ++r)
      for (int q = 0; q < Nl; ++q) A[r * Nl + q] = r == q ? 1.0 : 0.0;
    return;
  }
  // the loop inverted the row-permuted block P A (row q of it is row piv[q] of A):
  // A^-1 = (P A)^-1 P, i.e. column q of the result moves to column piv[q]
  double tmp[32];
  for (int r = 0; r < Nl; ++r) {
    for (int q = 0; q < Nl; ++q) tmp[piv[q]] = A[r * Nl + q];
    for (int q = 0; q < Nl; ++q) A[r * Nl + q] = tmp[q];
  }
}

int launch_probe_v_dir(ilh_ctx* c, float* d, int comp, int col, double tau, float* yz, int tcomp, int tcol,
                       double* tD) {
  NodeGrid g{{c->ng[0], c->ng[1], c->ng[2]}};
  const ProbeTake tk{tcomp, tcol, yz ? tD : nullptr, 0, nullptr};
  hipLaunchKernelGGL(k_probe_v_dir, dim3(nblk(c->nblock, 8192)), dim3(TPB), 0, c->stream, d, c->N, c->dim, g,
                     c->k + 1, comp, col, (float)tau, c->nblock, yz, c->Nl, tk);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}
int launch_probe_e_dir(ilh_ctx* c, float* d, int j, float* yz, int tcomp, int tcol, double* tD, int tj,
                       double* tB) {
  NodeGrid g{{c->ng[0], c->ng[1], c->ng[2]}};
  const ProbeTake tk{tcomp, tcol, yz ? tD : nullptr, tj, yz ? tB : nullptr};
  hipLaunchKernelGGL(k_probe_e_dir, dim3(nblk(c->nblock, 8192)), dim3(TPB), 0, c->stream, d, c->N, c->dim, g, c->k + 1,
                     c->Nl, j, c->nblock, yz, tk);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}
int launch_probe_e_take(ilh_ctx* c, const float* y, int j, double* B) {
  hipLaunchKernelGGL(k_probe_e_take, dim3(nblk(c->Ne * c->Nl, 8192)), dim3(TPB), 0, c->stream, y, 2 * c->nh1, c->Ne,
                     c->Nl, j, B);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}
// The same inversion with the block size fixed at compile time (N_l <= 9: the 2D and 3D energy
// blocks of orders up to 3 in 2D, 2 in 3D): each work-group copies its 64 blocks to LDS with
// coalesced loads, each lane inverts one block held in registers (the row exchanges of the
// partial pivoting and the final column permutation as selects, so no register is indexed at
// run time), and the results go back through LDS.  The arithmetic and its order are those of
// k_invert_blocks; the per-lane global walk of that kernel took 190 us for the 5,376 blocks of
// the triple point, most of it the latency of its dependent uncoalesced accesses.
template <int NL>
__global__ void __launch_bounds__(64) k_invert_blocks_n(double* B, int64_t Ne) {
  constexpr int S = NL * NL;
  __shared__ double sA[64 * S];
  const int64_t e0 = (int64_t)blockIdx.x * 64;
  const int nb = (int)(Ne - e0 < 64 ? Ne - e0 : 64);
  double* base = B + e0 * S;
  for (int i = threadIdx.x; i < nb * S; i += 64) sA[i] = base[i];
  __syncthreads();
  const int t = threadIdx.x;
  if (t < nb) {
    double A[NL][NL];
    int piv[NL];
#pragma unroll
    for (int r = 0; r < NL; ++r) {
      piv[r] = r;
#pragma unroll
      for (int q = 0; q < NL; ++q) A[r][q] = sA[t * S + r * NL + q];
    }
    bool ok = true;
#pragma unroll
    for (int c = 0; c < NL; ++c) {
      double best = fabs(A[c][c]);
      int p = c;
#pragma unroll
      for (int r = c + 1; r < NL; ++r) {
        const double v = fabs(A[r][c]);
        if (v > best) {
          best = v;
          p = r;
        }
      }
      ok = ok && best > 0.0;
#pragma unroll
      for (int r = c + 1; r < NL; ++r) {
        const bool sw = r == p;
#pragma unroll
        for (int q = 0; q < NL; ++q) {
          const double a = A[c][q], b = A[r][q];
          A[c][q] = sw ? b : a;
          A[r][q] = sw ? a : b;
        }
        const int pa = piv[c], pb = piv[r];
        piv[c] = sw ? pb : pa;
        piv[r] = sw ? pa : pb;
      }
      const double inv = 1.0 / A[c][c];
      A[c][c] = 1.0;
#pragma unroll
      for (int q = 0; q < NL; ++q) A[c][q] *= inv;
#pragma unroll
      for (int r = 0; r < NL; ++r) {
        if (r == c) continue;
        const double f = A[r][c];
        A[r][c] = 0.0;
#pragma unroll
        for (int q = 0; q < NL; ++q) A[r][q] -= f * A[c][q];
      }
    }
    // (P A)^-1 P: column q of the result moves to column piv[q]; a singular block -> identity
#pragma unroll
    for (int r = 0; r < NL; ++r)
#pragma unroll
      for (int tc = 0; tc < NL; ++tc) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < NL; ++q) v = piv[q] == tc ? A[r][q] : v;
        sA[t * S + r * NL + tc] = ok ? v : (r == tc ? 1.0 : 0.0);
      }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nb * S; i += 64) base[i] = sA[i];
}

int launch_invert_blocks(ilh_ctx* c, double* B) {
  if (c->Nl > 32) return fail(c, ILH_EINVAL, "energy blocks larger than 32");
  const dim3 grid((unsigned)((c->Ne + 63) / 64));
  switch (c->Nl) {
    case 1: hipLaunchKernelGGL(k_invert_blocks_n<1>, grid, dim3(64), 0, c->stream, B, c->Ne); break;
    case 4: hipLaunchKernelGGL(k_invert_blocks_n<4>, grid, dim3(64), 0, c->stream, B, c->Ne); break;
    case 8: hipLaunchKernelGGL(k_invert_blocks_n<8>, grid, dim3(64), 0, c->stream, B, c->Ne); break;
    case 9: hipLaunchKernelGGL(k_invert_blocks_n<9>, grid, dim3(64), 0, c->stream, B, c->Ne); break;
    default: hipLaunchKernelGGL(k_invert_blocks, grid, dim3(64), 0, c->stream, B, c->Ne, c->Nl);
  }
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

// z_v = r_v / D (probed diagonal), z_x = r_x + tau z_v (coupled) or r_x, z_e = Binv r_e per element;
// input scale and the extra last block as in k_precond
template <typename TV>
__global__ void k_precond_probe(const TV* __restrict__ r, const double* __restrict__ D,
                                const double* __restrict__ Binv, TV* z, float* z32, double tau, int coupled,
                                int64_t nh1, int64_t Ne, int Nl, TV* zero_v, const double* tau_dev,
                                const double* rs, const GivensJob g) {
  if (g.skip && *g.skip != 0.0) return;
  if (g.part && blockIdx.x == 0) {  // first, so its serial chain overlaps the rest of the grid
    sum_givens_block(g);
    return;
  }
  const double sc = g.part ? scale_from_partials(g.part, g.np) : (rs ? *rs : 1.0);
  const int64_t i = (blockIdx.x - (g.part ? 1 : 0)) * (int64_t)blockDim.x + threadIdx.x;
  if (zero_v && i < nh1) zero_v[i] = TV(0);  // velocity rows of the next Jacobian action's output
  if (tau_dev) tau = *tau_dev;
  if (i < nh1) {
    const double zv = sc * (double)r[nh1 + i] / D[i];
    const double zx = coupled ? tau * zv + sc * (double)r[i] : sc * (double)r[i];
    z[i] = (TV)zx;
    z[nh1 + i] = (TV)zv;
    if (z32) {
      z32[i] = (float)zx;
      z32[nh1 + i] = (float)zv;
    }
  } else if (i < nh1 + Ne * Nl) {
    const int64_t k = i - nh1, e = k / Nl;
    const int rr = (int)(k % Nl);
    const double* Bi = Binv + (e * Nl + rr) * Nl;
    double acc = 0;
    for (int j = 0; j < Nl; ++j) acc += Bi[j] * (double)r[2 * nh1 + e * Nl + j];
    acc *= sc;
    z[2 * nh1 + k] = (TV)acc;
    if (z32) z32[2 * nh1 + k] = (float)acc;
  }
}

template <typename TV>
int launch_precond_probe(ilh_ctx* c, const TV* r, TV* z, float* z32, double tau, int coupled,
                         TV* zero_v, const double* tau_dev, const double* rs, const GivensJob* job) {
  const int64_t n = c->nh1 + c->Ne * c->Nl;
  const GivensJob g = job ? *job : GivensJob{};
  const unsigned nb = (unsigned)((n + TPB - 1) / TPB) + (job ? 1u : 0u);
  hipLaunchKernelGGL(k_precond_probe<TV>, dim3(nb), dim3(TPB), 0, c->stream, r, c->pdv, c->peinv, z, z32, tau, coupled,
                     c->nh1, c->Ne, c->Nl, zero_v, tau_dev, rs, g);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}
template int launch_precond_probe<double>(ilh_ctx*, const double*, double*, float*, double, int, double*,
                                          const double*, const double*, const GivensJob*);
template int launch_precond_probe<float>(ilh_ctx*, const float*, float*, float*, double, int, float*,
                                         const double*, const double*, const GivensJob*);

// ------------------------------------------------------------------ mass operators
// y += M_V x (values-only partial assembly).  bc != 0: constrained inputs read as zero and
// constrained outputs receive x (the eliminated operator Mhat).
template <int DIM, int D1D, int Q1D, int NE>
__global__ void __launch_bounds__(256) k_mass(const KParams P, const double* x, double* y, int bc) {
  constexpr int NQ = (DIM == 2) ? Q1D * Q1D : Q1D * Q1D * Q1D;
  constexpr int ND = (DIM == 2) ? D1D * D1D : D1D * D1D * D1D;
  constexpr int NT = NQ * NE;
  constexpr int LBUF = (DIM == 2) ? D1D * Q1D : (D1D * D1D * Q1D + D1D * Q1D * Q1D);
  __shared__ double sB[Q1D * D1D];
  __shared__ double sX[NE][DIM][ND];
  __shared__ double sW[NE][DIM][LBUF > NQ ? LBUF : NQ];
  __shared__ double sQ[NE][DIM][NQ];
  const int tid = threadIdx.x, z = tid / NQ, q = tid % NQ;
  const int qx = q % Q1D, qy = (q / Q1D) % Q1D, qz = (DIM == 3) ? q / (Q1D * Q1D) : 0;
  const int e0 = blockIdx.x * NE, k = P.k;
  const int64_t N = P.N, s1 = P.ng[0], s2 = (int64_t)P.ng[0] * P.ng[1];
  for (int i = tid; i < Q1D * D1D; i += NT) sB[i] = P.tab[i];
  for (int i = tid; i < NE * DIM * ND; i += NT) {
    const int li = i % ND, t = i / ND, c = t % DIM, zz = t / DIM, e = e0 + zz;
    double val = 0;
    if (e < P.Ne) {
      const int a = li % D1D, b = (li / D1D) % D1D, cc = (DIM == 3) ? li / (D1D * D1D) : 0;
      const int ex = e % P.n[0], ey = (e / P.n[0]) % P.n[1], ez = (DIM == 3) ? e / (P.n[0] * P.n[1]) : 0;
      const int I = k * ex + a, J = k * ey + b, K = k * ez + cc;
      const int gc = (c == 0) ? I : (c == 1 ? J : K);
      const bool cons = on_wall(P.walls, c, gc, P.ng[c]);
      val = (bc && cons) ? 0.0 : x[c * N + I + s1 * J + s2 * K];
    }
    sX[zz][c][li] = val;
  }
  __syncthreads();
  double vq[DIM];
  if constexpr (DIM == 2) {
    for (int i = tid; i < NE * 2 * D1D * Q1D; i += NT) {
      const int qxx = i % Q1D, t = i / Q1D, b = t % D1D, t2 = t / D1D, c = t2 & 1, zz = t2 >> 1;
      double acc = 0;
#pragma unroll
      for (int a = 0; a < D1D; ++a) acc += sB[qxx * D1D + a] * sX[zz][c][a + D1D * b];
      sW[zz][c][b * Q1D + qxx] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      double acc = 0;
#pragma unroll
      for (int b = 0; b < D1D; ++b) acc += sB[qy * D1D + b] * sW[z][c][b * Q1D + qx];
      vq[c] = acc;
    }
  } else {
    for (int i = tid; i < NE * 3 * D1D * D1D * Q1D; i += NT) {
      const int qxx = i % Q1D, t = i / Q1D, bcc = t % (D1D * D1D), t2 = t / (D1D * D1D), c = t2 % 3, zz = t2 / 3;
      double acc = 0;
#pragma unroll
      for (int a = 0; a < D1D; ++a) acc += sB[qxx * D1D + a] * sX[zz][c][a + D1D * bcc];
      sW[zz][c][bcc * Q1D + qxx] = acc;
    }
    __syncthreads();
    for (int i = tid; i < NE * 3 * D1D * Q1D * Q1D; i += NT) {
      const int qxx = i % Q1D, t = i / Q1D, qyy = t % Q1D, t2 = t / Q1D, cc = t2 % D1D, t3 = t2 / D1D, c = t3 % 3,
                zz = t3 / 3;
      double acc = 0;
#pragma unroll
      for (int b = 0; b < D1D; ++b) acc += sB[qyy * D1D + b] * sW[zz][c][(cc * D1D + b) * Q1D + qxx];
      sW[zz][c][D1D * D1D * Q1D + (cc * Q1D + qyy) * Q1D + qxx] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double acc = 0;
#pragma unroll
      for (int cc = 0; cc < D1D; ++cc) acc += sB[qz * D1D + cc] * sW[z][c][D1D * D1D * Q1D + (cc * Q1D + qy) * Q1D + qx];
      vq[c] = acc;
    }
  }
  const int e = e0 + z;
  const double mq = (e < P.Ne) ? P.mq[(int64_t)e * NQ + q] : 0.0;
#pragma unroll
  for (int c = 0; c < DIM; ++c) sQ[z][c][q] = mq * vq[c];
  __syncthreads();
  if constexpr (DIM == 2) {
    for (int i = tid; i < NE * 2 * D1D * Q1D; i += NT) {
      const int qxx = i % Q1D, t = i / Q1D, b = t % D1D, t2 = t / D1D, c = t2 & 1, zz = t2 >> 1;
      double acc = 0;
#pragma unroll
      for (int qyy = 0; qyy < Q1D; ++qyy) acc += sB[qyy * D1D + b] * sQ[zz][c][qxx + Q1D * qyy];
      sW[zz][c][b * Q1D + qxx] = acc;
    }
  } else {
    for (int i = tid; i < NE * 3 * D1D * Q1D * Q1D; i += NT) {
      const int qxx = i % Q1D, t = i / Q1D, qyy = t % Q1D, t2 = t / Q1D, cc = t2 % D1D, t3 = t2 / D1D, c = t3 % 3,
                zz = t3 / 3;
      double acc = 0;
#pragma unroll
      for (int qzz = 0; qzz < Q1D; ++qzz) acc += sB[qzz * D1D + cc] * sQ[zz][c][qxx + Q1D * (qyy + Q1D * qzz)];
      sW[zz][c][D1D * D1D * Q1D + (cc * Q1D + qyy) * Q1D + qxx] = acc;
    }
    __syncthreads();
    for (int i = tid; i < NE * 3 * D1D * D1D * Q1D; i += NT) {
      const int qxx = i % Q1D, t = i / Q1D, bcc = t % (D1D * D1D), t2 = t / (D1D * D1D), c = t2 % 3, zz = t2 / 3;
      const int b = bcc % D1D, cc = bcc / D1D;
      double acc = 0;
#pragma unroll
      for (int qyy = 0; qyy < Q1D; ++qyy) acc += sB[qyy * D1D + b] * sW[zz][c][D1D * D1D * Q1D + (cc * Q1D + qyy) * Q1D + qxx];
      sW[zz][c][bcc * Q1D + qxx] = acc;
    }
  }
  __syncthreads();
  for (int i = tid; i < NE * DIM * ND; i += NT) {
    const int li = i % ND, t = i / ND, c = t % DIM, zz = t / DIM, e2 = e0 + zz;
    if (e2 >= P.Ne) continue;
    const int a = li % D1D, bcc = li / D1D;
    double acc = 0;
#pragma unroll
    for (int qxx = 0; qxx < Q1D; ++qxx) acc += sB[qxx * D1D + a] * sW[zz][c][bcc * Q1D + qxx];
    const int b = bcc % D1D, cc = (DIM == 3) ? bcc / D1D : 0;
    const int ex = e2 % P.n[0], ey = (e2 / P.n[0]) % P.n[1], ez = (DIM == 3) ? e2 / (P.n[0] * P.n[1]) : 0;
    const int I = k * ex + a, J = k * ey + b, K = k * ez + cc;
    const int64_t gi = c * N + I + s1 * J + s2 * K;
    const int gc = (c == 0) ? I : (c == 1 ? J : K);
    const bool cons = on_wall(P.walls, c, gc, P.ng[c]);
    if (bc && cons) {
      const bool owner = (a < k || ex == P.n[0] - 1) && (b < k || ey == P.n[1] - 1) &&
                         (DIM == 2 || cc < k || ez == P.n[2] - 1);
      if (owner) unsafeAtomicAdd(&y[gi], x[gi]);
    } else {
      unsafeAtomicAdd(&y[gi], acc);
    }
  }
}

template <int DIM, int K>
static void launch_mass_t(ilh_ctx* c, const double* x, double* y, int bc) {
  constexpr int Q1D = 2 * K;
  constexpr int NQ = (DIM == 2) ? Q1D * Q1D : Q1D * Q1D * Q1D;
  constexpr int NE = (256 / NQ) > 0 ? (256 / NQ) : 1;
  const int grid = (int)((c->Ne + NE - 1) / NE);
  hipLaunchKernelGGL((k_mass<DIM, K + 1, Q1D, NE>), dim3(grid), dim3(NQ * NE), 0, c->stream, c->kp, x, y, bc);
}

static int mass_apply(ilh_ctx* c, const double* x, double* y, int bc) {
  int st = launch_fill(c, y, 0.0, c->nh1);
  if (st) return st;
  const int slot = tstart(c, 2);
  if (c->dim == 2) {
    switch (c->k) {
      case 1: launch_mass_t<2, 1>(c, x, y, bc); break;
      case 2: launch_mass_t<2, 2>(c, x, y, bc); break;
      case 3: launch_mass_t<2, 3>(c, x, y, bc); break;
      case 4: launch_mass_t<2, 4>(c, x, y, bc); break;
    }
  } else {
    switch (c->k) {
      case 1: launch_mass_t<3, 1>(c, x, y, bc); break;
      case 2: launch_mass_t<3, 2>(c, x, y, bc); break;
      case 3: launch_mass_t<3, 3>(c, x, y, bc); break;
    }
  }
  tstop(c, slot);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

int launch_mass_v(ilh_ctx* c, const double* x, double* y, int bc) { return mass_apply(c, x, y, bc); }

// x_e = s_e Minv_ref b_e  (M_E,e = rho0_e |J0| Mref on the affine initial mesh)
// x_e = scale_e Minv_e b_e with Minv_e = Minv + e * stride (stride 0: one reference inverse for
// every element of an affine initial mesh, scaled by 1 / (rho0 |J0|)_e; stride Nl^2: per-element
// inverses of a curved initial mesh, scale nullptr)
__global__ void k_me_inv(const double* Minv, int64_t stride, const double* scale, const double* b, double* x,
                         int64_t Ne, int Nl) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= Ne * Nl) return;
  const int64_t e = i / Nl;
  const int r = (int)(i % Nl);
  const double* Me = Minv + e * stride;
  double acc = 0;
  for (int j = 0; j < Nl; ++j) acc += Me[r * Nl + j] * b[e * Nl + j];
  x[i] = scale ? scale[e] * acc : acc;
}
int launch_mass_e_inv(ilh_ctx* c, const double* b, double* x) {
  const int64_t n = c->Ne * c->Nl;
  if (n == 0) return ILH_OK;
  hipLaunchKernelGGL(k_me_inv, dim3((unsigned)((n + TPB - 1) / TPB)), dim3(TPB), 0, c->stream, c->MEinv,
                     c->me_stride, c->me_scale, b, x, c->Ne, c->Nl);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

// ------------------------------------------------------------------ device-scalar PCG
// scalars s[0] = rz, s[1] = pAp, s[2] = rz_new, s[3] = bb, s[4] = rr
__global__ void k_pcg_update_xr(double* x, double* r, const double* p, const double* Ap, const double* s, int64_t n) {
  const double alpha = s[1] != 0.0 ? s[0] / s[1] : 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    x[i] += alpha * p[i];
    r[i] -= alpha * Ap[i];
  }
}
__global__ void k_pcg_update_p(double* p, const double* z, double* s, int64_t n) {
  const double beta = s[0] != 0.0 ? s[2] / s[0] : 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = z[i] + beta * p[i];
}
__global__ void k_copy_scalar(double* s, int dst, int src) {
  if (threadIdx.x == 0 && blockIdx.x == 0) s[dst] = s[src];
}

int pcg_mass_v(ilh_ctx* c, const double* b, double* x, double rtol, int maxit, int check, int* iters,
               double* relres) {
  const int64_t n = c->nh1;
  double* r = c->pcgbuf;
  double* z = r + n;
  double* p = z + n;
  double* Ap = p + n;
  double* s = Ap + n;
  int st;
  if ((st = launch_fill(c, x, 0.0, n))) return st;
  ILH_HIP(c, hipMemcpyAsync(r, b, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if ((st = launch_jacobi(c, r, z))) return st;
  ILH_HIP(c, hipMemcpyAsync(p, z, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if ((st = dot_dev(c, r, z, n, s + 0))) return st;
  double bb = 0;
  if (check > 0) {
    if ((st = dot_host(c, b, b, n, &bb))) return st;
    if (bb == 0.0) {
      if (iters) *iters = 0;
      if (relres) *relres = 0.0;
      return ILH_OK;
    }
  }
  int it = 0;
  double rel = -1.0;
  for (; it < maxit; ++it) {
    if ((st = mass_apply(c, p, Ap, 1))) return st;
    if ((st = dot_dev(c, p, Ap, n, s + 1))) return st;
    hipLaunchKernelGGL(k_pcg_update_xr, dim3(nblk(n)), dim3(TPB), 0, c->stream, x, r, p, Ap, s, n);
    if ((st = launch_jacobi(c, r, z))) return st;
    if ((st = dot_dev(c, r, z, n, s + 2))) return st;
    hipLaunchKernelGGL(k_pcg_update_p, dim3(nblk(n)), dim3(TPB), 0, c->stream, p, z, s, n);
    hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, c->stream, s, 0, 2);
    ILH_HIP(c, hipGetLastError());
    if (check > 0 && ((it + 1) % check == 0 || it + 1 == maxit)) {
      double rr;
      if ((st = dot_host(c, r, r, n, &rr))) return st;
      rel = std::sqrt(rr / bb);
      if (rel <= rtol) {
        ++it;
        break;
      }
    }
  }
  if (iters) *iters = it;
  if (relres) *relres = rel;
  return ILH_OK;
}

// ------------------------------------------------------------------ per-qp diagnostics
// Dense (non sum-factorised) evaluation at each quadrature point: used only for
// diagnostics and set-up, never inside the Newton-Krylov loop.
enum Diag { D_MINDET = 0, D_DT = 1, D_L1 = 2, D_IE = 3, D_INITE = 4 };

template <int DIM>
__device__ inline double sigma_min(const double J[DIM][DIM]) {
  // smallest singular value = sqrt(smallest eigenvalue of J^T J)
  double A[DIM][DIM];
  for (int i = 0; i < DIM; ++i)
    for (int j = 0; j < DIM; ++j) {
      double acc = 0;
      for (int c = 0; c < DIM; ++c) acc += J[c][i] * J[c][j];
      A[i][j] = acc;
    }
  if constexpr (DIM == 2) {
    const double tr = A[0][0] + A[1][1];
    const double det = A[0][0] * A[1][1] - A[0][1] * A[1][0];
    const double disc = sqrt(fmax(0.25 * tr * tr - det, 0.0));
    const double lmax = 0.5 * tr + disc;
    return sqrt(fmax(det / lmax, 0.0));
  } else {
    // eigenvalues of a symmetric 3x3 matrix (trigonometric solution of the cubic)
    const double p1 = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const double qq = (A[0][0] + A[1][1] + A[2][2]) / 3.0;
    if (p1 == 0.0) return sqrt(fmin(A[0][0], fmin(A[1][1], A[2][2])));
    const double p2 = (A[0][0] - qq) * (A[0][0] - qq) + (A[1][1] - qq) * (A[1][1] - qq) +
                      (A[2][2] - qq) * (A[2][2] - qq) + 2.0 * p1;
    const double p = sqrt(p2 / 6.0);
    double Bm[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Bm[i][j] = (A[i][j] - (i == j ? qq : 0.0)) / p;
    const double detB = Bm[0][0] * (Bm[1][1] * Bm[2][2] - Bm[1][2] * Bm[2][1]) -
                        Bm[0][1] * (Bm[1][0] * Bm[2][2] - Bm[1][2] * Bm[2][0]) +
                        Bm[0][2] * (Bm[1][0] * Bm[2][1] - Bm[1][1] * Bm[2][0]);
    double rr = fmin(fmax(detB / 2.0, -1.0), 1.0);
    const double phi = acos(rr) / 3.0;
    const double l1 = qq + 2.0 * p * cos(phi);
    const double l3 = qq + 2.0 * p * cos(phi + 2.0943951023931954923);
    (void)l1;
    return sqrt(fmax(l3, 0.0));
  }
}

__device__ inline double prob_velocity(int prob, int c, const double* X) {
  const double pi = 3.14159265358979323846;
  if (prob == ILH_PROBLEM_TG2D) {
    return c == 0 ? sin(pi * X[0]) * cos(pi * X[1]) : -cos(pi * X[0]) * sin(pi * X[1]);
  }
  if (prob == ILH_PROBLEM_TG3D) {
    if (c == 0) return sin(pi * X[0]) * cos(pi * X[1]) * cos(pi * X[2]);
    if (c == 1) return -cos(pi * X[0]) * sin(pi * X[1]) * cos(pi * X[2]);
    return 0.0;
  }
  return 0.0;
}

// tab layout: B [Q1D][D1D], G [Q1D][D1D], BL [Q1D][L1D], w1 [Q1D], xg [Q1D], gll [D1D]
template <int DIM>
__global__ void __launch_bounds__(256) k_diag(const KParams P, int mode, int prob, const double* u, double cfl,
                                              double* part) {
  __shared__ double sB[64], sG[64], sBL[64], sW1[8];
  const int k = P.k, D1D = k + 1, Q1D = 2 * k, L1D = k;
  const int NQ = (DIM == 2) ? Q1D * Q1D : Q1D * Q1D * Q1D;
  for (int i = threadIdx.x; i < Q1D * D1D; i += blockDim.x) {
    sB[i] = P.tab[i];
    sG[i] = P.tab[Q1D * D1D + i];
  }
  for (int i = threadIdx.x; i < Q1D * L1D; i += blockDim.x) sBL[i] = P.tab[2 * Q1D * D1D + i];
  for (int i = threadIdx.x; i < Q1D; i += blockDim.x) sW1[i] = P.tab[2 * Q1D * D1D + Q1D * L1D + i];
  __syncthreads();
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)P.Ne * NQ;
  const bool is_min = (mode == D_MINDET || mode == D_DT);
  double val = is_min ? 1e300 : 0.0;
  if (gid < total) {
    const int e = (int)(gid / NQ), q = (int)(gid % NQ);
    const int qi[3] = {q % Q1D, (q / Q1D) % Q1D, (DIM == 3) ? q / (Q1D * Q1D) : 0};
    const int ex = e % P.n[0], ey = (e / P.n[0]) % P.n[1], ez = (DIM == 3) ? e / (P.n[0] * P.n[1]) : 0;
    const int64_t N = P.N, s1 = P.ng[0], s2 = (int64_t)P.ng[0] * P.ng[1];
    double J[DIM][DIM], Gv[DIM][DIM], xq[DIM], vq[DIM];
    for (int c = 0; c < DIM; ++c) {
      xq[c] = vq[c] = 0;
      for (int a = 0; a < DIM; ++a) J[c][a] = Gv[c][a] = 0;
    }
    const int NDn = (DIM == 2) ? D1D * D1D : D1D * D1D * D1D;
    if (mode != D_IE) {
      for (int li = 0; li < NDn; ++li) {
        const int nl[3] = {li % D1D, (li / D1D) % D1D, (DIM == 3) ? li / (D1D * D1D) : 0};
        double w = 1, g[DIM];
        for (int d = 0; d < DIM; ++d) g[d] = 1;
        for (int d = 0; d < DIM; ++d) {
          const double bv = sB[qi[d] * D1D + nl[d]], gv = sG[qi[d] * D1D + nl[d]];
          w *= bv;
          for (int d2 = 0; d2 < DIM; ++d2) g[d2] *= (d2 == d) ? gv : bv;
        }
        const int64_t node = (k * ex + nl[0]) + s1 * (k * ey + nl[1]) + s2 * (k * ez + nl[2]);
        for (int c = 0; c < DIM; ++c) {
          const double xv = u[c * N + node];
          const double vv = u[DIM * N + c * N + node];
          xq[c] += w * xv;
          vq[c] += w * vv;
          for (int d = 0; d < DIM; ++d) {
            J[c][d] += g[d] * xv;
            Gv[c][d] += g[d] * vv;
          }
        }
      }
    }
    double eq = 0;
    if (mode == D_DT || mode == D_IE) {
      const int NLn = (DIM == 2) ? L1D * L1D : L1D * L1D * L1D;
      for (int j = 0; j < NLn; ++j) {
        const int al = j % L1D, bl = (j / L1D) % L1D, cl = (DIM == 3) ? j / (L1D * L1D) : 0;
        double ph = sBL[qi[0] * L1D + al] * sBL[qi[1] * L1D + bl];
        if (DIM == 3) ph *= sBL[qi[2] * L1D + cl];
        eq += ph * u[2 * DIM * N + (int64_t)e * NLn + j];
      }
    }
    if (mode == D_MINDET) {
      double Ji[DIM][DIM], det;
      inv_det<DIM, double>(J, Ji, det);
      val = det;
    } else if (mode == D_IE) {
      val = P.mq[gid] * eq;
    } else if (mode == D_DT) {
      double Ji[DIM][DIM], det;
      inv_det<DIM, double>(J, Ji, det);
      const double gam = P.gamma[e];
      double ep, r;
      e_plus<double>(eq, P.eps_e, ep, r);
      const double cs = sqrt(gam * (gam - 1) * ep);
      double nu = 0;  // mu / rho
      if (P.visc) {
        double div = 0;
        for (int c = 0; c < DIM; ++c)
          for (int a = 0; a < DIM; ++a) div += Gv[c][a] * Ji[a][c];
        const double h = P.h0 * ((DIM == 2) ? sqrt(det / P.detJ0[gid]) : cbrt(det / P.detJ0[gid]));
        const double dv = h * div;
        const double dsc = P.dsc_mode ? 2.0 * h * cs * P.hc_inv : P.dsc_w;
        const double aabs = sqrt(dv * dv + dsc * dsc);
        const double psi = 0.5 + 0.5 * tanh(-dv / (2 * dsc) - P.psi_shift);
        nu = h * (P.q2 * aabs + P.q1 * cs * psi);
      }
      const double hmin = sigma_min<DIM>(J) / k;
      const double inv_dt = cs / hmin + 2.5 * nu / (hmin * hmin);
      val = cfl / inv_dt;
    } else if (mode == D_L1) {
      double Ji[DIM][DIM], det;
      inv_det<DIM, double>(J, Ji, det);
      double err2 = 0;
      for (int c = 0; c < DIM; ++c) {
        const double d = vq[c] - prob_velocity(prob, c, xq);
        err2 += d * d;
      }
      double wq = 1;
      for (int d = 0; d < DIM; ++d) wq *= sW1[qi[d]];
      val = wq * det * sqrt(err2);
    }
  }
  double r = is_min ? block_min<256>(val) : block_sum<256>(val);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

static int diag_dev(ilh_ctx* c, int mode, const double* u, double cfl, double* d_out) {
  const int NQ = c->Q;
  const int64_t total = c->Ne * (int64_t)NQ;
  const int nb = (int)((total + 255) / 256);
  double* part = c->ws;  // nb doubles
  if (c->ws_len < nb + 1) return fail(c, ILH_EINVAL, "workspace too small for diagnostics");
  if (c->dim == 2)
    hipLaunchKernelGGL(k_diag<2>, dim3(nb), dim3(256), 0, c->stream, c->kp, mode, c->s.problem, u, cfl, part);
  else
    hipLaunchKernelGGL(k_diag<3>, dim3(nb), dim3(256), 0, c->stream, c->kp, mode, c->s.problem, u, cfl, part);
  const bool is_min = (mode == D_MINDET || mode == D_DT);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(TPB), 0, c->stream, part, nb, d_out, is_min ? 1 : 0);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
}

static int diag_host(ilh_ctx* c, int mode, const double* u, double cfl, double* out) {
  double* d_out = c->red + c->red_blocks * 65 + 1;
  int st = diag_dev(c, mode, u, cfl, d_out);
  if (st) return st;
  ILH_HIP(c, hipMemcpyAsync(c->red_host, d_out, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  ILH_HIP(c, hipStreamSynchronize(c->stream));
  *out = c->red_host[0];
  return ILH_OK;
}

int min_detj_host(ilh_ctx* c, const double* x, double* out) { return diag_host(c, D_MINDET, x, 0.0, out); }
int min_detj_dev(ilh_ctx* c, const double* x, double* d_out) { return diag_dev(c, D_MINDET, x, 0.0, d_out); }
int dt_estimate_host(ilh_ctx* c, const double* u, double cfl, double* out) { return diag_host(c, D_DT, u, cfl, out); }
int l1_error_host(ilh_ctx* c, const double* u, double* out) { return diag_host(c, D_L1, u, 0.0, out); }
int energy_host(ilh_ctx* c, const double* u, double* ke, double* ie) {
  int st = diag_host(c, D_IE, u, 0.0, ie);
  if (st) return st;
  // KE = 1/2 v^T M_V v
  double* Mv = c->pcgbuf;
  const double* v = u + c->nh1;
  if ((st = mass_apply(c, v, Mv, 0))) return st;
  double vmv;
  if ((st = dot_host(c, v, Mv, c->nh1, &vmv))) return st;
  *ke = 0.5 * vmv;
  return ILH_OK;
}

// ------------------------------------------------------------------ initial state
// nodes: x0 on the affine mesh, v0 = nodal interpolation of the problem velocity
template <int DIM>
__global__ void k_init_nodes(const KParams P, int prob, double lo0, double lo1, double lo2, double h0, double h1,
                             double h2, const double* x0, double* u) {
  const int64_t node = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (node >= P.N) return;
  const int k = P.k, Q1D = 2 * k, D1D = k + 1, L1D = k;
  const double* gll = P.tab + 2 * Q1D * D1D + Q1D * L1D + 2 * Q1D;
  const double lo[3] = {lo0, lo1, lo2}, hh[3] = {h0, h1, h2};
  int64_t rem = node;
  double X[3] = {0, 0, 0};
  int gi[3];
  for (int d = 0; d < DIM; ++d) {
    gi[d] = (int)(rem % P.ng[d]);
    rem /= P.ng[d];
    int ex = gi[d] / k;
    if (ex > P.n[d] - 1) ex = P.n[d] - 1;
    const int loc = gi[d] - k * ex;
    X[d] = lo[d] + hh[d] * (ex + gll[loc]);
  }
  if (x0)
    for (int d = 0; d < DIM; ++d) X[d] = x0[d * P.N + node];
  for (int c = 0; c < DIM; ++c) {
    u[c * P.N + node] = X[c];
    const bool cons = on_wall(P.walls, c, gi[c], P.ng[c]);
    u[DIM * P.N + c * P.N + node] = cons ? 0.0 : prob_velocity(prob, c, X);
  }
}

__device__ inline double prob_energy(int prob, const double* X, double gam, double e0c) {
  const double pi = 3.14159265358979323846;
  if (prob == ILH_PROBLEM_TG2D) {
    const double p = 0.25 * (cos(2 * pi * X[0]) + cos(2 * pi * X[1])) + 1.0;
    return p / (gam - 1.0);
  }
  if (prob == ILH_PROBLEM_TG3D) {
    const double p = 1.0 + (cos(2 * pi * X[0]) + cos(2 * pi * X[1])) * (cos(2 * pi * X[2]) + 2.0) / 16.0;
    return p / (gam - 1.0);
  }
  return e0c;
}

// rhs_j = sum_q m_q e0(x0_q) phi_j(xi_q), one thread per (element, j)
template <int DIM>
__global__ void k_init_rhs(const KParams P, int prob, const double* e0, double lo0, double lo1, double lo2,
                           double h0, double h1, double h2, const double* x0, double* rhs) {
  const int k = P.k, Q1D = 2 * k, D1D = k + 1, L1D = k;
  const int NLn = (DIM == 2) ? L1D * L1D : L1D * L1D * L1D;
  const int NQ = (DIM == 2) ? Q1D * Q1D : Q1D * Q1D * Q1D;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)P.Ne * NLn) return;
  const int e = (int)(i / NLn), j = (int)(i % NLn);
  const double* BL = P.tab + 2 * Q1D * D1D;
  const double* xg = P.tab + 2 * Q1D * D1D + Q1D * L1D + Q1D;
  const int jl[3] = {j % L1D, (j / L1D) % L1D, (DIM == 3) ? j / (L1D * L1D) : 0};
  const int ei[3] = {e % P.n[0], (e / P.n[0]) % P.n[1], (DIM == 3) ? e / (P.n[0] * P.n[1]) : 0};
  const double lo[3] = {lo0, lo1, lo2}, hh[3] = {h0, h1, h2};
  const double gam = P.gamma[e];
  double acc = 0;
  for (int q = 0; q < NQ; ++q) {
    const int qi[3] = {q % Q1D, (q / Q1D) % Q1D, (DIM == 3) ? q / (Q1D * Q1D) : 0};
    double X[3] = {0, 0, 0}, ph = 1;
    for (int d = 0; d < DIM; ++d) {
      X[d] = lo[d] + hh[d] * (ei[d] + xg[qi[d]]);
      ph *= BL[qi[d] * L1D + jl[d]];
    }
    if (x0) {  // curved initial mesh: x0(xi_q) = sum_n x0_n w_n(xi_q)
      const int NDn = (DIM == 2) ? D1D * D1D : D1D * D1D * D1D;
      for (int d = 0; d < DIM; ++d) X[d] = 0;
      for (int li = 0; li < NDn; ++li) {
        const int a[3] = {li % D1D, (li / D1D) % D1D, (DIM == 3) ? li / (D1D * D1D) : 0};
        double wn = 1;
        int64_t node = 0, stride = 1;
        for (int d = 0; d < DIM; ++d) {
          wn *= P.tab[qi[d] * D1D + a[d]];
          node += (int64_t)(k * ei[d] + a[d]) * stride;
          stride *= P.ng[d];
        }
        for (int d = 0; d < DIM; ++d) X[d] += wn * x0[d * P.N + node];
      }
    }
    acc += P.mq[(int64_t)e * NQ + q] * prob_energy(prob, X, gam, e0[e]) * ph;
  }
  rhs[i] = acc;
}

int init_state_dev(ilh_ctx* c, double* u, const double*) {
  const double h[3] = {(c->hi[0] - c->lo[0]) / c->n[0], (c->hi[1] - c->lo[1]) / c->n[1],
                       c->dim == 3 ? (c->hi[2] - c->lo[2]) / c->n[2] : 1.0};
  const int nb = (int)((c->N + 255) / 256);
  if (c->dim == 2)
    hipLaunchKernelGGL(k_init_nodes<2>, dim3(nb), dim3(256), 0, c->stream, c->kp, c->s.problem, c->lo[0], c->lo[1],
                       c->lo[2], h[0], h[1], h[2], c->x0, u);
  else
    hipLaunchKernelGGL(k_init_nodes<3>, dim3(nb), dim3(256), 0, c->stream, c->kp, c->s.problem, c->lo[0], c->lo[1],
                       c->lo[2], h[0], h[1], h[2], c->x0, u);
  const int64_t nl = c->Ne * c->Nl;
  double* rhs = c->ws;
  if (c->ws_len < nl) return fail(c, ILH_EINVAL, "workspace too small for the initial state");
  const int nb2 = (int)((nl + 255) / 256);
  if (c->dim == 2)
    hipLaunchKernelGGL(k_init_rhs<2>, dim3(nb2), dim3(256), 0, c->stream, c->kp, c->s.problem, c->e0, c->lo[0],
                       c->lo[1], c->lo[2], h[0], h[1], h[2], c->x0, rhs);
  else
    hipLaunchKernelGGL(k_init_rhs<3>, dim3(nb2), dim3(256), 0, c->stream, c->kp, c->s.problem, c->e0, c->lo[0],
                       c->lo[1], c->lo[2], h[0], h[1], h[2], c->x0, rhs);
  ILH_HIP(c, hipGetLastError());
  return launch_mass_e_inv(c, rhs, u + 2 * c->nh1);
}

}  // namespace ilh

// Learned Newton initial guess: per-element features, a BF16/FP32 MLP on MFMA, and the
// assembly of the predicted element-local stage rates into a block vector.
//
// MLP tensors: every width w is padded to P(w) = 32 ceil(w / 32); padding entries are zero.
//   W_l  [P(w_{l+1})][P(w_l)]  BF16 (uint16 storage), WT_l = transpose of W_l
//   b_l  [P(w_{l+1})]          FP32
//   activations [batch][P(w)]  FP32 (rounded to BF16 where they enter an MFMA)
// Dense products use v_mfma_f32_16x16x32_bf16: BF16 operands, FP32 accumulation.
// Hidden layers use GELU in its erf form; the last layer is linear.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "ilh_internal.h"

namespace ilh {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

static inline int pad32(int w) { return (w + 31) / 32 * 32; }

// round-to-nearest-even FP32 -> BF16 bits (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

__device__ __forceinline__ bf16x8 pack8(const float* v) {
  bf16x8 r;
  for (int j = 0; j < 8; ++j) {
    const uint16_t h = f2bf(v[j]);
    r[j] = __builtin_bit_cast(__bf16, h);
  }
  return r;
}
__device__ __forceinline__ bf16x8 load8bf(const uint16_t* p) {
  bf16x8 r;
  for (int j = 0; j < 8; ++j) r[j] = __builtin_bit_cast(__bf16, p[j]);
  return r;
}

// ---------------------------------------------------------------------------------------
// Z[b][n] = sum_k bf(X[b][k]) W[n][k] + bias[n];  A = gelu(Z) (act) or Z.
// Work-group: 4 waves x 16 rows = 64 batch rows; each wave computes all Np/16 column tiles.
// MFMA 16x16x32 operand layout: lane l holds row/col (l % 16) and the 8 consecutive k of
// block (l / 16); the accumulator holds column (l % 16), rows 4 (l / 16) + 0..3.
template <int KP, int NP>
__global__ void __launch_bounds__(256) k_dense_fwd(const float* __restrict__ X, const uint16_t* __restrict__ W,
                                                   const float* __restrict__ bias, int batch, int act,
                                                   float* __restrict__ Z, float* __restrict__ A) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row0 = blockIdx.x * 64 + wave * 16;
  const int r = row0 + (lane & 15), kb = (lane >> 4) * 8;
  bf16x8 af[KP / 32];
#pragma unroll
  for (int s = 0; s < KP / 32; ++s) {
    float v[8];
    for (int j = 0; j < 8; ++j) v[j] = (r < batch) ? X[(int64_t)r * KP + s * 32 + kb + j] : 0.0f;
    af[s] = pack8(v);
  }
#pragma unroll
  for (int t = 0; t < NP / 16; ++t) {
    const int n = t * 16 + (lane & 15);
    f32x4 acc = {0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < KP / 32; ++s) {
      const bf16x8 bf = load8bf(W + (int64_t)n * KP + s * 32 + kb);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[s], bf, acc, 0, 0, 0);
    }
    const float bn = bias[n];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int rr = row0 + (lane >> 4) * 4 + j;
      if (rr < batch) {
        const float z = acc[j] + bn;
        Z[(int64_t)rr * NP + n] = z;
        A[(int64_t)rr * NP + n] = act ? gelu(z) : z;
      }
    }
  }
}

// dX[b][k] = sum_n bf(dZ[b][n]) W[n][k]  (B operand from WT [KP][NP]: WT[k][n]);
// if gz != null: dX *= gelu'(gz[b][k]) (the previous layer's pre-activation).
template <int KP, int NP>
__global__ void __launch_bounds__(256) k_dense_bwd_data(const float* __restrict__ dZ, const uint16_t* __restrict__ WT,
                                                        int batch, const float* __restrict__ gz, float* __restrict__ dX) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row0 = blockIdx.x * 64 + wave * 16;
  const int r = row0 + (lane & 15), kb = (lane >> 4) * 8;
  bf16x8 af[NP / 32];
#pragma unroll
  for (int s = 0; s < NP / 32; ++s) {
    float v[8];
    for (int j = 0; j < 8; ++j) v[j] = (r < batch) ? dZ[(int64_t)r * NP + s * 32 + kb + j] : 0.0f;
    af[s] = pack8(v);
  }
#pragma unroll
  for (int t = 0; t < KP / 16; ++t) {
    const int k = t * 16 + (lane & 15);
    f32x4 acc = {0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < NP / 32; ++s) {
      const bf16x8 bf = load8bf(WT + (int64_t)k * NP + s * 32 + kb);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[s], bf, acc, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int rr = row0 + (lane >> 4) * 4 + j;
      if (rr < batch) {
        float v = acc[j];
        if (gz) v *= gelu_d(gz[(int64_t)rr * KP + k]);
        dX[(int64_t)rr * KP + k] = v;
      }
    }
  }
}

// dW[n][k] += sum_b bf(dZ[b][n]) bf(X[b][k]) over a chunk of 256 batch rows per work-group
// (A operand = dZ^T: rows n, k-dim = batch; B operand = X: cols k).  db[n] += sum_b dZ[b][n].
// Grid: x = batch chunks, y = groups of output tiles (each wave one 16 x 16 tile at a time), so
// that a batch of a few thousand rows still spreads over the whole chip.
template <int KP, int NP>
__global__ void __launch_bounds__(256) k_dense_bwd_weight(const float* __restrict__ dZ, const float* __restrict__ X,
                                                          int batch, float* __restrict__ dW, float* __restrict__ db) {
  constexpr int NT = (NP / 16) * (KP / 16);  // output tiles
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int b0 = blockIdx.x * 256;
  const int kb = (lane >> 4) * 8;
  for (int t = blockIdx.y * 4 + wave; t < NT; t += 4 * gridDim.y) {
    const int tn = t / (KP / 16), tk = t % (KP / 16);
    const int n = tn * 16 + (lane & 15), k = tk * 16 + (lane & 15);
    f32x4 acc = {0, 0, 0, 0};
    for (int s = 0; s < 8; ++s) {
      float va[8], vb[8];
      for (int j = 0; j < 8; ++j) {
        const int bb = b0 + s * 32 + kb + j;
        va[j] = (bb < batch) ? dZ[(int64_t)bb * NP + n] : 0.0f;
        vb[j] = (bb < batch) ? X[(int64_t)bb * KP + k] : 0.0f;
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(pack8(va), pack8(vb), acc, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int nn = tn * 16 + (lane >> 4) * 4 + j;
      unsafeAtomicAdd(&dW[(int64_t)nn * KP + k], acc[j]);
    }
  }
  // bias gradient (first tile group)
  if (blockIdx.y != 0) return;
  for (int n = threadIdx.x; n < NP; n += 256) {
    float acc = 0;
    for (int bb = b0; bb < b0 + 256 && bb < batch; ++bb) acc += dZ[(int64_t)bb * NP + n];
    unsafeAtomicAdd(&db[n], acc);
  }
}

// dY = (Y - T) mask / batch ; loss partial sums 0.5 (Y - T)^2 mask / batch
__global__ void k_mse(const float* Y, const float* Tt, int64_t n, int ncols, int nvalid, int batch, float* dY,
                      double* part) {
  __shared__ double sh[4];
  double acc = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(i % ncols);
    float d = (c < nvalid) ? (Y[i] - Tt[i]) : 0.0f;
    dY[i] = d / batch;
    acc += 0.5 * (double)d * d / batch;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// Adam on FP32 master parameters; the weight part is rounded to BF16 into W and WT.
__global__ void k_adam(int64_t n, float* p, const float* g, float* m1, float* m2, float b1, float b2, float lr,
                       float bc1, float bc2, float eps) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.0f - b1) * gi;
    const float b = b2 * m2[i] + (1.0f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    p[i] -= lr * (a * bc1) / (sqrtf(b * bc2) + eps);
  }
}
__global__ void k_pack(const float* Wm, int rows, int cols, uint16_t* W, uint16_t* WT) {
  const int64_t n = (int64_t)rows * cols;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(i / cols), c = (int)(i % cols);
    const uint16_t h = f2bf(Wm[i]);
    W[i] = h;
    WT[(int64_t)c * rows + r] = h;
  }
}

__global__ void k_sum_part(const double* part, int np, double* out) {
  __shared__ double sh[4];
  double acc = 0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) acc += part[i];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) *out = sh[0] + sh[1] + sh[2] + sh[3];
}

// ---------------------------------------------------------------------------------------
// Learned-guess features and targets (2D).  Per element e with local H1 node (a, b) and
// L2 dof j:  features = [v_c(a,b)/vs (c = 0, 1) | e_j/es | corner_c - centre_c)/xs (4 corners)
//                        | optionally base_v/kvs | base_e/kes],  row stride ld, zero padded.
struct FeatArgs {
  const double* u;
  const double* base;  // nullable: no base block
  double vs, es, xs, kvs, kes;
  const float* mu;  // nullable: no normalisation
  const float* sd;
};

// feature i of element e (0 past the feature count)
__device__ __forceinline__ float feature_value(const KParams& P, const FeatArgs& A, int64_t e, int i) {
  const int k = P.k, D1D = k + 1, ND = D1D * D1D, NL = k * k;
  const int ex = (int)(e % P.n[0]), ey = (int)(e / P.n[0]);
  const int64_t N = P.N, nh1 = 2 * N, ng0 = P.ng[0];
  const double* u = A.u;
  const int nbase = A.base ? 2 * ND + NL : 0;
  const int nin = 2 * ND + NL + 8 + nbase;
  double val = 0.0;
  if (i < 2 * ND) {
    const int c = i / ND, li = i % ND, a = li % D1D, b = li / D1D;
    val = u[nh1 + c * N + (int64_t)(k * ey + b) * ng0 + k * ex + a] / A.vs;
  } else if (i < 2 * ND + NL) {
    val = u[2 * nh1 + e * NL + (i - 2 * ND)] / A.es;
  } else if (i < 2 * ND + NL + 8) {
    const int j = i - 2 * ND - NL, corner = j / 2, c = j % 2;
    const int a = (corner & 1) ? k : 0, b = (corner & 2) ? k : 0;
    double cen = 0;
    for (int q = 0; q < 4; ++q)
      cen += u[c * N + (int64_t)(k * ey + ((q & 2) ? k : 0)) * ng0 + k * ex + ((q & 1) ? k : 0)];
    val = (u[c * N + (int64_t)(k * ey + b) * ng0 + k * ex + a] - 0.25 * cen) / A.xs;
  } else if (i < nin) {
    const int j = i - 2 * ND - NL - 8;
    if (j < 2 * ND) {
      const int c = j / ND, li = j % ND, a = li % D1D, b = li / D1D;
      val = A.base[nh1 + c * N + (int64_t)(k * ey + b) * ng0 + k * ex + a] / A.kvs;
    } else {
      val = A.base[2 * nh1 + e * NL + (j - 2 * ND)] / A.kes;
    }
  }
  if (A.mu && i < nin) val = (val - (double)A.mu[i]) / (double)A.sd[i];
  return (float)val;
}

__global__ void k_features(const KParams P, const FeatArgs A, float* feat, int ld) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.y + threadIdx.y;
  if (e >= P.Ne) return;
  float* f = feat + e * ld;
  for (int i = threadIdx.x; i < ld; i += blockDim.x) f[i] = feature_value(P, A, e, i);
}

// ---------------------------------------------------------------------------------------
// Fused inference: the features of a tile of 16 elements, every layer and the store of the
// network output in one launch.  Each work-group first copies all weights (BF16) and biases into
// LDS and then walks element tiles; the eight waves compute the features of the tile together and
// split each layer's 16-column output tiles, the activations passing between layers through two
// alternating LDS tiles in the MFMA operand layout.  The operand rounding (BF16), the
// accumulation order and the epilogue are those of k_dense_fwd, so the output is the layered
// forward's.  Weight rows are padded by 8 BF16 (16 bytes) in LDS, so the 16 lanes of a quarter
// wave read 16 different rows from 16 different bank groups.
constexpr int FZ_MAXL = 8;
constexpr int FZ_WLDS = 57344;  // BF16 weight elements in LDS (padded rows): 112 KiB
constexpr int FZ_BLDS = FZ_MAXL * 128;
constexpr int FZ_ALD = 128 + 8;  // activation tile row (BF16, padded)

struct FusedNet {
  int nl;
  int kp[FZ_MAXL], np[FZ_MAXL];  // padded widths of each layer
  int wg[FZ_MAXL];                // offset of layer l in the global W (KP x NP blocks)
  int ws[FZ_MAXL];                // offset of layer l in the LDS copy (rows of KP + 8)
  int bo[FZ_MAXL];                // offset of layer l's bias
};

constexpr int FZ_T = 512;  // threads of the work-group (8 waves)

__global__ void __launch_bounds__(FZ_T) k_guess_fused(const KParams P, const FeatArgs FA, const FusedNet F,
                                                     const uint16_t* __restrict__ W, const float* __restrict__ bias,
                                                     float* __restrict__ pred, int ld_out) {
  __shared__ __attribute__((aligned(16))) uint16_t sW[FZ_WLDS];
  __shared__ float sB[FZ_BLDS];
  __shared__ __attribute__((aligned(16))) uint16_t sA[2][16][FZ_ALD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // weights: 8 BF16 (16 bytes) per copy, rows of KP to rows of KP + 8, eight copies in flight
  for (int l = 0; l < F.nl; ++l) {
    const int KP = F.kp[l], NP = F.np[l], KC = KP / 8, tot = NP * KC;
    for (int i0 = tid; i0 < tot; i0 += FZ_T * 8) {
      uint4 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = min(i0 + FZ_T * u, tot - 1);
        const int n = i / KC, kc = i - n * KC;
        v[u] = *reinterpret_cast<const uint4*>(W + F.wg[l] + n * KP + kc * 8);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = i0 + FZ_T * u;
        if (i < tot) {
          const int n = i / KC, kc = i - n * KC;
          *reinterpret_cast<uint4*>(sW + F.ws[l] + n * (KP + 8) + kc * 8) = v[u];
        }
      }
    }
    for (int i = tid; i < NP; i += FZ_T) sB[F.bo[l] + i] = bias[F.bo[l] + i];
  }
  const int64_t ntiles = (P.Ne + 15) / 16;
  const int kb = (lane >> 4) * 8;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t row0 = tile * 16;
    // layer 0 input: the features of the tile's 16 elements, BF16, all threads
    const int KP0 = F.kp[0];
    for (int i = tid; i < 16 * KP0; i += FZ_T) {
      const int r = i / KP0, f = i - r * KP0;
      const int64_t e = row0 + r;
      sA[0][r][f] = f2bf(e < P.Ne ? feature_value(P, FA, e, f) : 0.0f);
    }
    __syncthreads();  // the weights (first tile) and the features are in place
    for (int l = 0; l < F.nl; ++l) {
      const int KP = F.kp[l], NP = F.np[l];
      const bool last = l == F.nl - 1;
      const uint16_t* Wl = sW + F.ws[l];
      const int cur = l & 1;
      bf16x8 af[4];
#pragma unroll
      for (int s = 0; s < 4; ++s)
        if (s < KP / 32) af[s] = *reinterpret_cast<const bf16x8*>(&sA[cur][lane & 15][s * 32 + kb]);
      for (int t = wave; t < NP / 16; t += FZ_T / 64) {
        const int n = t * 16 + (lane & 15);
        f32x4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          if (s < KP / 32) {
            const bf16x8 bf = *reinterpret_cast<const bf16x8*>(Wl + n * (KP + 8) + s * 32 + kb);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[s], bf, acc, 0, 0, 0);
          }
        }
        const float bn = sB[F.bo[l] + n];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int rl = (lane >> 4) * 4 + j;
          const float z = acc[j] + bn;
          if (last) {
            const int64_t rr = row0 + rl;
            if (rr < P.Ne && n < ld_out) pred[rr * ld_out + n] = z;
          } else {
            sA[cur ^ 1][rl][n] = f2bf(gelu(z));
          }
        }
      }
      __syncthreads();  // the next layer's input is complete, this layer's is no longer read
    }
  }
}

// targets: element-local [(k_v - base_v)/kvs | (k_e - base_e)/kes], row stride ld
__global__ void k_targets(const KParams P, const double* kk, const double* base, double kvs, double kes,
                          const float* osc, float* t, int ld) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.y + threadIdx.y;
  if (e >= P.Ne) return;
  const int k = P.k, D1D = k + 1, ND = D1D * D1D, NL = k * k;
  const int ex = (int)(e % P.n[0]), ey = (int)(e / P.n[0]);
  const int64_t N = P.N, nh1 = 2 * N, ng0 = P.ng[0];
  for (int i = threadIdx.x; i < ld; i += blockDim.x) {
    double val = 0.0;
    if (i < 2 * ND) {
      const int c = i / ND, li = i % ND, a = li % D1D, b = li / D1D;
      const int64_t g = nh1 + c * N + (int64_t)(k * ey + b) * ng0 + k * ex + a;
      val = (kk[g] - (base ? base[g] : 0.0)) / kvs;
    } else if (i < 2 * ND + NL) {
      const int64_t g = 2 * nh1 + e * NL + (i - 2 * ND);
      val = (kk[g] - (base ? base[g] : 0.0)) / kes;
    }
    if (osc && i < 2 * ND + NL) val /= (double)osc[i];
    t[e * ld + i] = (float)val;
  }
}

// assembly, step 1: acc_v[node] += kvs * pred_v (sum over the elements containing the node)
__global__ void k_assemble_acc(const KParams P, const float* pred, int ld, double kvs, const float* osc, double* acc) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.y + threadIdx.y;
  if (e >= P.Ne) return;
  const int k = P.k, D1D = k + 1, ND = D1D * D1D;
  const int ex = (int)(e % P.n[0]), ey = (int)(e / P.n[0]);
  const int64_t N = P.N, ng0 = P.ng[0];
  for (int i = threadIdx.x; i < 2 * ND; i += blockDim.x) {
    const int c = i / ND, li = i % ND, a = li % D1D, b = li / D1D;
    const double sc = osc ? (double)osc[i] : 1.0;
    unsafeAtomicAdd(&acc[c * N + (int64_t)(k * ey + b) * ng0 + k * ex + a], kvs * sc * (double)pred[e * ld + i]);
  }
}
// step 2: k_v = base_v + acc / multiplicity (0 on constrained rows), k_x = u_v + tau k_v
__global__ void k_assemble_nodes(const KParams P, const double* acc, const double* base, const double* u, double tau,
                                 double* kout) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= 2 * P.N) return;
  const int64_t N = P.N, node = i % N;
  const int c = (int)(i / N), k = P.k;
  const int I = (int)(node % P.ng[0]), J = (int)(node / P.ng[0]);
  const int mx = (I % k == 0 && I > 0 && I < P.ng[0] - 1) ? 2 : 1;
  const int my = (J % k == 0 && J > 0 && J < P.ng[1] - 1) ? 2 : 1;
  const int gc = (c == 0) ? I : J, ngc = P.ng[c];
  const bool cons = on_wall(P.walls, c, gc, ngc);
  const double kv = cons ? 0.0 : base[2 * N + i] + acc[i] / (mx * my);
  kout[2 * N + i] = kv;
  kout[i] = u[2 * N + i] + tau * kv;
}
__global__ void k_assemble_e(const KParams P, const float* pred, int ld, double kes, const float* osc,
                             const double* base, double* kout) {
  const int NL = P.k * P.k, ND = (P.k + 1) * (P.k + 1);
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)P.Ne * NL) return;
  const int64_t e = i / NL, j = i % NL, off = 4 * P.N;
  const double sc = osc ? (double)osc[2 * ND + j] : 1.0;
  kout[off + i] = base[off + i] + kes * sc * (double)pred[e * ld + 2 * ND + j];
}

// ---------------------------------------------------------------------------------------
template <int KP, int NP>
static void fwd_t(ilh_ctx* c, const float* X, const uint16_t* W, const float* b, int batch, int act, float* Z,
                  float* A) {
  hipLaunchKernelGGL((k_dense_fwd<KP, NP>), dim3((batch + 63) / 64), dim3(256), 0, c->stream, X, W, b, batch, act, Z,
                     A);
}
template <int KP, int NP>
static void bwdd_t(ilh_ctx* c, const float* dZ, const uint16_t* WT, int batch, const float* gz, float* dX) {
  hipLaunchKernelGGL((k_dense_bwd_data<KP, NP>), dim3((batch + 63) / 64), dim3(256), 0, c->stream, dZ, WT, batch, gz,
                     dX);
}
template <int KP, int NP>
static void bwdw_t(ilh_ctx* c, const float* dZ, const float* X, int batch, float* dW, float* db) {
  constexpr int NT = (NP / 16) * (KP / 16);
  hipLaunchKernelGGL((k_dense_bwd_weight<KP, NP>), dim3((batch + 255) / 256, (NT + 3) / 4), dim3(256), 0, c->stream, dZ,
                     X, batch, dW, db);
}

// dispatch on padded (KP, NP) in {32, 64, 96, 128}^2
#define ILH_DISPATCH(FN, KP_, NP_, ...)                                                       \
  do {                                                                                        \
    const int _k = (KP_), _n = (NP_);                                                         \
    if (_k == 64 && _n == 128) FN<64, 128>(__VA_ARGS__);                                      \
    else if (_k == 128 && _n == 128) FN<128, 128>(__VA_ARGS__);                               \
    else if (_k == 128 && _n == 64) FN<128, 64>(__VA_ARGS__);                                 \
    else if (_k == 32 && _n == 128) FN<32, 128>(__VA_ARGS__);                                 \
    else if (_k == 96 && _n == 128) FN<96, 128>(__VA_ARGS__);                                 \
    else if (_k == 128 && _n == 32) FN<128, 32>(__VA_ARGS__);                                 \
    else if (_k == 128 && _n == 96) FN<128, 96>(__VA_ARGS__);                                 \
    else if (_k == 32 && _n == 32) FN<32, 32>(__VA_ARGS__);                                   \
    else if (_k == 64 && _n == 64) FN<64, 64>(__VA_ARGS__);                                   \
    else if (_k == 64 && _n == 32) FN<64, 32>(__VA_ARGS__);                                   \
    else if (_k == 32 && _n == 64) FN<32, 64>(__VA_ARGS__);                                   \
    else return fail(c, ILH_EINVAL, "unsupported MLP layer width (padded widths 32..128)");   \
  } while (0)

static int check_widths(ilh_ctx* c, int nl, const int* w) {
  if (nl < 1 || nl > 8) return fail(c, ILH_EINVAL, "1..8 layers");
  for (int l = 0; l <= nl; ++l)
    if (w[l] < 1 || w[l] > 128) return fail(c, ILH_EINVAL, "MLP widths must be in 1..128");
  return ILH_OK;
}

}  // namespace ilh

using namespace ilh;

extern "C" {

int ilh_guess_features(ilh_ctx* c, const double* u, const double* base, double vs, double es, double xs,
                       double kvs, double kes, const float* mu, const float* sd, float* feat, int ld) {
  ILH_TRY
  if (!c || !u || !feat || c->dim != 2) return fail(c, ILH_EINVAL, "guess features: 2D only, non-null u/feat");
  const int ND = (c->k + 1) * (c->k + 1), NL = c->k * c->k;
  const int nin = 2 * ND + NL + 8 + (base ? 2 * ND + NL : 0);
  if (ld < nin) return fail(c, ILH_EINVAL, "feature row stride too small");
  if (!(vs > 0 && es > 0 && xs > 0 && kvs > 0 && kes > 0)) return fail(c, ILH_EINVAL, "scales must be > 0");
  const FeatArgs fa{u, base, vs, es, xs, kvs, kes, mu, sd};
  hipLaunchKernelGGL(k_features, dim3((unsigned)((c->Ne + 3) / 4)), dim3(64, 4), 0, c->stream, c->kp, fa, feat, ld);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
  ILH_CATCH(c)
}

int ilh_guess_targets(ilh_ctx* c, const double* kk, const double* base, double kvs, double kes, const float* osc,
                      float* t, int ld) {
  ILH_TRY
  if (!c || !kk || !t || c->dim != 2) return fail(c, ILH_EINVAL, "guess targets: 2D only");
  const int ND = (c->k + 1) * (c->k + 1), NL = c->k * c->k;
  if (ld < 2 * ND + NL || !(kvs > 0 && kes > 0)) return fail(c, ILH_EINVAL, "target stride/scales");
  hipLaunchKernelGGL(k_targets, dim3((unsigned)((c->Ne + 3) / 4)), dim3(64, 4), 0, c->stream, c->kp, kk, base, kvs, kes,
                     osc, t, ld);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
  ILH_CATCH(c)
}

int ilh_guess_assemble(ilh_ctx* c, const float* pred, int ld, double kvs, double kes, const float* osc,
                       const double* base, const double* u, double tau, double* kout) {
  ILH_TRY
  if (!c || !pred || !base || !u || !kout || c->dim != 2) return fail(c, ILH_EINVAL, "guess assemble: 2D only");
  const int ND = (c->k + 1) * (c->k + 1), NL = c->k * c->k;
  if (ld < 2 * ND + NL) return fail(c, ILH_EINVAL, "prediction stride too small");
  double* acc = c->pcgbuf;  // nh1 doubles
  int st = launch_fill(c, acc, 0.0, c->nh1);
  if (st) return st;
  hipLaunchKernelGGL(k_assemble_acc, dim3((unsigned)((c->Ne + 3) / 4)), dim3(64, 4), 0, c->stream, c->kp, pred, ld, kvs,
                     osc, acc);
  hipLaunchKernelGGL(k_assemble_nodes, dim3((unsigned)((c->nh1 + 255) / 256)), dim3(256), 0, c->stream, c->kp, acc,
                     base, u, tau, kout);
  hipLaunchKernelGGL(k_assemble_e, dim3((unsigned)((c->nl2 + 255) / 256)), dim3(256), 0, c->stream, c->kp, pred, ld,
                     kes, osc, base, kout);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
  ILH_CATCH(c)
}

int ilh_mlp_forward(ilh_ctx* c, int nl, const int* widths, const uint16_t* W, const float* b, const float* x,
                    int batch, float* zs, float* acts) {
  ILH_TRY
  if (!c || !widths || !W || !b || !x || !zs || !acts || batch < 0) return ILH_EINVAL;
  int st = check_widths(c, nl, widths);
  if (st) return st;
  if (batch == 0) return ILH_OK;
  int64_t wo = 0, bo = 0, ao = 0;
  const float* in = x;
  for (int l = 0; l < nl; ++l) {
    const int KP = pad32(widths[l]), NP = pad32(widths[l + 1]);
    float* Z = zs + ao;
    float* A = acts + ao;
    ILH_DISPATCH(fwd_t, KP, NP, c, in, W + wo, b + bo, batch, l < nl - 1 ? 1 : 0, Z, A);
    in = A;
    wo += (int64_t)KP * NP;
    bo += NP;
    ao += (int64_t)batch * NP;
  }
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
  ILH_CATCH(c)
}

int ilh_guess_mlp_fused(ilh_ctx* c, const ilh_guess_model* m, const double* u, const double* base, float* pred,
                        int ld) {
  ILH_TRY
  if (!c || !m || !u || !pred || !m->W || !m->b || c->dim != 2) return fail(c, ILH_EINVAL, "fused guess MLP: 2D, non-null");
  int st = check_widths(c, m->nl, m->widths);
  if (st) return st;
  if (m->nl > FZ_MAXL) return fail(c, ILH_EINVAL, "fused guess MLP: at most 8 layers");
  const int ND = (c->k + 1) * (c->k + 1), NL = c->k * c->k;
  const int nin = 2 * ND + NL + 8 + (m->with_base ? 2 * ND + NL : 0);
  if (m->widths[0] != nin || m->widths[m->nl] != 2 * ND + NL)
    return fail(c, ILH_EINVAL, "fused guess MLP: widths do not match the features and outputs of this mesh");
  if (m->with_base && !base) return fail(c, ILH_EINVAL, "fused guess MLP: the model takes the base iterate");
  FusedNet F{};
  F.nl = m->nl;
  int wg = 0, ws = 0, bo = 0;
  for (int l = 0; l < m->nl; ++l) {
    F.kp[l] = pad32(m->widths[l]);
    F.np[l] = pad32(m->widths[l + 1]);
    F.wg[l] = wg;
    F.ws[l] = ws;
    F.bo[l] = bo;
    wg += F.kp[l] * F.np[l];
    ws += F.np[l] * (F.kp[l] + 8);
    bo += F.np[l];
  }
  if (ws > FZ_WLDS) return fail(c, ILH_EINVAL, "fused guess MLP: the weights exceed the LDS budget");
  if (ld < F.np[m->nl - 1]) return fail(c, ILH_EINVAL, "prediction stride below the padded output width");
  if ((reinterpret_cast<uintptr_t>(m->W) & 15) != 0) return fail(c, ILH_EINVAL, "fused guess MLP: W not 16-byte aligned");
  const FeatArgs fa{u, m->with_base ? base : nullptr, m->vscale, m->escale, m->xscale, m->kvscale, m->kescale,
                    m->mu, m->sd};
  // one work-group per compute unit at most (the LDS holds one), each walking several tiles
  const int64_t ntiles = (c->Ne + 15) / 16;
  const unsigned nb = (unsigned)std::min<int64_t>(ntiles, 256);
  hipLaunchKernelGGL(k_guess_fused, dim3(nb), dim3(FZ_T), 0, c->stream, c->kp, fa, F, m->W, m->b, pred, ld);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
  ILH_CATCH(c)
}

int ilh_mlp_backward(ilh_ctx* c, int nl, const int* widths, const uint16_t* WT, const float* x, const float* zs,
                     const float* acts, const float* target, int batch, float* dW, float* db, float* work,
                     double* loss) {
  ILH_TRY
  if (!c || !widths || !WT || !x || !zs || !acts || !target || !dW || !db || !work || batch <= 0) return ILH_EINVAL;
  int st = check_widths(c, nl, widths);
  if (st) return st;
  int64_t wtot = 0, btot = 0, atot = 0;
  std::vector<int64_t> woff(nl), boff(nl), aoff(nl);
  for (int l = 0; l < nl; ++l) {
    const int KP = pad32(widths[l]), NP = pad32(widths[l + 1]);
    woff[l] = wtot;
    boff[l] = btot;
    aoff[l] = atot;
    wtot += (int64_t)KP * NP;
    btot += NP;
    atot += (int64_t)batch * NP;
  }
  if ((st = launch_fillf(c, dW, 0.0f, wtot))) return st;
  if ((st = launch_fillf(c, db, 0.0f, btot))) return st;
  // work: two buffers of [batch][128]
  float* g0 = work;
  float* g1 = work + (int64_t)batch * 128;
  const int NPL = pad32(widths[nl]);
  const int64_t nout = (int64_t)batch * NPL;
  const int nbm = 256;
  hipLaunchKernelGGL(k_mse, dim3(nbm), dim3(256), 0, c->stream, acts + aoff[nl - 1], target, nout, NPL, widths[nl],
                     batch, g0, c->red);
  float* dZ = g0;
  for (int l = nl - 1; l >= 0; --l) {
    const int KP = pad32(widths[l]), NP = pad32(widths[l + 1]);
    const float* Xin = (l == 0) ? x : acts + aoff[l - 1];
    ILH_DISPATCH(bwdw_t, KP, NP, c, dZ, Xin, batch, dW + woff[l], db + boff[l]);
    if (l > 0) {
      float* dX = (dZ == g0) ? g1 : g0;
      ILH_DISPATCH(bwdd_t, KP, NP, c, dZ, WT + woff[l], batch, zs + aoff[l - 1], dX);
      dZ = dX;
    }
  }
  ILH_HIP(c, hipGetLastError());
  if (loss) {
    double* d_out = c->red + c->red_blocks * 65 + 2;
    hipLaunchKernelGGL(k_sum_part, dim3(1), dim3(256), 0, c->stream, c->red, nbm, d_out);
    ILH_HIP(c, hipMemcpyAsync(c->red_host + 2, d_out, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    ILH_HIP(c, hipStreamSynchronize(c->stream));
    *loss = c->red_host[2];
  }
  return ILH_OK;
  ILH_CATCH(c)
}

int ilh_mlp_adam(ilh_ctx* c, int64_t n, float* p, const float* g, float* m1, float* m2, int step, double lr,
                 double beta1, double beta2, double eps) {
  ILH_TRY
  if (!c || !p || !g || !m1 || !m2 || n < 0 || step < 1) return ILH_EINVAL;
  const double bc1 = 1.0 / (1.0 - std::pow(beta1, step)), bc2 = 1.0 / (1.0 - std::pow(beta2, step));
  hipLaunchKernelGGL(k_adam, dim3(1024), dim3(256), 0, c->stream, n, p, g, m1, m2, (float)beta1, (float)beta2,
                     (float)lr, (float)bc1, (float)bc2, (float)eps);
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
  ILH_CATCH(c)
}

int ilh_mlp_pack(ilh_ctx* c, int nl, const int* widths, const float* Wmaster, uint16_t* W, uint16_t* WT) {
  ILH_TRY
  if (!c || !widths || !Wmaster || !W || !WT) return ILH_EINVAL;
  int st = check_widths(c, nl, widths);
  if (st) return st;
  int64_t off = 0;
  for (int l = 0; l < nl; ++l) {
    const int KP = pad32(widths[l]), NP = pad32(widths[l + 1]);
    hipLaunchKernelGGL(k_pack, dim3(256), dim3(256), 0, c->stream, Wmaster + off, NP, KP, W + off, WT + off);
    off += (int64_t)KP * NP;
  }
  ILH_HIP(c, hipGetLastError());
  return ILH_OK;
  ILH_CATCH(c)
}

}  // extern "C"

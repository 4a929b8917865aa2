// Host side of the ilh library: discretisation set-up, the C ABI and the host-driven
// Newton-Krylov stage solver (Sec. 3.5) whose vectors and kernels live on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ilh_internal.h"

// Static scratch of ilh_jvp_noalloc: one array per GPU, held until the process ends.  Host code
// never uses the name `scratch` as an address (on the host it is only a stand-in for the symbol):
// each device's address comes from hipGetSymbolAddress, resolved once per device at context
// creation with that device current, and kernels receive that address.
static __device__ __align__(256) unsigned char scratch[ILH_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// This device's address of `scratch` (dev must be the current device).
int resolve_scratch(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return ILH_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return ILH_EHIP;
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return ILH_OK;
}
}  // namespace

using ilh::EArgs;

namespace ilh {

int fail(ilh_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}
int hip_fail(ilh_ctx* c, hipError_t e, const char* what) {
  if (c) c->err = std::string(what) + ": " + hipGetErrorString(e);
  return (e == hipErrorOutOfMemory) ? ILH_ENOMEM : ILH_EHIP;
}

// ---------------------------------------------------------------- 1D bases (host, FP64)
// Legendre P_n and its derivative on [-1, 1] by the three-term recurrence.
static void legendre(int n, double x, double& p, double& dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    p = 1.0;
    dp = 0.0;
    return;
  }
  for (int k = 2; k <= n; ++k) {
    const double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = pk;
  }
  p = p1;
  dp = (std::fabs(x) < 1.0) ? n * (x * p1 - p0) / (x * x - 1.0) : 0.5 * n * (n + 1) * std::pow(x, n + 1);
}

// Gauss-Legendre points/weights on [0, 1] (Newton on P_n from Chebyshev guesses).
static void gauss(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(n, z, p, dp);
      const double dz = p / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p, dp;
    legendre(n, z, p, dp);
    x[n - 1 - i] = 0.5 * (z + 1.0);
    w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);  // = 2/((1-z^2) P'^2) on [-1,1], halved
  }
}

// Gauss-Lobatto-Legendre points on [0, 1]: endpoints and the roots of P_k'.
static std::vector<double> gll(int k) {
  std::vector<double> x(k + 1);
  x[0] = 0.0;
  x[k] = 1.0;
  for (int i = 1; i < k; ++i) {
    double z = -std::cos(M_PI * i / k);
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(k, z, p, dp);
      // P'' from the Legendre equation (1 - z^2) P'' = 2 z P' - k (k+1) P
      const double ddp = (2.0 * z * dp - k * (k + 1.0) * p) / (1.0 - z * z);
      const double dz = dp / ddp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = 0.5 * (z + 1.0);
  }
  return x;
}

static double binom(int n, int k) {
  double r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

static bool invert(std::vector<double>& A, int n) {  // Gauss-Jordan with partial pivoting
  std::vector<double> I(n * n, 0.0);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) return false;
    for (int j = 0; j < n; ++j) {
      std::swap(A[c * n + j], A[piv * n + j]);
      std::swap(I[c * n + j], I[piv * n + j]);
    }
    const double d = A[c * n + c];
    for (int j = 0; j < n; ++j) {
      A[c * n + j] /= d;
      I[c * n + j] /= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = A[r * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        A[r * n + j] -= f * A[c * n + j];
        I[r * n + j] -= f * I[c * n + j];
      }
    }
  }
  A = I;
  return true;
}

static constexpr int TPOOL = 4096;  // event pairs

int tflush(ilh_ctx* c) {
  if (c->tused == 0) return ILH_OK;
  ILH_HIP(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i < c->tused; ++i) {
    if (c->tcls[i] < 0) continue;  // dropped
    float ms = 0.f;
    ILH_HIP(c, hipEventElapsedTime(&ms, c->tev[2 * i], c->tev[2 * i + 1]));
    c->tms[c->tcls[i]] += ms;
    c->tcnt[c->tcls[i]] += 1;
  }
  c->tused = 0;
  ++c->tgen;
  return ILH_OK;
}

void tdrop(ilh_ctx* c, int slot, int64_t gen) {
  if (slot >= 0 && gen == c->tgen && slot < c->tused) c->tcls[slot] = -1;
}

int tstart(ilh_ctx* c, int cls) {
  if (!c->timing) return -1;
  if (c->tused == TPOOL && tflush(c) != ILH_OK) return -1;
  const int slot = c->tused++;
  c->tcls[slot] = cls;
  if (hipEventRecord(c->tev[2 * slot], c->stream) != hipSuccess) return -1;
  return slot;
}

void tstop(ilh_ctx* c, int slot) {
  if (slot >= 0) (void)hipEventRecord(c->tev[2 * slot + 1], c->stream);
}

int tstart_k(ilh_ctx* c, int cls) {
  if (!c->timing) return -1;
  if (c->tused == TPOOL && tflush(c) != ILH_OK) return -1;
  const int slot = c->tused++;
  c->tcls[slot] = cls;
  c->xev0 = c->tev[2 * slot];
  c->xev1 = c->tev[2 * slot + 1];
  return slot;
}

void tstop_k(ilh_ctx* c, int slot) {
  if (slot < 0) return;
  if (c->xev0) {
    (void)hipEventRecord(c->xev0, c->stream);
    (void)hipEventRecord(c->xev1, c->stream);
    c->xev0 = c->xev1 = nullptr;
  }
}

template <typename T>
static int dalloc(ilh_ctx* c, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  ILH_HIP(c, hipMalloc((void**)p, count * sizeof(T)));
  return ILH_OK;
}

// Krylov workspace for restart length m: the basis V, Z in FP64 (kry) or FP32 (kryf, f32 = true),
// and two FP32 block vectors (kry32) for the cast actions and the probed preconditioner.
static int ensure_solver_ws(ilh_ctx* c, int m, bool f32 = false) {
  int st;
  if (!c->kry32 && (st = dalloc(c, &c->kry32, (size_t)2 * c->nblock))) return st;
  if (f32) {
    if (c->kryf && c->kryf_m >= m) return ILH_OK;
    if (c->kryf) (void)hipFree(c->kryf);
    c->kryf = nullptr;
    if ((st = dalloc(c, &c->kryf, (size_t)(2 * m + 1) * c->nblock))) return st;
    c->kryf_m = m;
    return ILH_OK;
  }
  if (c->kry && c->kry_m >= m) return ILH_OK;
  if (c->kry) (void)hipFree(c->kry);
  c->kry = nullptr;
  if ((st = dalloc(c, &c->kry, (size_t)(2 * m + 1) * c->nblock))) return st;
  c->kry_m = m;
  return ILH_OK;
}

}  // namespace ilh

using namespace ilh;

extern "C" {

const char* ilh_status_string(int s) {
  switch (s) {
    case ILH_OK: return "ok";
    case ILH_EINVAL: return "invalid argument";
    case ILH_EHIP: return "HIP error";
    case ILH_ENOMEM: return "out of device memory";
    case ILH_ETANGLED: return "mesh tangled (det J <= 0 after line search)";
    case ILH_ENOCONV: return "Newton did not converge";
    case ILH_ENONFINITE: return "non-finite residual";
  }
  return "unknown status";
}

void ilh_setup_defaults(ilh_setup* s, int problem) {
  const int dim = s->dim, n0 = s->n[0], n1 = s->n[1], n2 = s->n[2], k = s->order_v;
  std::memset(s, 0, sizeof(*s));
  s->dim = dim;
  s->n[0] = n0;
  s->n[1] = n1;
  s->n[2] = n2;
  s->order_v = k;
  s->problem = problem;
  s->q1 = 0.5;
  s->q2 = 1.0;
  s->psi0 = 0.5;
  s->dscale_mode = ILH_DSCALE_CONST;
  s->dscale_width = 1e-3;
  s->eps_e = 1e-6;
  s->tg_source = (problem == ILH_PROBLEM_TG2D) ? 1 : 0;
  for (int d = 0; d < 3; ++d) {
    s->lo[d] = 0.0;
    s->hi[d] = 1.0;
  }
}

void ilh_newton_defaults(ilh_newton_opts* o) {
  o->tol = 1e-10;
  o->max_newton = 30;
  o->restart = 15;
  o->gmres_rtol = 1e-6;
  o->gmres_maxit = 150;
  o->jvp_prec = 32;
  o->max_halvings = 10;
  o->pcg_iters = 0;
  o->prec_coupled = 1;
  o->guess_fallback = 1;
  o->ls_residual = 1;
  o->prec_probe = 0;
  o->prec_lag = 0;
  o->graphs = 0;
  o->basis64 = 0;
  o->cgs2 = 0;
}

const char* ilh_last_error(const ilh_ctx* c) { return c ? c->err.c_str() : "null context"; }

int ilh_set_stream(ilh_ctx* c, void* stream) {
  ILH_TRY
  if (!c) return ILH_EINVAL;
  c->stream = (hipStream_t)stream;
  return ILH_OK;
  ILH_CATCH(c)
}

int ilh_sizes(const ilh_ctx* c, int64_t* nh1, int64_t* nl2, int64_t* nb, int64_t* nq) {
  if (!c) return ILH_EINVAL;
  if (nh1) *nh1 = c->nh1;
  if (nl2) *nl2 = c->nl2;
  if (nb) *nb = c->nblock;
  if (nq) *nq = c->nqp;
  return ILH_OK;
}

void ilh_destroy(ilh_ctx* c) {
  if (!c) return;
  void* ptrs[] = {c->gsp, c->kryf, c->x0, c->rj0, c->j0e, c->tab, c->tabf, c->mq, c->detJ0, c->gamma, c->rho0, c->e0, c->MEinv, c->Mdiag,
                  c->w64, c->w32, c->red, c->ws, c->pcgbuf, c->kry, c->nwt, c->kry32, c->hdev, c->gmd, c->sdk, c->rkw, c->pdv, c->peinv, c->gscr, c->gres, c->pgb, c->dmin_part};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (void* p : c->qd)
    if (p) (void)hipFree(p);
  for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
  if (c->pev) (void)hipEventDestroy(c->pev);
  for (hipGraphExec_t e : c->gexec)
    if (e) (void)hipGraphExecDestroy(e);
  if (c->capstream) (void)hipStreamDestroy(c->capstream);
  if (c->red_host) (void)hipHostFree(c->red_host);
  if (c->hest) (void)hipHostFree(c->hest);
  delete c;
}

// Body of ilh_create; *made receives the context as soon as it exists, so that the exported
// wrapper can release it when a host allocation throws part-way.  Every error return below
// releases the context itself.
static int create_ctx(const ilh_setup* s, void* stream, ilh_ctx** out, ilh_ctx** made) {
  if (!s || !out) return ILH_EINVAL;
  *out = nullptr;
  ilh_ctx* c = new ilh_ctx();
  *made = c;
  c->s = *s;
  c->stream = (hipStream_t)stream;
  auto bad = [&](const std::string& m) {
    // creation failures are reported through stderr because no context survives
    std::fprintf(stderr, "ilh_create: %s\n", m.c_str());
    ilh_destroy(c);
    return ILH_EINVAL;
  };
  const int dim = s->dim, k = s->order_v;
  if (dim != 2 && dim != 3) return bad("dim must be 2 or 3");
  if (k < 1 || (dim == 2 && k > 4) || (dim == 3 && k > 3)) return bad("order_v out of range");
  if (s->nq1d != 0 && s->nq1d != 2 * k) return bad("only nq1d = 2k is built");
  for (int d = 0; d < dim; ++d)
    if (s->n[d] < 1) return bad("n must be >= 1");
  const int prob = s->problem;
  if (prob < 0 || prob > ILH_PROBLEM_UNIFORM) return bad("unknown problem");
  if ((prob == ILH_PROBLEM_TG2D || prob == ILH_PROBLEM_TRIPLE) && dim != 2) return bad("problem is 2D");
  if (prob == ILH_PROBLEM_TG3D && dim != 3) return bad("problem is 3D");
  if (s->tg_source && prob != ILH_PROBLEM_TG2D) return bad("tg_source requires TG2D");
  if (prob == ILH_PROBLEM_CUSTOM && (!s->rho0_elem || !s->gamma_elem || !s->e0_elem))
    return bad("custom problem needs rho0/gamma/e0 arrays");
  if (s->eps_e <= 0) return bad("eps_e must be > 0");
  if (s->visc_on && s->dscale_mode == ILH_DSCALE_CONST && !(s->dscale_width > 0)) return bad("dscale_width must be > 0");
  if (s->visc_on && (s->psi0 <= 0 || s->psi0 >= 1)) return bad("psi0 must lie in (0, 1)");
  if (s->free_faces < 0 || s->free_faces >= (1 << (2 * dim))) return bad("free_faces has bits beyond the box's faces");
  c->general = s->x0 != nullptr || s->free_faces != 0;
  const int walls = ((1 << (2 * dim)) - 1) & ~s->free_faces;

  c->dim = dim;
  c->k = k;
  c->D1D = k + 1;
  c->Q1D = 2 * k;
  c->L1D = k;
  c->Nh = (int)std::pow(k + 1, dim);
  c->Nl = (int)std::pow(k, dim);
  c->Q = (int)std::pow(2 * k, dim);
  // box
  if (prob == ILH_PROBLEM_TG2D || prob == ILH_PROBLEM_TG3D) {
    for (int d = 0; d < 3; ++d) {
      c->lo[d] = 0.0;
      c->hi[d] = 1.0;
    }
  } else if (prob == ILH_PROBLEM_TRIPLE) {
    c->lo[0] = 0;
    c->lo[1] = 0;
    c->hi[0] = 7;
    c->hi[1] = 3;
  } else {
    for (int d = 0; d < dim; ++d) {
      c->lo[d] = s->lo[d];
      c->hi[d] = s->hi[d];
      if (!(c->hi[d] > c->lo[d])) return bad("box must have hi > lo");
    }
  }
  c->Ne = 1;
  c->N = 1;
  for (int d = 0; d < dim; ++d) {
    c->n[d] = s->n[d];
    c->ng[d] = k * s->n[d] + 1;
    c->Ne *= s->n[d];
    c->N *= c->ng[d];
  }
  if (c->Ne > 2147483647LL / c->Q) return bad("mesh too large for 32-bit element indexing");
  c->nh1 = dim * c->N;
  c->nl2 = c->Ne * c->Nl;
  c->nblock = 2 * c->nh1 + c->nl2;
  c->nqp = c->Ne * c->Q;
  const int D1D = c->D1D, Q1D = c->Q1D, L1D = c->L1D;

  // 1D tables
  std::vector<double> xg, wg;
  gauss(Q1D, xg, wg);
  const std::vector<double> xn = gll(k);
  std::vector<double> B(Q1D * D1D), G(Q1D * D1D), BL(Q1D * L1D);
  for (int q = 0; q < Q1D; ++q) {
    const double t = xg[q];
    for (int a = 0; a < D1D; ++a) {
      double num = 1, den = 1, der = 0;
      for (int b = 0; b < D1D; ++b) {
        if (b == a) continue;
        num *= t - xn[b];
        den *= xn[a] - xn[b];
      }
      for (int m = 0; m < D1D; ++m) {
        if (m == a) continue;
        double pr = 1;
        for (int b = 0; b < D1D; ++b)
          if (b != a && b != m) pr *= t - xn[b];
        der += pr;
      }
      B[q * D1D + a] = num / den;
      G[q * D1D + a] = der / den;
    }
    for (int j = 0; j < L1D; ++j)
      BL[q * L1D + j] = binom(k - 1, j) * std::pow(t, j) * std::pow(1 - t, k - 1 - j);
  }
  std::vector<double> tab;
  tab.insert(tab.end(), B.begin(), B.end());
  tab.insert(tab.end(), G.begin(), G.end());
  tab.insert(tab.end(), BL.begin(), BL.end());
  tab.insert(tab.end(), wg.begin(), wg.end());
  tab.insert(tab.end(), xg.begin(), xg.end());
  tab.insert(tab.end(), xn.begin(), xn.end());
  std::vector<float> tabf(tab.begin(), tab.end());
  c->h_B = B;
  c->h_G = G;
  c->h_BL = BL;
  c->h_gll = xn;
  c->h_w1 = wg;

  // per-element material data
  std::vector<double> rho0(c->Ne, 1.0), gam(c->Ne, 5.0 / 3.0), e0(c->Ne, 0.0);
  double h[3] = {1, 1, 1};
  for (int d = 0; d < dim; ++d) h[d] = (c->hi[d] - c->lo[d]) / c->n[d];
  if (prob == ILH_PROBLEM_TRIPLE) {
    for (int64_t e = 0; e < c->Ne; ++e) {
      const int ex = (int)(e % c->n[0]), ey = (int)(e / c->n[0]);
      const double xc = c->lo[0] + h[0] * (ex + 0.5), yc = c->lo[1] + h[1] * (ey + 0.5);
      double r, p, g;
      if (xc < 1.0) { r = 1.0; p = 1.0; g = 1.5; }
      else if (yc < 1.5) { r = 1.0; p = 0.1; g = 1.4; }
      else { r = 0.125; p = 0.1; g = 1.5; }
      rho0[e] = r;
      gam[e] = g;
      e0[e] = p / ((g - 1.0) * r);
    }
  } else if (prob == ILH_PROBLEM_UNIFORM) {
    std::fill(gam.begin(), gam.end(), 1.4);
    std::fill(e0.begin(), e0.end(), 2.5);
  }
  if (s->rho0_elem) std::copy(s->rho0_elem, s->rho0_elem + c->Ne, rho0.begin());
  if (s->gamma_elem) std::copy(s->gamma_elem, s->gamma_elem + c->Ne, gam.begin());
  if (s->e0_elem) std::copy(s->e0_elem, s->e0_elem + c->Ne, e0.begin());
  for (int64_t e = 0; e < c->Ne; ++e)
    if (!(rho0[e] > 0) || !(gam[e] > 1)) return bad("rho0 must be > 0 and gamma > 1");

  // quadrature data: affine Cartesian elements, det J0 = prod h_d (a curved initial mesh x0
  // replaces it per point below)
  double detJ0 = 1;
  for (int d = 0; d < dim; ++d) detJ0 *= h[d];
  const int Q = c->Q;
  std::vector<double> qw(Q);
  for (int q = 0; q < Q; ++q) {
    double w = 1;
    int r = q;
    for (int d = 0; d < dim; ++d) {
      w *= wg[r % Q1D];
      r /= Q1D;
    }
    qw[q] = w;
  }
  c->h_qw = qw;
  std::vector<double> mq(c->nqp), dj0(c->nqp, detJ0), rj0(c->Ne), j0e(c->Ne, detJ0);
  for (int64_t e = 0; e < c->Ne; ++e) rj0[e] = rho0[e] * detJ0;
  const int Nh = c->Nh;
  const int64_t s1 = c->ng[0], s2 = (int64_t)c->ng[0] * c->ng[1];
  // global index of element-local H1 node li of element e
  auto gnode = [&](int64_t e, int li) -> int64_t {
    const int ex = (int)(e % c->n[0]), ey = (int)((e / c->n[0]) % c->n[1]),
              ez = dim == 3 ? (int)(e / ((int64_t)c->n[0] * c->n[1])) : 0;
    const int a = li % D1D, b = (li / D1D) % D1D, cc = dim == 3 ? li / (D1D * D1D) : 0;
    return (k * ex + a) + s1 * (k * ey + b) + s2 * (k * ez + cc);
  };
  // reference gradient of local node li at quadrature point q (direction dd) and its value
  auto wgrad = [&](int li, int q, int dd) {
    const int a[3] = {li % D1D, (li / D1D) % D1D, dim == 3 ? li / (D1D * D1D) : 0};
    const int qi[3] = {q % Q1D, (q / Q1D) % Q1D, dim == 3 ? q / (Q1D * Q1D) : 0};
    double v = 1;
    for (int d = 0; d < dim; ++d) v *= (d == dd ? G : B)[qi[d] * D1D + a[d]];
    return v;
  };
  if (s->x0) {
    // curved initial mesh (Sec. 2.1: the positions are an H1 field): J0 = sum_n x0_n (x) grad w_n
    // and m_q = rho0 det J0 w_q at every quadrature point
    for (int64_t e = 0; e < c->Ne; ++e) {
      double jsum = 0;
      for (int q = 0; q < Q; ++q) {
        double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (int li = 0; li < Nh; ++li) {
          const int64_t g = gnode(e, li);
          for (int dd = 0; dd < dim; ++dd) {
            const double gw = wgrad(li, q, dd);
            for (int cc = 0; cc < dim; ++cc) J[cc][dd] += s->x0[cc * c->N + g] * gw;
          }
        }
        const double dj = dim == 2 ? J[0][0] * J[1][1] - J[0][1] * J[1][0]
                                   : J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                                         J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                                         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        if (!(dj > 0)) return bad("x0: det J0 <= 0 at a quadrature point");
        dj0[e * Q + q] = dj;
        jsum += dj * qw[q];
      }
      double wsum = 0;
      for (int q = 0; q < Q; ++q) wsum += qw[q];
      j0e[e] = jsum / wsum;  // not read by the generic kernels; kept meaningful
      rj0[e] = rho0[e] * j0e[e];
    }
  }
  for (int64_t e = 0; e < c->Ne; ++e)
    for (int q = 0; q < Q; ++q) mq[e * Q + q] = rho0[e] * dj0[e * Q + q] * qw[q];
  // L2 mass: M_E,e = rho0_e detJ0 (M1 x M1 [x M1]) with the 1D Bernstein mass M1
  std::vector<double> M1(L1D * L1D, 0.0);
  for (int i = 0; i < L1D; ++i)
    for (int j = 0; j < L1D; ++j)
      for (int q = 0; q < Q1D; ++q) M1[i * L1D + j] += wg[q] * BL[q * L1D + i] * BL[q * L1D + j];
  if (!invert(M1, L1D)) return bad("singular L2 mass");
  const int Nl = c->Nl;
  std::vector<double> me(Nl * Nl + c->Ne);
  for (int i = 0; i < Nl; ++i)
    for (int j = 0; j < Nl; ++j) {
      double v = 1;
      int ri = i, rj = j;
      for (int d = 0; d < dim; ++d) {
        v *= M1[(ri % L1D) * L1D + (rj % L1D)];
        ri /= L1D;
        rj /= L1D;
      }
      me[i * Nl + j] = v;
    }
  for (int64_t e = 0; e < c->Ne; ++e) me[Nl * Nl + e] = 1.0 / (rho0[e] * detJ0);
  if (s->x0) {
    // curved: the element blocks M_E,e(i, j) = sum_q m_q phi_i phi_j are not multiples of one
    // reference block; each is inverted on its own
    me.assign((size_t)c->Ne * Nl * Nl, 0.0);
    std::vector<double> blk(Nl * Nl), phi(Nl);
    for (int64_t e = 0; e < c->Ne; ++e) {
      std::fill(blk.begin(), blk.end(), 0.0);
      for (int q = 0; q < Q; ++q) {
        const int qi[3] = {q % Q1D, (q / Q1D) % Q1D, dim == 3 ? q / (Q1D * Q1D) : 0};
        for (int j = 0; j < Nl; ++j) {
          const int jl[3] = {j % L1D, (j / L1D) % L1D, dim == 3 ? j / (L1D * L1D) : 0};
          double v = 1;
          for (int d = 0; d < dim; ++d) v *= BL[qi[d] * L1D + jl[d]];
          phi[j] = v;
        }
        for (int i = 0; i < Nl; ++i)
          for (int j = 0; j < Nl; ++j) blk[i * Nl + j] += mq[e * Q + q] * phi[i] * phi[j];
      }
      if (!invert(blk, Nl)) return bad("singular L2 mass block");
      std::copy(blk.begin(), blk.end(), me.begin() + e * Nl * Nl);
    }
  }
  // H1 mass diagonal (tensor product of 1D sums) with ones on constrained rows
  std::vector<double> d1(D1D, 0.0);
  for (int a = 0; a < D1D; ++a)
    for (int q = 0; q < Q1D; ++q) d1[a] += wg[q] * B[q * D1D + a] * B[q * D1D + a];
  std::vector<double> diag(c->N, 0.0);
  if (s->x0) {  // diag(M_s)(n) = sum over elements and points of m_q w_n(xi_q)^2
    for (int64_t e = 0; e < c->Ne; ++e)
      for (int li = 0; li < Nh; ++li) {
        double v = 0;
        for (int q = 0; q < Q; ++q) {
          const double wv = wgrad(li, q, -1);
          v += mq[e * Q + q] * wv * wv;
        }
        diag[gnode(e, li)] += v;
      }
  }
  for (int64_t e = 0; e < (s->x0 ? 0 : c->Ne); ++e) {
    const int ex = (int)(e % c->n[0]), ey = (int)((e / c->n[0]) % c->n[1]),
              ez = dim == 3 ? (int)(e / ((int64_t)c->n[0] * c->n[1])) : 0;
    for (int li = 0; li < Nh; ++li) {
      const int a = li % D1D, b = (li / D1D) % D1D, cc = dim == 3 ? li / (D1D * D1D) : 0;
      double v = rho0[e] * detJ0 * d1[a] * d1[b] * (dim == 3 ? d1[cc] : 1.0);
      diag[(k * ex + a) + s1 * (k * ey + b) + s2 * (k * ez + cc)] += v;
    }
  }
  std::vector<double> Md(c->nh1);
  for (int cc = 0; cc < dim; ++cc)
    for (int64_t node = 0; node < c->N; ++node) {
      int64_t r = node;
      int gi[3] = {0, 0, 0};
      for (int d = 0; d < dim; ++d) {
        gi[d] = (int)(r % c->ng[d]);
        r /= c->ng[d];
      }
      const bool cons = on_wall(walls, cc, gi[cc], c->ng[cc]);
      Md[cc * c->N + node] = cons ? 1.0 : diag[node];
    }

  // viscosity parameters
  double vol = 1;
  for (int d = 0; d < dim; ++d) vol *= c->hi[d] - c->lo[d];
  if (s->x0) {  // |Omega_0| of the curved mesh by quadrature
    vol = 0;
    for (int64_t e = 0; e < c->Ne; ++e)
      for (int q = 0; q < Q; ++q) vol += dj0[e * Q + q] * qw[q];
  }
  const double h0 = s->h0 > 0 ? s->h0 : std::pow(vol / c->Ne, 1.0 / dim) / k;
  const double hc = s->h_coarse > 0 ? s->h_coarse : h0;

  int st;
  const size_t ntab = tab.size();
  if ((st = dalloc(c, &c->tab, ntab)) || (st = dalloc(c, &c->tabf, ntab)) || (st = dalloc(c, &c->mq, c->nqp)) ||
      (st = dalloc(c, &c->detJ0, c->nqp)) || (st = dalloc(c, &c->gamma, c->Ne)) || (st = dalloc(c, &c->rho0, c->Ne)) ||
      (st = dalloc(c, &c->e0, c->Ne)) || (st = dalloc(c, &c->MEinv, me.size())) || (st = dalloc(c, &c->Mdiag, c->nh1)) ||
      (st = dalloc(c, &c->w64, c->nblock)) || (st = dalloc(c, &c->w32, c->nblock)) ||
      (st = dalloc(c, &c->red, (size_t)c->red_blocks * 66 + 256)) || (st = dalloc(c, &c->pcgbuf, 4 * c->nh1 + 16)) ||
      (st = dalloc(c, &c->rj0, c->Ne)) || (st = dalloc(c, &c->j0e, c->Ne)) ||
      (s->x0 && (st = dalloc(c, &c->x0, c->nh1)))) {
    std::fprintf(stderr, "ilh_create: %s\n", c->err.c_str());
    ilh_destroy(c);
    return st;
  }
  c->ws_len = std::max<int64_t>(c->nl2, (c->nqp + 255) / 256 + 16);
  if ((st = dalloc(c, &c->ws, c->ws_len))) {
    ilh_destroy(c);
    return st;
  }
  if (hipHostMalloc((void**)&c->red_host, 64 * sizeof(double)) != hipSuccess) {
    ilh_destroy(c);
    return ILH_ENOMEM;
  }
  auto up = [&](void* d, const void* h, size_t bytes) { return hipMemcpy(d, h, bytes, hipMemcpyHostToDevice); };
  if (up(c->tab, tab.data(), ntab * 8) || up(c->tabf, tabf.data(), ntab * 4) || up(c->mq, mq.data(), c->nqp * 8) ||
      up(c->detJ0, dj0.data(), c->nqp * 8) || up(c->gamma, gam.data(), c->Ne * 8) ||
      up(c->rho0, rho0.data(), c->Ne * 8) || up(c->e0, e0.data(), c->Ne * 8) ||
      up(c->MEinv, me.data(), me.size() * 8) || up(c->Mdiag, Md.data(), c->nh1 * 8) ||
      up(c->rj0, rj0.data(), c->Ne * 8) || up(c->j0e, j0e.data(), c->Ne * 8) ||
      (s->x0 && up(c->x0, s->x0, c->nh1 * 8))) {
    std::fprintf(stderr, "ilh_create: upload failed\n");
    ilh_destroy(c);
    return ILH_EHIP;
  }
  KParams& P = c->kp;
  P.dim = dim;
  P.k = k;
  for (int d = 0; d < 3; ++d) {
    P.n[d] = d < dim ? c->n[d] : 1;
    P.ng[d] = d < dim ? c->ng[d] : 1;
  }
  P.Ne = (int)c->Ne;
  P.N = c->N;
  P.tab = c->tab;
  P.tabf = c->tabf;
  P.mq = c->mq;
  P.detJ0 = c->detJ0;
  P.gamma = c->gamma;
  P.rj0 = c->rj0;
  P.j0e = c->j0e;
  P.eps_e = s->eps_e;
  P.visc = s->visc_on;
  P.dsc_mode = s->dscale_mode;
  P.tg_source = s->tg_source;
  P.q1 = s->q1;
  P.q2 = s->q2;
  P.h0 = h0;
  P.hc_inv = 1.0 / hc;
  P.dsc_w = s->dscale_width;
  P.psi_shift = s->visc_on ? std::atanh(1.0 - 2.0 * s->psi0) : 0.0;
  P.walls = walls;
  {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || resolve_scratch(dev, &c->scratch) != ILH_OK) {
      std::fprintf(stderr, "ilh_create: could not resolve the static scratch array on this device\n");
      ilh_destroy(c);
      return ILH_EHIP;
    }
  }
  if (s->x0) {
    c->me_stride = (int64_t)Nl * Nl;
    c->me_scale = nullptr;
  } else {
    c->me_stride = 0;
    c->me_scale = c->MEinv + Nl * Nl;
  }
  if (c->general) c->jvp_variant = 1;
  *out = c;
  return ILH_OK;
}

int ilh_create(const ilh_setup* s, void* stream, ilh_ctx** out) {
  ilh_ctx* made = nullptr;
  int st;
  try {
    return create_ctx(s, stream, out, &made);
  } catch (const std::bad_alloc&) {
    st = ILH_ENOMEM;
  } catch (...) {
    st = ILH_EINVAL;
  }
  // an exception left the context half-built (create_ctx frees it on every error return)
  std::fprintf(stderr, "ilh_create: %s\n", st == ILH_ENOMEM ? "host allocation failed" : "unexpected C++ exception");
  ilh_destroy(made);
  if (out) *out = nullptr;
  return st;
}

int ilh_init_state(ilh_ctx* c, double* u) {
  ILH_TRY
  if (!c || !u) return ILH_EINVAL;
  return init_state_dev(c, u, nullptr);
  ILH_CATCH(c)
}

int ilh_force(ilh_ctx* c, const double* w, double* f1, double* ftv) {
  ILH_TRY
  if (!c || !w || !f1 || !ftv) return ILH_EINVAL;
  int st = launch_fill(c, f1, 0.0, c->nh1);
  if (st) return st;
  EArgs<double> a{w, w + c->nh1, w + 2 * c->nh1, nullptr, nullptr, 0.0, f1, ftv};
  return launch_elem(c, M_FORCE, 64, &a, nullptr);
  ILH_CATCH(c)
}

int ilh_force_jvp(ilh_ctx* c, int prec, const double* w, const void* dw, void* df1, void* dftv) {
  ILH_TRY
  if (!c || !w || !dw || !df1 || !dftv) return ILH_EINVAL;
  int st;
  if (prec == 64) {
    if ((st = launch_fill(c, (double*)df1, 0.0, c->nh1))) return st;
    EArgs<double> a{w, w + c->nh1, w + 2 * c->nh1, nullptr, (const double*)dw, 1.0, (double*)df1, (double*)dftv};
    return launch_elem(c, M_FJVP, 64, &a, nullptr);
  }
  if (prec == 32) {
    if ((st = launch_cast_d2f(c, c->w32, w, c->nblock))) return st;
    if ((st = launch_fillf(c, (float*)df1, 0.0f, c->nh1))) return st;
    EArgs<float> a{w, c->w32 + c->nh1, c->w32 + 2 * c->nh1, nullptr, (const float*)dw, 1.0, (float*)df1,
                   (float*)dftv};
    return launch_elem(c, M_FJVP, 32, nullptr, &a);
  }
  return fail(c, ILH_EINVAL, "prec must be 32 or 64");
  ILH_CATCH(c)
}

// The stage residual; the kernels accumulate the velocity rows of r, so they start from zero:
// zeroed here unless the caller has zeroed them already (zero_v false)
static int residual_into(ilh_ctx* c, const double* k, const double* u, double tau, double* r, bool zero_v) {
  int st = zero_v ? launch_fill(c, r + c->nh1, 0.0, c->nh1) : ILH_OK;
  if (st) return st;
  const int slot = tstart_k(c, 1);
  if (c->jvp_variant != 1 && res2d_available(c)) {
    st = launch_res2d(c, k, u, tau, r);
  } else if (c->jvp_variant != 1 && res3d_available(c)) {
    st = launch_res3d(c, k, u, tau, r);
  } else {
    EArgs<double> a{u, u + c->nh1, u + 2 * c->nh1, k, nullptr, tau, r, nullptr};
    st = launch_elem(c, M_RESID, 64, &a, nullptr);
  }
  tstop_k(c, slot);
  return st;
}

// R(k1) into r1 and R(k2) into r2 at the same u and tau, the velocity rows of both zero on entry:
// one launch where the 2D strip kernel applies, else two
static int residual_pair(ilh_ctx* c, const double* k1, double* r1, const double* k2, double* r2, const double* u,
                         double tau) {
  if (c->jvp_variant != 1 && res2d_available(c)) {
    const int slot = tstart_k(c, 1);
    const int st = launch_res2d(c, k1, u, tau, r1, nullptr, k2, r2);
    tstop_k(c, slot);
    return st;
  }
  const int st = residual_into(c, k1, u, tau, r1, false);
  return st ? st : residual_into(c, k2, u, tau, r2, false);
}

int ilh_residual(ilh_ctx* c, const double* k, const double* u, double tau, double* r) {
  ILH_TRY
  if (!c || !k || !u || !r) return ILH_EINVAL;
  return residual_into(c, k, u, tau, r, true);
  ILH_CATCH(c)
}

// The strip residual with the smallest det J of the stage positions, one pass for both; false
// (nothing launched) where no strip residual kernel applies
static bool residual_detj_available(const ilh_ctx* c) {
  return c->jvp_variant != 1 && (res2d_available(c) || res3d_available(c));
}
// the same, with the per-work-group minima left in c->dmin_part (*ng of them) for the caller's
// final reduction; the velocity rows of r must be zero on entry
static int residual_detj_part(ilh_ctx* c, const double* k, const double* u, double tau, double* r, int* ng) {
  int st;
  const bool d2 = res2d_available(c);
  *ng = d2 ? res2d_groups(c) : res3d_groups(c);
  if (!c->dmin_part && (st = dalloc(c, &c->dmin_part, (size_t)*ng))) return st;
  const int slot = tstart_k(c, 1);
  st = d2 ? launch_res2d(c, k, u, tau, r, c->dmin_part) : launch_res3d(c, k, u, tau, r, c->dmin_part);
  tstop_k(c, slot);
  return st;
}


int ilh_linearize(ilh_ctx* c, const double* k, const double* u, double tau) {
  ILH_TRY
  if (!c || !k || !u) return ILH_EINVAL;
  int st;
  if ((st = launch_waxpy(c, c->w64, u, tau, k, c->nblock))) return st;
  c->lin_tau = tau;
  c->qd_ok[0] = c->qd_ok[1] = false;
  if (c->jvp_variant == 0 && (lin2d_available(c) || lin3d_available(c))) return ILH_OK;  // they read w64 only
  return launch_cast_d2f(c, c->w32, c->w64, c->nblock);
  ILH_CATCH(c)
}

// The linearised action on an output whose velocity rows the caller has zeroed
static int jvp_lin_zeroed(ilh_ctx* c, int prec, const void* dk, void* jdk) {
  int st;
  if (c->jvp_variant == 0 && (lin2d_available(c) || lin3d_available(c))) {
    const bool d3 = c->dim == 3;
    const int p = prec == 64 ? 1 : 0;
    if (!c->qd_ok[p]) {
      const int ls = tstart_k(c, 5);
      st = d3 ? launch_lin3d(c, prec) : launch_lin2d(c, prec);
      tstop_k(c, ls);
      if (st) return st;
      c->qd_ok[p] = true;
    }
    const int slot = tstart_k(c, 0);
    st = d3 ? launch_jvp3d_q(c, prec, dk, jdk) : launch_jvp2d_q(c, prec, dk, jdk);
    tstop_k(c, slot);
    return st;
  }
  if (prec == 64) {
    EArgs<double> a{c->w64, c->w64 + c->nh1, c->w64 + 2 * c->nh1, nullptr, (const double*)dk, c->lin_tau,
                    (double*)jdk, nullptr};
    const int slot = tstart_k(c, 0);
    st = c->jvp_variant == 1 ? ILH_EINVAL : launch_jvp2d(c, 64, &a, nullptr);
    if (st == ILH_EINVAL) st = launch_elem(c, M_JVP, 64, &a, nullptr);
    tstop_k(c, slot);
    return st;
  }
  EArgs<float> a{c->w64, c->w32 + c->nh1, c->w32 + 2 * c->nh1, nullptr, (const float*)dk, c->lin_tau,
                 (float*)jdk, nullptr};
  const int slot = tstart_k(c, 0);
  st = c->jvp_variant == 1 ? ILH_EINVAL : launch_jvp2d(c, 32, nullptr, &a);
  if (st == ILH_EINVAL) st = launch_elem(c, M_JVP, 32, nullptr, &a);
  tstop_k(c, slot);
  return st;
}

int ilh_jvp_lin(ilh_ctx* c, int prec, const void* dk, void* jdk) {
  ILH_TRY
  if (!c || !dk || !jdk) return ILH_EINVAL;
  if (prec != 32 && prec != 64) return fail(c, ILH_EINVAL, "prec must be 32 or 64");
  int st;
  if (prec == 64) {
    if ((st = launch_fill(c, (double*)jdk + c->nh1, 0.0, c->nh1))) return st;
  } else {
    if ((st = launch_fillf(c, (float*)jdk + c->nh1, 0.0f, c->nh1))) return st;
  }
  return jvp_lin_zeroed(c, prec, dk, jdk);
  ILH_CATCH(c)
}

int ilh_jvp(ilh_ctx* c, int prec, const double* k, const double* u, double tau, const void* dk, void* jdk) {
  ILH_TRY
  int st = ilh_linearize(c, k, u, tau);
  if (st) return st;
  return ilh_jvp_lin(c, prec, dk, jdk);
  ILH_CATCH(c)
}

int ilh_jvp_noalloc(ilh_ctx* c, int prec, const double* k, const double* u, double tau, const void* dk,
                    void* jdk) {
  ILH_TRY
  if (!c || !k || !u || !dk || !jdk) return ILH_EINVAL;
  if (prec != 32 && prec != 64) return fail(c, ILH_EINVAL, "prec must be 32 or 64");
  if (!c->scratch) return fail(c, ILH_EINVAL, "no static scratch on this context's device");
  // scratch layout: w = u + tau k (FP64) | FP32 shadow of w (recomputing kernels) or the tangent
  // coefficients of precision prec (linearised kernels), each part 256-byte aligned
  auto al = [](int64_t b) { return (b + 255) / 256 * 256; };
  const bool lin = c->jvp_variant == 0 && (lin2d_available(c) || lin3d_available(c));
  const int64_t off1 = al(c->nblock * 8);
  const int64_t part2 = lin ? (c->dim == 3 ? lin3d_coef_bytes(c, prec) : lin2d_coef_bytes(c, prec)) : c->nblock * 4;
  const int64_t need = off1 + al(part2);
  if (need > (int64_t)ILH_NOALLOC_SCRATCH_BYTES)
    return fail(c, ILH_EINVAL, "ilh_jvp_noalloc: this mesh needs " + std::to_string(need) +
                                   " bytes of scratch, the static array holds " +
                                   std::to_string((long long)ILH_NOALLOC_SCRATCH_BYTES));
  unsigned char* base = (unsigned char*)c->scratch;
  const int p = prec == 64 ? 1 : 0;
  // run ilh_jvp on the scratch buffers in place of the context's own, then restore the context's
  // linearisation point (its buffers are not touched; enqueued kernels keep the addresses they got)
  double* w64 = c->w64;
  float* w32 = c->w32;
  void* qd = c->qd[p];
  const bool ok0 = c->qd_ok[0], ok1 = c->qd_ok[1];
  const double tau0 = c->lin_tau;
  c->w64 = (double*)base;
  if (lin)
    c->qd[p] = base + off1;
  else
    c->w32 = (float*)(base + off1);
  const int st = ilh_jvp(c, prec, k, u, tau, dk, jdk);
  c->w64 = w64;
  c->w32 = w32;
  c->qd[p] = qd;
  c->qd_ok[0] = ok0;
  c->qd_ok[1] = ok1;
  c->lin_tau = tau0;
  return st;
  ILH_CATCH(c)
}

int ilh_vjp_lin(ilh_ctx* c, int prec, const void* y, void* jty) {
  ILH_TRY
  if (!c || !y || !jty) return ILH_EINVAL;
  if (prec != 32 && prec != 64) return fail(c, ILH_EINVAL, "prec must be 32 or 64");
  const bool d3 = c->dim == 3;
  if (!(d3 ? lin3d_available(c) : lin2d_available(c)))
    return fail(c, ILH_EINVAL, "the transpose action is built for 2D meshes with k = 2, 3 and 3D with k = 2");
  int st;
  if (prec == 64) {
    if ((st = launch_fill(c, (double*)jty, 0.0, 2 * c->nh1))) return st;
  } else {
    if ((st = launch_fillf(c, (float*)jty, 0.0f, 2 * c->nh1))) return st;
  }
  const int p = prec == 64 ? 1 : 0;
  if (!c->qd_ok[p]) {
    const int ls = tstart_k(c, 5);
    st = d3 ? launch_lin3d(c, prec) : launch_lin2d(c, prec);
    tstop_k(c, ls);
    if (st) return st;
    c->qd_ok[p] = true;
  }
  const int slot = tstart_k(c, 6);
  st = d3 ? launch_vjp3d_q(c, prec, y, jty) : launch_vjp2d_q(c, prec, y, jty);
  tstop_k(c, slot);
  return st;
  ILH_CATCH(c)
}

int ilh_vjp(ilh_ctx* c, int prec, const double* k, const double* u, double tau, const void* y, void* jty) {
  ILH_TRY
  int st = ilh_linearize(c, k, u, tau);
  if (st) return st;
  return ilh_vjp_lin(c, prec, y, jty);
  ILH_CATCH(c)
}

int ilh_mass_v_apply(ilh_ctx* c, const double* x, double* y) {
  ILH_TRY
  if (!c || !x || !y) return ILH_EINVAL;
  return launch_mass_v(c, x, y, 0);
  ILH_CATCH(c)
}

int ilh_mass_v_solve(ilh_ctx* c, const double* b, double* x, double rtol, int maxit, int* iters, double* relres) {
  ILH_TRY
  if (!c || !b || !x || maxit < 0) return ILH_EINVAL;
  int it = 0;
  double rel = 0;
  int st = pcg_mass_v(c, b, x, rtol, maxit, 1, &it, &rel);
  if (st) return st;
  if (iters) *iters = it;
  if (relres) *relres = rel;
  if (rel > rtol) return fail(c, ILH_ENOCONV, "PCG did not reach rtol");
  return ILH_OK;
  ILH_CATCH(c)
}

int ilh_mass_e_inv(ilh_ctx* c, const double* b, double* x) {
  ILH_TRY
  if (!c || !b || !x) return ILH_EINVAL;
  return launch_mass_e_inv(c, b, x);
  ILH_CATCH(c)
}

int ilh_energy(ilh_ctx* c, const double* u, double* ke, double* ie) {
  ILH_TRY
  if (!c || !u || !ke || !ie) return ILH_EINVAL;
  return energy_host(c, u, ke, ie);
  ILH_CATCH(c)
}

int ilh_min_detj(ilh_ctx* c, const double* w, double* m) {
  ILH_TRY
  if (!c || !w || !m) return ILH_EINVAL;
  return min_detj_host(c, w, m);
  ILH_CATCH(c)
}

int ilh_dt_estimate(ilh_ctx* c, const double* u, double cfl, double* dt) {
  ILH_TRY
  if (!c || !u || !dt || !(cfl > 0)) return ILH_EINVAL;
  return dt_estimate_host(c, u, cfl, dt);
  ILH_CATCH(c)
}

int ilh_l1_velocity_error(ilh_ctx* c, const double* u, double* err) {
  ILH_TRY
  if (!c || !u || !err) return ILH_EINVAL;
  if (c->s.problem != ILH_PROBLEM_TG2D && c->s.problem != ILH_PROBLEM_TG3D)
    return fail(c, ILH_EINVAL, "L1 error needs an analytic Taylor-Green velocity");
  return l1_error_host(c, u, err);
  ILH_CATCH(c)
}

int ilh_rate(ilh_ctx* c, const double* u, double* f) {
  ILH_TRY
  if (!c || !u || !f) return ILH_EINVAL;
  int st;
  const int64_t nh1 = c->nh1;
  // the residual at k = 0, tau = 0 holds F 1 (free rows) and -F^T v - b
  if ((st = ensure_solver_ws(c, 1))) return st;
  double* zero = c->kry;
  double* r = c->kry + c->nblock;
  if ((st = launch_fill(c, zero, 0.0, c->nblock))) return st;
  if ((st = ilh_residual(c, zero, u, 0.0, r))) return st;
  // f_e = M_E^-1 (F^T v + b) = -M_E^-1 R_e(0)
  if ((st = launch_axpby(c, r + 2 * nh1, 0.0, r, -1.0, c->nl2))) return st;
  if ((st = launch_mass_e_inv(c, r + 2 * nh1, f + 2 * nh1))) return st;
  // f_v = -Mhat^-1 P_u F 1 ; R_v(0) = F 1 on free rows and 0 on constrained rows
  if ((st = launch_axpby(c, r + nh1, 0.0, r, -1.0, nh1))) return st;
  int it;
  double rel;
  if ((st = pcg_mass_v(c, r + nh1, f + nh1, 1e-14, 500, 10, &it, &rel))) return st;
  ILH_HIP(c, hipMemcpyAsync(f, u + nh1, nh1 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  return ILH_OK;
  ILH_CATCH(c)
}

// a = -Mhat^-1 P_u F(w) 1 (the velocity rate, wall rows zero), using f1 [nh1] as scratch
static int velocity_rate(ilh_ctx* c, const double* w, double* f1, double* ftv, double* a) {
  int st;
  if ((st = ilh_force(c, w, f1, ftv))) return st;
  if ((st = launch_scale_free(c, f1, -1.0, f1))) return st;
  int it;
  double rel;
  return pcg_mass_v(c, f1, a, 1e-14, 500, 10, &it, &rel);
}

// de = M_E^-1 (F(w)^T vt + b(x_w)) using r [nl2] as scratch
static int energy_rate(ilh_ctx* c, const double* w, const double* vt, double* r, double* de) {
  EArgs<double> a{w, w + c->nh1, w + 2 * c->nh1, nullptr, vt, 0.0, nullptr, r};
  int st = launch_elem(c, M_ERATE, 64, &a, nullptr);
  if (st) return st;
  return launch_mass_e_inv(c, r, de);
}

int ilh_rk2avg_step(ilh_ctx* c, double* u, double dt) {
  ILH_TRY
  if (!c || !u || !(dt > 0)) return ILH_EINVAL;
  if (c->dim != 2) return fail(c, ILH_EINVAL, "the explicit RK2-average step is built for 2D");
  int st;
  const int64_t nh1 = c->nh1, nl2 = c->nl2, nb = c->nblock;
  if (!c->rkw && (st = dalloc(c, &c->rkw, 3 * nb))) return st;
  double* uh = c->rkw;           // half-step state [block]
  double* a = c->rkw + nb;       // velocity rate [nh1]
  double* f1 = a + nh1;          // F 1 scratch [nh1]
  double* vb = f1 + nh1;         // averaged velocity [nh1]
  double* r = vb + nh1;          // energy scratch [nl2]
  double* de = r + nl2;          // energy rate [nl2]
  double *x = u, *v = u + nh1, *e = u + 2 * nh1;
  double *xh = uh, *vh = uh + nh1, *eh = uh + 2 * nh1;
  // half step: v_h = v + dt/2 a(u), e_h = e + dt/2 M_E^-1 (F(u)^T v_h + b(x)), x_h = x + dt/2 v_h
  if ((st = velocity_rate(c, u, f1, r, a))) return st;
  if ((st = launch_waxpy(c, vh, v, 0.5 * dt, a, nh1))) return st;
  if ((st = energy_rate(c, u, vh, r, de))) return st;
  if ((st = launch_waxpy(c, eh, e, 0.5 * dt, de, nl2))) return st;
  if ((st = launch_waxpy(c, xh, x, 0.5 * dt, vh, nh1))) return st;
  // full step: v+ = v + dt a(u_h), vbar = (v + v+)/2, e+ = e + dt M_E^-1 (F(u_h)^T vbar + b(x_h)),
  // x+ = x + dt vbar
  if ((st = velocity_rate(c, uh, f1, r, a))) return st;
  if ((st = launch_waxpy(c, vb, v, 0.5 * dt, a, nh1))) return st;
  if ((st = energy_rate(c, uh, vb, r, de))) return st;
  if ((st = launch_axpby(c, e, dt, de, 1.0, nl2))) return st;
  if ((st = launch_axpby(c, x, dt, vb, 1.0, nh1))) return st;
  return launch_axpby(c, v, dt, a, 1.0, nh1);
  ILH_CATCH(c)
}

int ilh_plain_guess(ilh_ctx* c, const double* u, const double* k1, const double* k2, int nhist, double tau,
                    double* out) {
  ILH_TRY
  if (!c || !u || !out) return ILH_EINVAL;
  int st;
  if (nhist > 0) {
    if (!k1 || (nhist >= 2 && !k2)) return fail(c, ILH_EINVAL, "missing history vector");
    return launch_extrap(c, out, u, k1, k2, nhist >= 2 ? 2 : 1, tau);  // one pass, position block included
  }
  if ((st = ilh_rate(c, u, out))) return st;
  if (tau > 0.0) {
    // out_x = u_v + tau out_v
    ILH_HIP(c, hipMemcpyAsync(out, u + c->nh1, c->nh1 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    if ((st = launch_axpby(c, out, tau, out + c->nh1, 1.0, c->nh1))) return st;
  }
  return ILH_OK;
  ILH_CATCH(c)
}

}  // extern "C"

// ---------------------------------------------------------------- Newton-Krylov
namespace ilh {

static double nrm2(ilh_ctx* c, const double* x, int64_t n, int* st) {
  double v = 0;
  *st = dot_host(c, x, x, n, &v);
  return std::sqrt(v);
}

// two adjacent device scalars (in the reduction buffer's scalar area) and their host copies:
// results enqueued one after the other are read with a single synchronisation
static double* dev_pair(ilh_ctx* c) { return c->red + (int64_t)c->red_blocks * 65 + 8; }
static int read_pair(ilh_ctx* c, double* a, double* b) {
  ILH_HIP(c, hipMemcpyAsync(c->red_host + 4, dev_pair(c), 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  ILH_HIP(c, hipStreamSynchronize(c->stream));
  *a = c->red_host[4];
  *b = c->red_host[5];
  return ILH_OK;
}

// y = x / beta; beta is also stored to *beta_out, the scale of the stored vector y, 1, to *s0
// and the FGMRES cycle's tag to *tag_out
// y = x / beta with the cycle's Arnoldi scalars: h[240] = beta, h[252] = the residual target,
// h[255] = the cycle's tag, s_0 = h[256] = 1, and the stage factor h[250] = tau that the step
// kernels read
// (beta2 nullable: beta = sqrt(*beta2), the norm of a restart residual formed on the device; a
// zero norm gives a zero basis vector, whose cycle then ends at its first column)
template <typename TV>
__global__ void k_scale_copy(TV* y, const double* x, double beta_h, int64_t n, double* h, double target,
                             double tag, double tau, const double* beta2) {
  const double beta = beta2 ? sqrt(*beta2) : beta_h;
  const double f = beta > 0.0 ? 1.0 / beta : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    h[250] = tau;
    h[240] = beta;
    h[252] = target;
    h[255] = tag;
    h[256] = 1.0;
    h[HDEV_LGSE] = 0.0;
  }
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (TV)(x[i] * f);
}

// Exact diagonal blocks of the Jacobian at the current linearisation point, read off by FP32
// Jacobian actions on coloured unit directions: the diagonal of the velocity block (mode 2:
// directions (0, e, 0)) or of the velocity block with the position block eliminated (mode 1:
// directions (tau e, e, 0)), and every element's energy block.
static int build_probe_prec(ilh_ctx* c, int mode) {
  int st;
  if (!c->pdv && (st = dalloc(c, &c->pdv, (size_t)c->nh1))) return st;
  if (!c->peinv && (st = dalloc(c, &c->peinv, (size_t)c->Ne * c->Nl * c->Nl))) return st;
  float* d = c->kry32;
  float* y = c->kry32 + c->nblock;
  const int M = c->k + 1;
  const int ncol = c->dim == 3 ? M * M * M : M * M;
  // each direction kernel first takes the previous probe's entries from the action output y,
  // then zeroes y's velocity rows for the next action; the last probe is read off on its own
  int pcomp = -1, pcol = -1;  // the previous velocity probe
  for (int comp = 0; comp < c->dim; ++comp)
    for (int col = 0; col < ncol; ++col) {
      if ((st = launch_probe_v_dir(c, d, comp, col, mode == 1 ? c->lin_tau : 0.0, y, pcomp, pcol,
                                   pcomp >= 0 ? c->pdv : nullptr)))
        return st;
      if ((st = jvp_lin_zeroed(c, 32, d, y))) return st;
      pcomp = comp;
      pcol = col;
    }
  for (int j = 0; j < c->Nl; ++j) {
    if ((st = launch_probe_e_dir(c, d, j, y, pcomp, pcol, j == 0 ? c->pdv : nullptr, j - 1,
                                 j > 0 ? c->peinv : nullptr)))
      return st;
    if ((st = jvp_lin_zeroed(c, 32, d, y))) return st;
  }
  if ((st = launch_probe_e_take(c, y, c->Nl - 1, c->peinv))) return st;
  return launch_invert_blocks(c, c->peinv);
}

// The FGMRES basis V, Z is stored in TV: FP64, or FP32 when the Jacobian actions inside FGMRES
// run in FP32 (the orthogonalisation, Hessenberg matrix, rotations and the solution update stay
// FP64; the basis vectors carry the 1e-7 relative rounding the FP32 actions already have).
template <typename TV>
struct Solver {
  static constexpr bool F32 = sizeof(TV) == 4;
  TV* basis() const {
    if constexpr (F32)
      return c->kryf;
    else
      return c->kry;
  }
  ilh_ctx* c;
  const ilh_newton_opts* o;
  double tau;
  int jvp_calls = 0;

  // next_out (nullable): the FP64 output of the Jacobian action that will read z; when the
  // FP32 action can write it directly, the preconditioner kernel also zeroes its velocity rows.
  // rs (nullable, device): the input vector is *rs times r.
  // job (nullable): the Givens update of the Arnoldi step that produced r, run by an extra block
  // of the preconditioner launch (or, for the PCG form, as its own launch first); *rs is the
  // scale that update stores, which the other blocks of the launch form from the same partial
  // sums, so the preconditioned vector is that of the normalised basis vector.
  int precond(const TV* r, TV* z, TV* next_out = nullptr, const double* rs = nullptr,
              const GivensJob* job = nullptr) {
    int st;
    const int slot = tstart(c, 4);
    st = precond_body(r, z, next_out, rs, job);
    tstop(c, slot);
    return st;
  }

  const TV* z32_of = nullptr;  // FP64 basis: the vector whose FP32 copy is in kry32 (written by precond)
  const TV* zeroed_v = nullptr;  // the basis vector whose velocity rows precond zeroed
  bool took_direct = false;  // an action took the direct FP32 path (tau read from the device)

  // FP32 linearised 2D actions write the FP64 Krylov vector directly
  bool direct64() const { return o->jvp_prec == 32 && c->jvp_variant == 0 && lin2d_available(c); }

  int precond_body(const TV* r, TV* z, TV* next_out, const double* rs, const GivensJob* job) {
    const int64_t nh1 = c->nh1;
    int st;
    z32_of = nullptr;
    zeroed_v = nullptr;
    TV* zv = (next_out && direct64()) ? next_out + nh1 : nullptr;
    const double* tdev = c->hdev + 250;  // tau on the device (set at the start of each solve)
    if (o->prec_probe) {
      float* z32 = (o->jvp_prec == 32 && !F32) ? c->kry32 : nullptr;
      if ((st = launch_precond_probe(c, r, z, z32, tau, o->prec_coupled, zv, tdev, rs, job))) return st;
      if (z32) z32_of = z;
      if (zv) zeroed_v = next_out;
      return ILH_OK;
    }
    if (o->pcg_iters <= 0) {
      float* z32 = (o->jvp_prec == 32 && !F32) ? c->kry32 : nullptr;
      if ((st = launch_precond(c, r, z, z32, tau, o->prec_coupled, zv, tdev, rs, job))) return st;
      if (z32) z32_of = z;
      if (zv) zeroed_v = next_out;
      return ILH_OK;
    }
    if constexpr (F32) {
      return fail(c, ILH_EINVAL, "the PCG velocity block needs the FP64 basis");
    } else {
    if (job && (st = launch_sum_givens(c, *job))) return st;
    ILH_HIP(c, hipMemcpyAsync(z, r, nh1 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    if (o->pcg_iters > 0) {
      if ((st = pcg_mass_v(c, r + nh1, z + nh1, 0.0, o->pcg_iters, 0, nullptr, nullptr))) return st;
    } else {
      if ((st = launch_jacobi(c, r + nh1, z + nh1))) return st;
    }
    if ((st = launch_mass_e_inv(c, r + 2 * nh1, z + 2 * nh1))) return st;
    if (o->prec_coupled)
      if ((st = launch_axpby(c, z, tau, z + nh1, 1.0, nh1))) return st;
    if (rs && (st = launch_scale_dev(c, z, rs, c->nblock))) return st;  // the operator is linear
    return ILH_OK;
    }
  }

  // skip (nullable, device): used by the FP32 action written straight into the Krylov basis,
  // which returns at once when *skip is nonzero
  bool skippable = false;  // the last action was one that a set flag turns into no work
  int skip_slot = -1;      // its timer slot and generation
  int64_t skip_gen = -1;
  // the last action did no work (its step's flag was set): neither counted nor timed
  void drop_skipped() {
    if (!skippable) return;
    --jvp_calls;
    tdrop(c, skip_slot, skip_gen);
    skippable = false;
  }
  // the action on a basis vector (FP32 basis: an FP32 action reading Z_j and writing V_{j+1} itself)
  int apply_basis(const TV* x, TV* y, const double* skip = nullptr) {
    if constexpr (!F32) {
      return apply(x, y, skip);
    } else {
      int st;
      ++jvp_calls;
      skippable = false;
      const bool zeroed = (y == zeroed_v);
      zeroed_v = nullptr;
      if (zeroed && direct64()) {
        if (!c->qd_ok[0]) {
          const int ls = tstart_k(c, 5);
          st = launch_lin2d(c, 32);
          tstop_k(c, ls);
          if (st) return st;
          c->qd_ok[0] = true;
        }
        took_direct = true;
        const int slot = tstart_k(c, 0);
        st = launch_jvp2d_q_f32to32(c, x, y, c->hdev + 250, skip);
        tstop_k(c, slot);
        skippable = skip != nullptr;
        skip_slot = slot;
        skip_gen = c->tgen;
        return st;
      }
      return ilh_jvp_lin(c, 32, x, y);
    }
  }

  // the action on FP64 vectors (restart residuals; with an FP64 basis, every action)
  int apply(const double* x, double* y, const double* skip = nullptr) {
    int st;
    ++jvp_calls;
    skippable = false;
    if (o->jvp_prec == 32) {
      float* x32 = c->kry32;
      float* y32 = c->kry32 + c->nblock;
      // the preconditioner leaves the FP32 copy of its output in x32; it is used once
      const bool have32 = !F32 && ((const void*)x == (const void*)z32_of);
      const bool zeroed = !F32 && ((const void*)y == (const void*)zeroed_v);
      z32_of = nullptr;
      zeroed_v = nullptr;
      if (have32 && zeroed && direct64()) {
        if (!c->qd_ok[0]) {
          const int ls = tstart_k(c, 5);
          st = launch_lin2d(c, 32);
          tstop_k(c, ls);
          if (st) return st;
          c->qd_ok[0] = true;
        }
        took_direct = true;
        const int slot = tstart_k(c, 0);
        st = launch_jvp2d_q_f32to64(c, x32, y, c->hdev + 250, skip);
        tstop_k(c, slot);
        skippable = skip != nullptr;
        skip_slot = slot;
        skip_gen = c->tgen;
        return st;
      }
      if (direct64()) {
        // (restart residuals) the FP32 copy of x and the zero velocity rows of y in one launch,
        // then the action writes the FP64 y itself at the host's tau
        if (!have32 && (st = launch_cast_d2f(c, x32, x, c->nblock, y + c->nh1, c->nh1))) return st;
        if (have32 && (st = launch_fill(c, y + c->nh1, 0.0, c->nh1))) return st;
        if (!c->qd_ok[0]) {
          const int ls = tstart_k(c, 5);
          st = launch_lin2d(c, 32);
          tstop_k(c, ls);
          if (st) return st;
          c->qd_ok[0] = true;
        }
        const int slot = tstart_k(c, 0);
        st = launch_jvp2d_q_f32to64(c, x32, y, nullptr, nullptr);
        tstop_k(c, slot);
        return st;
      }
      if (!have32 && (st = launch_cast_d2f(c, x32, x, c->nblock))) return st;
      if ((st = ilh_jvp_lin(c, 32, x32, y32))) return st;
      return launch_cast_f2d(c, y, y32, c->nblock);
    }
    return ilh_jvp_lin(c, 64, x, y);
  }

  // One Arnoldi step j: w = J z_j, two Gram-Schmidt passes, then the Givens update of step j,
  // run by an extra block of the preconditioner launch for the next basis vector (z_{j+1} =
  // P v_{j+1}) or, at the last basis index, on its own; its reduction also stores the residual
  // estimate and the cycle's tag in mapped host memory (c->hest), which the host polls.  The basis
  // vectors are stored unnormalised: v_j = s_j x (stored V_j), s_j = 1 / |w| set by step j-1's
  // norm reduction; the preconditioner and the pass coefficients take the scale, so no pass
  // rescales the vector.  On entry Z_j holds z_j (from the previous step, or the cycle start).
  // Every launch of step j > 0 reads step j-1's end flag and does nothing when it is set (the
  // host enqueues step j before it reads step j-1's estimate).
  int arnoldi_step(int j, int m) {
    const int64_t n = c->nblock;
    TV* V = basis();
    TV* Z = V + (int64_t)(m + 1) * n;
    double* hd = c->hdev;
    double* s = hd + 256;
    TV* Zj = Z + (int64_t)j * n;
    TV* w = V + (int64_t)(j + 1) * n;
    const double* skip = j > 0 ? hd + HDEV_FLAG + j - 1 : nullptr;
    int st;
    if ((st = apply_basis(Zj, w, skip))) return st;
    // classical Gram-Schmidt, twice: h1 = V^T w; w -= V h1 fused with h2 = V^T w; w -= V h2
    const int slot = tstart(c, 3);
    if ((st = multidot_fused(c, V, n, j + 1, w, n, hd, s, hd + 480, skip))) return st;
    if ((st = maxpy_multidot(c, w, V, n, j + 1, hd + 480, n, s, hd + 72, hd + 560, skip))) return st;
    GivensJob job;
    if ((st = multiaxpy_nrm(c, w, V, n, j + 1, hd + 560, -1.0, n, hd, c->gmd, j, m, c->hest_dev, &job, skip)))
      return st;
    tstop(c, slot);
    if (j + 1 < m) {
      TV* next = V + (int64_t)(j + 2) * n;
      return precond(w, Z + (int64_t)(j + 1) * n, next, s + j + 1, &job);
    }
    return launch_sum_givens(c, job);
  }

  // The lagged form (Gram-Schmidt with the second pass lagged one step; scheme at the kernels):
  // the preconditioners of the mass-matrix or probed-block kind, which the update sweep applies
  bool lagged() const { return !o->cgs2 && o->pcg_iters <= 0; }

  // Arnoldi step j of the lagged form in a cycle of L columns: j < L applies J to z_j (in Z_j,
  // formed from u_j by step j - 1 or the cycle start) into slot j + 1, runs the dot sweep, the
  // final block and the update sweep (v_j, u_{j+1} and, when step j + 1 is a full step, z_{j+1});
  // j == L is the closing step (dot sweep on u_L and the final block).  The final block of step
  // j finishes column j - 1 and stores its residual estimate; when the cycle ends there it sets
  // the cycle-end flag, and every launch enqueued after it returns at once.
  int lag_step(int j, int m, int L) {
    const int64_t n = c->nblock;
    TV* V = basis();
    TV* Z = V + (int64_t)(m + 1) * n;
    double* hd = c->hdev;
    const double* skip = hd + HDEV_LGSE;
    const bool full = j < L;
    TV* w = full ? V + (int64_t)(j + 1) * n : nullptr;
    int st;
    if (full && (st = apply_basis(Z + (int64_t)j * n, w, skip))) return st;
    const int slot = tstart(c, 3);
    int np = 0;
    if ((st = lgs_dots<TV>(c, V, n, j, V + (int64_t)j * n, w, n, c->gsp, &np, skip))) return st;
    if ((st = lgs_final(c, c->gsp, np, j, m, full ? 1 : 0, hd, c->gmd, c->hest_dev, skip))) return st;
    if (full) {
      const bool next = j + 1 < L;  // step j + 1 applies J to z_{j+1}
      TV* zn = next ? Z + (int64_t)(j + 1) * n : nullptr;
      TV* out = (next && direct64()) ? V + (int64_t)(j + 2) * n : nullptr;
      float* z32 = (next && o->jvp_prec == 32 && !F32) ? c->kry32 : nullptr;
      if ((st = lgs_update<TV>(c, V, n, j, hd, zn, z32, out, o->prec_probe, o->prec_coupled, hd + 250, c->hest_dev,
                               hd + HDEV_LGSE)))
        return st;
      z32_of = z32 ? zn : nullptr;
      zeroed_v = out;
    }
    tstop(c, slot);
    return ILH_OK;
  }

  // Graph replay applies when every kernel of the step reads its varying inputs from device
  // memory (tau) and no kernel of it synchronises: linearised FP32 2D actions with the mass or
  // probed preconditioner, kernel timing off.
  bool graphable() const { return o->graphs && !c->timing && direct64() && o->pcg_iters <= 0; }

  uint64_t graph_key(int m) const {
    uint64_t k = 1469598103934665603ull;
    auto mix = [&](uint64_t v) { k = (k ^ v) * 1099511628211ull; };
    const void* ptrs[] = {basis(), c->kry32, c->hdev, c->hest_dev, c->gmd, c->red, c->qd[0], c->Mdiag, c->MEinv,
                          c->pdv, c->peinv, c->rj0};
    for (const void* q : ptrs) mix((uint64_t)(uintptr_t)q);
    mix((uint64_t)m);
    mix((uint64_t)o->prec_probe);
    mix((uint64_t)o->prec_coupled);
    mix((uint64_t)c->apply_rows);
    mix((uint64_t)c->apply_waves);
    mix((uint64_t)c->nblock);
    mix((uint64_t)lagged());
    return k;
  }

  // The captured step j (captured on first use for this configuration; the lagged form keeps two
  // per basis index: with and without z_{j+1}, i.e. j + 1 < L or not).
  int graph_for(int j, int m, int L, hipGraphExec_t* out) {
    const uint64_t key = graph_key(m);
    if (key != c->gkey) {
      for (hipGraphExec_t e : c->gexec)
        if (e) (void)hipGraphExecDestroy(e);
      c->gexec.assign(128, nullptr);
      c->gkey = key;
    }
    const int gi = lagged() ? 2 * j + (j + 1 < L ? 1 : 0) : j;
    if (!c->gexec[gi]) {
      // Step j - 1 (replayed, so its host-side records were not made) or the cycle start left the
      // FP32 copy of z_j and zeroed the velocity rows of V_{j+1}: the captured action must take the
      // direct FP32 path, which reads tau from the device (a captured host tau would go stale).
      const int64_t n = c->nblock;
      z32_of = basis() + (int64_t)(m + 1) * n + (int64_t)j * n;
      zeroed_v = basis() + (int64_t)(j + 1) * n;
      took_direct = false;
      if (!c->capstream) ILH_HIP(c, hipStreamCreateWithFlags(&c->capstream, hipStreamNonBlocking));
      hipStream_t saved = c->stream;
      c->stream = c->capstream;
      ILH_HIP(c, hipStreamBeginCapture(c->capstream, hipStreamCaptureModeThreadLocal));
      const int calls = jvp_calls;  // the replays count the action
      const int st = lagged() ? lag_step(j, m, L) : arnoldi_step(j, m);
      jvp_calls = calls;
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(c->capstream, &g);
      c->stream = saved;
      if (st || !took_direct) {
        if (g) (void)hipGraphDestroy(g);
        return st ? st : fail(c, ILH_EINVAL, "graph capture: the Arnoldi step did not take the device-tau action");
      }
      ILH_HIP(c, e);
      hipGraphExec_t ex = nullptr;
      const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      ILH_HIP(c, ei);
      c->gexec[gi] = ex;
    }
    *out = c->gexec[gi];
    return ILH_OK;
  }

  // FGMRES: solve J x = b, x starts at 0.  Returns total iterations in *its.  beta_b >= 0 is
  // |b| when the caller already has it (no reduction and synchronisation for it).
  // The Givens rotations, the residual estimate and the triangular solve run on the device;
  // the host enqueues Arnoldi step j before it reads step j-1's residual estimate (stored by
  // the device in mapped host memory and tagged per cycle), so the stream never drains between
  // steps.  A step enqueued after the one that ended the cycle is discarded: its launches return
  // at once on that step's end flag (and where the host alone ends the cycle, at the iteration
  // limit, it only touches V_{j+1}, Z_j, column j and g_j, g_{j+1}, none of which the solution
  // over the first j columns reads).
  int fgmres(const double* b, double* x, int* its, double beta_b = -1.0) {
    const int64_t n = c->nblock;
    const int m = std::max(1, std::min(o->restart, 64));
    TV* V = basis();
    TV* Z = V + (int64_t)(m + 1) * n;
    double* hd = c->hdev;
    double* G = c->gmd;
    int st;
    // x is written by the first cycle's x = Z y (no zero fill ahead of it); every return path
    // before that writes zeros
    bool x_set = false;
    double beta = beta_b;
    if (!(beta >= 0.0)) {
      beta = nrm2(c, b, n, &st);
      if (st) return st;
    }
    *its = 0;
    if (beta == 0.0) return launch_fill(c, x, 0.0, n);
    const double target = o->gmres_rtol * beta;
    const double* beta2_dev = nullptr;  // set once a restart forms the residual norm on the device
    const double* rhs = b;
    double* rbuf = c->nwt + 3 * n;  // tmp vector
    int total = 0;
    const bool use_graph = graphable();
    if (use_graph && !c->qd_ok[0]) {  // the linearisation stays outside the captured steps
      if ((st = launch_lin2d(c, 32))) return st;
      c->qd_ok[0] = true;
    }
    while (true) {
      // V0 = r / beta (beta, the target and the cycle's tag to the device), z_0 = P V0
      const double tag = (c->est_tag += 1.0);
      hipLaunchKernelGGL(k_scale_copy<TV>, dim3(1024), dim3(256), 0, c->stream, V, rhs, beta, n, hd, target, tag,
                         tau, beta2_dev);
      if ((st = precond(V, Z, V + n))) return st;
      int j_end = 0;
      bool stop = false;  // converged or out of iterations
      bool dev_end = false;  // the step's end flag is set on the device
      // read step jj's estimate; true when the cycle ends after it
      auto check = [&](int jj, bool& end) -> int {
        // wait for the tag the step's reduction stores after its estimate; the stream running
        // dry without it (every enqueued kernel done) is an error, so the wait always ends
        const volatile double* est = c->hest;
        const auto t0 = std::chrono::steady_clock::now();
        auto arrived = [&]() { return est[4 * jj + 1] == tag && est[4 * jj + 3] == tag; };
        for (unsigned spins = 1; !arrived(); ++spins) {
          __builtin_ia32_pause();
          if ((spins & 1023) == 0) {
            const hipError_t q = hipStreamQuery(c->stream);
            if (q != hipSuccess && q != hipErrorNotReady) ILH_HIP(c, q);
            if (q == hipSuccess && !arrived()) {
              // the stream is done: the tag must arrive (host-mapped stores can trail the
              // completion the stream reports); give it 10 ms before calling it missing
              const auto td = std::chrono::steady_clock::now();
              while (!arrived() && std::chrono::steady_clock::now() - td < std::chrono::milliseconds(10))
                __builtin_ia32_pause();
            }
            if (q == hipSuccess && !arrived()) {
              // the device's view: cycle-end flag, target, and the previous column's estimate
              double dv[HDEV_LEN];
              (void)hipMemcpy(dv, hd, sizeof(dv), hipMemcpyDeviceToHost);
              const int pj = jj > 0 ? jj - 1 : 0;
              char msg[512];
              std::snprintf(msg, sizeof msg,
                            "FGMRES: a finished step left no residual estimate (column %d, tag %.17g, found %.17g, "
                            "columns read %d, end flag %g; column %d: host %.17g %.17g tag %.17g, device %.17g "
                            "%.17g; target host %.17g device %.17g)",
                            jj, tag, (double)est[4 * jj + 1], total, dv[HDEV_LGSE], pj, (double)est[4 * pj],
                            (double)est[4 * pj + 2], (double)est[4 * pj + 1], dv[352 + 2 * pj], dv[353 + 2 * pj],
                            target, dv[252]);
              return fail(c, ILH_EHIP, msg);
            }
            if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(120))
              return fail(c, ILH_EHIP, "FGMRES: timed out waiting for a residual estimate");
          }
        }
        std::atomic_thread_fence(std::memory_order_acquire);
        const double res = est[4 * jj], hn = est[4 * jj + 2];
        if (!std::isfinite(hn) || !std::isfinite(res)) return fail(c, ILH_ENONFINITE, "non-finite Krylov vector");
        ++total;
        stop = res <= target || total >= o->gmres_maxit;
        end = stop || hn == 0.0;
        dev_end = res <= target || hn == 0.0;  // the test the device made (its end flag)
        return ILH_OK;
      };
      bool end = false;
      if (lagged()) {
        // columns this cycle may finish; step j finishes column j - 1 (its update sweep hands the
        // estimate to the host), and the closing step L finishes the last.  The host keeps one
        // step enqueued beyond the one whose estimate it waits for, so that the stream has work
        // while it reads and enqueues the next (one step is 30 us or more of kernels, four
        // launches take less); the step after the one that ends the cycle returns at once (its
        // action too when it is the direct FP32 one, which reads the flag).  Two steps ahead
        // measured slower: 0.612 vs 0.602 ms per C2 step, 8.5 vs 8.2 ms on the triple point.
        const int ahead = 1;
        const int L = std::max(1, std::min(m, o->gmres_maxit - total));
        struct Rec {
          bool sk;  // the step's action returns at once once the flag is set
          int slot;
          int64_t gen;
        };
        Rec rec[65];
        int next = 0;  // next step to enqueue
        int col = 0;   // next column to read
        while (true) {
          while (next <= L && next <= col + 1 + ahead) {
            if (use_graph && next < L) {
              hipGraphExec_t ex;
              if ((st = graph_for(next, m, L, &ex))) return st;
              ILH_HIP(c, hipGraphLaunch(ex, c->stream));
              ++jvp_calls;
              rec[next] = Rec{true, -1, -1};
            } else {
              if ((st = lag_step(next, m, L))) return st;
              rec[next] = Rec{skippable, skip_slot, skip_gen};
            }
            ++next;
          }
          if ((st = check(col, end))) return st;
          ++col;
          if (end) {
            // step col's final block ended the cycle at column col - 1; the full steps enqueued
            // after it returned at once (a host-only end, at the iteration limit, is column L - 1)
            for (int s2 = col + 1; s2 < next; ++s2)
              if (s2 < L && rec[s2].sk) {
                --jvp_calls;
                tdrop(c, rec[s2].slot, rec[s2].gen);
              }
            j_end = col;
            break;
          }
          if (col == L) {
            j_end = L;
            break;
          }
        }
      }
      for (int j = 0; j < m && !end && !lagged(); ++j) {
        // step j - 1 is the last one the iteration limit allows: step j is not enqueued
        const bool enqueue = !(j >= 1 && total + 1 >= o->gmres_maxit);
        if (!enqueue) {
        } else if (use_graph) {
          hipGraphExec_t ex;
          if ((st = graph_for(j, m, m, &ex))) return st;
          ILH_HIP(c, hipGraphLaunch(ex, c->stream));
          ++jvp_calls;
          skippable = j > 0;  // timing is off in graph replay
          skip_slot = -1;
        } else if ((st = arnoldi_step(j, m))) {
          return st;
        }
        if (j >= 1) {
          if ((st = check(j - 1, end))) return st;
          if (end) {
            j_end = j;  // step j was speculative
            if (dev_end && enqueue) drop_skipped();  // and its launches returned at once
          }
        }
      }
      if (!end && !lagged()) {  // the cycle filled the basis: read its last step
        if ((st = check(m - 1, end))) return st;
        j_end = m;
      }
      // y = H^-1 g (upper triangular), x += Z y (x = Z y in the first cycle)
      if ((st = launch_trisolve_maxpy<TV>(c, x, Z, n, G, j_end, n, x_set))) return st;
      x_set = true;
      if (stop) break;
      // restart: r = b - J x, its |r|^2 left on the device for the next cycle's scaling kernel
      // (no synchronisation; a restart residual that already meets the target, which the
      // cycle's own estimates make rare, ends the next cycle at its first column)
      if (total >= o->gmres_maxit) break;
      if ((st = apply(x, rbuf))) return st;
      if ((st = launch_axpby(c, rbuf, 1.0, b, -1.0, n))) return st;
      rhs = rbuf;
      if ((st = dot_dev(c, rbuf, rbuf, n, hd + HDEV_RBETA2))) return st;
      beta2_dev = hd + HDEV_RBETA2;
    }
    *its = total;
    return ILH_OK;
  }
};

// The linearisation at k (state u + tau k) with its tangent coefficients formed at once for the
// action precision prec (the linearised variant; else the state copies only)
static int linearize_now(ilh_ctx* c, const double* k, const double* u, double tau, int prec) {
  int st;
  if ((st = ilh_linearize(c, k, u, tau))) return st;
  if (c->jvp_variant == 0 && (lin2d_available(c) || lin3d_available(c))) {
    const int ls = tstart_k(c, 5);
    st = c->dim == 3 ? launch_lin3d(c, prec) : launch_lin2d(c, prec);
    tstop_k(c, ls);
    if (st) return st;
    c->qd_ok[prec == 64 ? 1 : 0] = true;
  }
  return ILH_OK;
}

template <typename TV>
static int stage_solve_t(ilh_ctx* c, const double* u, double tau, const double* k_guess, double* k_out,
                         const ilh_newton_opts* o, ilh_step_stats* st_out, const double** k_final) {
  const int64_t n = c->nblock;
  int st;
  ilh_step_stats stats;
  std::memset(&stats, 0, sizeof(stats));
  const int m = std::max(1, std::min(o->restart, 64));
  if ((st = ensure_solver_ws(c, m, sizeof(TV) == 4))) return st;
  if (!c->gsp && (st = dalloc(c, &c->gsp, (size_t)132 * 1024))) return st;
  if (!c->nwt && (st = dalloc(c, &c->nwt, 8 * (size_t)n))) return st;
  if (!c->hdev && (st = dalloc(c, &c->hdev, HDEV_LEN))) return st;
  if (!c->hest) {
    if (hipHostMalloc((void**)&c->hest, 272 * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess)
      return fail(c, ILH_ENOMEM, "pinned host buffer");
    std::memset(c->hest, 0, 272 * sizeof(double));  // no tag (tags start at 1)
    ILH_HIP(c, hipHostGetDevicePointer((void**)&c->hest_dev, c->hest, 0));
  }
  if (!c->gmd && (st = dalloc(c, &c->gmd, 64 * 64 + 3 * 65))) return st;
  // The iterate k is only read: every Newton update writes a trial buffer (kA or kB), which then
  // becomes the iterate; the guess and the zero vector serve as iterates without a copy.
  double* kA = c->nwt;
  double* kB = c->nwt + 6 * n;
  const double* k = nullptr;
  double* r = c->nwt + n;
  double* dk = c->nwt + 2 * n;
  double* trial = c->nwt + 4 * n;
  double* zero = c->nwt + 5 * n;
  double* rt = c->nwt + 7 * n;
  Solver<TV> S{c, o, tau};
  double* dsc = dev_pair(c);
  double* pa = c->red;                   // partial sums of the first norm of a pair
  double* pb = c->red + c->red_blocks;   // and of the second
  double* hp = c->hest_dev + 256;        // the pair, in mapped host memory
  auto read_hp = [&](double* a, double* b) -> int {
    ILH_HIP(c, hipStreamSynchronize(c->stream));
    *a = c->hest[256];
    *b = c->hest[257];
    return ILH_OK;
  };
  // The first pair (|R(0)|, |R(guess)|) is read while the stream already runs the linearisation
  // at the first iterate, which is then taken in the common case (the iterate kept and not yet
  // within the tolerance): an event marks the end of the pair's reduction, the linearisation
  // is enqueued behind it, and the host waits for the event only.  A rejected guess or a met
  // tolerance discards that linearisation (the next one overwrites it).
  const double* k_lin = nullptr;  // the iterate the stream has been linearised at
  auto read_first = [&](const double* kspec, double* a, double* b) -> int {
    int s1;
    if (o->max_newton < 1) return read_hp(a, b);
    if (!c->pev) ILH_HIP(c, hipEventCreateWithFlags(&c->pev, hipEventDisableTiming));
    ILH_HIP(c, hipEventRecord(c->pev, c->stream));
    if ((s1 = linearize_now(c, kspec, u, tau, o->jvp_prec))) return s1;
    k_lin = kspec;
    ILH_HIP(c, hipEventSynchronize(c->pev));
    *a = c->hest[256];
    *b = c->hest[257];
    return ILH_OK;
  };
  if (!c->zero_ok) {
    if ((st = launch_fill(c, zero, 0.0, n))) return st;
    c->zero_ok = true;  // nothing else writes this part of the workspace
  }
  int npa = 0, npb = 0;
  // the velocity rows of both residual buffers zeroed by one launch
  if ((st = k_guess ? launch_fill2(c, rt + c->nh1, r + c->nh1, 0.0, c->nh1) : launch_fill(c, rt + c->nh1, 0.0, c->nh1)))
    return st;
  // R(0) in rt, and R(k_guess) in r (one launch for the two where the 2D strip kernel applies)
  if ((st = k_guess ? residual_pair(c, zero, rt, k_guess, r, u, tau) : residual_into(c, zero, u, tau, rt, false)))
    return st;
  if ((st = k_guess ? dot_part2(c, rt, rt, r, r, n, pa, pb, &npa) : dot_part(c, rt, rt, n, pa, &npa))) return st;
  npb = npa;
  double r0 = 0.0, nr = 0.0;
  if (k_guess) {
    // |R(0)| and |R(k_guess)| read together
    if ((st = launch_pair_final(c, pa, npa, 0, pb, npb, 0, hp))) return st;
    if ((st = read_first(k_guess, &r0, &nr))) return st;
    r0 = std::sqrt(r0);
    nr = std::sqrt(nr);
    stats.res0 = r0;
    stats.res_init = nr;
    k = k_guess;
    if (o->guess_fallback && !(nr <= r0)) {
      // the initial iterate is worse than k = 0: start from zero instead (its residual is in rt)
      stats.guess_rejected = 1;
      k = zero;
      std::swap(r, rt);
      nr = r0;
    }
  } else {
    double unused;
    if ((st = launch_pair_final(c, pa, npa, 0, pa, npa, 0, hp))) return st;
    if ((st = read_first(zero, &r0, &unused))) return st;
    r0 = std::sqrt(r0);
    nr = r0;
    stats.res0 = r0;
    k = zero;
    std::swap(r, rt);
    stats.res_init = r0;
  }
  int status = ILH_OK;
  int it = 0;
  for (;; ++it) {
    if (it < 32) stats.res_hist[it] = r0 > 0 ? nr / r0 : nr;
    stats.res_final = nr;
    if (!std::isfinite(nr)) {
      status = ILH_ENONFINITE;
      c->err = "non-finite residual";
      break;
    }
    if (nr <= o->tol * r0) break;
    if (it >= o->max_newton) {
      status = ILH_ENOCONV;
      c->err = "Newton reached max_newton";
      break;
    }
    if (!(it == 0 && k == k_lin) && (st = ilh_linearize(c, k, u, tau))) return st;
    if (o->prec_probe && (it == 0 || !o->prec_lag) && (st = build_probe_prec(c, o->prec_probe))) return st;
    // the Newton direction is -x with J x = R(k): the solve takes r as its right-hand side and
    // the trials step by -alpha x
    int gits = 0;
    if ((st = S.fgmres(r, dk, &gits, nr))) return st;
    stats.gmres_iters += gits;
    double* kt = (k == kB) ? kA : kB;
    // backtracking: det J > 0 at every quadrature point of the stage positions, and (when
    // enabled) sufficient decrease ||R(k + a dk)|| <= (1 - 1e-4 a) ||R(k)||
    double alpha = 1.0, best = INFINITY, best_alpha = 0.0;
    bool ok = false, any_valid = false, nonfinite = false;
    for (int h = 0; h <= o->max_halvings; ++h) {
      // the trial residual is formed before det J > 0 is known (it is discarded otherwise), so
      // that one synchronisation reads both; the strip residual kernel returns det J itself
      double md, nrt2;
      if (residual_detj_available(c)) {
        // the trial iterate and the zero velocity rows of its residual in one launch
        if ((st = launch_waxpy(c, kt, k, -alpha, dk, n, rt + c->nh1, c->nh1))) return st;
        int ng = 0;
        if ((st = residual_detj_part(c, kt, u, tau, rt, &ng))) return st;
        if ((st = dot_part(c, rt, rt, n, pb, &npb))) return st;
        if ((st = launch_pair_final(c, c->dmin_part, ng, 1, pb, npb, 0, hp))) return st;
        if ((st = read_hp(&md, &nrt2))) return st;
      } else {
        if ((st = launch_waxpy(c, kt, k, -alpha, dk, n))) return st;
        if ((st = launch_waxpy(c, trial, u, tau, kt, c->nh1))) return st;
        if ((st = min_detj_dev(c, trial, dsc))) return st;
        if ((st = ilh_residual(c, kt, u, tau, rt))) return st;
        if ((st = dot_dev(c, rt, rt, n, dsc + 1))) return st;
        if ((st = read_pair(c, &md, &nrt2))) return st;
      }
      // a NaN det J (non-finite stage positions) or a non-finite residual at valid positions
      // is reported as ENONFINITE if no trial succeeds, not as tangling
      if (std::isnan(md) || (md > 0.0 && !std::isfinite(nrt2))) nonfinite = true;
      if (md > 0.0 && std::isfinite(nrt2)) {
        any_valid = true;
        const double nrt = std::sqrt(nrt2);
        if (!o->ls_residual || nrt <= (1.0 - 1e-4 * alpha) * nr) {
          ok = true;
          nr = nrt;
          break;
        }
        if (nrt < best) {
          best = nrt;
          best_alpha = alpha;
        }
      }
      alpha *= 0.5;
      ++stats.halvings;
    }
    if (!ok && any_valid && std::isfinite(best)) {
      // no sufficient decrease within the halvings: take the best valid trial
      alpha = best_alpha;
      if ((st = launch_waxpy(c, kt, k, -alpha, dk, n))) return st;
      if ((st = ilh_residual(c, kt, u, tau, rt))) return st;
      nr = nrm2(c, rt, n, &st);
      if (st) return st;
      ok = true;
    }
    if (!ok) {
      status = nonfinite ? ILH_ENONFINITE : ILH_ETANGLED;
      c->err = nonfinite ? "line search: non-finite stage positions or residual"
                         : "line search could not keep det J > 0";
      break;
    }
    k = kt;
    std::swap(r, rt);
  }
  stats.newton_iters = it;
  stats.newton_max = it;
  stats.jvp_calls = S.jvp_calls;
  stats.status = status;
  if (k_final && status == ILH_OK) {
    // the caller finishes the step from the final iterate (its buffer stays valid until the
    // context's next call): no copy and no synchronisation here
    *k_final = k;
    if (st_out) *st_out = stats;
    return status;
  }
  if (k_out) {
    if (k_out != k) ILH_HIP(c, hipMemcpyAsync(k_out, k, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  } else if (k != c->nwt) {
    // without k_out, the final iterate is left at the head of the Newton workspace
    ILH_HIP(c, hipMemcpyAsync(c->nwt, k, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  }
  ILH_HIP(c, hipStreamSynchronize(c->stream));
  if (st_out) *st_out = stats;
  return status;
}

// FP32 Jacobian actions orthogonalise an FP32 basis unless the options ask for FP64 (basis64) or
// the velocity block of the preconditioner runs PCG (FP64 vectors)
// k_final (nullable): on success the final iterate's address is returned there instead of being
// copied to k_out (or the workspace), and the stream is not synchronised
static int stage_solve(ilh_ctx* c, const double* u, double tau, const double* k_guess, double* k_out,
                       const ilh_newton_opts* o, ilh_step_stats* st_out, const double** k_final = nullptr) {
  const bool f32 = o->jvp_prec == 32 && !o->basis64 && o->pcg_iters <= 0;
  return f32 ? stage_solve_t<float>(c, u, tau, k_guess, k_out, o, st_out, k_final)
             : stage_solve_t<double>(c, u, tau, k_guess, k_out, o, st_out, k_final);
}

}  // namespace ilh

extern "C" {

int ilh_set_viscosity_scale(ilh_ctx* c, int mode, double width) {
  ILH_TRY
  if (!c) return ILH_EINVAL;
  if (mode != ILH_DSCALE_CONST && mode != ILH_DSCALE_FORMULA) return fail(c, ILH_EINVAL, "unknown delta_scale mode");
  if (mode == ILH_DSCALE_CONST && !(width > 0)) return fail(c, ILH_EINVAL, "dscale width must be > 0");
  c->kp.dsc_mode = mode;
  if (mode == ILH_DSCALE_CONST) c->kp.dsc_w = width;
  c->s.dscale_mode = mode;
  c->s.dscale_width = c->kp.dsc_w;
  c->qd_ok[0] = c->qd_ok[1] = false;  // the tangent coefficients depend on it
  return ILH_OK;
  ILH_CATCH(c)
}

int ilh_set_apply_rows(ilh_ctx* c, int rows) {
  ILH_TRY
  if (!c) return ILH_EINVAL;
  if (rows < 0) return fail(c, ILH_EINVAL, "apply rows must be >= 0");
  c->apply_rows = rows;
  return ILH_OK;
  ILH_CATCH(c)
}

int ilh_set_apply_waves(ilh_ctx* c, int waves) {
  ILH_TRY
  if (!c) return ILH_EINVAL;
  if (waves < 0 || waves > 2) return fail(c, ILH_EINVAL, "apply waves must be 0, 1 or 2");
  c->apply_waves = waves;
  return ILH_OK;
  ILH_CATCH(c)
}

int ilh_set_kernel_variant(ilh_ctx* c, int variant) {
  ILH_TRY
  if (!c) return ILH_EINVAL;
  if (variant < 0 || variant > 2) return fail(c, ILH_EINVAL, "kernel variant must be 0, 1 or 2");
  if (c->general && variant != 1)
    return fail(c, ILH_EINVAL, "curved initial meshes and faces without walls run on the generic kernels (variant 1)");
  if (variant != c->jvp_variant) c->qd_ok[0] = c->qd_ok[1] = false;
  // the recompute kernels read the FP32 shadow of w, which the linearised variant does not keep
  if (variant != 0 && c->w64) {
    const int st = launch_cast_d2f(c, c->w32, c->w64, c->nblock);
    if (st) return st;
  }
  c->jvp_variant = variant;
  return ILH_OK;
  ILH_CATCH(c)
}

int ilh_timing_enable(ilh_ctx* c, int on) {
  ILH_TRY
  if (!c) return ILH_EINVAL;
  int st = tflush(c);
  if (st) return st;
  if (c->tev.empty()) {
    c->tev.resize(2 * TPOOL);
    c->tcls.resize(TPOOL);
    for (auto& e : c->tev) ILH_HIP(c, hipEventCreate(&e));
  }
  c->timing = on != 0;
  for (int i = 0; i < ILH_TIMING_CLASSES; ++i) {
    c->tms[i] = 0;
    c->tcnt[i] = 0;
  }
  return ILH_OK;
  ILH_CATCH(c)
}

int ilh_timing_read(ilh_ctx* c, double* ms, int64_t* cnt) {
  ILH_TRY
  if (!c || !ms || !cnt) return ILH_EINVAL;
  int st = tflush(c);
  if (st) return st;
  for (int i = 0; i < ILH_TIMING_CLASSES; ++i) {
    ms[i] = c->tms[i];
    cnt[i] = c->tcnt[i];
  }
  return ILH_OK;
  ILH_CATCH(c)
}

int ilh_stage_solve(ilh_ctx* c, const double* ubase, double tau, const double* k_guess, double* k_out,
                    const ilh_newton_opts* o, ilh_step_stats* st) {
  ILH_TRY
  if (!c || !ubase || !o) return ILH_EINVAL;
  if (o->restart < 1 || o->gmres_maxit < 1 || o->max_newton < 0 || (o->jvp_prec != 32 && o->jvp_prec != 64))
    return fail(c, ILH_EINVAL, "bad Newton options");
  return stage_solve(c, ubase, tau, k_guess, k_out, o, st);
  ILH_CATCH(c)
}

int ilh_implicit_step(ilh_ctx* c, double* u, double dt, const double* k_guess, double* k_out,
                      const ilh_newton_opts* o, ilh_step_stats* st) {
  ILH_TRY
  if (!c || !u || !o || !(dt > 0)) return ILH_EINVAL;
  if (o->restart < 1 || o->gmres_maxit < 1 || o->max_newton < 0 || (o->jvp_prec != 32 && o->jvp_prec != 64))
    return fail(c, ILH_EINVAL, "bad Newton options");
  const double* kf = nullptr;
  int status = stage_solve(c, u, 0.5 * dt, k_guess, k_out, o, st, &kf);
  if (status != ILH_OK) return status;
  // u <- u + dt k, and the stage rate to k_out, in one pass
  int s2 = launch_step_update(c, u, dt, kf, (k_out && k_out != kf) ? k_out : nullptr, c->nblock);
  if (s2) return s2;
  ILH_HIP(c, hipStreamSynchronize(c->stream));
  return ILH_OK;
  ILH_CATCH(c)
}

// SDIRK tableaux of Sec. 4 from their published closed forms.  SD2: implicit midpoint.  SD3:
// Alexander's three-stage, L-stable, third-order method; gamma is the root in (1/6, 1/2) of
// g^3 - 3 g^2 + 3/2 g - 1/6 (Newton's method from 0.44), c2 = (1 + gamma)/2, last row
// -(6g^2 - 16g + 1)/4, (6g^2 - 20g + 5)/4, gamma.  SD4: Crouzeix's three-stage fourth-order
// method; gamma = 1/2 + cos(pi/18)/sqrt(3), rows (gamma), (1/2 - gamma, gamma),
// (2 gamma, 1 - 4 gamma, gamma), weights b1 = b3 = 1/(6 (1 - 2 gamma)^2), b2 = 1 - 2 b1.
struct SdirkTab {
  int s = 0;
  double a[3][3] = {};
  double b[3] = {};
};

static bool sdirk_tab(int scheme, SdirkTab* t) {
  *t = SdirkTab{};
  if (scheme == 2) {
    t->s = 1;
    t->a[0][0] = 0.5;
    t->b[0] = 1.0;
    return true;
  }
  if (scheme == 3) {
    double g = 0.44;
    for (int i = 0; i < 60; ++i) g -= (((g - 3.0) * g + 1.5) * g - 1.0 / 6.0) / ((3.0 * g - 6.0) * g + 1.5);
    const double b1 = -(6.0 * g * g - 16.0 * g + 1.0) / 4.0, b2 = (6.0 * g * g - 20.0 * g + 5.0) / 4.0;
    t->s = 3;
    t->a[0][0] = t->a[1][1] = t->a[2][2] = g;
    t->a[1][0] = 0.5 * (1.0 + g) - g;
    t->a[2][0] = b1;
    t->a[2][1] = b2;
    t->b[0] = b1;
    t->b[1] = b2;
    t->b[2] = g;
    return true;
  }
  if (scheme == 4) {
    const double g = 0.5 + std::cos(M_PI / 18.0) / std::sqrt(3.0);
    const double b1 = 1.0 / (6.0 * (1.0 - 2.0 * g) * (1.0 - 2.0 * g));
    t->s = 3;
    t->a[0][0] = t->a[1][1] = t->a[2][2] = g;
    t->a[1][0] = 0.5 - g;
    t->a[2][0] = 2.0 * g;
    t->a[2][1] = 1.0 - 4.0 * g;
    t->b[0] = t->b[2] = b1;
    t->b[1] = 1.0 - 2.0 * b1;
    return true;
  }
  return false;
}

int ilh_guess_infer(ilh_ctx* c, const ilh_guess_model* m, const double* u, const double* base, double tau,
                    double* k, int* used) {
  ILH_TRY
  if (!c || !m || !u || !base || !k || m->nl < 1 || m->nl > 7 || !m->W || !m->b) return ILH_EINVAL;
  auto pad = [](int w) { return (w + 31) / 32 * 32; };
  for (int l = 0; l <= m->nl; ++l)
    if (m->widths[l] < 1 || m->widths[l] > 128) return fail(c, ILH_EINVAL, "guess model widths must be 1..128");
  const int64_t ne = c->Ne;
  const int p0 = pad(m->widths[0]), pl = pad(m->widths[m->nl]);
  int64_t tot = 0;
  for (int l = 1; l <= m->nl; ++l) tot += ne * pad(m->widths[l]);
  const int64_t need = ne * p0 + 2 * tot;
  int st;
  if (c->gscr_len < need) {
    if (c->gscr) (void)hipFree(c->gscr);
    c->gscr = nullptr;
    c->gscr_len = 0;
    if ((st = dalloc(c, &c->gscr, (size_t)need))) return st;
    c->gscr_len = need;
  }
  if (!c->gres && (st = dalloc(c, &c->gres, (size_t)c->nblock))) return st;
  float* feat = c->gscr;
  float* zs = feat + ne * p0;
  float* acts = zs + tot;
  float* out = acts + tot - ne * pl;
  // one launch (features and every layer, weights in LDS) where the model fits, else the
  // features and the layer-by-layer forward
  const int ND = (c->k + 1) * (c->k + 1), NLd = c->k * c->k;
  const bool widths_ok = m->widths[0] == 2 * ND + NLd + 8 + (m->with_base ? 2 * ND + NLd : 0) &&
                         m->widths[m->nl] == 2 * ND + NLd;
  int64_t lds = 0;
  for (int l = 0; l < m->nl; ++l) lds += (int64_t)pad(m->widths[l + 1]) * (pad(m->widths[l]) + 8);
  const bool fused = widths_ok && lds <= 57344 && (reinterpret_cast<uintptr_t>(m->W) & 15) == 0;
  if (fused) {
    if ((st = ilh_guess_mlp_fused(c, m, u, base, out, pl))) return st;
  } else {
    // the features are written for all p0 columns (padding zero)
    if ((st = ilh_guess_features(c, u, m->with_base ? base : nullptr, m->vscale, m->escale, m->xscale, m->kvscale,
                                 m->kescale, m->mu, m->sd, feat, p0)))
      return st;
    if ((st = ilh_mlp_forward(c, m->nl, m->widths, m->W, m->b, feat, (int)ne, zs, acts))) return st;
  }
  if ((st = ilh_guess_assemble(c, out, pl, m->kvscale, m->kescale, m->osc, base, u, tau, k))) return st;
  // judge: residual norms of the learned and the plain iterate
  if ((st = ilh_residual(c, k, u, tau, c->gres))) return st;
  const double nl = nrm2(c, c->gres, c->nblock, &st);
  if (st) return st;
  if ((st = ilh_residual(c, base, u, tau, c->gres))) return st;
  const double nb = nrm2(c, c->gres, c->nblock, &st);
  if (st) return st;
  const bool use = std::isfinite(nl) && (nl < nb || !std::isfinite(nb));
  if (!use) ILH_HIP(c, hipMemcpyAsync(k, base, c->nblock * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  ILH_HIP(c, hipStreamSynchronize(c->stream));
  if (used) *used = use ? 1 : 0;
  return ILH_OK;
  ILH_CATCH(c)
}

int ilh_plain_guess_fallback(ilh_ctx* c, const double* u, const double* k1, const double* k2, int nhist,
                             double tau, double* out, int* which) {
  ILH_TRY
  if (!c || !u || !out) return ILH_EINVAL;
  int st;
  if ((st = ilh_plain_guess(c, u, k1, k2, nhist, tau, out))) return st;
  if (which) *which = nhist < 2 ? (nhist < 0 ? 0 : nhist) : 2;
  if (nhist < 2) return ILH_OK;
  const int64_t n = c->nblock;
  if (!c->pgb && (st = dalloc(c, &c->pgb, 2 * (size_t)n))) return st;
  double* cand = c->pgb;
  double* res = c->pgb + n;
  if ((st = ilh_plain_guess(c, u, k1, nullptr, 1, tau, cand))) return st;
  double* dsc = dev_pair(c);
  if ((st = ilh_residual(c, out, u, tau, res))) return st;
  if ((st = dot_dev(c, res, res, n, dsc))) return st;
  if ((st = ilh_residual(c, cand, u, tau, res))) return st;
  if ((st = dot_dev(c, res, res, n, dsc + 1))) return st;
  double re = 0.0, r1 = 0.0;
  if ((st = read_pair(c, &re, &r1))) return st;
  // keep the extrapolation unless its residual is not finite or larger than the previous rate's
  if (!(re <= r1) && std::isfinite(r1)) {
    ILH_HIP(c, hipMemcpyAsync(out, cand, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    if (which) *which = 1;
  }
  return ILH_OK;
  ILH_CATCH(c)
}

int ilh_probe_blocks(ilh_ctx* c, int mode, double* dv, double* einv) {
  ILH_TRY
  if (!c || (mode != 1 && mode != 2)) return ILH_EINVAL;
  int st;
  if ((st = ensure_solver_ws(c, 1))) return st;
  if ((st = build_probe_prec(c, mode))) return st;
  if (dv) ILH_HIP(c, hipMemcpyAsync(dv, c->pdv, c->nh1 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (einv)
    ILH_HIP(c, hipMemcpyAsync(einv, c->peinv, (size_t)c->Ne * c->Nl * c->Nl * sizeof(double), hipMemcpyDeviceToDevice,
                              c->stream));
  return ILH_OK;
  ILH_CATCH(c)
}

int ilh_invert_blocks(ilh_ctx* c, double* blocks) {
  ILH_TRY
  if (!c || !blocks) return ILH_EINVAL;
  return launch_invert_blocks(c, blocks);
  ILH_CATCH(c)
}

int ilh_sdirk_step(ilh_ctx* c, double* u, double dt, int scheme, const double* k_guess, double* k_out,
                   const ilh_newton_opts* o, ilh_step_stats* st) {
  ILH_TRY
  if (!c || !u || !o || !(dt > 0)) return ILH_EINVAL;
  if (o->restart < 1 || o->gmres_maxit < 1 || o->max_newton < 0 || (o->jvp_prec != 32 && o->jvp_prec != 64))
    return fail(c, ILH_EINVAL, "bad Newton options");
  SdirkTab T;
  if (!sdirk_tab(scheme, &T)) return fail(c, ILH_EINVAL, "scheme must be 2 (SD2), 3 (SD3) or 4 (SD4)");
  const int64_t n = c->nblock;
  int rc;
  if (!c->sdk && (rc = dalloc(c, &c->sdk, 5 * (size_t)n))) return rc;
  double* ub = c->sdk + 3 * n;
  ilh_step_stats acc;
  std::memset(&acc, 0, sizeof(acc));
  for (int i = 0; i < T.s; ++i) {
    double* ki = c->sdk + (int64_t)i * n;
    // stage base u + dt sum_{j<i} a_ij k_j
    ILH_HIP(c, hipMemcpyAsync(ub, u, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    for (int j = 0; j < i; ++j)
      if ((rc = launch_axpby(c, ub, dt * T.a[i][j], c->sdk + (int64_t)j * n, 1.0, n))) return rc;
    const double* guess = i ? c->sdk + (int64_t)(i - 1) * n : k_guess;
    ilh_step_stats sst;
    std::memset(&sst, 0, sizeof(sst));
    const int status = stage_solve(c, ub, T.a[i][i] * dt, guess, ki, o, &sst);
    acc.newton_iters += sst.newton_iters;
    acc.newton_max = std::max(acc.newton_max, sst.newton_iters);
    acc.gmres_iters += sst.gmres_iters;
    acc.jvp_calls += sst.jvp_calls;
    acc.halvings += sst.halvings;
    acc.guess_rejected += sst.guess_rejected;
    acc.res0 = sst.res0;
    acc.res_init = sst.res_init;
    acc.res_final = sst.res_final;
    std::memcpy(acc.res_hist, sst.res_hist, sizeof(acc.res_hist));
    acc.status = status;
    if (status != ILH_OK) {
      if (st) *st = acc;
      return status;  // u unchanged
    }
  }
  for (int i = 0; i < T.s; ++i)
    if ((rc = launch_axpby(c, u, dt * T.b[i], c->sdk + (int64_t)i * n, 1.0, n))) return rc;
  if (k_out)
    ILH_HIP(c, hipMemcpyAsync(k_out, c->sdk + (int64_t)(T.s - 1) * n, n * sizeof(double), hipMemcpyDeviceToDevice,
                              c->stream));
  ILH_HIP(c, hipStreamSynchronize(c->stream));
  if (st) *st = acc;
  return ILH_OK;
  ILH_CATCH(c)
}

int ilh_adaptive_step(ilh_ctx* c, double* u, double* dt, double dt_max, int scheme, const double* k_guess,
                      double* k_out, const ilh_newton_opts* o, ilh_step_stats* st, int max_reject, int* rejected,
                      double* dt_taken) {
  ILH_TRY
  if (!c || !u || !dt || !o || !(*dt > 0) || !(dt_max > 0) || max_reject < 0) return ILH_EINVAL;
  SdirkTab T;
  if (!sdirk_tab(scheme, &T)) return fail(c, ILH_EINVAL, "scheme must be 2 (SD2), 3 (SD3) or 4 (SD4)");
  const int64_t n = c->nblock;
  int rc;
  if (!c->sdk && (rc = dalloc(c, &c->sdk, 5 * (size_t)n))) return rc;
  double* backup = c->sdk + 4 * n;
  ILH_HIP(c, hipMemcpyAsync(backup, u, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  double h = std::min(*dt, dt_max);
  int nrej = 0, last = ILH_ENOCONV;
  for (;;) {
    ilh_step_stats s1;
    std::memset(&s1, 0, sizeof(s1));
    const int status = ilh_sdirk_step(c, u, h, scheme, k_guess, k_out, o, &s1);
    if (status == ILH_OK && s1.newton_max < 4) {
      *dt = s1.newton_max <= 1 ? 1.05 * h : h;
      if (dt_taken) *dt_taken = h;
      if (rejected) *rejected = nrej;
      if (st) *st = s1;
      return ILH_OK;
    }
    if (status != ILH_OK && status != ILH_ENOCONV && status != ILH_ETANGLED && status != ILH_ENONFINITE)
      return status;  // an error of the library or the device, not of the step
    if (status == ILH_OK)  // accepted by Newton but too many iterations: undo the update
      ILH_HIP(c, hipMemcpyAsync(u, backup, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    else
      last = status;
    if (++nrej > max_reject) {
      ILH_HIP(c, hipStreamSynchronize(c->stream));
      if (rejected) *rejected = nrej;
      if (st) *st = s1;
      return fail(c, last, "step-size control: too many rejected trials");
    }
    h *= 0.85;
  }
  ILH_CATCH(c)
}

}  // extern "C"

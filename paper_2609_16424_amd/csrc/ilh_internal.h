// Internal declarations of the ilh library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstdint>
#include <new>
#include <string>
#include <vector>

#include "ilh.h"

namespace ilh {

// Element kernel modes.
enum Mode { M_FORCE = 0, M_RESID = 1, M_FJVP = 2, M_JVP = 3, M_ERATE = 4 };

// Scalar parameters of the quadrature-point kernel and the structured mesh, passed by
// value to every element kernel.
struct KParams {
  int dim, k;
  int n[3];     // elements per direction
  int ng[3];    // H1 node grid extents (k n + 1)
  int Ne;
  int64_t N;    // H1 nodes
  const double* tab;   // 1D tables: B [Q1D][D1D], G [Q1D][D1D], BL [Q1D][L1D] (FP64)
  const float* tabf;   // the same tables rounded to FP32
  const double* mq;    // [Ne][Q] quadrature mass rho0 detJ0 w_q
  const double* detJ0; // [Ne][Q]
  const double* gamma; // [Ne]
  const double* rj0;   // [Ne] rho0 |J0| per element (affine initial mesh): m_q = rj0 w_q
  const double* j0e;   // [Ne] |J0| per element
  double eps_e;
  int visc, dsc_mode, tg_source;
  double q1, q2, h0, hc_inv, dsc_w, psi_shift;
  int walls;    // bit 2d: the face x_d = lo_d is a wall (v.n = 0), bit 2d + 1: the face x_d = hi_d
};

// Component c of the node with grid index g along direction c (of ngc) is constrained when the
// node lies on a wall face normal to c.
__host__ __device__ inline bool on_wall(int walls, int c, int64_t g, int64_t ngc) {
  return (g == 0 && ((walls >> (2 * c)) & 1)) || (g == ngc - 1 && ((walls >> (2 * c + 1)) & 1));
}

// Pointers of one element-kernel launch.  The meaning depends on the mode:
//  FORCE : x, v, e = state w;                      out = F 1 [H1], out2 = F^T v [L2]
//  RESID : x, v, e = u (FP64);  kk = k block;       out = R [block]
//  FJVP  : x, v, e = state w;   dk = direction;     out = d(F 1), out2 = d(F^T v)
//  JVP   : x (FP64), v, e = state; dk = direction;  out = J dk [block]
//  ERATE : x, v, e = state w;   dk = test velocity vt [H1];  out2 = F(w)^T vt + b(x) [L2] (2D)
template <typename T>
struct EArgs {
  const double* x;
  const T* v;
  const T* e;
  const double* kk;
  const T* dk;
  double tau;
  T* out;
  T* out2;
};

// 1D tables of the 2D element kernels, passed by value (kernel-argument memory).
template <typename T, int D1D, int Q1D>
struct Tab2 {
  T B[Q1D][D1D];
  T G[Q1D][D1D];
  T BL[Q1D][D1D - 1];
  T W[Q1D];
};

}  // namespace ilh

struct ilh_ctx {
  ilh_setup s;
  hipStream_t stream = nullptr;
  int dim = 2, k = 1, D1D = 2, Q1D = 2, L1D = 1, Nh = 4, Nl = 1, Q = 4;
  int n[3] = {1, 1, 1}, ng[3] = {1, 1, 1};
  int64_t N = 0, Ne = 0, nh1 = 0, nl2 = 0, nblock = 0, nqp = 0;
  double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
  ilh::KParams kp{};
  // device constant data
  double* tab = nullptr;
  float* tabf = nullptr;
  double* mq = nullptr;
  double* detJ0 = nullptr;
  double* gamma = nullptr;
  double* rho0 = nullptr;
  double* e0 = nullptr;
  double* MEinv = nullptr;  // affine initial mesh: [Nl][Nl] reference inverse + [Ne] scales; curved: [Ne][Nl][Nl]
  int64_t me_stride = 0;    // element stride of MEinv's blocks (0: one reference block)
  const double* me_scale = nullptr;  // per-element scale of the reference block (nullptr: none)
  double* x0 = nullptr;     // [nh1] initial node positions of a curved initial mesh (else nullptr)
  bool general = false;     // curved initial mesh or faces without walls: generic element kernels only
  void* scratch = nullptr;  // this device's address of the library's static scratch array (ilh_jvp_noalloc)
  double* Mdiag = nullptr;  // [nh1] diag(M_V), 1 on constrained rows
  double* qw = nullptr;     // [Q] reference weights (host copy below)
  std::vector<double> h_qw, h_B, h_G, h_BL, h_gll, h_qpts, h_w1;
  double* rj0 = nullptr;    // [Ne]
  double* j0e = nullptr;    // [Ne]
  // linearisation point
  double* w64 = nullptr;    // [nblock]
  float* w32 = nullptr;     // [nblock] (x part unused)
  double lin_tau = 0.0;
  // reduction scratch
  double* red = nullptr;        // device partials
  double* dmin_part = nullptr;  // per-work-group det J minima of the strip residual
  double* red_host = nullptr;   // pinned host
  int red_blocks = 1024;
  // solver workspace
  double* ws = nullptr;         // general FP64 workspace
  int64_t ws_len = 0;
  float* ws32 = nullptr;
  int64_t ws32_len = 0;
  double* pcgbuf = nullptr;     // [4 nh1 + 16] PCG vectors and device scalars
  // Krylov / Newton workspace (allocated on first use)
  int kry_m = 0;
  double* kry = nullptr;        // V [(m+1)][nblock], Z [m][nblock]
  float* gscr = nullptr;        // learned-guess features and activations (allocated on first use)
  int64_t gscr_len = 0;
  double* gres = nullptr;       // learned-guess judge residual [nblock]
  double* pgb = nullptr;        // plain-guess fallback: candidate and residual [2][nblock] (first use)
  double* pdv = nullptr;        // probed diagonal of the velocity block [nh1]
  double* peinv = nullptr;      // inverted probed energy blocks [Ne][Nl][Nl]
  double* rkw = nullptr;        // explicit RK2-average workspace [2 nblock] (allocated on first use)
  double* sdk = nullptr;        // SDIRK stage rates and stage base [4][nblock] (allocated on first use)
  double* nwt = nullptr;        // Newton vectors: k, r, dk, tmp, zero, w [6][nblock]
  float* kry32 = nullptr;       // z32, w32 [2][nblock]
  int kryf_m = 0;
  float* kryf = nullptr;        // FP32 Krylov basis (FP32 Jacobian actions): V [(m+1)][nblock], Z [m][nblock]
  bool zero_ok = false;          // the zero block vector of the Newton workspace is filled
  double* gsp = nullptr;        // partial sums of the lagged Gram-Schmidt dot sweep [132][1024]
  double* hdev = nullptr;       // [HDEV_LEN] device scalars of the Arnoldi step
  double* hest = nullptr;       // pinned, coherent: per Arnoldi column j the records {|g_j+1|, tag} and
                                // {h_j+1,j, tag} at [4j, 4j + 4); [256, 258) a pair of norms
  double* hest_dev = nullptr;   // its device (mapped) address
  double est_tag = 0.0;         // tag of the current FGMRES cycle (host counter)
  double* gmd = nullptr;        // device Givens state of FGMRES: H [64][64], cs, sn [64], g [65]
  hipStream_t capstream = nullptr;         // stream the Arnoldi-step graphs are captured on
  std::vector<hipGraphExec_t> gexec;       // captured Arnoldi step per basis index
  uint64_t gkey = 0;                       // configuration the graphs were captured for
  int apply_rows = 0;           // element rows per apply wave of the linearised kernels (0: by mesh size)
  int apply_waves = 0;          // waves per strip of the 2D FP32 linearised apply (0: by mesh size)
  int jvp_variant = 0;          // 0 linearised (where available), 1 generic, 2 register-resident recompute
  void* qd[2] = {nullptr, nullptr};  // stored tangent coefficients, FP32 / FP64 (linearised variant)
  bool qd_ok[2] = {false, false};    // valid for the current linearisation point
  // kernel timing (HIP events)
  bool timing = false;
  std::vector<hipEvent_t> tev;  // pairs
  std::vector<int> tcls;
  int tused = 0;
  int64_t tgen = 0;  // flushes so far (a pending slot index is valid within one generation)
  hipEvent_t xev0 = nullptr, xev1 = nullptr;  // open single-kernel slot, taken by the next klaunch
  hipEvent_t pev = nullptr;  // end of the Newton solve's first norm pair (read while later work runs)
  double tms[ILH_TIMING_CLASSES] = {};
  int64_t tcnt[ILH_TIMING_CLASSES] = {};
  std::string err;
};

namespace ilh {

// error helpers
int fail(ilh_ctx* c, int code, const std::string& msg);
int hip_fail(ilh_ctx* c, hipError_t e, const char* what);

// Set the context's message without letting an exception escape (used on the ABI's
// exception paths, where the allocation inside std::string may itself fail).
inline int guard_fail(ilh_ctx* c, int code, const char* msg) noexcept {
  if (c) {
    try {
      c->err = msg;
    } catch (...) {
    }
  }
  return code;
}

// Every extern "C" body that can allocate on the host runs inside ILH_TRY ... ILH_CATCH(ctx):
// a failed host allocation becomes ILH_ENOMEM and any other C++ exception ILH_EINVAL, so no
// exception crosses the ABI.
#define ILH_TRY try {
#define ILH_CATCH(ctx)                                                         \
  }                                                                            \
  catch (const std::bad_alloc&) {                                              \
    return ilh::guard_fail(ctx, ILH_ENOMEM, "host allocation failed");         \
  }                                                                            \
  catch (...) {                                                                \
    return ilh::guard_fail(ctx, ILH_EINVAL, "unexpected C++ exception");       \
  }

#define ILH_HIP(ctx, call)                               \
  do {                                                   \
    hipError_t _e = (call);                              \
    if (_e != hipSuccess) return ilh::hip_fail(ctx, _e, #call); \
  } while (0)

// kernel timing: tstart returns a slot (or -1 when timing is off), tstop closes it
int tstart(ilh_ctx* c, int cls);
void tstop(ilh_ctx* c, int slot);
int tflush(ilh_ctx* c);
// forget pending slot `slot` of generation `gen` (a launch that did no work), if still pending
void tdrop(ilh_ctx* c, int slot, int64_t gen);
// Single-kernel slot: the events are not recorded as stream markers but attached to the next
// kernel launched through klaunch, so they bracket that dispatch alone.  tstop_k records both
// (an empty interval) if no launch took them.
int tstart_k(ilh_ctx* c, int cls);
void tstop_k(ilh_ctx* c, int slot);

// Launch on the ctx stream, handing it the open single-kernel timing events, if any.
template <typename F, typename... Args>
inline void klaunch(ilh_ctx* c, F kernel, dim3 grid, dim3 block, uint32_t shm, Args... args) {
  hipEvent_t e0 = c->xev0, e1 = c->xev1;
  c->xev0 = c->xev1 = nullptr;
  hipExtLaunchKernelGGL(kernel, grid, block, shm, c->stream, e0, e1, 0u, args...);
}

// kernel launchers (ilh_ops.hip)
int launch_elem(ilh_ctx* c, int mode, int prec, const EArgs<double>* a64, const EArgs<float>* a32);
// register-resident 2D Jacobian action (k = 2, 3); ILH_EINVAL when not specialised
int launch_jvp2d(ilh_ctx* c, int prec, const EArgs<double>* a64, const EArgs<float>* a32);
// linearised 2D Jacobian action (k = 2, 3): coefficients at (w64, lin_tau), then apply
bool lin2d_available(const ilh_ctx* c);
int launch_lin2d(ilh_ctx* c, int prec);
int launch_jvp2d_q(ilh_ctx* c, int prec, const void* dk, void* out);
int launch_vjp2d_q(ilh_ctx* c, int prec, const void* y, void* out);
int launch_vjp3d_q(ilh_ctx* c, int prec, const void* y, void* out);
int lin2d_nqd(const ilh_ctx* c);
int64_t lin2d_stride(const ilh_ctx* c);
// bytes of the stored tangent coefficients of one precision (2D / 3D linearised kernels)
int64_t lin2d_coef_bytes(const ilh_ctx* c, int prec);
int64_t lin3d_coef_bytes(const ilh_ctx* c, int prec);
// linearised 3D Jacobian action (Q2Q1, no source)
bool lin3d_available(const ilh_ctx* c);
int launch_lin3d(ilh_ctx* c, int prec);
int launch_jvp3d_q(ilh_ctx* c, int prec, const void* dk, void* out);
int launch_fill(ilh_ctx* c, double* p, double v, int64_t n);
int launch_fill2(ilh_ctx* c, double* p, double* q, double v, int64_t n);  // p = q = v, one launch
// u <- u + dt k; with kc, k copied there by the same launch
int launch_step_update(ilh_ctx* c, double* u, double dt, const double* k, double* kc, int64_t n);
int launch_fillf(ilh_ctx* c, float* p, float v, int64_t n);
int launch_axpby(ilh_ctx* c, double* y, double a, const double* x, double b, int64_t n);  // y = a x + b y
// w = u + t k; with z, its first nz (<= n) entries are zeroed by the same launch
int launch_waxpy(ilh_ctx* c, double* w, const double* u, double t, const double* k, int64_t n, double* z = nullptr,
                 int64_t nz = 0);
// y = (float) x; with z, its first nz (<= n) entries are zeroed by the same launch
int launch_cast_d2f(ilh_ctx* c, float* y, const double* x, int64_t n, double* z = nullptr, int64_t nz = 0);
int launch_cast_f2d(ilh_ctx* c, double* y, const float* x, int64_t n);
int launch_mass_v(ilh_ctx* c, const double* x, double* y, int zero_first);
int launch_mass_e_inv(ilh_ctx* c, const double* b, double* x);
int launch_jacobi(ilh_ctx* c, const double* r, double* z);   // z = r / Mdiag
int launch_scale_free(ilh_ctx* c, double* y, double a, const double* x);  // H1: y = a x, constrained rows 0
// reductions: dot products of n-length vectors, result on host (synchronizes)
int dot_host(ilh_ctx* c, const double* x, const double* y, int64_t n, double* out);
// device-side dot into d_out (no sync)
int dot_dev(ilh_ctx* c, const double* x, const double* y, int64_t n, double* d_out);
// the block partial sums of x . y into part (*np of them)
int dot_part(ilh_ctx* c, const double* x, const double* y, int64_t n, double* part, int* np);
// x . y into part and x2 . y2 into part2 (np partials each) by one launch
int dot_part2(ilh_ctx* c, const double* x, const double* y, const double* x2, const double* y2, int64_t n,
              double* part, double* part2, int* np);
// out[0], out[1] = sum (mode 0) or minimum (mode 1) of each partial set, one launch
int launch_pair_final(ilh_ctx* c, const double* pa, int na, int ma, const double* pb, int nb, int mb, double* out);
// out = k1 or 2 k1 - k2 (nhist 1 or 2), position block u_v + tau out_v when tau > 0
int launch_extrap(ilh_ctx* c, double* out, const double* u, const double* k1, const double* k2, int nhist,
                  double tau);
// Arnoldi scalars: [0, 72) and [72, 144) the two Gram-Schmidt passes, 144 the norm, [160, 224)
// the update coefficients, 240 beta, 250 tau, 252 the cycle's residual target, 255 the cycle's
// tag, [256, 321) the basis scales s_j (basis vector j = s_j x the stored vector), [352, 480)
// (|g_j+1|, h_j+1,j) per step, [480, 545) and [560, 625) the two passes' coefficients times s_j
// (the coefficients of the stored vectors), [640, 704) the step-end flags: flag j (HDEV_FLAG + j)
// is 1 when step j ended the cycle (residual estimate at most the target, or a zero norm), and
// every kernel of step j + 1 then returns at once
constexpr int HDEV_FLAG = 640;
// [704, 769): the first-pass coefficients of the previous Arnoldi step, 769 the inverse scale of
// the stored once-orthogonalised vector, 770 the cycle-end flag (0 while the cycle runs, s + 1
// once the final block of step s found the end) (Gram-Schmidt with the second pass lagged one
// step)
constexpr int HDEV_LGSP = 704;
constexpr int HDEV_LGSE = 770;
// 771: |r|^2 of a restart residual, formed on the device and read by the next cycle's scaling
constexpr int HDEV_RBETA2 = 771;
constexpr int HDEV_LEN = 776;
// y = H(0:n, 0:n)^-1 g
int launch_trisolve(ilh_ctx* c, const double* G, int m, int n, double* y);
// x += Z y with y = H(0:jn, 0:jn)^-1 g, one launch (accumulate = false: x = Z y, x need not be
// initialised; with jn = 0 it is zeroed)
template <typename TV>
int launch_trisolve_maxpy(ilh_ctx* c, double* x, const TV* Z, int64_t ldz, const double* G, int jn, int64_t n,
                          bool accumulate = true);
// Norm reduction and Givens update of Arnoldi step j: the partial sums of |w|^2 (part, np blocks),
// the Arnoldi scalars h, the rotations G (layout at givens_update), and the mapped host buffer of
// residual estimates (hest, nullable).  Runs as its own one-block kernel, or as the extra last
// block of the next preconditioner launch.
struct GivensJob {
  const double* part = nullptr;
  int np = 0;
  double* h = nullptr;
  double* G = nullptr;
  int j = 0;
  int m = 0;
  double* hest = nullptr;
  const double* skip = nullptr;  // nullable: nonzero *skip (the previous step's flag) skips the launch
};
int launch_sum_givens(ilh_ctx* c, const GivensJob& job);
// y *= *s (s on the device)
int launch_scale_dev(ilh_ctx* c, double* y, const double* s, int64_t n);
// the Krylov kernels take the basis in FP64 or FP32 (TV); every product and sum is FP64
template <typename TV>
int multiaxpy_dev(ilh_ctx* c, double* w, const TV* V, int64_t ldv, int m, const double* h, double sign, int64_t n);
// fused versions: w read once per 8 basis vectors.  d_out[j] = s_j V_j . w (s nullable: 1),
// d_outs (nullable) [j] = s_j d_out[j]
// skip (nullable, device): the launches return at once when *skip is nonzero
template <typename TV>
int multidot_fused(ilh_ctx* c, const TV* V, int64_t ldv, int m, const TV* w, int64_t n, double* d_out,
                   const double* s = nullptr, double* d_outs = nullptr, const double* skip = nullptr);
// w -= sum_j cf[j] V_j, then the products of the updated w as in multidot_fused
template <typename TV>
int maxpy_multidot(ilh_ctx* c, TV* w, const TV* V, int64_t ldv, int m, const double* cf, int64_t n,
                   const double* s, double* d_out, double* d_outs, const double* skip = nullptr);
// input *rs r (rs nullable: 1); job (nullable): run that Givens update in an extra block of the
// same launch, the other blocks then form the scale it stores (1 / |r|) from its partial sums
template <typename TV>
int launch_precond(ilh_ctx* c, const TV* r, TV* z, float* z32, double tau, int coupled,
                   TV* zero_v = nullptr, const double* tau_dev = nullptr, const double* rs = nullptr,
                   const GivensJob* job = nullptr);
// probed diagonal blocks of the Jacobian (preconditioner option prec_probe); the direction
// kernels also zero the velocity rows of yz (nullable: the output of the action they feed),
// after taking from it the previous probe's entries: the velocity diagonal of probe
// (tcomp, tcol) into tD, column tj of the energy blocks into tB (each nullable)
int launch_probe_v_dir(ilh_ctx* c, float* d, int comp, int col, double tau, float* yz = nullptr, int tcomp = -1,
                       int tcol = -1, double* tD = nullptr);
int launch_probe_e_dir(ilh_ctx* c, float* d, int j, float* yz = nullptr, int tcomp = -1, int tcol = -1,
                       double* tD = nullptr, int tj = -1, double* tB = nullptr);
int launch_probe_e_take(ilh_ctx* c, const float* y, int j, double* B);
int launch_invert_blocks(ilh_ctx* c, double* B);
template <typename TV>
int launch_precond_probe(ilh_ctx* c, const TV* r, TV* z, float* z32, double tau, int coupled,
                         TV* zero_v = nullptr, const double* tau_dev = nullptr, const double* rs = nullptr,
                         const GivensJob* job = nullptr);
// w += sign sum_j cf[j] V_j with the partial sums of |w|^2 of the result; *job receives the Givens
// update of step j that finishes it (into h[144], then from the pass coefficients h[0..j],
// h[72..72+j], and the next basis scale h[256 + j + 1] = 1 / |w|; hest (nullable, host-mapped)
// receives the step's (|g_j+1|, h_j+1,j) with the cycle's tag, records {value, tag} at [4j, 4j + 4))
template <typename TV>
int multiaxpy_nrm(ilh_ctx* c, TV* w, const TV* V, int64_t ldv, int m, const double* cf, double sign,
                  int64_t n, double* h, double* G, int j, int mm, double* hest, GivensJob* job,
                  const double* skip = nullptr);
// Gram-Schmidt with the second pass lagged one step (the scheme is described at the kernels):
// the dot sweep of step j (w nullable: the closing step) into part (np partials per sum), the
// final block, and the update sweep with the preconditioner of the next basis vector (z nullable:
// none; probe selects the probed blocks instead of the mass-matrix ones).
template <typename TV>
int lgs_dots(ilh_ctx* c, const TV* V, int64_t ldv, int j, const TV* uj, const TV* w, int64_t n, double* part,
             int* np, const double* skip);
int lgs_final(ilh_ctx* c, const double* part, int np, int j, int m, int has_w, double* h, double* G, double* hest,
              const double* skip);
template <typename TV>
int lgs_update(ilh_ctx* c, TV* V, int64_t ldv, int j, const double* h, TV* z, float* z32, TV* zero_v, int probe,
               int coupled, const double* tau_dev, double* hest, const double* end);
// (skip nullable: the kernel returns at once when *skip is nonzero)
int launch_jvp2d_q_f32to64(ilh_ctx* c, const float* dk, double* out, const double* tau_dev,
                           const double* skip = nullptr);
int launch_jvp2d_q_f32to32(ilh_ctx* c, const float* dk, float* out, const double* tau_dev,
                           const double* skip = nullptr);
// Stage residual on the strip lane maps (2D k = 2, 3; 3D k = 2 without the TG source):
// r = R(k; u, tau), the velocity rows of r zero on entry
bool res2d_available(const ilh_ctx* c);
// dmin (nullable, res2d_groups(c) entries): each work-group's smallest det J over its quadrature
// points at the stage positions u_x + tau k_x
// (k2, r2 nullable: a second residual R(k2) into r2 by the same launch, without det J)
int launch_res2d(ilh_ctx* c, const double* k, const double* u, double tau, double* r, double* dmin = nullptr,
                 const double* k2 = nullptr, double* r2 = nullptr);
int res2d_groups(const ilh_ctx* c);
// *out = min_i part[i], i < np (device)
int launch_min_final(ilh_ctx* c, const double* part, int np, double* out);
bool res3d_available(const ilh_ctx* c);
int launch_res3d(ilh_ctx* c, const double* k, const double* u, double tau, double* r, double* dmin = nullptr);
int res3d_groups(const ilh_ctx* c);
int min_detj_host(ilh_ctx* c, const double* x, double* out);
int min_detj_dev(ilh_ctx* c, const double* x, double* d_out);  // result stays on the device (no sync)
int dt_estimate_host(ilh_ctx* c, const double* u, double cfl, double* out);
int l1_error_host(ilh_ctx* c, const double* u, double* out);
int energy_host(ilh_ctx* c, const double* u, double* ke, double* ie);
int init_state_dev(ilh_ctx* c, double* u, const double* rhs_l2);
// PCG for M_V with device-resident scalars (no host synchronisation).  If check != 0 the
// residual is tested on the host every `check` iterations.
int pcg_mass_v(ilh_ctx* c, const double* b, double* x, double rtol, int maxit, int check,
               int* iters, double* relres);

// MLP and guess (ilh_mlp.hip)
int guess_features(ilh_ctx* c, const double* u, double vs, double es, double xs, float* f, int nin);
int guess_targets(ilh_ctx* c, const double* k, double kvs, double kes, float* t, int nout);
int guess_assemble(ilh_ctx* c, const float* pred, int nout, double kvs, double kes,
                   const double* base, const double* u, double tau, double* k);

}  // namespace ilh

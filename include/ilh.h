/*
 * ilh.h -- C ABI of the MI355X (gfx950) implicit high-order Lagrangian hydrodynamics library.
 *
 * The library evaluates, matrix-free, the curvilinear finite element force operator of
 * Andrej et al., "Implicit Lagrangian Hydrodynamics with High-Order Finite Elements"
 * (Sec. 2.1 eqs. v_semi, e_semi, matrices; Sec. 2.2 partial assembly, eq. decompose),
 * its Jacobian action (Sec. 3.1 eq. pa_jac_action) as a hand-written tangent, and the
 * implicit-midpoint Newton-Krylov stage solve (Sec. 3.5 eqs. nonlinear_system,
 * newton_linear).
 *
 * Conventions for every call:
 *  - Pointer arguments are DEVICE pointers owned by the caller unless marked "host".
 *    The library never frees or retains them.
 *  - Work is enqueued on the context's HIP stream (see ilh_create / ilh_set_stream).
 *    Calls that return host scalars or statistics synchronize that stream; all others
 *    are asynchronous.
 *  - Vectors are FP64 unless a precision argument says otherwise.
 *  - Layouts.  N = number of H1 nodes, Ne = elements, Nl = k^d L2 dofs per element.
 *      H1 vector  [d][N]   component-major; nodes lexicographic on the (k*n_x+1) x ...
 *                          grid, first direction fastest.
 *      L2 vector  [Ne][Nl] element-major; elements lexicographic, first direction fastest;
 *                          within an element the Bernstein basis is lexicographic.
 *      block      [x | v | e] = 2 H1 vectors followed by one L2 vector.
 *  - Boundary conditions: v.n = 0 on every wall face of the box (every face unless the set-up's
 *    free_faces lists it; Sec. 4.2 states walls for its test).  Component c of a node on a wall
 *    face normal to direction c is "constrained".
 *  - Return value: an ILH_* status code.  No C++ exception crosses the ABI.  On error
 *    ilh_last_error() describes the failure; outputs are unspecified.
 */
#ifndef ILH_H
#define ILH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ILH_OK = 0,
  ILH_EINVAL = 1,     /* bad sizes, options or pointers                          */
  ILH_EHIP = 2,       /* a HIP runtime call failed (message holds the HIP error) */
  ILH_ENOMEM = 3,     /* device allocation failed                                */
  ILH_ETANGLED = 4,   /* line search could not keep every det J > 0              */
  ILH_ENOCONV = 5,    /* Newton reached its iteration limit                      */
  ILH_ENONFINITE = 6  /* a non-finite residual norm appeared                     */
};

enum {
  ILH_PROBLEM_CUSTOM = 0,  /* rho0/gamma/e0 per element from the setup arrays        */
  ILH_PROBLEM_TG2D = 1,    /* 2D Taylor-Green vortex on [0,1]^2, gamma 5/3, rho 1   */
  ILH_PROBLEM_TG3D = 2,    /* 3D Taylor-Green vortex on [0,1]^3, gamma 5/3, rho 1   */
  ILH_PROBLEM_TRIPLE = 3,  /* three-state triple point on [0,7]x[0,3], v = 0         */
  ILH_PROBLEM_UNIFORM = 4  /* rho 1, gamma 1.4, e 2.5, v 0 (closed-form checks)      */
};

enum { ILH_DSCALE_CONST = 0, ILH_DSCALE_FORMULA = 1 };

typedef struct ilh_ctx ilh_ctx;

/* Discretisation and physics set-up (all fields host memory).
 * Sec. 2.1 (Q_k Q_{k-1} spaces), Sec. 3.4 (smoothed viscosity, energy regularisation). */
typedef struct {
  int dim;              /* 2 or 3 */
  int n[3];             /* elements per direction */
  double lo[3], hi[3];  /* box; ignored for the analytic problems, which fix their box */
  int order_v;          /* kinematic order k (1..4 in 2D, 1..3 in 3D); energy order k-1 */
  int nq1d;             /* Gauss-Legendre points per direction; 0 selects 2k (only 2k is built) */
  int problem;          /* ILH_PROBLEM_* */
  const double* rho0_elem;  /* host [Ne] or NULL: initial density per element */
  const double* gamma_elem; /* host [Ne] or NULL: ideal-gas gamma per element */
  const double* e0_elem;    /* host [Ne] or NULL: initial specific energy per element */
  int visc_on;          /* smoothed artificial viscosity mu_imp, eq. visc_mu_imp */
  double q1, q2;        /* eq. visc_mu_imp coefficients (paper default 0.5, 1) */
  double psi0;          /* switch value at zero compression, eq. visc_imp_switch (0.5) */
  int dscale_mode;      /* ILH_DSCALE_CONST: delta_scale = dscale_width;
                           ILH_DSCALE_FORMULA: delta_scale = 2 (h/h_coarse) c_s, eq. visc_imp_scale */
  double dscale_width;
  double h0;            /* initial length scale of eq. visc_imp_h; <= 0 selects (|Omega|/Ne)^(1/d)/k */
  double h_coarse;      /* <= 0 selects h0 */
  double eps_e;         /* energy regularisation width, eq. energy_regularization (1e-6) */
  int tg_source;        /* TG2D only: add the energy source that keeps the vortex steady */
  const double* x0;     /* host [dim][N] or NULL: initial node positions, an H1 vector in the layout
                           below (Sec. 2.1: the mesh positions are a field of the kinematic space, so
                           the initial mesh may be curved).  NULL: the box's affine nodes.  Given,
                           det J0 and m_q = rho0 det J0 w_q are formed at every quadrature point and
                           M_E^-1 per element; det J0 <= 0 anywhere is ILH_EINVAL.  The element-to-
                           node numbering stays that of the box grid (its logical structure) */
  int free_faces;       /* bit 2d set: no wall on the face x_d = lo_d (v.n = 0 is not imposed there);
                           bit 2d+1: likewise on x_d = hi_d.  0: walls on every face (the paper's
                           test problems).  x0 != NULL or free_faces != 0 selects the generic element
                           kernels (kernel variant 1) for every operator; the transpose action is
                           then not available */
} ilh_setup;

/* Fill *s with the defaults above for the given problem (dim, n, k set by the caller). */
void ilh_setup_defaults(ilh_setup* s, int problem);

/* Build the mesh, DOF maps, 1D basis tables, quadrature data m_q = rho0 detJ0 w_q
 * (pointwise mass conservation, Sec. 2.1, rho = rho0 / |J|) and the L2 mass inverse blocks on the device
 * (Sec. 2.2).  stream: a hipStream_t (NULL = default stream).  *out receives the context (NULL
 * on failure).  Errors: ILH_EINVAL for inconsistent set-ups (printed to stderr, as no context
 * survives), ILH_ENOMEM when a host or device allocation fails, ILH_EHIP for other HIP errors. */
int ilh_create(const ilh_setup* s, void* stream, ilh_ctx** out);
void ilh_destroy(ilh_ctx* ctx);
int ilh_set_stream(ilh_ctx* ctx, void* stream);
const char* ilh_last_error(const ilh_ctx* ctx);
const char* ilh_status_string(int status);

/* Sizes (host outputs, any may be NULL): H1 vector length d*N, L2 length Ne*Nl,
 * block length, and the number of quadrature points Ne*(2k)^d. */
int ilh_sizes(const ilh_ctx* ctx, int64_t* n_h1vec, int64_t* n_l2, int64_t* n_block,
              int64_t* n_qp);

/* Initial state u [block] (Sec. 2.1: x, v in the kinematic space, e in the thermodynamic space):
 * x0 = mesh nodes (the set-up's x0 when given), v0 = nodal interpolation of the problem's
 * velocity (zero on constrained components), e0 = rho-weighted L2 projection
 * M_E e0 = int rho0 e0(x) phi (the paper leaves the projection to its references; this is the
 * mass-weighted one).  Asynchronous; u is device memory of n_block doubles. */
int ilh_init_state(ilh_ctx* ctx, double* u);

/* Force actions at state w [block] (eq. matrices, eqs. v_semi/e_semi):
 * f1 [H1] = F(w) 1 (no boundary conditions), ftv [L2] = F(w)^T w_v. */
int ilh_force(ilh_ctx* ctx, const double* w, double* f1, double* ftv);

/* Tangent of the force actions at w [block, FP64] along dw [block]:
 * df1 = d(F 1)[dw], dftv = d(F^T v)[dw] (eq. pa_jac_action with the hand-written
 * derivative of the quadrature-point kernel).  prec = 64: dw/df1/dftv are double;
 * prec = 32: they are float and the pointwise arithmetic runs in FP32. */
int ilh_force_jvp(ilh_ctx* ctx, int prec, const double* w, const void* dw, void* df1,
                  void* dftv);

/* Stage residual R(k; tau, u) at w = u + tau k (eq. nonlinear_system), all [block]:
 *   R_x = k_x - w_v
 *   R_v = M_V k_v + F(w) 1          (constrained rows: R_v = k_v)
 *   R_e = M_E k_e - F(w)^T w_v - b(w_x)   (b: TG energy source, else 0).
 * 2D (k = 2, 3) and 3D (k = 2, no TG source): strip kernels on the lane maps of the linearised
 * kernels (unless kernel variant 1 is selected); otherwise the generic element kernel. */
int ilh_residual(ilh_ctx* ctx, const double* k, const double* u, double tau, double* r);

/* Store the linearisation point of the next ilh_jvp_lin calls: w = u + tau k in FP64 inside
 * the context (and, for the recomputing kernel variants, its FP32 shadow of velocity and
 * energy).  Stored tangent coefficients of an earlier point are invalidated; the first
 * ilh_jvp_lin of each precision recomputes them. */
int ilh_linearize(ilh_ctx* ctx, const double* k, const double* u, double tau);

/* Jacobian action J dk = dR/dk [dk] at the stored linearisation point (eq. newton_linear):
 *   (J dk)_x = dk_x - tau dk_v
 *   (J dk)_v = M_V dk_v + d(F 1)[tau dk]            (constrained rows: dk_v)
 *   (J dk)_e = M_E dk_e - d(F^T w_v)[tau dk] - db[tau dk_x].
 * prec = 64: dk, jdk are double [block]; prec = 32: float [block], FP32 arithmetic (the
 * linearised variant applies FP64-evaluated coefficients rounded to FP32; the recomputing
 * variants read positions in FP64 and make them element-relative before rounding).  The first
 * call of a precision after ilh_linearize evaluates and stores that precision's tangent
 * coefficients (linearised variant: 2D, k = 2, 3, 12 to 18 values per quadrature point;
 * 3D, k = 2, 20 or 29; allocated on first use and kept until ilh_destroy). */
int ilh_jvp_lin(ilh_ctx* ctx, int prec, const void* dk, void* jdk);

/* ilh_linearize followed by ilh_jvp_lin. */
int ilh_jvp(ilh_ctx* ctx, int prec, const double* k, const double* u, double tau,
            const void* dk, void* jdk);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): ilh_jvp with the same kernels and result, whose own
 * storage -- the point w = u + tau k (FP64) and the tangent coefficients of precision prec (the
 * FP32 shadow of w for the recomputing kernels) -- lives in a static device array of the library
 * of ILH_NOALLOC_SCRATCH_BYTES per GPU instead of buffers the context allocates on first use.  The
 * call allocates nothing (no hipMalloc or hipFree; the library makes no host allocation on success).  The array is
 * held by every GPU the library runs on until the process ends; its address on a device is taken
 * when the first context is created there.  Limit: 8 n_block bytes plus the coefficients (2D Q3Q2
 * without viscosity: 48 (FP32) or 96 (FP64) bytes per quadrature point) must fit, e.g. 2D Q3Q2 up
 * to 128x128 elements in either precision, 3D Q2Q1 up to 32^3 in FP32; larger meshes: ILH_EINVAL
 * (nothing launched).  Every call on one GPU shares that GPU's array and leaves its contents
 * there; calls that overlap on one GPU (from several contexts or streams) race.  Nothing in the
 * array needs to start at zero.  The context's own linearisation point (ilh_linearize) is left
 * as it was.  Arguments, precision and layouts as for ilh_jvp. */
#define ILH_NOALLOC_SCRATCH_BYTES (256u * 1024u * 1024u)
int ilh_jvp_noalloc(ilh_ctx* ctx, int prec, const double* k, const double* u, double tau,
                    const void* dk, void* jdk);

/* Transpose Jacobian action J^T y at the stored linearisation point (the transpose of
 * eq. pa_jac_action; Sec. 3.4 notes that transpose actions keep the gather - pointwise -
 * scatter structure):
 *   (J^T y)_x = y_x + d(F 1)^T[y~_v] + (terms of d(F^T w_v) and db along dk_x)^T[y_e]
 *   (J^T y)_v = M_V y~_v - tau y_x + d(F 1)^T[y~_v] + d(F^T w_v)^T[y_e] + y_v on constrained rows
 *   (J^T y)_e = M_E y_e + (derivatives along dk_e)^T[y~_v, y_e]
 * where y~_v is y_v with its constrained rows set to zero (those rows of R are the identity)
 * and every derivative carries the stage factor tau as in ilh_jvp_lin.  It uses the same
 * stored tangent coefficients as ilh_jvp_lin (evaluated on the first call of a precision after
 * ilh_linearize) and satisfies <y, J dk> = <J^T y, dk> to rounding.  prec = 64: y, jty double
 * [block]; prec = 32: float [block], FP32 arithmetic.  Built for 2D meshes with k = 2, 3
 * and 3D meshes with k = 2 without the TG source (otherwise ILH_EINVAL). */
int ilh_vjp_lin(ilh_ctx* ctx, int prec, const void* y, void* jty);

/* ilh_linearize followed by ilh_vjp_lin. */
int ilh_vjp(ilh_ctx* ctx, int prec, const double* k, const double* u, double tau,
            const void* y, void* jty);

/* y [H1] = M_V x [H1] (partial assembly, eq. matrices; no boundary conditions). */
int ilh_mass_v_apply(ilh_ctx* ctx, const double* x, double* y);

/* Solve Mhat x = b, Mhat = P_u M_V P_u + P_c (identity on constrained DOFs), by
 * Jacobi-preconditioned CG (Sec. 2.2) to ||r|| <= rtol ||b|| or maxit iterations.
 * iters, relres: host outputs (nullable).  Returns ILH_ENOCONV if rtol was not met. */
int ilh_mass_v_solve(ilh_ctx* ctx, const double* b, double* x, double rtol, int maxit,
                     int* iters, double* relres);

/* x [L2] = M_E^{-1} b [L2], exactly, with the per-element inverse blocks (eq. matrices: M_E is
 * block diagonal because the thermodynamic space is discontinuous).  Asynchronous. */
int ilh_mass_e_inv(ilh_ctx* ctx, const double* b, double* x);

/* Kinetic 1/2 v^T M_V v and internal 1^T M_E e energies of u (host outputs), FP64.  Their sum
 * is the total energy that eqs. v_semi and e_semi conserve exactly (F 1 paired with v equals
 * 1 paired with F^T v); it is the energy check of the implicit step.  Synchronises. */
int ilh_energy(ilh_ctx* ctx, const double* u, double* ke, double* ie);

/* Minimum of det J over all quadrature points of the positions of w [block] (host output;
 * synchronises).  The Newton line search of Sec. 3.5 keeps this positive.  A non-finite position
 * gives NaN (the minimum propagates NaN). */
int ilh_min_detj(ilh_ctx* ctx, const double* w, double* min_detj);

/* Explicit time-step estimate cfl * min_q h_min / (c_s + 2.5 mu / (rho h_min)),
 * h_min = smallest singular value of J_q / k (host output; synchronises).  Sec. 4 measures
 * implicit steps in multiples of the explicit CFL step ("FS-CFL") and refers to the explicit
 * estimate of its references; this is that estimate as read here. */
int ilh_dt_estimate(ilh_ctx* ctx, const double* u, double cfl, double* dt);

/* TG2D only: int |v_h - v_exact(x)|_2 dx over the current mesh (host output). */
int ilh_l1_velocity_error(ilh_ctx* ctx, const double* u, double* err);

/* Explicit rate f(u) = [u_v; -Mhat^-1 P_u F(u) 1; M_E^-1 (F(u)^T u_v + b)] [block]. */
int ilh_rate(ilh_ctx* ctx, const double* u, double* f);

/* Plain initial iterate of a stage solve: nhist = 0 -> out = f(u) (ilh_rate);
 * nhist = 1 -> out = k1; nhist >= 2 -> out = 2 k1 - k2 (linear extrapolation of the two
 * previous converged stage rates).  If tau > 0 the position block is then made consistent
 * with the position equation, out_x = u_v + tau out_v (R_x = 0 exactly).
 * k1, k2 [block] may be NULL when unused. */
int ilh_plain_guess(ilh_ctx* ctx, const double* u, const double* k1, const double* k2,
                    int nhist, double tau, double* out);

/* ilh_plain_guess with a fallback: for nhist >= 2, out receives the better -- the smaller finite
 * residual norm ||R(.; tau, u)|| -- of the extrapolation 2 k1 - k2 and the previous rate k1 (both
 * with out_x = u_v + tau out_v); fewer rates: as ilh_plain_guess.  *which (host, nullable): 2 the
 * extrapolation, 1 the previous rate, 0 the explicit rate.  The extrapolation of a step whose
 * predecessor moved the mesh fast can tangle the stage mesh; the previous rate is then the next
 * simplest iterate before the solver's own fallback to k = 0.  Two block vectors of workspace
 * (allocated on first use).  Synchronises (two norms). */
int ilh_plain_guess_fallback(ilh_ctx* ctx, const double* u, const double* k1, const double* k2, int nhist,
                             double tau, double* out, int* which);

/* Newton-Krylov options (host).  Converged when ||R(k)|| <= tol ||R(0; tau, u)||. */
typedef struct {
  double tol;          /* relative nonlinear tolerance (1e-10 for the benchmarks) */
  int max_newton;      /* Newton iteration cap */
  int restart;         /* FGMRES restart length (<= 64; default 15) */
  double gmres_rtol;   /* relative tolerance of each linear solve */
  int gmres_maxit;     /* FGMRES iteration cap per Newton iteration */
  int jvp_prec;        /* 32 or 64: precision of the Jacobian actions inside FGMRES */
  int max_halvings;    /* line-search halvings (det J > 0, residual decrease) */
  int pcg_iters;       /* Jacobi-PCG iterations of the velocity-mass preconditioner block
                          (0 = diagonal only) */
  int prec_coupled;    /* 1: after the mass blocks, set z_x = r_x + tau z_v */
  int guess_fallback;  /* 1: start from k = 0 when ||R(k_guess)|| > ||R(0)|| */
  int ls_residual;     /* 1: the line search also requires ||R|| to decrease (Armijo, 1e-4);
                          0: det J > 0 only */
  int prec_probe;      /* 0: block preconditioner with the masses (Jacobi of M_V, exact M_E^-1);
                          1, 2: with the exact diagonal blocks of the Jacobian, read off by
                          Jacobian actions on coloured unit directions once per Newton iterate
                          (eq. blockdiag_prec): the exact element blocks M_E - tau dF^T/de,
                          inverted per element, and Jacobi of M_V + tau dF/dv + tau^2 dF/dx
                          (1: position block eliminated) or of M_V + tau dF/dv (2);
                          d (k+1)^d + k^d extra actions per iterate */
  int prec_lag;        /* with prec_probe: 0 rebuild the blocks at every Newton iterate, 1 only
                          at the first iterate of each stage solve (lagged, Sec. 3.5) */
  int graphs;          /* 1: replay each Arnoldi step (preconditioner, FP32 linearised 2D
                          action, Gram-Schmidt with the Givens update) as a HIP graph captured
                          once per context and basis index (not while kernel timing is enabled,
                          nor with pcg_iters > 0); 0 (default): launch its kernels one by one,
                          measured faster on this stack (graph launch costs more than the
                          kernel launches it replaces) */
  int basis64;         /* with jvp_prec = 32: 0 (default) stores the FGMRES basis V, Z in FP32
                          (orthogonalisation sums, Hessenberg matrix, rotations and the update
                          of the Newton direction stay FP64; the basis then carries the 1e-7
                          rounding the FP32 actions have anyway, and the sweeps over it move
                          half the bytes), 1 keeps it in FP64.  FP64 actions and pcg_iters > 0
                          always use the FP64 basis */
  int cgs2;            /* FGMRES orthogonalisation (Sec. 3.5; both are classical Gram-Schmidt
                          twice, so the basis is orthonormal to the same order): 0 (default) takes
                          the second pass of each basis vector one Arnoldi step late, together
                          with the first pass of the next vector (one dot-product sweep and one
                          update sweep over the basis per step, the preconditioner and the
                          Givens update inside them: four launches per step; the residual
                          estimate of a column is known one step later, so a converging cycle
                          runs one more Jacobian action); 1 runs both passes in the step (three
                          sweeps, seven launches).  pcg_iters > 0 always uses 1 */
} ilh_newton_opts;

typedef struct {
  int status;            /* ILH_* */
  int newton_iters;
  int gmres_iters;       /* total over the Newton iterations */
  int jvp_calls;
  int halvings;          /* total line-search halvings */
  int guess_rejected;    /* 1 if the initial iterate was replaced by k = 0 */
  double res0;           /* ||R(0; tau, u)|| */
  double res_init;       /* ||R(k_guess)|| */
  double res_final;      /* ||R(k)|| at exit */
  double res_hist[32];   /* ||R(k^m)|| / res0, m = 0..min(newton_iters, 31) */
  int newton_max;        /* most Newton iterations of any stage of the step */
} ilh_step_stats;

void ilh_newton_defaults(ilh_newton_opts* o);

/* One implicit midpoint step (Sec. 4.1: MFEM ImplicitMidpointSolver; eq. nonlinear_system
 * with tau = dt/2): solve R(k; dt/2, u) = 0 from k_guess (NULL: zero), then u <- u + dt k.
 * u [block] in/out, k_out [block] receives k (may be NULL).  o, st: host.
 * On ETANGLED/ENOCONV/ENONFINITE u is left unchanged. */
int ilh_implicit_step(ilh_ctx* ctx, double* u, double dt, const double* k_guess,
                      double* k_out, const ilh_newton_opts* o, ilh_step_stats* st);

/* One SDIRK stage solve: R(k; tau, ubase) = 0 from k_guess (NULL: zero); k_out receives k.
 * Higher-order SDIRK steps are built from these stage solves. */
int ilh_stage_solve(ilh_ctx* ctx, const double* ubase, double tau, const double* k_guess,
                    double* k_out, const ilh_newton_opts* o, ilh_step_stats* st);

/* The diagonal blocks of eq. blockdiag_prec at the stored linearisation point (ilh_linearize),
 * as the preconditioner option prec_probe = mode (1 or 2) builds them from FP32 Jacobian
 * actions on coloured unit directions: dv [N_h1] receives the diagonal of the velocity block
 * M_V + tau dF/dv (mode 2), with tau^2 dF/dx added (mode 1: position block eliminated);
 * constrained rows 1.  einv [N_e][N_l][N_l] receives the inverses of the element blocks
 * M_E - tau dF^T/de (row-major).  Device pointers, nullable.  Other modes: ILH_EINVAL. */
int ilh_probe_blocks(ilh_ctx* ctx, int mode, double* dv, double* einv);

/* The inversion that ilh_probe_blocks and the probed preconditioner apply to the element blocks
 * of eq. blockdiag_prec, on caller data: blocks [N_e][N_l][N_l] (device, row-major, the
 * context's N_e and N_l) are replaced in place by their inverses (Gauss-Jordan elimination with
 * partial pivoting in FP64); a block with a zero pivot column is replaced by the identity.
 * Asynchronous. */
int ilh_invert_blocks(ilh_ctx* ctx, double* blocks);

/* One SDIRK step of Sec. 4 (scheme 2 = SD2, the implicit midpoint rule; 3 = SD3, the
 * three-stage L-stable third-order method of Alexander; 4 = SD4, the three-stage fourth-order
 * method of Crouzeix).  Stage i solves R(k_i; a_ii dt, u + dt sum_{j<i} a_ij k_j) = 0 by the
 * same Newton-Krylov stage solve as ilh_stage_solve, from k_guess (NULL: zero) for stage 1
 * and from k_{i-1} for later stages; then u <- u + dt sum_i b_i k_i.  k_out (nullable)
 * receives the last stage rate.  st (host) sums the iteration counts over the stages and
 * keeps the residual history of the last stage.  On failure u is left unchanged.  Stage
 * storage (4 block vectors) is allocated on first use. */
int ilh_sdirk_step(ilh_ctx* ctx, double* u, double dt, int scheme, const double* k_guess, double* k_out,
                   const ilh_newton_opts* o, ilh_step_stats* st);

/* One explicit step of the RK2-average scheme, the explicit RK2 reference of Sec. 4 (defined
 * there by reference to Dobrev et al. 2012, Sec. 7.1):
 *   v_h = v + dt/2 a(u),  e_h = e + dt/2 M_E^-1 (F(u)^T v_h + b(x)),  x_h = x + dt/2 v_h,
 *   v+ = v + dt a(u_h),   vbar = (v + v+)/2,
 *   e+ = e + dt M_E^-1 (F(u_h)^T vbar + b(x_h)),  x+ = x + dt vbar,
 * with a(w) = -Mhat^-1 P_u F(w) 1 (velocity mass solve with the wall rows held at zero, PCG to
 * 1e-14) and b the TG energy source (else 0).  The averaged velocity makes the total energy
 * change exactly dt 1^T b(x_h).  u [block] is updated in place.  2D only (ILH_EINVAL in 3D);
 * uses 3 block vectors of workspace (allocated on first use). */
int ilh_rk2avg_step(ilh_ctx* ctx, double* u, double dt);

/* One accepted step under the Newton-based step-size control of Sec. 4 ("Implicit time step
 * control"), with the SDIRK scheme of ilh_sdirk_step.
 *   dt (host, in/out): in, the proposed step; out, the proposed next step: 1.05 x the accepted
 *     step when every stage needed at most one Newton iteration, the accepted step otherwise.
 *   dt_max: upper bound of this step (for instance the time left).
 *   A trial whose stages need four or more Newton iterations, or whose solve fails, is rejected:
 *   u is restored and the trial repeats with 85 % of its size, at most max_reject times (then
 *   the failure status, or ILH_ENOCONV, is returned with u unchanged).
 *   rejected, dt_taken (host, out, nullable): rejected trials and the accepted step.
 *   st (host, nullable) describes the accepted trial.
 * Every trial starts stage 1 from k_guess (NULL: zero).  Uses one more block vector of stage
 * storage than ilh_sdirk_step. */
int ilh_adaptive_step(ilh_ctx* ctx, double* u, double* dt, double dt_max, int scheme, const double* k_guess,
                      double* k_out, const ilh_newton_opts* o, ilh_step_stats* st, int max_reject,
                      int* rejected, double* dt_taken);

/* Change the smoothing scale delta_scale of the viscosity (Sec. 3.4, eqs. visc_imp_abs,
 * visc_imp_switch, visc_imp_scale) for the calls that follow: mode ILH_DSCALE_CONST with the given
 * width, or ILH_DSCALE_FORMULA (2 (h/h_coarse) c_s; width ignored).  Used for a continuation in the
 * smoothing width within a step (solve with a wide scale, then narrow it from that solution).
 * Stored tangent coefficients are invalidated.  No effect without viscosity.  ILH_EINVAL for an
 * unknown mode or a width <= 0. */
int ilh_set_viscosity_scale(ilh_ctx* ctx, int mode, double width);

/* ---- measurement --------------------------------------------------------------------- */
/* Kernel timing with HIP events recorded on the context stream around each launch of the
 * timed kernel classes: 0 = Jacobian-action element kernel, 1 = residual element kernel,
 * 2 = velocity-mass element kernel, 3 = Krylov orthogonalisation (multi-dot / multi-axpy),
 * 4 = other Newton-Krylov vector kernels, 5 = linearisation kernel of the linearised
 * Jacobian action (once per linearisation point and precision), 6 = transpose-action kernel.
 * For classes 0, 1, 5 and 6 the events are attached to the kernel dispatch itself.  ilh_timing_enable(ctx, 1) resets the
 * counters; ilh_timing_read synchronises the stream and returns, per class, the summed kernel
 * time in milliseconds and the number of timed launches (host arrays of ILH_TIMING_CLASSES). */
#define ILH_TIMING_CLASSES 7
/* Select the Jacobian-action kernels (all compute the same operator, for cross-checking):
 *   0 (default) linearised: where one exists (2D, k = 2, 3; 3D, k = 2 without the TG
 *     source), the tangent coefficients of every quadrature point are evaluated once per
 *     linearisation point and precision (FP64 arithmetic, stored in the precision of the
 *     action) and each action applies them;
 *   1 generic LDS-staged element kernel recomputing the state's quadrature data (it also
 *     takes over the residual, which otherwise runs on the strip kernels where they exist);
 *   2 register-resident 2D kernel recomputing the state's quadrature data (2D, k = 2, 3).
 * Other values: ILH_EINVAL. */
int ilh_set_kernel_variant(ilh_ctx* ctx, int variant);
/* Work split of the linearised apply kernels: one wave walks `rows` consecutive element rows
 * (2D) or element layers (3D) of its strip, so that node sums shared between those rows stay on
 * chip and only nodes shared with other waves are added atomically.  rows = 0 (default) picks
 * the count from the mesh size: 1 on meshes whose one-row grid has few waves per SIMD, up to 8
 * on large meshes.  The result does not depend on it beyond the order of FP additions.
 * rows < 0: ILH_EINVAL. */
int ilh_set_apply_rows(ilh_ctx* ctx, int rows);
/* Waves per strip of the 2D FP32 linearised Jacobian-action kernel: 1 (one wave takes every
 * quadrature row of its strip of elements) or 2 (the two waves of a work-group share the strip:
 * each takes half of the quadrature rows, and the direction's gathers and the node sums are
 * spread over both, which halves each wave's chain of dependent row steps on meshes whose
 * one-wave grid leaves SIMDs idle).  waves = 0 (default) picks 2 on meshes whose one-wave grid
 * has fewer than 1,024 waves (one per SIMD), else 1.  FP64 actions always use one wave.  The
 * result does not depend on it beyond the order of FP additions.  Other values: ILH_EINVAL. */
int ilh_set_apply_waves(ilh_ctx* ctx, int waves);
int ilh_timing_enable(ilh_ctx* ctx, int on);
int ilh_timing_read(ilh_ctx* ctx, double* ms, int64_t* launches);

/* ---- learned Newton initial guess (per-element MLP) ------------------------------------ */
/* Not part of the paper: a per-element MLP predicts the correction of the plain initial
 * iterate of each implicit stage (2D only).  Element-local layouts, element e with local H1
 * node (a, b) (index a + (k+1) b) and L2 dof j:
 *   features [Ne][ld]  float: v_c(a,b)/vscale (c = 0, 1) | e_j/escale |
 *                      (corner - element centre)/xscale for corners (0,0),(k,0),(0,k),(k,k) |
 *                      if base != NULL: base_v/kvscale | base_e/kescale;  zero padded to ld.
 *   targets  [Ne][ld]  float: (k_v - base_v)/kvscale | (k_e - base_e)/kescale (base NULL = 0).
 * ilh_guess_assemble turns predictions of that layout into a block vector: the velocity
 * part is averaged over the elements sharing each node and added to base (constrained rows
 * 0), the energy part is added element-locally, and k_x = u_v + tau k_v. */
int ilh_guess_features(ilh_ctx* ctx, const double* u, const double* base, double vscale,
                       double escale, double xscale, double kvscale, double kescale,
                       const float* mu, const float* sd, float* feat, int ld);
int ilh_guess_targets(ilh_ctx* ctx, const double* k, const double* base, double kvscale,
                      double kescale, const float* oscale, float* targ, int ld);
int ilh_guess_assemble(ilh_ctx* ctx, const float* pred, int ld, double kvscale, double kescale,
                       const float* oscale, const double* base, const double* u, double tau,
                       double* k);
/* Optional per-column arrays (device, float, nullable): features are standardised as
 * (f - mu[i]) / sd[i] after the scalar scaling; targets are divided by oscale[i] and
 * predictions multiplied by oscale[i] before assembly. */

/* A trained per-element guess model: device pointers owned by the caller.  Layouts as for
 * ilh_mlp_forward (W, b) and ilh_guess_features / ilh_guess_assemble (mu, sd, osc, scales). */
typedef struct {
  int nl;               /* layers (1..7) */
  int widths[8];        /* widths[0..nl], each 1..128 */
  const uint16_t* W;    /* BF16 weights */
  const float* b;       /* biases */
  const float* mu;      /* feature standardisation (nullable) */
  const float* sd;      /* (nullable) */
  const float* osc;     /* output scale (nullable) */
  double vscale, escale, xscale, kvscale, kescale;
  int with_base;        /* the features include the plain iterate's element rates */
} ilh_guess_model;

/* Learned initial iterate of a stage (callers that run the learned guess before each Newton
 * solve): features of (u, base), MLP forward, assembly (k_x = u_v + tau k_v); the stage
 * residual R(.; tau, u) judges the result against base, and k receives the learned iterate if
 * its residual norm is finite and smaller than base's (or base's is not finite), else a copy
 * of base.  u, base, k: device [block]; m, used (1 if learned, nullable): host.  Scratch for
 * the features, activations and one residual is kept in the context (allocated on first
 * use).  Synchronises (the judge reads two norms). */
int ilh_guess_infer(ilh_ctx* ctx, const ilh_guess_model* m, const double* u, const double* base, double tau,
                    double* k, int* used);

/* Features of (u, base) and the whole MLP of m in one launch: pred [Ne][ld] (float, device)
 * receives the network output of every element, equal to ilh_guess_features followed by
 * ilh_mlp_forward (same BF16 rounding, accumulation order and epilogue).  Each work-group keeps
 * every layer's BF16 weights and biases in LDS and walks tiles of 16 elements.  ILH_EINVAL when
 * the widths do not match this mesh's features (widths[0]) and outputs (widths[nl]), when the
 * padded weights exceed 112 KiB of LDS (rows padded by 8 entries), when ld is below the padded
 * output width, or when m->W is not 16-byte aligned.  ilh_guess_infer takes this path when the
 * model fits.  No synchronisation. */
int ilh_guess_mlp_fused(ilh_ctx* ctx, const ilh_guess_model* m, const double* u, const double* base,
                        float* pred, int ld);

/* MLP on MFMA (BF16 operands, FP32 accumulation): widths w[0..nl] (each 1..128), hidden
 * layers GELU (erf form), last layer linear.  Every width is padded to P(w) = 32 ceil(w/32);
 * padding entries are zero.  Concatenated over layers l = 0..nl-1:
 *   W  bf16 (uint16) [P(w_{l+1})][P(w_l)],  WT its transpose,  b float [P(w_{l+1})],
 *   zs / acts float [batch][P(w_{l+1})]: pre-activations / outputs of each layer.
 * x float [batch][P(w_0)].  The network output is the last acts block. */
int ilh_mlp_forward(ilh_ctx* ctx, int nl, const int* widths /*host*/, const uint16_t* W,
                    const float* b, const float* x, int batch, float* zs, float* acts);

/* Gradients of the loss 0.5/batch sum_{rows, cols < w_nl} (y - t)^2 (t [batch][P(w_nl)]):
 * dW (float, layout of W) and db (float), both overwritten.  work: float
 * [2 * batch * 128] scratch.  loss (host, nullable) receives the loss (synchronises). */
int ilh_mlp_backward(ilh_ctx* ctx, int nl, const int* widths /*host*/, const uint16_t* WT,
                     const float* x, const float* zs, const float* acts, const float* target,
                     int batch, float* dW, float* db, float* work, double* loss);

/* Adam step on n FP32 master parameters p with gradient g and moments m1, m2 (step >= 1):
 * p -= lr mhat / (sqrt(vhat) + eps) with bias-corrected moments mhat, vhat. */
int ilh_mlp_adam(ilh_ctx* ctx, int64_t n, float* p, const float* g, float* m1, float* m2,
                 int step, double lr, double beta1, double beta2, double eps);

/* Round the FP32 master weights (layout of W) to BF16 into W and its transpose WT. */
int ilh_mlp_pack(ilh_ctx* ctx, int nl, const int* widths /*host*/, const float* Wmaster,
                 uint16_t* W, uint16_t* WT);

#ifdef __cplusplus
}
#endif

#endif

"""ctypes declarations of the libilh.so C ABI (include/ilh.h).  Marshalling only."""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libilh.so")

ILH_OK, ILH_EINVAL, ILH_EHIP, ILH_ENOMEM, ILH_ETANGLED, ILH_ENOCONV, ILH_ENONFINITE = range(7)
PROBLEMS = {"custom": 0, "tg2d": 1, "tg3d": 2, "triple": 3, "uniform": 4}


class Setup(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("n", C.c_int * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("order_v", C.c_int), ("nq1d", C.c_int), ("problem", C.c_int),
        ("rho0_elem", C.POINTER(C.c_double)), ("gamma_elem", C.POINTER(C.c_double)),
        ("e0_elem", C.POINTER(C.c_double)),
        ("visc_on", C.c_int), ("q1", C.c_double), ("q2", C.c_double), ("psi0", C.c_double),
        ("dscale_mode", C.c_int), ("dscale_width", C.c_double), ("h0", C.c_double),
        ("h_coarse", C.c_double), ("eps_e", C.c_double), ("tg_source", C.c_int),
        ("x0", C.POINTER(C.c_double)), ("free_faces", C.c_int),
    ]


class NewtonOpts(C.Structure):
    _fields_ = [
        ("tol", C.c_double), ("max_newton", C.c_int), ("restart", C.c_int),
        ("gmres_rtol", C.c_double), ("gmres_maxit", C.c_int), ("jvp_prec", C.c_int),
        ("max_halvings", C.c_int), ("pcg_iters", C.c_int), ("prec_coupled", C.c_int),
        ("guess_fallback", C.c_int), ("ls_residual", C.c_int), ("prec_probe", C.c_int),
        ("prec_lag", C.c_int), ("graphs", C.c_int), ("basis64", C.c_int), ("cgs2", C.c_int),
    ]


class StepStats(C.Structure):
    _fields_ = [
        ("status", C.c_int), ("newton_iters", C.c_int), ("gmres_iters", C.c_int),
        ("jvp_calls", C.c_int), ("halvings", C.c_int), ("guess_rejected", C.c_int), ("res0", C.c_double),
        ("res_init", C.c_double), ("res_final", C.c_double), ("res_hist", C.c_double * 32),
        ("newton_max", C.c_int),
    ]


class GuessModel(C.Structure):
    _fields_ = [
        ("nl", C.c_int), ("widths", C.c_int * 8), ("W", C.c_void_p), ("b", C.c_void_p), ("mu", C.c_void_p),
        ("sd", C.c_void_p), ("osc", C.c_void_p), ("vscale", C.c_double), ("escale", C.c_double),
        ("xscale", C.c_double), ("kvscale", C.c_double), ("kescale", C.c_double), ("with_base", C.c_int),
    ]


P = C.c_void_p
D = C.c_double
I = C.c_int
I64 = C.c_int64

SIGNATURES = {
    "ilh_setup_defaults": (None, [C.POINTER(Setup), I]),
    "ilh_create": (I, [C.POINTER(Setup), P, C.POINTER(P)]),
    "ilh_destroy": (None, [P]),
    "ilh_set_stream": (I, [P, P]),
    "ilh_last_error": (C.c_char_p, [P]),
    "ilh_status_string": (C.c_char_p, [I]),
    "ilh_sizes": (I, [P, C.POINTER(I64), C.POINTER(I64), C.POINTER(I64), C.POINTER(I64)]),
    "ilh_init_state": (I, [P, P]),
    "ilh_force": (I, [P, P, P, P]),
    "ilh_force_jvp": (I, [P, I, P, P, P, P]),
    "ilh_residual": (I, [P, P, P, D, P]),
    "ilh_linearize": (I, [P, P, P, D]),
    "ilh_jvp_lin": (I, [P, I, P, P]),
    "ilh_jvp": (I, [P, I, P, P, D, P, P]),
    "ilh_jvp_noalloc": (I, [P, I, P, P, D, P, P]),
    "ilh_mass_v_apply": (I, [P, P, P]),
    "ilh_mass_v_solve": (I, [P, P, P, D, I, C.POINTER(I), C.POINTER(D)]),
    "ilh_mass_e_inv": (I, [P, P, P]),
    "ilh_energy": (I, [P, P, C.POINTER(D), C.POINTER(D)]),
    "ilh_min_detj": (I, [P, P, C.POINTER(D)]),
    "ilh_dt_estimate": (I, [P, P, D, C.POINTER(D)]),
    "ilh_l1_velocity_error": (I, [P, P, C.POINTER(D)]),
    "ilh_rate": (I, [P, P, P]),
    "ilh_plain_guess": (I, [P, P, P, P, I, D, P]),
    "ilh_plain_guess_fallback": (I, [P, P, P, P, I, D, P, C.POINTER(I)]),
    "ilh_newton_defaults": (None, [C.POINTER(NewtonOpts)]),
    "ilh_implicit_step": (I, [P, P, D, P, P, C.POINTER(NewtonOpts), C.POINTER(StepStats)]),
    "ilh_stage_solve": (I, [P, P, D, P, P, C.POINTER(NewtonOpts), C.POINTER(StepStats)]),
    "ilh_sdirk_step": (I, [P, P, D, I, P, P, C.POINTER(NewtonOpts), C.POINTER(StepStats)]),
    "ilh_probe_blocks": (I, [P, I, P, P]),
    "ilh_invert_blocks": (I, [P, P]),
    "ilh_guess_infer": (I, [P, C.POINTER(GuessModel), P, P, D, P, C.POINTER(I)]),
    "ilh_guess_mlp_fused": (I, [P, C.POINTER(GuessModel), P, P, P, I]),
    "ilh_adaptive_step": (I, [P, P, C.POINTER(D), D, I, P, P, C.POINTER(NewtonOpts), C.POINTER(StepStats), I,
                              C.POINTER(I), C.POINTER(D)]),
    "ilh_timing_enable": (I, [P, I]),
    "ilh_set_viscosity_scale": (I, [P, I, D]),
    "ilh_set_kernel_variant": (I, [P, I]),
    "ilh_set_apply_rows": (I, [P, I]),
    "ilh_set_apply_waves": (I, [P, I]),
    "ilh_vjp_lin": (I, [P, I, P, P]),
    "ilh_vjp": (I, [P, I, P, P, D, P, P]),
    "ilh_rk2avg_step": (I, [P, P, D]),
    "ilh_timing_read": (I, [P, C.POINTER(D), C.POINTER(I64)]),
    "ilh_guess_features": (I, [P, P, P, D, D, D, D, D, P, P, P, I]),
    "ilh_guess_targets": (I, [P, P, P, D, D, P, P, I]),
    "ilh_guess_assemble": (I, [P, P, I, D, D, P, P, P, D, P]),
    "ilh_mlp_forward": (I, [P, I, C.POINTER(I), P, P, P, I, P, P]),
    "ilh_mlp_backward": (I, [P, I, C.POINTER(I), P, P, P, P, P, I, P, P, P, C.POINTER(D)]),
    "ilh_mlp_adam": (I, [P, I64, P, P, P, P, I, D, D, D, D]),
    "ilh_mlp_pack": (I, [P, I, C.POINTER(I), P, P, P]),
}

_lib = None


def load():
    """Load libilh.so (built in-tree by __graft_entry__.build()).  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libilh.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        if not hasattr(lib, name):
            continue
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return list(SIGNATURES)

"""MI355X (gfx950) implicit high-order Lagrangian hydrodynamics.

Python binding of libilh.so (include/ilh.h): every call marshals torch device tensors to
the C ABI and runs on the library's HIP kernels.  There is no CPU fallback: if the
library is not built, or no GPU is present, the calls raise.
"""
import ctypes as C

import torch

from . import _lib
from ._lib import NewtonOpts, Setup, StepStats, PROBLEMS

__all__ = ["Hydro", "IlhError", "ForceFn", "ResidualFn", "newton_options", "make_sedov"]


class IlhError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("ilh status %d: %s" % (status, msg))
        self.status = status


def newton_options(**kw):
    lib = _lib.load()
    o = NewtonOpts()
    lib.ilh_newton_defaults(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _raw(t):
    """The plain tensor under functorch wrappers (torch.func transforms hand those to custom rules)."""
    while torch._C._functorch.is_functorch_wrapped_tensor(t):
        t = torch._C._functorch.get_unwrapped(t)
    return t


def _ptr(t):
    return C.c_void_p(_raw(t).data_ptr())


class Hydro:
    """One discretisation context on one GPU (wraps ilh_ctx)."""

    def __init__(self, problem, n, k, visc=False, dscale_mode="const", dscale_width=1e-3, q1=0.5,
                 q2=1.0, psi0=0.5, h0=0.0, h_coarse=0.0, tg_source=None, rho0=None, gamma=None,
                 e0=None, lo=None, hi=None, x0=None, free_faces=0, device="cuda"):
        """x0 (host array of d * N positions, nullable): a curved initial mesh; free_faces: bit
        mask of box faces without the wall condition (bit 2d: x_d = lo_d, bit 2d+1: x_d = hi_d)."""
        self.lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("ilh needs a ROCm GPU; none is visible")
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        s = Setup()
        s.dim = len(n)
        for d in range(len(n)):
            s.n[d] = int(n[d])
        s.order_v = int(k)
        self.lib.ilh_setup_defaults(C.byref(s), PROBLEMS[problem])
        s.visc_on = int(bool(visc))
        s.dscale_mode = {"const": 0, "formula": 1}[dscale_mode]
        s.dscale_width, s.q1, s.q2, s.psi0 = dscale_width, q1, q2, psi0
        s.h0, s.h_coarse = h0, h_coarse
        if tg_source is not None:
            s.tg_source = int(bool(tg_source))
        if lo is not None:
            for d in range(len(lo)):
                s.lo[d] = lo[d]
        if hi is not None:
            for d in range(len(hi)):
                s.hi[d] = hi[d]
        self._keep = []
        for name, arr in (("rho0_elem", rho0), ("gamma_elem", gamma), ("e0_elem", e0)):
            if arr is not None:
                a = (C.c_double * len(arr))(*[float(x) for x in arr])
                self._keep.append(a)
                setattr(s, name, C.cast(a, C.POINTER(C.c_double)))
        if x0 is not None:
            import numpy as np
            a = np.ascontiguousarray(np.asarray(x0, dtype=np.float64).ravel())
            self._keep.append(a)
            s.x0 = a.ctypes.data_as(C.POINTER(C.c_double))
        s.free_faces = int(free_faces)
        self.setup = s
        ctx = C.c_void_p()
        with torch.cuda.device(self.device):
            st = self.lib.ilh_create(C.byref(s), C.c_void_p(torch.cuda.current_stream().cuda_stream),
                                     C.byref(ctx))
        if st != 0:
            raise IlhError(st, "ilh_create failed (see stderr)")
        self.ctx = ctx
        nh1, nl2, nb, nq = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        self.lib.ilh_sizes(ctx, C.byref(nh1), C.byref(nl2), C.byref(nb), C.byref(nq))
        self.nh1, self.nl2, self.nblock, self.nqp = nh1.value, nl2.value, nb.value, nq.value
        self.dim, self.k, self.n = len(n), int(k), tuple(int(v) for v in n)
        self.Ne = 1
        for v in self.n:
            self.Ne *= v

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            try:
                torch.cuda.synchronize(self.device)
            except Exception:
                pass
            self.lib.ilh_destroy(ctx)
            self.ctx = None

    # ---- helpers ----
    def _check(self, st):
        if st != 0:
            raise IlhError(st, self.lib.ilh_last_error(self.ctx).decode())

    def _stream(self):
        self.lib.ilh_set_stream(self.ctx, C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def _vec(self, t, n, dtype=torch.float64, name="vector"):
        if not isinstance(t, torch.Tensor) or t.device != self.device or t.dtype != dtype:
            raise TypeError("%s must be a %s tensor on %s" % (name, dtype, self.device))
        if not t.is_contiguous() or t.numel() != n:
            raise ValueError("%s must be contiguous with %d elements (got %d)" % (name, n, t.numel()))
        return _ptr(t)

    def new(self, n=None, dtype=torch.float64):
        return torch.zeros(self.nblock if n is None else n, dtype=dtype, device=self.device)

    def split(self, u):
        return u[:self.nh1], u[self.nh1:2 * self.nh1], u[2 * self.nh1:]

    # ---- ABI wrappers ----
    def init_state(self):
        u = self.new()
        self._stream()
        self._check(self.lib.ilh_init_state(self.ctx, _ptr(u)))
        return u

    def force(self, w):
        f1, ftv = self.new(self.nh1), self.new(self.nl2)
        self._stream()
        self._check(self.lib.ilh_force(self.ctx, self._vec(w, self.nblock, name="w"), _ptr(f1), _ptr(ftv)))
        return f1, ftv

    def force_jvp(self, w, dw, prec=64):
        dt = torch.float64 if prec == 64 else torch.float32
        df1, dftv = self.new(self.nh1, dt), self.new(self.nl2, dt)
        self._stream()
        self._check(self.lib.ilh_force_jvp(self.ctx, prec, self._vec(w, self.nblock, name="w"),
                                           self._vec(dw, self.nblock, dt, "dw"), _ptr(df1), _ptr(dftv)))
        return df1, dftv

    def residual(self, k, u, tau, out=None):
        r = self.new() if out is None else out
        self._stream()
        self._check(self.lib.ilh_residual(self.ctx, self._vec(k, self.nblock, name="k"),
                                          self._vec(u, self.nblock, name="u"), float(tau), _ptr(r)))
        return r

    def linearize(self, k, u, tau):
        self._stream()
        self._check(self.lib.ilh_linearize(self.ctx, self._vec(k, self.nblock, name="k"),
                                           self._vec(u, self.nblock, name="u"), float(tau)))

    def jvp_lin(self, dk, prec=64, out=None):
        dt = torch.float64 if prec == 64 else torch.float32
        o = self.new(dtype=dt) if out is None else out
        self._stream()
        self._check(self.lib.ilh_jvp_lin(self.ctx, prec, self._vec(dk, self.nblock, dt, "dk"),
                                         self._vec(o, self.nblock, dt, "out")))
        return o

    def jvp(self, k, u, tau, dk, prec=64):
        self.linearize(k, u, tau)
        return self.jvp_lin(dk, prec)

    def vjp_lin(self, y, prec=64, out=None):
        """Transpose Jacobian action J^T y at the stored linearisation point (2D k = 2, 3; 3D k = 2)."""
        dt = torch.float64 if prec == 64 else torch.float32
        o = self.new(dtype=dt) if out is None else out
        self._stream()
        self._check(self.lib.ilh_vjp_lin(self.ctx, prec, self._vec(y, self.nblock, dt, "y"),
                                         self._vec(o, self.nblock, dt, "out")))
        return o

    def jvp_noalloc(self, k, u, tau, dk, prec=64, out=None):
        """ilh_jvp_noalloc: the Jacobian action with the library's static scratch (allocates nothing
        on the device; `out`, if given, receives the result so that the call makes no allocation
        through torch either)."""
        dt = torch.float64 if prec == 64 else torch.float32
        o = self.new(dtype=dt) if out is None else out
        self._stream()
        self._check(self.lib.ilh_jvp_noalloc(self.ctx, prec, self._vec(k, self.nblock, name="k"),
                                             self._vec(u, self.nblock, name="u"), float(tau),
                                             self._vec(dk, self.nblock, dt, "dk"),
                                             self._vec(o, self.nblock, dt, "out")))
        return o

    def vjp(self, k, u, tau, y, prec=64):
        self.linearize(k, u, tau)
        return self.vjp_lin(y, prec)

    def rk2avg_step(self, u, dt):
        """One explicit RK2-average step, u updated in place (2D)."""
        self._stream()
        self._check(self.lib.ilh_rk2avg_step(self.ctx, self._vec(u, self.nblock, name="u"), float(dt)))
        return u

    def mass_v_apply(self, x):
        y = self.new(self.nh1)
        self._stream()
        self._check(self.lib.ilh_mass_v_apply(self.ctx, self._vec(x, self.nh1, name="x"), _ptr(y)))
        return y

    def mass_v_solve(self, b, rtol=1e-12, maxit=500):
        x = self.new(self.nh1)
        it, rel = C.c_int(), C.c_double()
        self._stream()
        self._check(self.lib.ilh_mass_v_solve(self.ctx, self._vec(b, self.nh1, name="b"), _ptr(x),
                                              float(rtol), int(maxit), C.byref(it), C.byref(rel)))
        return x, it.value, rel.value

    def mass_e_inv(self, b):
        x = self.new(self.nl2)
        self._stream()
        self._check(self.lib.ilh_mass_e_inv(self.ctx, self._vec(b, self.nl2, name="b"), _ptr(x)))
        return x

    def energy(self, u):
        ke, ie = C.c_double(), C.c_double()
        self._stream()
        self._check(self.lib.ilh_energy(self.ctx, self._vec(u, self.nblock, name="u"), C.byref(ke), C.byref(ie)))
        return ke.value, ie.value

    def min_detj(self, w):
        m = C.c_double()
        self._stream()
        self._check(self.lib.ilh_min_detj(self.ctx, self._vec(w, self.nblock, name="w"), C.byref(m)))
        return m.value

    def dt_estimate(self, u, cfl):
        dt = C.c_double()
        self._stream()
        self._check(self.lib.ilh_dt_estimate(self.ctx, self._vec(u, self.nblock, name="u"), float(cfl),
                                             C.byref(dt)))
        return dt.value

    def l1_error(self, u):
        e = C.c_double()
        self._stream()
        self._check(self.lib.ilh_l1_velocity_error(self.ctx, self._vec(u, self.nblock, name="u"), C.byref(e)))
        return e.value

    def rate(self, u):
        f = self.new()
        self._stream()
        self._check(self.lib.ilh_rate(self.ctx, self._vec(u, self.nblock, name="u"), _ptr(f)))
        return f

    def plain_guess(self, u, history, tau=0.0, fallback=False):
        """Explicit rate, last rate, or linear extrapolation of the last two (most recent last);
        with tau > 0 the position block is set to u_v + tau k_v.  fallback: the better of the
        extrapolation and the last rate by stage residual (ilh_plain_guess_fallback)."""
        out = torch.empty(self.nblock, dtype=torch.float64, device=self.device)  # every block is written
        k1 = self._vec(history[-1], self.nblock, name="k1") if len(history) >= 1 else None
        k2 = self._vec(history[-2], self.nblock, name="k2") if len(history) >= 2 else None
        self._stream()
        if fallback:
            which = C.c_int(0)
            self._check(self.lib.ilh_plain_guess_fallback(self.ctx, self._vec(u, self.nblock, name="u"), k1, k2,
                                                          min(len(history), 2), float(tau), _ptr(out),
                                                          C.byref(which)))
            self.last_plain_choice = which.value
            return out
        self._check(self.lib.ilh_plain_guess(self.ctx, self._vec(u, self.nblock, name="u"), k1, k2,
                                             min(len(history), 2), float(tau), _ptr(out)))
        return out

    def probe_blocks(self, mode=1):
        """(velocity-block diagonal [nh1], inverted energy blocks [Ne, Nl, Nl]) at the stored
        linearisation point; mode 1 eliminates the position block, mode 2 does not."""
        nl = self.nl2 // self.Ne
        dv = self.new(self.nh1)
        einv = self.new(self.Ne * nl * nl)
        self._stream()
        self._check(self.lib.ilh_probe_blocks(self.ctx, int(mode), _ptr(dv), _ptr(einv)))
        return dv, einv.view(self.Ne, nl, nl)

    def invert_blocks(self, blocks):
        """In place: each [Nl, Nl] block of blocks [Ne, Nl, Nl] (FP64, on the device) replaced by
        its inverse, as the probed preconditioner inverts its element blocks (a block with a zero
        pivot column becomes the identity)."""
        nl = self.nl2 // self.Ne
        self._stream()
        self._check(self.lib.ilh_invert_blocks(self.ctx, self._vec(blocks.view(-1), self.Ne * nl * nl,
                                                                     name="blocks")))
        return blocks

    JVP_VARIANTS = {"lin": 0, "generic": 1, "recompute": 2}

    def set_viscosity_scale(self, mode, width=0.0):
        """delta_scale of the viscosity from now on: mode "const" (width) or "formula"."""
        self._check(self.lib.ilh_set_viscosity_scale(self.ctx, {"const": 0, "formula": 1}[mode], float(width)))

    def set_kernel_variant(self, variant):
        """Jacobian-action kernels: "lin" (default), "generic" or "recompute" (or 0, 1, 2)."""
        v = self.JVP_VARIANTS[variant] if isinstance(variant, str) else int(variant)
        self._stream()
        self._check(self.lib.ilh_set_kernel_variant(self.ctx, v))

    def set_apply_rows(self, rows):
        """Element rows (2D) or layers (3D) walked by one wave of the linearised apply kernels;
        0 chooses by mesh size."""
        self._check(self.lib.ilh_set_apply_rows(self.ctx, int(rows)))

    def set_apply_waves(self, waves):
        """Waves per element strip of the 2D FP32 linearised apply kernel (1 or 2); 0 chooses by
        mesh size."""
        self._check(self.lib.ilh_set_apply_waves(self.ctx, int(waves)))

    def timing(self, on=True):
        self._check(self.lib.ilh_timing_enable(self.ctx, int(bool(on))))

    def timing_read(self):
        names = ("jvp", "residual", "mass", "krylov", "precond", "linearize", "transpose")
        ms = (C.c_double * len(names))()
        cnt = (C.c_int64 * len(names))()
        self._check(self.lib.ilh_timing_read(self.ctx, ms, cnt))
        return {nm: (ms[i], cnt[i]) for i, nm in enumerate(names)}

    def stage_solve(self, ubase, tau, guess=None, opts=None):
        opts = opts or newton_options()
        k = self.new()
        st = StepStats()
        self._stream()
        g = self._vec(guess, self.nblock, name="guess") if guess is not None else None
        code = self.lib.ilh_stage_solve(self.ctx, self._vec(ubase, self.nblock, name="u"), float(tau), g,
                                        _ptr(k), C.byref(opts), C.byref(st))
        return k, _stats(st, code)

    def implicit_step(self, u, dt, guess=None, opts=None, raise_on_fail=True):
        """u <- u + dt k with k = f(u + dt/2 k) (in place); returns (k, stats dict)."""
        opts = opts or newton_options()
        k = torch.empty(self.nblock, dtype=torch.float64, device=self.device)  # written by the library
        st = StepStats()
        self._stream()
        g = self._vec(guess, self.nblock, name="guess") if guess is not None else None
        code = self.lib.ilh_implicit_step(self.ctx, self._vec(u, self.nblock, name="u"), float(dt), g,
                                          _ptr(k), C.byref(opts), C.byref(st))
        stats = _stats(st, code)
        if code != 0 and raise_on_fail:
            raise IlhError(code, self.lib.ilh_last_error(self.ctx).decode())
        return k, stats

    SDIRK = {"sd2": 2, "sd3": 3, "sd4": 4}

    def sdirk_step(self, u, dt, scheme="sd3", guess=None, opts=None, raise_on_fail=True):
        """One SDIRK step (SD2 / SD3 / SD4) in place on u; returns (last stage rate, stats)."""
        opts = opts or newton_options()
        k = self.new()
        st = StepStats()
        self._stream()
        g = self._vec(guess, self.nblock, name="guess") if guess is not None else None
        code = self.lib.ilh_sdirk_step(self.ctx, self._vec(u, self.nblock, name="u"), float(dt),
                                       self.SDIRK[scheme], g, _ptr(k), C.byref(opts), C.byref(st))
        stats = _stats(st, code)
        if code != 0 and raise_on_fail:
            raise IlhError(code, self.lib.ilh_last_error(self.ctx).decode())
        return k, stats

    def adaptive_step(self, u, dt, dt_max, scheme="sd2", guess=None, opts=None, max_reject=30):
        """One accepted step of the Newton-based step-size control (in place on u).
        Returns (last stage rate, stats, accepted step, proposed next step, rejected trials)."""
        opts = opts or newton_options()
        k = self.new()
        st = StepStats()
        h = C.c_double(float(dt))
        taken = C.c_double(0.0)
        nrej = C.c_int(0)
        self._stream()
        g = self._vec(guess, self.nblock, name="guess") if guess is not None else None
        code = self.lib.ilh_adaptive_step(self.ctx, self._vec(u, self.nblock, name="u"), C.byref(h),
                                          float(dt_max), self.SDIRK[scheme], g, _ptr(k), C.byref(opts),
                                          C.byref(st), int(max_reject), C.byref(nrej), C.byref(taken))
        if code != 0:
            raise IlhError(code, self.lib.ilh_last_error(self.ctx).decode())
        return k, _stats(st, code), taken.value, h.value, nrej.value


def _stats(st, code):
    n = min(st.newton_iters, 31)
    return dict(status=code, newton=st.newton_iters, newton_max=st.newton_max, gmres=st.gmres_iters,
                jvp_calls=st.jvp_calls,
                halvings=st.halvings, guess_rejected=st.guess_rejected, res0=st.res0, res_init=st.res_init, res_final=st.res_final,
                hist=[st.res_hist[i] for i in range(n + 1)])


def make_sedov(n, k, visc=True, h_coarse=None):
    """2D Sedov blast (Sec. 4.2): unit square, walls, gamma 1.4, rho 1, v 0, the deposited
    energy 0.25 as a constant specific energy in the element at the origin (zero elsewhere),
    the smoothed viscosity with delta_scale = 2 (h / h_coarse) c_s.  h_coarse defaults to the
    isotropic length of a 1 x 1 base mesh of the same order (1/k)."""
    ne = int(n) * int(n)
    e0 = [0.0] * ne
    e0[0] = 0.25 * n * n
    hc = 1.0 / k if h_coarse is None else h_coarse
    return Hydro("custom", (n, n), k, visc=visc, dscale_mode="formula", h_coarse=hc, rho0=[1.0] * ne,
                 gamma=[1.4] * ne, e0=e0, lo=(0.0, 0.0), hi=(1.0, 1.0), tg_source=False)


class ForceFn(torch.autograd.Function):
    """(F(w) 1, F(w)^T w_v) with a forward-mode derivative from the hand-written tangent kernel.

    forward(hydro, w) -> (f1, ftv); jvp(dw) -> (d f1, d ftv) via ilh_force_jvp (FP64).  Forward
    mode only (see backward).
    """

    @staticmethod
    def forward(hydro, w):
        return hydro.force(w.detach().contiguous())

    @staticmethod
    def setup_context(ctx, inputs, output):
        hydro, w = inputs
        ctx.hydro = hydro
        ctx.save_for_forward(w)

    @staticmethod
    def jvp(ctx, _hydro_t, dw):
        (w,) = ctx.saved_tensors
        return ctx.hydro.force_jvp(w.detach().contiguous(), dw.contiguous(), 64)

    @staticmethod
    def backward(ctx, *grads):
        # The library's transpose action (ilh_vjp_lin) is that of the stage residual, which adds
        # the masses and replaces the wall rows by the identity; the bare force actions carry no
        # boundary conditions, so their transpose is not recoverable from it.  Reverse mode is
        # provided for the residual (ResidualFn.backward), not for the force alone.
        raise NotImplementedError("ForceFn has forward mode only; use ResidualFn for reverse mode")


class ResidualFn(torch.autograd.Function):
    """R(k; tau, u) with forward-mode derivative J dk from ilh_jvp and reverse-mode derivative
    J^T g from ilh_vjp (FP64; the reverse mode is built for 2D meshes with k = 2, 3 and 3D with k = 2)."""

    @staticmethod
    def forward(hydro, k, u, tau):
        return hydro.residual(k.detach().contiguous(), u.detach().contiguous(), float(tau))

    @staticmethod
    def setup_context(ctx, inputs, output):
        hydro, k, u, tau = inputs
        ctx.hydro, ctx.tau = hydro, float(tau)
        ctx.save_for_forward(k, u)
        ctx.save_for_backward(k, u)

    @staticmethod
    def jvp(ctx, _h, dk, du, _t):
        k, u = ctx.saved_tensors
        if du is not None and bool(torch.any(du != 0)):
            raise NotImplementedError("tangents in u are not supported; differentiate in k")
        if dk is None:
            dk = torch.zeros_like(k)
        return ctx.hydro.jvp(k.detach().contiguous(), u.detach().contiguous(), ctx.tau, dk.contiguous(), 64)

    @staticmethod
    def backward(ctx, g):
        if ctx.needs_input_grad[2]:
            raise NotImplementedError("gradients in u are not supported; differentiate in k")
        k, u = ctx.saved_tensors
        gk = ctx.hydro.vjp(k.detach().contiguous(), u.detach().contiguous(), ctx.tau, g.contiguous(), 64)
        return None, gk, None, None


def __getattr__(name):
    if name == "learned":
        import importlib
        return importlib.import_module(".learned", __name__)
    raise AttributeError(name)

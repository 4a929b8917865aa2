"""Learned Newton initial guess for the implicit stage solve (2D).

A per-element MLP maps element features of the current state (and of the plain
extrapolated iterate) to a correction of that plain iterate; the element predictions are
assembled (shared velocity nodes averaged) into a block vector.  The library's residual
is the judge: the learned iterate is used only when its stage residual is smaller than
the plain iterate's, otherwise the solve starts from the plain iterate.

Everything numerical runs in libilh.so: features, MLP forward/backward (BF16 MFMA with
FP32 accumulation), Adam, assembly, residuals and the Newton-Krylov solves.  Python only
orchestrates (batching, bookkeeping, file I/O).

Command line:
  python -m paper_2609_16424_amd.learned train --runs 200 --steps 30 --out MODEL.npz
  python -m paper_2609_16424_amd.learned eval --model MODEL.npz --seeds 1000-1009
"""
import argparse
import ctypes as C
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import Hydro, IlhError, _lib, newton_options

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_MODEL = os.path.join(HERE, "models", "guess_triple_q3q2.npz")        # 8x explicit step
MODEL_4X = os.path.join(HERE, "models", "guess_triple_q3q2_4x.npz")          # 4x explicit step

# triple-point regions: (rho, p, gamma) for x < 1; x > 1, y < 1.5; x > 1, y > 1.5
TRIPLE = ((1.0, 1.0, 1.5), (1.0, 0.1, 1.4), (0.125, 0.1, 1.5))


def pad32(w):
    return (w + 31) // 32 * 32


def triple_materials(nx, ny, scale=None, shift=0.0):
    """Per-element (rho0, gamma, e0) of the triple point on [0,7]x[0,3], optionally with the
    region densities/pressures multiplied by scale[r] = (s_rho, s_p) and the interfaces
    moved by `shift`."""
    h = (7.0 / nx, 3.0 / ny)
    rho = np.empty(nx * ny)
    gam = np.empty(nx * ny)
    e0 = np.empty(nx * ny)
    for ey in range(ny):
        for ex in range(nx):
            xc = (ex + 0.5) * h[0] - shift
            yc = (ey + 0.5) * h[1] - shift
            r = 0 if xc < 1.0 else (1 if yc < 1.5 else 2)
            r0, p0, g = TRIPLE[r]
            sr, sp = (1.0, 1.0) if scale is None else scale[r]
            e = ex + nx * ey
            rho[e], gam[e] = r0 * sr, g
            e0[e] = p0 * sp / ((g - 1.0) * r0 * sr)
    return rho, gam, e0


def perturbation(seed):
    """Seeded perturbation of a training/evaluation run: region rho, p in U(0.8, 1.2),
    interface shift j/16 with j in {-2..2}."""
    rng = np.random.default_rng(seed)
    scale = [(rng.uniform(0.8, 1.2), rng.uniform(0.8, 1.2)) for _ in range(3)]
    shift = rng.integers(-2, 3) / 16.0
    return scale, shift


VISC = {"mode": "formula", "width": 1e-3, "h_coarse": 1.0 / 3.0}


def model_newton_options(z):
    """Newton-Krylov options a committed model is evaluated with (its preconditioner settings;
    the GMRES restart length only changes how the inexact Newton steps are reached)."""
    pp = int(z["prec_probe"]) if "prec_probe" in z else 0
    pl = int(z["prec_lag"]) if "prec_lag" in z else 0
    return newton_options(tol=1e-10, jvp_prec=32, max_newton=30, restart=15, gmres_maxit=150,
                          prec_probe=pp, prec_lag=pl)


def make_triple(nx, ny, k, seed=None):
    """Triple point with the smoothed viscosity.  Default delta_scale: the paper's formula
    2 (h / h_coarse) c_s with h_coarse the isotropic length of the 7 x 3 base mesh (1/k)."""
    scale, shift = (None, 0.0) if seed is None else perturbation(seed)
    rho, gam, e0 = triple_materials(nx, ny, scale, shift)
    hc = VISC["h_coarse"] * 3.0 / k
    return Hydro("custom", (nx, ny), k, visc=True, dscale_mode=VISC["mode"], dscale_width=VISC["width"],
                 h_coarse=hc, rho0=rho, gamma=gam, e0=e0, lo=(0.0, 0.0), hi=(7.0, 3.0), tg_source=False)


class GuessMLP:
    """MLP parameters on the GPU: FP32 master weights + BF16 copies (W, W^T) + Adam moments."""

    def __init__(self, hydro, widths, seed=0):
        self.h = hydro
        self.lib = hydro.lib
        self.widths = list(widths)
        self.nl = len(widths) - 1
        P = [pad32(w) for w in widths]
        self.P = P
        self.wsz = [P[l + 1] * P[l] for l in range(self.nl)]
        self.bsz = [P[l + 1] for l in range(self.nl)]
        self.nW = sum(self.wsz)
        self.nparam = self.nW + sum(self.bsz)
        dev = hydro.device
        self.master = torch.zeros(self.nparam, dtype=torch.float32, device=dev)
        g = torch.Generator().manual_seed(seed)
        off = 0
        for l in range(self.nl):
            w = torch.zeros(P[l + 1], P[l])
            w[:widths[l + 1], :widths[l]] = torch.randn(widths[l + 1], widths[l], generator=g) * math.sqrt(2.0 / widths[l])
            if l == self.nl - 1:
                w *= 0.1
            self.master[off:off + self.wsz[l]] = w.reshape(-1).to(dev)
            off += self.wsz[l]
        self.m1 = torch.zeros_like(self.master)
        self.m2 = torch.zeros_like(self.master)
        self.grad = torch.zeros_like(self.master)
        self.W = torch.zeros(self.nW, dtype=torch.int16, device=dev)
        self.WT = torch.zeros(self.nW, dtype=torch.int16, device=dev)
        self.step_count = 0
        self.cw = (C.c_int * len(widths))(*widths)
        self.pack()

    def _p(self, t):
        return C.c_void_p(t.data_ptr())

    def pack(self):
        self.h._stream()
        self.h._check(self.lib.ilh_mlp_pack(self.h.ctx, self.nl, self.cw, self._p(self.master), self._p(self.W),
                                            self._p(self.WT)))

    @property
    def bias(self):
        return self.master[self.nW:]

    def forward(self, x):
        """x [B][P(w0)] float32 -> (zs, acts) concatenated, and the output view [B][P(wL)]."""
        B = x.shape[0]
        tot = sum(B * p for p in self.P[1:])
        zs = torch.empty(tot, dtype=torch.float32, device=x.device)
        acts = torch.empty(tot, dtype=torch.float32, device=x.device)
        self.h._stream()
        self.h._check(self.lib.ilh_mlp_forward(self.h.ctx, self.nl, self.cw, self._p(self.W), self._p(self.bias),
                                               self._p(x), B, self._p(zs), self._p(acts)))
        out = acts[tot - B * self.P[-1]:].view(B, self.P[-1])
        return zs, acts, out

    def train_step(self, x, t, lr, work):
        B = x.shape[0]
        zs, acts, _ = self.forward(x)
        loss = C.c_double()
        self.h._stream()
        self.h._check(self.lib.ilh_mlp_backward(self.h.ctx, self.nl, self.cw, self._p(self.WT), self._p(x),
                                                self._p(zs), self._p(acts), self._p(t), B,
                                                self._p(self.grad), self._p(self.grad[self.nW:]), self._p(work),
                                                C.byref(loss)))
        self.step_count += 1
        self.h._check(self.lib.ilh_mlp_adam(self.h.ctx, self.nparam, self._p(self.master), self._p(self.grad),
                                            self._p(self.m1), self._p(self.m2), self.step_count, lr, 0.9, 0.999,
                                            1e-8))
        self.pack()
        return loss.value

    def state(self):
        return {"widths": np.array(self.widths), "master": self.master.cpu().numpy()}

    def load_state(self, st):
        assert list(st["widths"]) == self.widths, "width mismatch"
        self.master.copy_(torch.from_numpy(st["master"]).to(self.master.device))
        self.pack()


class LearnedGuess:
    """Plain iterate + MLP correction, with the residual as judge and plain as fallback."""

    def __init__(self, hydro, mlp, scales, with_base=True, norm=None):
        self.h, self.mlp, self.sc, self.with_base = hydro, mlp, scales, with_base
        dev = hydro.device
        self.norm = None if norm is None else {k: torch.as_tensor(v, dtype=torch.float32, device=dev).contiguous()
                                               for k, v in norm.items()}
        k = hydro.k
        self.nout = 2 * (k + 1) ** 2 + k * k
        self.nin = self.nout + 8 + (self.nout if with_base else 0)
        assert mlp.widths[0] == self.nin and mlp.widths[-1] == self.nout
        self.ld_in = pad32(self.nin)
        self.ld_out = pad32(self.nout)
        self.feat = torch.zeros(hydro.Ne, self.ld_in, dtype=torch.float32, device=hydro.device)
        self.used = 0
        self.calls = 0

    def features(self, u, base):
        s = self.sc
        self.h._stream()
        nm = self.norm
        self.h._check(self.h.lib.ilh_guess_features(self.h.ctx, self.h._vec(u, self.h.nblock),
                                                    self.h._vec(base, self.h.nblock) if self.with_base else None,
                                                    s["vs"], s["es"], s["xs"], s["kvs"], s["kes"],
                                                    C.c_void_p(nm["mu"].data_ptr()) if nm else None,
                                                    C.c_void_p(nm["sd"].data_ptr()) if nm else None,
                                                    C.c_void_p(self.feat.data_ptr()), self.ld_in))
        return self.feat

    def predict(self, u, base, tau):
        x = self.features(u, base)
        _, _, out = self.mlp.forward(x)
        k = self.h.new()
        s = self.sc
        osc = C.c_void_p(self.norm["osc"].data_ptr()) if self.norm else None
        self.h._check(self.h.lib.ilh_guess_assemble(self.h.ctx, C.c_void_p(out.data_ptr()), self.ld_out, s["kvs"],
                                                    s["kes"], osc, self.h._vec(base, self.h.nblock),
                                                    self.h._vec(u, self.h.nblock), float(tau), C.c_void_p(k.data_ptr())))
        return k

    def predict_fused(self, u, base):
        """Network output [Ne][P(w_nl)] from ilh_guess_mlp_fused (features and every layer in one
        launch, the weights in LDS)."""
        out = torch.zeros(self.h.Ne, self.ld_out, dtype=torch.float32, device=self.h.device)
        self.h._stream()
        self.h._check(self.h.lib.ilh_guess_mlp_fused(self.h.ctx, C.byref(self.model()), self.h._vec(u, self.h.nblock),
                                                     self.h._vec(base, self.h.nblock) if self.with_base else None,
                                                     C.c_void_p(out.data_ptr()), self.ld_out))
        return out

    def predict_layered(self, u, base):
        """The same network output from ilh_guess_features and the layer-by-layer forward."""
        x = self.features(u, base)
        _, _, out = self.mlp.forward(x)
        return out

    def model(self):
        """Descriptor of this guess for ilh_guess_infer (device pointers stay owned here)."""
        m = _lib.GuessModel()
        m.nl = self.mlp.nl
        for i, w in enumerate(self.mlp.widths):
            m.widths[i] = int(w)
        m.W = self.mlp.W.data_ptr()
        m.b = self.mlp.bias.data_ptr()
        if self.norm:
            m.mu, m.sd, m.osc = (self.norm[k].data_ptr() for k in ("mu", "sd", "osc"))
        s = self.sc
        m.vscale, m.escale, m.xscale, m.kvscale, m.kescale = s["vs"], s["es"], s["xs"], s["kvs"], s["kes"]
        m.with_base = int(self.with_base)
        return m

    def guess(self, u, hist, tau):
        """Returns (k_guess, used_learned): one fused library call (features, MLP, assembly,
        residual judge against the plain iterate)."""
        base = self.h.plain_guess(u, hist, tau)
        k = self.h.new()
        used = C.c_int(0)
        self.h._stream()
        self.h._check(self.h.lib.ilh_guess_infer(self.h.ctx, C.byref(self.model()), self.h._vec(u, self.h.nblock),
                                                 self.h._vec(base, self.h.nblock), float(tau),
                                                 C.c_void_p(k.data_ptr()), C.byref(used)))
        self.calls += 1
        self.used += used.value
        return k, bool(used.value)


def default_scales(hydro, u0):
    """Normalisation scalars from the initial state (velocity unit from the sound speed)."""
    nh1 = hydro.nh1
    e = u0[2 * nh1:]
    es = float(torch.mean(torch.abs(e)))
    vs = math.sqrt(max(es, 1e-12))
    h = 7.0 / hydro.n[0]
    return {"vs": vs, "es": es, "xs": h, "kvs": vs / h * 0.1, "kes": es / h * vs * 0.1}


def run_plain(h, u, dt, steps, opts, record=None, scales=None):
    """Plain-guess trajectory; record (features, targets) of every step when asked."""
    hist = []
    stats = []
    for _ in range(steps):
        base = h.plain_guess(u, hist, 0.5 * dt)
        u_prev = u.clone()
        k, st = h.implicit_step(u, dt, guess=base, opts=opts, raise_on_fail=False)
        if st["status"] != 0:
            u.copy_(u_prev)
            stats.append(st)
            break
        if record is not None:
            record(u_prev, base, k)
        hist = (hist + [k])[-2:]
        stats.append(st)
    return stats


def generate(nx, ny, k, seeds, steps, cfl_factor, opts, scales_ref=None, log=None):
    """Trajectories of the perturbed triple point; returns features, targets (GPU tensors)."""
    feats, targs = [], []
    scales = scales_ref
    for s in seeds:
        h = make_triple(nx, ny, k, seed=s)
        u = h.init_state()
        if scales is None:
            scales = default_scales(h, u)
        dt = cfl_factor * h.dt_estimate(u, 0.5)
        nout = 2 * (k + 1) ** 2 + k * k
        nin = nout + 8 + nout
        ldi, ldo = pad32(nin), pad32(nout)

        def record(u_prev, base, kk):
            f = torch.zeros(h.Ne, ldi, dtype=torch.float32, device=h.device)
            t = torch.zeros(h.Ne, ldo, dtype=torch.float32, device=h.device)
            h._check(h.lib.ilh_guess_features(h.ctx, h._vec(u_prev, h.nblock), h._vec(base, h.nblock), scales["vs"],
                                              scales["es"], scales["xs"], scales["kvs"], scales["kes"], None, None,
                                              C.c_void_p(f.data_ptr()), ldi))
            h._check(h.lib.ilh_guess_targets(h.ctx, h._vec(kk, h.nblock), h._vec(base, h.nblock), scales["kvs"],
                                             scales["kes"], None, C.c_void_p(t.data_ptr()), ldo))
            feats.append(f)
            targs.append(t)

        t0 = time.time()
        st = run_plain(h, u, dt, steps, opts, record, scales)
        if log:
            log("run seed %d: %d steps, newton %s, %.2fs" % (s, len(st), [x["newton"] for x in st][:8], time.time() - t0))
        del h
    return torch.cat(feats), torch.cat(targs), scales


def column_stats(X, T, nin, nout):
    """Per-column standardisation of the features and output scales of the targets."""
    mu = torch.zeros(X.shape[1], device=X.device)
    sd = torch.ones(X.shape[1], device=X.device)
    mu[:nin] = X[:, :nin].mean(0)
    sdx = X[:, :nin].std(0)
    sd[:nin] = torch.clamp(sdx, min=1e-6 + 1e-3 * float(sdx.max()))
    osc = torch.ones(T.shape[1], device=T.device)
    sdt = T[:, :nout].std(0)
    osc[:nout] = torch.clamp(sdt, min=1e-12 + 1e-3 * float(sdt.max()))
    return {"mu": mu, "sd": sd, "osc": osc}


def train(model, X, T, epochs, batch, lr, log=None):
    n = X.shape[0]
    work = torch.empty(2 * batch * 128, dtype=torch.float32, device=X.device)
    g = torch.Generator(device=X.device).manual_seed(0)
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g, device=X.device)
        tot, cnt = 0.0, 0
        lr_ep = lr * 0.5 * (1 + math.cos(math.pi * ep / max(epochs, 1)))
        for i in range(0, n - batch + 1, batch):
            idx = perm[i:i + batch]
            tot += model.train_step(X[idx].contiguous(), T[idx].contiguous(), lr_ep, work)
            cnt += 1
        hist.append(tot / max(cnt, 1))
        if log:
            log("epoch %d loss %.4e" % (ep, hist[-1]))
    return hist


def evaluate(nx, ny, k, seeds, steps, cfl_factor, opts, model_state, scales, log=None):
    """Held-out comparison at equal final residual of four initial iterates: plain (the extrapolated
    iterate; the solver starts from k = 0 when that is better), plain_fallback (the extrapolation or
    the previous rate, whichever has the smaller stage residual, then the same k = 0 fallback),
    learned (the MLP's correction of the extrapolation, judged against it by the residual) and a
    zero-output control (the learned path's overhead with a network that outputs zero).  Every run of
    a seed goes on until its first failed step.  Each mode is summarised over its completed steps,
    and the learned run is compared with each other mode over matched steps: the step indices of a
    seed that both runs completed, so that both are timed on the same steps."""
    recs = {}
    for mode in ("plain", "plain_fallback", "learned", "zero"):
        recs[mode] = {}
        for s in seeds:
            h = make_triple(nx, ny, k, seed=s)
            u = h.init_state()
            dt = cfl_factor * h.dt_estimate(u, 0.5)
            lg = None
            if mode in ("learned", "zero"):
                mlp = GuessMLP(h, [int(w) for w in model_state["widths"]])
                if mode == "learned":
                    mlp.load_state(model_state)
                else:
                    mlp.master.zero_()
                    mlp.pack()
                norm = {k: model_state[k] for k in ("mu", "sd", "osc")} if "mu" in model_state else None
                lg = LearnedGuess(h, mlp, scales, norm=norm)
            hist, rows, failed = [], [], False
            torch.cuda.synchronize()
            for n in range(steps):
                t0 = time.perf_counter()
                if lg is None:
                    g, used = h.plain_guess(u, hist, 0.5 * dt, fallback=(mode == "plain_fallback")), False
                else:
                    g, used = lg.guess(u, hist, 0.5 * dt)
                torch.cuda.synchronize()
                t_guess = time.perf_counter() - t0
                k_, st = h.implicit_step(u, dt, guess=g, opts=opts, raise_on_fail=False)
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                if st["status"] != 0:
                    failed = True
                    break
                rows.append((wall, st["newton"], st["gmres"], st["res_init"] / max(st["res0"], 1e-300), used,
                             t_guess))
                hist = (hist + [k_])[-2:]
            recs[mode][s] = (rows, failed)
            del h
    out = {}
    for mode in recs:
        allr = [r for s in seeds for r in recs[mode][s][0]]
        ginit = [r[3] for r in allr]
        finite = [g for g in ginit if np.isfinite(g)]
        out[mode] = {"s_per_step": float(np.mean([r[0] for r in allr])) if allr else None,
                     "newton_per_step": float(np.mean([r[1] for r in allr])) if allr else None,
                     "gmres_per_step": float(np.mean([r[2] for r in allr])) if allr else None,
                     "steps": len(allr), "learned_used": int(sum(r[4] for r in allr)),
                     # the initial iterate's share of the step: plain extrapolation, or features,
                     # MLP inference, assembly and the residual judge (synchronised)
                     "guess_s_per_step": float(np.mean([r[5] for r in allr])) if allr else None,
                     "seeds_failed": [s for s in seeds if recs[mode][s][1]],
                     # a tangled stage state gives a non-finite initial residual
                     "median_initial_residual_ratio": float(np.median(finite)) if finite else None,
                     "non_finite_initial_residuals": len(ginit) - len(finite)}
        if log:
            log("%s: %s" % (mode, out[mode]))
    for other in ("plain", "plain_fallback", "zero"):
        m = {s: min(len(recs["learned"][s][0]), len(recs[other][s][0])) for s in seeds}
        a = [r for s in seeds for r in recs["learned"][s][0][:m[s]]]
        b = [r for s in seeds for r in recs[other][s][0][:m[s]]]
        if not a:
            continue
        out["learned_vs_" + other] = {
            "matched_steps": len(a),
            "s_per_step_learned": float(np.mean([r[0] for r in a])), "s_per_step_" + other: float(np.mean([r[0] for r in b])),
            "newton_learned": float(np.mean([r[1] for r in a])), "newton_" + other: float(np.mean([r[1] for r in b])),
            "gmres_learned": float(np.mean([r[2] for r in a])), "gmres_" + other: float(np.mean([r[2] for r in b])),
            "speedup_s_per_step": float(np.mean([r[0] for r in b]) / np.mean([r[0] for r in a]))}
    out["steps_per_seed"] = steps
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train", "eval", "probe", "mlpbench"])
    ap.add_argument("--nx", type=int, default=112)
    ap.add_argument("--ny", type=int, default=48)
    ap.add_argument("--order", type=int, default=3)
    ap.add_argument("--runs", type=int, default=200)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--cfl-factor", type=float, default=8.0)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--hidden", type=int, default=128)
    ap.add_argument("--model", default=DEFAULT_MODEL)
    ap.add_argument("--out", default=DEFAULT_MODEL)
    ap.add_argument("--eval-seeds", default="1000-1009")
    ap.add_argument("--report", default="")
    ap.add_argument("--zero-guess", action="store_true")
    ap.add_argument("--dscale", choices=["formula", "const"], default="formula")
    ap.add_argument("--pcg-iters", type=int, default=0)
    ap.add_argument("--prec-probe", type=int, default=2,
                    help="block preconditioner: 0 masses, 1/2 probed diagonal Jacobian blocks")
    ap.add_argument("--prec-lag", type=int, default=1, help="rebuild probed blocks once per stage solve")
    a = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)
    VISC["mode"] = a.dscale
    opts = newton_options(tol=1e-10, jvp_prec=32, max_newton=30, restart=15, gmres_maxit=150,
                          pcg_iters=a.pcg_iters, prec_probe=a.prec_probe, prec_lag=a.prec_lag)
    lo, hi = [int(v) for v in a.eval_seeds.split("-")]
    eval_seeds = list(range(lo, hi + 1))
    if a.cmd == "mlpbench":
        # the MLP kernels alone, for counter and timing passes: two epochs of training on 32,768
        # random samples (batch 4,096) and three learned guesses of the triple point (5,376 elements)
        z = np.load(a.model)
        widths = [int(w) for w in z["widths"]]
        h = make_triple(a.nx, a.ny, a.order, seed=1000)
        m = GuessMLP(h, widths, seed=0)
        g = torch.Generator(device=h.device).manual_seed(0)
        X = torch.randn(32768, pad32(widths[0]), device=h.device, generator=g)
        T = torch.randn(32768, pad32(widths[-1]), device=h.device, generator=g)
        t0 = time.time()
        train(m, X, T, 2, 4096, 1e-3)
        torch.cuda.synchronize()
        log("training: 2 epochs x 8 batches of 4096 in %.3f s" % (time.time() - t0))
        scales = dict(zip(("vs", "es", "xs", "kvs", "kes"), z["scales"].tolist()))
        m2 = GuessMLP(h, widths)
        m2.load_state({k: z[k] for k in ("widths", "master")})
        lg = LearnedGuess(h, m2, scales, norm={k: z[k] for k in ("mu", "sd", "osc")})
        u = h.init_state()
        dt = a.cfl_factor * h.dt_estimate(u, 0.5)
        for _ in range(3):
            lg.guess(u, [], 0.5 * dt)
        base = h.plain_guess(u, [], 0.5 * dt)
        for _ in range(3):  # the same network output through the features and layer-by-layer kernels
            lg.predict_layered(u, base)
        torch.cuda.synchronize()
        log("inference: 3 learned guesses (fused network launch) and 3 layer-by-layer forwards on %d elements"
            % h.Ne)
        return
    if a.cmd == "probe":
        h = make_triple(a.nx, a.ny, a.order, seed=None)
        u = h.init_state()
        dt = a.cfl_factor * h.dt_estimate(u, 0.5)
        log("dt %.4g" % dt)
        t0 = time.time()
        if a.zero_guess:
            st = []
            for i in range(a.steps):
                k_, s_ = h.implicit_step(u, dt, guess=None, opts=opts, raise_on_fail=False)
                st.append(s_)
                if s_["status"]:
                    break
        else:
            st = run_plain(h, u, dt, a.steps, opts)
        for i, s in enumerate(st):
            log("step %d status %d newton %d gmres %d res %.2e hist %s" % (
                i, s["status"], s["newton"], s["gmres"], s["res_final"] / max(s["res0"], 1e-300),
                " ".join("%.1e" % v for v in s["hist"][:12])))
        log("%.3f s/step" % ((time.time() - t0) / max(len(st), 1)))
        return 0
    if a.cmd == "train":
        t0 = time.time()
        X, T, scales = generate(a.nx, a.ny, a.order, range(a.runs), a.steps, a.cfl_factor, opts, log=log)
        log("dataset %s in %.1fs" % (tuple(X.shape), time.time() - t0))
        nout = 2 * (a.order + 1) ** 2 + a.order ** 2
        nin = 2 * nout + 8
        widths = [nin, a.hidden, a.hidden, a.hidden, nout]
        norm = column_stats(X, T, nin, nout)
        X = (X - norm["mu"]) / norm["sd"]
        X[:, nin:] = 0.0
        T = T / norm["osc"]
        h = make_triple(a.nx, a.ny, a.order)
        mlp = GuessMLP(h, widths, seed=0)
        t1 = time.time()
        hist = train(mlp, X, T, a.epochs, a.batch, a.lr, log=log)
        log("trained in %.1fs" % (time.time() - t1))
        st = mlp.state()
        st.update({k: v.cpu().numpy() for k, v in norm.items()})
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        np.savez(a.out, widths=st["widths"], master=st["master"], mu=st["mu"], sd=st["sd"], osc=st["osc"],
                 scales=np.array([scales[k] for k in ("vs", "es", "xs", "kvs", "kes")]),
                 loss=np.array(hist), cfl_factor=np.array(a.cfl_factor), runs=np.array(a.runs),
                 steps=np.array(a.steps), prec_probe=np.array(a.prec_probe), prec_lag=np.array(a.prec_lag))
        log("saved %s" % a.out)
        del X, T
        res = evaluate(a.nx, a.ny, a.order, eval_seeds, a.steps, a.cfl_factor, opts, st, scales, log=log)
        if a.report:
            json.dump({"train_loss": hist, "eval": res, "runs": a.runs, "steps": a.steps}, open(a.report, "w"))
        return 0
    if a.cmd == "eval":
        z = np.load(a.model)
        scales = dict(zip(("vs", "es", "xs", "kvs", "kes"), z["scales"].tolist()))
        res = evaluate(a.nx, a.ny, a.order, eval_seeds, a.steps, a.cfl_factor, opts,
                       {k: z[k] for k in ("widths", "master", "mu", "sd", "osc")}, scales, log=log)
        if a.report:
            json.dump(res, open(a.report, "w"))
        return 0


if __name__ == "__main__":
    sys.exit(main())

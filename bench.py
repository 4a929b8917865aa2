#!/usr/bin/env python3
"""Benchmark of the implicit Lagrangian hydrodynamics hot path on one MI355X.

Workload (default): 2D Taylor-Green vortex on [0,1]^2, 128 x 128 quadrilaterals, Q3Q2
(36 quadrature points per element, 589,824 in total), gamma 5/3, no viscosity, implicit
midpoint steps at 4x the explicit CFL-0.5 time step, FP64 residual / mass solves / Newton
test, FP32 Jacobian actions inside FGMRES, Newton tolerance 1e-10.

A timed "step" is one implicit midpoint step: plain initial iterate, then Newton-FGMRES
(residual, Jacobian actions, mass preconditioner, detJ line search) and the update.

Printed JSON line:
  value       Jacobian-action throughput in quadrature points per second: N_qp times the
              number of FP32 Jacobian actions inside the timed steps, divided by their summed
              kernel time plus that of the linearisation launches they used (HIP events
              attached by the library to each dispatch on its stream);
  ms_per_step wall time per implicit step (host synchronised at both ends);
  roofline    algorithmic bytes of one Jacobian-action (apply) launch -- the state, the direction
              and the result (three block vectors) and m_q per point, 19 B per quadrature point in
              FP32 -- over its mean launch time, vs 8 TB/s; design_bytes / bandwidth_frac count
              what this implementation moves instead (its stored tangent coefficients included);
              traffic = counter-measured bytes per launch, and valu = counted VALU instructions
              per launch with the fraction of the issue peak they occupy at the measured launch
              time, when recorded for the current kernel sources;
  cpu_baseline the CPU oracle's complex-step Jacobian action at C2 on all cores of the CPU share
              (cpu_oracle: 1 core and all cores, residual and Jacobian actions, C1-C4 and R-A).
Run with --gpus N, N > 1: exits, this build runs on one GPU only.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0

# HBM traffic of one FP32 Jacobian-action launch (FP32 output: the FP32 Krylov basis) at 128x128
# Q3Q2 without viscosity, from two
# rocprofv3 counter passes (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what
# the same counter reads for a copy-shaped kernel of known size (--copy-probe-mib).  The record
# holds only while the kernel sources hash to the value it was taken with; otherwise traffic is
# reported as null.
# The kernel's sources: its file, the headers of its device code, and of the internal header the
# part the device code sees (kernel parameters, tables, wall test: everything before the host-side
# context struct, whose later declarations do not change the kernel).
TRAFFIC_SOURCES = ("paper_2609_16424_amd/csrc/ilh_jvplin2d.hip", "paper_2609_16424_amd/csrc/ilh_lin.h",
                   "paper_2609_16424_amd/csrc/ilh_pointwise.h", "paper_2609_16424_amd/csrc/ilh_internal.h")
TRAFFIC_SOURCE_END = {"paper_2609_16424_amd/csrc/ilh_internal.h": b"struct ilh_ctx {"}
TRAFFIC_RECORD = {"sha256": "27386b64d2e5349a588d80bf98687b40352c5154e35d5c37b3c61c3dacac98fb",
                  "variant": "lin", "n": 128, "order": 3,
                  "fetch_kib": 16609.3, "fetch_scale": 262144.0 / 131080.04,
                  "write_kib": 3704.6, "write_scale": 262144.0 / 262144.0}


def sources_sha256():
    h = hashlib.sha256()
    root = os.path.dirname(os.path.abspath(__file__))
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(root, rel), "rb") as f:
            data = f.read()
        end = TRAFFIC_SOURCE_END.get(rel)
        if end is not None:
            data = data[:data.index(end)]
        h.update(data)
    return h.hexdigest()


# VALU instructions per launch of the same kernel (rocprofv3 --pmc SQ_INSTS_VALU, same sources):
# the issue peak of wave64 FP32 (unpacked) / FP64 VALU instructions is 1024 SIMDs x 2.4 GHz / 4.
VALU_RECORD = {"sha256": TRAFFIC_RECORD["sha256"], "variant": "lin", "n": 128, "order": 3,
               "instructions": 2137047.3}
VALU_ISSUE_PEAK = 1024 * 2.4e9 / 4


def recorded_valu(n, k, variant, launch_s):
    r = VALU_RECORD
    if variant != r["variant"] or (n, k) != (r["n"], r["order"]) or sources_sha256() != r["sha256"]:
        return None
    return {"instructions_per_launch": r["instructions"], "issue_peak_per_s": VALU_ISSUE_PEAK,
            "busy": r["instructions"] / (launch_s * VALU_ISSUE_PEAK)}


def recorded_traffic(n, k, variant):
    r = TRAFFIC_RECORD
    if variant != r["variant"] or r["sha256"] is None or (n, k) != (r["n"], r["order"]) or sources_sha256() != r["sha256"]:
        return None
    return 1024.0 * (r["fetch_kib"] * r["fetch_scale"] + r["write_kib"] * r["write_scale"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=128, help="elements per side")
    ap.add_argument("--order", type=int, default=3)
    ap.add_argument("--cfl-factor", type=float, default=4.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-ra", action="store_true",
                    help="add the 1024^2 Q3Q2 shape to the CPU oracle legs (about 2-3 minutes more)")
    ap.add_argument("--no-fp64-leg", action="store_true")
    ap.add_argument("--jvp-variant", choices=("lin", "generic", "recompute"), default="lin",
                    help="Jacobian-action kernels: linearised (stored tangent coefficients), generic element "
                         "kernel, or register-resident recompute kernel")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--learned-seeds", default="1000-1004")
    ap.add_argument("--learned-steps", type=int, default=30)
    ap.add_argument("--no-c4", action="store_true", help="skip the triple-point precision and step-control legs")
    ap.add_argument("--no-sedov", action="store_true", help="skip the Sedov explicit-vs-implicit leg")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a copy-shaped elementwise kernel (dst = -src) over this many MiB three "
                         "times: the byte calibration for HBM traffic counters")
    ap.add_argument("--roofline-shape", type=int, default=1024,
                    help="also time the JVP on an n x n Q3Q2 state of this size (0 = off)")
    ap.add_argument("--roofline-shape-3d", type=int, default=128,
                    help="also time the JVP on an n^3 Q2Q1 3D Taylor-Green state of this size (0 = off)")
    return ap.parse_args()


def n_coef(H):
    """Stored tangent coefficients per quadrature point of the linearised kernels: J^-1 and
    grad_xi v J^-1 (2 d^2), P and dP/de (or the viscous stress, m_q nu and three coefficients
    of d nu), m_q grad s with the TG source (d)."""
    d = H.dim
    return 2 * d * d + (d * (d + 1) // 2 + 5 if H.setup.visc_on else 2) + (d if H.setup.tg_source else 0)


def jvp_bytes(H, prec, variant="lin"):
    """Algorithmic HBM bytes of one Jacobian-action launch: every array read or written once.

    lin:       direction dk and output J dk, the stored tangent coefficients (n_coef per point)
               and the per-element rho0 |J0| (quadrature-mass factor).
    recompute: state x (FP64), v and e (FP32 shadow, or FP64), dk, J dk and per-element
               rho0 |J0|, |J0| and gamma (affine initial mesh).
    generic:   as recompute, with per-point m_q instead of the per-element factors.
    """
    w = 4 if prec == 32 else 8
    vec = H.nblock * w
    if variant == "lin":
        return 2 * vec + n_coef(H) * H.nqp * w + H.Ne * 8
    state = H.nh1 * 8 + (H.nh1 + H.nl2) * w
    qdata = H.nqp * 8 + H.Ne * 8 if variant == "generic" else 3 * H.Ne * 8
    return state + 2 * vec + qdata


def alg_bytes(H, prec):
    """Algorithmic HBM bytes of one Jacobian action (or residual) by the method's own count: the
    unique vectors it touches once each -- the state w, the direction dk and the result (three
    block vectors) -- and the quadrature mass m_q per point (+ det J0 per point with viscosity);
    nothing the implementation chooses to store (tangent coefficients) is counted.  2D Q3Q2:
    19 (FP32) / 38 (FP64) bytes per point; 3D Q2Q1: 14.6 / 29.1."""
    w = 4 if prec == 32 else 8
    return 3 * H.nblock * w + H.nqp * w * (2 if H.setup.visc_on else 1)


def lin_bytes(H, prec):
    """Algorithmic bytes of one linearisation launch: state w (FP64) read, coefficients written,
    per-element rho0 |J0|, |J0|, gamma read."""
    return H.nblock * 8 + n_coef(H) * H.nqp * (4 if prec == 32 else 8) + 3 * H.Ne * 8


def res_bytes(H):
    """Algorithmic bytes of one stage-residual launch: u and k read, R written (FP64 block
    vectors), per-element rho0 |J0|, |J0| and gamma read (strip kernels)."""
    return 3 * H.nblock * 8 + 3 * H.Ne * 8


def residual_rate(H, k, u, tau, launches):
    """Mean launch time of the stage residual (library kernel events) -> dict."""
    r = H.new()
    for _ in range(2):
        H.residual(k, u, tau, out=r)
    H.timing(True)
    for _ in range(launches):
        H.residual(k, u, tau, out=r)
    t = H.timing_read()
    H.timing(False)
    avg = 1e-3 * t["residual"][0] / max(t["residual"][1], 1)
    b = alg_bytes(H, 64)
    bd = res_bytes(H)
    return {"avg_launch_us": 1e6 * avg, "qps": H.nqp / avg, "bytes_per_launch": b,
            "achieved_GBs": b / avg / 1e9, "frac": b / avg / 1e9 / HBM_PEAK_GBS,
            "design_bytes_per_launch": bd, "bandwidth_frac": bd / avg / 1e9 / HBM_PEAK_GBS}


KERNEL_NAMES = {"lin": "k_jvp2d_q<4,6,float,visc=0,src=1,out=float,waves=1>", "generic": "k_elem2d<4,6,JVP,float,7>",
                "recompute": "k_jvp2d<4,6,float,visc=0,src=1>"}


def run_steps(H, u, dt, nsteps, opts, hist, ilh):
    stats = []
    for _ in range(nsteps):
        g = H.plain_guess(u, hist, 0.5 * dt)
        k, st = H.implicit_step(u, dt, guess=g, opts=opts)
        hist.append(k)
        if len(hist) > 2:
            hist.pop(0)
        stats.append(st)
    return stats


def triple_point_legs(ilh, torch):
    """C4 (triple point 112x48 Q3Q2, smoothed viscosity): (i) 8 fixed steps at 8x the explicit
    step with FP32 and with FP64 Jacobian actions, probed block preconditioner (Newton and GMRES
    counts, state difference);
    (ii) the Newton-based step-size control of Sec. 4 started from 8x the explicit step, SD2,
    10 accepted steps."""
    from paper_2609_16424_amd import learned as L
    res = {}
    states = {}
    for prec in (32, 64):
        h = L.make_triple(112, 48, 3)
        u = h.init_state()
        dt = 8.0 * h.dt_estimate(u, 0.5)
        opts = ilh.newton_options(tol=1e-10, jvp_prec=prec, max_newton=30, restart=15, gmres_maxit=150,
                                  prec_probe=2, prec_lag=1)
        hist, newton, gmres = [], [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(8):
            g = h.plain_guess(u, hist, 0.5 * dt)
            k, st = h.implicit_step(u, dt, guess=g, opts=opts)
            hist = (hist + [k])[-2:]
            newton.append(st["newton"])
            gmres.append(st["gmres"])
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / 8
        states[prec] = u.clone()
        # one more step with kernel events: the Jacobian action on the shocked state
        h.timing(True)
        g = h.plain_guess(u, hist, 0.5 * dt)
        h.implicit_step(u, dt, guess=g, opts=opts)
        tm = h.timing_read()
        h.timing(False)
        jms, jn = tm["jvp"]
        res["fixed_8x_fp%d" % prec] = {"newton_per_step": float(np.mean(newton)), "gmres_per_step": float(np.mean(gmres)),
                                       "s_per_step": el,
                                       "jvp_qps_shocked_state": h.nqp * jn / (1e-3 * (jms + tm["linearize"][0])),
                                       "jvp_apply_avg_us": 1e3 * jms / max(jn, 1)}
    res["fixed_8x_rel_state_diff_fp32_vs_fp64"] = float(torch.linalg.norm(states[32] - states[64]) /
                                                         torch.linalg.norm(states[64]))
    h = L.make_triple(112, 48, 3)
    u = h.init_state()
    dt_exp = h.dt_estimate(u, 0.5)
    dt = 8.0 * dt_exp
    opts = ilh.newton_options(tol=1e-10, jvp_prec=32, max_newton=30, restart=15, gmres_maxit=150)
    hist, rej, ratios, newton = [], [], [], []
    for _ in range(10):
        g = h.plain_guess(u, hist, 0.5 * dt)
        k, st, taken, dt, nrej = h.adaptive_step(u, dt, 10.0, "sd2", guess=g, opts=opts, max_reject=40)
        hist = (hist + [k])[-2:]
        rej.append(nrej)
        ratios.append(taken / dt_exp)
        newton.append(st["newton_max"])
    res["step_control_from_8x"] = {"rejected_trials": rej, "accepted_dt_over_explicit": ratios[-1],
                                   "newton_per_step": float(np.mean(newton))}
    return res


def c1_leg(ilh, torch):
    """M1: the C1 configuration (2D TG 8x8 Q2Q1, 10 implicit midpoint steps, dt 0.01, tol 1e-10) on the
    GPU, FP64 and FP32 Jacobian actions: s/step (latency-bound at 1,024 quadrature points)."""
    out = {}
    for prec in (64, 32):
        H = ilh.Hydro("tg2d", (8, 8), 2)
        u = H.init_state()
        opts = ilh.newton_options(tol=1e-10, jvp_prec=prec)
        e0 = sum(H.energy(u))
        hist, newton, gmres = [], [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            g = H.plain_guess(u, hist)
            kk, st = H.implicit_step(u, 0.01, guess=g, opts=opts)
            hist = (hist + [kk])[-2:]
            newton.append(st["newton"])
            gmres.append(st["gmres"])
        torch.cuda.synchronize()
        out["fp%d" % prec] = {"s_per_step": (time.perf_counter() - t0) / 10, "newton_per_step": float(np.mean(newton)),
                              "gmres_per_step": float(np.mean(gmres)),
                              "rel_energy_change": (sum(H.energy(u)) - e0) / e0}
    out["workload"] = "C1: 2D Taylor-Green 8x8 Q2Q1, 10 implicit midpoint steps, dt 0.01, Newton tol 1e-10"
    return out


def oracle_step_estimate(cpu, name, newton, gmres):
    """Oracle s/implicit step from its measured per-point rates and the iteration counts of the run:
    (Newton + 1) residuals and one complex-step action per GMRES iteration (the mass solves of its
    preconditioner and the orthogonalisation are left out, so this is a lower bound)."""
    e = cpu["shapes"][name]
    nqp = e["n_qp"]
    res = {}
    for tag in ("1core", "all_cores"):
        res["s_per_step_" + tag] = ((newton + 1) * nqp / e["residual"]["qps_" + tag] +
                                    gmres * nqp / e["jvp_cs"]["qps_" + tag])
    res.update(newton_per_step=newton, gmres_per_step=gmres,
               how="estimate: (Newton + 1) x residual + GMRES x complex-step action at the measured rates")
    return res


def c4_configured_width_leg(ilh, torch, steps=20, widths=(1e-1, 3e-2, 1e-2, 3e-3)):
    """C4 as configured: the triple point 112x48 Q3Q2 at 8x the explicit step with the smoothing
    width delta_scale = 1e-3 (constant), FP32 Jacobian actions, probed block preconditioner.
    (i) direct: each step solved at width 1e-3 from the plain iterate, until the first failure;
    (ii) continuation in the width within each step: stage solves at the wider scales `widths`,
    each from the previous one's solution, then the step at 1e-3 from that iterate.
    Per step: status, Newton and GMRES iterations, line-search halvings, residual history."""
    from paper_2609_16424_amd import learned as L
    out = {"workload": "2D triple point 112x48 Q3Q2, delta_scale = 1e-3 (constant), 8x explicit CFL, "
                       "FP32 Jacobian actions, tol 1e-10, probed block preconditioner (mode 2, lag 1)"}
    for mode in ("direct", "continuation"):
        H = L.make_triple(112, 48, 3)
        H.set_viscosity_scale("const", 1e-3)
        u = H.init_state()
        dt = 8.0 * H.dt_estimate(u, 0.5)
        opts = ilh.newton_options(tol=1e-10, jvp_prec=32, max_newton=30, restart=15, gmres_maxit=150,
                                  prec_probe=2, prec_lag=1)
        hist, recs = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ok_steps = 0
        for n in range(steps):
            g = H.plain_guess(u, hist, 0.5 * dt)
            cont = []
            if mode == "continuation":
                for w in widths:
                    H.set_viscosity_scale("const", w)
                    kc, stc = H.stage_solve(u, 0.5 * dt, guess=g, opts=opts)
                    cont.append([w, stc["status"], stc["newton"]])
                    if stc["status"] == 0:
                        g = kc
                H.set_viscosity_scale("const", 1e-3)
            k, st = H.implicit_step(u, dt, guess=g, opts=opts, raise_on_fail=False)
            recs.append({"status": st["status"], "newton": st["newton"], "gmres": st["gmres"],
                         "halvings": st["halvings"], "res_hist": [float("%.3e" % x) for x in st["hist"][:12]]})
            if cont:
                recs[-1]["continuation"] = cont
            if st["status"] != 0:
                break
            ok_steps += 1
            hist = (hist + [k])[-2:]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[mode] = {"steps_converged": ok_steps, "steps_tried": len(recs),
                     "s_per_step": el / max(1, len(recs)), "per_step": recs}
        del H, u
    # (iii) the paper's Newton-based step control (Sec. 4) from 8x at width 1e-3: how far the step
    # has to shrink for Newton to converge within three iterations
    H = L.make_triple(112, 48, 3)
    H.set_viscosity_scale("const", 1e-3)
    u = H.init_state()
    dt_exp = H.dt_estimate(u, 0.5)
    dt = 8.0 * dt_exp
    opts = ilh.newton_options(tol=1e-10, jvp_prec=32, max_newton=30, restart=15, gmres_maxit=150,
                              prec_probe=2, prec_lag=1)
    hist, ratios, rej = [], [], []
    try:
        for _ in range(10):
            g = H.plain_guess(u, hist, 0.5 * dt)
            k, st, taken, dt, nrej = H.adaptive_step(u, dt, 10.0, "sd2", guess=g, opts=opts, max_reject=40)
            hist = (hist + [k])[-2:]
            ratios.append(taken / dt_exp)
            rej.append(nrej)
        out["step_control_from_8x"] = {"accepted_dt_over_explicit": ratios, "rejected_trials": rej}
    except Exception as e:  # the control gives up after max_reject trials
        out["step_control_from_8x"] = {"accepted_dt_over_explicit": ratios, "rejected_trials": rej,
                                       "failure": str(e)}
    return out


def _peak_density_radius(H, u):
    """Radius of the element with the largest mass / area (area from its boundary nodes)."""
    n, k = H.n[0], H.k
    x = u[:H.nh1].view(2, -1).cpu().numpy()
    ng = k * n + 1
    X, Y = x[0].reshape(ng, ng), x[1].reshape(ng, ng)
    best = (0.0, 0.0)
    for ey in range(n):
        for ex in range(n):
            idx = ([(ex * k + a, ey * k) for a in range(k)] + [(ex * k + k, ey * k + b) for b in range(k)] +
                   [(ex * k + k - a, ey * k + k) for a in range(k)] + [(ex * k, ey * k + k - b) for b in range(k)])
            px = np.array([X[j, i] for i, j in idx])
            py = np.array([Y[j, i] for i, j in idx])
            area = 0.5 * abs(np.dot(px, np.roll(py, -1)) - np.dot(py, np.roll(px, -1)))
            rho = (1.0 / (n * n)) / area
            if rho > best[0]:
                best = (rho, float(np.hypot(px.mean(), py.mean())))
    return best


def sedov_leg(ilh, torch, n=16, k=3, T=0.8):
    """2D Sedov blast (Sec. 4.2), n x n Q3Q2, to T = 0.8: the explicit RK2-average scheme at
    CFL 0.5 against implicit midpoint at FS-CFL 2 (dt = 2 x the explicit estimate, each step),
    wall time, steps, energy, shock position (radius of the densest element; the exact
    self-similar shock is at 0.898)."""
    out = {}
    for mode in ("explicit_rk2_cfl0.5", "implicit_midpoint_fscfl2"):
        H = ilh.make_sedov(n, k)
        u = H.init_state()
        e0 = sum(H.energy(u))
        opts = ilh.newton_options(tol=1e-10, jvp_prec=32, max_newton=30, restart=15, gmres_maxit=150,
                                  prec_probe=2, prec_lag=1)
        t, steps, hist, newton, gmres = 0.0, 0, [], 0, 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while t < T - 1e-12:
            if mode.startswith("explicit"):
                dt = min(0.5 * H.dt_estimate(u, 1.0), T - t)
                H.rk2avg_step(u, dt)
            else:
                dt = min(2.0 * H.dt_estimate(u, 1.0), T - t)
                g = H.plain_guess(u, hist, 0.5 * dt)
                kk, st = H.implicit_step(u, dt, guess=g, opts=opts)
                hist = (hist + [kk])[-2:]
                newton += st["newton"]
                gmres += st["gmres"]
            t += dt
            steps += 1
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        peak, r = _peak_density_radius(H, u)
        entry = {"steps": steps, "wall_s": wall, "s_per_step": wall / steps,
                 "rel_energy_change": (sum(H.energy(u)) - e0) / e0, "peak_density": peak, "peak_radius": r}
        if newton:
            entry.update(newton_per_step=newton / steps, gmres_per_step=gmres / steps)
        out[mode] = entry
        del H, u
    # the paper's step control from FS-CFL 2 with its default solver settings (Newton relative
    # tolerance 1e-5, at most 10 iterations, linear solves to 1e-12, zero initial iterate)
    H = ilh.make_sedov(n, k)
    u = H.init_state()
    e0 = sum(H.energy(u))
    opts = ilh.newton_options(tol=1e-5, max_newton=10, restart=30, gmres_rtol=1e-12, gmres_maxit=400,
                              jvp_prec=64, ls_residual=0, guess_fallback=0, prec_probe=2, prec_lag=1)
    t, steps, rej = 0.0, 0, 0
    dt = H.dt_estimate(u, 2.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    try:
        while t < T - 1e-12:
            _, st, taken, dt, nrej = H.adaptive_step(u, dt, T - t, "sd2", guess=None, opts=opts, max_reject=60)
            t += taken
            steps += 1
            rej += nrej
        torch.cuda.synchronize()
        peak, r = _peak_density_radius(H, u)
        out["implicit_step_control_paper_settings"] = {
            "steps": steps, "rejected": rej, "wall_s": time.perf_counter() - t0,
            "rel_energy_change": (sum(H.energy(u)) - e0) / e0, "peak_radius": r,
            "paper_implicit_steps": 205}
    except Exception as e:
        out["implicit_step_control_paper_settings"] = {"steps": steps, "rejected": rej, "failure": str(e)}
    del H, u
    out["implicit_speedup_wall"] = out["explicit_rk2_cfl0.5"]["wall_s"] / out["implicit_midpoint_fscfl2"]["wall_s"]
    out["workload"] = "2D Sedov %dx%d Q%dQ%d, gamma 1.4, smoothed viscosity, T = %g; exact shock radius 0.898" % (
        n, n, k, k - 1, T)
    return out


# ---------------------------------------------------------------------------------------------
# CPU oracle baseline.  Runs first, before the GPU is initialised, so that the worker processes are
# forked from a process without a GPU context.  Every figure times the oracle as it stands (plain
# NumPy FP64 / complex128): its element force evaluation (oracle.hydro.Hydro.force on a chunk of
# elements, the whole per-element work of a residual or Jacobian action) on a bounded sample of
# each workload, on one core and on all cores of the CPU share (one process per core, BLAS
# threads 1, each process a different chunk of the same size: weak scaling), plus full implicit
# steps of the oracle at C1.
_CPU = {}


def _cpu_worker(args):
    """Time one oracle operation on one element chunk (runs in a forked worker or inline)."""
    from threadpoolctl import threadpool_limits
    op, lo, hi = args
    O, w, dk, tau = _CPU["O"], _CPU["w"], _CPU["dk"], _CPU["tau"]
    els = np.arange(lo, hi)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        if op == "residual":
            O.force(w, elements=els)
        elif op == "jvp_cs":
            O.force(w + 1j * 1e-30 * tau * dk, elements=els)
        else:  # two-residual central difference
            O.force(w + 1e-7 * tau * dk, elements=els)
            O.force(w - 1e-7 * tau * dk, elements=els)
        return time.perf_counter() - t0


def _cpu_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        share = len(os.sched_getaffinity(0))
    except AttributeError:
        share = os.cpu_count() or 1
    return model, os.cpu_count(), share


def cpu_legs(with_ra=False, target_s=0.7):
    """The oracle on the host CPU: qp/s of its residual force kernel and of its Jacobian action
    (complex step; two-residual central difference) at the C1-C4 shapes (and R-A with with_ra),
    1 core and all cores; oracle s/implicit step at C1 (10 steps, dt 0.01, tol 1e-10)."""
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    from oracle.hydro import Hydro as OHydro, ViscosityOptions
    from oracle import krylov
    import seeded_inputs as si
    model, nproc, share = _cpu_info()
    workers = max(1, min(16, share))  # the machine's CPU share for one GPU is 16 cores
    shapes = [("C1", "tg2d", (8, 8), 2, None), ("C2", "tg2d", (128, 128), 3, None),
              ("C3", "tg3d", (32, 32, 32), 2, None), ("C4", "triple", (112, 48), 3, "formula")]
    if with_ra:
        # 1024^2: building the oracle takes ~40 s and each subset evaluation gathers the whole
        # mesh (~1 s per call), so the sample takes larger chunks there
        shapes.append(("R-A", "tg2d", (1024, 1024), 3, None))
    out = {"cpu_model": model, "nproc": nproc, "cpu_share": share, "workers": workers, "shapes": {}}
    t_all = time.perf_counter()
    for name, prob, n, k, visc in shapes:
        tb = time.perf_counter()
        vo = ViscosityOptions(on=visc is not None, mode=visc or "const", h_coarse=(1.0 / k if prob == "triple" else None))
        with threadpool_limits(1):
            O = OHydro(prob, n, k, visc=vo)
            u = O.init_state()
        build_s = time.perf_counter() - tb
        h = float(np.min(O.mesh.h)) / k
        w = si.perturb_state(u, 3, O.nh1, 0.02 * h, 0.02, 0.01) if prob != "tg3d" else si.displace_positions(u, O.nh1, 0.05)
        dk = si.block_direction(4, O.nh1, O.nl2, h, 1.0, 1.0)
        _CPU.update(O=O, w=w, dk=dk, tau=0.5 * O.dt_estimate(w, 2.0))
        entry = {"n_elements": O.mesh.Ne, "n_qp": O.mesh.Ne * O.Q, "oracle_build_s": build_s}
        Q = O.Q
        for op in ("residual", "jvp_cs", "jvp_fd"):
            # chunk sized for about target_s of one core's work (at most the whole mesh): the
            # oracle's subset evaluation gathers the whole mesh first, so a call costs a + b ne
            m1 = min(O.mesh.Ne, 128)
            m2 = min(O.mesh.Ne, 256)
            ta = min(_cpu_worker((op, 0, m1)) for _ in range(2))
            tb_ = min(_cpu_worker((op, 0, m2)) for _ in range(2))
            slope = max((tb_ - ta) / max(m2 - m1, 1), 1e-7) if m2 > m1 else ta / m1
            tgt = target_s if name != "R-A" else 8.0
            ne = int(min(O.mesh.Ne, max(m1, (tgt - max(ta - m1 * slope, 0.0)) / slope)))
            t1 = min(_cpu_worker((op, 0, ne)) for _ in range(2))
            one = ne * Q / t1
            chunks = [(op, (i * ne) % max(1, O.mesh.Ne - ne + 1), (i * ne) % max(1, O.mesh.Ne - ne + 1) + ne)
                      for i in range(workers)]
            ctx = mp.get_context("fork")
            with ctx.Pool(workers) as pool:
                pool.map(_cpu_worker, chunks[:workers])  # warm the workers
                tw = time.perf_counter()
                pool.map(_cpu_worker, chunks)
                wall = time.perf_counter() - tw
            entry[op] = {"qps_1core": one, "qps_all_cores": workers * ne * Q / wall, "chunk_elements": ne}
        out["shapes"][name] = entry
        _CPU.clear()
        del O, u, w, dk
    # full oracle implicit steps at C1 (the oracle's Newton-FGMRES with complex-step actions)
    with threadpool_limits(1):
        O = OHydro("tg2d", (8, 8), 2)
        u0 = O.init_state()
        t0 = time.perf_counter()
        _, _, st = krylov.run_midpoint(O, u0, 0.01, 10)
        c1 = (time.perf_counter() - t0) / 10
    out["oracle_s_per_step_C1_1core"] = c1
    out["oracle_C1_newton_gmres_per_step"] = [float(np.mean([x["newton"] for x in st])),
                                              float(np.mean([x["gmres"] for x in st]))]
    out["wall_s"] = time.perf_counter() - t_all
    return out


def cpu_baseline_line(cpu):
    """The contract's cpu_baseline object: the oracle's complex-step Jacobian action at C2 on all cores."""
    e = cpu["shapes"]["C2"]["jvp_cs"]
    return {"value": e["qps_all_cores"], "unit": "quad-pts/s", "cores": cpu["workers"], "kind": "oracle",
            "sample": "oracle complex-step Jacobian action (element force in complex128) on %d processes x %d "
                      "elements of the 128x128 Q3Q2 Taylor-Green state (1 BLAS thread each); 1 core: %.3g qp/s; "
                      "CPU %s, nproc %s, CPU share %s" % (cpu["workers"], e["chunk_elements"], e["qps_1core"],
                                                          cpu["cpu_model"], cpu["nproc"], cpu["cpu_share"])}


def _finite(v):
    """JSON has no NaN or infinity: a non-finite figure is reported as null."""
    if isinstance(v, dict):
        return {k: _finite(x) for k, x in v.items()}
    if isinstance(v, (list, tuple)):
        return [_finite(x) for x in v]
    if isinstance(v, float) and not np.isfinite(v):
        return None
    return v


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on exactly one GPU (no sharding or collectives); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_legs(with_ra=args.cpu_ra)  # before the GPU is initialised (forked workers)
    import torch
    import paper_2609_16424_amd as ilh

    n, k = args.n, args.order
    H = ilh.Hydro("tg2d", (n, n), k)
    H.set_kernel_variant(args.jvp_variant)
    u0 = H.init_state()
    dt = args.cfl_factor * H.dt_estimate(u0, 0.5)
    opts32 = ilh.newton_options(tol=1e-10, jvp_prec=32)
    opts64 = ilh.newton_options(tol=1e-10, jvp_prec=64)

    # warm-up from the initial state
    u = u0.clone()
    hist = []
    run_steps(H, u, dt, args.warmup, opts32, hist, ilh)
    u_start = u.clone()
    hist_start = [h.clone() for h in hist]
    torch.cuda.synchronize()

    # timed FP32-JVP leg (no per-kernel events)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = run_steps(H, u, dt, args.steps, opts32, hist, ilh)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = 1e3 * (t1 - t0) / args.steps
    # the same steps again with kernel events (kernel-by-kernel launches) for the per-kernel times
    u_ev, hist_ev = u_start.clone(), [h.clone() for h in hist_start]
    H.timing(True)
    torch.cuda.synchronize()
    t0e = time.perf_counter()
    run_steps(H, u_ev, dt, args.steps, opts32, hist_ev, ilh)
    torch.cuda.synchronize()
    t1e = time.perf_counter()
    tim = H.timing_read()
    H.timing(False)
    ms_per_step_events = 1e3 * (t1e - t0e) / args.steps
    jvp_ms, jvp_n = tim["jvp"]
    lin_ms, lin_n = tim["linearize"]
    jvp_avg_s = 1e-3 * jvp_ms / max(jvp_n, 1)
    # Jacobian actions per second of kernel time, the linearisation launches charged to them
    value = H.nqp * jvp_n / (1e-3 * (jvp_ms + lin_ms))
    bytes32 = jvp_bytes(H, 32, args.jvp_variant)
    # inside FGMRES the linearised FP32 action writes the (FP32) Krylov basis vector itself
    bytes_loop = bytes32
    alg32 = alg_bytes(H, 32)
    achieved = alg32 / jvp_avg_s / 1e9
    # the same kernel back to back at the last linearisation point (no other kernels between)
    dkb = torch.randn(H.nblock, device=u.device, dtype=torch.float32,
                      generator=torch.Generator(device=u.device).manual_seed(7))
    outb = torch.empty_like(dkb)
    H.jvp_lin(dkb, 32, outb)
    H.timing(True)
    for _ in range(50):
        H.jvp_lin(dkb, 32, outb)
    tb_ = H.timing_read()
    H.timing(False)
    burst_us = 1e3 * tb_["jvp"][0] / max(tb_["jvp"][1], 1)
    # the transpose action J^T y at the same point, back to back (same bytes moved)
    H.vjp_lin(dkb, 32, outb)
    H.timing(True)
    for _ in range(50):
        H.vjp_lin(dkb, 32, outb)
    tv_ = H.timing_read()
    H.timing(False)
    vjp_us = 1e3 * tv_["transpose"][0] / max(tv_["transpose"][1], 1)
    # the stage residual at the last stage increment, back to back
    res_c2 = dict(residual_rate(H, hist[-1], u, 0.5 * dt, 20), kernel="k_res2d<4,6,src=1> (FP64)")
    u32 = u.clone()
    newton = [s["newton"] for s in stats]
    gmres = [s["gmres"] for s in stats]
    ke, ie = H.energy(u32)

    extra = {}
    # the same steps with both Gram-Schmidt passes inside each Arnoldi step (three basis sweeps and
    # seven launches per step, against two sweeps and four with the second pass lagged)
    u = u_start.clone()
    hist = [h.clone() for h in hist_start]
    opts_two = ilh.newton_options(tol=1e-10, jvp_prec=32, cgs2=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st_two = run_steps(H, u, dt, args.steps, opts_two, hist, ilh)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    extra["gram_schmidt"] = {
        "lagged_second_pass_ms_per_step": ms_per_step,
        "two_passes_in_step_ms_per_step": 1e3 * (t1 - t0) / args.steps,
        "gmres_per_step_lagged": float(np.mean(gmres)),
        "gmres_per_step_two_passes": float(np.mean([s["gmres"] for s in st_two])),
        "jvp_calls_per_step_lagged": float(np.mean([s["jvp_calls"] for s in stats])),
        "jvp_calls_per_step_two_passes": float(np.mean([s["jvp_calls"] for s in st_two])),
        "rel_state_diff": float(torch.linalg.norm(u - u32) / torch.linalg.norm(u32)),
    }
    if not args.no_fp64_leg:
        u = u_start.clone()
        hist = [h.clone() for h in hist_start]
        H.timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st64 = run_steps(H, u, dt, args.steps, opts64, hist, ilh)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        tim64 = H.timing_read()
        H.timing(False)
        j64_ms, j64_n = tim64["jvp"]
        l64_ms, l64_n = tim64["linearize"]
        extra["all_fp64"] = {
            "ms_per_step": 1e3 * (t1 - t0) / args.steps,
            "jvp_qps": H.nqp * j64_n / (1e-3 * (j64_ms + l64_ms)),
            "jvp_apply_avg_us": 1e3 * j64_ms / max(j64_n, 1),
            "linearize_avg_us": 1e3 * l64_ms / max(l64_n, 1),
            "newton_per_step": float(np.mean([s["newton"] for s in st64])),
            "gmres_per_step": float(np.mean([s["gmres"] for s in st64])),
            "rel_state_diff_vs_fp32_jvp": float(torch.linalg.norm(u - u32) / torch.linalg.norm(u)),
        }

    roof_extra = None
    if args.roofline_shape:
        m = args.roofline_shape
        HR = ilh.Hydro("tg2d", (m, m), 3)
        HR.set_kernel_variant(args.jvp_variant)
        uR = HR.init_state()
        uR[:HR.nh1] += 0.05 * uR[HR.nh1:2 * HR.nh1]
        kR = torch.zeros_like(uR)
        HR.linearize(kR, uR, 0.5 * HR.dt_estimate(uR, 2.0))
        dk = torch.randn(HR.nblock, device=uR.device, dtype=torch.float64,
                         generator=torch.Generator(device=uR.device).manual_seed(3))
        dk32 = dk.float()
        out32 = torch.empty_like(dk32)
        for _ in range(3):
            HR.jvp_lin(dk32, 32, out32)
        HR.timing(True)
        for _ in range(20):
            HR.jvp_lin(dk32, 32, out32)
        for _ in range(5):  # re-linearise: one linearisation launch each (linearised variant)
            HR.linearize(kR, uR, 0.5 * HR.dt_estimate(uR, 2.0))
            HR.jvp_lin(dk32, 32, out32)
        tr = HR.timing_read()
        HR.timing(False)
        avg = 1e-3 * tr["jvp"][0] / tr["jvp"][1]
        bR = jvp_bytes(HR, 32, args.jvp_variant)
        aR = alg_bytes(HR, 32)
        roof_extra = {"shape": "%dx%d Q3Q2 TG (displaced)" % (m, m), "n_qp": HR.nqp,
                      "jvp_qps": HR.nqp / avg, "achieved_GBs": aR / avg / 1e9,
                      "frac": aR / avg / 1e9 / HBM_PEAK_GBS, "bytes_per_launch": aR, "avg_launch_us": 1e6 * avg,
                      "design_bytes_per_launch": bR, "bandwidth_frac": bR / avg / 1e9 / HBM_PEAK_GBS}
        if tr["linearize"][1]:
            lavg = 1e-3 * tr["linearize"][0] / tr["linearize"][1]
            roof_extra["linearize"] = {"avg_launch_us": 1e6 * lavg, "bytes_per_launch": lin_bytes(HR, 32),
                                       "achieved_GBs": lin_bytes(HR, 32) / lavg / 1e9}
        # FP64 action at the same shape
        out64 = torch.empty_like(dk)
        for _ in range(3):
            HR.jvp_lin(dk, 64, out64)
        HR.timing(True)
        for _ in range(10):
            HR.jvp_lin(dk, 64, out64)
        t64 = HR.timing_read()
        HR.timing(False)
        a64 = 1e-3 * t64["jvp"][0] / t64["jvp"][1]
        b64 = jvp_bytes(HR, 64, args.jvp_variant)
        al64 = alg_bytes(HR, 64)
        roof_extra["fp64"] = {"avg_launch_us": 1e6 * a64, "jvp_qps": HR.nqp / a64, "bytes_per_launch": al64,
                              "achieved_GBs": al64 / a64 / 1e9, "frac": al64 / a64 / 1e9 / HBM_PEAK_GBS,
                              "design_bytes_per_launch": b64, "bandwidth_frac": b64 / a64 / 1e9 / HBM_PEAK_GBS}
        # FP32 action against FP64 on the same direction (the FP32 path rounds dk too)
        roof_extra["fp32_vs_fp64_rel_err"] = float(torch.linalg.norm(out32.double() - out64) / torch.linalg.norm(out64))
        kres = 1e-3 * dk  # a small stage increment for the residual
        roof_extra["residual"] = dict(residual_rate(HR, kres, uR, 0.5 * HR.dt_estimate(uR, 2.0), 10),
                                      kernel="k_res2d<4,6,src=1> (FP64)")
        del HR, uR, kR, dk, dk32, out32, out64, kres
        torch.cuda.empty_cache()

    roof_3d = None
    if args.roofline_shape_3d:
        roof_3d = {}
        for m, visc in ((args.roofline_shape_3d, False), (args.roofline_shape_3d, True), (32, False)):
            H3 = ilh.Hydro("tg3d", (m, m, m), 2, visc=visc, dscale_mode="formula" if visc else "const",
                           h_coarse=1.0 / 2.0)
            H3.set_kernel_variant(args.jvp_variant)
            u3 = H3.init_state()
            u3[:H3.nh1] += 0.05 * u3[H3.nh1:2 * H3.nh1]
            k3 = torch.zeros_like(u3)
            H3.linearize(k3, u3, 0.5 * H3.dt_estimate(u3, 2.0))
            entry = {"shape": "%d^3 Q2Q1 3D TG (displaced)%s" % (m, ", viscosity" if visc else ""), "n_qp": H3.nqp}
            outs3 = {}
            for prec in (32, 64):
                dt_ = torch.float32 if prec == 32 else torch.float64
                d3 = torch.randn(H3.nblock, device=u3.device, dtype=torch.float64,
                                 generator=torch.Generator(device=u3.device).manual_seed(5)).to(dt_)
                o3 = torch.empty_like(d3)
                H3.timing(True)
                for _ in range(2):
                    H3.jvp_lin(d3, prec, o3)
                tw = H3.timing_read()  # did the warm-up launch a linearisation?
                kind = "lin" if tw["linearize"][1] else "generic"
                H3.timing(True)
                for _ in range(10):
                    H3.jvp_lin(d3, prec, o3)
                t3 = H3.timing_read()
                H3.timing(False)
                a3 = 1e-3 * t3["jvp"][0] / t3["jvp"][1]
                b3 = jvp_bytes(H3, prec, kind)
                al3 = alg_bytes(H3, prec)
                outs3[prec] = o3.double().clone()
                entry["fp%d" % prec] = {"kernel_variant": kind, "avg_launch_us": 1e6 * a3, "jvp_qps": H3.nqp / a3,
                                        "bytes_per_launch": al3, "achieved_GBs": al3 / a3 / 1e9,
                                        "frac": al3 / a3 / 1e9 / HBM_PEAK_GBS,
                                        "design_bytes_per_launch": b3,
                                        "bandwidth_frac": b3 / a3 / 1e9 / HBM_PEAK_GBS,
                                        "linearize_avg_us": (1e3 * tw["linearize"][0] / tw["linearize"][1]
                                                             if tw["linearize"][1] else None)}
                del d3, o3
            entry["fp32_vs_fp64_rel_err"] = float(torch.linalg.norm(outs3[32] - outs3[64]) / torch.linalg.norm(outs3[64]))
            del outs3
            # the stage residual (FP64 strip kernel)
            k3r = 1e-3 * torch.randn(H3.nblock, device=u3.device, dtype=torch.float64,
                                     generator=torch.Generator(device=u3.device).manual_seed(6))
            entry["residual"] = dict(residual_rate(H3, k3r, u3, 0.5 * H3.dt_estimate(u3, 2.0), 5),
                                     kernel="k_res3d<3,4> (FP64)")
            del k3r
            roof_3d["%d%s" % (m, "_visc" if visc else "")] = entry
            del H3, u3, k3
            torch.cuda.empty_cache()

    learned = {}
    if not args.no_learned:
        from paper_2609_16424_amd import learned as L
        lo, hi = [int(v) for v in args.learned_seeds.split("-")]
        for key, path in (("learned_guess_c5", L.DEFAULT_MODEL), ("learned_guess_c5_4x", L.MODEL_4X)):
            if not os.path.exists(path):
                continue
            z = np.load(path)
            scales = dict(zip(("vs", "es", "xs", "kvs", "kes"), z["scales"].tolist()))
            opts_c4 = L.model_newton_options(z)
            res = L.evaluate(112, 48, 3, list(range(lo, hi + 1)), args.learned_steps, float(z["cfl_factor"]),
                             opts_c4, {k: z[k] for k in ("widths", "master", "mu", "sd", "osc")}, scales)
            learned[key] = {
                "workload": "2D triple point 112x48 Q3Q2, smoothed viscosity, %gx explicit CFL, held-out "
                            "perturbation seeds %s, %d steps each, tol 1e-10, block preconditioner mode %d "
                            "(lag %d)" % (float(z["cfl_factor"]), args.learned_seeds, args.learned_steps,
                                          opts_c4.prec_probe, opts_c4.prec_lag),
                "plain": res["plain"], "plain_fallback": res["plain_fallback"], "learned": res["learned"],
                "zero_output_control": res["zero"],
                "matched": {k: res[k] for k in res if k.startswith("learned_vs_")},
                "speedup_s_per_step": res["learned_vs_plain"]["speedup_s_per_step"]}

    if args.copy_probe_mib:
        nb = args.copy_probe_mib << 20
        src = torch.ones(nb // 4, device="cuda", dtype=torch.float32)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    c1 = c1_leg(ilh, torch)
    c4 = None
    c4w = None
    if not args.no_c4:
        c4 = triple_point_legs(ilh, torch)
        c4w = c4_configured_width_leg(ilh, torch)
    sedov = None
    if not args.no_sedov:
        sedov = sedov_leg(ilh, torch)


    out = {
        "metric": "JVP quad-pts/s (% HBM roofline); s/implicit step, learned-guess vs plain",
        "value": value,
        "unit": "quad-pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (Jacobian action) / f64 (residual, masses, Newton)",
        "data": "synthetic (analytic Taylor-Green initial state)",
        "config": {"workload": "2D Taylor-Green %dx%d Q%dQ%d, gamma 5/3, no viscosity, implicit midpoint at "
                               "%gx explicit CFL 0.5 (dt=%.4g), Newton tol 1e-10, FP32 GMRES JVP" %
                               (n, n, k, k - 1, args.cfl_factor, dt),
                   "n_qp": H.nqp, "n_block": H.nblock},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": recorded_traffic(n, k, args.jvp_variant),
                     "kernel": KERNEL_NAMES[args.jvp_variant], "bytes_per_launch": alg32,
                     "bytes_count": "algorithmic: state, direction and result (3 block vectors) + m_q, "
                                    "FP32: %.1f B per quadrature point" % (alg32 / H.nqp),
                     "design_bytes_per_launch": bytes_loop,
                     "bandwidth_frac": bytes_loop / jvp_avg_s / 1e9 / HBM_PEAK_GBS,
                     "avg_launch_us": 1e6 * jvp_avg_s, "launches": jvp_n,
                     "avg_launch_us_back_to_back_fp32_output": burst_us,
                     "valu": recorded_valu(n, k, args.jvp_variant, jvp_avg_s)},
        "transpose_action": {"kernel": "k_vjp2d_q<4,6,float,visc=0,src=1>", "avg_launch_us_back_to_back": vjp_us,
                             "qps": H.nqp / (1e-6 * vjp_us), "bytes_per_launch": alg32,
                             "frac": alg32 / (1e-6 * vjp_us) / 1e9 / HBM_PEAK_GBS,
                             "design_bytes_per_launch": bytes32,
                             "bandwidth_frac": bytes32 / (1e-6 * vjp_us) / 1e9 / HBM_PEAK_GBS},
        "jvp_variant": args.jvp_variant,
        "jvp_apply_qps": H.nqp / jvp_avg_s,
        "residual": res_c2,
        "linearize": {"launches": lin_n, "avg_launch_us": 1e3 * lin_ms / max(lin_n, 1),
                      "bytes_per_launch": lin_bytes(H, 32) if lin_n else None,
                      "jvp_launches_per_linearization": jvp_n / lin_n if lin_n else None},
        "cpu_baseline": cpu_baseline_line(cpu) if cpu else None,
        "cpu_oracle": cpu,
        "s_per_implicit_step_plain": ms_per_step / 1e3,
        "ms_per_step_with_kernel_events": ms_per_step_events,
        "newton_per_step": float(np.mean(newton)),
        "gmres_per_step": float(np.mean(gmres)),
        "kernel_ms_per_step": {kname: v[0] / args.steps for kname, v in tim.items()},
        "energy_after": ke + ie,
    }
    out["c1_m1"] = c1
    if cpu:
        est = {"C2": oracle_step_estimate(cpu, "C2", float(np.mean(newton)), float(np.mean(gmres)))}
        if c4:
            f = c4["fixed_8x_fp32"]
            est["C4"] = oracle_step_estimate(cpu, "C4", f["newton_per_step"], f["gmres_per_step"])
        est["C1_measured_1core"] = cpu["oracle_s_per_step_C1_1core"]
        out["oracle_s_per_implicit_step"] = est
    out.update(extra)
    out.update(learned)
    if "learned_guess_c5" in learned:
        mt = learned["learned_guess_c5"]["matched"]["learned_vs_plain"]
        out["s_per_implicit_step_learned_c5"] = mt["s_per_step_learned"]
        out["s_per_implicit_step_plain_c5"] = mt["s_per_step_plain"]
        out["c5_matched_steps"] = mt["matched_steps"]
    if roof_extra:
        out["roofline_large_shape"] = roof_extra
    if roof_3d:
        out["roofline_3d"] = roof_3d
    if c4:
        out["c4_triple_point"] = c4
    if c4w:
        out["c4_configured_width"] = c4w
    if sedov:
        out["sedov_2d"] = sedov
    print(json.dumps(_finite(out), allow_nan=False))


if __name__ == "__main__":
    main()

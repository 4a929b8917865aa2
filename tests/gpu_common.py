"""Shared helpers of the GPU parity tests (oracle on the CPU, HIP library on the GPU)."""
import numpy as np
import torch

import seeded_inputs as si


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def maxrel(a, b):
    """Entry-wise bound: max |a - b| over max |b| (a few wrong entries of a long vector show here
    even when the 2-norm ratio hides them)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    mb = np.abs(b).max() if b.size else 0.0
    return float(np.abs(a - b).max() / (mb if mb > 0 else 1.0)) if b.size else 0.0


def blocks_close(a, b, nh1, tol):
    """Both bounds on every block [x | v | e] of a block vector: the 2-norm ratio and the
    entry-wise max bound, each block against its own scale.  Returns the worst ratio to tol."""
    worst = 0.0
    for sl in (slice(0, nh1), slice(nh1, 2 * nh1), slice(2 * nh1, None)):
        bb = np.asarray(b)[sl]
        if bb.size == 0 or not np.any(bb):
            continue
        worst = max(worst, rel(np.asarray(a)[sl], bb) / tol, maxrel(np.asarray(a)[sl], bb) / tol)
    return worst


def close(a, b, tol, nh1=None):
    """Both parity bounds: the 2-norm ratio rel(a, b) <= tol and the entry-wise bound
    max |a - b| <= tol max |b|; with nh1, the entry-wise bound holds on each block [x | v | e]
    against that block's own largest entry (a block of b that is all zero against the whole)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if not rel(a, b) <= tol:
        return False
    parts = [slice(None)] if nh1 is None else [slice(0, nh1), slice(nh1, 2 * nh1), slice(2 * nh1, None)]
    scale_all = np.abs(b).max() if b.size else 0.0
    for sl in parts:
        bb, aa = b[sl], a[sl]
        if bb.size == 0:
            continue
        sc = np.abs(bb).max()
        if sc == 0.0:
            sc = scale_all
        if not np.abs(aa - bb).max() <= tol * (sc if sc > 0 else 1.0):
            return False
    return True


def to_dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def to_np(t):
    return t.detach().double().cpu().numpy()


def make_pair(problem, n, k, visc=None, width=1e-3, **kw):
    """(oracle Hydro, GPU Hydro) for the same discretisation."""
    from oracle.hydro import Hydro as OHydro, ViscosityOptions
    import paper_2609_16424_amd as ilh
    vo = ViscosityOptions(on=visc is not None, mode=visc or "const", width=width)
    O = OHydro(problem, n, k, visc=vo, **kw)
    G = ilh.Hydro(problem, n, k, visc=visc is not None, dscale_mode=visc or "const",
                  dscale_width=width, tg_source=O.use_source)
    return O, G


def random_state(O, seed, amp=0.03):
    u = O.init_state()
    h = float(np.min(O.mesh.h)) / O.k
    return si.perturb_state(u, seed, O.nh1, amp * h, 0.3, 0.2)


def random_dir(O, seed):
    h = float(np.min(O.mesh.h)) / O.k
    return si.block_direction(seed, O.nh1, O.nl2, sx=h, sv=1.0, se=1.0)


def jvp_local(O, k, u, tau, dk, adj, h=1.0e-30):
    """The oracle's complex-step Jacobian action J dk = Im R(k + i h dk; tau, u) / h with the force
    evaluated on the elements `adj` only (oracle.hydro.Hydro.force(elements=...)).  The result is
    exact at every row whose elements all lie in `adj` (and everywhere when dk is supported on
    the degrees of freedom of `adj`): the other elements' contributions have no imaginary part
    there.  Used for sampled rows and columns of the action at full benchmark size."""
    nh1 = O.nh1
    m = O.mesh
    kc = k + 1j * h * dk
    wc = u + tau * kc
    adj = np.asarray(sorted(set(int(a) for a in adj)))
    F1, Ftv_sub = O.force(wc, elements=adj)
    kx, kv, ke = O.split(dk)
    out_x = kx - tau * kv
    out_v = np.where(O.cons, kv, O.mass_v(kv) + F1.imag / h)
    Ftv = np.zeros((m.Ne, m.Nl))
    Ftv[adj] = Ftv_sub.imag / h
    out_e = O.mass_e(ke) - Ftv.ravel()
    if O.use_source and np.any(kx):
        out_e = out_e - O.energy_source(wc[:nh1]).imag / h
    return np.concatenate([out_x, out_v, out_e])


def elements_of_dof(O, j):
    """Elements whose residual rows depend on block degree of freedom j."""
    nh1, m = O.nh1, O.mesh
    if j < 2 * nh1:
        node = j % m.N
        return np.nonzero((m.conn == node).any(axis=1))[0]
    return np.array([(j - 2 * nh1) // m.Nl])

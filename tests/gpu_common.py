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

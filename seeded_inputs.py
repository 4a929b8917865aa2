"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle timing leg.

Holds only random-number generation and plain array arithmetic on given arrays (no step
of the hydrodynamics method): Gaussian directions scaled per block, and perturbations of
a given state.  Both the GPU path and the CPU oracle receive the arrays made here.
"""
import numpy as np


def block_direction(seed, nh1, nl2, sx=1.0, sv=1.0, se=1.0):
    """N(0,1) block vector [x | v | e] with per-block scales."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal(2 * nh1 + nl2)
    d[:nh1] *= sx
    d[nh1:2 * nh1] *= sv
    d[2 * nh1:] *= se
    return d


def perturb_state(u, seed, nh1, ax, av, ae_rel):
    """u + (ax, av) N(0,1) on the x and v blocks; e multiplied by (1 + ae_rel N(0,1))."""
    rng = np.random.default_rng(seed)
    w = np.array(u, dtype=np.float64, copy=True)
    w[:nh1] += ax * rng.standard_normal(nh1)
    w[nh1:2 * nh1] += av * rng.standard_normal(nh1)
    w[2 * nh1:] *= 1.0 + ae_rel * rng.standard_normal(w.size - 2 * nh1)
    return w


def displace_positions(u, nh1, amp):
    """x <- x + amp * v (the velocity block of u): a smooth mesh displacement."""
    w = np.array(u, dtype=np.float64, copy=True)
    w[:nh1] += amp * w[nh1:2 * nh1]
    return w


def zero_rows(d, mask_rows):
    """Zero the entries of d listed by the boolean mask (e.g. constrained velocity rows)."""
    d = np.array(d, copy=True)
    d[mask_rows] = 0.0
    return d


def curved_positions(x0, lo, hi, amp):
    """A smooth interior displacement of the node positions x0 [dim][N] of a box mesh:
    x_c <- x_c + amp (hi_c - lo_c) prod_a sin(pi t_a), t_a = (x_a - lo_a)/(hi_a - lo_a).
    It vanishes on the box faces, so the boundary nodes stay where they are."""
    x0 = np.asarray(x0, dtype=np.float64)
    dim = x0.shape[0]
    bump = np.ones(x0.shape[1])
    for a in range(dim):
        bump *= np.sin(np.pi * (x0[a] - lo[a]) / (hi[a] - lo[a]))
    out = x0.copy()
    for c in range(dim):
        out[c] += amp * (hi[c] - lo[c]) * bump * (1.0 if c % 2 == 0 else -0.5)
    return out

"""ilh_jvp_noalloc (the Jacobian action with its storage in the library's static scratch array)
against ilh_jvp on the same context: two calls in a row on one GPU, the second on a smaller mesh,
in both precisions and on the linearised and the generic kernels; the context's own linearisation
point is left as it was; a mesh whose storage exceeds the array is rejected."""
import numpy as np
import pytest
import torch

import paper_2609_16424_amd as ilh
import seeded_inputs as si
from gpu_common import close, to_dev, to_np

pytestmark = pytest.mark.gpu


def _inputs(G, seed):
    u0 = to_np(G.init_state())
    h = 1.0 / (G.k * max(G.n))
    u = si.perturb_state(u0, seed, G.nh1, 0.05 * h, 0.05, 0.02)
    k = si.block_direction(seed + 1, G.nh1, G.nl2, 0.1 * h, 0.1, 0.1)
    dk = si.block_direction(seed + 2, G.nh1, G.nl2, h, 1.0, 1.0)
    tau = 0.5 * G.dt_estimate(to_dev(u), 2.0)
    return to_dev(u), to_dev(k), dk, tau


def _compare(G, seed):
    u, k, dk, tau = _inputs(G, seed)
    for prec, tol in ((64, 1e-12), (32, 1e-5)):
        dt = torch.float64 if prec == 64 else torch.float32
        d = to_dev(dk, dt)
        ref = to_np(G.jvp(k, u, tau, d, prec))
        out = torch.empty(G.nblock, dtype=dt, device=u.device)
        got = to_np(G.jvp_noalloc(k, u, tau, d, prec, out=out))
        assert close(got, ref, tol, G.nh1), (prec, np.abs(got - ref).max())


def test_noalloc_matches_jvp_two_calls_second_smaller():
    big = ilh.Hydro("tg2d", (128, 128), 3)          # the benchmark mesh: 2D Q3Q2 128 x 128
    _compare(big, 10)
    small = ilh.Hydro("triple", (14, 6), 2, visc=True, dscale_mode="formula", h_coarse=0.5)
    _compare(small, 20)                             # same GPU, same array, smaller input


def test_noalloc_3d_and_generic_kernels():
    _compare(ilh.Hydro("tg3d", (8, 6, 5), 2), 30)  # 3D linearised kernels
    g = ilh.Hydro("tg3d", (4, 3, 3), 3)              # no linearised kernel at k = 3: generic path
    _compare(g, 40)


def test_noalloc_leaves_the_context_linearisation():
    G = ilh.Hydro("tg2d", (24, 20), 3)
    u, k, dk, tau = _inputs(G, 50)
    d = to_dev(dk)
    G.linearize(k, u, tau)
    a = to_np(G.jvp_lin(d, 64))
    u2, k2, dk2, tau2 = _inputs(G, 60)
    G.jvp_noalloc(k2, u2, tau2, to_dev(dk2), 64)
    b = to_np(G.jvp_lin(d, 64))
    assert close(b, a, 1e-14, G.nh1)


def test_noalloc_rejects_meshes_beyond_the_array():
    G = ilh.Hydro("tg2d", (1024, 1024), 3)           # 2D Q3Q2 1024^2 needs ~2.2 GB of storage
    z = torch.zeros(G.nblock, dtype=torch.float64, device="cuda")
    with pytest.raises(ilh.IlhError) as e:
        G.jvp_noalloc(z, z, 1e-3, z, 64, out=torch.empty_like(z))
    assert e.value.status == ilh._lib.ILH_EINVAL
    assert "scratch" in str(e.value)

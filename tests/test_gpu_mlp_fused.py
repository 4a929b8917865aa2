"""The fused learned-guess inference launch (ilh_guess_mlp_fused: the features of (u, base) and
every MLP layer in one kernel, BF16 weights and biases held in LDS) against the features kernel
followed by the layer-by-layer MFMA forward.  Both round the same operands to BF16, accumulate
in the same order and apply the same epilogue, so the outputs must agree bit for bit; the cases
cover a few tiles of 16 elements, many tiles with a partial last one, the base block and
the standardisation on or off, two to four layers (padded widths the layered forward takes), and
the committed trained model on a triple-point state (336 tiles)."""
import os

import numpy as np
import pytest
import torch

import paper_2609_16424_amd as ilh
import seeded_inputs as si
from paper_2609_16424_amd import learned as L

pytestmark = pytest.mark.gpu


def _guess(h, hidden, with_base, normed, seed):
    k = h.k
    nout = 2 * (k + 1) ** 2 + k * k
    nin = nout + 8 + (nout if with_base else 0)
    widths = [nin] + list(hidden) + [nout]
    mlp = L.GuessMLP(h, widths, seed=seed)
    g = torch.Generator(device=h.device).manual_seed(seed + 1)
    off = mlp.nW
    for l in range(mlp.nl):  # biases on the true widths, zero padding
        n = widths[l + 1]
        mlp.master[off:off + n] = 0.1 * torch.randn(n, generator=g, device=h.device)
        off += mlp.P[l + 1]
    norm = None
    if normed:
        rng = np.random.default_rng(seed + 2)
        norm = {"mu": (0.1 * rng.standard_normal(L.pad32(nin))).astype(np.float32),
                "sd": (1.0 + 0.5 * rng.random(L.pad32(nin))).astype(np.float32),
                "osc": (1.0 + rng.random(L.pad32(nout))).astype(np.float32)}
    scales = {"vs": 0.7, "es": 1.3, "xs": 1.0 / h.n[0], "kvs": 0.3, "kes": 0.9}
    return L.LearnedGuess(h, mlp, scales, with_base=with_base, norm=norm)


def _state(h, seed):
    u = h.init_state()
    w = si.perturb_state(u.cpu().numpy(), seed, h.nh1, 1e-3 / h.n[0], 0.05, 0.02)
    u = torch.from_numpy(w).to(h.device)
    base = h.plain_guess(u, [], 0.01)
    return u, base


@pytest.mark.parametrize("n,k,hidden,with_base,normed", [
    ((9, 7), 2, (64,), False, False),
    ((40, 30), 2, (128, 64), True, True),
    ((13, 11), 3, (128, 128, 128), True, False),
    ((21, 17), 3, (32, 64, 128), False, True),
])
def test_fused_equals_layered(n, k, hidden, with_base, normed):
    h = ilh.Hydro("tg2d", n, k)
    lg = _guess(h, hidden, with_base, normed, seed=11 * k + len(hidden))
    u, base = _state(h, 5)
    a = lg.predict_fused(u, base)
    b = lg.predict_layered(u, base)
    assert torch.isfinite(b).all()
    assert torch.equal(a, b), float((a - b).abs().max())


def test_fused_rejects_mismatched_widths():
    h = ilh.Hydro("tg2d", (6, 5), 2)
    lg = _guess(h, (32,), False, False, seed=3)
    u, base = _state(h, 1)
    lg.with_base = True  # the features would include a base block the widths do not cover
    with pytest.raises(ilh.IlhError):
        lg.predict_fused(u, base)


@pytest.mark.skipif(not os.path.exists(L.DEFAULT_MODEL), reason="no trained model committed")
def test_fused_equals_layered_trained_model():
    z = np.load(L.DEFAULT_MODEL)
    scales = dict(zip(("vs", "es", "xs", "kvs", "kes"), z["scales"].tolist()))
    h = L.make_triple(112, 48, 3, seed=1002)
    u = h.init_state()
    dt = float(z["cfl_factor"]) * h.dt_estimate(u, 0.5)
    opts = L.model_newton_options(z)
    hist = []
    for _ in range(2):
        kk, _ = h.implicit_step(u, dt, guess=h.plain_guess(u, hist, 0.5 * dt), opts=opts)
        hist = (hist + [kk])[-2:]
    mlp = L.GuessMLP(h, [int(w) for w in z["widths"]])
    mlp.load_state({key: z[key] for key in ("widths", "master")})
    lg = L.LearnedGuess(h, mlp, scales, norm={key: z[key] for key in ("mu", "sd", "osc")})
    base = h.plain_guess(u, hist, 0.5 * dt)
    a = lg.predict_fused(u, base)
    b = lg.predict_layered(u, base)
    assert torch.equal(a, b), float((a - b).abs().max())

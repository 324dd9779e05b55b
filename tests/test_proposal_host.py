"""Host-side pieces of the learned proposal (CPU, no GPU): the symmetry-
invariant alignment loss of the supervised warm start, and the symmetries
it relies on, checked on the float64 oracle."""
import math

import numpy as np
import torch

import oracle as O
from paper_2506_22935_amd.proposal import alignment_loss, median_all


def test_images_of_the_weighted_isl_are_equal():
    # a global phase, a linear phase ramp, time reversal and conjugation
    # leave the weighted ISL of a code unchanged (W depends on |tau| and
    # |k_c| only): the codes the alignment loss identifies are equally good
    n, m = 24, 64
    rng = np.random.default_rng(5)
    s = np.exp(1j * rng.uniform(0, 2 * math.pi, n))
    u, v = rng.uniform(0, 1, 31), rng.uniform(0, 1, 31)
    lp = O.LossParams(w_isl=1.0, h_tau=2, h_k=1, u=u, v=v, eps=1e-12)

    def wisl(x):
        return O.loss_terms(O.chi(x, m), O.energy(x), n, lp)["isl"]

    ref = wisl(s)
    ramp = np.exp(1j * 0.37 * np.arange(n))
    for img in (s * np.exp(0.9j), s * ramp, s[::-1], np.conj(s), np.conj(s[::-1]) * ramp):
        assert abs(wisl(img) - ref) <= 1e-12 * ref
    # a quadratic phase is not such a symmetry: it shears |chi| along k
    assert abs(wisl(s * np.exp(0.05j * np.arange(n) ** 2)) - ref) > 1e-6 * ref


def test_alignment_loss_zero_on_every_image():
    torch.manual_seed(0)
    tgt = torch.rand(3, 16, dtype=torch.float64) * 2 * math.pi
    rev = torch.flip(tgt, dims=[1])
    ramp = 2 * math.pi * 5 / (8 * 16) * torch.arange(16, dtype=torch.float64)  # a slope on the search grid
    for img in (tgt + 0.7, rev - 1.1, -tgt + 2.0, -rev, tgt + ramp, -rev - 3 * ramp + 0.2):
        loss, g = alignment_loss(img, tgt)
        assert abs(loss) < 1e-12
        assert float(g.abs().max()) < 1e-12


def test_alignment_loss_gradient_finite_differences():
    torch.manual_seed(1)
    B, n = 3, 16
    tgt = torch.rand(B, n, dtype=torch.float64) * 2 * math.pi
    phi = torch.rand(B, n, dtype=torch.float64) * 2 * math.pi
    loss, g = alignment_loss(phi, tgt)
    assert 0.0 < loss < 1.0
    h = 1e-6
    num = torch.zeros_like(phi)
    for b in range(B):
        for k in range(n):
            p = phi.clone()
            p[b, k] += h
            lp = alignment_loss(p, tgt)[0]
            p[b, k] -= 2 * h
            lm = alignment_loss(p, tgt)[0]
            num[b, k] = (lp - lm) / (2 * h)
    assert float((num - g).abs().max()) <= 1e-7 * float(g.abs().max())


def test_median_counts_misses_as_infinite():
    inf = float("inf")
    assert median_all(torch.tensor([1.0, 2.0, 3.0])) == 2.0
    assert median_all(torch.tensor([1.0, inf, inf])) == inf
    assert median_all(torch.tensor([1.0, 2.0, inf, inf])) == 2.0  # lower median of an even count
    assert median_all(torch.tensor([5.0, 1.0, inf, 3.0, inf])) == 5.0

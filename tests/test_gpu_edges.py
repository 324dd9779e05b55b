"""Degenerate and boundary cases of the HIP path against the oracle (GPU).

Covered: the shortest waveforms (N = 1, 2, 3), N = M/2 exactly and M = 8N,
lag windows of one and three rows, single-cell and full-lag mainlobes, a
waveform with leading and trailing zeros, and a zero-energy waveform
(documented to give NaN losses, not a fault).
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_2506_22935_amd import workloads as W

pytestmark = pytest.mark.gpu
EPS = 1e-12
TOL_A = 1e-5
TOL_G = 1e-4


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def af():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_22935_amd import af as af_mod
    return af_mod


def dev(s):
    return torch.from_numpy(np.ascontiguousarray(s.astype(np.complex64))).cuda()


def ref64(s):
    return O.to_c64_exact(s.astype(np.complex64))


def cancel_floor(dlde, s):
    """Float32 floor of a gradient that is a difference of two large parts.
    Normalised losses are scale-free, so dL/dE * s cancels the per-cell part
    along s (for N = 1 the gradient is exactly 0): the float32 result keeps a
    few units of roundoff of |dL/dE| * max|s|."""
    return 8.0 * 2.0 ** -24 * abs(dlde) * np.max(np.abs(s))


def grad_close(got, ref, what, floor=0.0):
    bar = max(TOL_G * np.max(np.abs(ref)), floor, 1e-7)
    err = np.max(np.abs(got - ref))
    assert err <= bar, "%s: err %.3e bar %.3e" % (what, err, bar)


@pytest.mark.parametrize("n,m,T", [(1, 128, -1), (2, 128, -1), (3, 128, -1), (16, 128, -1), (64, 128, -1),
                                   (100, 256, 0), (100, 256, 1), (511, 1024, 3)])
def test_forward_edges(af, n, m, T):
    say("forward edge", n, m, T)
    s = W.random_code(n, seed=900 + n)
    plan = af.Plan([n], [m], [T], eps=EPS)
    mag, chi, e = plan.forward(dev(s), mag=True, chi=True)
    torch.cuda.synchronize()
    Tn = n - 1 if T < 0 else T
    sr = ref64(s)
    E = O.energy(sr)
    c_ref = O.chi(sr, m, Tn)
    assert abs(e.item() - E) <= 1e-6 * E
    assert np.max(np.abs(plan.grid(mag, 0).cpu().numpy() - O.magnitude(c_ref, E, EPS))) <= TOL_A
    assert np.max(np.abs(plan.grid(chi, 0).cpu().numpy() - c_ref)) <= TOL_A * E


@pytest.mark.parametrize("n,m,T", [(1, 128, -1), (2, 128, -1), (100, 256, 0), (100, 256, 1), (511, 1024, 3)])
def test_backward_edges(af, n, m, T):
    say("backward edge", n, m, T)
    s = W.random_code(n, seed=950 + n)
    Tn = n - 1 if T < 0 else T
    sr = ref64(s)
    a_ref = O.magnitude(O.chi(sr, m, Tn), O.energy(sr), EPS)
    ga = (W.upstream_grid(2 * Tn + 1, m, seed=n) * a_ref).astype(np.float32)
    plan = af.Plan([n], [m], [T], eps=EPS)
    ws = plan.new_workspace()
    plan.forward(dev(s), mag=False, ws=ws)
    g = plan.backward(dev(s), torch.from_numpy(ga.ravel()).cuda(), ws=ws)
    torch.cuda.synchronize()
    ref = O.magnitude_backward(sr, m, Tn, ga.astype(np.float64), EPS)
    E = O.energy(sr)
    p = np.abs(O.chi(sr, m, Tn)) ** 2 / E ** 2
    dlde = np.sum(ga * p / (E * a_ref))  # size of the energy term that cancels
    grad_close(g.cpu().numpy().astype(np.complex128), ref, "backward %d/%d/%d" % (n, m, T), cancel_floor(dlde, sr))


@pytest.mark.parametrize("n,m,h_tau,h_k", [(1, 128, 1, 1), (3, 128, 1, 1), (200, 512, 0, 0), (64, 256, 63, 0),
                                           (128, 256, 2, 4)])
@pytest.mark.parametrize("lp", [dict(w_isl=1.0, w_psl=0.0, temp=0.05), dict(w_isl=1.0, w_psl=1.0, temp=0.05)])
def test_loss_mainlobe_edges(af, n, m, h_tau, h_k, lp):
    # single-cell mainlobe, a mainlobe over every lag, wider windows, and the
    # shortest waveforms; both the fused ISL pass and the fused ISL + soft-PSL
    say("loss edge", n, m, h_tau, h_k, lp)
    s = W.random_code(n, seed=1000 + n + h_k)
    plan = af.Plan([n], [m], h_tau=h_tau, h_k=h_k, eps=EPS)
    terms, g, _ = plan.loss(dev(s), grad=True, **lp)
    torch.cuda.synchronize()
    ref = O.loss_and_grad(ref64(s), m, n - 1, O.LossParams(h_tau=h_tau, h_k=h_k, eps=EPS, **lp))
    t = terms.cpu().numpy()[0]
    assert abs(t[0] - ref["loss"]) <= 1e-4 * abs(ref["loss"]) + 1e-5
    assert abs(t[1] - ref["isl"]) <= 1e-4 * abs(ref["isl"]) + 1e-5
    # dL/dE of a normalised loss is of the order of 2 loss / E
    grad_close(g.cpu().numpy().astype(np.complex128), ref["g"], "loss edge",
               cancel_floor(2.0 * abs(ref["loss"]) / O.energy(ref64(s)), ref64(s)))


def test_zero_padded_waveform(af):
    # leading and trailing zeros inside the declared length
    say("zero-padded waveform")
    n, m = 300, 1024
    s = W.random_code(n, seed=77).astype(np.complex64)
    s[:40] = 0
    s[-70:] = 0
    plan = af.Plan([n], [m], eps=EPS)
    terms, g, mag = plan.loss(dev(s), w_isl=1.0, w_psl=1.0, temp=0.05, grad=True, mag=True)
    torch.cuda.synchronize()
    sr = ref64(s)
    ref = O.loss_and_grad(sr, m, n - 1, O.LossParams(eps=EPS, w_isl=1.0, w_psl=1.0, temp=0.05))
    assert np.max(np.abs(plan.grid(mag, 0).cpu().numpy() - ref["a"])) <= TOL_A
    assert abs(terms[0, 0].item() - ref["loss"]) <= 1e-4 * abs(ref["loss"])
    grad_close(g.cpu().numpy().astype(np.complex128), ref["g"], "zero-padded")


def test_zero_energy_gives_nan_not_a_fault(af):
    say("zero energy")
    n, m = 64, 128
    plan = af.Plan([n], [m], eps=EPS)
    terms, g, _ = plan.loss(dev(np.zeros(n, dtype=np.complex64)), w_isl=1.0, w_psl=1.0, grad=True)
    torch.cuda.synchronize()
    assert terms[0, 3].item() == 0.0  # E
    assert np.isnan(terms[0, 0].item())

"""Cross-ambiguity of two waveforms on the HIP path against the oracle
(GPU): the magnitude and chi_su grids, and the backward for both inputs, over
one-waveform and uneven plans, aperiodic and periodic (circular lags) and
both in one plan (the cross-AF extension of the paper's limitations
section)."""
import sys

import numpy as np
import pytest
import torch

import oracle as O

pytestmark = pytest.mark.gpu
EPS = 1e-12


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def af():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_22935_amd import af as afmod
    return afmod


def rand_c64(n, seed):
    rng = np.random.default_rng(seed)
    return O.to_c64_exact((rng.standard_normal(n) + 1j * rng.standard_normal(n)) / np.sqrt(2.0))


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.complex64))).cuda()


@pytest.mark.parametrize("n,m,T", [(64, 128, -1), (100, 256, 30), (300, 1024, -1), (1000, 2048, 200),
                                   (2048, 4096, 40), (4096, 8192, 12), (1, 128, -1)])
def test_cross_forward(af, n, m, T):
    say("cross forward", n, m, T)
    s, u = rand_c64(n, 2000 + n), rand_c64(n, 3000 + n)
    Tn = n - 1 if T < 0 else T
    plan = af.Plan([n], [m], [T], eps=EPS)
    mag, chi, e = plan.cross_forward(to_dev(s), to_dev(u), mag=True, chi=True)
    torch.cuda.synchronize()
    Es, Eu = O.energy(s), O.energy(u)
    assert abs(e[0, 0].item() - Es) <= 1e-5 * Es and abs(e[0, 1].item() - Eu) <= 1e-5 * Eu
    rows = 2 * Tn + 1
    bins = None if n * m <= 2048 * 2048 else np.random.default_rng(n).choice(m, 256, replace=False)
    ref = O.cross_chi(s, u, m, Tn, bins)
    a_ref = np.sqrt(np.abs(ref) ** 2 / (Es * Eu) + EPS)
    g_mag = mag.cpu().numpy().reshape(rows, m).astype(np.float64)
    g_chi = chi.cpu().numpy().reshape(rows, m).astype(np.complex128)
    if bins is not None:
        g_mag, g_chi = g_mag[:, bins], g_chi[:, bins]
    assert np.max(np.abs(g_mag - a_ref)) <= 1e-5
    scale = np.sqrt(Es * Eu)
    assert np.max(np.abs(g_chi - ref)) <= 1e-5 * scale


def test_cross_with_itself_is_the_af(af):
    say("cross u = s")
    n, m = 200, 512
    s = rand_c64(n, 5)
    plan = af.Plan([n], [m], eps=EPS)
    mag, _, _ = plan.cross_forward(to_dev(s), to_dev(s))
    torch.cuda.synchronize()
    ref = O.magnitude(O.chi(s, m, n - 1), O.energy(s), EPS)
    assert np.max(np.abs(mag.cpu().numpy().reshape(ref.shape) - ref)) <= 1e-5


@pytest.mark.parametrize("n,m,T", [(64, 128, -1), (100, 256, 30), (300, 1024, -1), (1000, 2048, 100),
                                   (2048, 4096, 24), (4096, 8192, 6)])
def test_cross_backward(af, n, m, T):
    say("cross backward", n, m, T)
    s, u = rand_c64(n, 4000 + n), rand_c64(n, 5000 + n)
    Tn = n - 1 if T < 0 else T
    w = np.random.default_rng(n + 1).standard_normal((2 * Tn + 1, m)).astype(np.float32)
    plan = af.Plan([n], [m], [T], eps=EPS)
    gs, gu = plan.cross_backward(to_dev(s), to_dev(u), torch.from_numpy(w.ravel()).cuda())
    gs2, gu2 = plan.cross_backward(to_dev(s), to_dev(u), torch.from_numpy(w.ravel()).cuda())
    torch.cuda.synchronize()
    rs, ru = O.cross_magnitude_backward(s, u, m, Tn, w.astype(np.float64), EPS)
    for g, r, name in ((gs, rs, "s"), (gu, ru, "u")):
        err = np.max(np.abs(g.cpu().numpy().astype(np.complex128) - r))
        assert err <= 1e-4 * np.max(np.abs(r)), (name, err, np.max(np.abs(r)))
    # deterministic: no atomics
    assert torch.equal(gs, gs2) and torch.equal(gu, gu2)


def test_cross_uneven_batch(af):
    say("cross uneven")
    sizes, ms, Ts = [64, 100, 300, 37], [128, 256, 1024, 128], [-1, 20, 60, -1]
    ss = [rand_c64(n, 6000 + n) for n in sizes]
    us = [rand_c64(n, 7000 + n) for n in sizes]
    plan = af.Plan(sizes, ms, Ts, eps=EPS)
    rows = [2 * (n - 1 if T < 0 else T) + 1 for n, T in zip(sizes, Ts)]
    ws_ = [np.random.default_rng(i).standard_normal((r, m)).astype(np.float32) for i, (r, m) in
           enumerate(zip(rows, ms))]
    sd, ud = to_dev(np.concatenate(ss)), to_dev(np.concatenate(us))
    mag, _, _ = plan.cross_forward(sd, ud)
    gs, gu = plan.cross_backward(sd, ud, torch.from_numpy(np.concatenate([w.ravel() for w in ws_])).cuda())
    torch.cuda.synchronize()
    mg, gsn, gun = mag.cpu().numpy(), gs.cpu().numpy(), gu.cpu().numpy()
    go = so = 0
    for s, u, n, m, T, r, w in zip(ss, us, sizes, ms, Ts, rows, ws_):
        Tn = n - 1 if T < 0 else T
        ref = np.sqrt(np.abs(O.cross_chi(s, u, m, Tn)) ** 2 / (O.energy(s) * O.energy(u)) + EPS)
        assert np.max(np.abs(mg[go:go + r * m].reshape(r, m) - ref)) <= 1e-5, n
        rs, ru = O.cross_magnitude_backward(s, u, m, Tn, w.astype(np.float64), EPS)
        assert np.max(np.abs(gsn[so:so + n] - rs)) <= 1e-4 * np.max(np.abs(rs)), n
        assert np.max(np.abs(gun[so:so + n] - ru)) <= 1e-4 * np.max(np.abs(ru)), n
        go += r * m
        so += n


@pytest.mark.parametrize("n", [64, 256, 1024, 4096])
def test_cross_periodic_forward(af, n):
    # the periodic cross-AF (circular lags, N x N grid) against the oracle's
    # defining sum; sampled bins at N = 4096
    say("cross periodic forward", n)
    s, u = rand_c64(n, 8000 + n), rand_c64(n, 8100 + n)
    plan = af.Plan([n], [n], eps=EPS, periodic=True)
    mag, chi, e = plan.cross_forward(to_dev(s), to_dev(u), mag=True, chi=True)
    torch.cuda.synchronize()
    Es, Eu = O.energy(s), O.energy(u)
    assert abs(e[0, 0].item() - Es) <= 1e-5 * Es and abs(e[0, 1].item() - Eu) <= 1e-5 * Eu
    bins = None if n <= 1024 else np.random.default_rng(n).choice(n, 64, replace=False)
    ref = O.cross_chi_circular(s, u, bins)
    a_ref = np.sqrt(np.abs(ref) ** 2 / (Es * Eu) + EPS)
    g_mag = mag.cpu().numpy().reshape(n, n).astype(np.float64)
    g_chi = chi.cpu().numpy().reshape(n, n).astype(np.complex128)
    if bins is not None:
        g_mag, g_chi = g_mag[:, bins], g_chi[:, bins]
    assert np.max(np.abs(g_mag - a_ref)) <= 1e-5
    assert np.max(np.abs(g_chi - ref)) <= 1e-5 * np.sqrt(Es * Eu)


def test_cross_periodic_with_itself_is_the_periodic_af(af):
    say("cross periodic u = s")
    n = 256
    s = rand_c64(n, 8200)
    plan = af.Plan([n], [n], eps=EPS, periodic=True)
    mag, _, _ = plan.cross_forward(to_dev(s), to_dev(s))
    torch.cuda.synchronize()
    ref = O.magnitude(O.chi_circular(s), O.energy(s), EPS)
    assert np.max(np.abs(mag.cpu().numpy().reshape(n, n) - ref)) <= 1e-5


@pytest.mark.parametrize("n", [64, 256, 1024])
def test_cross_periodic_backward(af, n):
    say("cross periodic backward", n)
    s, u = rand_c64(n, 8300 + n), rand_c64(n, 8400 + n)
    w = np.random.default_rng(n + 7).standard_normal((n, n)).astype(np.float32)
    plan = af.Plan([n], [n], eps=EPS, periodic=True)
    gs, gu = plan.cross_backward(to_dev(s), to_dev(u), torch.from_numpy(w.ravel()).cuda())
    gs2, gu2 = plan.cross_backward(to_dev(s), to_dev(u), torch.from_numpy(w.ravel()).cuda())
    torch.cuda.synchronize()
    rs, ru = O.cross_magnitude_backward_circular(s, u, w.astype(np.float64), EPS)
    for g, r, name in ((gs, rs, "s"), (gu, ru, "u")):
        err = np.max(np.abs(g.cpu().numpy().astype(np.complex128) - r))
        assert err <= 1e-4 * np.max(np.abs(r)), (name, err, np.max(np.abs(r)))
    assert torch.equal(gs, gs2) and torch.equal(gu, gu2)


def test_cross_mixed_periodic_and_aperiodic(af):
    # periodic and aperiodic waveforms of several sizes in one plan
    say("cross mixed lag kinds")
    sizes, ms, per = [64, 100, 256, 300, 128], [64, 256, 256, 1024, 128], [True, False, True, False, True]
    ss = [rand_c64(n, 8500 + i) for i, n in enumerate(sizes)]
    us = [rand_c64(n, 8600 + i) for i, n in enumerate(sizes)]
    plan = af.Plan(sizes, ms, eps=EPS, periodic=per)
    rows = [n if p else 2 * n - 1 for n, p in zip(sizes, per)]
    ws_ = [np.random.default_rng(40 + i).standard_normal((r, m)).astype(np.float32) for i, (r, m) in
           enumerate(zip(rows, ms))]
    sd, ud = to_dev(np.concatenate(ss)), to_dev(np.concatenate(us))
    mag, _, _ = plan.cross_forward(sd, ud)
    gs, gu = plan.cross_backward(sd, ud, torch.from_numpy(np.concatenate([w.ravel() for w in ws_])).cuda())
    torch.cuda.synchronize()
    mg, gsn, gun = mag.cpu().numpy(), gs.cpu().numpy(), gu.cpu().numpy()
    go = so = 0
    for s, u, n, m, p, r, w in zip(ss, us, sizes, ms, per, rows, ws_):
        c = O.cross_chi_circular(s, u) if p else O.cross_chi(s, u, m, n - 1)
        ref = np.sqrt(np.abs(c) ** 2 / (O.energy(s) * O.energy(u)) + EPS)
        assert np.max(np.abs(mg[go:go + r * m].reshape(r, m) - ref)) <= 1e-5, n
        if p:
            rs, ru = O.cross_magnitude_backward_circular(s, u, w.astype(np.float64), EPS)
        else:
            rs, ru = O.cross_magnitude_backward(s, u, m, n - 1, w.astype(np.float64), EPS)
        assert np.max(np.abs(gsn[so:so + n] - rs)) <= 1e-4 * np.max(np.abs(rs)), n
        assert np.max(np.abs(gun[so:so + n] - ru)) <= 1e-4 * np.max(np.abs(ru)), n
        go += r * m
        so += n


@pytest.mark.parametrize("n,m,T", [(600, 16384, 20), (5000, 16384, 10), (9000, 32768, 6)])
def test_cross_forward_large_m(af, n, m, T):
    # M = 16384 and 32768: one row per work group, samples from global memory;
    # sampled bins against the oracle's defining sum
    say("cross forward large M", n, m, T)
    s, u = rand_c64(n, 8700 + n), rand_c64(n, 8800 + n)
    plan = af.Plan([n], [m], [T], eps=EPS)
    mag, chi, e = plan.cross_forward(to_dev(s), to_dev(u), mag=True, chi=True)
    torch.cuda.synchronize()
    Es, Eu = O.energy(s), O.energy(u)
    assert abs(e[0, 0].item() - Es) <= 1e-5 * Es and abs(e[0, 1].item() - Eu) <= 1e-5 * Eu
    rows = 2 * T + 1
    bins = np.sort(np.random.default_rng(m + n).choice(m, 128, replace=False))
    ref = O.cross_chi(s, u, m, T, bins)
    a_ref = np.sqrt(np.abs(ref) ** 2 / (Es * Eu) + EPS)
    g_mag = mag.cpu().numpy().reshape(rows, m)[:, bins].astype(np.float64)
    g_chi = chi.cpu().numpy().reshape(rows, m)[:, bins].astype(np.complex128)
    assert np.max(np.abs(g_mag - a_ref)) <= 1e-5
    assert np.max(np.abs(g_chi - ref)) <= 1e-5 * np.sqrt(Es * Eu)


@pytest.mark.parametrize("n,m,T", [(600, 16384, 12), (3000, 16384, 4), (600, 32768, 6)])
def test_cross_backward_large_m(af, n, m, T):
    say("cross backward large M", n, m, T)
    s, u = rand_c64(n, 8900 + n), rand_c64(n, 9000 + n)
    w = np.random.default_rng(m).standard_normal((2 * T + 1, m)).astype(np.float32)
    plan = af.Plan([n], [m], [T], eps=EPS)
    gs, gu = plan.cross_backward(to_dev(s), to_dev(u), torch.from_numpy(w.ravel()).cuda())
    gs2, gu2 = plan.cross_backward(to_dev(s), to_dev(u), torch.from_numpy(w.ravel()).cuda())
    torch.cuda.synchronize()
    rs, ru = O.cross_magnitude_backward(s, u, m, T, w.astype(np.float64), EPS)
    for g, r, name in ((gs, rs, "s"), (gu, ru, "u")):
        err = np.max(np.abs(g.cpu().numpy().astype(np.complex128) - r))
        assert err <= 1e-4 * np.max(np.abs(r)), (name, err, np.max(np.abs(r)))
    assert torch.equal(gs, gs2) and torch.equal(gu, gu2)


def test_cross_rejections(af):
    from paper_2506_22935_amd import _lib
    s = to_dev(rand_c64(128, 1))
    plan = af.Plan([128], [256], eps=EPS)
    g = torch.zeros(255 * 256, dtype=torch.float32, device="cuda")
    with pytest.raises(_lib.AfError) as ei:
        plan.cross_backward(s, s, g, ws=torch.empty(256, dtype=torch.uint8, device="cuda"))
    assert ei.value.code == -5


def test_cross_autograd_user_loss(af):
    # a user loss through torch autograd: L = sum w a on the cross-AF grid
    say("cross autograd")
    from paper_2506_22935_amd.autograd import cross_af_magnitude
    n, m, T = 200, 512, 50
    s0, u0 = rand_c64(n, 91), rand_c64(n, 92)
    w = np.random.default_rng(93).standard_normal((2 * T + 1) * m).astype(np.float32)
    plan = af.Plan([n], [m], [T], eps=EPS)
    s = to_dev(s0).requires_grad_(True)
    u = to_dev(u0).requires_grad_(True)
    a = cross_af_magnitude(s, u, plan)
    (a * torch.from_numpy(w).cuda()).sum().backward()
    torch.cuda.synchronize()
    rs, ru = O.cross_magnitude_backward(s0, u0, m, T, w.reshape(2 * T + 1, m).astype(np.float64), EPS)
    # torch's gradient of a real loss at a complex leaf is 2 dL/d conj(.)
    for g, r in ((s.grad, rs), (u.grad, ru)):
        gg = g.cpu().numpy().astype(np.complex128) / 2
        assert np.max(np.abs(gg - r)) <= 1e-4 * np.max(np.abs(r))

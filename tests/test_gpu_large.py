"""The large lag-window workload (GPU only): an N=16384 LFM chirp (time-
bandwidth 1000) with N(0, 0.3) rad phase noise, lags |tau| <= 2048,
M = 32768, forward and backward under a workspace budget.

Parity at this size: sampled rows against the direct-sum oracle; the full
gradient against the oracle's FFT-step route; store and recompute modes give
identical bits.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_2506_22935_amd import workloads as W

pytestmark = pytest.mark.gpu
EPS = 1e-12
N, M, T = 16384, 32768, 2048


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_22935_amd import af
    s = W.unimodular(W.lfm_noisy_phases(N, 1000.0, 0.3, seed=0))
    return dict(af=af, s=s, sr=O.to_c64_exact(s), sd=torch.from_numpy(s).cuda())


def test_large_forward_sampled_rows(setup):
    say("large forward rows")
    af, sd, sr = setup["af"], setup["sd"], setup["sr"]
    plan = af.Plan([N], [M], [T], eps=EPS, store_mode=2)
    mag, _, e = plan.forward(sd, mag=True)
    torch.cuda.synchronize()
    E = O.energy(sr)
    assert abs(e.item() - E) <= 1e-6 * E
    rng = np.random.default_rng(1)
    taus = [0, 1, -1, T, -T] + [int(x) for x in rng.integers(-T, T + 1, 3)]
    ref = O.magnitude(O.chi_rows(sr, M, taus), E, EPS)
    grid = plan.grid(mag, 0)
    for i, tau in enumerate(taus):
        got = grid[tau + T].cpu().numpy()
        assert np.max(np.abs(got - ref[i])) <= 1e-5, tau


def test_large_backward_store_and_recompute(setup):
    say("large backward")
    af, sd, sr = setup["af"], setup["sd"], setup["sr"]
    E = O.energy(sr)
    # upstream u * a (well conditioned), a from the oracle's FFT-step rows
    up = np.empty((2 * T + 1, M), dtype=np.float32)
    for i0 in range(0, 2 * T + 1, 256):
        i1 = min(2 * T + 1, i0 + 256)
        rows = O.chi_rows_fft(sr, M, range(i0 - T, i1 - T))
        a = O.magnitude(rows, E, EPS)
        u = np.random.default_rng(1000 + i0).standard_normal(a.shape)
        up[i0:i1] = (u * a).astype(np.float32)
    upd = torch.from_numpy(up.ravel()).cuda()
    grads = {}
    for store in (1, 2):
        plan = af.Plan([N], [M], [T], eps=EPS, store_mode=store)
        assert plan.summary()["stores"] == (1 if store == 1 else 0)
        ws = plan.new_workspace()
        plan.forward(sd, mag=False, ws=ws)
        grads[store] = plan.backward(sd, upd, ws=ws).cpu()
    torch.cuda.synchronize()
    assert torch.equal(grads[1], grads[2])
    ref = O.magnitude_backward_fft(sr, M, T, up.astype(np.float64), EPS)
    g = grads[1].numpy().astype(np.complex128)
    assert np.max(np.abs(g - ref)) <= 1e-4 * np.max(np.abs(ref))


def test_budget_decides_store_or_recompute(setup):
    say("budget")
    af = setup["af"]
    from paper_2506_22935_amd import _lib
    big = af.Plan([N], [M], [T], eps=EPS, store_mode=0, budget_bytes=16 << 30)
    assert big.summary()["stores"] == 1
    store_bytes = big.summary()["store_bytes"]
    small = af.Plan([N], [M], [T], eps=EPS, store_mode=0, budget_bytes=store_bytes // 2)
    assert small.summary()["stores"] == 0
    with pytest.raises(_lib.AfError) as ei:
        af.Plan([N], [M], [T], eps=EPS, store_mode=0, budget_bytes=1 << 10)
    assert ei.value.code == -3
    with pytest.raises(_lib.AfError) as ei:
        af.Plan([N], [M], [T], eps=EPS, store_mode=1, budget_bytes=store_bytes // 2)
    assert ei.value.code == -3


@pytest.mark.parametrize("variant", [2])
@pytest.mark.parametrize("n,m,T", [(6000, 16384, 300), (N, M, 200)])
def test_halves_in_turn_variants(setup, variant, n, m, T):
    # the halves-in-turn variant at both of its sizes with random-phase codes
    # and small windows: sampled forward rows against the direct sums, the
    # magnitude backward against the oracle's FFT-step route
    say("halves in turn", variant, n, m, T)
    af = setup["af"]
    s = W.random_code(n, seed=40 + n)
    sr = O.to_c64_exact(s)
    sd = torch.from_numpy(s).cuda()
    plan = af.Plan([n], [m], [T], eps=EPS, store_mode=2, variant=variant)
    assert plan.summary()["variant"] == variant
    ws = plan.new_workspace()
    mag, _, _ = plan.forward(sd, mag=True, ws=ws)
    E = O.energy(sr)
    taus = [0, 1, -1, T, -T, T // 2]
    ref = O.magnitude(O.chi_rows(sr, m, taus), E, EPS)
    grid = plan.grid(mag, 0).cpu().numpy()
    for i, tau in enumerate(taus):
        assert np.max(np.abs(grid[tau + T] - ref[i])) <= 1e-5, tau
    a = O.magnitude(O.chi_rows_fft(sr, m, range(-T, T + 1)), E, EPS)
    up = (np.random.default_rng(n).standard_normal(a.shape) * a).astype(np.float32)
    g = plan.backward(sd, torch.from_numpy(up.ravel()).cuda(), ws=ws).cpu().numpy().astype(np.complex128)
    gref = O.magnitude_backward_fft(sr, m, T, up.astype(np.float64), EPS)
    assert np.max(np.abs(g - gref)) <= 1e-4 * np.max(np.abs(gref))

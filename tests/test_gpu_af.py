"""Parity of the HIP path against the float64 oracle (GPU only).

Bars (stated in the design notes):
  a = sqrt(|chi|^2/E^2 + eps):   |a_gpu - a_ref| <= 1e-5      (peak = 1)
  chi / E:                        |chi_gpu - chi_ref| / E <= 1e-5
  gradients:                      max|g - g_ref| <= 1e-4 max|g_ref|
  loss values:                    relative 1e-4 (float32 sums over 10^6+ cells)
Every case prints its name before touching the GPU.
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
FLOOR_DRAWS = 5  # noise draws behind a float32 conditioning floor (the largest counts)


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def af():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_22935_amd import af as afmod
    return afmod


def to_dev(s):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(s, dtype=np.complex64))).cuda()


def packed(codes):
    return to_dev(np.concatenate(codes))


def ref_c64(s):
    return O.to_c64_exact(s)


def check_grad(g, ref, what):
    err = np.max(np.abs(g - ref))
    scale = np.max(np.abs(ref))
    assert err <= TOL_G * scale, "%s: grad err %.3e vs %.3e" % (what, err, TOL_G * scale)


SHAPES = [
    # (n, m, max_lag): several tiles, ragged lengths, lag windows, M = 4N
    (64, 128, -1),
    (100, 256, 40),
    (37, 128, -1),
    (700, 2048, -1),
    (1024, 2048, -1),
    (300, 2048, 120),
    (1000, 4096, -1),
]


@pytest.mark.parametrize("n,m,T", SHAPES)
def test_forward_magnitude_and_chi(af, n, m, T):
    say("forward", n, m, T)
    s = W.random_code(n, seed=n + m)
    plan = af.Plan([n], [m], [T], eps=EPS)
    mag, chi, e = plan.forward(to_dev(s), mag=True, chi=True)
    torch.cuda.synchronize()
    Tn = n - 1 if T < 0 else T
    sr = ref_c64(s)
    E = O.energy(sr)
    c_ref = O.chi(sr, m, Tn)
    a_ref = O.magnitude(c_ref, E, EPS)
    a = plan.grid(mag, 0).cpu().numpy()
    c = plan.grid(chi, 0).cpu().numpy()
    assert abs(e.item() - E) <= 1e-6 * E
    assert np.max(np.abs(a - a_ref)) <= TOL_A
    assert np.max(np.abs(c - c_ref)) <= TOL_A * E


def fp32_sensitivity(s, m, T, ga, draws=FLOOR_DRAWS):
    """How far the float64 gradient moves when chi carries float32-level
    noise (one unit roundoff of E per cell), the largest over several noise
    draws: the conditioning floor of a magnitude upstream that does not
    vanish where |chi| does."""
    E = O.energy(s)
    c = O.chi(s, m, T)

    def grad(cc):
        p = O.power(cc, E)
        a = np.sqrt(p + EPS)
        return O.grad_from_upstream(s, m, T, ga * cc / (2 * E * E * a), -float(np.sum(ga * p / (E * a))))

    g0 = grad(c)
    worst = 0.0
    for seed in range(draws):
        rng = np.random.default_rng(seed)
        noise = 2.0 ** -24 * E * (rng.standard_normal(c.shape) + 1j * rng.standard_normal(c.shape)) / np.sqrt(2)
        worst = max(worst, float(np.max(np.abs(grad(c + noise) - g0))))
    return worst, g0


BWD_SHAPES = [(64, 128, -1), (700, 2048, -1), (1024, 2048, -1), (100, 256, 40), (1000, 4096, -1)]


@pytest.mark.parametrize("n,m,T", BWD_SHAPES)
@pytest.mark.parametrize("store", [1, 2])
def test_backward_magnitude(af, n, m, T, store):
    # upstream u * a (a user loss whose derivative vanishes with |chi|, e.g.
    # sum w a^2 / 2): well conditioned, so the 1e-4 bar applies
    say("backward", n, m, T, "store" if store == 1 else "recompute")
    s = W.random_code(n, seed=3 * n + m)
    Tn = n - 1 if T < 0 else T
    sr = ref_c64(s)
    a_ref = O.magnitude(O.chi(sr, m, Tn), O.energy(sr), EPS)
    ga = (W.upstream_grid(2 * Tn + 1, m, seed=n) * a_ref).astype(np.float32)
    plan = af.Plan([n], [m], [T], eps=EPS, store_mode=store)
    sd = to_dev(s)
    ws = plan.new_workspace()
    plan.forward(sd, mag=True, ws=ws)
    g = plan.backward(sd, torch.from_numpy(ga.ravel()).cuda(), ws=ws)
    torch.cuda.synchronize()
    ref = O.magnitude_backward(sr, m, Tn, ga.astype(np.float64), EPS)
    check_grad(g.cpu().numpy().astype(np.complex128), ref, "backward %d/%d" % (n, m))


@pytest.mark.parametrize("n,m,T", [(64, 128, -1), (300, 1024, -1)])
def test_backward_random_upstream_within_fp32_conditioning(af, n, m, T):
    # a fully random dL/da: exact zeros of chi (the unimodular zero-lag row
    # vanishes at every even bin when M = 2N) have no float32 phase, so the
    # bar is the oracle's own sensitivity to float32 noise on chi
    say("backward random upstream", n, m, T)
    s = W.random_code(n, seed=3 * n + m)
    Tn = n - 1 if T < 0 else T
    sr = ref_c64(s)
    ga = W.upstream_grid(2 * Tn + 1, m, seed=n)
    floor, ref = fp32_sensitivity(sr, m, Tn, ga.astype(np.float64))
    plan = af.Plan([n], [m], [T], eps=EPS)
    sd = to_dev(s)
    ws = plan.new_workspace()
    plan.forward(sd, mag=False, ws=ws)  # store mode: the backward reads these spectra
    g = plan.backward(sd, torch.from_numpy(ga.ravel()).cuda(), ws=ws)
    torch.cuda.synchronize()
    err = np.max(np.abs(g.cpu().numpy().astype(np.complex128) - ref))
    bar = max(TOL_G * np.max(np.abs(ref)), 2.0 * floor)
    say("  grad err/bar %.3f (floor %.3e)" % (err / bar, floor))
    assert err <= bar, (err, floor)


def test_store_equals_recompute_bitwise(af):
    say("store == recompute")
    n, m = 700, 2048
    s = to_dev(W.random_code(n, seed=5))
    ga = torch.from_numpy(W.upstream_grid(2 * n - 1, m, seed=6).ravel()).cuda()
    outs = []
    for store in (1, 2):
        plan = af.Plan([n], [m], eps=EPS, store_mode=store)
        ws = plan.new_workspace()
        plan.forward(s, mag=False, ws=ws)
        outs.append(plan.backward(s, ga, ws=ws).cpu())
    assert torch.equal(outs[0], outs[1])


LOSSES = [
    dict(w_isl=1.0, w_psl=1.0, temp=0.05),   # the single-waveform workload's loss
    dict(w_isl=1.0, w_psl=0.0, temp=0.05),   # fused ISL pass
    dict(w_isl=0.0, w_psl=1.0, temp=0.1),
]


def softpsl_fp32_floor(s, m, T, lp, draws=FLOOR_DRAWS):
    """Sensitivity of the soft-PSL part of the gradient to float32 noise on
    chi (one unit roundoff of E per cell), the largest over several noise
    draws.  Cells where chi vanishes exactly keep a soft-max weight but have
    no float32 phase.  For a unimodular code at M = 2N that is the zero-lag
    row at every even bin (|chi(0, k)| = |sin(pi k N / M) / sin(pi k / M)|);
    the floor applies to those inputs only, every other case is held to the
    plain bar."""
    if not lp["w_psl"]:
        return 0.0
    pp = O.LossParams(w_isl=0.0, w_psl=lp["w_psl"], temp=lp["temp"], eps=EPS)
    c = O.chi(s, m, T)
    g0 = O.loss_grad_from_chi(s, m, T, c, pp)["g"]
    worst = 0.0
    for seed in range(draws):
        rng = np.random.default_rng(seed)
        noise = 2.0 ** -24 * O.energy(s) * (rng.standard_normal(c.shape) +
                                             1j * rng.standard_normal(c.shape)) / np.sqrt(2)
        g1 = O.loss_grad_from_chi(s, m, T, c + noise, pp)["g"]
        worst = max(worst, float(np.max(np.abs(g1 - g0))))
    return worst


def unimodular_zero_row(s, m):
    """Does the zero-lag row of chi vanish exactly off k = 0?  For a
    constant-modulus code it does at every even bin when M = 2N, the only such
    shape the tests draw."""
    return m == 2 * len(s) and np.allclose(np.abs(s), 1.0, atol=1e-6)


def grad_bar(s, m, T, lp, ref_g):
    """The gradient bar: 1e-4 of max|g_ref|; for unimodular codes at M = 2N
    at least twice the float32 floor of the soft-PSL part."""
    plain = TOL_G * np.max(np.abs(ref_g))
    floor = softpsl_fp32_floor(s, m, T, lp) if unimodular_zero_row(s, m) else 0.0
    return max(plain, 2.0 * floor), floor


# (loss, passes): passes 0 runs one fused pass where the loss allows it, 1
# forces forward + backward; w_psl == 0 always runs the single fused ISL pass
LOSS_CASES = [(LOSSES[0], 0), (LOSSES[0], 1), (LOSSES[1], 0), (LOSSES[2], 0), (LOSSES[2], 1)]


@pytest.mark.parametrize("n,m", [(64, 128), (1024, 2048), (333, 1024)])
@pytest.mark.parametrize("lp,passes", LOSS_CASES)
def test_loss_and_grad(af, n, m, lp, passes):
    say("loss", n, m, lp, passes)
    s = W.random_code(n, seed=7 * n)
    plan = af.Plan([n], [m], h_tau=1, h_k=1, eps=EPS, loss_passes=passes)
    terms, g, _ = plan.loss(to_dev(s), grad=True, **lp)
    torch.cuda.synchronize()
    sr = ref_c64(s)
    ref = O.loss_and_grad(sr, m, n - 1, O.LossParams(h_tau=1, h_k=1, eps=EPS, **lp))
    t = terms.cpu().numpy()[0]
    assert abs(t[0] - ref["loss"]) <= 1e-4 * abs(ref["loss"]) + 1e-6
    assert abs(t[1] - ref["isl"]) <= 1e-4 * abs(ref["isl"])
    if lp["w_psl"]:
        assert abs(t[2] - ref["softpsl"]) <= 1e-5 * max(1.0, abs(ref["softpsl"]))
    err = np.max(np.abs(g.cpu().numpy().astype(np.complex128) - ref["g"]))
    bar, floor = grad_bar(sr, m, n - 1, lp, ref["g"])
    say("  grad err/bar %.3f (err %.3e, bar %.3e, floor %.3e)" % (err / bar, err, bar, floor))
    assert err <= bar, "loss grad err %.3e vs bar %.3e (floor %.3e)" % (err, bar, floor)


# Non-unimodular inputs at the plain bar, no floor: complex Gaussian samples
# leave no AF cell exactly zero, so the soft-PSL gradient is well
# conditioned.  64 x 128, 1024 x 2048 and the M = 8192 class (variant 1).
GAUSS_LOSSES = [dict(w_isl=0.0, w_psl=1.0, temp=0.1), dict(w_isl=1.0, w_psl=1.0, temp=0.05)]
_gauss_ref = {}


def gauss_reference(n, m, li):
    key = (n, m, li)
    if key not in _gauss_ref:
        s = W.complex_gaussian(n, seed=11 * n + m)
        sr = ref_c64(s)
        lp = GAUSS_LOSSES[li]
        _gauss_ref[key] = (s, O.loss_and_grad(sr, m, n - 1, O.LossParams(h_tau=1, h_k=1, eps=EPS, **lp)))
    return _gauss_ref[key]


@pytest.mark.parametrize("n,m", [(64, 128), (1024, 2048), (2500, 8192)])
@pytest.mark.parametrize("li", [0, 1])
@pytest.mark.parametrize("passes", [0, 1])
def test_softpsl_gaussian_plain_bar(af, n, m, li, passes):
    lp = GAUSS_LOSSES[li]
    say("softpsl gaussian", n, m, lp, passes)
    s, ref = gauss_reference(n, m, li)
    plan = af.Plan([n], [m], h_tau=1, h_k=1, eps=EPS, loss_passes=passes)
    terms, g, _ = plan.loss(to_dev(s), grad=True, **lp)
    torch.cuda.synchronize()
    t = terms.cpu().numpy()[0]
    assert abs(t[0] - ref["loss"]) <= 1e-4 * abs(ref["loss"]) + 1e-6
    assert abs(t[2] - ref["softpsl"]) <= 1e-5 * max(1.0, abs(ref["softpsl"]))
    err = np.max(np.abs(g.cpu().numpy().astype(np.complex128) - ref["g"]))
    bar = TOL_G * np.max(np.abs(ref["g"]))
    say("  grad err/bar %.3f (err %.3e, bar %.3e)" % (err / bar, err, bar))
    assert err <= bar, "gaussian loss grad err %.3e vs bar %.3e" % (err, bar)


def loss_vs_oracle(af, plan, codes, ms, Ts, lp, what):
    """plan.loss against the oracle for every waveform of a packed batch."""
    s = packed(codes)
    terms, g, _ = plan.loss(s, grad=True, **lp)
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.complex128)
    t = terms.cpu().numpy()
    for b, (code, m, T) in enumerate(zip(codes, ms, Ts)):
        n = len(code)
        sr = ref_c64(code)
        ref = O.loss_and_grad(sr, m, T, O.LossParams(h_tau=1, h_k=1, eps=EPS, **lp))
        assert abs(t[b, 0] - ref["loss"]) <= 1e-4 * abs(ref["loss"]) + 1e-6, "%s loss %d" % (what, b)
        if lp["w_psl"]:
            assert abs(t[b, 2] - ref["softpsl"]) <= 1e-5 * max(1.0, abs(ref["softpsl"])), "%s softpsl %d" % (what, b)
        gb = g[plan.s_offsets[b]:plan.s_offsets[b] + n]
        err = np.max(np.abs(gb - ref["g"]))
        bar, floor = grad_bar(sr, m, T, lp, ref["g"])
        say("  %s %d: grad err/bar %.3f (floor %.3e)" % (what, b, err / bar, floor))
        assert err <= bar, "%s grad %d: err %.3e bar %.3e" % (what, b, err, bar)


@pytest.mark.parametrize("passes", [0, 1])
def test_isl_softpsl_uneven_batch(af, passes):
    # ISL + soft-PSL over waveforms of several lengths and sizes: the fused
    # pass (second slabs on the mainlobe lags of every waveform) and the
    # forward + backward passes
    say("isl+softpsl uneven", passes)
    ns = [64, 100, 255, 256, 511, 700, 1023, 90]
    ms = [W.next_pow2(2 * n) for n in ns]
    ms[-1] = 4 * ms[-1]
    codes = [W.random_code(n, seed=300 + i) for i, n in enumerate(ns)]
    plan = af.Plan(ns, ms, eps=EPS, loss_passes=passes)
    loss_vs_oracle(af, plan, codes, ms, [n - 1 for n in ns], dict(w_isl=1.0, w_psl=0.5, temp=0.05), "uneven")


def test_softpsl_partial_window_fused(af):
    # soft-PSL alone over a partial lag window: eligible for the fused pass
    # (no ISL part), the grids hold 2T + 1 rows
    say("softpsl partial window")
    ns, Ts = [300, 512], [40, 200]
    ms = [1024, 1024]
    codes = [W.random_code(n, seed=400 + i) for i, n in enumerate(ns)]
    plan = af.Plan(ns, ms, max_lags=Ts, eps=EPS)
    loss_vs_oracle(af, plan, codes, ms, Ts, dict(w_isl=0.0, w_psl=1.0, temp=0.1), "partial")


def test_small_temperature_uses_running_maximum(af):
    # T = 0.01 is below the fixed-shift rule: forward + backward passes with
    # per-iteration maxima
    say("small temperature")
    n, m = 128, 256
    codes = [W.random_code(n, seed=501)]
    plan = af.Plan([n], [m], eps=EPS)
    loss_vs_oracle(af, plan, codes, [m], [n - 1], dict(w_isl=1.0, w_psl=1.0, temp=0.01), "small T")


def test_autotune_picks_a_fitting_variant(af, tmp_path, monkeypatch):
    # two size classes; the tuner times every variant that fits each class
    # and the plan keeps computing the same loss and gradient afterwards
    say("autotune")
    ns, ms = [256, 256, 700], [512, 512, 2048]
    codes = [W.random_code(n, seed=600 + i) for i, n in enumerate(ns)]
    plan = af.Plan(ns, ms, eps=EPS)
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("GRAF_AF_TUNE_CACHE", str(cache))
    v, best = plan.autotune(packed(codes))
    # per class: M = 2048 fits variants 0, 3 and 4; or one launch of both (6)
    assert v in (0, 3, 4, 6) and best > 0.0
    assert plan.summary()["variant"] == v
    loss_vs_oracle(af, plan, codes, ms, [n - 1 for n in ns], dict(w_isl=1.0, w_psl=0.0, temp=0.05), "autotuned")
    # the choice is cached for these shapes: a second plan takes it without
    # timing, and the cache file holds one line for it
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].split()[0].startswith("gfx950")
    again = af.Plan(ns, ms, eps=EPS)
    v2, best2 = again.autotune(packed(codes))
    assert (v2, best2) == (v, best) and again.summary() == plan.summary()
    assert len(cache.read_text().splitlines()) == 1


def test_fused_loss_graph_replay_matches_eager(af):
    # ISL + soft-PSL Adam steps on one waveform through the fused loss pass
    # and the reduce-plus-Adam kernel, captured in a HIP graph (device step
    # counter, exit counter): every replay must equal the eager steps
    say("fused loss graph replay")
    n, m, K = 1024, 2048, 4
    plan = af.Plan([n], [m], eps=EPS)
    phi0 = torch.from_numpy(W.random_phases(n, seed=21).astype(np.float32)).cuda()
    st_e = af.PhaseState(phi0.clone())
    terms_e = torch.empty(1, 4, device="cuda")
    eager = []
    for _ in range(3 * K):
        plan.optim_step(st_e, w_isl=1.0, w_psl=1.0, lr=0.01, terms=terms_e)
        eager.append((st_e.phi.clone(), terms_e.clone()))
    torch.cuda.synchronize()
    st_g = af.PhaseState(phi0.clone())
    terms_g = torch.empty(1, 4, device="cuda")
    ws = plan.workspace
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            for _ in range(K):
                plan.optim_step(st_g, w_isl=1.0, w_psl=1.0, lr=0.01, terms=terms_g, ws=ws)
    torch.cuda.synchronize()
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        phi_e, terms_ref = eager[(rep + 1) * K - 1]
        assert int(st_g.step.item()) == (rep + 1) * K
        assert torch.equal(st_g.phi, phi_e), "replay %d" % rep
        assert torch.equal(terms_g, terms_ref), "replay %d" % rep
        _ = (st_g.phi * 2).sum().item()  # unrelated eager work between replays


def test_fused_pass_matches_two_passes(af):
    # the same loss and gradient from the fused pass (auto) and from forced
    # forward + backward passes
    say("fused vs two passes")
    n, m = 1024, 2048
    s = to_dev(W.random_code(n, seed=31))
    a = af.Plan([n], [m], eps=EPS).loss(s, w_isl=1.0, w_psl=1.0, temp=0.05)
    b = af.Plan([n], [m], eps=EPS, loss_passes=1).loss(s, w_isl=1.0, w_psl=1.0, temp=0.05)
    torch.cuda.synchronize()
    ga, gb = a[1].cpu().numpy(), b[1].cpu().numpy()
    assert np.max(np.abs(ga - gb)) <= 1e-4 * np.max(np.abs(gb))
    assert np.allclose(a[0].cpu().numpy(), b[0].cpu().numpy(), rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("variant", [1, 5, 6])
def test_m8192_variants(af, variant):
    # the kernel variants for M = 8192 (512-thread groups; 32 points per lane
    # with one wave per SIMD; the one-launch kernel): forward, ISL loss and
    # ISL + soft-PSL loss
    say("M=8192 variant", variant)
    ns, m = [300, 1000], 8192
    codes = [W.random_code(n, seed=700 + n) for n in ns]
    plan = af.Plan(ns, [m, m], eps=EPS, variant=variant)
    assert plan.summary()["variant"] == variant
    s = packed(codes)
    mag, _, _ = plan.forward(s, mag=True)
    terms, g, _ = plan.loss(s, w_isl=1.0, w_psl=0.0)
    terms2, g2, _ = plan.loss(s, w_isl=1.0, w_psl=1.0, temp=0.05)
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.complex128)
    g2 = g2.cpu().numpy().astype(np.complex128)
    for b, n in enumerate(ns):
        sr = ref_c64(codes[b])
        ref = O.loss_and_grad(sr, m, n - 1, O.LossParams(eps=EPS))
        assert np.max(np.abs(plan.grid(mag, b).cpu().numpy() - ref["a"])) <= TOL_A, "mag %d" % b
        assert abs(terms[b, 1].item() - ref["isl"]) <= 1e-4 * ref["isl"]
        check_grad(g[plan.s_offsets[b]:plan.s_offsets[b] + n], ref["g"], "M=8192 v%d wave %d" % (variant, b))
        ref2 = O.loss_and_grad(sr, m, n - 1, O.LossParams(eps=EPS, w_isl=1.0, w_psl=1.0, temp=0.05))
        assert abs(terms2[b, 0].item() - ref2["loss"]) <= 1e-4 * abs(ref2["loss"])
        check_grad(g2[plan.s_offsets[b]:plan.s_offsets[b] + n], ref2["g"], "M=8192 psl v%d wave %d" % (variant, b))


def test_weighted_isl_batch(af):
    # descriptor-weighted ISL on a slice of the proposal workload (N=256, M=512)
    say("weighted isl batch")
    B, n, m = 6, 256, 512
    d = W.descriptors(B, seed=11)
    codes = [W.random_code(n, seed=100 + b) for b in range(B)]
    band = np.concatenate([d["u"], d["v"]], axis=1).astype(np.float32)
    plan = af.Plan([n] * B, [m] * B, h_tau=d["h_tau"].tolist(), h_k=d["h_k"].tolist(), eps=EPS)
    terms, g, _ = plan.loss(packed(codes), w_isl=1.0, w_psl=0.0, band_w=torch.from_numpy(band.ravel()).cuda())
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.complex128)
    t = terms.cpu().numpy()
    for b in range(B):
        lp = O.LossParams(w_isl=1.0, w_psl=0.0, h_tau=int(d["h_tau"][b]), h_k=int(d["h_k"][b]),
                          u=d["u"][b].astype(np.float64), v=d["v"][b].astype(np.float64), eps=EPS)
        ref = O.loss_and_grad(ref_c64(codes[b]), m, n - 1, lp)
        assert abs(t[b, 1] - ref["isl"]) <= 1e-4 * ref["isl"]
        check_grad(g[b * n:(b + 1) * n], ref["g"], "weighted %d" % b)


def test_uneven_batch(af):
    say("uneven batch")
    ns = [64, 65, 100, 255, 256, 257, 511, 700, 1023, 1500, 2047, 90]
    ms = [W.next_pow2(2 * n) for n in ns]
    ms[-1] = 4 * ms[-1]  # one waveform with M = 8 N
    codes = [W.random_code(n, seed=200 + i) for i, n in enumerate(ns)]
    plan = af.Plan(ns, ms, eps=EPS)
    s = packed(codes)
    mag, _, e = plan.forward(s, mag=True)
    terms, g, _ = plan.loss(s, w_isl=1.0, w_psl=0.0)
    torch.cuda.synchronize()
    mag = mag.cpu()
    g = g.cpu().numpy().astype(np.complex128)
    t = terms.cpu().numpy()
    for b, (n, m) in enumerate(zip(ns, ms)):
        sr = ref_c64(codes[b])
        ref = O.loss_and_grad(sr, m, n - 1, O.LossParams(eps=EPS))
        a_ref = ref["a"]
        assert np.max(np.abs(plan.grid(mag, b).numpy() - a_ref)) <= TOL_A, "mag %d" % b
        assert abs(t[b, 1] - ref["isl"]) <= 1e-4 * ref["isl"], "isl %d" % b
        check_grad(g[plan.s_offsets[b]:plan.s_offsets[b] + n], ref["g"], "uneven %d" % b)


def test_deterministic(af):
    say("determinism")
    n, m = 1024, 2048
    s = to_dev(W.random_code(n, seed=9))
    plan = af.Plan([n], [m], eps=EPS)
    a = plan.loss(s, w_isl=1.0, w_psl=1.0)
    b = plan.loss(s, w_isl=1.0, w_psl=1.0)
    torch.cuda.synchronize()
    assert torch.equal(a[0].cpu(), b[0].cpu())
    assert torch.equal(a[1].cpu(), b[1].cpu())


def test_optim_step_matches_oracle(af):
    say("optim step")
    n, m = 256, 512
    phi = W.random_phases(n, seed=12).astype(np.float32)
    plan = af.Plan([n], [m], eps=EPS)
    st = af.PhaseState(torch.from_numpy(phi).cuda())
    terms = torch.empty(1, 4, device="cuda")
    plan.optim_step(st, w_isl=1.0, w_psl=1.0, lr=0.01, terms=terms)
    torch.cuda.synchronize()
    s0 = ref_c64(np.exp(1j * phi.astype(np.float64)))
    ref = O.loss_and_grad(s0, m, n - 1, O.LossParams(w_isl=1.0, w_psl=1.0, eps=EPS))
    dphi = O.phase_grad(s0, ref["g"])
    x, _, _ = O.adam_step(phi.astype(np.float64), dphi, np.zeros(n), np.zeros(n), 1, lr=0.01)
    # first Adam step moves every phase by lr * sign(grad) (up to eps)
    got = st.phi.cpu().numpy()
    strong = np.abs(dphi) > 1e-3 * np.max(np.abs(dphi))
    assert np.max(np.abs(got - x)[strong]) <= 1e-5
    assert int(st.step.item()) == 1
    assert abs(terms[0, 0].item() - ref["loss"]) <= 1e-4 * ref["loss"]
    s_new = st.s.cpu().numpy()
    assert np.max(np.abs(s_new - np.exp(1j * got.astype(np.float64)))) <= 1e-6


def test_autograd_magnitude(af):
    say("autograd magnitude")
    from paper_2506_22935_amd.autograd import af_magnitude
    n, m = 128, 256
    s0 = W.random_code(n, seed=13)
    plan = af.Plan([n], [m], eps=EPS)
    s = to_dev(s0).requires_grad_(True)
    a = af_magnitude(s, plan)
    # L = sum u a^2 / 2: dL/da = u a vanishes with |chi| (well conditioned)
    u = torch.from_numpy(W.upstream_grid(2 * n - 1, m, seed=14).ravel()).cuda()
    (0.5 * u * a * a).sum().backward()
    torch.cuda.synchronize()
    sr = ref_c64(s0)
    a_ref = O.magnitude(O.chi(sr, m, n - 1), O.energy(sr), EPS)
    ga = u.cpu().numpy().reshape(2 * n - 1, m).astype(np.float64) * a_ref
    ref = O.magnitude_backward(sr, m, n - 1, ga, EPS)
    check_grad(s.grad.cpu().numpy().astype(np.complex128) / 2, ref, "autograd")


def test_autograd_loss_finite_difference(af):
    say("autograd loss fd")
    from paper_2506_22935_amd.autograd import af_loss
    n, m = 64, 128
    s0 = W.random_code(n, seed=15).astype(np.complex128)
    plan = af.Plan([n], [m], eps=EPS)
    s = to_dev(s0).requires_grad_(True)
    L = af_loss(s, plan, w_isl=1.0, w_psl=1.0)
    L.sum().backward()
    grad = s.grad.cpu().numpy().astype(np.complex128)
    # directional derivative in float64 on the oracle: 2 Re<g_torch/2, d> = dL
    d = np.random.default_rng(16).standard_normal(n) + 1j * np.random.default_rng(17).standard_normal(n)
    h = 1e-4
    lp = O.LossParams(w_isl=1.0, w_psl=1.0, eps=EPS)
    fp = O.loss_terms(O.chi(s0 + h * d, m), O.energy(s0 + h * d), n, lp)["loss"]
    fm = O.loss_terms(O.chi(s0 - h * d, m), O.energy(s0 - h * d), n, lp)["loss"]
    fd = (fp - fm) / (2 * h)
    assert abs(np.real(np.vdot(grad, d)) - fd) <= 1e-3 * abs(fd)


@pytest.mark.parametrize("bad", [dict(n=100, m=128), dict(n=64, m=100), dict(n=64, m=64)])
def test_plan_rejects_bad_shapes(af, bad):
    from paper_2506_22935_amd import _lib
    with pytest.raises(_lib.AfError) as ei:
        af.Plan([bad["n"]], [bad["m"]])
    assert ei.value.code == -2

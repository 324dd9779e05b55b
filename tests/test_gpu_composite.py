"""L_match of the composite loss (Sec. 5.2) on the HIP path against the
oracle (GPU): the AF in power matched to a target surface over every cell,
alone and with ISL and the hard PSL, on the aperiodic and the periodic AF."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
from paper_2506_22935_amd import workloads as W

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


def to_dev(s):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(s, dtype=np.complex64))).cuda()


def check_grad(g, ref, what):
    err = np.max(np.abs(g - ref))
    assert err <= 1e-4 * np.max(np.abs(ref)), "%s: grad err %.3e vs %.3e" % (what, err, np.max(np.abs(ref)))


@pytest.mark.parametrize("n,m,T,periodic", [(100, 256, -1, False), (300, 1024, 40, False), (128, 128, -1, True),
                                            (1024, 2048, -1, False)])
@pytest.mark.parametrize("w_isl", [0.0, 1.0])
def test_match_loss_and_gradient(af, n, m, T, periodic, w_isl):
    say("match", n, m, T, periodic, w_isl)
    s = W.random_code(n, seed=1000 + n)
    Tn = n - 1 if T < 0 else T
    rows = n if periodic else 2 * Tn + 1
    target = np.random.default_rng(n + Tn).uniform(0.0, 0.01, (rows, m)).astype(np.float32)
    plan = af.Plan([n], [m], [T], eps=EPS, periodic=periodic)
    terms, g, _ = plan.loss(to_dev(s), w_isl=w_isl, w_psl=0.0, match=torch.from_numpy(target.ravel()).cuda(),
                            w_match=3.0)
    torch.cuda.synchronize()
    sr = O.to_c64_exact(s)
    params = O.LossParams(w_isl=w_isl, eps=EPS, match=target.astype(np.float64), w_match=3.0)
    ref = O.loss_and_grad_circular(sr, params) if periodic else O.loss_and_grad(sr, m, Tn, params)
    assert abs(terms[0, 0].item() - ref["loss"]) <= 1e-4 * ref["loss"], (terms[0, 0].item(), ref["loss"])
    check_grad(g.cpu().numpy().astype(np.complex128), ref["g"], "match %d %d" % (n, m))


def test_match_with_hard_psl_and_value_only(af):
    say("match + hard PSL")
    n, m = 128, 256
    for seed in range(1100, 1150):
        s = W.random_code(n, seed=seed)
        sr = O.to_c64_exact(s)
        c = O.chi(sr, m)
        p = O.power(c, O.energy(sr))
        side = ~O.mainlobe_mask(m, n - 1, 1, 1)
        top = np.sort(np.unique(np.round(p[side], 9)))
        if top[-1] - top[-2] > 1e-4 * top[-1]:
            break
    target = np.random.default_rng(5).uniform(0.0, 0.01, p.shape).astype(np.float32)
    plan = af.Plan([n], [m], eps=EPS)
    kw = dict(w_isl=0.5, w_psl=1.0, psl_hard=True, match=torch.from_numpy(target.ravel()).cuda(), w_match=2.0)
    terms, g, _ = plan.loss(to_dev(s), grad=True, **kw)
    terms0, _, _ = plan.loss(to_dev(s), grad=False, **kw)
    torch.cuda.synchronize()
    base = O.loss_and_grad(sr, m, n - 1, O.LossParams(w_isl=0.5, eps=EPS, match=target.astype(np.float64),
                                                      w_match=2.0))
    ex = O.experiment_loss_and_grad(sr, m, 0.0, h_tau=1, h_k=1, eps=EPS)
    for tt in (terms, terms0):
        assert abs(tt[0, 0].item() - (base["loss"] + ex["psl"])) <= 1e-4 * tt[0, 0].item()
    check_grad(g.cpu().numpy().astype(np.complex128), base["g"] + ex["g"], "match + hard PSL")


def test_match_at_its_own_surface_and_rejections(af):
    say("match own surface")
    from paper_2506_22935_amd import _lib
    n, m = 256, 512
    s = W.random_code(n, seed=1200)
    sr = O.to_c64_exact(s)
    p = O.power(O.chi(sr, m), O.energy(sr)).astype(np.float32)
    plan = af.Plan([n], [m], eps=EPS)
    tgt = torch.from_numpy(p.ravel()).cuda()
    terms, g, _ = plan.loss(to_dev(s), w_isl=0.0, match=tgt, w_match=1.0)
    torch.cuda.synchronize()
    # float32 AF against its float64 surface: only roundoff remains
    assert terms[0, 0].item() <= 1e-9 * p.size
    # L_match with the soft PSL is not a supported combination
    with pytest.raises(_lib.AfError) as ei:
        plan.loss(to_dev(s), w_isl=0.0, w_psl=1.0, match=tgt, w_match=1.0)
    assert ei.value.code == -2


def rand_c64(n, seed, modulated=True):
    rng = np.random.default_rng(seed)
    s = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    if not modulated:
        s = np.exp(1j * np.angle(s))
    return O.to_c64_exact(s / np.sqrt(2.0))


@pytest.mark.parametrize("n,m,T,periodic", [(100, 256, -1, False), (300, 1024, 40, False), (128, 128, -1, True),
                                            (1024, 2048, -1, False), (256, 256, -1, True)])
@pytest.mark.parametrize("w_isl", [0.0, 1.0])
def test_soft_width_loss_and_gradient(af, n, m, T, periodic, w_isl):
    say("width", n, m, T, periodic, w_isl)
    s = rand_c64(n, 1300 + n)
    Tn = n - 1 if T < 0 else T
    plan = af.Plan([n], [m], [T], eps=EPS, periodic=periodic)
    terms, g, _ = plan.loss(to_dev(s), w_isl=w_isl, w_psl=0.0, w_width=0.5, gamma=8.0)
    terms0, _, _ = plan.loss(to_dev(s), w_isl=w_isl, w_psl=0.0, w_width=0.5, gamma=8.0, grad=False)
    torch.cuda.synchronize()
    params = O.LossParams(w_isl=w_isl, eps=EPS, w_width=0.5, gamma=8.0)
    ref = O.loss_and_grad_circular(s, params) if periodic else O.loss_and_grad(s, m, Tn, params)
    for tt in (terms, terms0):
        assert abs(tt[0, 0].item() - ref["loss"]) <= 1e-4 * ref["loss"], (tt[0, 0].item(), ref["loss"])
    check_grad(g.cpu().numpy().astype(np.complex128), ref["g"], "width %d %d" % (n, m))


@pytest.mark.parametrize("n,m,T,periodic", [(200, 512, -1, False), (256, 256, -1, True)])
def test_every_composite_term_together(af, n, m, T, periodic):
    say("all terms", n, m, periodic)
    s = rand_c64(n, 1400 + n)
    Tn = n - 1
    rows = n if periodic else 2 * Tn + 1
    target = np.random.default_rng(7).uniform(0.0, 0.02, (rows, m)).astype(np.float32)
    plan = af.Plan([n], [m], [T], eps=EPS, periodic=periodic)
    kw = dict(w_isl=0.3, w_psl=1.0, psl_hard=True, match=torch.from_numpy(target.ravel()).cuda(), w_match=2.0,
              w_width=0.25, gamma=5.0, w_const=1.5, w_smooth=0.75)
    terms, g, _ = plan.loss(to_dev(s), **kw)
    torch.cuda.synchronize()
    params = O.LossParams(w_isl=0.3, eps=EPS, match=target.astype(np.float64), w_match=2.0, w_width=0.25,
                          gamma=5.0, w_const=1.5, w_smooth=0.75)
    base = O.loss_and_grad_circular(s, params) if periodic else O.loss_and_grad(s, m, Tn, params)
    ex = O.experiment_loss_and_grad(s, m, 0.0, h_tau=1, h_k=1, periodic=periodic, eps=EPS)
    want = base["loss"] + ex["psl"]
    assert abs(terms[0, 0].item() - want) <= 1e-4 * want, (terms[0, 0].item(), want)
    check_grad(g.cpu().numpy().astype(np.complex128), base["g"] + ex["g_psl"], "all terms")


@pytest.mark.parametrize("sizes,ms,Ts", [([100, 37, 512], [256, 128, 1024], [-1, -1, 60]),
                                         ([9000], [32768], [100])])
def test_waveform_terms_any_class(af, sizes, ms, Ts):
    # var(|s|) and the smoothness term alone: no AF gradient, any size class
    # (the N = 9000 plan runs the halves-in-turn variant)
    say("const + smooth", sizes)
    ss = [rand_c64(n, 1500 + n) for n in sizes]
    plan = af.Plan(sizes, ms, Ts, eps=EPS)
    terms, g, _ = plan.loss(to_dev(np.concatenate(ss)), w_isl=0.0, w_const=1.5, w_smooth=0.75)
    torch.cuda.synchronize()
    gg = g.cpu().numpy().astype(np.complex128)
    off = 0
    for b, s in enumerate(ss):
        vc, gc = O.modulus_variance(s)
        vs, gs = O.phase_smoothness(s)
        want = 1.5 * vc + 0.75 * vs
        assert abs(terms[b, 0].item() - want) <= 1e-4 * want, (b, terms[b, 0].item(), want)
        check_grad(gg[off:off + len(s)], 1.5 * gc + 0.75 * gs, "const+smooth %d" % len(s))
        off += len(s)


def test_waveform_terms_in_the_adam_step(af):
    # one Adam step on the phases of the ISL + smoothness loss against the
    # oracle's gradient through phi and its Adam step
    say("adam smooth")
    n, m = 128, 256
    phi = np.random.default_rng(9).uniform(-np.pi, np.pi, n).astype(np.float32)
    plan = af.Plan([n], [m], eps=EPS)
    st = af.PhaseState(torch.from_numpy(phi).cuda())
    plan.optim_step(st, w_isl=1.0, w_smooth=2.0, lr=0.01)
    torch.cuda.synchronize()
    s = np.exp(1j * phi.astype(np.float64))
    ref = O.loss_and_grad(s, m, n - 1, O.LossParams(w_isl=1.0, eps=EPS, w_smooth=2.0))
    gphi = O.phase_grad(s, ref["g"])
    want, _, _ = O.adam_step(phi.astype(np.float64), gphi, np.zeros(n), np.zeros(n), 1)
    # the first Adam step moves each phase by lr sign(g) (up to eps): compare
    # where the gradient is clear of zero, and bound the step everywhere
    got = st.phi.cpu().numpy().astype(np.float64)
    clear = np.abs(gphi) > 1e-3 * np.max(np.abs(gphi))
    assert clear.sum() > n // 2
    assert np.max(np.abs(got - want)[clear]) < 1e-5
    assert np.max(np.abs(got - phi)) <= 0.01 * (1 + 1e-4)


@pytest.mark.parametrize("unit", [False, True])
def test_spectral_projection(af, unit):
    say("projection", unit)
    sizes = [100, 37, 512, 1]
    ss = [rand_c64(n, 1600 + n) for n in sizes]
    masks = []
    for n in sizes:
        k = np.arange(n)
        kc = np.abs(np.where(k < (n + 1) // 2, k, k - n))
        masks.append(np.where(kc <= n // 5, 1.0, np.where(kc <= n // 4, 0.5, 0.0)).astype(np.float32))
    plan = af.Plan(sizes, [256, 128, 1024, 128], eps=EPS)
    sd = to_dev(np.concatenate(ss))
    md = torch.from_numpy(np.concatenate(masks)).cuda()
    out = plan.project(sd, md, unit=unit)
    inplace = sd.clone()
    plan.project(inplace, md, unit=unit, out=inplace)
    uonly = plan.project(sd, None, unit=True)
    torch.cuda.synchronize()
    o, ip, uo = (x.cpu().numpy().astype(np.complex128) for x in (out, inplace, uonly))
    assert np.array_equal(o, ip)
    off = 0
    for s, mk in zip(ss, masks):
        y = O.spectral_projection(s, mk.astype(np.float64))
        got = o[off:off + len(s)]
        if unit:
            # directions agree where the projected sample is clear of zero
            clear = np.abs(y) > 1e-2 * np.max(np.abs(y))
            assert np.max(np.abs(np.abs(got) - 1.0)) < 1e-6
            assert np.max(np.abs(got[clear] - y[clear] / np.abs(y[clear]))) < 1e-4, len(s)
        else:
            assert np.max(np.abs(got - y)) <= 1e-5 * np.max(np.abs(y)), len(s)
        assert np.max(np.abs(uo[off:off + len(s)] - s / np.abs(s))) < 1e-6
        off += len(s)


def test_new_terms_rejections(af):
    from paper_2506_22935_amd import _lib
    n, m = 128, 256
    plan = af.Plan([n], [m], eps=EPS)
    s = to_dev(rand_c64(n, 1))
    with pytest.raises(_lib.AfError) as ei:
        plan.loss(s, w_isl=0.0, w_psl=1.0, w_width=1.0)  # the width with the soft PSL
    assert ei.value.code == -2
    with pytest.raises(_lib.AfError) as ei:
        plan.loss(s, w_isl=1.0, w_width=1.0, gamma=-1.0)
    assert ei.value.code == -1
    big = af.Plan([5000], [16384], [100], eps=EPS)
    with pytest.raises(_lib.AfError) as ei:
        big.project(to_dev(rand_c64(5000, 2)), torch.ones(5000, device="cuda"))  # mask beyond N = 4096
    assert ei.value.code == -2


@pytest.mark.parametrize("n,m,periodic", [(100, 256, False), (128, 128, True), (1000, 2048, False)])
def test_multi_scenario_weights(af, n, m, periodic):
    # Eq. 24 over three target-profile scenarios: the GPU combines the grids
    # once and runs one pass; the oracle sums the scenario losses one by one
    say("multi-scenario", n, m, periodic)
    s = rand_c64(n, 1700 + n)
    T = n - 1
    rows, cols = (n, n) if periodic else (2 * T + 1, m)
    rng = np.random.default_rng(n)
    grids = [(rng.uniform(0, 1, (rows, cols)) * (rng.uniform(0, 1, (rows, 1)) < 0.4)).astype(np.float32)
             for _ in range(3)]
    lams = np.array([0.5, 2.0, 1.25], dtype=np.float32)
    plan = af.Plan([n], [m], eps=EPS, periodic=periodic)
    comb = plan.scenario_combine(torch.from_numpy(np.stack([g.ravel() for g in grids])).cuda(),
                                 torch.from_numpy(lams).cuda())
    terms, g, _ = plan.loss(to_dev(s), w_isl=0.0, cell_w=comb, w_cell=1.0)
    terms_h, g_h, _ = plan.loss(to_dev(s), w_isl=0.0, w_psl=1.0, psl_hard=True, cell_w=comb, w_cell=1.0)
    torch.cuda.synchronize()
    ref_comb = O.combine_scenario_weights([g_.astype(np.float64) for g_ in grids], lams.astype(np.float64))
    assert np.max(np.abs(comb.cpu().numpy().reshape(rows, cols) - ref_comb)) <= 1e-6 * np.max(ref_comb)
    scen = [O.LossParams(w_isl=0.0, eps=EPS, cell_w=g_.astype(np.float64), w_cell=1.0) for g_ in grids]
    L, gref = O.multi_scenario_loss_and_grad(s, m, T, scen, lams.astype(np.float64), periodic=periodic)
    assert abs(terms[0, 0].item() - L) <= 1e-4 * L, (terms[0, 0].item(), L)
    check_grad(g.cpu().numpy().astype(np.complex128), gref, "multi-scenario")
    # with the hard PSL of the experiment loss on top
    ex = O.experiment_loss_and_grad(s, m, 0.0, h_tau=1, h_k=1, periodic=periodic, eps=EPS)
    assert abs(terms_h[0, 0].item() - (L + ex["psl"])) <= 1e-4 * (L + ex["psl"])
    check_grad(g_h.cpu().numpy().astype(np.complex128), gref + ex["g_psl"], "multi-scenario + hard PSL")


def test_cell_weights_rejections(af):
    from paper_2506_22935_amd import _lib
    plan = af.Plan([128], [256], eps=EPS)
    s = to_dev(rand_c64(128, 3))
    w = torch.ones(255 * 256, dtype=torch.float32, device="cuda")
    with pytest.raises(_lib.AfError) as ei:
        plan.loss(s, w_isl=0.0, w_psl=1.0, cell_w=w, w_cell=1.0)  # with the soft PSL
    assert ei.value.code == -2
    with pytest.raises(_lib.AfError) as ei:
        plan.loss(s, w_isl=0.0, w_cell=1.0)  # weight without a grid
    assert ei.value.code == -1


def unique_max_code(n, m, T, seed0):
    # a code whose largest sidelobe power is unique (the hard PSL's cell is
    # then the same for float32 and float64)
    side = ~O.mainlobe_mask(m, T, 1, 1)
    for seed in range(seed0, seed0 + 40):
        s = rand_c64(n, seed)
        c = O.chi(s, m, T)
        p = O.power(c, O.energy(s))
        top = np.sort(np.unique(np.round(p[side], 9)))
        if top[-1] - top[-2] > 1e-4 * top[-1]:
            return s, c, side
    raise AssertionError("no code with a unique maximum")


@pytest.mark.parametrize("n,m,T", [(600, 16384, 20), (1500, 32768, 10)])
def test_hard_psl_alone_halves_in_turn(af, n, m, T):
    # the forward pass alone records the maximum (the extended forward
    # instance of the 1024-thread halves-in-turn variant); its gradient is
    # the single-cell adjoint
    say("hard PSL halves in turn", n, m, T)
    s, c, side = unique_max_code(n, m, T, 2200)
    E = O.energy(s)
    plan = af.Plan([n], [m], [T], eps=EPS)
    assert plan.summary()["variant"] == 2
    terms, g, _ = plan.loss(to_dev(s), w_isl=0.0, w_psl=1.0, psl_hard=True)
    torch.cuda.synchronize()
    psl, cell = O.hard_psl(c, E, side)
    G = np.zeros_like(c)
    G[cell] = c[cell] / (E * E)
    g_psl = O.grad_from_upstream(s, m, T, G, -2.0 * psl / E)
    assert abs(terms[0, 0].item() - psl) <= 1e-4 * psl, (terms[0, 0].item(), psl)
    check_grad(g.cpu().numpy().astype(np.complex128), g_psl, "hard PSL M = %d" % m)


@pytest.mark.parametrize("variant,n,m,T", [(0, 300, 1024, 40), (3, 300, 1024, 40), (4, 1500, 4096, 30),
                                           (1, 3000, 8192, 20), (5, 3000, 8192, 20), (2, 600, 16384, 20),
                                           (2, 1500, 32768, 10)])
def test_extended_terms_every_variant(af, variant, n, m, T):
    # every extended term at once (hard PSL, L_match, width, cell weights,
    # var(|s|), smoothness, ISL) on each variant's extended instances, with
    # a lag window (variant 2: the halves-in-turn variant of M >= 16384)
    say("extended terms variant", variant, n, m, T)
    rows = 2 * T + 1
    side = ~O.mainlobe_mask(m, T, 1, 1)
    for seed in range(2100, 2140):
        s = rand_c64(n, seed)
        c = O.chi(s, m, T)
        E = O.energy(s)
        p = O.power(c, E)
        top = np.sort(np.unique(np.round(p[side], 9)))
        if top[-1] - top[-2] > 1e-4 * top[-1]:
            break
    rng = np.random.default_rng(variant)
    target = rng.uniform(0, 2e-3, (rows, m)).astype(np.float32)
    cellw = (rng.uniform(0, 1, (rows, m)) * (rng.uniform(0, 1, (rows, 1)) < 0.3)).astype(np.float32)
    plan = af.Plan([n], [m], [T], eps=EPS, variant=variant)
    assert plan.summary()["variant"] == variant
    kw = dict(w_isl=0.3, w_psl=1.0, psl_hard=True, match=torch.from_numpy(target.ravel()).cuda(), w_match=5.0,
              w_width=0.2, gamma=5.0, cell_w=torch.from_numpy(cellw.ravel()).cuda(), w_cell=0.5, w_const=1.0,
              w_smooth=0.5)
    terms, g, _ = plan.loss(to_dev(s), **kw)
    torch.cuda.synchronize()
    params = O.LossParams(w_isl=0.3, eps=EPS, match=target.astype(np.float64), w_match=5.0, w_width=0.2, gamma=5.0,
                          cell_w=cellw.astype(np.float64), w_cell=0.5, w_const=1.0, w_smooth=0.5)
    base = O.loss_grad_from_chi(s, m, T, c, params)
    psl, cell = O.hard_psl(c, E, side)
    G = np.zeros_like(c)
    G[cell] = c[cell] / (E * E)
    g_psl = O.grad_from_upstream(s, m, T, G, -2.0 * psl / E)
    want = base["loss"] + psl
    assert abs(terms[0, 0].item() - want) <= 1e-4 * want, (terms[0, 0].item(), want)
    check_grad(g.cpu().numpy().astype(np.complex128), base["g"] + g_psl, "variant %d" % variant)

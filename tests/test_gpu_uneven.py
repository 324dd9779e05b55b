"""Uneven batches in one plan: every Doppler size class in one persistent
launch over one work queue (the default), or one launch per class with the
classes concurrent; the optimiser step and its HIP-graph capture (GPU only).

The batch is the uneven workload: 512 random-phase codes, N log-uniform in
[64, 4096] (seed 0), M = next power of two >= 2N, full lag grid each, ISL.
"""
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


@pytest.fixture(scope="module")
def batch(af):
    ns, ms, phases = W.uneven_batch(512, seed=0)
    codes = [W.unimodular(p) for p in phases]
    plan = af.Plan(ns.tolist(), ms.tolist(), eps=EPS)
    s = torch.from_numpy(np.concatenate(codes)).cuda()
    return dict(ns=ns, ms=ms, phases=phases, codes=codes, plan=plan, s=s)


def isl_grad_fft(s, m):
    """Oracle ISL (uniform weights, mainlobe 1x1) and its gradient through
    the FFT-step route: dISL/da = 2 W a turns magnitude_backward into the
    ISL adjoint (W chi / E^2 per cell)."""
    n = len(s)
    T = n - 1
    E = O.energy(s)
    W_ = O.isl_weights(n, m, T, 1, 1)
    rows = O.chi_rows_fft(s, m, range(-T, T + 1))
    a = O.magnitude(rows, E, EPS)
    isl = float(np.sum(W_ * O.power(rows, E)))
    g = O.magnitude_backward_fft(s, m, T, 2.0 * W_ * a, EPS)
    return isl, g


def test_uneven_full_batch_sampled_parity(af, batch):
    say("uneven full batch")
    plan, s = batch["plan"], batch["s"]
    terms, g, _ = plan.loss(s, w_isl=1.0, w_psl=0.0)
    torch.cuda.synchronize()
    terms = terms.cpu().numpy()
    g = g.cpu().numpy().astype(np.complex128)
    ns, ms = batch["ns"], batch["ms"]
    # direct oracle on the shortest waveforms, FFT-step oracle on a long one
    order = np.argsort(ns)
    picks = list(order[:4]) + [order[len(order) // 2], order[-1]]
    for b in picks:
        n, m = int(ns[b]), int(ms[b])
        sr = O.to_c64_exact(batch["codes"][b])
        if n <= 300:
            ref = O.loss_and_grad(sr, m, n - 1, O.LossParams(eps=EPS))
            isl, gref = ref["isl"], ref["g"]
        else:
            isl, gref = isl_grad_fft(sr, m)
        gb = g[plan.s_offsets[b]:plan.s_offsets[b] + n]
        assert abs(terms[b, 1] - isl) <= 1e-4 * isl, (b, n, terms[b, 1], isl)
        assert np.max(np.abs(gb - gref)) <= 1e-4 * np.max(np.abs(gref)), (b, n)
    # every waveform: the normalised loss is scale and phase invariant, so
    # sum conj(s) g = 0 (a property that holds at any size)
    s_np = s.cpu().numpy().astype(np.complex128)
    for b in range(len(ns)):
        o, n = plan.s_offsets[b], int(ns[b])
        sb, gb = s_np[o:o + n], g[o:o + n]
        assert abs(np.vdot(sb, gb)) <= 1e-3 * np.linalg.norm(sb) * np.linalg.norm(gb), b


def test_graph_replay_matches_eager(af):
    say("graph replay")
    ns, ms, phases = W.uneven_batch(48, seed=3)
    plan = af.Plan(ns.tolist(), ms.tolist(), eps=EPS)
    phi0 = torch.from_numpy(np.concatenate(phases).astype(np.float32)).cuda()
    K = 5
    # eager reference
    st_e = af.PhaseState(phi0.clone())
    terms_e = torch.empty(plan.batch, 4, device="cuda")
    for _ in range(2 * K):
        plan.optim_step(st_e, w_isl=1.0, lr=0.01, terms=terms_e)
    torch.cuda.synchronize()
    # captured: K steps per graph, replayed twice with eager work in between
    st_g = af.PhaseState(phi0.clone())
    terms_g = torch.empty(plan.batch, 4, device="cuda")
    ws = plan.workspace
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            for _ in range(K):
                plan.optim_step(st_g, w_isl=1.0, lr=0.01, terms=terms_g, ws=ws)
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    _ = (st_g.phi * 2).sum().item()  # unrelated eager work between replays
    g.replay()
    torch.cuda.synchronize()
    assert int(st_g.step.item()) == 2 * K
    assert torch.equal(st_g.phi, st_e.phi)
    assert torch.equal(st_g.s, st_e.s)
    assert torch.equal(terms_g, terms_e)


def test_adam_steps_decrease_isl(af):
    say("adam decreases isl")
    ns, ms, phases = W.uneven_batch(16, seed=4)
    plan = af.Plan(ns.tolist(), ms.tolist(), eps=EPS)
    st = af.PhaseState(torch.from_numpy(np.concatenate(phases).astype(np.float32)).cuda())
    terms = torch.empty(plan.batch, 4, device="cuda")
    plan.optim_step(st, w_isl=1.0, lr=0.01, terms=terms)
    first = terms[:, 1].clone()
    for _ in range(50):
        plan.optim_step(st, w_isl=1.0, lr=0.01, terms=terms)
    torch.cuda.synchronize()
    assert bool((terms[:, 1] < first).all())
    # the device loss terms agree with the oracle at the final phases
    phi = st.phi.cpu().numpy().astype(np.float64)
    b = int(np.argmin(ns))
    o, n, m = plan.s_offsets[b], int(ns[b]), int(ms[b])
    sr = O.to_c64_exact(np.exp(1j * phi[o:o + n]))
    plan.loss(st.s, w_isl=1.0, out_terms=terms, grad=False)
    torch.cuda.synchronize()
    ref = O.loss_and_grad(sr, m, n - 1, O.LossParams(eps=EPS))
    assert abs(terms[b, 1].item() - ref["isl"]) <= 1e-4 * ref["isl"]


def small_uneven(af, count, seed, **kw):
    ns, ms, phases = W.uneven_batch(count, seed=seed)
    codes = [W.unimodular(p) for p in phases]
    plan = af.Plan(ns.tolist(), ms.tolist(), eps=EPS, **kw)
    return ns, ms, codes, plan, torch.from_numpy(np.concatenate(codes)).cuda()


def test_one_launch_matches_per_class_and_oracle(af):
    # the default plan of an uneven batch is one launch of the one-launch
    # kernel (variant 6); per-class launches give the same loss and gradient
    # up to float32 summation order, and both match the oracle
    say("one launch vs per class")
    ns, ms, codes, one, s = small_uneven(af, 40, 7)
    assert len(set(ms.tolist())) > 2
    assert one.summary()["variant"] == 6
    per = af.Plan(ns.tolist(), ms.tolist(), eps=EPS, one_launch=False)
    assert per.summary()["variant"] != 6
    lp = dict(w_isl=1.0, w_psl=1.0, temp=0.05)
    t1, g1, a1 = one.loss(s, grad=True, mag=True, **lp)
    t2, g2, a2 = per.loss(s, grad=True, mag=True, **lp)
    torch.cuda.synchronize()
    t1, t2 = t1.cpu().numpy(), t2.cpu().numpy()
    g1 = g1.cpu().numpy().astype(np.complex128)
    g2 = g2.cpu().numpy().astype(np.complex128)
    assert np.allclose(t1, t2, rtol=1e-5, atol=1e-6)
    assert float((a1 - a2).abs().max()) <= 1e-6
    for b in range(len(ns)):
        o, n = one.s_offsets[b], int(ns[b])
        gb1, gb2 = g1[o:o + n], g2[o:o + n]
        assert np.max(np.abs(gb1 - gb2)) <= 1e-5 * np.max(np.abs(gb2)), b
    order = np.argsort(ns)
    for b in list(order[:3]) + [order[-1]]:
        n, m = int(ns[b]), int(ms[b])
        if n > 700:
            continue
        ref = O.loss_and_grad(O.to_c64_exact(codes[b]), m, n - 1,
                              O.LossParams(eps=EPS, h_tau=1, h_k=1, w_isl=1.0, w_psl=1.0, temp=0.05))
        assert abs(t1[b, 0] - ref["loss"]) <= 1e-4 * abs(ref["loss"])
        o = one.s_offsets[b]
        assert np.max(np.abs(g1[o:o + n] - ref["g"])) <= 1e-4 * np.max(np.abs(ref["g"])), b


def test_one_launch_largest_size_edges(af):
    # the largest transform (M = 8192) stages its samples unpadded and clamps
    # the lag product's index: N = M/2 (every shifted index past the samples
    # is clamped), the smallest N of that size, and N between, beside sizes
    # whose stride-256 pass reads the pass table at a stride (M = 1024, 2048)
    say("one launch, M = 8192 edges")
    ns = [4096, 2049, 3001, 500, 1000, 64]
    ms = [8192, 8192, 8192, 1024, 2048, 128]
    codes = [W.random_code(n, seed=970 + i) for i, n in enumerate(ns)]
    s = torch.from_numpy(np.concatenate(codes)).cuda()
    one = af.Plan(ns, ms, eps=EPS)
    per = af.Plan(ns, ms, eps=EPS, one_launch=False)
    assert one.summary()["variant"] == 6 and per.summary()["variant"] != 6
    lp = dict(w_isl=1.0, w_psl=1.0, temp=0.05)
    t1, g1, a1 = one.loss(s, grad=True, mag=True, **lp)
    t2, g2, a2 = per.loss(s, grad=True, mag=True, **lp)
    torch.cuda.synchronize()
    assert np.allclose(t1.cpu().numpy(), t2.cpu().numpy(), rtol=1e-5, atol=1e-6)
    assert float((a1 - a2).abs().max()) <= 1e-6
    g1 = g1.cpu().numpy().astype(np.complex128)
    g2 = g2.cpu().numpy().astype(np.complex128)
    for b, n in enumerate(ns):
        o = one.s_offsets[b]
        assert np.max(np.abs(g1[o:o + n] - g2[o:o + n])) <= 1e-5 * np.max(np.abs(g2[o:o + n])), b
    # the sizes the oracle runs in seconds, against the oracle
    t1 = t1.cpu().numpy()
    for b in (3, 5):
        n, m = ns[b], ms[b]
        ref = O.loss_and_grad(O.to_c64_exact(codes[b]), m, n - 1,
                              O.LossParams(eps=EPS, h_tau=1, h_k=1, w_isl=1.0, w_psl=1.0, temp=0.05))
        assert abs(t1[b, 0] - ref["loss"]) <= 1e-4 * abs(ref["loss"])
        o = one.s_offsets[b]
        assert np.max(np.abs(g1[o:o + n] - ref["g"])) <= 1e-4 * np.max(np.abs(ref["g"])), b


@pytest.mark.parametrize("mmax", [2048, 4096])
def test_one_launch_smaller_largest_size(af, mmax):
    # plans whose largest M is 2048 or 4096: the stride-256 pass table holds
    # only the entries those sizes read (whole indices of the plan's table)
    say("one launch, largest M", mmax)
    ns = [mmax // 2, mmax // 4 - 3, 300, 100, 40]
    ms = [mmax, mmax // 2, 1024, 256, 128]
    codes = [W.random_code(n, seed=990 + i) for i, n in enumerate(ns)]
    s = torch.from_numpy(np.concatenate(codes)).cuda()
    one = af.Plan(ns, ms, eps=EPS)
    per = af.Plan(ns, ms, eps=EPS, one_launch=False)
    assert one.summary()["variant"] == 6 and per.summary()["variant"] != 6
    t1, g1, a1 = one.loss(s, w_isl=1.0, grad=True, mag=True)
    t2, g2, a2 = per.loss(s, w_isl=1.0, grad=True, mag=True)
    torch.cuda.synchronize()
    assert np.allclose(t1.cpu().numpy(), t2.cpu().numpy(), rtol=1e-5, atol=1e-6)
    assert float((a1 - a2).abs().max()) <= 1e-6
    g1 = g1.cpu().numpy().astype(np.complex128)
    g2 = g2.cpu().numpy().astype(np.complex128)
    for b, n in enumerate(ns):
        o = one.s_offsets[b]
        assert np.max(np.abs(g1[o:o + n] - g2[o:o + n])) <= 1e-5 * np.max(np.abs(g2[o:o + n])), b


def test_one_launch_is_deterministic(af):
    # work groups take items by atomic ticket, so the assignment changes from
    # run to run; every item writes its own slab and record, so the results
    # may not
    say("one launch deterministic")
    ns, ms, codes, plan, s = small_uneven(af, 64, 9)
    assert plan.summary()["variant"] == 6
    outs = []
    for _ in range(3):
        t, g, _ = plan.loss(s, w_isl=1.0, grad=True)
        outs.append((t.cpu(), g.cpu()))
    torch.cuda.synchronize()
    for t, g in outs[1:]:
        assert torch.equal(t, outs[0][0]) and torch.equal(g, outs[0][1])


def test_one_launch_periodic_sizes(af):
    # periodic waveforms of five sizes (N = M = 64 ... 4096) in one launch,
    # ISL + soft-PSL against the oracle's periodic loss
    say("one launch periodic")
    ns = [64, 4096, 128, 256, 1024, 64, 512]
    codes = [W.complex_gaussian(n, seed=900 + i) for i, n in enumerate(ns)]
    plan = af.Plan(ns, ns, eps=EPS, periodic=True)
    assert plan.summary()["variant"] == 6
    s = torch.from_numpy(np.concatenate(codes)).cuda()
    lp = dict(w_isl=1.0, w_psl=1.0, temp=0.05)
    t, g, _ = plan.loss(s, grad=True, **lp)
    torch.cuda.synchronize()
    t = t.cpu().numpy()
    g = g.cpu().numpy().astype(np.complex128)
    for b, n in enumerate(ns):
        if n > 1024:
            continue
        ref = O.loss_and_grad_circular(O.to_c64_exact(codes[b]),
                                       O.LossParams(eps=EPS, h_tau=1, h_k=1, w_isl=1.0, w_psl=1.0, temp=0.05))
        assert abs(t[b, 0] - ref["loss"]) <= 1e-4 * abs(ref["loss"]), b
        o = plan.s_offsets[b]
        assert np.max(np.abs(g[o:o + n] - ref["g"])) <= 1e-4 * np.max(np.abs(ref["g"])), b


def test_one_launch_every_mode_matches_per_class(af):
    # every pass of the one-launch kernel against per-class launches (each of
    # which the other tests hold to the oracle): forward with a and chi
    # grids, the magnitude backward (stored and recomputed spectra), the
    # two-pass soft-PSL loss (running maxima), and the extended epilogue
    # terms (hard PSL, L_match, mainlobe width, cell weights)
    say("one launch, every mode")
    ns = [64, 100, 200, 300, 500, 90]
    ms = [128, 256, 512, 1024, 1024, 512]
    codes = [W.random_code(n, seed=950 + i) for i, n in enumerate(ns)]
    s = torch.from_numpy(np.concatenate(codes)).cuda()
    plans = {}
    for one in (True, False):
        for store in (1, 2):
            plans[(one, store)] = af.Plan(ns, ms, eps=EPS, one_launch=one, store_mode=store)
    assert plans[(True, 1)].summary()["variant"] == 6 and plans[(False, 1)].summary()["variant"] != 6
    E = np.array([float(np.sum(np.abs(c.astype(np.complex128)) ** 2)) for c in codes])

    def close(x, y, tol, what):
        x, y = x.cpu().numpy(), y.cpu().numpy()
        assert np.max(np.abs(x - y)) <= tol, (what, float(np.max(np.abs(x - y))), tol)

    # forward: a and chi
    out = {}
    for one in (True, False):
        p = plans[(one, 1)]
        mag, chi, e = p.forward(s, mag=True, chi=True, ws=p.new_workspace())
        out[one] = (mag, chi, e)
    torch.cuda.synchronize()
    close(out[True][0], out[False][0], 2e-6, "a")
    close(torch.view_as_real(out[True][1]), torch.view_as_real(out[False][1]), 2e-6 * E.max(), "chi")
    close(out[True][2], out[False][2], 1e-6 * E.max(), "E")
    # magnitude backward, both store modes
    cells = plans[(True, 1)].total_cells
    ga = torch.from_numpy(W.upstream_grid(1, cells, seed=77).ravel()).cuda() * out[False][0]
    grads = {}
    for key, p in plans.items():
        ws = p.new_workspace()
        p.forward(s, mag=False, ws=ws)
        grads[key] = p.backward(s, ga, ws=ws)
    torch.cuda.synchronize()
    ref = grads[(False, 2)]
    scale = float(ref.abs().max())
    for key, g in grads.items():
        close(torch.view_as_real(g), torch.view_as_real(ref), 1e-5 * scale, "backward %s" % (key,))
    # two-pass soft PSL (T = 0.01: running maxima, forward then backward)
    lp = dict(w_isl=1.0, w_psl=1.0, temp=0.01)
    res = {one: plans[(one, 2)].loss(s, **lp) for one in (True, False)}
    torch.cuda.synchronize()
    close(res[True][0], res[False][0], 1e-5 * float(res[False][0].abs().max()), "two-pass terms")
    close(torch.view_as_real(res[True][1]), torch.view_as_real(res[False][1]),
          1e-5 * float(res[False][1].abs().max()), "two-pass grad")
    # extended terms
    target = torch.rand(cells, device="cuda") * 0.01
    cw = torch.rand(cells, device="cuda")
    lp = dict(w_isl=1.0, match=target, w_match=0.5, w_width=0.01, gamma=10.0, cell_w=cw, w_cell=0.1)
    res = {one: plans[(one, 2)].loss(s, **lp) for one in (True, False)}
    torch.cuda.synchronize()
    close(res[True][0], res[False][0], 1e-5 * float(res[False][0].abs().max()), "ext terms")
    close(torch.view_as_real(res[True][1]), torch.view_as_real(res[False][1]),
          1e-5 * float(res[False][1].abs().max()), "ext grad")
    # the hard PSL (the forward pass with the extended epilogue): its value
    # (a maximum, robust to rounding; its cell and gradient could move between
    # near-equal sidelobes, so only the value is compared)
    lp = dict(w_isl=0.0, w_psl=1.0, psl_hard=True, match=target, w_match=0.5)
    fwd_only = {one: plans[(one, 2)].loss(s, grad=False, **lp) for one in (True, False)}
    torch.cuda.synchronize()
    close(fwd_only[True][0], fwd_only[False][0], 1e-5 * float(fwd_only[False][0].abs().max()), "ext forward")

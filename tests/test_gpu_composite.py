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
    # nor the hard PSL on the halves-in-turn variant (M >= 16384)
    big = af.Plan([9000], [32768], [100], eps=EPS)
    with pytest.raises(_lib.AfError) as ei:
        big.loss(to_dev(W.random_code(9000, seed=1)), w_isl=0.0, w_psl=1.0, psl_hard=True)
    assert ei.value.code == -2

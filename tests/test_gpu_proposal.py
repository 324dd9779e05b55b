"""What the learned proposal gains over the method without it (GPU only).

A small training run (fresh shaping weights each step) on N=256, M=512
codes; on held-out descriptors the network's proposals must start far below
random phases and stay ahead of plain Adam from random phases after the same
number of refinement steps.  The float64 oracle re-judges the weighted ISL of
a sample of the final codes.  Parity of the loss itself is covered in
test_gpu_af.py; this test is about the learned part.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O

pytestmark = pytest.mark.gpu
EPS = 1e-12


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def test_learned_proposal_beats_random_start():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_22935_amd import proposal as P
    n, m = 256, 512
    say("train proposer")
    pr = P.Proposer(n, m, seed=0)
    P.train(pr, n, m, batch=256, steps=600, seed=11)
    te = P.DescriptorBatch(n, m, 128, seed=12)
    say("evaluate")
    res = P.evaluate(pr, te, plain_steps=300, refine_steps=50, fallback_steps=300, seed=13)
    # the proposal alone is far better than a random start, and proposal + 50
    # refinement steps is better than 50 plain steps from random phases
    assert res["isl_proposal"] < 0.8 * res["isl_random"]
    plain50 = float(res["traj_plain"][50].mean())
    assert res["isl_after_refine"] < plain50
    # the oracle judges a sample of the learned, refined codes in float64
    phi = res["phi_learned_refined"].cpu().numpy().astype(np.float64).reshape(te.batch, n)
    got = P.weighted_isl(te, res["phi_learned_refined"]).cpu().numpy()
    for b in range(4):
        s = O.to_c64_exact(np.exp(1j * phi[b]))
        lp = O.LossParams(w_isl=1.0, h_tau=int(te.h_tau[b]), h_k=int(te.h_k[b]),
                          u=te.u[b].astype(np.float64), v=te.v[b].astype(np.float64), eps=EPS)
        ref = O.loss_terms(O.chi(s, m), O.energy(s), n, lp)["isl"]
        assert abs(got[b] - ref) <= 1e-4 * ref

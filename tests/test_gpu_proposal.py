"""What the learned proposal gains over the method without it (GPU only).

The network trains through the AF loss on fresh draws of the shaping
weights (N=256, M=512, batch 4096).  On held-out descriptors (another seed):
  * its proposals start far below random phases;
  * proposal + 50 refinement steps beats 50 plain steps from random phases;
  * the median time to reach, per descriptor, the weighted ISL that plain
    Adam has after 2000 steps is shorter for the learned path, the median
    taken over every descriptor with those that never reach it counted as
    inf (so more than half must reach it);
and the float64 oracle re-judges the weighted ISL of a sample of the codes.
Parity of the loss itself is covered in test_gpu_af.py.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O

pytestmark = pytest.mark.gpu
EPS = 1e-12
N, M = 256, 512


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def trained():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_22935_amd import proposal as P
    say("train proposer: batch 4096, 6000 steps")
    pr = P.Proposer(N, M, seed=0)
    P.train(pr, N, M, batch=4096, steps=6000, seed=11)
    te = P.DescriptorBatch(N, M, 1024, seed=12)
    say("evaluate on 1024 held-out descriptors")
    res = P.evaluate(pr, te, plain_steps=2000, refine_steps=50, fallback_steps=2000, seed=13)
    say("  reach within 50 %.3f, with fallback %.3f; median ms plain %.1f learned %.1f"
        % (res["reach_within_refine"], res["reach_with_fallback"], res["median_plain_ms"],
           res["median_learned_ms"]))
    return P, pr, te, res


def test_proposal_beats_random_start(trained):
    _, _, _, res = trained
    assert res["isl_proposal"] < 0.8 * res["isl_random"]
    plain50 = float(res["traj_plain"][50].mean())
    assert res["isl_after_refine"] < plain50


def test_learned_reaches_plain_isl_in_less_time(trained):
    _, _, _, res = trained
    # medians over every held-out descriptor, misses counted as inf
    assert res["reach_with_fallback"] > 0.5
    assert res["median_learned_ms"] < res["median_plain_ms"]


def test_oracle_rejudges_the_codes(trained):
    P, _, te, res = trained
    phi = res["phi_learned_refined"].cpu().numpy().astype(np.float64).reshape(te.batch, N)
    got = P.weighted_isl(te, res["phi_learned_refined"]).cpu().numpy()
    for b in range(4):
        s = O.to_c64_exact(np.exp(1j * phi[b]))
        lp = O.LossParams(w_isl=1.0, h_tau=int(te.h_tau[b]), h_k=int(te.h_k[b]),
                          u=te.u[b].astype(np.float64), v=te.v[b].astype(np.float64), eps=EPS)
        ref = O.loss_terms(O.chi(s, M), O.energy(s), N, lp)["isl"]
        assert abs(got[b] - ref) <= 1e-4 * ref

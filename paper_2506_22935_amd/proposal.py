"""Learned phase-code proposals (paper Sec. 6.1, Fig. 1, and the direct
refinement of Sec. 6.2 as the fallback).

A sidelobe-mask descriptor d = [h_tau/16, h_k/16, u_1..u_31, v_1..v_31]
sets the mainlobe half-widths and the separable ISL shaping weights
W[tau, k] = u[floor(31|tau|/N)] v[floor(31|k_c|/(M/2+1))] (0 on the mainlobe).
The network maps d to N phases; s = exp(j phi); the loss is the weighted ISL
of the ambiguity function.

Pipeline:
  1. plain optimiser (Adam on phases from random phases) on training
     descriptors -> target codes;
  2. supervised pre-training on those codes, with a loss invariant under the
     symmetries that leave the weighted ISL unchanged: a global phase, a
     linear phase ramp, time reversal and conjugation (|chi| is the same
     under the first three and mirrored in k under the last, and W depends
     on |k_c| only);
  3. fine-tuning through the differentiable AF loss: d -> net -> phi -> s ->
     weighted ISL -> dL/d conj(s) -> dL/dphi -> net backward -> Adam;
  4. use: net(d) then a few plain refinement steps.
"""
import math
import time

import numpy as np
import torch

from . import af
from . import mlp as MLPm
from . import workloads as W


class DescriptorBatch:
    """Descriptors on the device plus the plan that carries their masks."""

    def __init__(self, n, m, batch, seed, eps=1e-12):
        d = W.descriptors(batch, seed=seed)
        self.n, self.m, self.batch = n, m, batch
        self.h_tau, self.h_k = d["h_tau"], d["h_k"]
        self.d = torch.from_numpy(d["d"]).cuda()
        self.band = torch.from_numpy(np.concatenate([d["u"], d["v"]], axis=1).astype(np.float32).ravel()).cuda()
        self.u, self.v = d["u"], d["v"]
        self.plan = af.Plan([n] * batch, [m] * batch, h_tau=self.h_tau.tolist(), h_k=self.h_k.tolist(), eps=eps)
        self.ws = self.plan.workspace

    def resample_shaping(self, seed):
        """New shaping weights u, v (same mainlobes, so the same plan): a fresh
        draw from the descriptor distribution."""
        rng = np.random.default_rng(seed)
        u = rng.uniform(0.0, 1.0, size=(self.batch, 31))
        v = rng.uniform(0.0, 1.0, size=(self.batch, 31))
        d = self.d.cpu().numpy()
        d[:, 2:33], d[:, 33:64] = u, v
        self.d.copy_(torch.from_numpy(d.astype(np.float32)))
        self.band.copy_(torch.from_numpy(np.concatenate([u, v], axis=1).astype(np.float32).ravel()))
        self.u, self.v = u.astype(np.float32), v.astype(np.float32)


def plain_optimize(db, steps, lr=0.01, seed=0, phi0=None, record=True):
    """Adam on phases from random (or given) phases; returns the phase state
    and the per-step weighted ISL [steps, B] (loss at the start of each step)."""
    if phi0 is None:
        rng = np.random.default_rng(seed)
        phi0 = torch.from_numpy(rng.uniform(0, 2 * np.pi, db.batch * db.n).astype(np.float32)).cuda()
    st = af.PhaseState(phi0.clone())
    traj = torch.empty(max(steps, 1), db.batch, 4, device="cuda")
    for t in range(steps):
        db.plan.optim_step(st, w_isl=1.0, band_w=db.band, lr=lr, ws=db.ws, terms=traj[t])
    return st, traj[:steps, :, 1]


def weighted_isl(db, phi):
    s = torch.empty(phi.numel(), dtype=torch.complex64, device="cuda")
    af.phase_to_signal(phi.contiguous().view(-1), s)
    terms, _, _ = db.plan.loss(s, w_isl=1.0, band_w=db.band, grad=False, ws=db.ws)
    return terms[:, 1]


RAMP_OVERSAMPLE = 8  # linear-phase slopes searched on a grid of 2 pi / (8 N)


def alignment_loss(phi, target_phi):
    """Symmetry-invariant distance between phase codes [B, N] and its
    gradient.  |chi|, and with it the weighted ISL (whose weights depend on
    |tau| and |k_c| only), is unchanged by a global phase, a linear phase
    ramp (a frequency offset multiplies each lag product by a constant),
    time reversal and conjugation.  Per code the loss is
    1 - max |mean_n e^{j(phi_n - phi'_n - a n)}| over the four images phi'
    of the target (itself, reversed, conjugated, both) and the ramp slope a
    (on a grid of RAMP_OVERSAMPLE N slopes, by an FFT); the global phase is
    maximised in closed form by the modulus.  Averaged over the batch.
    Returns (loss, dloss/dphi), the gradient taken at the best image and
    slope."""
    B, n = phi.shape
    rev = torch.flip(target_phi, dims=[1])
    images = torch.stack([target_phi, rev, -target_phi, -rev])  # [4, B, N]
    e = torch.polar(torch.ones_like(images), phi.unsqueeze(0) - images)
    K = RAMP_OVERSAMPLE * n
    zs = torch.fft.fft(e, n=K, dim=2) / n  # z(a_j), a_j = 2 pi j / K
    mag = zs.abs()
    best_j = mag.argmax(dim=2)  # [4, B]
    best_val = mag.gather(2, best_j.unsqueeze(2)).squeeze(2)  # [4, B]
    best_i = best_val.argmax(dim=0)  # [B]: the image closest to the code
    rows = torch.arange(B, device=phi.device)
    jb = best_j[best_i, rows]  # [B]
    a = (2.0 * math.pi / K) * jb.to(phi.dtype)
    nn = torch.arange(n, device=phi.device, dtype=phi.dtype)
    eb = e[best_i, rows] * torch.polar(torch.ones_like(phi), -a.unsqueeze(1) * nn.unsqueeze(0))
    zb = eb.mean(dim=1, keepdim=True)
    az = zb.abs().clamp_min(1e-12)
    loss = float((1 - az).mean())
    # with e_n = e^{j(phi_n - phi'_n - a n)}, dz/dphi_n = j e_n / N, so
    # d(1 - |z|)/dphi_n = Im(conj(z) e_n) / (N |z|); averaged over the batch
    dphi = (torch.conj(zb) * eb).imag / (az * n * B)
    return loss, dphi.contiguous()


class Proposer:
    """The network and its two training stages."""

    def __init__(self, n=256, m=512, hidden=(1024, 1024, 1024), seed=0):
        self.n, self.m = n, m
        self.net = MLPm.MLP((64,) + tuple(hidden) + (n,), seed=seed)

    def propose(self, d):
        phi, _ = self.net.forward(d)
        return phi

    def pretrain_step(self, d, target_phi, lr=1e-3):
        """Supervised step towards plain-optimiser codes with the
        symmetry-invariant alignment loss."""
        phi, cache = self.net.forward(d)
        loss, dphi = alignment_loss(phi, target_phi)
        dW, db_ = self.net.backward(dphi, MLPm.to_bf16(dphi), cache)
        self.net.adam(dW, db_, lr=lr)
        return loss

    def finetune_step(self, db, lr=1e-4, scale=1.0):
        """One step through the AF loss: mean weighted ISL over the batch."""
        phi, cache = self.net.forward(db.d)
        s = torch.empty(db.batch * db.n, dtype=torch.complex64, device="cuda")
        af.phase_to_signal(phi.view(-1), s)
        terms, g, _ = db.plan.loss(s, w_isl=1.0, band_w=db.band, grad=True, ws=db.ws)
        dphi = torch.empty(db.batch, db.n, dtype=torch.float32, device="cuda")
        dphi16 = torch.empty(db.batch, db.n, dtype=torch.bfloat16, device="cuda")
        # mean over the batch: scale the upstream by 1/B
        MLPm.phase_grad(s, g, dphi, None)
        dphi.mul_(scale / db.batch)
        MLPm.to_bf16(dphi, dphi16)
        dW, dbias = self.net.backward(dphi, dphi16, cache)
        self.net.adam(dW, dbias, lr=lr)
        return terms[:, 1]


def time_to_target(traj, target, step_ms, offset_ms=0.0):
    """First step at which each waveform's ISL is <= its target, as ms
    (inf where never); traj [steps, B] holds the loss at the start of each step."""
    hit = traj <= target[None, :]
    steps = traj.shape[0]
    first = torch.where(hit.any(dim=0), hit.float().argmax(dim=0), torch.full_like(target, steps, dtype=torch.long))
    ms = offset_ms + first.double() * step_ms
    ms[~hit.any(dim=0)] = float("inf")
    return ms


def median_all(t):
    """Median over every descriptor, those that never reach the target
    counted as inf (the lower median of an even count)."""
    v, _ = torch.sort(t.double())
    return float(v[(v.numel() - 1) // 2])


def timed_ms(fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, (time.perf_counter() - t0) * 1e3


def train(proposer, n, m, batch=4096, steps=3000, lr=1e-3, lr_late=3e-4, seed=1, pretrain_steps=0,
          pretrain_draws=2, pretrain_plain_steps=2000, log=None):
    """Fine-tune through the AF loss on fresh descriptor draws (same mainlobes,
    new shaping weights every step); with pretrain_steps > 0, first a
    supervised warm start on the codes the plain optimiser finds for
    pretrain_draws draws of the shaping weights (symmetry-invariant loss)."""
    tr = DescriptorBatch(n, m, batch, seed=seed)
    if pretrain_steps:
        sets = []
        for k in range(pretrain_draws):
            if k:
                tr.resample_shaping(seed * 7919 + k)
            st, traj = plain_optimize(tr, pretrain_plain_steps, lr=0.01, seed=seed + 7 + k)
            sets.append((tr.d.clone(), st.phi.view(batch, n).clone()))
            if log:
                log("pretrain targets %d: plain-%d mean weighted ISL %.3f" % (k, pretrain_plain_steps,
                                                                             float(traj[-1].mean())))
        for it in range(pretrain_steps):
            d, tgt = sets[it % len(sets)]
            loss = proposer.pretrain_step(d, tgt, lr=lr)
            if log and (it % 1000 == 0 or it == pretrain_steps - 1):
                log("pretrain step %d: alignment loss %.4f" % (it, loss))
    isl = None
    for it in range(steps):
        tr.resample_shaping(seed * 1_000_003 + it)
        isl = proposer.finetune_step(tr, lr=lr if it < (2 * steps) // 3 else lr_late)
        if log and (it % 1000 == 0 or it == steps - 1):
            log("train step %d: mean weighted ISL %.3f" % (it, float(isl.mean())))
    return float(isl.mean()) if isl is not None else float("nan")


def evaluate(proposer, db, plain_steps=2000, refine_steps=50, fallback_steps=2000, seed=3, log=None):
    """Time to reach, per descriptor, the weighted ISL that plain Adam (lr 0.01,
    from random phases) has after plain_steps steps: plain from random versus
    network proposal + plain refinement (up to refine_steps, then the same
    optimiser continues as the fallback up to fallback_steps)."""
    (st_p, traj_p), ms_p = timed_ms(lambda: plain_optimize(db, plain_steps, lr=0.01, seed=seed))
    step_ms = ms_p / plain_steps
    target = traj_p[-1].clone()
    t_plain = time_to_target(traj_p, target, step_ms)
    phi, ms_net = timed_ms(lambda: proposer.propose(db.d))
    (st_l, traj_l), ms_l = timed_ms(lambda: plain_optimize(db, fallback_steps + 1, lr=0.01,
                                                           phi0=phi.view(-1).contiguous()))
    step_ms_l = ms_l / (fallback_steps + 1)
    t_learned = time_to_target(traj_l, target, step_ms_l, offset_ms=ms_net)
    within = time_to_target(traj_l[:refine_steps + 1], target, step_ms_l, offset_ms=ms_net)
    fin_p = torch.isfinite(t_plain)
    fin_l = torch.isfinite(t_learned)
    # ISL at equal wall time: plain after as many steps as the learned path's
    # proposal + refine_steps take, and the learned path after plain's budget
    eq_steps = min(plain_steps - 1, int(round((ms_net + refine_steps * step_ms_l) / step_ms)))
    res = dict(
        step_ms=step_ms, net_ms=ms_net, plain_steps=plain_steps, refine_steps=refine_steps,
        isl_random=float(traj_p[0].mean()), isl_plain_final=float(target.mean()),
        isl_proposal=float(traj_l[0].mean()), isl_after_refine=float(traj_l[min(refine_steps, traj_l.shape[0] - 1)].mean()),
        reach_within_refine=float(torch.isfinite(within).float().mean()),
        reach_with_fallback=float(fin_l.float().mean()),
        reach_plain=float(fin_p.float().mean()),
        # medians over every descriptor, inf where the target is never reached
        median_plain_ms=median_all(t_plain),
        median_learned_ms=median_all(t_learned),
        # medians over the descriptors that reach it (reported, not compared)
        median_plain_reached_ms=float(t_plain[fin_p].median()) if bool(fin_p.any()) else float("inf"),
        median_learned_reached_ms=float(t_learned[fin_l].median()) if bool(fin_l.any()) else float("inf"),
        learned_faster_frac=float((t_learned < t_plain).float().mean()),
        equal_time_steps=eq_steps,
        isl_plain_at_equal_time=float(traj_p[eq_steps].mean()),
        isl_learned_after_plain_budget=float(traj_l[min(plain_steps, traj_l.shape[0] - 1)].mean()),
        phi_plain=st_p.phi, phi_learned_refined=st_l.phi, traj_learned=traj_l, traj_plain=traj_p)
    if log:
        log("evaluate: plain %.3f ms/step; ISL random %.2f plain-%d %.2f proposal %.2f +%d refine %.2f; "
            "reach within %d: %.3f, with fallback %.3f; median time (all descriptors, inf if never) plain %.1f "
            "ms learned %.1f ms; plain at equal time (%d steps) %.2f"
            % (step_ms, res["isl_random"], plain_steps, res["isl_plain_final"], res["isl_proposal"], refine_steps,
               res["isl_after_refine"], refine_steps, res["reach_within_refine"], res["reach_with_fallback"],
               res["median_plain_ms"], res["median_learned_ms"], eq_steps, res["isl_plain_at_equal_time"]))
    return res

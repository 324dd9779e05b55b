"""Python face of libgraf_af.so: plans, the three AF calls and the phase
optimiser step, on torch device tensors.  Argument marshalling only: every
step of the computation runs in the library's HIP kernels.

Conventions (see include/graf_af.h): packed complex64 waveforms, packed
float32 grids [2T+1][M] per waveform, gradients as dL/d conj(s).
"""
import ctypes

import torch

from . import _lib as L

_DEV = "cuda"


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


class Plan:
    """A batch layout: per waveform N, M, lag half-width T and mainlobe
    half-widths.  Waveforms pack back to back in s; grids pack back to back.
    periodic (bool or one per waveform): the circular AF of N = M bins with
    [N][N] grids (row tau in [0, N)) instead of the aperiodic [2T+1][M].
    """

    def __init__(self, lengths, ms, max_lags=None, h_tau=1, h_k=1, eps=1e-12, store_mode=0,
                 budget_bytes=0, variant=-1, segment_iters=0, loss_passes=0, periodic=False, one_launch=True):
        lengths = [int(n) for n in lengths]
        ms = [int(m) for m in ms]
        B = len(lengths)
        if len(ms) != B:
            raise ValueError("lengths and ms differ in length")
        periodic = [bool(periodic)] * B if isinstance(periodic, (bool, int)) else [bool(x) for x in periodic]
        max_lags = [n - 1 for n in lengths] if max_lags is None else [int(t) for t in max_lags]
        max_lags = [n - 1 if t < 0 else t for n, t in zip(lengths, max_lags)]
        h_tau = [int(h_tau)] * B if isinstance(h_tau, int) else [int(x) for x in h_tau]
        h_k = [int(h_k)] * B if isinstance(h_k, int) else [int(x) for x in h_k]
        waves = (L.AfWave * B)()
        s_off = g_off = 0
        self.s_offsets, self.grid_offsets, self.rows = [], [], []
        for b in range(B):
            w = waves[b]
            w.n, w.m, w.max_lag = lengths[b], ms[b], max_lags[b]
            w.h_tau, w.h_k = h_tau[b], h_k[b]
            w.flags = L.AF_WAVE_PERIODIC if periodic[b] else 0
            w.s_off, w.grid_off = s_off, g_off
            rows = lengths[b] if periodic[b] else 2 * max_lags[b] + 1
            self.s_offsets.append(s_off)
            self.grid_offsets.append(g_off)
            self.rows.append(rows)
            s_off += lengths[b]
            g_off += rows * ms[b]
        self.batch, self.lengths, self.ms, self.max_lags = B, lengths, ms, max_lags
        self.periodic = periodic
        self.total_samples, self.total_cells = s_off, g_off
        opts = L.AfPlanOpts(eps=float(eps), store_mode=int(store_mode), budget_bytes=int(budget_bytes),
                            variant=int(variant), segment_iters=int(segment_iters),
                            loss_passes=int(loss_passes), launch_mode=0 if one_launch else 1)
        h = ctypes.c_void_p()
        L.check("af_plan_create", L.lib().af_plan_create(B, waves, ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        self._refresh()

    def _refresh(self):
        sz = ctypes.c_size_t()
        L.check("af_plan_workspace_size", L.lib().af_plan_workspace_size(self._h, ctypes.byref(sz)))
        self.workspace_bytes = int(sz.value)
        self._ws = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                L.lib().af_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    # ------------------------------------------------------------------
    def summary(self):
        s = L.AfPlanSummary()
        L.check("af_plan_get_summary", L.lib().af_plan_get_summary(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in L.AfPlanSummary._fields_}

    def new_workspace(self):
        return torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8, device=_DEV)

    @property
    def workspace(self):
        if self._ws is None or self._ws.numel() < self.workspace_bytes:
            self._ws = self.new_workspace()
        return self._ws

    def grid(self, flat, b):
        """View of waveform b's grid ([2T+1, M], periodic [N, N]) inside a
        packed grid tensor."""
        o = self.grid_offsets[b]
        return flat[o:o + self.rows[b] * self.ms[b]].view(self.rows[b], self.ms[b])

    def owner_index(self, device):
        """int64[total_samples]: the waveform each packed sample belongs to."""
        if getattr(self, "_owner", None) is None or self._owner.device != torch.device(device):
            self._owner = torch.repeat_interleave(torch.arange(self.batch, device=device),
                                                  torch.tensor(self.lengths, device=device))
        return self._owner

    def signal(self, flat, b):
        o = self.s_offsets[b]
        return flat[o:o + self.lengths[b]]

    def autotune(self, s):
        _need(s, torch.complex64, "s")
        ws = torch.empty(max(self.workspace_bytes * 4, 1 << 20), dtype=torch.uint8, device=_DEV)
        v = ctypes.c_int32()
        ms = ctypes.c_float()
        L.check("af_plan_autotune", L.lib().af_plan_autotune(self._h, _ptr(s), _ptr(ws), ws.numel(), _stream(),
                                                              ctypes.byref(v), ctypes.byref(ms)))
        self._refresh()
        return int(v.value), float(ms.value)

    # ------------------------------------------------------------------
    def forward(self, s, mag=True, chi=False, ws=None, out_mag=None):
        """Returns (a grids float32 or None, chi complex64 or None, E float32[B])."""
        _need(s, torch.complex64, "s")
        ws = self.workspace if ws is None else ws
        m = None
        if mag:
            m = out_mag if out_mag is not None else torch.empty(self.total_cells, dtype=torch.float32, device=_DEV)
        c = torch.empty(self.total_cells, dtype=torch.complex64, device=_DEV) if chi else None
        e = torch.empty(self.batch, dtype=torch.float32, device=_DEV)
        L.check("af_forward", L.lib().af_forward(self._h, _ptr(s), _ptr(m), _ptr(c), _ptr(e), _ptr(ws),
                                                 ws.numel(), _stream()))
        return m, c, e

    def backward(self, s, grad_mag, ws=None, out=None):
        """dL/d conj(s) for an upstream dL/da (packed float32 grids)."""
        _need(s, torch.complex64, "s")
        _need(grad_mag, torch.float32, "grad_mag")
        ws = self.workspace if ws is None else ws
        g = out if out is not None else torch.empty(self.total_samples, dtype=torch.complex64, device=_DEV)
        L.check("af_backward", L.lib().af_backward(self._h, _ptr(s), _ptr(grad_mag), _ptr(g), _ptr(ws),
                                                   ws.numel(), _stream()))
        return g

    @staticmethod
    def loss_params(w_isl=1.0, w_psl=0.0, temp=0.05, band_w=None, psl_hard=False, w_spec=0.0, match=None,
                    w_match=0.0, w_width=0.0, gamma=10.0, w_const=0.0, w_smooth=0.0, cell_w=None, w_cell=0.0):
        if band_w is not None:
            _need(band_w, torch.float32, "band_w")
        if match is not None:
            _need(match, torch.float32, "match")
        if cell_w is not None:
            _need(cell_w, torch.float32, "cell_w")
        p = L.AfLossParams(w_isl=float(w_isl), w_psl=float(w_psl), psl_temp=float(temp),
                           band_w=None if band_w is None else band_w.data_ptr(), psl_hard=1 if psl_hard else 0,
                           w_spec=float(w_spec), match_target=None if match is None else match.data_ptr(),
                           w_match=float(w_match), w_width=float(w_width), gamma=float(gamma),
                           w_const=float(w_const), w_smooth=float(w_smooth),
                           cell_w=None if cell_w is None else cell_w.data_ptr(), w_cell=float(w_cell))
        p._keep = (band_w, match, cell_w)  # keep the tensors alive while the struct is in use
        return p

    def loss(self, s, w_isl=1.0, w_psl=0.0, temp=0.05, band_w=None, grad=True, mag=False, ws=None,
             out_terms=None, out_grad=None, psl_hard=False, w_spec=0.0, match=None, w_match=0.0, w_width=0.0,
             gamma=10.0, w_const=0.0, w_smooth=0.0, cell_w=None, w_cell=0.0):
        """Built-in loss.  Returns (terms float32[B,4] = (L, ISL, PSL term, E),
        dL/d conj(s) or None, a grids or None).  psl_hard: the hard PSL
        (power ratio) instead of the soft one; w_spec: weight of the spectral
        variance (the experiment loss: w_psl=1, psl_hard=True,
        w_spec=lambda*alpha); match, w_match: L_match against a target power
        grid laid out like the a grid; w_width, gamma: the soft mainlobe
        width; w_const: var(|s|); w_smooth: the phase-smoothness term;
        cell_w, w_cell: a per-cell weight grid laid out like the a grid."""
        _need(s, torch.complex64, "s")
        ws = self.workspace if ws is None else ws
        lp = self.loss_params(w_isl, w_psl, temp, band_w, psl_hard, w_spec, match, w_match, w_width, gamma,
                              w_const, w_smooth, cell_w, w_cell)
        t = out_terms if out_terms is not None else torch.empty(self.batch, 4, dtype=torch.float32, device=_DEV)
        g = None
        if grad:
            g = out_grad if out_grad is not None else torch.empty(self.total_samples, dtype=torch.complex64,
                                                                 device=_DEV)
        m = torch.empty(self.total_cells, dtype=torch.float32, device=_DEV) if mag else None
        L.check("af_loss", L.lib().af_loss(self._h, _ptr(s), ctypes.byref(lp), _ptr(t), _ptr(m), _ptr(g),
                                           _ptr(ws), ws.numel(), _stream()))
        return t, g, m

    def loss_no_alloc(self, s, terms, grad=None, mag=None, w_isl=1.0, w_psl=0.0, temp=0.05, band_w=None,
                      psl_hard=False, w_spec=0.0, match=None, w_match=0.0, w_width=0.0, gamma=10.0, w_const=0.0,
                      w_smooth=0.0, cell_w=None, w_cell=0.0):
        """loss() through af_loss_no_alloc: the workspace is the library's own
        device array (no workspace argument, nothing allocated by the call).
        terms, grad (nullable) and mag (nullable) are caller-owned outputs."""
        _need(s, torch.complex64, "s")
        lp = self.loss_params(w_isl, w_psl, temp, band_w, psl_hard, w_spec, match, w_match, w_width, gamma,
                              w_const, w_smooth, cell_w, w_cell)
        L.check("af_loss_no_alloc", L.lib().af_loss_no_alloc(self._h, _ptr(s), ctypes.byref(lp), _ptr(terms),
                                                             _ptr(mag), _ptr(grad), _stream()))

    def loss_stage(self, stage, s, terms, grad, mag, w_isl=1.0, w_psl=0.0, temp=0.05, band_w=None, ws=None,
                   psl_hard=False, w_spec=0.0, match=None, w_match=0.0, w_width=0.0, gamma=10.0, w_const=0.0,
                   w_smooth=0.0, cell_w=None, w_cell=0.0):
        """Run one stage (0 forward, 1 backward and the per-waveform terms, 2
        reduce) of loss(); for timing."""
        ws = self.workspace if ws is None else ws
        lp = self.loss_params(w_isl, w_psl, temp, band_w, psl_hard, w_spec, match, w_match, w_width, gamma,
                              w_const, w_smooth, cell_w, w_cell)
        L.check("af_loss_stage", L.lib().af_loss_stage(self._h, int(stage), _ptr(s), ctypes.byref(lp), _ptr(terms),
                                                       _ptr(mag), _ptr(grad), _ptr(ws), ws.numel(), _stream()))

    def optim_step(self, state, w_isl=1.0, w_psl=0.0, temp=0.05, band_w=None, lr=0.01, betas=(0.9, 0.999),
                   eps=1e-8, ws=None, terms=None, psl_hard=False, w_spec=0.0, match=None, w_match=0.0,
                   w_width=0.0, gamma=10.0, w_const=0.0, w_smooth=0.0, cell_w=None, w_cell=0.0):
        """One Adam step on the phases held in `state` (see PhaseState)."""
        ws = self.workspace if ws is None else ws
        lp = self.loss_params(w_isl, w_psl, temp, band_w, psl_hard, w_spec, match, w_match, w_width, gamma,
                              w_const, w_smooth, cell_w, w_cell)
        ad = L.AfAdamParams(lr=float(lr), beta1=float(betas[0]), beta2=float(betas[1]), eps=float(eps))
        L.check("af_optim_step", L.lib().af_optim_step(
            self._h, _ptr(state.phi), _ptr(state.m), _ptr(state.v), _ptr(state.s), _ptr(state.step),
            ctypes.byref(lp), ctypes.byref(ad), _ptr(terms), _ptr(ws), ws.numel(), _stream()))


    def spectral_variance(self, s, grad=False, ws=None):
        """Spectral variance of each waveform's N-point spectrum (Sec. 7.1.1)
        and, with grad, its dV/d conj(s).  Returns (float32[B], grad or None)."""
        _need(s, torch.complex64, "s")
        ws = self.workspace if ws is None else ws
        v = torch.empty(self.batch, dtype=torch.float32, device=_DEV)
        g = torch.empty(self.total_samples, dtype=torch.complex64, device=_DEV) if grad else None
        L.check("af_spectral_variance", L.lib().af_spectral_variance(self._h, _ptr(s), _ptr(v), _ptr(g), _ptr(ws),
                                                                     ws.numel(), _stream()))
        return v, g

    def project(self, s, mask=None, unit=False, out=None):
        """Projection step of projected descent (Sec. 6.2): with mask (float32,
        one weight per bin of each waveform's N-point DFT, packed like s) the
        masked spectrum transformed back; with unit, then onto the unit
        circle.  out may be s (in place).  Returns out."""
        _need(s, torch.complex64, "s")
        if mask is not None:
            _need(mask, torch.float32, "mask")
        out = torch.empty_like(s) if out is None else out
        L.check("af_project", L.lib().af_project(self._h, _ptr(s), _ptr(mask), 1 if unit else 0, _ptr(out),
                                                 _stream()))
        return out


    def scenario_combine(self, grids, lambdas):
        """sum_s lambdas[s] grids[s] over the plan's cells (Eq. 24's linear
        scenario terms as one weight grid): grids float32 [S, cells],
        lambdas float32 [S] (device).  Returns float32 [cells]."""
        _need(grids, torch.float32, "grids")
        _need(lambdas, torch.float32, "lambdas")
        if grids.dim() != 2 or grids.shape[1] != self.total_cells or lambdas.numel() != grids.shape[0]:
            raise ValueError("grids must be [S, %d] with S lambdas" % self.total_cells)
        out = torch.empty(self.total_cells, dtype=torch.float32, device=_DEV)
        L.check("af_scenario_combine", L.lib().af_scenario_combine(self._h, grids.shape[0], _ptr(grids),
                                                                   _ptr(lambdas), _ptr(out), _stream()))
        return out

    def cross_workspace(self):
        """Device workspace for cross_backward (allocated once per plan)."""
        if getattr(self, "_cross_ws", None) is None:
            n = ctypes.c_size_t(0)
            L.check("af_cross_workspace_size", L.lib().af_cross_workspace_size(self._h, ctypes.byref(n)))
            self._cross_ws = torch.empty(max(int(n.value), 256), dtype=torch.uint8, device=_DEV)
        return self._cross_ws

    def cross_forward(self, s, u, mag=True, chi=False):
        """Cross-ambiguity of s and u (packed like the plan's input): returns
        (a grids or None, chi_su grids or None, float32[B, 2] = E_s, E_u)."""
        _need(s, torch.complex64, "s")
        _need(u, torch.complex64, "u")
        m = torch.empty(self.total_cells, dtype=torch.float32, device=_DEV) if mag else None
        c = torch.empty(self.total_cells, dtype=torch.complex64, device=_DEV) if chi else None
        e = torch.empty(self.batch, 2, dtype=torch.float32, device=_DEV)
        L.check("af_cross_forward", L.lib().af_cross_forward(self._h, _ptr(s), _ptr(u), _ptr(m), _ptr(c), _ptr(e),
                                                             _stream()))
        return m, c, e

    def cross_backward(self, s, u, grad_mag, ws=None):
        """(dL/d conj(s), dL/d conj(u)) for the upstream dL/da grid."""
        _need(s, torch.complex64, "s")
        _need(u, torch.complex64, "u")
        _need(grad_mag, torch.float32, "grad_mag")
        ws = self.cross_workspace() if ws is None else ws
        gs = torch.empty_like(s)
        gu = torch.empty_like(u)
        L.check("af_cross_backward", L.lib().af_cross_backward(self._h, _ptr(s), _ptr(u), _ptr(grad_mag), _ptr(gs),
                                                               _ptr(gu), _ptr(ws), ws.numel(), _stream()))
        return gs, gu


class PhaseState:
    """Phases, Adam moments, the device step counter and s = exp(j phi)."""

    def __init__(self, phi):
        _need(phi, torch.float32, "phi")
        self.phi = phi
        self.m = torch.zeros_like(phi)
        self.v = torch.zeros_like(phi)
        self.step = torch.zeros(1, dtype=torch.int32, device=phi.device)
        self.s = torch.empty(phi.numel(), dtype=torch.complex64, device=phi.device)
        phase_to_signal(self.phi, self.s)


def phase_to_signal(phi, s):
    _need(phi, torch.float32, "phi")
    _need(s, torch.complex64, "s")
    L.check("af_phase_to_signal", L.lib().af_phase_to_signal(_ptr(phi), _ptr(s), phi.numel(), _stream()))
    return s


def single(n, m=None, max_lag=-1, **kw):
    """Plan for one waveform of n samples (M defaults to 2n rounded up to a power of two)."""
    m = m or 1 << (2 * n - 1).bit_length()
    return Plan([n], [m], [max_lag], **kw)

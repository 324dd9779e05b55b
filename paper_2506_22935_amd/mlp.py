"""The proposal network (paper Sec. 6.1, Fig. 1): design parameters ->
network -> phases.  Dense layers with exact GELU between them; BF16 weights
and activations, FP32 accumulation, FP32 master weights for Adam.  Every
layer, gradient and update runs in the library's kernels; this class only
holds the tensors and orders the calls.
"""
import ctypes

import numpy as np
import torch

from . import _lib as L

NT, NN, TN = 0, 1, 2
E_F32, E_BIAS_F32, E_BIAS_GELU, E_GELU_BWD = 0, 1, 2, 3


def _p(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _st():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


_WS = {}  # device -> uint8 workspace shared by the split-k GEMMs and column sums (stream-ordered)


def _workspace(nbytes, device):
    key = torch.device(device).index if torch.device(device).index is not None else torch.cuda.current_device()
    ws = _WS.get(key)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(max(nbytes, 1 << 20), dtype=torch.uint8, device=device)
        _WS[key] = ws
    return ws


def gemm_config(m, n, k, tile=0, split_k=0):
    """(tile, split_k, workspace bytes) the library uses for this shape."""
    t, s, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t()
    L.check("af_gemm_config", L.lib().af_gemm_config(m, n, k, tile, split_k, ctypes.byref(t), ctypes.byref(s),
                                                     ctypes.byref(b)))
    return t.value, s.value, b.value


def gemm(layout, epi, m, n, k, a, b, bias=None, aux=None, out_f32=None, out_bf16=None, tile=0, split_k=0):
    _, _, need = gemm_config(m, n, k, tile, split_k)
    ws = _workspace(need, a.device) if need else None
    L.check("af_gemm_bf16", L.lib().af_gemm_bf16(layout, epi, m, n, k, _p(a), _p(b), _p(bias), _p(aux),
                                                 _p(out_f32), _p(out_bf16), tile, split_k, _p(ws),
                                                 need, _st()))


def to_bf16(x, out=None):
    out = torch.empty(x.shape, dtype=torch.bfloat16, device=x.device) if out is None else out
    L.check("af_to_bf16", L.lib().af_to_bf16(x.numel(), _p(x), _p(out), _st()))
    return out


def colsum(x, out):
    need = ctypes.c_size_t()
    L.check("af_colsum_workspace_size", L.lib().af_colsum_workspace_size(x.shape[0], x.shape[1], ctypes.byref(need)))
    ws = _workspace(need.value, x.device)
    L.check("af_colsum", L.lib().af_colsum(x.shape[0], x.shape[1], _p(x), _p(out), _p(ws), need.value, _st()))
    return out


def phase_grad(s, grad_s, out, out_bf16=None):
    L.check("af_phase_grad", L.lib().af_phase_grad(out.numel(), _p(s), _p(grad_s), _p(out), _p(out_bf16), _st()))
    return out


class MLP:
    """sizes = (in, hidden..., out); the default is the proposal network
    64 -> 1024 -> 1024 -> 1024 -> 256."""

    def __init__(self, sizes=(64, 1024, 1024, 1024, 256), seed=0, device="cuda"):
        rng = np.random.default_rng(seed)
        self.sizes = tuple(int(x) for x in sizes)
        self.W, self.b = [], []
        for i in range(len(sizes) - 1):
            fan_in = sizes[i]
            lim = 1.0 / np.sqrt(fan_in)
            self.W.append(torch.from_numpy(rng.uniform(-lim, lim, (sizes[i + 1], fan_in)).astype(np.float32)).to(device))
            self.b.append(torch.from_numpy(rng.uniform(-lim, lim, sizes[i + 1]).astype(np.float32)).to(device))
        self.W16 = [to_bf16(w) for w in self.W]
        self.mW = [torch.zeros_like(w) for w in self.W]
        self.vW = [torch.zeros_like(w) for w in self.W]
        self.mb = [torch.zeros_like(b) for b in self.b]
        self.vb = [torch.zeros_like(b) for b in self.b]
        self.step = 0

    @property
    def layers(self):
        return len(self.W)

    def forward(self, x):
        """x: float32 [B, in].  Returns (out float32 [B, out], cache)."""
        B = x.shape[0]
        a = to_bf16(x.contiguous())
        acts, pres = [a], []
        for i in range(self.layers):
            n_out, n_in = self.W[i].shape
            z = torch.empty(B, n_out, dtype=torch.float32, device=x.device)
            if i < self.layers - 1:
                a_next = torch.empty(B, n_out, dtype=torch.bfloat16, device=x.device)
                gemm(NT, E_BIAS_GELU, B, n_out, n_in, a, self.W16[i], bias=self.b[i], out_f32=z, out_bf16=a_next)
                acts.append(a_next)
                a = a_next
            else:
                gemm(NT, E_BIAS_F32, B, n_out, n_in, a, self.W16[i], bias=self.b[i], out_f32=z)
            pres.append(z)
        return pres[-1], dict(acts=acts, pres=pres)

    def backward(self, dout, dout_bf16, cache):
        """dout: float32 [B, out] = dL/d out (and its bfloat16 copy).
        Returns (dW list float32, db list float32)."""
        B = dout.shape[0]
        dW = [None] * self.layers
        db = [None] * self.layers
        dz, dz16 = dout, dout_bf16
        for i in range(self.layers - 1, -1, -1):
            n_out, n_in = self.W[i].shape
            dW[i] = torch.empty(n_out, n_in, dtype=torch.float32, device=dout.device)
            gemm(TN, E_F32, n_out, n_in, B, dz16, cache["acts"][i], out_f32=dW[i])
            db[i] = colsum(dz, torch.empty(n_out, dtype=torch.float32, device=dout.device))
            if i > 0:
                dz_prev = torch.empty(B, n_in, dtype=torch.float32, device=dout.device)
                dz16_prev = torch.empty(B, n_in, dtype=torch.bfloat16, device=dout.device)
                gemm(NN, E_GELU_BWD, B, n_in, n_out, dz16, self.W16[i], aux=cache["pres"][i - 1], out_f32=dz_prev,
                     out_bf16=dz16_prev)
                dz, dz16 = dz_prev, dz16_prev
        return dW, db

    def adam(self, dW, db, lr=1e-3, betas=(0.9, 0.999), eps=1e-8):
        self.step += 1
        ad = L.AfAdamParams(lr=float(lr), beta1=float(betas[0]), beta2=float(betas[1]), eps=float(eps))
        for i in range(self.layers):
            L.check("af_adam_update", L.lib().af_adam_update(self.W[i].numel(), _p(self.W[i]), _p(dW[i]),
                                                             _p(self.mW[i]), _p(self.vW[i]), self.step,
                                                             ctypes.byref(ad), _p(self.W16[i]), _st()))
            L.check("af_adam_update", L.lib().af_adam_update(self.b[i].numel(), _p(self.b[i]), _p(db[i]),
                                                             _p(self.mb[i]), _p(self.vb[i]), self.step,
                                                             ctypes.byref(ad), None, _st()))

    def state(self):
        """Tensors that checkpoint the network and its optimiser."""
        return dict(W=self.W, b=self.b, mW=self.mW, vW=self.vW, mb=self.mb, vb=self.vb, step=self.step)

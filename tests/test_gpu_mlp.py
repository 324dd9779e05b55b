"""The BF16-MFMA proposal network against the float64 oracle (GPU only).

The oracle rounds GEMM operands to bfloat16 exactly where the kernels store
bfloat16 and sums in float64; the kernels sum bf16 x bf16 products (exact in
float32) in float32.  Their sums differ by float32 accumulation error
(~sqrt(K) 2^-24 relative); where that straddles a bfloat16 rounding boundary
of a stored activation, the two round to neighbouring bf16 values (2^-8
relative) and the difference propagates.  Bars: max error <= 2e-2 of the
output scale and mean error <= 2e-3 of it, which a wrong layout, index or
epilogue exceeds by orders of magnitude.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def M():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_22935_amd import mlp
    return mlp


def close(got, ref, what, max_rel=2e-2, mean_rel=2e-3):
    scale = np.max(np.abs(ref))
    err = np.abs(got - ref)
    assert err.max() <= max_rel * scale, "%s: max err %.3e scale %.3e" % (what, err.max(), scale)
    assert err.mean() <= mean_rel * np.mean(np.abs(ref)) + 1e-7 * scale, "%s: mean err %.3e" % (what, err.mean())


def test_gemm_layouts_exact_small_integers(M):
    # integer-valued bf16 operands: every product and sum is exact in float32,
    # so each layout must match the float64 product exactly
    say("gemm layouts")
    rng = np.random.default_rng(0)
    m, n, k = 128, 64, 192
    A = rng.integers(-4, 5, (m, k)).astype(np.float32)
    Bnk = rng.integers(-4, 5, (n, k)).astype(np.float32)
    ref = A.astype(np.float64) @ Bnk.T.astype(np.float64)
    out = torch.empty(m, n, device="cuda")
    to16 = lambda x: M.to_bf16(torch.from_numpy(np.ascontiguousarray(x)).cuda())
    M.gemm(M.NT, M.E_F32, m, n, k, to16(A), to16(Bnk), out_f32=out)
    assert np.array_equal(out.cpu().numpy(), ref)
    M.gemm(M.NN, M.E_F32, m, n, k, to16(A), to16(Bnk.T), out_f32=out)
    assert np.array_equal(out.cpu().numpy(), ref)
    M.gemm(M.TN, M.E_F32, m, n, k, to16(A.T), to16(Bnk.T), out_f32=out)
    assert np.array_equal(out.cpu().numpy(), ref)


@pytest.mark.parametrize("layout", [0, 1, 2])
@pytest.mark.parametrize("tile,split", [(1, 1), (2, 1), (3, 1), (4, 1), (5, 1), (6, 1), (7, 1), (8, 1), (1, 2), (2, 4),
                                        (3, 12), (4, 3), (5, 2), (6, 3), (7, 6), (8, 2)])
def test_gemm_tiles_and_splits_exact(M, layout, tile, split):
    # every tile shape and split-k path, several tiles in m and n, integer
    # operands (exact in float32): the result equals the float64 product
    say("gemm tile", layout, tile, split)
    rng = np.random.default_rng(10 + tile + 5 * split)
    m, n, k = 256, 384, 768
    A = rng.integers(-4, 5, (m, k)).astype(np.float32)
    Bnk = rng.integers(-4, 5, (n, k)).astype(np.float32)
    ref = A.astype(np.float64) @ Bnk.T.astype(np.float64)
    to16 = lambda x: M.to_bf16(torch.from_numpy(np.ascontiguousarray(x)).cuda())
    a = to16(A.T) if layout == M.TN else to16(A)
    b = to16(Bnk) if layout == M.NT else to16(Bnk.T)
    out = torch.full((m, n), float("nan"), device="cuda")
    M.gemm(layout, M.E_F32, m, n, k, a, b, out_f32=out, tile=tile, split_k=split)
    assert np.array_equal(out.cpu().numpy(), ref)


@pytest.mark.parametrize("split", [1, 4])
def test_gemm_split_epilogues(M, split):
    # the split-k reduction applies every epilogue like the one-pass kernel
    say("gemm split epilogues", split)
    rng = np.random.default_rng(20 + split)
    m, n, k = 128, 256, 512
    A = rng.standard_normal((m, k)).astype(np.float32)
    W = (rng.standard_normal((n, k)) * 0.05).astype(np.float32)
    b = rng.standard_normal(n).astype(np.float32)
    aux = rng.standard_normal((m, n)).astype(np.float32)
    a16, w16 = M.to_bf16(torch.from_numpy(A).cuda()), M.to_bf16(torch.from_numpy(W).cuda())
    Z = O.bf16_round(A).astype(np.float64) @ O.bf16_round(W).T.astype(np.float64)
    outs = {}
    for epi in (M.E_F32, M.E_BIAS_F32, M.E_BIAS_GELU, M.E_GELU_BWD):
        f = torch.empty(m, n, device="cuda")
        h = torch.empty(m, n, dtype=torch.bfloat16, device="cuda")
        M.gemm(M.NT, epi, m, n, k, a16, w16, bias=torch.from_numpy(b).cuda(), aux=torch.from_numpy(aux).cuda(),
               out_f32=f, out_bf16=h, tile=1, split_k=split)
        outs[epi] = (f.cpu().numpy(), h.float().cpu().numpy())
    sc = np.max(np.abs(Z))
    assert np.max(np.abs(outs[M.E_F32][0] - Z)) <= 1e-5 * sc
    assert np.max(np.abs(outs[M.E_BIAS_F32][0] - (Z + b))) <= 1e-5 * sc
    assert np.max(np.abs(outs[M.E_BIAS_GELU][0] - (Z + b))) <= 1e-5 * sc
    g = O.gelu(Z + b)
    assert np.max(np.abs(outs[M.E_BIAS_GELU][1] - g)) <= 2 ** -8 * np.max(np.abs(g)) + 1e-5 * sc
    dz = Z * O.gelu_grad(aux.astype(np.float64))
    assert np.max(np.abs(outs[M.E_GELU_BWD][0] - dz)) <= 1e-5 * np.max(np.abs(dz)) * 4
    assert np.max(np.abs(outs[M.E_GELU_BWD][1] - dz)) <= 2 ** -8 * np.max(np.abs(dz)) + 1e-5 * np.max(np.abs(dz))


@pytest.mark.parametrize("rows,cols", [(1, 64), (7, 300), (4096, 1024), (4096, 256), (513, 64)])
def test_colsum_vs_float64(M, rows, cols):
    say("colsum", rows, cols)
    rng = np.random.default_rng(rows + cols)
    x = rng.standard_normal((rows, cols)).astype(np.float32)
    out = torch.empty(cols, device="cuda")
    M.colsum(torch.from_numpy(x).cuda(), out)
    ref = x.astype(np.float64).sum(axis=0)
    # float32 sums of rows terms: error ~ sqrt(rows) 2^-24 |x|
    assert np.max(np.abs(out.cpu().numpy() - ref)) <= 8 * np.sqrt(rows) * 2 ** -24 * np.max(np.abs(x)) * 4 + 1e-6


def test_gemm_bias_gelu_epilogues(M):
    say("gemm epilogues")
    rng = np.random.default_rng(1)
    m, n, k = 64, 128, 64
    A = rng.standard_normal((m, k)).astype(np.float32)
    W = (rng.standard_normal((n, k)) * 0.2).astype(np.float32)
    b = rng.standard_normal(n).astype(np.float32)
    Ar, Wr = O.bf16_round(A), O.bf16_round(W)
    Z = Ar @ Wr.T + b
    z = torch.empty(m, n, device="cuda")
    a16 = torch.empty(m, n, dtype=torch.bfloat16, device="cuda")
    M.gemm(M.NT, M.E_BIAS_GELU, m, n, k, M.to_bf16(torch.from_numpy(A).cuda()),
           M.to_bf16(torch.from_numpy(W).cuda()), bias=torch.from_numpy(b).cuda(), out_f32=z, out_bf16=a16)
    assert np.max(np.abs(z.cpu().numpy() - Z)) <= 1e-5 * np.max(np.abs(Z))
    g = O.gelu(Z)
    assert np.max(np.abs(a16.float().cpu().numpy() - g)) <= 2 ** -8 * np.max(np.abs(g)) + 1e-6


def mlp_params(net):
    return [w.cpu().numpy().astype(np.float64) for w in net.W], [b.cpu().numpy().astype(np.float64) for b in net.b]


@pytest.mark.parametrize("sizes,B", [((64, 128, 128, 64), 128), ((64, 1024, 1024, 1024, 256), 256)])
def test_mlp_forward_backward_vs_oracle(M, sizes, B):
    say("mlp", sizes, B)
    net = M.MLP(sizes, seed=3)
    rng = np.random.default_rng(4)
    x = rng.uniform(0, 1, (B, sizes[0])).astype(np.float32)
    up = rng.standard_normal((B, sizes[-1])).astype(np.float32)
    out, cache = net.forward(torch.from_numpy(x).cuda())
    upd = torch.from_numpy(up).cuda()
    dW, db = net.backward(upd, M.to_bf16(upd), cache)
    torch.cuda.synchronize()
    Ws, bs = mlp_params(net)
    ref, rc = O.mlp_forward(x.astype(np.float64), Ws, bs, emulate_bf16=True)
    close(out.cpu().numpy(), ref, "forward")
    rdW, rdb = O.mlp_backward(up.astype(np.float64), Ws, rc, emulate_bf16=True)
    for i in range(len(Ws)):
        close(dW[i].cpu().numpy(), rdW[i], "dW%d" % i)
        close(db[i].cpu().numpy(), rdb[i], "db%d" % i)


def test_adam_update_matches_oracle(M):
    say("mlp adam")
    from paper_2506_22935_amd import _lib as L
    net = M.MLP((64, 64, 64), seed=5)
    rng = np.random.default_rng(6)
    W0 = net.W[0].cpu().numpy().astype(np.float64)
    g = rng.standard_normal(W0.shape).astype(np.float32)
    dW = [torch.from_numpy(g).cuda(), torch.zeros_like(net.W[1])]
    db = [torch.zeros_like(b) for b in net.b]
    net.adam(dW, db, lr=1e-3)
    net.adam(dW, db, lr=1e-3)
    torch.cuda.synchronize()
    x, m, v = W0, np.zeros_like(W0), np.zeros_like(W0)
    for t in (1, 2):
        x, m, v = O.adam_step(x, g.astype(np.float64), m, v, t, lr=1e-3)
    assert np.max(np.abs(net.W[0].cpu().numpy() - x)) <= 1e-6
    assert torch.equal(net.W16[0], net.W[0].to(torch.bfloat16))


def test_phase_grad_kernel(M):
    say("phase grad")
    rng = np.random.default_rng(7)
    phi = rng.uniform(0, 2 * np.pi, 512)
    s = np.exp(1j * phi).astype(np.complex64)
    g = (rng.standard_normal(512) + 1j * rng.standard_normal(512)).astype(np.complex64)
    out = torch.empty(512, device="cuda")
    M.phase_grad(torch.from_numpy(s).cuda(), torch.from_numpy(g).cuda(), out)
    ref = O.phase_grad(s.astype(np.complex128), g.astype(np.complex128))
    assert np.max(np.abs(out.cpu().numpy() - ref)) <= 1e-6 * np.max(np.abs(ref))

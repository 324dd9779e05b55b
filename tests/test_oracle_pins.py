"""Pins for the float64 oracle: closed forms, identities, brute force and
independent routes (numpy FFT, torch autograd, finite differences).

Each test checks the oracle against something other than itself, so a
dropped term, a wrong sign, a swapped index or a transposed operand in
``oracle/`` fails at least one of them.  CPU only.
"""
import math
import os

import numpy as np
import pytest
import torch

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def rand_complex(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def rand_unimodular(n, seed):
    rng = np.random.default_rng(seed)
    return np.exp(1j * rng.uniform(0, 2 * np.pi, n))


def fft_route(s, m, T):
    """chi through numpy's FFT of each zero-padded lag product."""
    n = len(s)
    out = np.empty((2 * T + 1, m), dtype=np.complex128)
    for i in range(2 * T + 1):
        tau = i - T
        r = np.zeros(m, dtype=np.complex128)
        lo, hi = max(0, tau), min(n, n + tau)
        r[lo:hi] = s[lo:hi] * np.conj(s[lo - tau:hi - tau])
        out[i] = np.fft.fft(r)
    return out


# --------------------------------------------------------------------------
# chi: closed forms and identities
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,m", [(37, 128), (16, 16), (64, 128)])
def test_origin_is_energy_and_peak(n, m):
    s = rand_complex(n, 1)
    c = O.chi(s, m)
    E = O.energy(s)
    T = n - 1
    assert abs(c[T, 0] - E) <= 1e-12 * E
    assert np.max(np.abs(c)) <= E * (1 + 1e-12)  # Cauchy-Schwarz


def test_matches_fft_route():
    s = rand_complex(50, 2)
    for m, T in [(128, 49), (64, 20), (256, 0)]:
        c = O.chi(s, m, T)
        ref = fft_route(s, m, T)
        assert np.max(np.abs(c - ref)) <= 1e-11 * O.energy(s)


def test_lag_doppler_symmetry():
    n, m = 33, 64
    s = rand_complex(n, 3)
    c = O.chi(s, m)
    T = n - 1
    taus = np.arange(-T, T + 1)
    k = np.arange(m)
    # chi(-tau, -k) = exp(-j 2 pi k tau / M) conj(chi(tau, k))
    lhs = c[::-1][:, (-k) % m]
    rhs = np.exp(-2j * np.pi * np.outer(taus, k) / m) * np.conj(c)
    assert np.max(np.abs(lhs - rhs)) <= 1e-11 * O.energy(s)


@pytest.mark.parametrize("n,m", [(32, 32), (32, 64), (20, 128)])
def test_moyal_volume(n, m):
    s = rand_complex(n, 4)
    c = O.chi(s, m)
    E = O.energy(s)
    assert abs(np.sum(np.abs(c) ** 2) - m * E * E) <= 1e-10 * m * E * E


def test_rectangular_pulse_dirichlet():
    n, m = 24, 64
    s = np.ones(n, dtype=np.complex128)
    c = O.chi(s, m)
    T = n - 1
    for i in range(2 * T + 1):
        L = n - abs(i - T)
        for k in range(m):
            if k == 0:
                ref = L
            else:
                ref = abs(math.sin(math.pi * k * L / m) / math.sin(math.pi * k / m))
            assert abs(abs(c[i, k]) - ref) <= 1e-10 * n
    # zero-Doppler cut is the triangle (N - |tau|) / N
    tri = (n - np.abs(np.arange(-T, T + 1))) / n
    assert np.allclose(np.abs(c[:, 0]) / n, tri, atol=1e-13)


def test_unimodular_zero_lag_row_is_phase_free():
    n, m = 40, 128
    s = rand_unimodular(n, 5)
    c = O.chi(s, m)
    row = np.abs(c[n - 1])
    k = np.arange(1, m)
    ref = np.abs(np.sin(np.pi * k * n / m) / np.sin(np.pi * k / m))
    assert abs(row[0] - n) < 1e-10
    assert np.max(np.abs(row[1:] - ref)) < 1e-10


def test_barker13_golden():
    code = abs_acf = None
    with open(os.path.join(HERE, "golden", "barker13.txt")) as f:
        for line in f:
            if line.startswith("code:"):
                code = np.array([float(x) for x in line.split()[1:]])
            elif line.startswith("abs_acf:"):
                abs_acf = np.array([float(x) for x in line.split()[1:]])
    s = code.astype(np.complex128)
    c = O.chi(s, 32)
    cut = np.abs(c[:, 0])
    T = 12
    assert np.allclose(cut[T:], abs_acf, atol=1e-12)
    assert np.allclose(cut[:T + 1][::-1], abs_acf, atol=1e-12)
    # PSL of the zero-Doppler cut: 1/13 in amplitude = -22.3 dB
    side = np.ones(2 * T + 1, dtype=bool)
    side[T] = False
    assert abs(20 * math.log10(cut[side].max() / 13.0) - (-22.2788)) < 1e-3


def test_psl_db_barker13():
    # the oracle's PSL reporter (Eq. 18 in dB) on the Barker-13 zero-Doppler
    # cut, from a power cut and from a magnitude cut, against the golden value
    golden = code = None
    with open(os.path.join(HERE, "golden", "barker13.txt")) as f:
        for line in f:
            if line.startswith("code:"):
                code = np.array([float(x) for x in line.split()[1:]])
            elif line.startswith("psl_db_zero_doppler:"):
                golden = float(line.split()[1])
    s = code.astype(np.complex128)
    T = 12
    c = O.chi(s, 32)[:, 0]
    E = O.energy(s)
    side = np.ones(2 * T + 1, dtype=bool)
    side[T] = False
    p = O.power(c, E)
    assert abs(O.psl_db(p, side) - golden) < 1e-3
    assert abs(O.psl_db(np.sqrt(p), side, is_power=False) - golden) < 1e-3
    # the origin is excluded: with it the level would be 0 dB
    assert abs(O.psl_db(p, np.ones_like(side))) < 1e-12
    # no sidelobe energy: -inf
    assert O.psl_db(np.where(side, 0.0, p), side) == -math.inf


def test_invariances():
    n, m = 21, 64
    s = rand_complex(n, 6)
    a = np.abs(O.chi(s, m))
    k = np.arange(m)
    # global phase: chi unchanged
    assert np.allclose(O.chi(s * np.exp(0.7j), m), O.chi(s, m), atol=1e-11)
    # a frequency offset only adds a lag-dependent phase: |chi| unchanged
    k0 = 5
    sm = s * np.exp(2j * np.pi * k0 * np.arange(n) / m)
    assert np.allclose(np.abs(O.chi(sm, m)), a, atol=1e-11)
    # a quadratic phase exp(j pi c n^2 / M) shears it: row tau moves by c*tau bins
    c = 3
    sq = s * np.exp(1j * np.pi * c * np.arange(n) ** 2 / m)
    aq = np.abs(O.chi(sq, m))
    for i, tau in enumerate(range(-(n - 1), n)):
        assert np.allclose(aq[i], a[i, (k - c * tau) % m], atol=1e-11)
    # conjugation flips Doppler
    assert np.allclose(np.abs(O.chi(np.conj(s), m)), a[:, (-k) % m], atol=1e-11)
    # time reversal keeps |chi|
    assert np.allclose(np.abs(O.chi(s[::-1].copy(), m)), a, atol=1e-11)


def test_lag_window_is_subgrid():
    n, m = 30, 64
    s = rand_complex(n, 7)
    full = O.chi(s, m)
    win = O.chi(s, m, 7)
    assert np.array_equal(win, full[n - 1 - 7:n - 1 + 8])


# --------------------------------------------------------------------------
# losses
# --------------------------------------------------------------------------

def test_isl_full_grid_moyal_pin():
    # uniform-weight ISL over the full grid = M - sum over the mainlobe of p
    n, m = 32, 64
    s = rand_unimodular(n, 8)
    c = O.chi(s, m)
    E = O.energy(s)
    t = O.loss_terms(c, E, n, O.LossParams(h_tau=1, h_k=1))
    main = O.mainlobe_mask(m, n - 1, 1, 1)
    assert abs(t["isl"] - (m - np.sum(O.power(c, E)[main]))) < 1e-9


def test_zero_lag_neighbour_power_at_m_2n():
    n, m = 256, 512
    s = rand_unimodular(n, 9)
    c = O.chi(s, m, 0)
    p = O.power(c, O.energy(s))
    exact = (math.sin(math.pi * n / m) / (n * math.sin(math.pi / m))) ** 2
    assert abs(p[0, 1] - exact) < 1e-12
    assert abs(exact - (2 / math.pi) ** 2) < 1e-4


def test_softpsl_bounds_and_limit():
    n, m = 24, 64
    s = rand_unimodular(n, 10)
    c = O.chi(s, m)
    E = O.energy(s)
    for temp in [0.05, 0.01, 0.001]:
        t = O.loss_terms(c, E, n, O.LossParams(temp=temp, w_psl=1.0))
        amax = t["a"][t["side"]].max()
        count = int(t["side"].sum())
        assert amax - 1e-12 <= t["softpsl"] <= amax + temp * math.log(count) + 1e-12
    t = O.loss_terms(c, E, n, O.LossParams(temp=1e-4, w_psl=1.0))
    assert abs(t["softpsl"] - t["a"][t["side"]].max()) < 1e-3


def test_weighted_isl_brute_force():
    n, m, T = 12, 32, 11
    rng = np.random.default_rng(11)
    u, v = rng.uniform(size=31), rng.uniform(size=31)
    s = rand_unimodular(n, 11)
    c = O.chi(s, m)
    E = O.energy(s)
    t = O.loss_terms(c, E, n, O.LossParams(h_tau=2, h_k=3, u=u, v=v))
    ref = 0.0
    for i in range(2 * T + 1):
        tau = i - T
        for k in range(m):
            kc = k - m if k >= m // 2 else k
            if abs(tau) <= 2 and abs(kc) <= 3:
                continue
            w = u[(31 * abs(tau)) // n] * v[(31 * abs(kc)) // (m // 2 + 1)]
            ref += w * abs(c[i, k]) ** 2 / E ** 2
    assert abs(t["isl"] - ref) < 1e-12


# --------------------------------------------------------------------------
# gradients
# --------------------------------------------------------------------------

def _loss_value(s, m, T, params):
    return O.loss_terms(O.chi(s, m, T), O.energy(s), len(s), params)["loss"]


def _fd_grad(f, s, h=1e-6):
    g = np.zeros(len(s), dtype=np.complex128)
    for p in range(len(s)):
        e = np.zeros(len(s), dtype=np.complex128)
        e[p] = h
        dx = (f(s + e) - f(s - e)) / (2 * h)
        dy = (f(s + 1j * e) - f(s - 1j * e)) / (2 * h)
        g[p] = 0.5 * (dx + 1j * dy)
    return g


CASES = [
    dict(w_isl=1.0, w_psl=0.0),
    dict(w_isl=0.0, w_psl=1.0, temp=0.05),
    dict(w_isl=1.0, w_psl=1.0, temp=0.05),
    dict(w_isl=0.7, w_psl=0.3, temp=0.2, h_tau=2, h_k=2, weighted=True),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("n,m,T", [(8, 16, 7), (13, 32, 12), (16, 32, 5)])
def test_loss_grad_finite_differences(case, n, m, T):
    case = dict(case)
    if case.pop("weighted", False):
        rng = np.random.default_rng(12)
        case.update(u=rng.uniform(size=31), v=rng.uniform(size=31))
    params = O.LossParams(**case)
    s = rand_complex(n, 13)
    g = O.loss_and_grad(s, m, T, params)["g"]
    fd = _fd_grad(lambda x: _loss_value(x, m, T, params), s)
    assert np.max(np.abs(g - fd)) <= 1e-6 * max(1.0, np.max(np.abs(fd)))


def test_magnitude_backward_finite_differences():
    n, m, T, eps = 11, 32, 10, 1e-12
    s = rand_complex(n, 14)
    ga = np.random.default_rng(15).standard_normal((2 * T + 1, m))
    g = O.magnitude_backward(s, m, T, ga, eps)

    def f(x):
        return float(np.sum(ga * O.magnitude(O.chi(x, m, T), O.energy(x), eps)))

    fd = _fd_grad(f, s)
    assert np.max(np.abs(g - fd)) <= 1e-6 * np.max(np.abs(fd))


def test_adjoint_dot_product_exact():
    # L = 2 Re <G, chi(s)>: dL/d conj(s) = adjoint(G); chi is quadratic in
    # (s, conj s), so a central difference of chi is exact up to rounding.
    n, m, T = 19, 64, 12
    s = rand_complex(n, 16)
    d = rand_complex(n, 17)
    rng = np.random.default_rng(18)
    G = rng.standard_normal((2 * T + 1, m)) + 1j * rng.standard_normal((2 * T + 1, m))
    g = O.grad_from_upstream(s, m, T, G, 0.0)
    t = 0.5
    dchi = (O.chi(s + t * d, m, T) - O.chi(s - t * d, m, T)) / (2 * t)
    lhs = 2 * np.real(np.vdot(g, d))
    rhs = 2 * np.real(np.vdot(G, dchi))
    assert abs(lhs - rhs) <= 1e-10 * abs(rhs)


@pytest.mark.parametrize("case", CASES[:3])
def test_normalised_loss_gradient_orthogonal_to_s(case):
    # scale and phase invariance of normalised losses: sum conj(s) g = 0
    n, m = 64, 128
    s = rand_complex(n, 19)
    g = O.loss_and_grad(s, m, n - 1, O.LossParams(**case))["g"]
    assert abs(np.vdot(s, g)) <= 1e-10 * np.linalg.norm(s) * np.linalg.norm(g)


def test_torch_autograd_route():
    # torch's .grad of a real loss w.r.t. a complex leaf is 2 dL/d conj(s)
    n, m, T = 24, 64, 23
    params = O.LossParams(w_isl=1.0, w_psl=0.5, temp=0.1, h_tau=1, h_k=1)
    s = rand_complex(n, 20)
    g = O.loss_and_grad(s, m, T, params)["g"]

    st = torch.tensor(s, dtype=torch.complex128, requires_grad=True)
    E = (st.abs() ** 2).sum()
    rows = []
    for tau in range(-T, T + 1):
        lo, hi = max(0, tau), min(n, n + tau)
        r = torch.zeros(m, dtype=torch.complex128)
        r = r.index_put((torch.arange(lo, hi),), st[lo:hi] * torch.conj(st[lo - tau:hi - tau]))
        rows.append(torch.fft.fft(r))
    c = torch.stack(rows)
    p = (c.abs() ** 2) / E ** 2
    a = torch.sqrt(p + params.eps)
    side = torch.tensor(~O.mainlobe_mask(m, T, 1, 1))
    isl = p[side].sum()
    soft = params.temp * torch.logsumexp(a[side] / params.temp, dim=0)
    (params.w_isl * isl + params.w_psl * soft).backward()
    assert np.max(np.abs(st.grad.numpy() / 2 - g)) <= 1e-9 * np.max(np.abs(g))


def test_phase_grad_chain():
    n, m = 16, 32
    phi = np.random.default_rng(21).uniform(0, 2 * np.pi, n)
    params = O.LossParams(w_isl=1.0, w_psl=1.0)

    def f(ph):
        return _loss_value(np.exp(1j * ph), m, n - 1, params)

    s = np.exp(1j * phi)
    dphi = O.phase_grad(s, O.loss_and_grad(s, m, n - 1, params)["g"])
    h = 1e-6
    fd = np.array([(f(phi + h * e) - f(phi - h * e)) / (2 * h) for e in np.eye(n)])
    assert np.max(np.abs(dphi - fd)) <= 1e-6 * np.max(np.abs(fd))


# --------------------------------------------------------------------------
# optimiser and network
# --------------------------------------------------------------------------

def test_adam_matches_torch():
    rng = np.random.default_rng(22)
    x0 = rng.standard_normal(10)
    grads = [rng.standard_normal(10) for _ in range(5)]
    xt = torch.tensor(x0, requires_grad=True)
    opt = torch.optim.Adam([xt], lr=0.01, betas=(0.9, 0.999), eps=1e-8)
    x, m, v = x0.copy(), np.zeros(10), np.zeros(10)
    for t, gr in enumerate(grads, start=1):
        opt.zero_grad()
        xt.grad = torch.tensor(gr)
        opt.step()
        x, m, v = O.adam_step(x, gr, m, v, t)
    assert np.max(np.abs(x - xt.detach().numpy())) < 1e-14


def test_adam_first_step_is_signed_lr():
    x, m, v = O.adam_step(np.zeros(3), np.array([2.0, -3.0, 0.5]), np.zeros(3), np.zeros(3), 1)
    assert np.allclose(x, -0.01 * np.sign([2.0, -3.0, 0.5]), atol=1e-9)


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(23)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-5, 5, 10000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 65504.0]])
    x32 = x.astype(np.float32)
    ref = torch.tensor(x32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(O.bf16_round(x32), ref)


def test_gelu_and_grad():
    x = np.linspace(-6, 6, 101)
    xt = torch.tensor(x, requires_grad=True)
    y = torch.nn.functional.gelu(xt)
    y.sum().backward()
    assert np.max(np.abs(O.gelu(x) - y.detach().numpy())) < 1e-14
    assert np.max(np.abs(O.gelu_grad(x) - xt.grad.numpy())) < 1e-14


def test_mlp_backward_matches_torch_and_fd():
    rng = np.random.default_rng(24)
    sizes = [6, 8, 8, 5]
    Ws = [rng.standard_normal((sizes[i + 1], sizes[i])) * 0.5 for i in range(3)]
    bs = [rng.standard_normal(sizes[i + 1]) * 0.1 for i in range(3)]
    x = rng.standard_normal((4, 6))
    up = rng.standard_normal((4, 5))
    out, cache = O.mlp_forward(x, Ws, bs, emulate_bf16=False)
    dW, db = O.mlp_backward(up, Ws, cache, emulate_bf16=False)

    Wt = [torch.tensor(w, requires_grad=True) for w in Ws]
    bt = [torch.tensor(b, requires_grad=True) for b in bs]
    a = torch.tensor(x)
    for i in range(3):
        a = a @ Wt[i].T + bt[i]
        if i < 2:
            a = torch.nn.functional.gelu(a)
    assert np.max(np.abs(a.detach().numpy() - out)) < 1e-13
    (a * torch.tensor(up)).sum().backward()
    for i in range(3):
        assert np.max(np.abs(dW[i] - Wt[i].grad.numpy())) < 1e-12
        assert np.max(np.abs(db[i] - bt[i].grad.numpy())) < 1e-12
    # finite difference on one weight
    h = 1e-6
    Wp = [w.copy() for w in Ws]
    Wp[1][2, 3] += h
    Wm = [w.copy() for w in Ws]
    Wm[1][2, 3] -= h
    fp = np.sum(O.mlp_forward(x, Wp, bs, False)[0] * up)
    fm = np.sum(O.mlp_forward(x, Wm, bs, False)[0] * up)
    assert abs((fp - fm) / (2 * h) - dW[1][2, 3]) < 1e-7


# --------------------------------------------------------------------------
# FFT-step route of the oracle (used at sizes the direct sums cannot reach)
# --------------------------------------------------------------------------

def test_fft_rows_match_direct_sum():
    n, m, T = 45, 128, 30
    s = rand_complex(n, 30)
    taus = [-30, -7, 0, 1, 29]
    direct = O.chi(s, m, T)[[t + T for t in taus]]
    assert np.max(np.abs(O.chi_rows_fft(s, m, taus) - direct)) <= 1e-11 * O.energy(s)


def test_fft_backward_matches_direct_sum():
    n, m, T, eps = 40, 128, 17, 1e-12
    s = rand_complex(n, 31)
    ga = np.random.default_rng(32).standard_normal((2 * T + 1, m))
    ref = O.magnitude_backward(s, m, T, ga, eps)
    got = O.magnitude_backward_fft(s, m, T, ga, eps, rows_per_block=7)
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_chi_rows_is_the_direct_grid():
    n, m, T = 29, 64, 28
    s = rand_complex(n, 33)
    taus = [-28, -3, 0, 5, 28]
    assert np.array_equal(O.chi_rows(s, m, taus), O.chi(s, m, T)[[t + T for t in taus]])


# --------------------------------------------------------------------------
# the periodic (circular) AF, Eqs. 2 and 7 and Algorithm 1
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [8, 16, 32])
def test_circular_is_folded_aperiodic(n):
    # with N Doppler bins, lag tau of the periodic product collects the
    # aperiodic lags tau and tau - N: chi_c(tau) = chi(tau) + chi(tau - N)
    s = rand_complex(n, 40 + n)
    cc = O.chi_circular(s)
    ca = O.chi(s, n)  # rows tau = -(N-1) .. N-1, M = N bins
    T = n - 1
    assert np.max(np.abs(cc[0] - ca[T])) <= 1e-12 * O.energy(s)
    for tau in range(1, n):
        assert np.max(np.abs(cc[tau] - (ca[T + tau] + ca[T + tau - n]))) <= 1e-12 * O.energy(s)


@pytest.mark.parametrize("n", [7, 16, 24])
def test_circular_moyal_origin_peak_symmetry(n):
    s = rand_complex(n, 50 + n)
    c = O.chi_circular(s)
    E = O.energy(s)
    # sum over the N x N grid of |chi_c|^2 = N E^2 (each sample product
    # |s[n]|^2 |s[n - tau]|^2 summed over tau gives E |s[n]|^2)
    assert abs(np.sum(np.abs(c) ** 2) - n * E * E) <= 1e-11 * n * E * E
    assert abs(c[0, 0] - E) <= 1e-12 * E
    assert np.max(np.abs(c)) <= E * (1 + 1e-12)
    # |chi_c(-tau, -k)| = |chi_c(tau, k)| with indices modulo N
    idx = (-np.arange(n)) % n
    assert np.max(np.abs(np.abs(c[idx][:, idx]) - np.abs(c))) <= 1e-11 * E


@pytest.mark.parametrize("n,u", [(16, 3), (64, 5), (15, 2), (13, 4)])
def test_zadoff_chu_periodic_af_is_a_line(n, u):
    # Zadoff-Chu: s[n] = exp(j pi u n^2 / N) (N even), exp(j pi u n (n+1) / N)
    # (N odd), gcd(u, N) = 1.  The periodic lag product is a pure tone of
    # frequency u tau, so |chi_c(tau, k)| = N where k = u tau mod N, else 0.
    k = np.arange(n)
    s = np.exp(1j * np.pi * u * (k * k if n % 2 == 0 else k * (k + 1)) / n)
    a = np.abs(O.chi_circular(s))
    line = np.zeros((n, n), dtype=bool)
    line[np.arange(n), (u * np.arange(n)) % n] = True
    assert np.max(np.abs(a[line] - n)) <= 1e-10 * n
    assert np.max(a[~line]) <= 1e-10 * n


def test_circular_rectangular_pulse():
    # s = 1: every periodic lag product is 1, so chi_c(tau, k) = N delta_k
    n = 32
    c = O.chi_circular(np.ones(n))
    ref = np.zeros((n, n))
    ref[:, 0] = n
    assert np.max(np.abs(c - ref)) <= 1e-10 * n


def test_circular_isl_complement_and_mask():
    # uniform full-grid ISL = N - sum of mainlobe power (periodic Moyal);
    # the mainlobe holds (2 h_tau + 1)(2 h_k + 1) cells
    n = 32
    s = rand_unimodular(n, 60)
    params = O.LossParams(w_isl=1.0, h_tau=2, h_k=1)
    t = O.loss_and_grad_circular(s, params)
    main = O.circular_mainlobe_mask(n, 2, 1)
    assert main.sum() == 5 * 3
    assert main[n - 2, 0] and main[2, n - 1] and not main[3, 0] and not main[0, 2]
    assert abs(t["isl"] - (n - np.sum(t["p"][main]))) <= 1e-10 * n


def _loss_value_circ(s, params):
    return O.loss_and_grad_circular(s, params)["loss"]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("n", [8, 12])
def test_circular_loss_grad_finite_differences(case, n):
    case = dict(case)
    if case.pop("weighted", False):
        rng = np.random.default_rng(14)
        case.update(u=rng.uniform(size=31), v=rng.uniform(size=31))
    params = O.LossParams(**case)
    s = rand_complex(n, 70 + n)
    g = O.loss_and_grad_circular(s, params)["g"]
    fd = _fd_grad(lambda x: _loss_value_circ(x, params), s)
    assert np.max(np.abs(g - fd)) <= 1e-6 * max(1.0, np.max(np.abs(fd)))


def test_circular_magnitude_backward_finite_differences():
    n, eps = 10, 1e-12
    s = rand_complex(n, 80)
    rng = np.random.default_rng(81)
    ga = rng.standard_normal((n, n))

    def f(x):
        c = O.chi_circular(x)
        return float(np.sum(ga * O.magnitude(c, O.energy(x), eps)))

    g = O.magnitude_backward_circular(s, ga, eps)
    fd = _fd_grad(f, s)
    assert np.max(np.abs(g - fd)) <= 1e-6 * max(1.0, np.max(np.abs(fd)))


def test_circular_normalised_gradient_orthogonal_to_s():
    # the normalised losses are invariant to s -> c s (c complex), so
    # sum_n conj(s_n) g_n = 0 for the periodic AF too
    s = rand_complex(16, 90)
    g = O.loss_and_grad_circular(s, O.LossParams(w_isl=1.0, w_psl=1.0, temp=0.1))["g"]
    assert abs(np.vdot(s, g)) <= 1e-12 * np.linalg.norm(s) * np.linalg.norm(g) * 16


def test_circular_rows_match_the_grid():
    s = rand_complex(64, 91)
    c = O.chi_circular(s)
    taus = [0, 1, 31, 32, 33, 63]
    assert np.max(np.abs(O.chi_circular_rows(s, taus) - c[taus])) <= 1e-12 * O.energy(s)


# --------------------------------------------------------------------------
# the experiment loss of Sec. 7.1.1: hard PSL + lambda alpha SpectralVariance
# --------------------------------------------------------------------------

def test_spectral_variance_closed_forms():
    n = 64
    # an impulse and a Zadoff-Chu code have flat spectra: V = 0
    assert O.spectral_variance(np.eye(n)[3])[0] <= 1e-30
    k = np.arange(n)
    assert O.spectral_variance(np.exp(1j * np.pi * 5 * k * k / n))[0] <= 1e-28
    # a constant code puts all power in bin 0: x = (1, 0, ..., 0)
    V = O.spectral_variance(np.ones(n))[0]
    assert abs(V - (1.0 / n - 1.0 / n ** 2)) <= 1e-15
    # matches numpy's FFT and population variance
    s = rand_complex(n, 95)
    P = np.abs(np.fft.fft(s)) ** 2
    assert abs(O.spectral_variance(s)[0] - np.var(P / P.sum())) <= 1e-15


@pytest.mark.parametrize("n", [8, 16, 13])
def test_spectral_variance_gradient_finite_differences(n):
    s = rand_complex(n, 96 + n)
    V, g = O.spectral_variance(s)
    fd = _fd_grad(lambda x: O.spectral_variance(x)[0], s)
    assert np.max(np.abs(g - fd)) <= 1e-7 * max(1e-3, np.max(np.abs(fd)))
    # V is invariant to s -> c s, so sum conj(s) g = 0
    assert abs(np.vdot(s, g)) <= 1e-12 * np.linalg.norm(s) * np.linalg.norm(g) * n


def test_hard_psl_is_the_brute_force_max():
    n, m = 16, 32
    s = rand_unimodular(n, 97)
    c = O.chi(s, m)
    E = O.energy(s)
    side = ~O.mainlobe_mask(m, n - 1, 1, 1)
    psl, cell = O.hard_psl(c, E, side)
    best = max(abs(c[i, k]) ** 2 / E ** 2 for i in range(2 * n - 1) for k in range(m) if side[i, k])
    assert abs(psl - best) <= 1e-15 and side[cell]
    assert abs(abs(c[cell]) ** 2 / E ** 2 - psl) <= 1e-15


@pytest.mark.parametrize("periodic,n,m", [(True, 8, 8), (True, 16, 16), (False, 8, 16)])
@pytest.mark.parametrize("lam", [0.0, 0.5, 2.0])
def test_experiment_loss_finite_differences(periodic, n, m, lam):
    # away from ties the hard max is smooth: central differences of L agree
    # with the subgradient on the maximising cell plus the spectral part
    s = rand_complex(n, 98 + n + int(periodic))

    def f(x):
        return O.experiment_loss_and_grad(x, m, lam, periodic=periodic)["loss"]

    r = O.experiment_loss_and_grad(s, m, lam, periodic=periodic)
    p = O.power(r["chi"], r["E"])[r["side"]]
    top = np.sort(np.unique(np.round(p, 14)))[-2:]
    assert top[1] - top[0] > 1e-6  # a unique maximum up to its twin cell
    fd = _fd_grad(f, s, h=1e-7)
    assert np.max(np.abs(r["g"] - fd)) <= 1e-5 * max(1.0, np.max(np.abs(fd)))


# --------------------------------------------------------------------------
# L_match of the composite loss (Sec. 5.2): sum (p - p_target)^2
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n,m,T", [(8, 16, 7), (13, 32, 4)])
def test_match_loss_finite_differences(n, m, T):
    rng = np.random.default_rng(n + T)
    target = rng.uniform(0, 0.2, (2 * T + 1, m))
    params = O.LossParams(w_isl=0.3, w_match=2.0, match=target)
    s = rand_complex(n, 120 + n)
    g = O.loss_and_grad(s, m, T, params)["g"]
    fd = _fd_grad(lambda x: _loss_value(x, m, T, params), s)
    assert np.max(np.abs(g - fd)) <= 1e-6 * max(1.0, np.max(np.abs(fd)))


def test_match_loss_is_zero_at_its_own_surface():
    # the target surface of the waveform itself is the minimum: L = 0, g = 0,
    # and a scaled or phase-rotated copy of s matches as well
    n, m = 16, 32
    s = rand_complex(n, 130)
    p = O.power(O.chi(s, m), O.energy(s))
    params = O.LossParams(w_isl=0.0, w_match=1.0, match=p)
    r = O.loss_and_grad(s, m, n - 1, params)
    assert r["match"] <= 1e-28 and np.max(np.abs(r["g"])) <= 1e-12
    r2 = O.loss_and_grad(2.5j * s, m, n - 1, params)
    assert r2["match"] <= 1e-26


# ---- remaining composite terms: soft mainlobe width (Eq. 21), var(|s|),
# phase smoothness, and the spectral-mask projection (Sec. 6.2)

def test_soft_width_sharp_limit_rectangular_pulse():
    # s = 1: p(tau, 0) = ((N - |tau|) / N)^2, above one half for tau <= 18 at
    # N = 64 (p(18) = 0.517, p(19) = 0.494): with a sharp sigmoid Eq. 21 counts
    # |tau| over those lags, 2 (1 + ... + 18) = 342
    n = 64
    s = np.ones(n, dtype=np.complex128)
    t = O.loss_and_grad(s, 128, n - 1, O.LossParams(w_isl=0.0, w_width=1.0, gamma=1e4))
    assert abs(t["width"] - 342.0) < 1e-9
    assert abs(t["loss"] - 342.0) < 1e-9
    # at gamma = 0 every row weighs one half: sum |tau| / 2 = N (N - 1) / 2
    t0 = O.loss_and_grad(s, 128, n - 1, O.LossParams(w_isl=0.0, w_width=1.0, gamma=0.0))
    assert abs(t0["width"] - n * (n - 1) / 2.0) < 1e-9


def test_soft_width_periodic_constant_code():
    # the periodic autocorrelation of a constant is N at every lag: p(tau, 0) = 1
    # and every row sits at sigma(gamma / 2); sum_tau |tau|_c = N^2 / 4
    n = 64
    s = np.full(n, 0.5 - 0.25j)
    for gamma in (0.5, 3.0):
        t = O.loss_and_grad_circular(s, O.LossParams(w_isl=0.0, w_width=1.0, gamma=gamma))
        assert abs(t["width"] - n * n / 4.0 / (1.0 + math.exp(-gamma / 2.0))) < 1e-9


def test_modulus_variance_and_smoothness_closed_forms():
    n = 40
    phi = np.random.default_rng(3).uniform(-np.pi, np.pi, n)
    s = np.exp(1j * phi)
    v, g = O.modulus_variance(s)
    assert v < 1e-28 and np.max(np.abs(g)) < 1e-15
    # two amplitude levels a, b in equal numbers: var = ((a - b) / 2)^2
    r = np.where(np.arange(n) % 2 == 0, 1.5, 0.25)
    v, _ = O.modulus_variance(r * s)
    assert abs(v - (1.25 / 2) ** 2) < 1e-14
    # linear phase step theta: (N - 1) |e^{j theta} - 1|^2 / N = (N - 1)(2 - 2 cos theta) / N
    theta = 0.3
    sm, _ = O.phase_smoothness(np.exp(1j * theta * np.arange(n)))
    assert abs(sm - (n - 1) * (2 - 2 * math.cos(theta)) / n) < 1e-14
    sm, g = O.phase_smoothness(np.full(n, 2.0 - 1.0j))
    assert sm == 0.0 and np.max(np.abs(g)) < 1e-15


@pytest.mark.parametrize("periodic", [False, True])
def test_width_const_smooth_finite_differences(periodic):
    n = 32
    s = rand_complex(n, 44) * (1.0 + 0.3 * np.cos(np.arange(n)))
    params = O.LossParams(w_isl=0.3, w_width=0.7, gamma=6.0, w_const=1.3, w_smooth=0.9)
    if periodic:
        f = lambda x: O.loss_and_grad_circular(x, params)["loss"]
        t = O.loss_and_grad_circular(s, params)
    else:
        f = lambda x: O.loss_and_grad(x, 64, n - 1, params)["loss"]
        t = O.loss_and_grad(s, 64, n - 1, params)
    g = _fd_grad(f, s)
    assert np.max(np.abs(t["g"] - g)) < 1e-6 * np.max(np.abs(g))
    # the pieces add up with their weights
    base = O.LossParams(w_isl=0.3)
    b = O.loss_and_grad_circular(s, base) if periodic else O.loss_and_grad(s, 64, n - 1, base)
    assert abs(t["loss"] - (b["loss"] + 0.7 * t["width"] + 1.3 * t["const"] + 0.9 * t["smooth"])) < 1e-9


def test_width_gradient_isolated_finite_differences():
    # the width term alone, including the origin-cell term, on a lag window
    n, m, T = 24, 64, 9
    s = rand_complex(n, 45)
    params = O.LossParams(w_isl=0.0, w_width=1.0, gamma=4.0)
    t = O.loss_and_grad(s, m, T, params)
    g = _fd_grad(lambda x: O.loss_and_grad(x, m, T, params)["loss"], s)
    assert np.max(np.abs(t["g"] - g)) < 1e-6 * np.max(np.abs(g))


def test_spectral_projection_two_tones():
    n = 48
    k = np.arange(n)
    a, b = 0.8 - 0.3j, -0.2 + 1.1j
    s = a * np.exp(2j * np.pi * 5 * k / n) + b * np.exp(2j * np.pi * 31 * k / n)
    mask = np.zeros(n)
    mask[5] = 1.0
    y = O.spectral_projection(s, mask)
    assert np.max(np.abs(y - a * np.exp(2j * np.pi * 5 * k / n))) < 1e-13
    # all-pass mask: identity; a 0/1 mask: idempotent; unit: on the circle
    assert np.max(np.abs(O.spectral_projection(s, np.ones(n)) - s)) < 1e-13
    s2 = rand_complex(n, 46)
    band = (np.abs(np.where(k < n // 2, k, k - n)) <= 10).astype(np.float64)
    y1 = O.spectral_projection(s2, band)
    assert np.max(np.abs(O.spectral_projection(y1, band) - y1)) < 1e-13
    yu = O.spectral_projection(s2, band, unit=True)
    assert np.max(np.abs(np.abs(yu) - 1.0)) < 1e-14
    assert np.max(np.abs(np.angle(yu * np.conj(y1)))) < 1e-12
    # a half-weight mask scales a tone by one half
    mask[5] = 0.5
    assert np.max(np.abs(O.spectral_projection(s, mask) - 0.5 * a * np.exp(2j * np.pi * 5 * k / n))) < 1e-13


# ---- cross-ambiguity (two waveforms)

def test_cross_af_with_itself_is_the_af():
    n, m, T = 40, 128, 17
    s = rand_complex(n, 50)
    c = O.cross_chi(s, s, m, T)
    ref = O.chi(s, m, T)
    assert np.max(np.abs(c - ref)) < 1e-10 * np.max(np.abs(ref))


def test_cross_af_swap_delay_and_volume():
    n, m = 48, 128
    s = rand_complex(n, 51)
    u = rand_complex(n, 52)
    c_su = O.cross_chi(s, u, m)
    c_us = O.cross_chi(u, s, m)
    T = n - 1
    tau = np.arange(-T, T + 1)[:, None]
    k = np.arange(m)[None, :]
    # chi_us(tau, k) = exp(-j 2 pi k tau / M) conj(chi_su(-tau, -k))
    flip = np.conj(c_su[::-1][:, (-np.arange(m)) % m])
    assert np.max(np.abs(c_us - np.exp(-2j * np.pi * k * tau / m) * flip)) < 1e-10 * np.max(np.abs(c_su))
    # cross Moyal volume: sum over the full grid of |chi_su|^2 = M E_s E_u
    vol = float(np.sum(np.abs(c_su) ** 2))
    assert abs(vol - m * O.energy(s) * O.energy(u)) < 1e-10 * vol
    # a delayed copy u[n] = s[n - d] moves the lag: chi_su(tau) = chi_ss(tau + d)
    d = 5
    s2 = s.copy()
    s2[n - d:] = 0.0
    u2 = np.zeros(n, dtype=np.complex128)
    u2[d:] = s2[:n - d]
    c = O.cross_chi(s2, u2, m)
    a = O.chi(s2, m, T)
    assert np.max(np.abs(c[:2 * T + 1 - d] - a[d:])) < 1e-10 * np.max(np.abs(a))
    # Cauchy-Schwarz: |chi_su|^2 <= E_s E_u
    assert np.max(np.abs(c_su) ** 2) <= O.energy(s) * O.energy(u) * (1 + 1e-12)


def test_cross_magnitude_backward_finite_differences():
    n, m, T = 14, 32, 9
    s = rand_complex(n, 53)
    u = rand_complex(n, 54)
    w = np.random.default_rng(55).standard_normal((2 * T + 1, m))
    eps = 1e-9

    def f(x, y):
        c = O.cross_chi(x, y, m, T)
        p = np.abs(c) ** 2 / (O.energy(x) * O.energy(y))
        return float(np.sum(w * np.sqrt(p + eps)))

    gs, gu = O.cross_magnitude_backward(s, u, m, T, w, eps)
    fs = _fd_grad(lambda x: f(x, u), s)
    fu = _fd_grad(lambda y: f(s, y), u)
    assert np.max(np.abs(gs - fs)) < 1e-6 * np.max(np.abs(fs))
    assert np.max(np.abs(gu - fu)) < 1e-6 * np.max(np.abs(fu))
    # with u = s the two gradients add up to the AF's magnitude backward
    ga, gb = O.cross_magnitude_backward(s, s, m, T, w, eps)
    ref = O.magnitude_backward(s, m, T, w, eps)
    assert np.max(np.abs(ga + gb - ref)) < 1e-9 * np.max(np.abs(ref))


def test_cross_af_periodic_pins():
    n = 16
    s = rand_complex(n, 56)
    u = rand_complex(n, 57)
    c = O.cross_chi_circular(s, u)
    # u = s: the periodic AF (the C core's direct sum)
    cs = O.cross_chi_circular(s, s)
    ref = O.chi_circular(s)
    assert np.max(np.abs(cs - ref)) < 1e-12 * np.max(np.abs(ref))
    # periodic lag tau collects the aperiodic cross lags tau and tau - N (M = N)
    ap = O.cross_chi(s, u, n)
    T = n - 1
    for tau in range(n):
        row = ap[T + tau] + (ap[T + tau - n] if tau > 0 else 0.0)
        assert np.max(np.abs(c[tau] - row)) < 1e-12 * np.max(np.abs(c))
    # Parseval over each row: sum over the grid of |chi_su|^2 = N E_s E_u
    vol = float(np.sum(np.abs(c) ** 2))
    assert abs(vol - n * O.energy(s) * O.energy(u)) < 1e-12 * vol
    # a circular delay of u moves the rows: u[n] = s[(n - d) mod N] gives
    # chi_su[tau] = chi_ss[(tau + d) mod N]
    d = 5
    c2 = O.cross_chi_circular(s, np.roll(s, d))
    assert np.max(np.abs(c2 - np.roll(ref, -d, axis=0))) < 1e-12 * np.max(np.abs(ref))
    # selected bins are the matching columns
    assert np.max(np.abs(O.cross_chi_circular(s, u, bins=[0, 3, 15]) - c[:, [0, 3, 15]])) < 1e-12


def test_cross_magnitude_backward_circular_finite_differences():
    n = 8
    s = rand_complex(n, 58)
    u = rand_complex(n, 59)
    w = np.random.default_rng(60).standard_normal((n, n))
    eps = 1e-9

    def f(x, y):
        c = O.cross_chi_circular(x, y)
        p = np.abs(c) ** 2 / (O.energy(x) * O.energy(y))
        return float(np.sum(w * np.sqrt(p + eps)))

    gs, gu = O.cross_magnitude_backward_circular(s, u, w, eps)
    fs = _fd_grad(lambda x: f(x, u), s)
    fu = _fd_grad(lambda y: f(s, y), u)
    assert np.max(np.abs(gs - fs)) < 1e-6 * np.max(np.abs(fs))
    assert np.max(np.abs(gu - fu)) < 1e-6 * np.max(np.abs(fu))
    # with u = s the two gradients add up to the periodic AF's magnitude
    # backward (the C core's adjoint)
    ga, gb = O.cross_magnitude_backward_circular(s, s, w, eps)
    ref = O.magnitude_backward_circular(s, w, eps)
    assert np.max(np.abs(ga + gb - ref)) < 1e-9 * np.max(np.abs(ref))


# ---- multi-scenario loss (Eq. 24) and per-cell weight grids

def test_cell_weights_reduce_to_weighted_isl():
    # a weight grid equal to the ISL weights (zero on the mainlobe) is the ISL
    n, m, T = 24, 64, 23
    s = rand_complex(n, 60)
    W = O.isl_weights(n, m, T, 1, 1)
    a = O.loss_and_grad(s, m, T, O.LossParams(w_isl=1.0))
    b = O.loss_and_grad(s, m, T, O.LossParams(w_isl=0.0, cell_w=W, w_cell=1.0))
    assert abs(a["loss"] - b["loss"]) < 1e-12 * a["loss"]
    assert np.max(np.abs(a["g"] - b["g"])) < 1e-12 * np.max(np.abs(a["g"]))


@pytest.mark.parametrize("periodic", [False, True])
def test_multi_scenario_is_one_pass_with_combined_weights(periodic):
    # Eq. 24 with weight-grid scenarios (target profiles), evaluated scenario
    # by scenario, equals one loss with the combined grid; finite differences
    n, m = 32, 64
    T = n - 1
    s = rand_complex(n, 61)
    rows = n if periodic else 2 * T + 1
    cols = n if periodic else m
    rng = np.random.default_rng(62)
    grids = [rng.uniform(0, 1, (rows, cols)) * (rng.uniform(0, 1, (rows, 1)) < 0.5) for _ in range(3)]
    lams = [0.5, 2.0, 1.25]
    scen = [O.LossParams(w_isl=0.0, cell_w=w, w_cell=1.0, w_smooth=0.1 * i) for i, w in enumerate(grids)]
    L, g = O.multi_scenario_loss_and_grad(s, m, T, scen, lams, periodic=periodic)
    one = O.LossParams(w_isl=0.0, cell_w=O.combine_scenario_weights(grids, lams), w_cell=1.0,
                       w_smooth=0.1 * (0 * 0.5 + 1 * 2.0 + 2 * 1.25))
    t = O.loss_and_grad_circular(s, one) if periodic else O.loss_and_grad(s, m, T, one)
    assert abs(L - t["loss"]) < 1e-11 * abs(L)
    assert np.max(np.abs(g - t["g"])) < 1e-11 * np.max(np.abs(g))
    f = (lambda x: O.multi_scenario_loss_and_grad(x, m, T, scen, lams, periodic=periodic)[0])
    gf = _fd_grad(f, s)
    assert np.max(np.abs(g - gf)) < 1e-6 * np.max(np.abs(gf))

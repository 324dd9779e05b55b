"""Float64 reference for everything the HIP path computes.

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` use it; the product path never does.

Conventions (shared by the definitions below and the paper's Secs. 3-5):
  * waveform s in C^N, zero outside [0, N); lags tau in [-T, T]; Doppler bins
    k in [0, M), M a power of two; centred bin k_c = ((k + M/2) mod M) - M/2.
  * chi[tau, k] = sum_n s[n] conj(s[n - tau]) exp(-j 2 pi k n / M)   (Eqs. 7-11)
  * E = sum |s|^2 = chi[0, 0] (the maximum of |chi|, Eq. 17's normaliser)
  * p = |chi|^2 / E^2 (the paper's chi, Eq. 12, divided by its peak)
  * a = sqrt(p + eps) (the eps-stabilised normalised magnitude)
  * every gradient is the conjugate Wirtinger derivative dL/d conj(.)
    (Sec. 3.3 Eq. 6 and Sec. 4.2 Eqs. 13-14).
Arrays are numpy; grids are [2T+1, M] with row i <-> tau = i - T.
"""
import math

import numpy as np
from scipy.special import erf

from . import _native

__all__ = [
    "to_c64_exact", "energy", "chi", "chi_rows", "magnitude", "power",
    "centred_bins", "mainlobe_mask", "isl_weights", "LossParams", "loss_terms",
    "loss_and_grad", "loss_grad_from_chi", "sigmoid", "soft_mainlobe_width", "modulus_variance",
    "phase_smoothness", "spectral_projection", "cross_chi", "cross_magnitude_backward", "cross_chi_circular",
    "cross_magnitude_backward_circular",
    "multi_scenario_loss_and_grad", "combine_scenario_weights", "magnitude_backward", "grad_from_upstream", "phase_grad",
    "adam_step", "bf16_round", "gelu", "gelu_grad", "mlp_forward",
    "mlp_backward", "psl_db", "chi_rows_fft", "magnitude_backward_fft",
    "chi_circular", "chi_circular_rows", "circular_lag_distance", "circular_mainlobe_mask", "circular_isl_weights",
    "loss_and_grad_circular", "magnitude_backward_circular",
    "spectral_variance", "hard_psl", "experiment_loss_and_grad",
]


# ----------------------------------------------------------------------------
# inputs
# ----------------------------------------------------------------------------

def to_c64_exact(s):
    """The complex64 value of s, widened to complex128 (the bits the GPU sees)."""
    return np.asarray(s).astype(np.complex64).astype(np.complex128)


def energy(s):
    """E = sum_n |s[n]|^2 (Sec. 4.3: the value of chi at the origin)."""
    s = np.asarray(s, dtype=np.complex128)
    return float(np.sum(s.real * s.real + s.imag * s.imag))


# ----------------------------------------------------------------------------
# the ambiguity function (Sec. 4.1, Eqs. 7-12)
# ----------------------------------------------------------------------------

def chi(s, m, max_lag=None):
    """Complex AF by its defining sum (C core, direct DFT, no FFT)."""
    s = np.asarray(s, dtype=np.complex128)
    T = s.shape[0] - 1 if max_lag is None or max_lag < 0 else int(max_lag)
    return _native.chi(s, int(m), T)


def chi_rows(s, m, taus):
    """Rows of chi for selected lags, by the same direct sums (C core)."""
    return _native.chi_rows(np.asarray(s, dtype=np.complex128), int(m), taus)


def power(c, E):
    """p = |chi|^2 / E^2."""
    return (c.real * c.real + c.imag * c.imag) / (E * E)


def magnitude(c, E, eps):
    """a = sqrt(|chi|^2 / E^2 + eps)."""
    return np.sqrt(power(c, E) + eps)


def psl_db(a_or_p, sidelobe, is_power=True):
    """Peak sidelobe level, Eq. 18, in dB of power relative to the origin."""
    v = a_or_p[sidelobe]
    pk = float(v.max()) if is_power else float(v.max()) ** 2
    return 10.0 * math.log10(pk) if pk > 0 else -math.inf


# ----------------------------------------------------------------------------
# regions and weights (Eqs. 18-19: the sidelobe region Omega_s)
# ----------------------------------------------------------------------------

def centred_bins(m):
    k = np.arange(m)
    return ((k + m // 2) % m) - m // 2


def mainlobe_mask(m, max_lag, h_tau, h_k):
    """True on the mainlobe |tau| <= h_tau and |k_c| <= h_k."""
    taus = np.arange(-max_lag, max_lag + 1)
    kc = centred_bins(m)
    return (np.abs(taus)[:, None] <= h_tau) & (np.abs(kc)[None, :] <= h_k)


def isl_weights(n, m, max_lag, h_tau, h_k, u=None, v=None):
    """ISL weight per cell: 0 on the mainlobe; 1 elsewhere, or the separable
    shaping weight u[floor(31|tau|/N)] * v[floor(31|k_c|/(M/2+1))] when the
    31-entry vectors u, v are given (integer floor division)."""
    main = mainlobe_mask(m, max_lag, h_tau, h_k)
    if u is None:
        W = np.ones((2 * max_lag + 1, m))
    else:
        u = np.asarray(u, dtype=np.float64)
        v = np.asarray(v, dtype=np.float64)
        taus = np.abs(np.arange(-max_lag, max_lag + 1))
        kc = np.abs(centred_bins(m))
        iu = (31 * taus) // n
        iv = (31 * kc) // (m // 2 + 1)
        W = u[iu][:, None] * v[iv][None, :]
    W[main] = 0.0
    return W


class LossParams:
    """L = w_isl ISL + w_psl softPSL + w_match Match + w_width Width
         + w_const Const + w_smooth Smooth.

    ISL = sum_{Omega_s} W p                         (Eq. 19, weighted)
    softPSL = T log sum_{Omega_s} exp(a / T)        (smooth stand-in for Eq. 18)
    Match = sum over every cell of (p - p_target)^2 (L_match of Sec. 5.2 with
            the AF in power, as the paper's chi, against a target surface
            p_target laid out like the grid)
    Width = sum over the lag rows of |tau| sigma(gamma (p(tau, 0) - p(0, 0)/2))
            (Eq. 21 on the power-normalised AF, whose half-power level is
            the -3 dB level of Eq. 20; |tau|_c on the periodic AF)
    Const = var(|s|)                                (L_const of Sec. 5.2)
    Smooth = sum_n |s[n+1] - s[n]|^2 / E            (phase continuity, Sec. 6.2)
    Cell = sum over every cell of W_cell p          (a per-cell weight grid laid out
            like the grid: the scenario profile of Eq. 24)
    """

    def __init__(self, w_isl=1.0, w_psl=0.0, temp=0.05, h_tau=1, h_k=1,
                 u=None, v=None, eps=1e-12, match=None, w_match=0.0,
                 w_width=0.0, gamma=10.0, w_const=0.0, w_smooth=0.0, cell_w=None, w_cell=0.0):
        self.match = None if match is None else np.asarray(match, dtype=np.float64)
        self.w_match = float(w_match)
        self.w_width, self.gamma = float(w_width), float(gamma)
        self.w_const, self.w_smooth = float(w_const), float(w_smooth)
        self.cell_w = None if cell_w is None else np.asarray(cell_w, dtype=np.float64)
        self.w_cell = float(w_cell)
        self.w_isl, self.w_psl, self.temp = float(w_isl), float(w_psl), float(temp)
        self.h_tau, self.h_k = int(h_tau), int(h_k)
        self.u = None if u is None else np.asarray(u, dtype=np.float64)
        self.v = None if v is None else np.asarray(v, dtype=np.float64)
        self.eps = float(eps)


def loss_terms(c, E, n, params):
    """Loss value and its pieces from a complex grid c (no gradient; the
    waveform-only terms Const and Smooth are not grid terms and are left out)."""
    T = (c.shape[0] - 1) // 2
    m = c.shape[1]
    side = ~mainlobe_mask(m, T, params.h_tau, params.h_k)
    W = isl_weights(n, m, T, params.h_tau, params.h_k, params.u, params.v)
    return _loss_terms_on(c, E, params, side, W, np.abs(np.arange(-T, T + 1)).astype(np.float64))


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * np.asarray(z, dtype=np.float64)))


def soft_mainlobe_width(p, lagd, gamma):
    """Eq. 21 on a power grid p: sum over the rows of lagd * sigma(gamma
    (p[row, 0] - p[origin, 0] / 2)), the origin being the row with lagd 0."""
    r0 = int(np.argmin(lagd))
    z = gamma * (p[:, 0] - 0.5 * p[r0, 0])
    return float(np.sum(lagd * sigmoid(z)))


def _loss_terms_on(c, E, params, side, W, lagd):
    """The loss pieces of a grid c with its sidelobe region, ISL weights and
    the lag distance |tau| of each row."""
    p = power(c, E)
    a = np.sqrt(p + params.eps)
    isl = float(np.sum(W * p))
    av = a[side]
    mx = float(av.max())
    S = float(np.sum(np.exp((av - mx) / params.temp)))
    soft = mx + params.temp * math.log(S)
    match = float(np.sum((p - params.match) ** 2)) if params.match is not None else 0.0
    width = soft_mainlobe_width(p, lagd, params.gamma)
    cell = float(np.sum(params.cell_w * p)) if params.cell_w is not None else 0.0
    loss = (params.w_isl * isl + params.w_psl * soft + params.w_match * match + params.w_width * width +
            params.w_cell * cell)
    return dict(loss=loss, isl=isl, softpsl=soft, match=match, width=width, cell=cell, psl_db=psl_db(p, side),
                p=p, a=a, side=side, W=W, lagd=lagd, lse_max=mx, lse_sum=S)


def modulus_variance(s):
    """L_const = var(|s|) (Sec. 5.2), the population variance, with its
    gradient (|s[n]| - mean|s|) s[n] / (N |s[n]|) (0 where s[n] = 0)."""
    s = np.asarray(s, dtype=np.complex128)
    r = np.abs(s)
    mu = float(r.mean())
    v = float(np.mean((r - mu) ** 2))
    with np.errstate(invalid="ignore", divide="ignore"):
        u = np.where(r > 0, s / np.where(r > 0, r, 1.0), 0.0)
    return v, (r - mu) * u / len(s)


def phase_smoothness(s):
    """Smooth = sum_{n < N-1} |s[n+1] - s[n]|^2 / E with its gradient
    (d[n-1] - d[n]) / E - Smooth s[n] / E, d[n] = s[n+1] - s[n] (zero outside
    [0, N-1)).  For a unit-modulus code it is 2/N sum (1 - cos(phase step))."""
    s = np.asarray(s, dtype=np.complex128)
    E = energy(s)
    d = s[1:] - s[:-1]
    D = float(np.sum(np.abs(d) ** 2))
    g = np.zeros_like(s)
    g[1:] += d
    g[:-1] -= d
    return D / E, g / E - (D / (E * E)) * s


def _add_waveform_terms(t, s, params):
    """Const and Smooth, which depend on s alone, added to t's loss and g."""
    vc, gc = modulus_variance(s)
    vs, gs = phase_smoothness(s)
    t["const"], t["smooth"] = vc, vs
    t["loss"] += params.w_const * vc + params.w_smooth * vs
    t["g"] = t["g"] + params.w_const * gc + params.w_smooth * gs
    return t


def spectral_projection(s, mask, unit=False):
    """Bandwidth limit of Sec. 6.2's projected descent: the N-point DFT of s
    times a real mask per bin, transformed back (inverse DFT with 1/N); with
    unit, then s / |s| onto the unit circle (1 where the result is 0)."""
    s = np.asarray(s, dtype=np.complex128)
    n = s.shape[0]
    k = np.arange(n)
    F = np.exp(-2j * np.pi * np.outer(k, k) / n)
    y = (np.conj(F).T @ (np.asarray(mask, dtype=np.float64) * (F @ s))) / n
    if unit:
        r = np.abs(y)
        y = np.where(r > 0, y / np.where(r > 0, r, 1.0), 1.0 + 0j)
    return y


def loss_and_grad(s, m, max_lag, params):
    """Loss of Sec. 5 and dL/d conj(s) through chi, E and a (Eqs. 13-15).

    Per cell: dL/d conj(chi) = w_isl W chi / E^2 + w_psl q chi / (2 E^2 a),
    q = softmax over Omega_s of a/T.  Energy: dL/dE = -2 w_isl ISL / E
    - w_psl sum q p / (E a).  Then g = adjoint(G) + dL/dE * s.
    """
    s = np.asarray(s, dtype=np.complex128)
    n = s.shape[0]
    T = n - 1 if max_lag is None or max_lag < 0 else int(max_lag)
    return loss_grad_from_chi(s, m, T, chi(s, m, T), params)


def loss_grad_from_chi(s, m, T, c, params):
    """loss_and_grad with the complex grid c supplied (c = chi(s) for the
    reference; tests pass a perturbed grid to measure conditioning)."""
    s = np.asarray(s, dtype=np.complex128)
    n = s.shape[0]
    E = energy(s)
    t = loss_terms(c, E, n, params)
    G, dLdE = _cell_upstream(t, c, E, params)
    g = grad_from_upstream(s, m, T, G, dLdE)
    t.update(g=g, G=G, dLdE=dLdE, chi=c, E=E)
    return _add_waveform_terms(t, s, params)


def _cell_upstream(t, c, E, params):
    """G = dL/d conj(chi) per cell and dL/dE from the loss pieces t."""
    a, p, side, W = t["a"], t["p"], t["side"], t["W"]
    q = np.zeros_like(a)
    q[side] = np.exp((a[side] - t["lse_max"]) / params.temp) / t["lse_sum"]
    coef = params.w_isl * W / (E * E) + params.w_psl * q / (2.0 * E * E * a)
    dLdE = (-2.0 * params.w_isl * t["isl"] / E
            - params.w_psl * float(np.sum(q * p / (E * a))))
    if params.match is not None and params.w_match != 0.0:
        # d/d conj(chi) of (p - p_t)^2 = 2 (p - p_t) chi / E^2; dp/dE = -2 p / E
        d = p - params.match
        coef = coef + params.w_match * 2.0 * d / (E * E)
        dLdE += params.w_match * float(np.sum(2.0 * d * (-2.0 * p / E)))
    if params.cell_w is not None and params.w_cell != 0.0:
        # d/d conj(chi) of W p = W chi / E^2; dp/dE = -2 p / E
        coef = coef + params.w_cell * params.cell_w / (E * E)
        dLdE += params.w_cell * float(np.sum(params.cell_w * (-2.0 * p / E)))
    if params.w_width != 0.0:
        # Eq. 21: dWidth/dp(tau, 0) = |tau| gamma sigma'(z_tau); the origin
        # cell also carries -gamma/2 sum |tau| sigma'(z_tau)
        lagd = t["lagd"]
        r0 = int(np.argmin(lagd))
        sg = sigmoid(params.gamma * (p[:, 0] - 0.5 * p[r0, 0]))
        u = lagd * params.gamma * sg * (1.0 - sg)  # zero on the origin row (lagd 0)
        u[r0] = -0.5 * float(np.sum(u))
        coef = np.array(coef, dtype=np.float64)
        coef[:, 0] += params.w_width * u / (E * E)
        dLdE += params.w_width * float(np.sum(u * (-2.0 * p[:, 0] / E)))
    G = coef * c
    return G, dLdE


def magnitude_backward(s, m, max_lag, grad_mag, eps):
    """dL/d conj(s) for an upstream dL/da on the magnitude grid.

    dL/d conj(chi) = g_a chi / (2 E^2 a); dL/dE = -sum g_a p / (E a).
    """
    s = np.asarray(s, dtype=np.complex128)
    n = s.shape[0]
    T = n - 1 if max_lag is None or max_lag < 0 else int(max_lag)
    E = energy(s)
    c = chi(s, m, T)
    p = power(c, E)
    a = np.sqrt(p + eps)
    ga = np.asarray(grad_mag, dtype=np.float64)
    G = ga * c / (2.0 * E * E * a)
    dLdE = -float(np.sum(ga * p / (E * a)))
    return grad_from_upstream(s, m, T, G, dLdE)


def grad_from_upstream(s, m, max_lag, G, dLdE):
    """g = sum over the chain rule of Eq. 15: the lag-product adjoint applied to
    the inverse DFT of G, plus the energy term dL/dE * s (dE/d conj(s) = s)."""
    s = np.asarray(s, dtype=np.complex128)
    return _native.adjoint(s, int(m), int(max_lag), G) + dLdE * s


def phase_grad(s, g):
    """dL/dphi for s = exp(j phi): 2 Im(conj(s) * dL/d conj(s))."""
    return 2.0 * np.imag(np.conj(s) * g)


# ----------------------------------------------------------------------------
# the periodic (circular) AF: the paper's own Eqs. 2 and 7 and Algorithm 1
# ----------------------------------------------------------------------------
# The lag index wraps modulo N and the Doppler transform has N bins (no zero
# padding): chi_c[tau, k] = sum_{n<N} s[n] conj(s[(n - tau) mod N])
# exp(-j 2 pi k n / N), tau, k in [0, N); grids are [N, N] with row tau.
# Lag tau and lag N - tau are the two signs of one circular lag: the
# mainlobe is |tau|_c = min(tau, N - tau) <= h_tau, |k_c| <= h_k, with k_c
# the centred bin over N.

def chi_circular(s):
    """Periodic AF by its defining sum (C core, direct DFT, no FFT)."""
    return _native.chi_circ(np.asarray(s, dtype=np.complex128))


def chi_circular_rows(s, taus):
    """Rows tau of the periodic AF for N a power of two, from the aperiodic
    direct sums with M = N: lag tau of the periodic product collects the
    aperiodic lags tau and tau - N (pinned against chi_circular)."""
    s = np.asarray(s, dtype=np.complex128)
    n = s.shape[0]
    out = np.empty((len(taus), n), dtype=np.complex128)
    for i, tau in enumerate(taus):
        tau = int(tau) % n
        out[i] = chi_rows(s, n, [tau])[0]
        if tau > 0:
            out[i] += chi_rows(s, n, [tau - n])[0]
    return out


def circular_lag_distance(n):
    tau = np.arange(n)
    return np.minimum(tau, n - tau)


def circular_mainlobe_mask(n, h_tau, h_k):
    return (circular_lag_distance(n)[:, None] <= h_tau) & (np.abs(centred_bins(n))[None, :] <= h_k)


def circular_isl_weights(n, h_tau, h_k, u=None, v=None):
    """As isl_weights with |tau|_c and N bins: u[floor(31 |tau|_c / N)] *
    v[floor(31 |k_c| / (N/2 + 1))] off the mainlobe (1 without u, v)."""
    if u is None:
        W = np.ones((n, n))
    else:
        u = np.asarray(u, dtype=np.float64)
        v = np.asarray(v, dtype=np.float64)
        iu = (31 * circular_lag_distance(n)) // n
        iv = (31 * np.abs(centred_bins(n))) // (n // 2 + 1)
        W = u[iu][:, None] * v[iv][None, :]
    W[circular_mainlobe_mask(n, h_tau, h_k)] = 0.0
    return W


def loss_and_grad_circular(s, params):
    """The loss of Sec. 5 on the periodic AF and dL/d conj(s): the per-cell
    upstream as in loss_and_grad, then the periodic lag-product adjoint."""
    s = np.asarray(s, dtype=np.complex128)
    n = s.shape[0]
    E = energy(s)
    c = chi_circular(s)
    side = ~circular_mainlobe_mask(n, params.h_tau, params.h_k)
    W = circular_isl_weights(n, params.h_tau, params.h_k, params.u, params.v)
    t = _loss_terms_on(c, E, params, side, W, circular_lag_distance(n).astype(np.float64))
    G, dLdE = _cell_upstream(t, c, E, params)
    g = _native.adjoint_circ(s, G) + dLdE * s
    t.update(g=g, G=G, dLdE=dLdE, chi=c, E=E)
    return _add_waveform_terms(t, s, params)


def magnitude_backward_circular(s, grad_mag, eps):
    """dL/d conj(s) for an upstream dL/da on the periodic magnitude grid."""
    s = np.asarray(s, dtype=np.complex128)
    E = energy(s)
    c = chi_circular(s)
    p = power(c, E)
    a = np.sqrt(p + eps)
    ga = np.asarray(grad_mag, dtype=np.float64)
    G = ga * c / (2.0 * E * E * a)
    dLdE = -float(np.sum(ga * p / (E * a)))
    return _native.adjoint_circ(s, G) + dLdE * s


# ----------------------------------------------------------------------------
# the experiment loss of Sec. 7.1.1: hard PSL + lambda alpha SpectralVariance
# ----------------------------------------------------------------------------

def spectral_variance(s):
    """V = var_j{ P_j / sum P }, P_j = |X_j|^2, X = the N-point DFT of s
    (no padding), population variance (mean of squared deviations from 1/N);
    returns (V, dV/d conj(s)).

    With x_j = P_j / S, S = sum P: dV/dP_j = 2 (x_j - sum_k x_k^2) / (N S),
    and dV/d conj(s[n]) = sum_j dV/dP_j X_j exp(+j 2 pi j n / N)."""
    s = np.asarray(s, dtype=np.complex128)
    n = s.shape[0]
    k = np.arange(n)
    F = np.exp(-2j * np.pi * np.outer(k, k) / n)  # DFT matrix by its definition
    X = F @ s
    P = X.real * X.real + X.imag * X.imag
    S = float(P.sum())
    x = P / S
    V = float(np.mean((x - 1.0 / n) ** 2))
    c = 2.0 * (x - float(np.sum(x * x))) / (n * S)
    g = np.conj(F).T @ (c * X)
    return V, g


def hard_psl(c, E, side):
    """PSL of Eq. 18 as a power ratio: max over the sidelobe cells of
    p = |chi|^2 / E^2; returns (PSL, (row, bin) of the maximum).  Ties take
    the first cell in row-major order."""
    p = power(c, E)
    pm = np.where(side, p, -np.inf)
    idx = int(np.argmax(pm))
    return float(pm.flat[idx]), np.unravel_index(idx, p.shape)


def experiment_loss_and_grad(s, m, lam, alpha=2000.0, h_tau=0, h_k=0, periodic=False, eps=1e-12):
    """L = PSL + lam * alpha * V (Sec. 7.1.1) and dL/d conj(s): the PSL
    subgradient sits on the maximising cell (dp/d conj(chi) = chi / E^2
    there, dPSL/dE = -2 PSL / E), the spectral part as in
    spectral_variance.  The grid is the periodic AF when periodic, else the
    aperiodic one with M bins and the full lag window."""
    s = np.asarray(s, dtype=np.complex128)
    n = s.shape[0]
    E = energy(s)
    if periodic:
        c = chi_circular(s)
        side = ~circular_mainlobe_mask(n, h_tau, h_k)
    else:
        c = chi(s, m, n - 1)
        side = ~mainlobe_mask(m, n - 1, h_tau, h_k)
    psl, cell = hard_psl(c, E, side)
    G = np.zeros_like(c)
    G[cell] = c[cell] / (E * E)
    gp = (_native.adjoint_circ(s, G) if periodic else _native.adjoint(s, m, n - 1, G)) - 2.0 * psl / E * s
    V, gv = spectral_variance(s)
    return dict(loss=psl + lam * alpha * V, psl=psl, cell=cell, spec_var=V, g=gp + lam * alpha * gv,
                g_psl=gp, g_spec=gv, chi=c, E=E, a=magnitude(c, E, eps), side=side)


# ----------------------------------------------------------------------------
# multi-scenario loss (Eq. 24): L_multi = sum_i lambda_i L_i(chi_s, scenario_i)
# ----------------------------------------------------------------------------

def multi_scenario_loss_and_grad(s, m, max_lag, scenarios, lambdas, periodic=False):
    """Eq. 24 as written: each scenario's loss (its own LossParams) on the
    same AF, weighted by lambda_i and summed, with the gradient likewise."""
    total, g = 0.0, None
    for params, lam in zip(scenarios, lambdas):
        t = loss_and_grad_circular(s, params) if periodic else loss_and_grad(s, m, max_lag, params)
        total += float(lam) * t["loss"]
        g = float(lam) * t["g"] if g is None else g + float(lam) * t["g"]
    return total, g


def combine_scenario_weights(grids, lambdas):
    """sum_i lambda_i W_i of per-cell weight grids (the linear scenario terms
    of Eq. 24 folded into one grid)."""
    out = np.zeros_like(np.asarray(grids[0], dtype=np.float64))
    for w, lam in zip(grids, lambdas):
        out = out + float(lam) * np.asarray(w, dtype=np.float64)
    return out


# ----------------------------------------------------------------------------
# cross-ambiguity of two waveforms (the cross-AF/MIMO extension the paper's
# limitations name): chi_su[tau, k] = sum_n s[n] conj(u[n - tau]) exp(-j 2 pi
# k n / M), equal to chi when u = s; normalised power p = |chi_su|^2 /
# (E_s E_u) <= 1 by Cauchy-Schwarz, a = sqrt(p + eps)
# ----------------------------------------------------------------------------

def _cross_products(s, u, max_lag):
    """Rows tau = -T..T of the lag products x_tau[n] = s[n] conj(u[n - tau])
    (zero where n - tau leaves [0, N))."""
    n = s.shape[0]
    X = np.zeros((2 * max_lag + 1, n), dtype=np.complex128)
    idx = np.arange(n)
    for i, tau in enumerate(range(-max_lag, max_lag + 1)):
        j = idx - tau
        ok = (j >= 0) & (j < n)
        X[i, ok] = s[ok] * np.conj(u[j[ok]])
    return X


def _dft_matrix(n, m, bins=None):
    """F[n, k] = exp(-j 2 pi k n / M) for the bins k (all M by default), from
    the integer product k n mod M."""
    k = np.arange(m, dtype=np.int64) if bins is None else np.asarray(bins, dtype=np.int64)
    kn = np.outer(np.arange(n, dtype=np.int64), k) % m
    return np.exp(-2j * np.pi * kn / m)


def cross_chi(s, u, m, max_lag=None, bins=None):
    """The cross-AF grid [2T+1, M] by its defining sum (a product matrix
    times the DFT matrix); with bins, only those columns."""
    s = np.asarray(s, dtype=np.complex128)
    u = np.asarray(u, dtype=np.complex128)
    n = s.shape[0]
    T = n - 1 if max_lag is None or max_lag < 0 else int(max_lag)
    return _cross_products(s, u, T) @ _dft_matrix(n, m, bins)


def cross_magnitude_backward(s, u, m, max_lag, grad_mag, eps):
    """(dL/d conj(s), dL/d conj(u)) for an upstream dL/da on the cross-AF
    magnitude grid.  Per cell G = g_a chi / (2 E_s E_u a); Q_tau[n] =
    sum_k G[tau, k] exp(+j 2 pi k n / M); then dL/d conj(s[n]) = sum_tau
    u[n - tau] Q_tau[n] and dL/d conj(u[m]) = sum_tau s[m + tau]
    conj(Q_tau[m + tau]); the energies add dL/dE_s s and dL/dE_u u with
    dL/dE_s = -sum g_a p / (2 a E_s) (and E_u alike)."""
    s = np.asarray(s, dtype=np.complex128)
    u = np.asarray(u, dtype=np.complex128)
    n = s.shape[0]
    T = n - 1 if max_lag is None or max_lag < 0 else int(max_lag)
    F = _dft_matrix(n, m)
    c = _cross_products(s, u, T) @ F
    Es, Eu = energy(s), energy(u)
    p = (c.real ** 2 + c.imag ** 2) / (Es * Eu)
    a = np.sqrt(p + eps)
    ga = np.asarray(grad_mag, dtype=np.float64)
    G = ga * c / (2.0 * Es * Eu * a)
    Q = G @ np.conj(F).T
    gs = np.zeros(n, dtype=np.complex128)
    gu = np.zeros(n, dtype=np.complex128)
    idx = np.arange(n)
    for i, tau in enumerate(range(-T, T + 1)):
        j = idx - tau
        ok = (j >= 0) & (j < n)
        gs[ok] += u[j[ok]] * Q[i, ok]
        np.add.at(gu, j[ok], s[ok] * np.conj(Q[i, ok]))
    q = float(np.sum(ga * p / a))
    return gs - q / (2.0 * Es) * s, gu - q / (2.0 * Eu) * u


# periodic form (the circular lags of Eq. 2 applied to the cross-AF): rows
# tau = 0..N-1, bins k over N, chi_su[tau, k] = sum_n s[n] conj(u[(n - tau)
# mod N]) exp(-j 2 pi k n / N)

def _cross_products_circular(s, u):
    """Rows tau = 0..N-1 of x_tau[n] = s[n] conj(u[(n - tau) mod N])."""
    n = s.shape[0]
    idx = np.arange(n)
    X = np.empty((n, n), dtype=np.complex128)
    for tau in range(n):
        X[tau] = s * np.conj(u[(idx - tau) % n])
    return X


def cross_chi_circular(s, u, bins=None):
    """The periodic cross-AF grid [N, N] by its defining sum; with bins,
    only those columns."""
    s = np.asarray(s, dtype=np.complex128)
    u = np.asarray(u, dtype=np.complex128)
    n = s.shape[0]
    return _cross_products_circular(s, u) @ _dft_matrix(n, n, bins)


def cross_magnitude_backward_circular(s, u, grad_mag, eps):
    """(dL/d conj(s), dL/d conj(u)) for an upstream dL/da on the periodic
    cross-AF magnitude grid: as cross_magnitude_backward with the sample
    indices taken modulo N and Q_tau[n] = sum_k G[tau, k] exp(+j 2 pi k n / N)."""
    s = np.asarray(s, dtype=np.complex128)
    u = np.asarray(u, dtype=np.complex128)
    n = s.shape[0]
    F = _dft_matrix(n, n)
    c = _cross_products_circular(s, u) @ F
    Es, Eu = energy(s), energy(u)
    p = (c.real ** 2 + c.imag ** 2) / (Es * Eu)
    a = np.sqrt(p + eps)
    ga = np.asarray(grad_mag, dtype=np.float64)
    G = ga * c / (2.0 * Es * Eu * a)
    Q = G @ np.conj(F).T
    gs = np.zeros(n, dtype=np.complex128)
    gu = np.zeros(n, dtype=np.complex128)
    idx = np.arange(n)
    for tau in range(n):
        j = (idx - tau) % n
        gs += u[j] * Q[tau]
        np.add.at(gu, j, s * np.conj(Q[tau]))
    q = float(np.sum(ga * p / a))
    return gs - q / (2.0 * Es) * s, gu - q / (2.0 * Eu) * u


# ----------------------------------------------------------------------------
# optimiser (Sec. 6.2 update, Sec. 7.1.2 settings: Adam, lr 0.01)
# ----------------------------------------------------------------------------

def adam_step(x, grad, m, v, t, lr=0.01, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step (Kingma & Ba), eps outside the square root.
    t is the 1-based step index.  Returns the new (x, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return x - lr * mh / (np.sqrt(vh) + eps), m, v


# ----------------------------------------------------------------------------
# proposal network (Sec. 6.1, Fig. 1: parameters -> network -> waveform)
# ----------------------------------------------------------------------------

def bf16_round(x):
    """Round float64 values to the nearest bfloat16 (ties to even), returned as
    float64.  Goes through float32 first, which is exact for values that are
    already float32 and otherwise adds one float32 rounding."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rnd = ((u >> 16) & 1) + 0x7FFF
    u = ((u + rnd) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(x):
    """Exact GELU: x * Phi(x)."""
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    """d GELU / dx = Phi(x) + x * phi(x)."""
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def mlp_forward(x, weights, biases, emulate_bf16=True):
    """Z_i = A_{i-1} W_i^T + b_i; A_i = GELU(Z_i) for hidden layers; the last
    layer is linear.  With emulate_bf16 the GEMM operands (inputs, weights,
    activations) are rounded to bfloat16 exactly where the GPU stores them in
    bfloat16; sums are exact float64.  Returns (output, cache)."""
    r = bf16_round if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    A = r(x)
    acts, pres = [A], []
    L = len(weights)
    for i, (W, b) in enumerate(zip(weights, biases)):
        Z = A @ r(W).T + np.asarray(b, dtype=np.float64)
        pres.append(Z)
        if i < L - 1:
            A = r(gelu(Z))
            acts.append(A)
        else:
            A = Z
    return A, dict(acts=acts, pres=pres)


def mlp_backward(dout, weights, cache, emulate_bf16=True):
    """Gradients of the network in mlp_forward for an upstream dL/d out.
    The upstream of every GEMM is rounded to bfloat16 where the GPU rounds it.
    Returns (dW list, db list)."""
    r = bf16_round if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    L = len(weights)
    dW, db = [None] * L, [None] * L
    dZ = np.asarray(dout, dtype=np.float64)
    for i in range(L - 1, -1, -1):
        dZr = r(dZ)
        dW[i] = dZr.T @ cache["acts"][i]
        db[i] = dZ.sum(axis=0)
        if i > 0:
            dA = dZr @ r(weights[i])
            dZ = dA * gelu_grad(cache["pres"][i - 1])
    return dW, db


# ----------------------------------------------------------------------------
# the same definitions with numpy's FFT as the Doppler-sum step, for sizes the
# direct sums cannot reach in seconds (pinned against the direct sums by tests)
# ----------------------------------------------------------------------------

def _lag_product(s, m, tau):
    n = s.shape[0]
    r = np.zeros(m, dtype=np.complex128)
    lo, hi = max(0, tau), min(n, n + tau)
    r[lo:hi] = s[lo:hi] * np.conj(s[lo - tau:hi - tau])
    return r, lo, hi


def chi_rows_fft(s, m, taus):
    """chi rows for the given lags: the Doppler sum of Eq. 11 by FFT."""
    s = np.asarray(s, dtype=np.complex128)
    out = np.empty((len(taus), m), dtype=np.complex128)
    for i, tau in enumerate(taus):
        out[i] = np.fft.fft(_lag_product(s, m, int(tau))[0])
    return out


def magnitude_backward_fft(s, m, max_lag, grad_mag, eps, rows_per_block=64):
    """magnitude_backward with FFT steps, streamed over lag rows: per row
    chi = FFT(r), G = g_a chi / (2 E^2 a), Q = M * IFFT(G), then the two
    adjoint terms of the lag product and the energy term.  grad_mag is an
    array [2T+1, M] or a callable (row index, a row) -> that row's dL/da."""
    s = np.asarray(s, dtype=np.complex128)
    n = s.shape[0]
    T = int(max_lag)
    E = energy(s)
    g = np.zeros(n, dtype=np.complex128)
    dLdE = 0.0
    for i0 in range(0, 2 * T + 1, rows_per_block):
        i1 = min(2 * T + 1, i0 + rows_per_block)
        for i in range(i0, i1):
            tau = i - T
            r, lo, hi = _lag_product(s, m, tau)
            c = np.fft.fft(r)
            p = power(c, E)
            a = np.sqrt(p + eps)
            ga = np.asarray(grad_mag(i, a) if callable(grad_mag) else grad_mag[i], dtype=np.float64)
            G = ga * c / (2.0 * E * E * a)
            dLdE -= float(np.sum(ga * p / (E * a)))
            Q = np.fft.ifft(G) * m
            # Q_tau[p] s[p - tau] for p in [lo, hi)
            g[lo:hi] += Q[lo:hi] * s[lo - tau:hi - tau]
            # conj(Q_tau[q]) s[q] added at p = q - tau for q in [lo, hi)
            g[lo - tau:hi - tau] += np.conj(Q[lo:hi]) * s[lo:hi]
    return g + dLdE * s

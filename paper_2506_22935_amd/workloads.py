"""Seeded synthetic inputs for every workload the library is measured and
tested on.

This module draws random numbers and lays out sizes; it holds none of the
ambiguity-function arithmetic, so the oracle and the HIP path can both take
their inputs from it.  All randomness is numpy's PCG64 (``default_rng``).

Workloads (sizes follow the paper's phase-coded setting, Sec. 7.1.2, widened
to the lag/Doppler grids this library covers):
  single_small  N=64,    M=128,   all 127 lags, random phase code
  single        N=1024,  M=2048,  all 2047 lags, random phase code
  uneven        512 random phase codes, N log-uniform in [64, 4096],
                M = next power of two >= 2N, all lags of each
  large         N=16384 LFM chirp (time-bandwidth 1000) + N(0, 0.3) rad phase
                noise, lags |tau| <= 2048, M=32768
  proposal      4096 sidelobe-mask descriptors (64 floats each), N=256, M=512
"""
import math

import numpy as np

TWO_PI = 2.0 * math.pi


def next_pow2(x):
    return 1 << (int(x) - 1).bit_length()


def random_phases(n, seed):
    """phi_n uniform on [0, 2 pi), float64."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, TWO_PI, size=n)


def unimodular(phases):
    """s = exp(j phi) rounded to complex64 (what the GPU receives)."""
    phases = np.asarray(phases, dtype=np.float64)
    return np.exp(1j * phases).astype(np.complex64)


def random_code(n, seed):
    return unimodular(random_phases(n, seed))


def complex_gaussian(n, seed):
    """Circular complex Gaussian samples (unit variance), rounded to complex64:
    a waveform whose modulus varies, so no AF cell vanishes exactly."""
    rng = np.random.default_rng(seed)
    z = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / math.sqrt(2.0)
    return z.astype(np.complex64)


def lfm_noisy_phases(n=16384, time_bandwidth=1000.0, sigma=0.3, seed=0):
    """Quadratic LFM phase pi*BT*(n/N - 1/2)^2 plus Gaussian phase noise."""
    rng = np.random.default_rng(seed)
    t = np.arange(n, dtype=np.float64) / n - 0.5
    return math.pi * time_bandwidth * t * t + sigma * rng.standard_normal(n)


def uneven_lengths(count=512, nmin=64, nmax=4096, seed=0):
    """N = round(exp(U[ln nmin, ln nmax])), clipped to [nmin, nmax]."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(math.log(nmin), math.log(nmax), size=count)
    return np.clip(np.rint(np.exp(x)).astype(np.int64), nmin, nmax)


def uneven_batch(count=512, nmin=64, nmax=4096, seed=0):
    """Lengths, M per waveform and one random phase code per waveform."""
    ns = uneven_lengths(count, nmin, nmax, seed)
    ms = np.array([next_pow2(2 * n) for n in ns], dtype=np.int64)
    rng = np.random.default_rng(seed + 1_000_003)
    phases = [rng.uniform(0.0, TWO_PI, size=int(n)) for n in ns]
    return ns, ms, phases


def descriptors(batch, seed=0, max_half_width=4):
    """Sidelobe-mask descriptors: integer mainlobe half-widths h_tau, h_k in
    [1, max_half_width] and 31 + 31 shaping weights u, v ~ U[0, 1].
    The network input is d = [h_tau/16, h_k/16, u, v] (64 floats)."""
    rng = np.random.default_rng(seed)
    h_tau = rng.integers(1, max_half_width + 1, size=batch)
    h_k = rng.integers(1, max_half_width + 1, size=batch)
    u = rng.uniform(0.0, 1.0, size=(batch, 31))
    v = rng.uniform(0.0, 1.0, size=(batch, 31))
    d = np.concatenate([h_tau[:, None] / 16.0, h_k[:, None] / 16.0, u, v], axis=1)
    return dict(d=d.astype(np.float32), h_tau=h_tau.astype(np.int32),
                h_k=h_k.astype(np.int32), u=u.astype(np.float32),
                v=v.astype(np.float32))


def upstream_grid(rows, m, seed):
    """A seeded float32 upstream gradient dL/da for a magnitude grid."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((rows, m)).astype(np.float32)


WORKLOADS = {
    "single_small": dict(n=64, m=128, max_lag=63),
    "single": dict(n=1024, m=2048, max_lag=1023),
    "uneven": dict(count=512, nmin=64, nmax=4096),
    "large": dict(n=16384, m=32768, max_lag=2048),
    "proposal": dict(batch=4096, n=256, m=512, max_lag=255),
}
